/*
 * Seeded synthetic "layered battery" linear systems.
 *
 * This module only produces inputs: a CSR matrix, its field map, and the
 * seeded vectors (exact solution, right-hand side, target) that the solver
 * and the CPU oracle both consume.  It contains none of the solver's
 * arithmetic.
 *
 * The paper's systems come from finite-element snapshots of a thermal
 * battery (Sec. 2, the solid/liquid voltage, continuity and Stefan-Maxwell
 * equations); those are not available, so a finite-volume stand-in with the
 * same block structure is assembled here:
 *   fields per cell, interleaved: phi_s, phi_e, p, c_1 [, c_2, c_3]
 *   5-point (2D) or 7-point (3D) two-point-flux stencils on unit cells,
 *   five layers along the last axis: collector / anode / separator /
 *   cathode / collector at height fractions 0.1 / 0.3 / 0.2 / 0.3 / 0.1.
 *
 * Row assembly order (fixes the floating-point result bit for bit):
 *   1. own-field transport, faces in order -x,+x,-y,+y[,-z,+z]:
 *        interior face: T = 2 k_i k_j / (k_i + k_j); if T > 0 add T on the
 *        diagonal and -T on the neighbour; species rows then add the
 *        first-order upwind convection (u = pt_i - pt_j): +max(u,0) on the
 *        diagonal and -max(-u,0) on the neighbour;
 *        boundary face with a Dirichlet condition: +2 k_i on the diagonal;
 *   2. species rows: + 1/dt on the diagonal;
 *   3. electrode cells (anode, cathode), k = j0(cell):
 *        phi_s row: +k (phi_s), -k (phi_e); phi_e row: -k (phi_s), +k (phi_e);
 *        species rows: -k/2 (phi_s), +k/2 (phi_e);
 *   4. species rows at cells where phi_e is active: mig * (phi_e stencil),
 *        faces in the same order: +mig*T_e on phi_e(cell), -mig*T_e on
 *        phi_e(neighbour).
 *   Identity rows (a single 1 on the diagonal): phi_s in the separator,
 *   phi_e in the collectors.
 *
 * Random numbers are counter based: u(stream, idx) =
 *   (splitmix64(seed ^ (stream * 0xD1B54A32D192ED03) ^ idx) >> 11) * 2^-53,
 * with splitmix64 the mixer of Steele, Lea and Flood (OOPSLA 2014).
 * Streams: 0 permeability, 1 j0, 2 x*, 3 pressure-mode parameters,
 * 4 target x_t, 5 finite-difference cells.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t nx, ny, nz;   /* nz == 0: two-dimensional grid, layers along y */
  int32_t nspecies;     /* 1 or 3 species fields after phi_s, phi_e, p */
  uint64_t seed;
  double diff[3];       /* species diffusivities */
  double inv_dt;        /* species mass term 1/dt */
  double mig;           /* migration factor on the phi_e stencil */
  double perm_lo, perm_hi;
  double j0_lo, j0_hi;
} synth_params;

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

double synth_u01(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(splitmix64(seed ^ (stream * 0xD1B54A32D192ED03ull) ^ idx) >> 11) *
         0x1.0p-53;
}

enum { L_COLL0 = 0, L_ANODE = 1, L_SEP = 2, L_CATH = 3, L_COLL1 = 4 };

/* layer of cell t (0..N-1) along the layered axis: first L with
 * (2t+1)*10 < 2N*C_L, C = 1,4,6,9,10 (cumulative tenths of the height). */
int32_t synth_layer(int32_t t, int32_t N) {
  static const int64_t C[5] = {1, 4, 6, 9, 10};
  for (int L = 0; L < 5; ++L)
    if ((int64_t)(2 * t + 1) * 10 < 2 * (int64_t)N * C[L]) return L;
  return 4;
}

typedef struct {
  int32_t nx, ny, nz, dim, nf, nl;  /* nl = size of layered axis */
  int64_t ncell;
  const synth_params *p;
  double *perm;  /* per cell */
  double *j0;    /* per cell */
  double *pt;    /* smooth pressure per cell */
  const double *j0_override;
} grid_t;

static double kappa(const grid_t *g, int f, int64_t cell, int layer) {
  switch (f) {
    case 0:
      if (layer == L_COLL0 || layer == L_COLL1) return 1e4;
      if (layer == L_SEP) return 0.0;
      return 1e2;
    case 1:
      if (layer == L_COLL0 || layer == L_COLL1) return 0.0;
      return 1.0;
    case 2:
      return g->perm[cell];
    default:
      return g->p->diff[f - 3];
  }
}

static double harm(double a, double b) {
  if (a == 0.0 || b == 0.0) return 0.0;
  return 2.0 * a * b / (a + b);
}

static void cell_coords(const grid_t *g, int64_t cell, int32_t x[3]) {
  x[0] = (int32_t)(cell % g->nx);
  int64_t r = cell / g->nx;
  x[1] = (int32_t)(r % g->ny);
  x[2] = (int32_t)(r / g->ny);
}

static int layer_of_cell(const grid_t *g, int64_t cell) {
  int32_t x[3];
  cell_coords(g, cell, x);
  return synth_layer(g->dim == 2 ? x[1] : x[2], g->nl);
}

/* neighbour of cell across face q (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z), -1 at the boundary */
static int64_t neighbour(const grid_t *g, int64_t cell, int q) {
  int32_t x[3];
  cell_coords(g, cell, x);
  int d = q >> 1, s = (q & 1) ? 1 : -1;
  int32_t n[3] = {g->nx, g->ny, g->nz};
  int32_t v = x[d] + s;
  if (v < 0 || v >= n[d]) return -1;
  int64_t stride = d == 0 ? 1 : (d == 1 ? g->nx : (int64_t)g->nx * g->ny);
  return cell + s * stride;
}

static int is_identity_row(int f, int layer) {
  if (f == 0 && layer == L_SEP) return 1;
  if (f == 1 && (layer == L_COLL0 || layer == L_COLL1)) return 1;
  return 0;
}

static int is_electrode(int layer) { return layer == L_ANODE || layer == L_CATH; }

/* Dirichlet faces: phi_s = 0 on the bottom faces, p = 0 on the top faces. */
static int dirichlet(const grid_t *g, int f, int q) {
  int last = g->dim - 1;
  if (f == 0 && q == 2 * last) return 1;
  if (f == 2 && q == 2 * last + 1) return 1;
  return 0;
}

/* per-row accumulator: at most 2*dim+3 distinct columns */
typedef struct {
  int64_t col[16];
  double val[16];
  int32_t dcell[16]; /* cell whose j0 the entry is linear in (-1: none) */
  double dcoef[16];
  int n;
} rowacc;

static void acc_add(rowacc *r, int64_t col, double v) {
  for (int i = 0; i < r->n; ++i)
    if (r->col[i] == col) {
      r->val[i] += v;
      return;
    }
  r->col[r->n] = col;
  r->val[r->n] = v;
  r->dcell[r->n] = -1;
  r->dcoef[r->n] = 0.0;
  r->n++;
}

static void acc_dj0(rowacc *r, int64_t col, int32_t cell, double coef) {
  for (int i = 0; i < r->n; ++i)
    if (r->col[i] == col) {
      r->dcell[i] = cell;
      r->dcoef[i] += coef;
      return;
    }
}

static void acc_sort(rowacc *r) {
  for (int i = 1; i < r->n; ++i) {
    int64_t c = r->col[i];
    double v = r->val[i], dc = r->dcoef[i];
    int32_t dl = r->dcell[i];
    int j = i - 1;
    while (j >= 0 && r->col[j] > c) {
      r->col[j + 1] = r->col[j];
      r->val[j + 1] = r->val[j];
      r->dcell[j + 1] = r->dcell[j];
      r->dcoef[j + 1] = r->dcoef[j];
      --j;
    }
    r->col[j + 1] = c;
    r->val[j + 1] = v;
    r->dcell[j + 1] = dl;
    r->dcoef[j + 1] = dc;
  }
}

static void assemble_row(const grid_t *g, int64_t row, rowacc *r) {
  const int nf = g->nf;
  int64_t cell = row / nf;
  int f = (int)(row % nf);
  int layer = layer_of_cell(g, cell);
  r->n = 0;
  if (is_identity_row(f, layer)) {
    acc_add(r, row, 1.0);
    return;
  }
  const int nq = 2 * g->dim;
  double kc = kappa(g, f, cell, layer);
  for (int q = 0; q < nq; ++q) {
    int64_t nb = neighbour(g, cell, q);
    if (nb >= 0) {
      double T = harm(kc, kappa(g, f, nb, layer_of_cell(g, nb)));
      if (T > 0.0) {
        acc_add(r, row, T);
        acc_add(r, nf * nb + f, -T);
      }
      if (f >= 3) {
        double u = g->pt[cell] - g->pt[nb];
        acc_add(r, row, u > 0.0 ? u : 0.0);
        acc_add(r, nf * nb + f, -(-u > 0.0 ? -u : 0.0));
      }
    } else if (dirichlet(g, f, q)) {
      acc_add(r, row, 2.0 * kc);
    }
  }
  if (f >= 3) acc_add(r, row, g->p->inv_dt);
  if (is_electrode(layer)) {
    double k = g->j0_override ? g->j0_override[cell] : g->j0[cell];
    int64_t cs = nf * cell + 0, ce = nf * cell + 1;
    if (f == 0) {
      acc_add(r, cs, k);
      acc_add(r, ce, -k);
      acc_dj0(r, cs, (int32_t)cell, 1.0);
      acc_dj0(r, ce, (int32_t)cell, -1.0);
    } else if (f == 1) {
      acc_add(r, cs, -k);
      acc_add(r, ce, k);
      acc_dj0(r, cs, (int32_t)cell, -1.0);
      acc_dj0(r, ce, (int32_t)cell, 1.0);
    } else if (f >= 3) {
      acc_add(r, cs, -0.5 * k);
      acc_add(r, ce, 0.5 * k);
      acc_dj0(r, cs, (int32_t)cell, -0.5);
      acc_dj0(r, ce, (int32_t)cell, 0.5);
    }
  }
  if (f >= 3 && !is_identity_row(1, layer)) {
    double ke = kappa(g, 1, cell, layer);
    for (int q = 0; q < nq; ++q) {
      int64_t nb = neighbour(g, cell, q);
      if (nb < 0) continue;
      double Te = harm(ke, kappa(g, 1, nb, layer_of_cell(g, nb)));
      if (Te > 0.0) {
        acc_add(r, nf * cell + 1, g->p->mig * Te);
        acc_add(r, nf * nb + 1, -(g->p->mig * Te));
      }
    }
  }
  acc_sort(r);
}

static const double TWO_PI = 6.283185307179586;

static int grid_init(grid_t *g, const synth_params *p, const double *j0_override) {
  memset(g, 0, sizeof(*g));
  g->p = p;
  g->nx = p->nx;
  g->ny = p->ny;
  g->nz = p->nz > 0 ? p->nz : 1;
  g->dim = p->nz > 0 ? 3 : 2;
  g->nl = g->dim == 2 ? g->ny : g->nz;
  g->nf = 3 + p->nspecies;
  g->ncell = (int64_t)g->nx * g->ny * g->nz;
  g->j0_override = j0_override;
  g->perm = (double *)malloc(sizeof(double) * g->ncell);
  g->j0 = (double *)malloc(sizeof(double) * g->ncell);
  g->pt = (double *)malloc(sizeof(double) * g->ncell);
  if (!g->perm || !g->j0 || !g->pt) return -1;
  /* smooth pressure modes: amplitude, wave numbers in {1,2,3}, phase */
  double amp[4], ph[4];
  int kw[4][3];
  for (int m = 0; m < 4; ++m) {
    amp[m] = 2.0 * synth_u01(p->seed, 3, 8 * m + 0) - 1.0;
    for (int d = 0; d < 3; ++d) kw[m][d] = 1 + (int)(3.0 * synth_u01(p->seed, 3, 8 * m + 1 + d));
    ph[m] = TWO_PI * synth_u01(p->seed, 3, 8 * m + 4);
  }
  const double plo = p->perm_lo, phi = p->perm_hi, jlo = p->j0_lo, jhi = p->j0_hi;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < g->ncell; ++c) {
    g->perm[c] = plo * pow(phi / plo, synth_u01(p->seed, 0, (uint64_t)c));
    g->j0[c] = jlo * pow(jhi / jlo, synth_u01(p->seed, 1, (uint64_t)c));
    int32_t x[3];
    cell_coords(g, c, x);
    int32_t nn[3] = {g->nx, g->ny, g->nz};
    double s = 0.0;
    for (int m = 0; m < 4; ++m) {
      double arg = ph[m];
      for (int d = 0; d < g->dim; ++d) arg += TWO_PI * kw[m][d] * (x[d] + 0.5) / nn[d];
      s += amp[m] * sin(arg);
    }
    g->pt[c] = s;
  }
  return 0;
}

static void grid_free(grid_t *g) {
  free(g->perm);
  free(g->j0);
  free(g->pt);
}

/* Number of rows of the system. */
int64_t synth_nrows(const synth_params *p) {
  int64_t nz = p->nz > 0 ? p->nz : 1;
  return (int64_t)p->nx * p->ny * nz * (3 + p->nspecies);
}

/* Pass 1: rowptr[0..n] (n+1 entries). Returns nnz, or -1 on failure. */
int64_t synth_rowptr(const synth_params *p, int64_t *rowptr) {
  grid_t g;
  if (grid_init(&g, p, NULL)) return -1;
  int64_t n = g.ncell * g.nf;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    rowacc r;
    assemble_row(&g, i, &r);
    rowptr[i + 1] = r.n;
  }
  rowptr[0] = 0;
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
  grid_free(&g);
  return rowptr[n];
}

/* Pass 2: columns, values, j0-derivative map (dcell, dcoef; may be NULL),
 * field of each row.  j0_override (per cell, may be NULL) replaces the
 * seeded exchange-current coefficients. */
int synth_fill(const synth_params *p, const double *j0_override, const int64_t *rowptr,
               int32_t *col, double *val, int32_t *dcell, double *dcoef,
               int32_t *field_of_row) {
  grid_t g;
  if (grid_init(&g, p, j0_override)) return -1;
  int64_t n = g.ncell * g.nf;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < n; ++i) {
    rowacc r;
    assemble_row(&g, i, &r);
    if (rowptr[i + 1] - rowptr[i] != r.n) {
      bad = 1;
      continue;
    }
    for (int k = 0; k < r.n; ++k) {
      col[rowptr[i] + k] = (int32_t)r.col[k];
      val[rowptr[i] + k] = r.val[k];
      if (dcell) dcell[rowptr[i] + k] = r.dcell[k];
      if (dcoef) dcoef[rowptr[i] + k] = r.dcoef[k];
    }
    if (field_of_row) field_of_row[i] = (int32_t)(i % g.nf);
  }
  grid_free(&g);
  return bad ? -2 : 0;
}

/* Per-cell data: layer, seeded j0, permeability, smooth pressure. */
int synth_cells(const synth_params *p, int32_t *layer, double *j0, double *perm, double *pt) {
  grid_t g;
  if (grid_init(&g, p, NULL)) return -1;
  for (int64_t c = 0; c < g.ncell; ++c) {
    if (layer) layer[c] = layer_of_cell(&g, c);
    if (j0) j0[c] = g.j0[c];
    if (perm) perm[c] = g.perm[c];
    if (pt) pt[c] = g.pt[c];
  }
  grid_free(&g);
  return 0;
}

/* Seeded uniform[-1,1] vector from a stream: out[i] = 2 u(stream, i) - 1. */
void synth_uniform_pm1(uint64_t seed, uint64_t stream, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = 2.0 * synth_u01(seed, stream, (uint64_t)i) - 1.0;
}

/* y = A x in ascending column order, products rounded before each add
 * (the library is built without floating-point contraction). */
void synth_matvec(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                  const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
    y[i] = s;
  }
}
