// CPU oracle for the block Gauss-Seidel / smoothed-aggregation AMG /
// flexible GMRES solve.  TEST INFRASTRUCTURE ONLY: nothing in the product
// path may link or call this file; only the tests, the smoke check and the
// benchmark's CPU-baseline leg use it.
//
// It is a plain, slow, single-threaded restatement of the method in double
// precision (with an optional single-precision V-cycle that mirrors the
// mixed-precision mode), written for readability, not speed.  It shares no
// code with the GPU library.
//
// What it follows (paper: "Multi-physics Preconditioning for Thermally
// Activated Batteries"):
//   * block splitting by physics field and the hierarchical block
//     Gauss-Seidel preconditioner: Sec. 3.2, eqs. (block-splitting),
//     (voltage-block), (non-voltage), (hierarchical-bgs-exact-inverse),
//     (non-voltage-bgs), (voltage-bgs).  The sweeps are taken block lower
//     triangular in the listed field order (the paper writes the mirrored,
//     upper form); each leaf block gets one SA-AMG V-cycle.
//   * flexible GMRES (Sec. 3.2, last paragraph) with restart m, classical
//     Gram-Schmidt applied twice, Givens rotations; the stopping test is
//     the relative residual of Sec. 4.1.
//   * smoothed aggregation AMG (Sec. 3.2.1): Galerkin coarse operators
//     (eq. galerkin) with R = P^T, prolongator smoothing of a tentative
//     prolongator, filtering of the matrix used for smoothing with lumping
//     of dropped entries, a diagonal weight equal to the absolute row sum of
//     the filtered matrix, Chebyshev smoothing of degree 2 in pre- and
//     post-position, a direct solve on the coarsest level.
// Where the paper leaves a choice open (strength measure, aggregation
// algorithm, eigenvalue estimate, Chebyshev interval, tentative prolongator
// scaling) the reading used is stated at the function that implements it.
//
// Floating-point conventions: built without contraction; every sum runs
// sequentially in ascending index order, products rounded before adding.
// Setup reductions over long vectors use 256-element chunks summed in order,
// then the chunk sums in order.
//
// Threads (OpenMP, for the CPU baseline timing only): loops whose iterations
// are independent run in parallel -- rows of a sparse product, element-wise
// vector updates, the rows of a dense elimination step, the fields'
// hierarchy setups.  Every reduction (dot products, norms, maxima) and every
// order-dependent step (aggregation, Gustavson products, transposes) stays
// sequential, so results are bitwise the same for any thread count.
#include <algorithm>
#include <omp.h>
#include <functional>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>
#include <vector>

namespace {

template <class T>
struct Csr {
  int n = 0, m = 0;  // rows, cols
  std::vector<int> rp, ci;
  std::vector<T> v;
  int64_t nnz() const { return (int64_t)ci.size(); }
};
using CsrD = Csr<double>;

template <class T, class S>
Csr<T> cast_csr(const Csr<S>& a) {
  Csr<T> b;
  b.n = a.n;
  b.m = a.m;
  b.rp = a.rp;
  b.ci = a.ci;
  b.v.resize(a.v.size());
  for (size_t k = 0; k < a.v.size(); ++k) b.v[k] = (T)a.v[k];
  return b;
}

// plain transpose: row j of the result lists (i, a_ij) in ascending i
template <class T>
Csr<T> transpose(const Csr<T>& a) {
  Csr<T> t;
  t.n = a.m;
  t.m = a.n;
  t.rp.assign(a.m + 1, 0);
  for (int i = 0; i < a.n; ++i)
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) t.rp[a.ci[k] + 1]++;
  for (int j = 0; j < a.m; ++j) t.rp[j + 1] += t.rp[j];
  t.ci.resize(a.ci.size());
  t.v.resize(a.v.size());
  std::vector<int> fill(t.rp.begin(), t.rp.end() - 1);
  for (int i = 0; i < a.n; ++i)
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      int p = fill[a.ci[k]]++;
      t.ci[p] = i;
      t.v[p] = a.v[k];
    }
  return t;
}

uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// ---------------------------------------------------------------- options
}  // namespace

extern "C" {
typedef struct {
  int32_t precision;    // 0: double everywhere; 1: single-precision V-cycle/sweep
  int32_t restart;      // GMRES restart length m
  int32_t max_iters;    // cap on total Arnoldi steps
  double rtol;          // true relative residual target ||b-Ax||/||b||
  int32_t cheb_degree;  // Chebyshev polynomial degree (pre and post)
  double cheb_ratio;    // lambda_min = lambda_max / ratio
  double cheb_boost;    // lambda_max = boost * estimate
  int32_t eig_iters;    // power iterations for eigenvalue estimates
  double sa_damping;    // omega = sa_damping / lambda(D_abs^-1 A_F)
  double omega_override;// >= 0: use this omega instead (tests); < 0: sa_damping / lambda
  int32_t coarse_max;   // stop coarsening at or below this many rows
  int32_t max_levels;   // including the finest level
  uint64_t seed;        // salt for aggregation priorities and start vectors
  double theta[16];     // strength-of-connection threshold per field
  int32_t exact_leaves; // tests: leaf solve = dense LU of the diagonal block
  int32_t block_jacobi; // 1: every coupling dropped (block Jacobi: each field on its own)
  int32_t nested;       // 1: each child of the outermost group is solved by an inner
                        //    flexible GMRES preconditioned by that child's own sweep
  int32_t inner_restart;   // inner GMRES restart length
  int32_t inner_max_iters; // cap on inner Arnoldi steps per solve
  double inner_rtol;       // inner target ||t - A_GG y|| / ||t||
  int32_t field_cheb_degree[16]; // > 0: Chebyshev degree of that field's V-cycle
  int32_t field_leaf[16]; // leaf solver per field: 0 SA-AMG V-cycle, 1 diagonal
                          // (one Jacobi sweep), 2 DD(0)-ILU(0)
  int32_t ilu_block;      // rows per ILU(0) subdomain (contiguous row blocks)
} or_options;
}

namespace {

// ------------------------------------------------------ strength of connection
// Reading of the strength measure (the paper only says the matrix used for
// prolongator smoothing is filtered): the classical smoothed-aggregation
// measure, compared by squares: (i,j) is strong when
//   a_ij * a_ij >= (theta^2 * |a_ii|) * |a_jj|,
// or when the transposed entry (j,i) is strong; diagonal entries excluded.
std::vector<char> strength(const CsrD& a, double theta) {
  std::vector<double> diag(a.n, 0.0);
  for (int i = 0; i < a.n; ++i)
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
      if (a.ci[k] == i) diag[i] = a.v[k];
  double th2 = theta * theta;
  std::vector<char> s(a.ci.size(), 0);
#pragma omp parallel for schedule(static) if (a.n > 4096)
  for (int i = 0; i < a.n; ++i)
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      int j = a.ci[k];
      if (j == i) continue;
      bool st = a.v[k] * a.v[k] >= (th2 * std::fabs(diag[i])) * std::fabs(diag[j]);
      if (!st) {  // transposed entry
        for (int q = a.rp[j]; q < a.rp[j + 1]; ++q)
          if (a.ci[q] == i) {
            st = a.v[q] * a.v[q] >= (th2 * std::fabs(diag[j])) * std::fabs(diag[i]);
            break;
          }
      }
      s[k] = st ? 1 : 0;
    }
  return s;
}

// ------------------------------------------------------------- aggregation
// Reading (the paper does not name its aggregation algorithm): maximal
// distance-2 independent set of the strength graph, chosen greedily in
// decreasing order of a hashed priority key(i) = hash32(i ^ salt) << 32 | i.
// Rows without off-diagonal entries are excluded (aggregate -1).
// Aggregate ids: roots ranked by ascending row index; then (phase 1) every
// row adjacent to a root joins it; (phase 2) every other row joins the
// phase-1 neighbour with the largest key; (phase 3) rows still left become
// singletons numbered after the roots in row order.
uint64_t agg_key(int i, uint64_t salt) {
  uint64_t h = splitmix64((uint64_t)(uint32_t)i ^ salt) >> 32;
  return (h << 32) | (uint64_t)(uint32_t)i;
}

struct AggResult {
  std::vector<int> agg;   // per row, -1 excluded
  std::vector<char> root;
  int nagg = 0;
};

AggResult aggregate(const CsrD& a, const std::vector<char>& strong, uint64_t salt) {
  const int n = a.n;
  AggResult r;
  std::vector<char> excluded(n, 1);
  for (int i = 0; i < n; ++i)
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
      if (a.ci[k] != i) excluded[i] = 0;
  // strong neighbours
  auto for_strong = [&](int i, auto&& fn) {
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
      if (strong[k]) fn(a.ci[k]);
  };
  std::vector<int> order;
  for (int i = 0; i < n; ++i)
    if (!excluded[i]) order.push_back(i);
  std::sort(order.begin(), order.end(),
            [&](int x, int y) { return agg_key(x, salt) > agg_key(y, salt); });
  // 0 undecided, 1 root, 2 within distance 2 of a root
  std::vector<char> state(n, 0);
  for (int v : order) {
    if (state[v] != 0) continue;
    state[v] = 1;
    for_strong(v, [&](int u) {
      if (state[u] == 0) state[u] = 2;
      for_strong(u, [&](int w) {
        if (state[w] == 0) state[w] = 2;
      });
    });
  }
  r.agg.assign(n, -1);
  r.root.assign(n, 0);
  int nroot = 0;
  for (int i = 0; i < n; ++i)
    if (!excluded[i] && state[i] == 1) {
      r.root[i] = 1;
      r.agg[i] = nroot++;
    }
  std::vector<int> phase1(n, -1);
  for (int i = 0; i < n; ++i) {
    if (excluded[i] || r.root[i]) continue;
    for_strong(i, [&](int u) {
      if (r.root[u]) phase1[i] = r.agg[u];
    });
  }
  std::vector<int> agg2(n, -1);
  for (int i = 0; i < n; ++i) {
    if (excluded[i] || r.root[i]) continue;
    if (phase1[i] >= 0) {
      agg2[i] = phase1[i];
      continue;
    }
    uint64_t best = 0;
    int bestagg = -1;
    for_strong(i, [&](int u) {
      if (phase1[u] >= 0 && !r.root[u]) {
        uint64_t ku = agg_key(u, salt);
        if (bestagg < 0 || ku > best) {
          best = ku;
          bestagg = phase1[u];
        }
      }
    });
    agg2[i] = bestagg;
  }
  int next = nroot;
  for (int i = 0; i < n; ++i) {
    if (excluded[i] || r.root[i]) continue;
    r.agg[i] = agg2[i] >= 0 ? agg2[i] : next++;
  }
  r.nagg = next;
  return r;
}

// ----------------------------------------------- filtering, weights, P, RAP
// Filtered matrix: strong off-diagonal entries are kept, every dropped entry
// of a row is added to that row's diagonal (in ascending column order).
// D_abs = absolute row sum of the filtered matrix.
void filter(const CsrD& a, const std::vector<char>& strong, CsrD& af, std::vector<double>& dabs) {
  af.n = a.n;
  af.m = a.m;
  af.rp.assign(a.n + 1, 0);
  af.ci.clear();
  af.v.clear();
  dabs.assign(a.n, 0.0);
  for (int i = 0; i < a.n; ++i) {
    double d = 0.0;
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
      if (a.ci[k] == i) d = a.v[k];
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
      if (a.ci[k] != i && !strong[k]) d += a.v[k];
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      int j = a.ci[k];
      if (j == i) {
        af.ci.push_back(i);
        af.v.push_back(d);
      } else if (strong[k]) {
        af.ci.push_back(j);
        af.v.push_back(a.v[k]);
      }
    }
    af.rp[i + 1] = (int)af.ci.size();
    double s = 0.0;
    for (int k = af.rp[i]; k < af.rp[i + 1]; ++k) s += std::fabs(af.v[k]);
    dabs[i] = s;
  }
}

// Sum of a long vector of products with a fixed association (the paper does
// not say how its eigenvalue estimate sums; this order is part of the
// reading): each run of 256 consecutive terms is summed in order, then the
// run sums are added in order.
double chunked_dot(const std::vector<double>& x, const std::vector<double>& y) {
  double total = 0.0;
  const size_t n = x.size();
  for (size_t c = 0; c < n; c += 256) {
    double s = 0.0;
    for (size_t i = c; i < std::min(n, c + 256); ++i) s += x[i] * y[i];
    total += s;
  }
  return total;
}

// Eigenvalue estimate of D^-1 B (reading: the usual power method with a
// Rayleigh quotient; the paper does not state its estimate): hashed start
// vector in [-1,1], `iters` steps each rescaled by the exact power of two
// that brings max|w| into [0.5,1), then lambda = (w . D^-1 B w) / (w . w).
// A row with d_i = 0 contributes 0 (with the absolute-row-sum weight of the
// filtered matrix, d_i = 0 only where that row of B is zero).
double power_estimate(const CsrD& b, const std::vector<double>& d, int iters, uint64_t salt) {
  const int n = b.n;
  std::vector<double> w(n), y(n);
  for (int i = 0; i < n; ++i)
    w[i] = 2.0 * ((double)(splitmix64((uint64_t)(uint32_t)i ^ salt) >> 11) * 0x1.0p-53) - 1.0;
  auto apply = [&]() {
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = b.rp[i]; k < b.rp[i + 1]; ++k) s += b.v[k] * w[b.ci[k]];
      y[i] = d[i] != 0.0 ? s / d[i] : 0.0;
    }
  };
  for (int it = 0; it < iters; ++it) {
    apply();
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = std::max(mx, std::fabs(y[i]));
    if (mx == 0.0) return 0.0;
    int e;
    std::frexp(mx, &e);
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) w[i] = std::ldexp(y[i], -e);
  }
  apply();
  return chunked_dot(w, y) / chunked_dot(w, w);
}

// Smoothed prolongator P = P_tent - omega D_abs^-1 A_F P_tent with a unit
// tentative prolongator (reading: the piecewise-constant aggregate
// indicator, so the coarse near-nullspace is the constant vector).  The
// pattern is structural: every aggregate met in the row is kept.  A row
// whose absolute row sum is 0 (every off-diagonal entry dropped and the
// lumped diagonal 0, i.e. a zero row of A_F) gets no smoothing term: its
// row of D_abs^-1 A_F is read as 0.
CsrD smooth_prolongator(const CsrD& af, const std::vector<double>& dabs, const std::vector<int>& agg,
                        int nagg, double omega) {
  CsrD p;
  p.n = af.n;
  p.m = nagg;
  p.rp.assign(af.n + 1, 0);
  for (int i = 0; i < af.n; ++i) {
    if (agg[i] >= 0) {
      std::vector<int> cols;
      for (int k = af.rp[i]; k < af.rp[i + 1]; ++k)
        if (agg[af.ci[k]] >= 0) cols.push_back(agg[af.ci[k]]);
      std::sort(cols.begin(), cols.end());
      cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
      double q = dabs[i] != 0.0 ? omega / dabs[i] : 0.0;
      for (int c : cols) {
        double s = 0.0;
        for (int k = af.rp[i]; k < af.rp[i + 1]; ++k)
          if (agg[af.ci[k]] == c) s += af.v[k];
        double t = (agg[i] == c) ? 1.0 : 0.0;
        p.ci.push_back(c);
        p.v.push_back(t - q * s);
      }
    }
    p.rp[i + 1] = (int)p.ci.size();
  }
  return p;
}

// C = A B (Gustavson): each output entry accumulates a_ik b_kj in ascending
// k; the pattern keeps every structurally produced entry.
CsrD spgemm(const CsrD& a, const CsrD& b) {
  CsrD c;
  c.n = a.n;
  c.m = b.m;
  c.rp.assign(a.n + 1, 0);
  std::vector<double> acc(b.m, 0.0);
  std::vector<int> mark(b.m, -1), cols;
  for (int i = 0; i < a.n; ++i) {
    cols.clear();
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      int kk = a.ci[k];
      for (int q = b.rp[kk]; q < b.rp[kk + 1]; ++q) {
        int j = b.ci[q];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += a.v[k] * b.v[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int j : cols) {
      c.ci.push_back(j);
      c.v.push_back(acc[j]);
    }
    c.rp[i + 1] = (int)c.ci.size();
  }
  return c;
}

// ------------------------------------------------------------- dense LU
struct DenseLU {
  int n = 0;
  std::vector<double> lu;  // row-major, L unit lower (below diag), U upper
  std::vector<int> piv;    // row interchanges: step k swapped rows k and piv[k]
};

// partial pivoting: the first row with maximal |a_ik| among i >= k
bool lu_factor(const CsrD& a, DenseLU& f) {
  const int n = a.n;
  f.n = n;
  f.lu.assign((size_t)n * n, 0.0);
  f.piv.assign(n, 0);
  for (int i = 0; i < n; ++i)
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) f.lu[(size_t)i * n + a.ci[k]] = a.v[k];
  double* m = f.lu.data();
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(m[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(m[(size_t)i * n + k]) > best) {
        best = std::fabs(m[(size_t)i * n + k]);
        p = i;
      }
    f.piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(m[(size_t)k * n + j], m[(size_t)p * n + j]);
#pragma omp parallel for schedule(static) if (n - k > 256)
    for (int i = k + 1; i < n; ++i) {
      double l = m[(size_t)i * n + k] / m[(size_t)k * n + k];
      m[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) m[(size_t)i * n + j] -= l * m[(size_t)k * n + j];
    }
  }
  return true;
}

// x = A^-1 b (transpose = 0) or A^-T b (transpose = 1), in double
void lu_solve(const DenseLU& f, const double* b, double* x, int transpose) {
  const int n = f.n;
  const double* m = f.lu.data();
  std::vector<double> y(b, b + n);
  if (!transpose) {
    for (int k = 0; k < n; ++k) std::swap(y[k], y[f.piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) y[i] -= m[(size_t)i * n + j] * y[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) y[i] -= m[(size_t)i * n + j] * y[j];
      y[i] /= m[(size_t)i * n + i];
    }
  } else {  // A = P^T L U  =>  A^T = U^T L^T P
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < i; ++j) y[i] -= m[(size_t)j * n + i] * y[j];
      y[i] /= m[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i)
      for (int j = i + 1; j < n; ++j) y[i] -= m[(size_t)j * n + i] * y[j];
    for (int k = n - 1; k >= 0; --k) std::swap(y[k], y[f.piv[k]]);
  }
  for (int i = 0; i < n; ++i) x[i] = y[i];
}

// ---------------------------------------------------------- AMG hierarchy
struct Level {
  CsrD A, AT, P, R;
  Csr<float> Af, ATf, Pf, Rf;
  std::vector<int> agg;
  std::vector<double> dinv;
  std::vector<float> dinvf;
  double lam_cheb = 0, lam_p = 0, omega = 0;
};

// Coarsest levels up to this many rows are solved by a dense LU.  A
// coarsening that stops above it (it stalls, or hits the level cap) ends in
// a smoothed coarsest level instead: one application of that level's
// Chebyshev polynomial from zero (the paper's coarse solver is a sparse
// direct one, which has no size limit; this reading keeps large strength
// thresholds usable).
constexpr int kDenseCoarseMax = 8000;

struct Amg {
  std::vector<Level> lv;  // lv.back() is the coarsest (direct solve, or smoothed)
  DenseLU lu;
  bool smoothed_coarsest = false;
  double theta = 0;
};

struct Status {
  int code = 0;
  std::string msg;
};
Status g_err;
int g_verbose = 0;  // progress lines on stderr during the system setup

int setup_amg(const CsrD& a0, double theta, const or_options& o, uint64_t salt_base, Amg& h, Status& err) {
  h.theta = theta;
  h.lv.clear();
  h.lv.emplace_back();
  h.lv[0].A = a0;
  for (int l = 0;; ++l) {
    Level& L = h.lv[l];
    bool last = L.A.n <= o.coarse_max || l + 1 >= o.max_levels;
    if (!last) {
      std::vector<char> s = strength(L.A, theta);
      AggResult ag = aggregate(L.A, s, salt_base + (uint64_t)l);
      if (ag.nagg == 0 || ag.nagg > 0.95 * L.A.n) {
        last = true;
      } else {
        CsrD af;
        std::vector<double> dabs;
        filter(L.A, s, af, dabs);
        L.lam_p = power_estimate(af, dabs, o.eig_iters, splitmix64(salt_base + 0x5000 + l));
        if (!(L.lam_p > 0.0)) {
          err = {-5, "non-positive eigenvalue estimate for prolongator smoothing"};
          return -5;
        }
        L.omega = o.omega_override >= 0 ? o.omega_override : o.sa_damping / L.lam_p;
        L.agg = ag.agg;
        L.P = smooth_prolongator(af, dabs, ag.agg, ag.nagg, L.omega);
        L.R = transpose(L.P);
        CsrD ap = spgemm(L.A, L.P);
        CsrD ac = spgemm(L.R, ap);
        h.lv.emplace_back();
        h.lv[l + 1].A = std::move(ac);
      }
    }
    Level& M = h.lv[l];
    if (last && M.A.n <= kDenseCoarseMax) {
      if (!lu_factor(M.A, h.lu)) {
        err = {-4, "singular coarsest-level matrix"};
        return -4;
      }
      break;
    }
    h.smoothed_coarsest = last;
    // Chebyshev data for level l: D = diag(A_l)
    M.dinv.assign(M.A.n, 0.0);
    std::vector<double> d(M.A.n, 0.0);
    for (int i = 0; i < M.A.n; ++i)
      for (int k = M.A.rp[i]; k < M.A.rp[i + 1]; ++k)
        if (M.A.ci[k] == i) d[i] = M.A.v[k];
    for (int i = 0; i < M.A.n; ++i) {
      if (d[i] == 0.0) {
        err = {-1, "zero diagonal entry"};
        return -1;
      }
      M.dinv[i] = 1.0 / d[i];
    }
    M.lam_cheb = power_estimate(M.A, d, o.eig_iters, splitmix64(salt_base + 0x9000 + l));
    if (last) break;  // smoothed coarsest level
  }
  for (auto& L : h.lv) {
    L.AT = transpose(L.A);
    L.Af = cast_csr<float>(L.A);
    L.ATf = cast_csr<float>(L.AT);
    L.Pf = cast_csr<float>(L.P);
    L.Rf = cast_csr<float>(L.R);
    L.dinvf.assign(L.dinv.begin(), L.dinv.end());
  }
  return 0;
}

// ------------------------------------------------------- V-cycle (T = value type)
template <class T>
const Csr<T>& mat(const Level& L, int which, int transpose);
template <>
const Csr<double>& mat<double>(const Level& L, int which, int transpose) {
  if (which == 0) return transpose ? L.AT : L.A;
  return which == 1 ? L.P : L.R;
}
template <>
const Csr<float>& mat<float>(const Level& L, int which, int transpose) {
  if (which == 0) return transpose ? L.ATf : L.Af;
  return which == 1 ? L.Pf : L.Rf;
}
template <class T>
const std::vector<T>& dinv_of(const Level& L);
template <>
const std::vector<double>& dinv_of<double>(const Level& L) { return L.dinv; }
template <>
const std::vector<float>& dinv_of<float>(const Level& L) { return L.dinvf; }

template <class T>
void spmv(const Csr<T>& a, const T* x, T* y) {
#pragma omp parallel for schedule(static) if (a.n > 4096)
  for (int i = 0; i < a.n; ++i) {
    T s = 0;
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) s += a.v[k] * x[a.ci[k]];
    y[i] = s;
  }
}

// Chebyshev smoothing of A x = b in D^-1 A (Saad, Iterative Methods for
// Sparse Linear Systems, Alg. 12.1) on [lmax/ratio, lmax], lmax =
// boost * estimate; `zero` means x starts at 0.
template <class T>
void chebyshev(const Level& L, const or_options& o, int transpose, const T* b, T* x, bool zero) {
  const Csr<T>& A = mat<T>(L, 0, transpose);
  const std::vector<T>& dinv = dinv_of<T>(L);
  const int n = A.n;
  double lmax = o.cheb_boost * L.lam_cheb, lmin = lmax / o.cheb_ratio;
  double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  double sigma = theta / delta, rho = 1.0 / sigma;
  std::vector<T> r(n), d(n), ad(n);
  if (zero) {
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) r[i] = b[i];
  } else {
    spmv(A, x, ad.data());
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) r[i] = b[i] - ad[i];
  }
  T c0 = (T)(1.0 / theta);
#pragma omp parallel for schedule(static) if (n > 4096)
  for (int i = 0; i < n; ++i) {
    d[i] = dinv[i] * r[i] * c0;
    x[i] = zero ? d[i] : x[i] + d[i];
  }
  for (int k = 1; k < o.cheb_degree; ++k) {
    spmv(A, d.data(), ad.data());
    double rho_new = 1.0 / (2.0 * sigma - rho);
    T c1 = (T)(rho_new * rho), c2 = (T)(2.0 * rho_new / delta);
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) {
      r[i] = r[i] - ad[i];
      d[i] = c1 * d[i] + c2 * (dinv[i] * r[i]);
      x[i] = x[i] + d[i];
    }
    rho = rho_new;
  }
}

// One V-cycle B_l b -> x on level l.  The adjoint (transpose = 1) uses
// A_l^T with the same P, R, D, polynomial and coarse factors, which makes it
// the exact transpose of the forward cycle.
template <class T>
void vcycle(const Amg& h, const or_options& o, int l, int transpose, const T* b, T* x) {
  const Level& L = h.lv[l];
  const int n = L.A.n;
  if (l + 1 == (int)h.lv.size() && h.smoothed_coarsest) {
    chebyshev<T>(L, o, transpose, b, x, true);
    return;
  }
  if (l + 1 == (int)h.lv.size()) {
    std::vector<double> bd(b, b + n), xd(n);
    lu_solve(h.lu, bd.data(), xd.data(), transpose);
    for (int i = 0; i < n; ++i) x[i] = (T)xd[i];
    return;
  }
  const Csr<T>& A = mat<T>(L, 0, transpose);
  const Csr<T>& P = mat<T>(L, 1, 0);
  const Csr<T>& R = mat<T>(L, 2, 0);
  chebyshev<T>(L, o, transpose, b, x, true);
  std::vector<T> r(n), ax(n), bc(R.n), xc(R.n), e(n);
  spmv(A, x, ax.data());
#pragma omp parallel for schedule(static) if (n > 4096)
  for (int i = 0; i < n; ++i) r[i] = b[i] - ax[i];
  spmv(R, r.data(), bc.data());
  vcycle<T>(h, o, l + 1, transpose, bc.data(), xc.data());
  spmv(P, xc.data(), e.data());
#pragma omp parallel for schedule(static) if (n > 4096)
  for (int i = 0; i < n; ++i) x[i] = x[i] + e[i];
  chebyshev<T>(L, o, transpose, b, x, false);
}

// ------------------------------------------------------------- other leaves
// DD(0)-ILU(0) (the species-block preconditioner of Sec. 3.2, with the
// domain decomposition of Sec. 3.1 without overlap): the block's rows are
// cut into contiguous subdomains of `ilu_block` rows; entries coupling two
// subdomains are dropped, and each subdomain block gets the incomplete LU
// factorisation with zero fill: L unit lower and U upper on the block's own
// pattern, computed row by row (IKJ order): for row i and each k < i in its
// pattern (ascending), l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for every
// j > k present in both rows i and k.
struct Ilu {
  int sub = 0;          // rows per subdomain
  CsrD F, FT;           // factors (L strictly below, U on and above the diagonal) and their transpose
  Csr<float> Ff, FTf;
  std::vector<int> dpos, dposT;  // position of each row's diagonal in F / FT
};

bool ilu0_setup(const CsrD& a, int sub, Ilu& f) {
  f.sub = sub;
  CsrD& F = f.F;
  F.n = F.m = a.n;
  F.rp.assign(a.n + 1, 0);
  for (int i = 0; i < a.n; ++i) {
    for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
      if (a.ci[k] / sub == i / sub) {
        F.ci.push_back(a.ci[k]);
        F.v.push_back(a.v[k]);
      }
    F.rp[i + 1] = (int)F.ci.size();
  }
  f.dpos.assign(a.n, -1);
  for (int i = 0; i < a.n; ++i)
    for (int k = F.rp[i]; k < F.rp[i + 1]; ++k)
      if (F.ci[k] == i) f.dpos[i] = k;
  for (int i = 0; i < a.n; ++i) {
    if (f.dpos[i] < 0) return false;
    for (int p = F.rp[i]; p < F.rp[i + 1] && F.ci[p] < i; ++p) {
      const int k = F.ci[p];
      const double l = F.v[p] / F.v[f.dpos[k]];
      F.v[p] = l;
      // a_ij -= l * u_kj for j > k in both rows (both sorted by column)
      int q = f.dpos[k] + 1;
      for (int r = p + 1; r < F.rp[i + 1]; ++r) {
        while (q < F.rp[k + 1] && F.ci[q] < F.ci[r]) ++q;
        if (q < F.rp[k + 1] && F.ci[q] == F.ci[r]) F.v[r] = F.v[r] - l * F.v[q];
      }
    }
    if (F.v[f.dpos[i]] == 0.0) return false;
  }
  f.FT = transpose(F);
  f.dposT.assign(a.n, -1);
  for (int i = 0; i < a.n; ++i)
    for (int k = f.FT.rp[i]; k < f.FT.rp[i + 1]; ++k)
      if (f.FT.ci[k] == i) f.dposT[i] = k;
  f.Ff = cast_csr<float>(F);
  f.FTf = cast_csr<float>(f.FT);
  return true;
}

template <class T>
const Csr<T>& ilu_mat(const Ilu& f, int transpose);
template <>
const Csr<double>& ilu_mat<double>(const Ilu& f, int transpose) { return transpose ? f.FT : f.F; }
template <>
const Csr<float>& ilu_mat<float>(const Ilu& f, int transpose) { return transpose ? f.FTf : f.Ff; }

// z = U^-1 L^-1 t (transpose: z = L^-T U^-T t, i.e. the same two sweeps on
// the transposed factors: a lower sweep with U^T, dividing by the diagonal,
// then an upper sweep with L^T, unit diagonal); each sum in ascending column
template <class T>
void ilu0_solve(const Ilu& f, int transpose, const T* t, T* z) {
  const Csr<T>& M = ilu_mat<T>(f, transpose);
  const std::vector<int>& dp = transpose ? f.dposT : f.dpos;
  const int n = M.n;
  std::vector<T> y(n);
  for (int i = 0; i < n; ++i) {  // lower sweep
    T s = t[i];
    for (int k = M.rp[i]; k < dp[i]; ++k) s = s - M.v[k] * y[M.ci[k]];
    y[i] = transpose ? s / M.v[dp[i]] : s;
  }
  for (int i = n - 1; i >= 0; --i) {  // upper sweep
    T s = y[i];
    for (int k = dp[i] + 1; k < M.rp[i + 1]; ++k) s = s - M.v[k] * z[M.ci[k]];
    z[i] = transpose ? s : s / M.v[dp[i]];
  }
}

// ----------------------------------------------------------- system context
struct Node {  // field-group tree node
  int lo = 0, hi = 0;   // row range in the permuted ordering
  int field = -1;       // leaf: field id
  std::vector<int> kids;
};

struct Ctx {
  or_options o;
  int n = 0, nf = 0;
  std::vector<int> perm;   // original row -> permuted row
  std::vector<int> iperm;  // permuted row -> original row
  std::vector<int> f_lo, f_hi;
  CsrD A, Ap, ApT;         // original, permuted, permuted transpose
  Csr<float> Apf, ApTf;
  std::vector<Amg> amg;    // per field
  std::vector<DenseLU> exact;  // per field (exact_leaves)
  std::vector<Node> nodes;     // nodes[0] = root
  std::vector<int> leaf_order;
  std::vector<or_options> fo;  // per-field options (Chebyshev degree)
  std::vector<std::vector<double>> dinv;  // diagonal leaves: 1 / a_ii (double and single)
  std::vector<std::vector<float>> dinvf;
  std::vector<Ilu> ilu;                   // ILU(0) leaves
  std::vector<CsrD> gA, gAT;   // nested form: diagonal block of each child of the root (and transpose)
};

int parse_tree(Ctx& c, const int* tree, int len) {
  c.nodes.clear();
  c.leaf_order.clear();
  std::vector<int> stack;
  std::vector<char> seen(c.nf, 0);
  for (int t = 0; t < len; ++t) {
    int code = tree[t];
    if (code == -1) {
      c.nodes.emplace_back();
      int id = (int)c.nodes.size() - 1;
      if (!stack.empty()) c.nodes[stack.back()].kids.push_back(id);
      stack.push_back(id);
    } else if (code == -2) {
      if (stack.empty()) return -1;
      stack.pop_back();
    } else if (code >= 0 && code < c.nf) {
      if (stack.empty() || seen[code]) return -1;
      seen[code] = 1;
      c.nodes.emplace_back();
      int id = (int)c.nodes.size() - 1;
      c.nodes[id].field = code;
      c.nodes[stack.back()].kids.push_back(id);
      c.leaf_order.push_back(code);
    } else {
      return -1;
    }
  }
  if (!stack.empty() || c.nodes.empty()) return -1;
  for (int f = 0; f < c.nf; ++f)
    if (!seen[f]) return -1;
  return 0;
}

void node_ranges(Ctx& c, int id) {
  Node& nd = c.nodes[id];
  if (nd.field >= 0) {
    nd.lo = c.f_lo[nd.field];
    nd.hi = c.f_hi[nd.field];
    return;
  }
  nd.lo = INT32_MAX;
  nd.hi = 0;
  for (int k : nd.kids) {
    node_ranges(c, k);
    nd.lo = std::min(nd.lo, c.nodes[k].lo);
    nd.hi = std::max(nd.hi, c.nodes[k].hi);
  }
}

CsrD block(const CsrD& ap, int lo, int hi) {  // diagonal block rows/cols [lo,hi)
  CsrD b;
  b.n = b.m = hi - lo;
  b.rp.assign(b.n + 1, 0);
  for (int i = lo; i < hi; ++i) {
    for (int k = ap.rp[i]; k < ap.rp[i + 1]; ++k)
      if (ap.ci[k] >= lo && ap.ci[k] < hi) {
        b.ci.push_back(ap.ci[k] - lo);
        b.v.push_back(ap.v[k]);
      }
    b.rp[i - lo + 1] = (int)b.ci.size();
  }
  return b;
}

// Leaf solve: one V-cycle (or the exact block solve in the test mode).
template <class T>
void leaf_solve(const Ctx& c, int f, int transpose, const T* t, T* z) {
  int n = c.f_hi[f] - c.f_lo[f];
  if (c.o.exact_leaves) {
    std::vector<double> td(t, t + n), zd(n);
    lu_solve(c.exact[f], td.data(), zd.data(), transpose);
    for (int i = 0; i < n; ++i) z[i] = (T)zd[i];
    return;
  }
  const int leaf = c.o.field_leaf[f];
  if (leaf == 1) {  // one Jacobi sweep from zero: exact for a diagonal block
    for (int i = 0; i < n; ++i) z[i] = std::is_same<T, float>::value ? t[i] * (T)c.dinvf[f][i] : t[i] * (T)c.dinv[f][i];
    return;
  }
  if (leaf == 2) {
    ilu0_solve<T>(c.ilu[f], transpose, t, z);
    return;
  }
  vcycle<T>(c.amg[f], c.fo[f], 0, transpose, t, z);
}

template <class T>
const Csr<T>& perm_mat(const Ctx& c, int transpose);
template <>
const Csr<double>& perm_mat<double>(const Ctx& c, int transpose) { return transpose ? c.ApT : c.Ap; }
template <>
const Csr<float>& perm_mat<float>(const Ctx& c, int transpose) { return transpose ? c.ApTf : c.Apf; }

// Hierarchical block Gauss-Seidel, forward form: the children of a group are
// visited in order; child k receives its part of the group's right-hand side
// minus the couplings to the children already solved, each term subtracted
// in ascending column order.  The transposed form visits the children in
// reverse order with the couplings of A^T to the children after it.
template <class T>
void bgs_node(const Ctx& c, int id, int transpose, const T* r, T* z) {
  const Node& nd = c.nodes[id];
  if (nd.field >= 0) {
    leaf_solve<T>(c, nd.field, transpose, r + nd.lo, z + nd.lo);
    return;
  }
  const Csr<T>& A = perm_mat<T>(c, transpose);
  const int nk = (int)nd.kids.size();
  for (int q = 0; q < nk; ++q) {
    const Node& ch = c.nodes[nd.kids[transpose ? nk - 1 - q : q]];
    int clo, chi;  // columns already solved within this group
    if (!transpose) {
      clo = nd.lo;
      chi = ch.lo;
    } else {
      clo = ch.hi;
      chi = nd.hi;
    }
    std::vector<T> t(c.n, (T)0);
#pragma omp parallel for schedule(static) if (ch.hi - ch.lo > 4096)
    for (int i = ch.lo; i < ch.hi; ++i) {
      T s = r[i];
      if (!c.o.block_jacobi)
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
          if (A.ci[k] >= clo && A.ci[k] < chi) s = s - A.v[k] * z[A.ci[k]];
      t[i] = s;
    }
    int cid = nd.kids[transpose ? nk - 1 - q : q];
    bgs_node<T>(c, cid, transpose, t.data(), z);
  }
}

// z = sweep of node `id` applied to r, in T precision (vectors of length n
// in the permuted ordering; only the node's rows are read and written)
void node_sweep(const Ctx& c, int id, int transpose, const double* r, double* z) {
  if (c.o.precision == 1) {
    std::vector<float> rf(c.n, 0.0f), zf(c.n, 0.0f);
#pragma omp parallel for schedule(static) if (c.n > 4096)
    for (int i = 0; i < c.n; ++i) rf[i] = (float)r[i];
    bgs_node<float>(c, id, transpose, rf.data(), zf.data());
#pragma omp parallel for schedule(static) if (c.n > 4096)
    for (int i = 0; i < c.n; ++i) z[i] = (double)zf[i];
  } else {
    std::vector<double> zz(c.n, 0.0);
    bgs_node<double>(c, id, transpose, r, zz.data());
    for (int i = 0; i < c.n; ++i) z[i] = zz[i];
  }
}

double dot(const std::vector<double>& x, const std::vector<double>& y) {
  double s = 0.0;
  for (size_t i = 0; i < x.size(); ++i) s += x[i] * y[i];
  return s;
}

// Flexible right-preconditioned GMRES(m) for A x = b (x holds the start):
// z_j = M(v_j) is stored, so M may change from step to step (Sec. 3.2, last
// paragraph).  Classical Gram-Schmidt applied twice; Givens rotations; the
// residual estimate |g_{j+1}| / ||b|| is checked after every step and the
// true residual at the end of every cycle.  Returns 0 converged, 1 cap hit.
int fgmres(const CsrD& A, int m, double rtol, int max_iters, const std::function<void(const double*, double*)>& M,
           const std::vector<double>& b, std::vector<double>& x, int* iters, double* hist, int cap, int* hlen) {
  const int n = A.n;
  *iters = 0;
  *hlen = 0;
  auto push = [&](double v) {
    if (hist && *hlen < cap) hist[*hlen] = v;
    (*hlen)++;
  };
  double bnorm = std::sqrt(dot(b, b));
  if (bnorm == 0.0) {
    std::fill(x.begin(), x.end(), 0.0);
    push(0.0);
    return 0;
  }
  std::vector<double> r(n), ax(n);
  auto true_resid = [&]() {
    spmv(A, x.data(), ax.data());
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) r[i] = b[i] - ax[i];
    return std::sqrt(dot(r, r));
  };
  double beta = true_resid();
  push(beta / bnorm);
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(n)), Z(m, std::vector<double>(n));
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), w(n), h1(m + 1), h2(m + 1);
  auto Hs = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  for (;;) {
    if (beta / bnorm <= rtol) return 0;
    if (*iters >= max_iters) return 1;
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i) V[0][i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      M(V[j].data(), Z[j].data());
      spmv(A, Z[j].data(), w.data());
      double w0 = std::sqrt(dot(w, w));
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<double>& hh = pass == 0 ? h1 : h2;
        for (int k = 0; k <= j; ++k) hh[k] = dot(V[k], w);
        // w -= V hh, each element in ascending k
#pragma omp parallel for schedule(static) if (n > 4096)
        for (int i = 0; i < n; ++i)
          for (int k = 0; k <= j; ++k) w[i] -= hh[k] * V[k][i];
      }
      for (int k = 0; k <= j; ++k) Hs(k, j) = h1[k] + h2[k];
      double hn = std::sqrt(dot(w, w));
      Hs(j + 1, j) = hn;
      if (hn > 0.0) {
#pragma omp parallel for schedule(static) if (n > 4096)
        for (int i = 0; i < n; ++i) V[j + 1][i] = w[i] / hn;
      }
      for (int k = 0; k < j; ++k) {
        double t1 = cs[k] * Hs(k, j) + sn[k] * Hs(k + 1, j);
        double t2 = -sn[k] * Hs(k, j) + cs[k] * Hs(k + 1, j);
        Hs(k, j) = t1;
        Hs(k + 1, j) = t2;
      }
      double a = Hs(j, j), bb = Hs(j + 1, j);
      double den = std::sqrt(a * a + bb * bb);
      cs[j] = a / den;
      sn[j] = bb / den;
      Hs(j, j) = den;
      Hs(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      (*iters)++;
      double est = std::fabs(g[j + 1]) / bnorm;
      push(est);
      jend = j + 1;
      if (est <= rtol || hn <= 1e-14 * w0 || *iters >= max_iters) break;
    }
    std::vector<double> y(jend);
    for (int i = jend - 1; i >= 0; --i) {
      double s = g[i];
      for (int k = i + 1; k < jend; ++k) s -= Hs(i, k) * y[k];
      y[i] = s / Hs(i, i);
    }
    // x += Z y, each element in ascending k
#pragma omp parallel for schedule(static) if (n > 4096)
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < jend; ++k) x[i] += y[k] * Z[k][i];
    beta = true_resid();
    if (hist && *hlen - 1 < cap) hist[*hlen - 1] = beta / bnorm;
  }
}

// Nested form (Sec. 3.2: the blocks of the outermost sweep are inverted by
// an inner GMRES(30) to a 1e-6 relative residual, preconditioned by their
// own block Gauss-Seidel sweeps): the children of the root are visited as in
// the sweep, child q receiving its right-hand side minus the couplings to
// the children already solved, and its block is solved by an inner flexible
// GMRES from a zero start, preconditioned by the child's sweep.  In the
// mixed mode each child's result is rounded to single precision, as the
// stored Krylov direction is.
void nested_precond(const Ctx& c, int transpose, const double* r, double* z) {
  const Node& root = c.nodes[0];
  const CsrD& A = transpose ? c.ApT : c.Ap;
  const int nk = (int)root.kids.size();
  std::fill(z, z + c.n, 0.0);
  for (int q = 0; q < nk; ++q) {
    const int kq = transpose ? nk - 1 - q : q;
    const int cid = root.kids[kq];
    const Node& ch = c.nodes[cid];
    const int clo = transpose ? ch.hi : root.lo, chi = transpose ? root.hi : ch.lo;
    const int m = ch.hi - ch.lo;
    std::vector<double> t(m), y(m, 0.0);
    for (int i = ch.lo; i < ch.hi; ++i) {
      double s = r[i];
      if (!c.o.block_jacobi)
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
          if (A.ci[k] >= clo && A.ci[k] < chi) s = s - A.v[k] * z[A.ci[k]];
      t[i - ch.lo] = s;
    }
    auto M = [&](const double* v, double* out) {
      std::vector<double> vf(c.n, 0.0), zf(c.n, 0.0);
      std::copy(v, v + m, vf.begin() + ch.lo);
      node_sweep(c, cid, transpose, vf.data(), zf.data());
      std::copy(zf.begin() + ch.lo, zf.begin() + ch.hi, out);
    };
    int it = 0, hl = 0;
    fgmres(transpose ? c.gAT[kq] : c.gA[kq], c.o.inner_restart, c.o.inner_rtol, c.o.inner_max_iters, M, t, y, &it,
           nullptr, 0, &hl);
    for (int i = 0; i < m; ++i) z[ch.lo + i] = c.o.precision == 1 ? (double)(float)y[i] : y[i];
  }
}

// z = M^-1 r in permuted ordering (result in double)
void precond(const Ctx& c, int transpose, const double* r, double* z) {
  if (c.o.nested)
    nested_precond(c, transpose, r, z);
  else
    node_sweep(c, 0, transpose, r, z);
}

// the outer solve: flexible GMRES on the permuted system
int gmres(const Ctx& c, int transpose, const std::vector<double>& b, std::vector<double>& x, int* iters,
          double* hist, int cap, int* hlen) {
  auto M = [&](const double* v, double* out) { precond(c, transpose, v, out); };
  return fgmres(transpose ? c.ApT : c.Ap, c.o.restart, c.o.rtol, c.o.max_iters, M, b, x, iters, hist, cap, hlen);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

typedef struct Ctx or_ctx;
typedef struct Amg or_amg;

void or_default_options(or_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = 0;
  o->restart = 50;
  o->max_iters = 2000;
  o->rtol = 1e-8;
  o->cheb_degree = 2;
  o->cheb_ratio = 30.0;
  o->cheb_boost = 1.1;
  o->eig_iters = 10;
  o->sa_damping = 4.0 / 3.0;
  o->omega_override = -1.0;
  o->coarse_max = 2000;
  o->max_levels = 10;
  o->seed = 0x2602ull;
  for (int f = 0; f < 16; ++f) o->theta[f] = 0.0;
  o->theta[0] = 0.04;
  o->exact_leaves = 0;
  o->block_jacobi = 0;
  o->nested = 0;
  o->inner_restart = 30;
  o->inner_max_iters = 300;
  o->inner_rtol = 1e-6;
  for (int f = 0; f < 16; ++f) o->field_cheb_degree[f] = 0;
  for (int f = 0; f < 16; ++f) o->field_leaf[f] = 0;
  o->ilu_block = 4096;
}

const char* or_last_error(void) { return g_err.msg.c_str(); }
// threads of the parallel loops (results do not depend on it)
void or_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int or_get_threads(void) { return omp_get_max_threads(); }
void or_set_verbose(int on) { g_verbose = on; }

static CsrD make_csr(int n, int m, const int* rp, const int* ci, const double* v) {
  CsrD a;
  a.n = n;
  a.m = m;
  a.rp.assign(rp, rp + n + 1);
  a.ci.assign(ci + rp[0], ci + rp[n]);
  a.v.assign(v + rp[0], v + rp[n]);
  return a;
}

// salt of field f's hierarchy
static uint64_t field_salt(uint64_t seed, int f) { return splitmix64(seed + 0x1000ull * (uint64_t)(f + 1)); }

// ---- single-block AMG (pins)
or_amg* or_amg_setup(int n, const int* rp, const int* ci, const double* v, double theta,
                     const or_options* o, uint64_t salt) {
  Amg* h = new Amg();
  CsrD a = make_csr(n, n, rp, ci, v);
  if (setup_amg(a, theta, *o, salt, *h, g_err) != 0) {
    delete h;
    return nullptr;
  }
  return h;
}
void or_amg_destroy(or_amg* h) { delete h; }
int or_amg_levels(const or_amg* h) { return (int)h->lv.size(); }
int or_amg_smoothed_coarsest(const or_amg* h) { return h->smoothed_coarsest ? 1 : 0; }
// which: 0 A, 1 P, 2 R, 3 A^T.  Returns nnz; fills when pointers non-null.
int64_t or_amg_get(const or_amg* h, int l, int which, int* nrows, int* ncols, int* rp, int* ci, double* v) {
  const Level& L = h->lv[l];
  const CsrD& a = which == 0 ? L.A : which == 1 ? L.P : which == 2 ? L.R : L.AT;
  if (nrows) *nrows = a.n;
  if (ncols) *ncols = a.m;
  if (rp) std::copy(a.rp.begin(), a.rp.end(), rp);
  if (ci) std::copy(a.ci.begin(), a.ci.end(), ci);
  if (v) std::copy(a.v.begin(), a.v.end(), v);
  return a.nnz();
}
void or_amg_agg(const or_amg* h, int l, int* agg) { std::copy(h->lv[l].agg.begin(), h->lv[l].agg.end(), agg); }
void or_amg_scalars(const or_amg* h, int l, double* out3) {
  out3[0] = h->lv[l].lam_cheb;
  out3[1] = h->lv[l].lam_p;
  out3[2] = h->lv[l].omega;
}
void or_amg_vcycle(const or_amg* h, const or_options* o, int transpose, int precision, const double* b,
                   double* x) {
  int n = h->lv[0].A.n;
  if (precision == 1) {
    std::vector<float> bf(b, b + n), xf(n);
    vcycle<float>(*h, *o, 0, transpose, bf.data(), xf.data());
    for (int i = 0; i < n; ++i) x[i] = xf[i];
  } else {
    vcycle<double>(*h, *o, 0, transpose, b, x);
  }
}
void or_amg_chebyshev(const or_amg* h, const or_options* o, int l, const double* b, double* x, int zero) {
  int n = h->lv[l].A.n;
  std::vector<double> xx(x, x + n);
  chebyshev<double>(h->lv[l], *o, 0, b, xx.data(), zero != 0);
  std::copy(xx.begin(), xx.end(), x);
}

// ---- building blocks (pins)
void or_strength(int n, const int* rp, const int* ci, const double* v, double theta, char* strong) {
  CsrD a = make_csr(n, n, rp, ci, v);
  std::vector<char> s = strength(a, theta);
  std::copy(s.begin(), s.end(), strong);
}
int or_aggregate(int n, const int* rp, const int* ci, const double* v, const char* strong, uint64_t salt,
                 int* agg, char* root) {
  CsrD a = make_csr(n, n, rp, ci, v);
  std::vector<char> s(strong, strong + a.nnz());
  AggResult r = aggregate(a, s, salt);
  std::copy(r.agg.begin(), r.agg.end(), agg);
  std::copy(r.root.begin(), r.root.end(), root);
  return r.nagg;
}
uint64_t or_agg_key(int i, uint64_t salt) { return agg_key(i, salt); }
double or_power_estimate(int n, const int* rp, const int* ci, const double* v, const double* d, int iters,
                         uint64_t salt) {
  CsrD a = make_csr(n, n, rp, ci, v);
  std::vector<double> dd(d, d + n);
  return power_estimate(a, dd, iters, salt);
}
void or_filter(int n, const int* rp, const int* ci, const double* v, const char* strong, int* frp, int* fci,
               double* fv, double* dabs) {
  CsrD a = make_csr(n, n, rp, ci, v), af;
  std::vector<char> s(strong, strong + a.nnz());
  std::vector<double> d;
  filter(a, s, af, d);
  std::copy(af.rp.begin(), af.rp.end(), frp);
  std::copy(af.ci.begin(), af.ci.end(), fci);
  std::copy(af.v.begin(), af.v.end(), fv);
  std::copy(d.begin(), d.end(), dabs);
}
// C = A B; returns nnz(C); fills when pointers are non-null (call twice)
int64_t or_spgemm(int n, int k, int m, const int* arp, const int* aci, const double* av, const int* brp,
                  const int* bci, const double* bv, int* crp, int* cci, double* cv) {
  CsrD a = make_csr(n, k, arp, aci, av), b = make_csr(k, m, brp, bci, bv);
  CsrD c = spgemm(a, b);
  if (crp) std::copy(c.rp.begin(), c.rp.end(), crp);
  if (cci) std::copy(c.ci.begin(), c.ci.end(), cci);
  if (cv) std::copy(c.v.begin(), c.v.end(), cv);
  return c.nnz();
}
int or_lu_solve(int n, const int* rp, const int* ci, const double* v, const double* b, double* x, int transpose) {
  CsrD a = make_csr(n, n, rp, ci, v);
  DenseLU f;
  if (!lu_factor(a, f)) return -4;
  lu_solve(f, b, x, transpose);
  return 0;
}

// ---- full system
or_ctx* or_setup(int n, const int* rp, const int* ci, const double* v, int nf, const int* field_of_row,
                 int tree_len, const int* tree, const or_options* o) {
  Ctx* c = new Ctx();
  c->o = *o;
  c->n = n;
  c->nf = nf;
  c->A = make_csr(n, n, rp, ci, v);
  if (parse_tree(*c, tree, tree_len) != 0) {
    g_err = {-1, "invalid field-group tree"};
    delete c;
    return nullptr;
  }
  // permutation: fields in depth-first leaf order, rows in original order within a field
  std::vector<int> pos(nf);
  for (int q = 0; q < nf; ++q) pos[c->leaf_order[q]] = q;
  std::vector<int> count(nf, 0);
  for (int i = 0; i < n; ++i) {
    if (field_of_row[i] < 0 || field_of_row[i] >= nf) {
      g_err = {-1, "field id out of range"};
      delete c;
      return nullptr;
    }
    count[field_of_row[i]]++;
  }
  c->f_lo.assign(nf, 0);
  c->f_hi.assign(nf, 0);
  int off = 0;
  for (int q = 0; q < nf; ++q) {
    int f = c->leaf_order[q];
    c->f_lo[f] = off;
    off += count[f];
    c->f_hi[f] = off;
  }
  c->perm.assign(n, 0);
  c->iperm.assign(n, 0);
  std::vector<int> fill(c->f_lo);
  for (int i = 0; i < n; ++i) {
    int p = fill[field_of_row[i]]++;
    c->perm[i] = p;
    c->iperm[p] = i;
  }
  CsrD& ap = c->Ap;
  ap.n = ap.m = n;
  ap.rp.assign(n + 1, 0);
  for (int p = 0; p < n; ++p) {
    int i = c->iperm[p];
    std::vector<std::pair<int, double>> row;
    for (int k = c->A.rp[i]; k < c->A.rp[i + 1]; ++k) row.push_back({c->perm[c->A.ci[k]], c->A.v[k]});
    std::sort(row.begin(), row.end(),
              [](const std::pair<int, double>& x, const std::pair<int, double>& y) { return x.first < y.first; });
    for (auto& e : row) {
      ap.ci.push_back(e.first);
      ap.v.push_back(e.second);
    }
    ap.rp[p + 1] = (int)ap.ci.size();
  }
  c->ApT = transpose(ap);
  c->Apf = cast_csr<float>(ap);
  c->ApTf = cast_csr<float>(c->ApT);
  node_ranges(*c, 0);
  if (o->inner_restart < 1 || o->inner_restart > 64 || o->inner_max_iters < 0 || !(o->inner_rtol >= 0.0)) {
    g_err = {-1, "invalid inner solver options"};
    delete c;
    return nullptr;
  }
  c->fo.assign(nf, *o);
  for (int f = 0; f < nf && f < 16; ++f)
    if (o->field_cheb_degree[f] > 0) c->fo[f].cheb_degree = o->field_cheb_degree[f];
  if (o->nested)
    for (int k : c->nodes[0].kids) {
      c->gA.push_back(block(ap, c->nodes[k].lo, c->nodes[k].hi));
      c->gAT.push_back(block(c->ApT, c->nodes[k].lo, c->nodes[k].hi));
    }
  c->amg.resize(nf);
  c->exact.resize(nf);
  c->ilu.resize(nf);
  c->dinv.resize(nf);
  c->dinvf.resize(nf);
  for (int f = 0; f < nf; ++f)
    if (o->field_leaf[f] < 0 || o->field_leaf[f] > 2 || o->ilu_block < 1) {
      g_err = {-1, "invalid leaf solver options"};
      delete c;
      return nullptr;
    }
  // the fields' leaf setups are independent: one field per thread
  std::vector<Status> st(nf);
  if (g_verbose) std::fprintf(stderr, "oracle: %d rows permuted; building %d field blocks\n", n, nf);
#pragma omp parallel for schedule(dynamic, 1)
  for (int f = 0; f < nf; ++f) {
    const double t0 = omp_get_wtime();
    CsrD blk = block(ap, c->f_lo[f], c->f_hi[f]);
    c->dinv[f].assign(blk.n, 0.0);
    c->dinvf[f].assign(blk.n, 0.0f);
    if (o->exact_leaves) {
      if (!lu_factor(blk, c->exact[f])) st[f] = {-4, "singular diagonal block"};
    } else if (o->field_leaf[f] == 1) {
      std::vector<double> d(blk.n, 0.0);
      for (int i = 0; i < blk.n; ++i)
        for (int k = blk.rp[i]; k < blk.rp[i + 1]; ++k)
          if (blk.ci[k] == i) d[i] = blk.v[k];
      for (int i = 0; i < blk.n; ++i) {
        if (d[i] == 0.0) {
          st[f] = {-1, "zero diagonal entry"};
          break;
        }
        c->dinv[f][i] = 1.0 / d[i];
        c->dinvf[f][i] = (float)c->dinv[f][i];
      }
    } else if (o->field_leaf[f] == 2) {
      if (!ilu0_setup(blk, o->ilu_block, c->ilu[f])) st[f] = {-4, "zero pivot in the incomplete factorisation"};
    } else {
      setup_amg(blk, o->theta[f], c->fo[f], field_salt(o->seed, f), c->amg[f], st[f]);
    }
    if (g_verbose)
      std::fprintf(stderr, "oracle: field %d (%d rows) set up in %.1f s\n", f, blk.n, omp_get_wtime() - t0);
  }
  for (int f = 0; f < nf; ++f)
    if (st[f].code != 0) {
      g_err = st[f];
      delete c;
      return nullptr;
    }
  return c;
}

void or_destroy(or_ctx* c) { delete c; }
// precision mode of later applies and solves (the hierarchy does not depend on it)
void or_set_precision(or_ctx* c, int precision) { c->o.precision = precision; }

int or_levels(const or_ctx* c, int f) { return (int)c->amg[f].lv.size(); }
const or_amg* or_field_amg(const or_ctx* c, int f) { return &c->amg[f]; }

// z = M^-1 r (or M^-T r), vectors in the original ordering
void or_apply(const or_ctx* c, const double* r, double* z, int transpose) {
  std::vector<double> rp(c->n), zp(c->n);
#pragma omp parallel for schedule(static) if (c->n > 4096)
  for (int i = 0; i < c->n; ++i) rp[c->perm[i]] = r[i];
  precond(*c, transpose, rp.data(), zp.data());
#pragma omp parallel for schedule(static) if (c->n > 4096)
  for (int i = 0; i < c->n; ++i) z[i] = zp[c->perm[i]];
}

// flat block lower (upper for transpose) Gauss-Seidel sweep over the leaves
// in depth-first order; equals the tree sweep for single sweeps (tests)
void or_apply_flat(const or_ctx* c, const double* r, double* z, int transpose) {
  std::vector<double> rp(c->n), zp(c->n, 0.0);
  for (int i = 0; i < c->n; ++i) rp[c->perm[i]] = r[i];
  const CsrD& A = transpose ? c->ApT : c->Ap;
  int nl = (int)c->leaf_order.size();
  for (int q = 0; q < nl; ++q) {
    int f = c->leaf_order[transpose ? nl - 1 - q : q];
    int lo = c->f_lo[f], hi = c->f_hi[f];
    std::vector<double> t(hi - lo);
    for (int i = lo; i < hi; ++i) {
      double s = rp[i];
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        int j = A.ci[k];
        if (transpose ? j >= hi : j < lo) s = s - A.v[k] * zp[j];
      }
      t[i - lo] = s;
    }
    leaf_solve<double>(*c, f, transpose, t.data(), zp.data() + lo);
  }
  for (int i = 0; i < c->n; ++i) z[i] = zp[c->perm[i]];
}

int or_solve(const or_ctx* c, const double* b, double* x, int use_x0, int transpose, int* iters, double* hist,
             int hist_cap, int* hist_len) {
  std::vector<double> bp(c->n), xp(c->n, 0.0);
  for (int i = 0; i < c->n; ++i) bp[c->perm[i]] = b[i];
  if (use_x0)
    for (int i = 0; i < c->n; ++i) xp[c->perm[i]] = x[i];
  int rc = gmres(*c, transpose, bp, xp, iters, hist, hist_cap, hist_len);
  for (int i = 0; i < c->n; ++i) x[i] = xp[c->perm[i]];
  return rc;
}

// grad_val[p] = -lambda[row(p)] * x[col(p)] on A's pattern (original ordering)
void or_grad_values(const or_ctx* c, const double* lambda, const double* x, double* grad) {
  for (int i = 0; i < c->n; ++i)
    for (int k = c->A.rp[i]; k < c->A.rp[i + 1]; ++k) grad[k] = -lambda[i] * x[c->A.ci[k]];
}

void or_permutation(const or_ctx* c, int* perm) { std::copy(c->perm.begin(), c->perm.end(), perm); }

}  // extern "C"
