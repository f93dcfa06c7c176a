/*
 * hbgs: block Gauss-Seidel / smoothed-aggregation AMG preconditioned
 * flexible GMRES on one AMD MI355X (gfx950).
 *
 * The operation (paper "Multi-physics Preconditioning for Thermally
 * Activated Batteries"): solve the monolithic multiphysics system A x = b of
 * eq. (block-splitting) with restarted flexible GMRES (Sec. 3.2, last
 * paragraph), right-preconditioned by one hierarchical block Gauss-Seidel
 * sweep over the physics field blocks (eqs. hierarchical-bgs-exact-inverse,
 * non-voltage-bgs, voltage-bgs; taken block lower triangular in the listed
 * field order), where each diagonal block is approximated by one
 * smoothed-aggregation AMG V-cycle (Sec. 3.2.1, eq. galerkin: degree-2
 * Chebyshev pre/post smoothing, filtered prolongator smoothing with an
 * absolute-row-sum weight, direct coarsest solve).  The stopping test is the
 * true relative residual ||b - A x|| / ||b|| (Sec. 4.1).
 *
 * Conventions for every call:
 *   - Matrices and vectors passed in are DEVICE pointers owned by the
 *     caller; the library copies what it keeps, so inputs may be freed after
 *     the call returns.  Arrays documented as "host" are host pointers.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it; calls that return host-side results (iteration
 *     counts, histories, statistics) synchronise it first.
 *   - CSR: rowptr[n+1], col[nnz] (int32, strictly increasing within each
 *     row, every row holds its diagonal), val[nnz] (double).  Rows/columns
 *     are in the caller's ordering; vectors use the same ordering.
 *   - Errors are negative status codes; hbgs_last_error() describes the
 *     last failure of the calling thread.  Non-convergence is not an error.
 *   - Calls on one context must not overlap (a context owns its workspace).
 */
#ifndef HBGS_H
#define HBGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbgs_ctx hbgs_ctx;

typedef enum {
  HBGS_OK = 0,
  HBGS_NOT_CONVERGED = 1, /* iteration cap hit; x holds the last iterate */
  HBGS_EINVAL = -1,       /* malformed input (CSR, field map, tree, options) */
  HBGS_ENOMEM = -2,       /* device allocation failed */
  HBGS_EHIP = -3,         /* HIP runtime error */
  HBGS_ESINGULAR = -4,    /* zero pivot in the coarsest-level factorisation */
  HBGS_ESETUP = -5        /* hierarchy could not be built (e.g. a non-positive eigenvalue
                             estimate, an overflowing product table) */
} hbgs_status;

#define HBGS_MAX_FIELDS 16
#define HBGS_MAX_LEVELS 16

typedef struct {
  int32_t precision;     /* 0: FP64 throughout; 1: mixed (FP32 V-cycles, couplings and
                            Krylov directions Z inside FP64 GMRES) */
  int32_t restart;       /* GMRES restart length m (default 50) */
  int32_t max_iters;     /* cap on total Arnoldi steps (default 2000) */
  double rtol;           /* target of ||b - A x|| / ||b|| (default 1e-8) */
  int32_t cheb_degree;   /* Chebyshev degree, pre and post (default 2) */
  double cheb_ratio;     /* lambda_min = lambda_max / ratio (default 30) */
  double cheb_boost;     /* lambda_max = boost * power estimate (default 1.1) */
  int32_t eig_iters;     /* power iterations per eigenvalue estimate (default 10) */
  double sa_damping;     /* omega = sa_damping / lambda(D_abs^-1 A_F) (default 4/3) */
  int32_t coarse_max;    /* coarsen until a level has at most this many rows (2000); the
                            coarsest level is solved with a dense inverse when it has at
                            most 8000 rows, and smoothed (one Chebyshev application from
                            zero) when coarsening stops above that (it stalls beyond 0.95
                            of the rows, or reaches max_levels) */
  int32_t max_levels;    /* levels per field, including the finest (default 10) */
  uint64_t seed;         /* salt of the aggregation priorities and start vectors */
  double theta[HBGS_MAX_FIELDS]; /* strength threshold per field (default 0.04 for
                                    field 0, 0 otherwise) */
  int32_t use_graphs;    /* 1: replay each GMRES iteration as a HIP graph captured on
                            its first use (per precision, direction and step; bitwise
                            the eager result; not used by the nested form or while
                            kernel timing is on).  A value update drops the graphs.
                            0 (default): launch kernels one by one */
  int32_t setup_concurrent; /* 1 (default): the fields' blocks and hierarchies are
                               built concurrently by one host thread per hardware
                               queue of the process (HIP's GPU_MAX_HW_QUEUES, 4 when
                               unset), each on its own stream (the first on the
                               caller's) taking the next unbuilt field; the results
                               do not depend on it.  0: one after another on the
                               caller's stream */
  int32_t block_jacobi;  /* 1: every coupling block is dropped, each field is solved on
                            its own (block Jacobi; all fields run concurrently); 0
                            (default): block Gauss-Seidel */
  int32_t nested;        /* 1: nested form of Sec. 3.2 -- each child of the outermost
                            group (e.g. the voltage and the non-voltage block) is solved
                            by an inner flexible GMRES preconditioned by that child's own
                            sweep, from a zero start; 0 (default): one sweep */
  int32_t inner_restart;   /* inner GMRES restart length, 1..64 (default 30) */
  int32_t inner_max_iters; /* cap on inner Arnoldi steps per inner solve (default 300) */
  double inner_rtol;       /* inner stopping test ||t - A_GG y|| / ||t|| (default 1e-6) */
  int32_t field_cheb_degree[HBGS_MAX_FIELDS]; /* > 0: Chebyshev degree of that field's
                            V-cycle (e.g. 4 on the voltage leaves, Sec. 4); 0: cheb_degree */
  int32_t field_leaf[HBGS_MAX_FIELDS]; /* leaf solver of each field's diagonal block:
                            0 (default) one SA-AMG V-cycle; 1 one Jacobi sweep z = D^-1 t
                            (exact for a diagonal block, e.g. the solid-species ODEs of
                            Sec. 3.2); 2 DD(0)-ILU(0): contiguous subdomains of ilu_block
                            rows without overlap, incomplete LU with zero fill in each
                            (the species-block choice of Sec. 3.2) */
  int32_t ilu_block;     /* rows per ILU(0) subdomain (default 4096) */
  int32_t build_transpose; /* 1 (default): the adjoint's operators (A_l^T on every level,
                              the transposed couplings and outer operator values, the
                              coarsest inverse transposed, transposed ILU factors) are
                              built with the hierarchy; 0: on the first transpose apply
                              or solve after each setup or value update, so forward-only
                              callers skip that work */
} hbgs_options;

typedef struct {
  int32_t n, n_fields;
  int64_t nnz;
  int32_t levels[HBGS_MAX_FIELDS];                   /* hierarchy depth per field */
  int32_t rows[HBGS_MAX_FIELDS][HBGS_MAX_LEVELS];    /* rows per level */
  int64_t nnz_a[HBGS_MAX_FIELDS][HBGS_MAX_LEVELS];   /* nnz(A_l) per level */
  int64_t nnz_p[HBGS_MAX_FIELDS][HBGS_MAX_LEVELS];   /* nnz(P_l) per level */
  double vcycle_bytes[2];   /* algorithmic HBM bytes of one preconditioner apply
                               (all field V-cycles + couplings), [0] FP64, [1] mixed */
  double spmv_bytes[2];     /* algorithmic bytes of one outer SpMV, [0] FP64 x, [1] FP32 x */
  double setup_seconds;     /* wall time of the last setup */
  double setup_field_seconds[HBGS_MAX_FIELDS]; /* wall time of each field's block
                               extraction and hierarchy build in the last setup */
  double setup_stage_seconds[8]; /* last setup, summed over fields (host wall time of
                               each stage, which includes its waits): [0] block and
                               coupling extraction, [1] strength and MIS-2
                               aggregation, [2] filtering, eigenvalue estimate and
                               prolongator smoothing, [3] R = P^T, [4] Galerkin
                               products, [5] coarsest factorisation and inverse,
                               [6] smoother data (diagonal inverses, Chebyshev
                               estimates), [7] transposes, FP32 copies, row
                               statistics and work vectors */
} hbgs_stats_t;

/* Fill *opt with the defaults listed above. */
void hbgs_default_options(hbgs_options *opt);

/* Build the preconditioner for A (device CSR, n rows, nnz entries) with the
 * field map field_of_row[n] (device, values in [0, n_fields)).
 * group_tree (host, tree_len entries) is the field-group tree in bracket
 * code: -1 opens a group, -2 closes it, f >= 0 is the leaf for field f; every
 * field appears exactly once and the outermost group encloses everything,
 * e.g. {-1, -1,0,1,-2, -1,2,-2, -1,3,-2, -2} for ((phi_s, phi_e), (p), (c)).
 * Sec. 3.2: fields are split into blocks, the sweep visits the leaves in
 * depth-first order.  All setup (permutation, splitting, strength, MIS-2
 * aggregation, prolongator smoothing, Galerkin products, coarsest factor)
 * runs on the device.  Each diagonal block must be structurally symmetric.
 * On success *out owns device memory until hbgs_destroy. */
hbgs_status hbgs_setup(hbgs_ctx **out, int32_t n, int64_t nnz, const int32_t *rowptr,
                       const int32_t *col, const double *val, int32_t n_fields,
                       const int32_t *field_of_row, int32_t tree_len, const int32_t *group_tree,
                       const hbgs_options *opt, void *stream);

/* Replace A's values (same pattern as at setup; device pointer, nnz entries).
 * rebuild_hierarchy != 0 rebuilds the whole preconditioner from the new
 * values; 0 replaces only the operator GMRES iterates with (and its
 * transpose) and keeps the current preconditioner, which then acts as a
 * preconditioner for the new matrix (e.g. for small perturbations). */
hbgs_status hbgs_set_values(hbgs_ctx *ctx, const double *val, int32_t rebuild_hierarchy, void *stream);

/* Select the precision mode of later apply/solve calls (0 FP64, 1 mixed). */
hbgs_status hbgs_set_precision(hbgs_ctx *ctx, int32_t precision);

/* Change the stopping rule of later solves: true relative residual rtol
 * (>= 0) and the cap on Arnoldi steps (>= 0). */
hbgs_status hbgs_set_tolerance(hbgs_ctx *ctx, double rtol, int32_t max_iters);

/* z = M^-1 r (transpose = 0) or z = M^-T r (transpose = 1): one block
 * Gauss-Seidel sweep (forward: lower, leaves in order; transposed: upper,
 * leaves in reverse order, with A^T couplings and adjoint V-cycles).
 * r, z: device, n doubles, caller's ordering; may not alias.  The call is
 * enqueued on `stream` and returns once z is complete (stream synchronised);
 * in the mixed mode the FP32 result is widened to FP64 exactly. */
hbgs_status hbgs_apply(hbgs_ctx *ctx, const double *r, double *z, int32_t transpose, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): z = M^-1 r
 * or M^-T r exactly as hbgs_apply computes it, with every temporary of the
 * call (the permuted input and output, 16 bytes per row at most) in a fixed
 * 64 MiB device buffer that the library holds on each device it runs on
 * until the process ends.  The call allocates nothing and does not
 * synchronise: it is enqueued on `stream` and z is ready when the stream
 * reaches that point.  r, z: device, n doubles, caller's ordering; may not
 * alias.  Returns HBGS_EINVAL (nothing enqueued) when the system has more
 * than 4,194,304 rows, for a nested-form context (its inner solvers need
 * their own workspace), or for transpose != 0 while the adjoint's operators
 * do not exist (build_transpose = 0 and no transpose call since the last
 * setup or value update).  Calls on one device share the buffer: calls
 * that overlap in time on one device (several host threads, or streams
 * that are not ordered with each other) race and must not be issued. */
hbgs_status hbgs_apply_noalloc(hbgs_ctx *ctx, const double *r, double *z, int32_t transpose, void *stream);

/* Solve A x = b (transpose = 0) or A^T x = b (transpose = 1) with flexible
 * right-preconditioned GMRES(m).  b, x: device, n doubles; x is the initial
 * guess when use_x0 != 0, else zero.  On return (stream synchronised):
 * *iters = total Arnoldi steps; hist (host, hist_cap entries, may be NULL)
 * holds the relative residual before the first step and after each step
 * (Givens estimate inside a cycle, true residual at each cycle end);
 * *hist_len = number of entries produced (may exceed hist_cap).
 * Returns HBGS_OK when the true relative residual <= rtol,
 * HBGS_NOT_CONVERGED when max_iters is reached first. b = 0 gives x = 0.
 * A b with a NaN or infinite entry returns HBGS_EINVAL (x unspecified). */
hbgs_status hbgs_solve(hbgs_ctx *ctx, const double *b, double *x, int32_t use_x0, int32_t transpose,
                       int32_t *iters, double *hist, int32_t hist_cap, int32_t *hist_len,
                       void *stream);

/* grad_val[p] = -lambda[row(p)] * x[col(p)] over A's pattern (the gradient
 * of a scalar loss with respect to A's values when lambda solves the adjoint
 * system A^T lambda = dL/dx).  Device pointers; grad_val has nnz entries. */
hbgs_status hbgs_grad_values(hbgs_ctx *ctx, const double *lambda, const double *x, double *grad_val,
                             void *stream);

/* Hierarchy sizes, algorithmic bytes and setup time (host struct). */
hbgs_status hbgs_stats(hbgs_ctx *ctx, hbgs_stats_t *out);

/* Host copy of one hierarchy object of field `field` (0-based, caller's
 * field ids) at level `level`: which = 0 A_l, 1 P_l, 2 R_l, 3 A_l^T.
 * Pass NULL arrays to query sizes (*n_rows, *n_cols, *nnz), then call
 * again with host arrays rowptr[n_rows+1], col[nnz], val[nnz].
 * Level-local indices; the finest level's rows are the field's rows in the
 * caller's order. */
hbgs_status hbgs_get_level(hbgs_ctx *ctx, int32_t field, int32_t level, int32_t which,
                           int32_t *n_rows, int32_t *n_cols, int64_t *nnz, int32_t *rowptr,
                           int32_t *col, double *val);

/* Host copy of level `level`'s aggregate ids (n_rows entries, -1 = row
 * excluded from aggregation) and its scalars out3 = {Chebyshev eigenvalue
 * estimate, prolongator-smoothing eigenvalue estimate, omega}. */
hbgs_status hbgs_get_aggregates(hbgs_ctx *ctx, int32_t field, int32_t level, int32_t *agg,
                                double *out3);

/* Kernel timing: `enable` = 0 off, -1 every kernel class, otherwise a bit
 * mask of classes (bit k = the k-th record reported by hbgs_kernel_times).
 * While on, each launch of a selected solve-phase kernel is bracketed by HIP
 * events recorded on its launch stream; durations are accumulated per class
 * (enabling resets the totals).  GMRES steps are launched one kernel at a
 * time (not replayed from graphs) while timing is on.  hbgs_kernel_times copies up to cap records
 * (name, total milliseconds, launch count, algorithmic bytes) and returns the
 * number of records, or a negative status. */
hbgs_status hbgs_profile(hbgs_ctx *ctx, int32_t enable);
int32_t hbgs_kernel_times(hbgs_ctx *ctx, char (*names)[48], double *total_ms, int64_t *launches,
                          double *bytes, int32_t cap);

/* Route the persistent device memory of contexts created afterwards (the
 * hierarchy and the GMRES workspace) through a caller's allocator, e.g. a
 * framework's caching allocator: alloc(bytes, user) returns device memory of
 * the current device or NULL (setup then fails with HBGS_ENOMEM);
 * free(ptr, user) releases it.  alloc may be called from the library's setup
 * threads concurrently.  NULL for both restores hipMalloc / hipFree.  Each
 * allocation is freed with the hook that made it, so the hook may change while
 * contexts are alive.  The chunks of the setup threads' scratch stacks (kept
 * for rebuilds until the context is destroyed) come from the hook too; the
 * few temporaries of hbgs_setup's pattern phase use HIP's stream-ordered
 * allocator.  Returns HBGS_EINVAL if exactly one of the two is NULL.
 * Process-wide; not to be called concurrently with hbgs_setup. */
hbgs_status hbgs_set_allocator(void *(*alloc)(size_t bytes, void *user), void (*free)(void *ptr, void *user),
                               void *user);

/* Test knob (process-wide; not to be called concurrently with hbgs_setup or
 * hbgs_set_values): the kernel path that every row of the Galerkin products'
 * sparse matrix products (eq. galerkin) takes.  0 (default): by the row's
 * size (narrow LDS tables shared by several rows, one wavefront per row, one
 * block per row, global-memory tables); 1: one wavefront per row; 2: the
 * numeric rows one block each; 3: every row through the global-memory
 * tables.  Every path accumulates each entry's products in ascending order
 * of the inner index, so the hierarchy is bitwise the same on each route.
 * Returns HBGS_EINVAL for any other value. */
hbgs_status hbgs_debug_spgemm_route(int32_t route);

/* Test knob (process-wide; not to be called while a solve or apply runs):
 * 1 (default): sparse matrix-vector products whose matrix has operand
 * tiles (built at setup where every block of rows reads its operand in at
 * most 48 spans of 64 consecutive entries) stage those spans in LDS instead
 * of gathering operand entries from memory; 0: always gather.  Both forms
 * compute the same products and row sums, so results are bitwise the same.
 * Returns HBGS_EINVAL for any other value. */
hbgs_status hbgs_debug_spmv_tiles(int32_t on);

void hbgs_destroy(hbgs_ctx *ctx);
const char *hbgs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HBGS_H */
