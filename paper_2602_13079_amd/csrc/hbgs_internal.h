// Internal declarations shared by the HIP translation units of libhbgs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <mutex>
#include <vector>

#include "hbgs.h"

namespace hbgs {

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);

struct Error {
  hbgs_status code;
};

#define HBGS_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::hbgs::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      throw ::hbgs::Error{e_ == hipErrorOutOfMemory ? HBGS_ENOMEM : HBGS_EHIP};     \
    }                                                                               \
  } while (0)

#define HBGS_FAIL(code, msg)      \
  do {                            \
    ::hbgs::set_error(msg);       \
    throw ::hbgs::Error{code};    \
  } while (0)

// ----------------------------------------------------- device memory owner
// Allocation hook for a context's persistent device memory (null: hipMalloc
// and hipFree).  Each allocation remembers the hook that made it.
struct Allocator {
  void* (*alloc)(size_t bytes, void* user) = nullptr;
  void (*free)(void* p, void* user) = nullptr;
  void* user = nullptr;
};
Allocator current_allocator();

// All device memory of a context goes through a Pool: persistent buffers
// live until the pool is destroyed, temporaries are released explicitly.
// An arena pool (the value-dependent hierarchy) carves allocations out of
// large chunks and keeps the chunks when cleared, so a rebuild of the same
// pattern allocates nothing.  Safe to use from several host threads.
class Scratch;
class Pool {
 public:
  explicit Pool(bool arena = false) : arena_(arena) {}
  // a temporary pool whose blocks come from the thread's scratch (when one
  // is set) and go back to it when the pool is cleared or destroyed
  struct FromScratch {};
  explicit Pool(FromScratch);
  ~Pool();
  void* get(size_t bytes);  // persistent
  void release(void* p);    // free one allocation early (arena: kept until clear)
  void clear();             // release everything (arena: chunks are kept for reuse)
  template <class T>
  T* make(size_t count) {
    return static_cast<T*>(get(count * sizeof(T) + (count == 0 ? sizeof(T) : 0)));
  }
  size_t bytes() const { return total_; }

 private:
  struct Block {
    void* p;
    size_t bytes;
    Allocator a;
    bool scratch;
  };
  struct Chunk {
    char* base;
    size_t size, used;
    Allocator a;
  };
  void* raw(size_t bytes, Allocator& a);
  std::mutex mu_;
  bool arena_;
  Scratch* scratch_ = nullptr;
  std::vector<Block> blocks_;
  std::vector<Chunk> chunks_;
  size_t total_ = 0;
};

// Setup work of one host thread runs on one stream; while a StreamScope is
// alive on a thread, that thread's temporaries are stream-ordered on it.
hipStream_t& tmp_stream();
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(tmp_stream()) { tmp_stream() = s; }
  ~StreamScope() { tmp_stream() = prev; }
};

// Scratch memory for the setup temporaries of one host thread: a stack of
// device chunks that is kept across rebuilds, so a rebuild of the same size
// makes no allocation call (allocation calls from several setup threads
// serialise in the runtime, and a free waits for the device).  The thread's
// temporaries are ordered on its one stream, so a freed block can back the
// next temporary at once.  Blocks are freed in any order; the stack shrinks
// when its top is free.  One thread at a time.
class Scratch {
 public:
  Scratch() = default;
  ~Scratch();
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  void* get(size_t bytes);
  void put(void* p);

 private:
  struct Chunk {
    char* base;
    size_t size, used;
    Allocator a;
  };
  struct Rec {
    void* p;
    size_t off;
    int chunk;
    bool freed;
  };
  std::vector<Chunk> chunks_;
  std::vector<Rec> stack_;
};
// the calling thread's scratch (null: temporaries use the runtime allocator)
Scratch*& tmp_scratch();
struct ScratchScope {
  Scratch* prev;
  explicit ScratchScope(Scratch* s) : prev(tmp_scratch()) { tmp_scratch() = s; }
  ~ScratchScope() { tmp_scratch() = prev; }
};

// Temporary device buffer (setup only): from the thread's scratch when one
// is set, else stream-ordered on the thread's setup stream when one is set,
// else hipMalloc / hipFree.
template <class T>
struct Tmp {
  T* p = nullptr;
  size_t count = 0;
  hipStream_t s = nullptr;
  bool async = false;
  Scratch* sc = nullptr;
  Tmp() = default;
  explicit Tmp(size_t n) { alloc(n); }
  void alloc(size_t n) {
    release();
    count = n;
    const size_t bytes = (n ? n : 1) * sizeof(T);
    if ((sc = tmp_scratch()) != nullptr) {
      p = static_cast<T*>(sc->get(bytes));
      return;
    }
    s = tmp_stream();
    async = false;
    if (s) {
      hipError_t e = hipMallocAsync((void**)&p, bytes, s);
      if (e == hipSuccess) {
        async = true;
        return;
      }
      if (e == hipErrorOutOfMemory) HBGS_HIP(e);
      (void)hipGetLastError();  // stream-ordered allocation unavailable: plain allocation
      p = nullptr;
    }
    HBGS_HIP(hipMalloc(&p, bytes));
  }
  void release() {
    if (p) {
      if (sc)
        sc->put(p);
      else if (async)
        (void)hipFreeAsync(p, s);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    sc = nullptr;
  }
  ~Tmp() { release(); }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

// ------------------------------------------------------------- device CSR
constexpr int COL_CHUNK = 256;  // entries sharing one base of packed column indices
// row-block sizes of the streaming SpMV, largest first: row_block(q) = 512 >> q
constexpr int kRowBlocks = 8;
__host__ __device__ constexpr int row_block(int q) { return 512 >> q; }
struct DCsr {
  int n = 0, m = 0;  // rows, columns
  int64_t nnz = 0;
  int* rp = nullptr;
  int* ci = nullptr;
  double* v = nullptr;
  float* vf = nullptr;  // FP32 copy of v (solve phase, mixed precision)
  int maxlen = 0;  // longest row
  // entries of the fullest block of row_block(q) consecutive rows (block b:
  // rows [b RB, min(n, (b + 1) RB))); with maxlen, selects the solve-phase
  // kernel shape
  int blkmax[kRowBlocks] = {};
  // packed column indices for the solve phase (null when a chunk of
  // COL_CHUNK consecutive entries spans 65536 columns or more):
  // col(k) = cb[k / COL_CHUNK] + cd[k]
  uint16_t* cd = nullptr;
  int* cb = nullptr;
  // operand tiles for the row-block SpMV that stages its operand in LDS
  // (tile_rb = 0: not built): block b of tile_rb rows reads the operand
  // only in the tiles of TILE_W consecutive entries listed at
  // tiles[b * TILE_MAX + j] (ascending, then -1), at most tile_cnt of them;
  // entry k reads slot lc[k] / TILE_W of that list, element lc[k] % TILE_W
  int tile_rb = 0, tile_cnt = 0;
  int* tiles = nullptr;
  uint16_t* lc = nullptr;
  float avg_row() const { return n ? (float)nnz / (float)n : 0.f; }
};
constexpr int TILE_W = 64;    // operand entries per tile
constexpr int TILE_MAX = 48;  // tiles per row block at most


// DD(0)-ILU(0) leaf of one field: factors on the subdomain-block pattern of
// the field's diagonal block (L strictly below the diagonal, unit diagonal
// implied; U on and above), the transposed factors' values on the same
// pattern (the block is structurally symmetric), and level schedules: within
// subdomain b the rows of level l are order[lev[sub[b] + l] ..
// lev[sub[b] + l + 1]) and depend only on rows of earlier levels (fwd: the
// lower sweep and the factorisation; bwd: the upper sweep).
struct IluLeaf {
  DCsr F;                 // F.v: factors; F.vf: FP32 copy
  double* vT = nullptr;   // transposed factors (same pattern)
  float* vTf = nullptr;
  int* dpos = nullptr;    // position of each row's diagonal entry
  int nsub = 0;
  int *ford = nullptr, *flev = nullptr, *fsub = nullptr;
  int *bord = nullptr, *blev = nullptr, *bsub = nullptr;
  double* yd = nullptr;   // intermediate vector of the two sweeps
  float* yf = nullptr;
};

// ------------------------------------------------------ launch helpers
inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 20) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// ======================================================== setup kernels
// (setup_kernels.hip, compiled without floating-point contraction so that
// every value matches a sequential, rounded-product-then-add evaluation)
namespace setup {
// exclusive prefix sums; out has n+1 entries (out[n] = total); returns total
int64_t scan_i32_to_i64(const int* in, int64_t* out, int64_t n, hipStream_t s);
int64_t scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);
int64_t counts_to_rowptr(const int* counts, int* rp, int n, hipStream_t s);  // int32 rowptr

void validate(int n, int64_t nnz, const int* rp, const int* ci, const double* v, int nf, const int* field,
              int* flags, hipStream_t s);
void field_histogram(int n, const int* field, int nf, int* counts, hipStream_t s);
void field_ranks(int n, const int* field, int f, const int* f_lo_dev, int* perm, hipStream_t s);
void field_ranks_all(int n, const int* field, int nf, const int* f_lo_host, int* perm, hipStream_t s);
void invert_perm(int n, const int* perm, int* iperm, hipStream_t s);
void permuted_lengths(int n, const int* rp, const int* perm, int* len, hipStream_t s);
void permute_fill(int n, const int* rp, const int* ci, const double* v, const int* perm, const int* iperm,
                  const int* rp_p, int* ci_p, double* v_p, int* pos_p, hipStream_t s);
void scatter_values(int64_t nnz, const double* v, const int* pos, double* v_p, hipStream_t s);

// transpose: t must have rp (m+1), ci, v allocated with a.nnz entries
void transpose(const DCsr& a, DCsr& t, hipStream_t s);
// sub-block: rows [r0,r1), columns [c0,c1) shifted by -coff; two passes
void block_count(const DCsr& a, int r0, int r1, int c0, int c1, int* cnt, hipStream_t s);
void block_fill(const DCsr& a, int r0, int r1, int c0, int c1, int coff, const int* rp_out, int* ci_out,
                double* v_out, hipStream_t s);

void diagonal(const DCsr& a, double* d, int* missing, hipStream_t s);
void strength(const DCsr& a, const double* d, double theta, char* strong, char* excluded, hipStream_t s);
// MIS-2 rounds: state 0 undecided, 1 root, 2 out, 3 excluded
void mis2_init(int n, const char* excluded, char* state, hipStream_t s);
void mis2_round(const DCsr& a, const char* strong, uint64_t salt, char* state, uint64_t* m1, char* r1,
                int* undecided, hipStream_t s);
void agg_roots(int n, const char* state, int* flag, hipStream_t s);
void agg_phase12(const DCsr& a, const char* strong, uint64_t salt, const char* state, const int64_t* root_rank,
                 int* agg, int* single_flag, hipStream_t s);
void agg_phase3(int n, const int* single_flag, const int64_t* single_rank, int nroot, int* agg, hipStream_t s);

void filter_count(const DCsr& a, const char* strong, int* cnt, hipStream_t s);
void filter_fill(const DCsr& a, const char* strong, const int* rp_f, int* ci_f, double* v_f, double* dabs,
                 hipStream_t s);

// power estimate of D^-1 B: returns lambda (host), syncs the stream
double power_estimate(const DCsr& b, const double* d, int iters, uint64_t salt, hipStream_t s);

void psmooth_count(const DCsr& af, const int* agg, int* cnt, hipStream_t s);
void psmooth_fill(const DCsr& af, const int* agg, const double* dabs, double omega, const int* rp_p, int* ci_p,
                  double* v_p, hipStream_t s);

// C = A B with in-order accumulation; allocates C's arrays from pool
void spgemm(const DCsr& a, const DCsr& b, DCsr& c, Pool& pool, hipStream_t s);
// kernel path of every product row (tests): 0 by row size, 1 one wavefront
// per row, 2 numeric rows one block each, 3 global-memory tables
void set_spgemm_route(int route);

// dense coarsest factor: returns 0 ok, -4 singular; inv (row-major n*n) = A^-1
int dense_inverse(const DCsr& a, double* inv, hipStream_t s);

void cast_f32(int64_t n, const double* in, float* out, hipStream_t s);
// A^T of a structurally symmetric A: same pattern, values gathered (no sort)
void transpose_symmetric(const DCsr& a, double* vt, hipStream_t s);
// q: 2 a.n rows, row 2i = row i of a, row 2i+1 = row i of b (a.m == b.m)
void interleave_rows(Pool& pool, const DCsr& a, const DCsr& b, DCsr& q, hipStream_t s);
// longest row of a and its fullest row blocks (a.maxlen, a.blkmax)
void row_stats(DCsr& a, hipStream_t s);
// the operand tiles of a's blocks of rb rows (a.tiles, a.lc, a.tile_cnt;
// a.tile_rb = rb), or none (a.tile_rb = 0) where a block has more than
// TILE_MAX tiles or more entries than one block's LDS staging holds
void build_tiles(Pool& pool, DCsr& a, int rb, hipStream_t s);
// DD(0)-ILU(0) of the n x n block a with subdomains of `sub` rows (factors,
// transposed factors, schedules, FP32 copies); returns -4 on a zero pivot
int ilu_setup(Pool& pool, const DCsr& a, int sub, IluLeaf& out, hipStream_t s);
void ilu_transpose(Pool& pool, IluLeaf& leaf, hipStream_t s);
// builds a.cd / a.cb when every chunk of COL_CHUNK entries fits a 16-bit
// offset from its smallest column (leaves them null otherwise)
void pack_columns(Pool& pool, DCsr& a, hipStream_t s);
// dense transpose of an n x n row-major matrix
void dense_transpose(int n, const double* in, double* out, hipStream_t s);
void reciprocal(int n, const double* d, double* dinv, float* dinvf, hipStream_t s);
void sort_rows(const DCsr& a, hipStream_t s);
}  // namespace setup

// ======================================================== solve kernels
namespace solve {
// rows per block of the streaming SpMV for matrix a with LDS staging of
// cap products per block (0: no row-block shape fits)
int rows_per_block(const DCsr& a, int cap, bool vec);
constexpr int ROWS_CAP_F32 = 4096, ROWS_CAP_F64 = 2048;
// use the operand tiles where a matrix has them (default) or never (tests)
void set_tiles(bool on);
// kernel classes tracked by the optional profiler
enum Kind {
  K_SPMV_OUTER = 0,
  K_SPMV_RESID,
  K_CHEB_PRE,
  K_CHEB_POST_A,
  K_CHEB_POST_B,
  K_CHEB_OTHER,
  K_RESID,
  K_RESTRICT,
  K_PROLONG,
  K_COARSE,
  K_COUPLE,
  K_DOT1,
  K_UPD_DOT2,
  K_REDUCE,
  K_GIVENS,
  K_SCALE,
  K_XUPDATE,
  K_PERMUTE,
  // the same V-cycle operations on levels below the finest one
  K_CHEB_PRE_C,
  K_CHEB_POST_A_C,
  K_CHEB_POST_B_C,
  K_CHEB_OTHER_C,
  K_RESID_C,
  K_RESTRICT_C,
  K_PROLONG_C,
  // one whole preconditioner application (every field's V-cycle and
  // coupling), timed from its first launch to its last on the caller's stream
  K_SWEEP,
  K_COUNT
};
extern const char* kind_names[K_COUNT];

struct ChebCoef {
  int degree;
  double c0;              // 1 / theta
  double c1[8], c2[8];    // step k >= 1: d = c1 d + c2 D^-1 r
};

// outer SpMV, y = A x with x double or float; resid: y = b - A x
// w = A z; e0/e1 (optional) are stamped with the kernel's start and end
void spmv_outer_f64(const DCsr& a, const double* x, double* y, hipStream_t s, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr);
void spmv_outer_mixed(const DCsr& a, const float* x, double* y, hipStream_t s, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
// t = v / vs - a z (FP64 values and result; z FP32 or FP64; vs a device
// scalar, or null for 1)
template <class TZ>
void couple_f64(const DCsr& a, const double* v, const TZ* z, double* t, const double* vs, hipStream_t s);
void spmv_resid_f64(const DCsr& a, const double* x, const double* b, double* r, hipStream_t s);

template <class T>
struct VcOps {
  // degree-2 pre-smoothing from a zero guess, one fused kernel, with the
  // first direction d0 = D^-1 b / theta precomputed by the rhs producer:
  // x = d0 + c1 d0 + c2 D^-1 (b - A d0)
  static void pre2(const DCsr& a, const T* dinv, const ChebCoef& c, const T* b, const T* d0, T* x, hipStream_t s);
  // d0 = (D^-1 b) / theta
  static void make_d0(int n, const T* b, const T* dinv, double c0, T* d0, hipStream_t s);
  // general degree, zero guess: r = b, d = D^-1 b / theta, x = d
  static void init0(int n, const T* dinv, const ChebCoef& c, const T* b, T* r, T* d, T* x, hipStream_t s);
  // post-smoothing start from x: r = b - A x, d = D^-1 r / theta (x not yet updated)
  static void post_start(const DCsr& a, const T* dinv, const ChebCoef& c, const T* b, const T* x, T* r, T* d,
                         hipStream_t s);
  // Chebyshev step k >= 1: r -= A d; dn = c1 d + c2 D^-1 r; x (+ d when add_d) += dn;
  // r and dn are stored only when keep
  static void step(const DCsr& a, const T* dinv, const ChebCoef& c, int k, bool add_d, bool keep, T* r,
                   const T* d, T* dn, T* x, hipStream_t s);
  static void add(int n, const T* d, T* x, hipStream_t s);
  static void resid(const DCsr& a, const T* b, const T* x, T* r, hipStream_t s);
  // bc = R r; when d0_c is given also d0_c = (Dc^-1 bc) * c0_c for the coarse level
  static void restrict_(const DCsr& rmat, const T* r, T* bc, const T* dinv_c, double c0_c, T* d0_c,
                        hipStream_t s);
  static void prolong(const DCsr& p, const T* xc, T* x, hipStream_t s);
  // prolongation fused with the post-smoother's start: with Q the rows of
  // A P (even) and P (odd) interleaved and r the residual b - A x from
  // before the coarse correction, one pass forms r = r - (A P) xc,
  // d = D^-1 r / theta and x = x + P xc, i.e. the residual and first
  // direction of the corrected x without re-reading A
  static void post_q(const DCsr& q, const T* dinv, const ChebCoef& c, const T* xc, T* r, T* x, T* d,
                     hipStream_t s);
  static void coarse(int n, const double* inv, int transpose, const T* b, T* x, hipStream_t s);
  static void ilu(const IluLeaf& f, int transpose, const T* t, T* z, hipStream_t s);
  // t = (T)(v / vs) - sum over coupling columns of a * z, rows of one field;
  // with d0 given also d0 = (D^-1 t) * c0 for the field's finest level.  vs
  // is a device scalar (null: 1) by which the sweep's input is divided
  static void couple(const DCsr& c, const double* v, const T* z, T* t, const T* dinv, double c0, T* d0,
                     const double* vs, hipStream_t s);
  // t = (T)(v / vs), and d0 as in couple
  static void cast_in(int n, const double* v, T* t, const T* dinv, double c0, T* d0, const double* vs,
                      hipStream_t s);
};

// GMRES pieces (FP64)
void permute_in(int n, const int* perm, const double* x, double* xp, hipStream_t s);   // xp[perm[i]] = x[i]
void permute_out(int n, const int* perm, const double* xp, double* x, hipStream_t s);  // x[i] = xp[perm[i]]
void permute_out_f32(int n, const int* perm, const float* xp, double* x, hipStream_t s);  // widening
int dot_blocks(int n);
// Givens step inputs: column j of the (m+1) x m Hessenberg matrix H, the
// rotations cs/sn, the rotated right-hand side g, and where to put the
// residual estimate (scal on the device, host_scal in pinned host memory
// or null)
struct GivensArgs {
  int j = 0, m = 0;
  const double* h1 = nullptr;
  double* H = nullptr;
  double* cs = nullptr;
  double* sn = nullptr;
  double* g = nullptr;
  double* scal = nullptr;
  double* host_scal = nullptr;
};
// Gram-Schmidt passes over the basis V_0..V_j (w = column j+1 of V), as
// per-block partial sums part[k * dot_blocks(n) + block]:
//   cgs_dots:        V_k . w (k <= j) and w . w
//   cgs_finish_dots: first V_j = (V_j - sum_{k<j} hp_k V_k) / scal[1] in
//                    place (finishing the previous step's basis vector),
//                    then as cgs_dots
//   cgs_update_dots: w -= V h1, then V_k . w (k <= j) and w . w
void cgs_dots(int n, int j, const double* V, size_t ldv, const double* w, double* part, hipStream_t s);
void cgs_finish_dots(int n, int j, double* V, size_t ldv, const double* w, const double* hp, const double* scal,
                     double* part, hipStream_t s);
void cgs_update_dots(int n, int j, const double* V, size_t ldv, double* w, const double* h1, double* part,
                     hipStream_t s);
// reduce the second pass into h2[0..j+1], then the Givens update of column
// j (scal[0] = |g_{j+1}|, scal[1] = h_{j+1,j}, scal[2] = ||w|| before
// orthogonalisation, also written to host_scal)
void reduce_givens(int n, int j, const double* part, double* h2, const GivensArgs& ga, hipStream_t s);
void mdot_reduce(int nvec, int nblocks, const double* part, double* out, hipStream_t s);
void backsolve(int jend, int m, const double* H, const double* g, double* y, hipStream_t s);
template <class TZ>
void xupdate(int n, int jend, const TZ* Z, size_t ldz, const double* y, double* x, hipStream_t s);
void norm2_partial(int n, const double* x, double* part, hipStream_t s);
void scale_copy(int n, const double* r, const double* part_sum, double* v, hipStream_t s);  // v = r / sqrt(sum)
void grad_values(int n, const int* rp, const int* ci, const double* lam, const double* x, double* g,
                 hipStream_t s);
// *diff |= (a[i] != b[i]) for some i
void compare_int(int64_t n, const int* a, const int* b, int* diff, hipStream_t s);
// *mask |= 1 << f for every field f (column ranges [lo[f], hi[f])) that a column of c falls in
void column_fields(const DCsr& c, int nf, const int* lo, const int* hi, int* mask, hipStream_t s);
}  // namespace solve

}  // namespace hbgs
