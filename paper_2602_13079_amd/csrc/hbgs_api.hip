// Host orchestration and C ABI of libhbgs: device setup pipeline, the
// block Gauss-Seidel sweep with per-field SA-AMG V-cycles, and flexible
// GMRES(m) with classical Gram-Schmidt applied twice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "hbgs_internal.h"

namespace hbgs {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

static std::mutex g_alloc_mu;
static Allocator g_alloc;
Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

// Fixed device buffer of hbgs_apply_noalloc: the permuted input (8 bytes
// per row) and the permuted output column (4 or 8 bytes per row), so at most
// 16 bytes per row.  Each device that loads the library holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: hbgs_setup looks the address up once per device (with that
// device current) and keeps it in scratch_dev.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int64_t kNoAllocMaxRows = (int64_t)(kNoAllocScratchBytes / 16);
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up once)
static void* scratch_dev() {
  int dev = 0;
  HBGS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) HBGS_FAIL(HBGS_EHIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HBGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) HBGS_FAIL(HBGS_EHIP, "no device address for the fixed scratch buffer");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

hipStream_t& tmp_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}
Scratch*& tmp_scratch() {
  static thread_local Scratch* s = nullptr;
  return s;
}

static void free_block(void* p, const Allocator& a) {
  if (a.free)
    a.free(p, a.user);
  else
    (void)hipFree(p);
}

void* Pool::raw(size_t bytes, Allocator& a) {
  void* p = nullptr;
  a = current_allocator();
  if (a.alloc) {
    p = a.alloc(bytes, a.user);
    if (!p) {
      set_error("device allocation of " + std::to_string(bytes) + " bytes failed in the user allocator");
      throw Error{HBGS_ENOMEM};
    }
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      set_error(std::string("device allocation of ") + std::to_string(bytes) + " bytes failed: " +
                hipGetErrorString(e));
      throw Error{HBGS_ENOMEM};
    }
  }
  return p;
}

Scratch::~Scratch() {
  for (auto& c : chunks_) free_block(c.base, c.a);
}
void* Scratch::get(size_t bytes) {
  const size_t need = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
  // the chunk holding the top of the stack, else the first
  size_t c = stack_.empty() ? 0 : (size_t)stack_.back().chunk;
  for (; c < chunks_.size(); ++c)
    if (chunks_[c].size - chunks_[c].used >= need) break;
  if (c == chunks_.size()) {  // grow: a new chunk at least twice the last
    Chunk k{};
    k.size = std::max<size_t>(need, chunks_.empty() ? size_t(64) << 20 : 2 * chunks_.back().size);
    k.a = current_allocator();
    if (k.a.alloc) {
      k.base = static_cast<char*>(k.a.alloc(k.size, k.a.user));
      if (!k.base) {
        set_error("device allocation of " + std::to_string(k.size) + " bytes failed in the user allocator");
        throw Error{HBGS_ENOMEM};
      }
    } else {
      hipError_t e = hipMalloc(&k.base, k.size);
      if (e != hipSuccess) {
        set_error(std::string("device allocation of ") + std::to_string(k.size) + " bytes failed: " +
                  hipGetErrorString(e));
        throw Error{HBGS_ENOMEM};
      }
    }
    k.used = 0;
    chunks_.push_back(k);
  }
  Chunk& k = chunks_[c];
  void* p = k.base + k.used;
  stack_.push_back({p, k.used, (int)c, false});
  k.used += need;
  return p;
}
void Scratch::put(void* p) {
  for (size_t q = stack_.size(); q-- > 0;)
    if (stack_[q].p == p) {
      stack_[q].freed = true;
      break;
    }
  while (!stack_.empty() && stack_.back().freed) {
    chunks_[stack_.back().chunk].used = stack_.back().off;
    stack_.pop_back();
  }
}

Pool::Pool(FromScratch) : arena_(false), scratch_(tmp_scratch()) {}
Pool::~Pool() {
  clear();
  for (auto& c : chunks_) free_block(c.base, c.a);
  chunks_.clear();
}
void Pool::clear() {
  std::lock_guard<std::mutex> lk(mu_);
  for (size_t q = blocks_.size(); q-- > 0;) {
    Block& b = blocks_[q];
    if (b.scratch)
      scratch_->put(b.p);
    else
      free_block(b.p, b.a);
  }
  blocks_.clear();
  for (auto& c : chunks_) c.used = 0;
  total_ = 0;
}
void* Pool::get(size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (arena_) {
    const size_t need = (bytes + 255) / 256 * 256;
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& c : chunks_)
      if (c.size - c.used >= need) {
        void* p = c.base + c.used;
        c.used += need;
        total_ += need;
        return p;
      }
    Chunk c{};
    c.size = std::max<size_t>(need, size_t(256) << 20);
    c.base = static_cast<char*>(raw(c.size, c.a));
    c.used = need;
    chunks_.push_back(c);
    total_ += need;
    return c.base;
  }
  Allocator a;
  if (scratch_) {
    void* p = scratch_->get(bytes);
    std::lock_guard<std::mutex> lk(mu_);
    blocks_.push_back({p, bytes, a, true});
    total_ += bytes;
    return p;
  }
  void* p = raw(bytes, a);
  std::lock_guard<std::mutex> lk(mu_);
  blocks_.push_back({p, bytes, a, false});
  total_ += bytes;
  return p;
}
void Pool::release(void* p) {
  if (arena_) return;
  std::lock_guard<std::mutex> lk(mu_);
  for (size_t i = 0; i < blocks_.size(); ++i)
    if (blocks_[i].p == p) {
      if (blocks_[i].scratch)
        scratch_->put(p);
      else
        free_block(p, blocks_[i].a);
      total_ -= blocks_[i].bytes;
      blocks_.erase(blocks_.begin() + i);
      return;
    }
}

static uint64_t splitmix64_host(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// ------------------------------------------------------------- profiler
struct Profiler {
  bool on = false;
  uint32_t mask = 0;  // kernel classes bracketed while on
  struct Rec {
    hipEvent_t a, b;
    int kind;
    double bytes;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> free_events;
  double total_ms[solve::K_COUNT] = {};
  int64_t launches[solve::K_COUNT] = {};
  double bytes[solve::K_COUNT] = {};
  hipEvent_t ev() {
    if (!free_events.empty()) {
      hipEvent_t e = free_events.back();
      free_events.pop_back();
      return e;
    }
    hipEvent_t e;
    HBGS_HIP(hipEventCreate(&e));
    return e;
  }
  // events for a launch of class k that stamps them itself (null when the
  // class is not being timed)
  void stamp(int k, double b, hipEvent_t* e0, hipEvent_t* e1) {
    *e0 = *e1 = nullptr;
    if (!on || !(mask >> k & 1u)) return;
    *e0 = ev();
    *e1 = ev();
    pending.push_back({*e0, *e1, k, b});
    if (pending.size() > 4096) flush();
  }
  void flush() {
    for (auto& r : pending) {
      HBGS_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      HBGS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      total_ms[r.kind] += ms;
      launches[r.kind] += 1;
      bytes[r.kind] += r.bytes;
      free_events.push_back(r.a);
      free_events.push_back(r.b);
    }
    pending.clear();
  }
  ~Profiler() {
    for (auto& r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : free_events) (void)hipEventDestroy(e);
  }
};

// brackets one kernel launch when profiling is on
struct Prof {
  Profiler* p;
  hipStream_t s;
  int kind;
  double bytes;
  hipEvent_t a = nullptr;
  Prof(Profiler& pr, hipStream_t st, int k, double b) : p(&pr), s(st), kind(k), bytes(b) {
    if (p->on && (p->mask >> k & 1u)) {
      a = p->ev();
      HBGS_HIP(hipEventRecord(a, s));
    }
  }
  ~Prof() {
    if (p->on && a) {
      hipEvent_t b = p->ev();
      (void)hipEventRecord(b, s);
      p->pending.push_back({a, b, kind, bytes});
      if (p->pending.size() > 4096) p->flush();
    }
  }
};

// ------------------------------------------------------------- structures
struct Level {
  DCsr A, AT, P, R;
  DCsr Q, QT;  // rows of A P and P interleaved (QT: A^T P and P), for the fused prolongation
  int* agg = nullptr;
  double* dinv = nullptr;
  float* dinvf = nullptr;
  double lam_cheb = 0, lam_p = 0, omega = 0;
  solve::ChebCoef cc{};
  // work vectors: rhs b, solution x, residual r, directions d / dn
  double *bd = nullptr, *xd = nullptr, *rd = nullptr, *dd = nullptr, *dnd = nullptr;
  float *bf = nullptr, *xf = nullptr, *rf = nullptr, *df = nullptr, *dnf = nullptr;
};

struct Field {
  int id = 0, lo = 0, hi = 0;
  std::vector<Level> lv;  // lv.back() is the coarsest level
  double* inv = nullptr;   // dense inverse of the coarsest operator (row-major)
  double* invT = nullptr;  // its transpose (adjoint apply)
  DCsr lower;             // rows of this field, columns of earlier leaves (global)
  DCsr upperT;            // rows of A^T in this field, columns of later leaves (global)
  double* td = nullptr;   // fine-level right-hand side
  float* tf = nullptr;
  uint32_t deps[2] = {0, 0};  // fields read by the coupling rows: [0] forward, [1] adjoint sweep
  double setup_seconds = 0.0;  // wall time of this field's part of the last setup
  double stage_seconds[8] = {};  // per setup stage (see hbgs_stats_t)
  int leaf = 0;                  // 0 SA-AMG V-cycle, 1 Jacobi sweep, 2 DD(0)-ILU(0)
  double bytes[2] = {};          // algorithmic bytes of its sweep step: [0] FP64, [1] mixed
  IluLeaf ilu;
  int n() const { return hi - lo; }
};

// Concurrent field V-cycles: a field's sweep step (coupling + V-cycle) only
// reads the z of the fields its coupling rows reference, so independent
// fields run on separate streams; events carry the dependencies.
struct SweepPlan {
  std::vector<int> order;   // fields in visiting order
  std::vector<int> stream;  // stream slot per position
  int nstreams = 1;
};
constexpr int MAX_SWEEP_STREAMS = 4;

// one captured GMRES iteration (key: precision, transpose, column j)
struct IterGraph {
  hipGraphExec_t exec = nullptr;
};

// Workspace of one flexible GMRES (the outer solve, or the inner solve of a
// group in the nested form): basis V ((m+1) x n, FP64, leading dimension ld),
// stored directions Z (m x n; FP32 in the mixed mode), right-hand side bp,
// iterate xp, Gram-Schmidt partial sums, Hessenberg data, and a pinned host
// slot that the Givens step writes the residual estimate to.
struct Krylov {
  int n = 0, m = 0;
  size_t ld = 0;
  double *V = nullptr, *Zd = nullptr;
  float* Zf = nullptr;
  double *bp = nullptr, *xp = nullptr, *r = nullptr, *part = nullptr, *h1 = nullptr, *h2 = nullptr,
         *hn2 = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *scal = nullptr;
  double* host = nullptr;      // pinned
  double* host_dev = nullptr;  // its device-side address
  Krylov() = default;
  Krylov(const Krylov&) = delete;
  Krylov& operator=(const Krylov&) = delete;
  ~Krylov() {
    if (host) (void)hipHostFree(host);
  }
  void ensure(Pool& pool, int n_, int m_, int precision) {
    if (V) {
      if (precision == 1 && !Zf) Zf = pool.make<float>((size_t)m * ld);
      if (precision == 0 && !Zd) Zd = pool.make<double>((size_t)m * ld);
      return;
    }
    n = n_;
    m = m_;
    ld = ((size_t)n + 63) / 64 * 64;
    V = pool.make<double>((size_t)(m + 1) * ld);
    if (precision == 1)
      Zf = pool.make<float>((size_t)m * ld);
    else
      Zd = pool.make<double>((size_t)m * ld);
    bp = pool.make<double>(n);
    xp = pool.make<double>(n);
    r = pool.make<double>(n);
    part = pool.make<double>((size_t)(m + 2) * solve::dot_blocks(n));
    h1 = pool.make<double>(m + 2);
    h2 = pool.make<double>(m + 2);
    hn2 = pool.make<double>(2);
    H = pool.make<double>((size_t)(m + 1) * m);
    cs = pool.make<double>(m);
    sn = pool.make<double>(m);
    g = pool.make<double>(m + 1);
    y = pool.make<double>(m);
    scal = pool.make<double>(4);
    // coherent (fine-grained): the Givens kernel's stores reach the host
    // while the rest of the step still runs
    HBGS_HIP(hipHostMalloc((void**)&host, 8 * sizeof(double), hipHostMallocCoherent));
    HBGS_HIP(hipHostGetDevicePointer((void**)&host_dev, host, 0));
  }
};

// Nested form: one child of the outermost group of the field tree.  Its
// fields are contiguous in the permuted ordering.
struct Group {
  int lo = 0, hi = 0;
  std::vector<int> fields;    // leaves in visiting order
  DCsr A, AT;                 // its diagonal block and transpose (columns relative to lo)
  DCsr lower, upperT;         // couplings to earlier / later groups (global columns)
  SweepPlan plan[2];          // the group's own sweep (forward, adjoint)
  std::unique_ptr<Krylov> K;  // inner solver workspace
  int n() const { return hi - lo; }
};

}  // namespace hbgs

struct hbgs_ctx {
  hbgs_options o{};
  int precision = 0;
  int n = 0, nf = 0;
  int64_t nnz = 0;
  hbgs::Pool pool;
  hbgs::Pool hier{true};  // value-dependent hierarchy (rebuilt by set_values; arena)
  void* noalloc_scratch = nullptr;  // this device's fixed scratch buffer (hbgs_apply_noalloc)
  // setup temporaries: one scratch per field's build thread, the last for
  // the calling thread
  hbgs::Scratch scratch[HBGS_MAX_FIELDS + 1];
  int *rp0 = nullptr, *ci0 = nullptr;  // caller's pattern
  int *perm = nullptr, *iperm = nullptr, *src = nullptr;
  int* posT = nullptr;  // position in A_p of each A_p^T entry
  // transposed operators: A_p^T's values follow A_p's (apt_fresh); the
  // hierarchy's transposed parts exist for the current hierarchy (hier_t)
  bool apt_fresh = false, hier_t = false;
  hbgs::DCsr Ap, ApT;
  std::vector<int> leaf_order, f_lo, f_hi;
  std::vector<hbgs::Field> F;
  // outer GMRES workspace (permuted ordering)
  int m = 0;
  hbgs::Krylov K;
  // nested form: the children of the outermost group
  std::vector<std::vector<int>> group_fields;
  std::vector<int> group_of;  // field -> index in group_fields
  std::vector<hbgs::Group> G;
  hbgs::Profiler prof;
  hbgs_stats_t stats{};
  // concurrent sweep
  hbgs::SweepPlan plan[2];
  hipStream_t fstream[hbgs::MAX_SWEEP_STREAMS] = {};
  hipEvent_t fdone[HBGS_MAX_FIELDS] = {};
  hipEvent_t fork = nullptr;
  // concurrent setup: one stream per field
  hipStream_t sstream[HBGS_MAX_FIELDS] = {};
  hipEvent_t setup_in = nullptr;
  // solve stream (graph capture needs a non-default stream) and graph cache
  hipStream_t sm = nullptr;
  hipEvent_t join_in = nullptr, join_out = nullptr;
  std::map<int, hbgs::IterGraph> graphs;
  void clear_graphs() {
    for (auto& kv : graphs)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
  }
  ~hbgs_ctx() {
    clear_graphs();
    if (sm) (void)hipStreamDestroy(sm);
    if (join_in) (void)hipEventDestroy(join_in);
    if (join_out) (void)hipEventDestroy(join_out);
    for (auto& st : fstream)
      if (st) (void)hipStreamDestroy(st);
    for (auto& e : fdone)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    for (auto& st : sstream)
      if (st) (void)hipStreamDestroy(st);
    if (setup_in) (void)hipEventDestroy(setup_in);
  }
};

namespace hbgs {

using solve::VcOps;

static void validate_options(const hbgs_options& o) {
  if (o.precision != 0 && o.precision != 1) HBGS_FAIL(HBGS_EINVAL, "precision must be 0 or 1");
  if (o.restart < 1 || o.restart > 64) HBGS_FAIL(HBGS_EINVAL, "restart must be in [1, 64]");
  if (o.max_iters < 0) HBGS_FAIL(HBGS_EINVAL, "max_iters must be >= 0");
  if (!(o.rtol >= 0.0)) HBGS_FAIL(HBGS_EINVAL, "rtol must be >= 0");
  if (o.cheb_degree < 1 || o.cheb_degree > 8) HBGS_FAIL(HBGS_EINVAL, "cheb_degree must be in [1, 8]");
  if (!(o.cheb_ratio > 1.0) || !(o.cheb_boost > 0.0)) HBGS_FAIL(HBGS_EINVAL, "bad Chebyshev interval options");
  if (o.eig_iters < 0 || !(o.sa_damping > 0.0)) HBGS_FAIL(HBGS_EINVAL, "bad eigenvalue / damping options");
  if (o.coarse_max < 1 || o.coarse_max > 8000) HBGS_FAIL(HBGS_EINVAL, "coarse_max must be in [1, 8000]");
  if (o.max_levels < 1 || o.max_levels > HBGS_MAX_LEVELS) HBGS_FAIL(HBGS_EINVAL, "max_levels out of range");
  if ((o.block_jacobi != 0 && o.block_jacobi != 1) || (o.nested != 0 && o.nested != 1) ||
      (o.setup_concurrent != 0 && o.setup_concurrent != 1))
    HBGS_FAIL(HBGS_EINVAL, "block_jacobi, nested and setup_concurrent must be 0 or 1");
  if (o.inner_restart < 1 || o.inner_restart > 64) HBGS_FAIL(HBGS_EINVAL, "inner_restart must be in [1, 64]");
  if (o.inner_max_iters < 0 || !(o.inner_rtol >= 0.0)) HBGS_FAIL(HBGS_EINVAL, "bad inner solver options");
  for (int f = 0; f < HBGS_MAX_FIELDS; ++f) {
    if (o.field_cheb_degree[f] < 0 || o.field_cheb_degree[f] > 8)
      HBGS_FAIL(HBGS_EINVAL, "field_cheb_degree must be in [0, 8]");
    if (o.field_leaf[f] < 0 || o.field_leaf[f] > 2) HBGS_FAIL(HBGS_EINVAL, "field_leaf must be 0, 1 or 2");
  }
  if (o.ilu_block < 1) HBGS_FAIL(HBGS_EINVAL, "ilu_block must be >= 1");
  if (o.build_transpose != 0 && o.build_transpose != 1) HBGS_FAIL(HBGS_EINVAL, "build_transpose must be 0 or 1");
}

static void parse_tree(hbgs_ctx* c, const int32_t* tree, int len) {
  std::vector<char> seen(c->nf, 0);
  int depth = 0, closed_root = 0;
  c->leaf_order.clear();
  c->group_fields.clear();
  for (int t = 0; t < len; ++t) {
    int code = tree[t];
    if (closed_root) HBGS_FAIL(HBGS_EINVAL, "group tree: entries after the outermost group");
    if (code == -1) {
      ++depth;
      if (depth == 2) c->group_fields.push_back({});
    } else if (code == -2) {
      if (depth == 0) HBGS_FAIL(HBGS_EINVAL, "group tree: unbalanced close");
      if (--depth == 0) closed_root = 1;
    } else if (code >= 0 && code < c->nf) {
      if (depth == 0 || seen[code]) HBGS_FAIL(HBGS_EINVAL, "group tree: field outside a group or repeated");
      seen[code] = 1;
      c->leaf_order.push_back(code);
      if (depth == 1) c->group_fields.push_back({});  // a leaf directly under the root: its own group
      c->group_fields.back().push_back(code);
    } else {
      HBGS_FAIL(HBGS_EINVAL, "group tree: invalid code");
    }
  }
  if (depth != 0 || !closed_root) HBGS_FAIL(HBGS_EINVAL, "group tree: unbalanced");
  for (int f = 0; f < c->nf; ++f)
    if (!seen[f]) HBGS_FAIL(HBGS_EINVAL, "group tree: a field is missing");
}

// extract rows [r0,r1) x columns [c0,c1) (shifted by -coff) of a into a new CSR
static DCsr extract(Pool& pool, const DCsr& a, int r0, int r1, int c0, int c1, int coff, int ncols,
                    hipStream_t s) {
  DCsr b;
  b.n = r1 - r0;
  b.m = ncols;
  Tmp<int> cnt(b.n);
  b.rp = pool.make<int>(b.n + 1);
  setup::block_count(a, r0, r1, c0, c1, cnt.p, s);
  b.nnz = setup::counts_to_rowptr(cnt.p, b.rp, b.n, s);
  b.ci = pool.make<int>(b.nnz);
  b.v = pool.make<double>(b.nnz);
  setup::block_fill(a, r0, r1, c0, c1, coff, b.rp, b.ci, b.v, s);
  return b;
}

static DCsr transpose_new(Pool& pool, const DCsr& a, hipStream_t s) {
  DCsr t;
  t.rp = pool.make<int>(a.m + 1);
  t.ci = pool.make<int>(a.nnz);
  t.v = pool.make<double>(a.nnz);
  setup::transpose(a, t, s);
  return t;
}

static void add_f32(Pool& pool, DCsr& a, hipStream_t s) {
  a.vf = pool.make<float>(a.nnz);
  setup::cast_f32(a.nnz, a.v, a.vf, s);
}

static solve::ChebCoef cheb_coef(const hbgs_options& o, double lam) {
  solve::ChebCoef c{};
  c.degree = o.cheb_degree;
  double lmax = o.cheb_boost * lam, lmin = lmax / o.cheb_ratio;
  double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
  double sigma = theta / delta, rho = 1.0 / sigma;
  c.c0 = 1.0 / theta;
  for (int k = 1; k < o.cheb_degree; ++k) {
    double rn = 1.0 / (2.0 * sigma - rho);
    c.c1[k] = rn * rho;
    c.c2[k] = 2.0 * rn / delta;
    rho = rn;
  }
  return c;
}

// pattern of a equals the pattern of its transpose
static bool structurally_symmetric_dev(const DCsr& a, hipStream_t s) {
  DCsr t;
  Pool tmp{Pool::FromScratch{}};
  t.rp = tmp.make<int>(a.m + 1);
  t.ci = tmp.make<int>(a.nnz);
  t.v = nullptr;
  DCsr pat = a;
  pat.v = nullptr;
  setup::transpose(pat, t, s);
  Tmp<int> diff(1);
  HBGS_HIP(hipMemsetAsync(diff.p, 0, sizeof(int), s));
  solve::compare_int(a.n + 1, a.rp, t.rp, diff.p, s);
  solve::compare_int(a.nnz, a.ci, t.ci, diff.p, s);
  int d = 0;
  HBGS_HIP(hipMemcpyAsync(&d, diff.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  return d == 0;
}

// host wall time per setup stage: to(q) closes the running stage and starts q
struct StageClock {
  double* acc;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  int cur = -1;
  explicit StageClock(double* a) : acc(a) {}
  void to(int q) {
    auto now = std::chrono::steady_clock::now();
    if (cur >= 0) acc[cur] += std::chrono::duration<double>(now - t).count();
    t = now;
    cur = q;
  }
  ~StageClock() { to(-1); }
};

// Coarsest levels up to this many rows are solved with a dense inverse; a
// coarsening that stops above it (stalled, or at the level cap) ends in a
// smoothed coarsest level: one application of its Chebyshev polynomial from
// zero.  (The paper's coarse solver is sparse direct and has no such limit.)
constexpr int kDenseCoarseMax = 8000;

// a level whose cycle smooths (every level but a dense-solved coarsest one)
static bool smoothed_level(const Field& F, size_t l) { return l + 1 < F.lv.size() || !F.inv; }

// SA-AMG hierarchy of one field's diagonal block (level 0 already set)
static void build_hierarchy(hbgs_ctx* c, Field& F, hipStream_t s) {
  const hbgs_options& o = c->o;
  StageClock clk(F.stage_seconds);
  Pool& pool = c->hier;
  const uint64_t salt_base = splitmix64_host(o.seed + 0x1000ull * (uint64_t)(F.id + 1));
  Tmp<int> flag1(1);
  for (int l = 0;; ++l) {
    const int n = F.lv[l].A.n;
    clk.to(6);
    Tmp<double> d(n);
    HBGS_HIP(hipMemsetAsync(flag1.p, 0, sizeof(int), s));
    setup::diagonal(F.lv[l].A, d.p, flag1.p, s);
    int missing = 0;
    HBGS_HIP(hipMemcpyAsync(&missing, flag1.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    if (missing) HBGS_FAIL(HBGS_EINVAL, "zero or missing diagonal entry in a field block");
    if (F.leaf != 0) {  // one-level leaf: diagonal inverse, or the incomplete factors
      Level& L = F.lv[0];
      if (!structurally_symmetric_dev(L.A, s))
        HBGS_FAIL(HBGS_EINVAL, "a diagonal field block is not structurally symmetric");
      clk.to(6);
      L.dinv = pool.make<double>(n);
      L.dinvf = pool.make<float>(n);
      setup::reciprocal(n, d.p, L.dinv, L.dinvf, s);
      if (F.leaf == 2) {
        clk.to(5);
        if (setup::ilu_setup(pool, L.A, o.ilu_block, F.ilu, s) != 0)
          HBGS_FAIL(HBGS_ESINGULAR, "zero pivot in the incomplete factorisation");
      }
      HBGS_HIP(hipStreamSynchronize(s));
      return;
    }
    bool last = n <= o.coarse_max || l + 1 >= o.max_levels;
    if (!last) {
      DCsr& A = F.lv[l].A;
      clk.to(1);
      Tmp<char> strong(A.nnz), excluded(n), state(n), r1(n);
      Tmp<uint64_t> m1(n);
      setup::strength(A, d.p, o.theta[F.id], strong.p, excluded.p, s);
      const uint64_t salt = salt_base + (uint64_t)l;
      setup::mis2_init(n, excluded.p, state.p, s);
      for (int round = 0;; ++round) {
        setup::mis2_round(A, strong.p, salt, state.p, m1.p, r1.p, flag1.p, s);
        int und = 0;
        HBGS_HIP(hipMemcpyAsync(&und, flag1.p, sizeof(int), hipMemcpyDeviceToHost, s));
        HBGS_HIP(hipStreamSynchronize(s));
        if (und == 0) break;
        if (round > n + 2) HBGS_FAIL(HBGS_ESETUP, "aggregation did not terminate");
      }
      Tmp<int> rflag(n), sflag(n);
      Tmp<int64_t> rrank(n + 1), srank(n + 1);
      setup::agg_roots(n, state.p, rflag.p, s);
      int64_t nroot = setup::scan_i32_to_i64(rflag.p, rrank.p, n, s);
      int* agg = pool.make<int>(n);
      setup::agg_phase12(A, strong.p, salt, state.p, rrank.p, agg, sflag.p, s);
      int64_t nsingle = setup::scan_i32_to_i64(sflag.p, srank.p, n, s);
      setup::agg_phase3(n, sflag.p, srank.p, (int)nroot, agg, s);
      int64_t nagg = nroot + nsingle;
      if (nagg == 0 || (double)nagg > 0.95 * n) {
        pool.release(agg);
        last = true;
      } else {
        F.lv[l].agg = agg;
        // filtered matrix and absolute-row-sum weight
        clk.to(2);
        DCsr af;
        af.n = af.m = n;
        Tmp<int> cnt(n), afrp(n + 1);
        setup::filter_count(A, strong.p, cnt.p, s);
        af.nnz = setup::counts_to_rowptr(cnt.p, afrp.p, n, s);
        Tmp<int> afci(af.nnz);
        Tmp<double> afv(af.nnz), dabs(n);
        af.rp = afrp.p;
        af.ci = afci.p;
        af.v = afv.p;
        setup::filter_fill(A, strong.p, af.rp, af.ci, af.v, dabs.p, s);
        double lam_p = setup::power_estimate(af, dabs.p, o.eig_iters, splitmix64_host(salt_base + 0x5000 + l), s);
        if (!(lam_p > 0.0)) HBGS_FAIL(HBGS_ESETUP, "non-positive eigenvalue estimate for prolongator smoothing");
        double omega = o.sa_damping / lam_p;
        F.lv[l].lam_p = lam_p;
        F.lv[l].omega = omega;
        DCsr P;
        P.n = n;
        P.m = (int)nagg;
        P.rp = pool.make<int>(n + 1);
        setup::psmooth_count(af, agg, cnt.p, s);
        P.nnz = setup::counts_to_rowptr(cnt.p, P.rp, n, s);
        P.ci = pool.make<int>(P.nnz);
        P.v = pool.make<double>(P.nnz);
        setup::psmooth_fill(af, agg, dabs.p, omega, P.rp, P.ci, P.v, s);
        clk.to(3);
        DCsr R = transpose_new(pool, P, s);
        clk.to(4);
        DCsr AP, Ac;
        Pool tmp_pool{Pool::FromScratch{}};
        setup::spgemm(A, P, AP, tmp_pool, s);
        setup::spgemm(R, AP, Ac, pool, s);
        // the fused prolongation pays where A P has no more entries than A
        // (coarse levels: about half; the finest level: 10-20% more, where
        // the separate prolongation and residual passes are as fast)
        if (AP.nnz <= A.nnz) setup::interleave_rows(pool, AP, P, F.lv[l].Q, s);
        F.lv[l].P = P;
        F.lv[l].R = R;
        F.lv.emplace_back();
        F.lv[l + 1].A = Ac;
      }
    }
    Level& L = F.lv[l];
    if (last && n <= kDenseCoarseMax) {
      clk.to(5);
      F.inv = pool.make<double>((size_t)n * n);
      if (setup::dense_inverse(L.A, F.inv, s) != 0) HBGS_FAIL(HBGS_ESINGULAR, "singular coarsest-level matrix");
      break;
    }
    clk.to(6);
    L.dinv = pool.make<double>(n);
    L.dinvf = pool.make<float>(n);
    setup::reciprocal(n, d.p, L.dinv, L.dinvf, s);
    L.lam_cheb = setup::power_estimate(L.A, d.p, o.eig_iters, splitmix64_host(salt_base + 0x9000 + l), s);
    hbgs_options of = o;
    if (o.field_cheb_degree[F.id] > 0) of.cheb_degree = o.field_cheb_degree[F.id];
    L.cc = cheb_coef(of, L.lam_cheb);
    if (last) break;  // beyond the dense limit: a smoothed coarsest level (F.inv stays null)
  }
  // solve-phase data: transposes, FP32 copies, work vectors
  clk.to(7);
  if (!structurally_symmetric_dev(F.lv[0].A, s))
    HBGS_FAIL(HBGS_EINVAL, "a diagonal field block is not structurally symmetric");
  for (size_t l = 0; l < F.lv.size(); ++l) {
    Level& L = F.lv[l];
    add_f32(pool, L.A, s);
    setup::row_stats(L.A, s);
    setup::pack_columns(pool, L.A, s);
    setup::build_tiles(pool, L.A, solve::rows_per_block(L.A, solve::ROWS_CAP_F32, true), s);
    if (l + 1 < F.lv.size()) {
      add_f32(pool, L.P, s);
      add_f32(pool, L.R, s);
      setup::row_stats(L.P, s);
      setup::row_stats(L.R, s);
      setup::pack_columns(pool, L.P, s);
      setup::pack_columns(pool, L.R, s);
      setup::build_tiles(pool, L.P, solve::rows_per_block(L.P, solve::ROWS_CAP_F32, true), s);
      if (L.Q.n) {
        add_f32(pool, L.Q, s);
        setup::row_stats(L.Q, s);
        setup::pack_columns(pool, L.Q, s);
        setup::build_tiles(pool, L.Q, solve::rows_per_block(L.Q, solve::ROWS_CAP_F32, true), s);
      }
    }
    const int n = L.A.n;
    L.bd = pool.make<double>(n);
    L.xd = pool.make<double>(n);
    L.rd = pool.make<double>(n);
    L.dd = pool.make<double>(n);
    L.dnd = pool.make<double>(n);
    L.bf = pool.make<float>(n);
    L.xf = pool.make<float>(n);
    L.rf = pool.make<float>(n);
    L.df = pool.make<float>(n);
    L.dnf = pool.make<float>(n);
  }
}

static double spmv_bytes(const DCsr& a, int tv, int tx, int ty, int extra_vec) {
  return (double)a.nnz * (tv + 4) + 4.0 * (a.n + 1) + (double)a.m * tx + (double)a.n * ty +
         (double)extra_vec * a.n * tv;
}

static void compute_stats(hbgs_ctx* c) {
  hbgs_stats_t& st = c->stats;
  st.n = c->n;
  st.n_fields = c->nf;
  st.nnz = c->nnz;
  for (int p = 0; p < 2; ++p) {
    int T = p == 0 ? 8 : 4;
    double b = 0;
    for (int f : c->leaf_order) {
      Field& F = c->F[f];
      double fb = 0;
      if (F.lower.nnz) fb += spmv_bytes(F.lower, T, T, T, 0) + 8.0 * F.n();
      if (F.leaf == 1) {
        fb += 3.0 * T * F.n();
      } else if (F.leaf == 2) {
        fb += 2.0 * spmv_bytes(F.ilu.F, T, T, T, 1);
      } else {
        for (size_t l = 0; l + 1 < F.lv.size(); ++l) {
          const Level& L = F.lv[l];
          const DCsr& A = L.A;
          fb += spmv_bytes(A, T, T, T, 1);          // pre (b, dinv gathered; x written)
          fb += spmv_bytes(A, T, T, T, 1);          // residual
          fb += spmv_bytes(L.R, T, T, T, 0);        // restriction
          fb += spmv_bytes(L.P, T, T, T, 1);        // prolongation (x read+write)
          fb += spmv_bytes(A, T, T, 2 * T, 2);      // post start
          fb += spmv_bytes(A, T, T, T, 3);          // post step
        }
        const Level& C = F.lv.back();
        const int nc = C.A.n;
        if (F.inv)
          fb += 8.0 * nc * nc + 2.0 * nc * T;
        else  // smoothed coarsest: the pre-smoothing polynomial only
          fb += (C.cc.degree - 1) * spmv_bytes(C.A, T, T, T, 3) + 4.0 * T * nc;
      }
      F.bytes[p] = fb;
      b += fb;
    }
    st.vcycle_bytes[p] = b;
    st.spmv_bytes[p] = spmv_bytes(c->Ap, 8, T, 8, 0);
  }
  for (int q = 0; q < 8; ++q) st.setup_stage_seconds[q] = 0.0;
  for (int f = 0; f < c->nf && f < HBGS_MAX_FIELDS; ++f) {
    const Field& F = c->F[f];
    for (int q = 0; q < 8; ++q) st.setup_stage_seconds[q] += F.stage_seconds[q];
    st.levels[f] = (int)F.lv.size();
    st.setup_field_seconds[f] = F.setup_seconds;
    for (size_t l = 0; l < F.lv.size() && l < HBGS_MAX_LEVELS; ++l) {
      st.rows[f][l] = F.lv[l].A.n;
      st.nnz_a[f][l] = F.lv[l].A.nnz;
      st.nnz_p[f][l] = l + 1 < F.lv.size() ? F.lv[l].P.nnz : 0;
    }
  }
}

// Stream slots for the sweep: a field continues the stream of the latest
// field (in visiting order) it depends on; a field without dependencies
// starts the next free slot.
static void plan_sweep(hbgs_ctx* c, const std::vector<int>& leaves, int tr, SweepPlan& p) {
  const int nl = (int)leaves.size();
  p.order.clear();
  p.stream.clear();
  p.nstreams = 0;
  std::vector<int> slot_of(c->nf, -1);
  for (int q = 0; q < nl; ++q) {
    int f = leaves[tr ? nl - 1 - q : q];
    int slot = -1;
    for (int k = q - 1; k >= 0 && slot < 0; --k)
      if (c->F[f].deps[tr] >> p.order[k] & 1u) slot = slot_of[p.order[k]];
    if (slot < 0) slot = p.nstreams < MAX_SWEEP_STREAMS ? p.nstreams++ : q % MAX_SWEEP_STREAMS;
    slot_of[f] = slot;
    p.order.push_back(f);
    p.stream.push_back(slot);
  }
  if (p.nstreams == 0) p.nstreams = 1;
  for (int k = 0; k < MAX_SWEEP_STREAMS; ++k)
    if (!c->fstream[k]) HBGS_HIP(hipStreamCreateWithFlags(&c->fstream[k], hipStreamNonBlocking));
  for (int f = 0; f < c->nf; ++f)
    if (!c->fdone[f]) HBGS_HIP(hipEventCreateWithFlags(&c->fdone[f], hipEventDisableTiming));
  if (!c->fork) HBGS_HIP(hipEventCreateWithFlags(&c->fork, hipEventDisableTiming));
  if (!c->sm) HBGS_HIP(hipStreamCreateWithFlags(&c->sm, hipStreamNonBlocking));
  if (!c->join_in) HBGS_HIP(hipEventCreateWithFlags(&c->join_in, hipEventDisableTiming));
  if (!c->join_out) HBGS_HIP(hipEventCreateWithFlags(&c->join_out, hipEventDisableTiming));
}

// per-field part of the value-dependent setup: diagonal block, couplings,
// SA-AMG hierarchy
// The adjoint's parts of one field (A_p^T's values must be current): the
// transposed couplings read by the reversed sweep; A_l^T on every level (A_l
// is structurally symmetric -- level 0 is checked, and Galerkin products
// R A P with R = P^T keep the property -- so A_l^T shares A_l's pattern and
// packed columns); the coarsest inverse transposed; the transposed ILU
// factors.  Counted in the solve-data stage.
static void build_field_T(hbgs_ctx* c, Field& F, hipStream_t s) {
  StageClock clk(F.stage_seconds);
  clk.to(7);
  Pool& pool = c->hier;
  int glo = 0, ghi = c->n;
  if (c->o.nested) {
    const std::vector<int>& gf = c->group_fields[c->group_of[F.id]];
    glo = c->f_lo[gf.front()];
    ghi = c->f_hi[gf.back()];
  }
  const bool bj = c->o.block_jacobi != 0;
  F.upperT = extract(pool, c->ApT, F.lo, F.hi, bj ? ghi : F.hi, ghi, glo, ghi - glo, s);
  add_f32(pool, F.upperT, s);
  setup::row_stats(F.upperT, s);
  setup::pack_columns(pool, F.upperT, s);
  setup::build_tiles(pool, F.upperT, solve::rows_per_block(F.upperT, solve::ROWS_CAP_F32, true), s);
  if (F.leaf == 2) setup::ilu_transpose(pool, F.ilu, s);
  if (F.leaf == 0) {
    for (size_t l = 0; l < F.lv.size(); ++l) {
      Level& L = F.lv[l];
      L.AT = L.A;  // pattern, row statistics and packed columns
      L.AT.v = pool.make<double>(L.A.nnz);
      setup::transpose_symmetric(L.A, L.AT.v, s);
      add_f32(pool, L.AT, s);
      if (L.Q.n) {  // A_l^T P_l for the adjoint's fused prolongation (same pattern as A_l P_l)
        DCsr ATP;
        Pool tmp_pool{Pool::FromScratch{}};
        setup::spgemm(L.AT, L.P, ATP, tmp_pool, s);
        setup::interleave_rows(pool, ATP, L.P, L.QT, s);
        add_f32(pool, L.QT, s);
        setup::row_stats(L.QT, s);
        setup::pack_columns(pool, L.QT, s);
      }
    }
    if (F.inv) {
      const int nc = F.lv.back().A.n;
      F.invT = pool.make<double>((size_t)nc * nc);
      setup::dense_transpose(nc, F.inv, F.invT, s);
    }
  }
  HBGS_HIP(hipStreamSynchronize(s));
}

static void build_field(hbgs_ctx* c, Field& F, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  std::fill(std::begin(F.stage_seconds), std::end(F.stage_seconds), 0.0);
  F.leaf = c->o.field_leaf[F.id];
  StageClock clk(F.stage_seconds);
  clk.to(0);
  F.lv.clear();
  F.lv.emplace_back();
  F.inv = F.invT = nullptr;  // set again if the new hierarchy ends in a dense-solved level
  F.lv[0].A = extract(c->hier, c->Ap, F.lo, F.hi, F.lo, F.hi, F.lo, F.n(), s);
  // couplings read by this field's sweep step: every earlier (later, for the
  // adjoint) field; in the nested form only those of its own group, with
  // columns relative to the group; none in block Jacobi
  int glo = 0, ghi = c->n;
  if (c->o.nested) {
    const std::vector<int>& gf = c->group_fields[c->group_of[F.id]];
    glo = c->f_lo[gf.front()];
    ghi = c->f_hi[gf.back()];
  }
  const bool bj = c->o.block_jacobi != 0;
  F.lower = extract(c->hier, c->Ap, F.lo, F.hi, glo, bj ? glo : F.lo, glo, ghi - glo, s);
  add_f32(c->hier, F.lower, s);
  setup::row_stats(F.lower, s);
  setup::pack_columns(c->hier, F.lower, s);
  setup::build_tiles(c->hier, F.lower, solve::rows_per_block(F.lower, solve::ROWS_CAP_F32, true), s);
  F.td = c->hier.make<double>(F.n());
  F.tf = c->hier.make<float>(F.n());
  HBGS_HIP(hipStreamSynchronize(s));
  clk.to(-1);
  build_hierarchy(c, F, s);
  if (c->o.build_transpose) build_field_T(c, F, s);
  HBGS_HIP(hipStreamSynchronize(s));
  F.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// hardware queues per process: HIP's GPU_MAX_HW_QUEUES, 4 when unset
static int hw_queues() {
  const char* e = std::getenv("GPU_MAX_HW_QUEUES");
  const int q = e ? std::atoi(e) : 4;
  return std::max(1, std::min(q, (int)HBGS_MAX_FIELDS));
}

// which fields each field's coupling rows read, forward (tr = 0: lower) or
// adjoint (tr = 1: upperT), with column ranges relative to the coupling's
// own column origin
static void field_deps(hbgs_ctx* c, int tr, hipStream_t s) {
  Tmp<int> masks(c->nf);
  HBGS_HIP(hipMemsetAsync(masks.p, 0, sizeof(int) * c->nf, s));
  std::vector<int> lo(c->nf), hi(c->nf);
  for (int f = 0; f < c->nf; ++f) {
    const int origin = c->o.nested ? c->f_lo[c->group_fields[c->group_of[f]].front()] : 0;
    for (int g = 0; g < c->nf; ++g) {
      lo[g] = c->f_lo[g] - origin;
      hi[g] = c->f_hi[g] - origin;
    }
    solve::column_fields(tr ? c->F[f].upperT : c->F[f].lower, c->nf, lo.data(), hi.data(), masks.p + f, s);
  }
  std::vector<int> hm(c->nf);
  HBGS_HIP(hipMemcpyAsync(hm.data(), masks.p, sizeof(int) * c->nf, hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  for (int f = 0; f < c->nf; ++f) c->F[f].deps[tr] = (uint32_t)hm[f];
}

// the adjoint's parts above the fields (after every build_field_T): the
// groups' transposed blocks, the adjoint dependencies and sweep plans
static void build_rest_T(hbgs_ctx* c, hipStream_t s) {
  for (Group& g : c->G) {
    const bool bj = c->o.block_jacobi != 0;
    g.AT = extract(c->hier, c->ApT, g.lo, g.hi, g.lo, g.hi, g.lo, g.n(), s);
    g.upperT = extract(c->hier, c->ApT, g.lo, g.hi, bj ? c->n : g.hi, c->n, 0, c->n, s);
    for (DCsr* a : {&g.AT, &g.upperT}) {
      setup::row_stats(*a, s);
      setup::pack_columns(c->hier, *a, s);
    }
  }
  field_deps(c, 1, s);
  plan_sweep(c, c->leaf_order, 1, c->plan[1]);
  for (Group& g : c->G) plan_sweep(c, g.fields, 1, g.plan[1]);
  c->hier_t = true;
}

// value-dependent part of setup: blocks, couplings, hierarchies.  The
// fields are independent here, so each is built by its own host thread on
// its own stream (the latency-bound steps of one field, such as the
// aggregation rounds and the factorisation steps, overlap the others').
static void build_values(hbgs_ctx* c, hipStream_t s) {
  ScratchScope main_scratch(&c->scratch[HBGS_MAX_FIELDS]);
  c->hier_t = false;
  c->clear_graphs();
  c->hier.clear();
  c->group_of.assign(c->nf, 0);
  for (size_t q = 0; q < c->group_fields.size(); ++q)
    for (int f : c->group_fields[q]) c->group_of[f] = (int)q;
  c->F.assign(c->nf, Field{});
  for (int f = 0; f < c->nf; ++f) {
    Field& F = c->F[f];
    F.id = f;
    F.lo = c->f_lo[f];
    F.hi = c->f_hi[f];
  }
  if (c->nf == 1 || !c->o.setup_concurrent) {
    StreamScope scope(s);
    ScratchScope scratch(&c->scratch[HBGS_MAX_FIELDS]);
    for (int f = 0; f < c->nf; ++f) build_field(c, c->F[f], s);
  } else {
    // One build thread per hardware queue the runtime gives this process
    // (streams beyond that share queues and would run one after another):
    // thread 0 works on the caller's stream, the others on their own, and
    // each takes the next unbuilt field until none is left.
    int dev = 0;
    HBGS_HIP(hipGetDevice(&dev));
    const int nw = std::min(c->nf, hw_queues());
    if (!c->setup_in) HBGS_HIP(hipEventCreateWithFlags(&c->setup_in, hipEventDisableTiming));
    for (int w = 1; w < nw; ++w)
      if (!c->sstream[w]) HBGS_HIP(hipStreamCreateWithFlags(&c->sstream[w], hipStreamNonBlocking));
    HBGS_HIP(hipEventRecord(c->setup_in, s));
    std::vector<int> code(c->nf, HBGS_OK);
    std::vector<std::string> msg(c->nf);
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    auto work = [&](int w) {
      hipStream_t sw = w == 0 ? s : c->sstream[w];
      int f = -1;
      try {
        HBGS_HIP(hipSetDevice(dev));
        if (w > 0) HBGS_HIP(hipStreamWaitEvent(sw, c->setup_in, 0));
        StreamScope scope(sw);
        ScratchScope scratch(&c->scratch[w]);
        while ((f = next.fetch_add(1)) < c->nf) build_field(c, c->F[f], sw);
      } catch (const Error& e) {
        if (f < 0 || f >= c->nf) f = 0;
        code[f] = e.code;
        msg[f] = g_last_error;
        next.store(c->nf);  // the others stop after their current field
      } catch (const std::exception& e) {
        if (f < 0 || f >= c->nf) f = 0;
        code[f] = HBGS_EHIP;
        msg[f] = std::string("exception: ") + e.what();
        next.store(c->nf);
      }
    };
    try {
      for (int w = 0; w < nw; ++w) th.emplace_back(work, w);
    } catch (...) {
      for (auto& t : th) t.join();
      throw;
    }
    for (auto& t : th) t.join();
    for (int f = 0; f < c->nf; ++f)
      if (code[f] != HBGS_OK) {
        // a failed build may leave work in flight on its stream: drain every
        // build stream before the caller can free what that work touches
        for (int w = 1; w < nw; ++w) (void)hipStreamSynchronize(c->sstream[w]);
        (void)hipStreamSynchronize(s);
        set_error(msg[f]);
        throw Error{(hbgs_status)code[f]};
      }
  }
  // nested form: each child of the outermost group, its diagonal block and
  // its couplings to the other children
  c->G.resize(c->o.nested ? c->group_fields.size() : 0);
  for (size_t q = 0; q < c->G.size(); ++q) {
    Group& g = c->G[q];
    g.fields = c->group_fields[q];
    g.lo = c->f_lo[g.fields.front()];
    g.hi = c->f_hi[g.fields.back()];
    g.A = extract(c->hier, c->Ap, g.lo, g.hi, g.lo, g.hi, g.lo, g.n(), s);
    const bool bj = c->o.block_jacobi != 0;
    g.lower = extract(c->hier, c->Ap, g.lo, g.hi, 0, bj ? 0 : g.lo, 0, c->n, s);
    for (DCsr* a : {&g.A, &g.lower}) {
      setup::row_stats(*a, s);
      setup::pack_columns(c->hier, *a, s);
    }
  }
  field_deps(c, 0, s);
  plan_sweep(c, c->leaf_order, 0, c->plan[0]);
  for (Group& g : c->G) plan_sweep(c, g.fields, 0, g.plan[0]);
  if (c->o.build_transpose) build_rest_T(c, s);
  HBGS_HIP(hipStreamSynchronize(s));
  compute_stats(c);
}

// --------------------------------------------------------------- V-cycle
template <class T>
struct Buf;
template <>
struct Buf<double> {
  static double* b(Level& L) { return L.bd; }
  static double* x(Level& L) { return L.xd; }
  static double* r(Level& L) { return L.rd; }
  static double* d(Level& L) { return L.dd; }
  static double* dn(Level& L) { return L.dnd; }
  static const double* dinv(const Level& L) { return L.dinv; }
  static double* t(Field& F) { return F.td; }
};
template <>
struct Buf<float> {
  static float* b(Level& L) { return L.bf; }
  static float* x(Level& L) { return L.xf; }
  static float* r(Level& L) { return L.rf; }
  static float* d(Level& L) { return L.df; }
  static float* dn(Level& L) { return L.dnf; }
  static const float* dinv(const Level& L) { return L.dinvf; }
  static float* t(Field& F) { return F.tf; }
};

// profiler class of a V-cycle operation on level l (finest level or below)
static int lk(int kind, int l) {
  if (l == 0) return kind;
  switch (kind) {
    case solve::K_CHEB_PRE: return solve::K_CHEB_PRE_C;
    case solve::K_CHEB_POST_A: return solve::K_CHEB_POST_A_C;
    case solve::K_CHEB_POST_B: return solve::K_CHEB_POST_B_C;
    case solve::K_CHEB_OTHER: return solve::K_CHEB_OTHER_C;
    case solve::K_RESID: return solve::K_RESID_C;
    case solve::K_RESTRICT: return solve::K_RESTRICT_C;
    case solve::K_PROLONG: return solve::K_PROLONG_C;
    default: return kind;
  }
}

template <class T>
static void vcycle(hbgs_ctx* c, Field& F, int l, int tr, const T* b, T* x, hipStream_t s) {
  using B = Buf<T>;
  const int TS = (int)sizeof(T);
  Level& L = F.lv[l];
  const int n = L.A.n;
  const bool coarsest = l + 1 == (int)F.lv.size();
  if (coarsest && F.inv) {
    Prof p(c->prof, s, solve::K_COARSE, 8.0 * n * n + 2.0 * n * TS);
    VcOps<T>::coarse(n, tr ? F.invT : F.inv, 0, b, x, s);
    return;
  }
  const DCsr& A = tr ? L.AT : L.A;
  const T* dinv = B::dinv(L);
  const solve::ChebCoef& cc = L.cc;
  T *r = B::r(L), *d = B::d(L), *dn = B::dn(L);
  // pre-smoothing from a zero guess (degree 2: d0 was written by the
  // producer of b into this level's d buffer)
  if (cc.degree == 2) {
    Prof p(c->prof, s, lk(solve::K_CHEB_PRE, l), spmv_bytes(A, TS, TS, TS, 2));
    VcOps<T>::pre2(A, dinv, cc, b, d, x, s);
  } else {
    {
      Prof p(c->prof, s, lk(solve::K_CHEB_OTHER, l), 4.0 * n * TS);
      VcOps<T>::init0(n, dinv, cc, b, r, d, x, s);
    }
    for (int k = 1; k < cc.degree; ++k) {
      Prof p(c->prof, s, lk(solve::K_CHEB_OTHER, l), spmv_bytes(A, TS, TS, 3 * TS, 2));
      VcOps<T>::step(A, dinv, cc, k, false, k + 1 < cc.degree, r, d, dn, x, s);
      std::swap(d, dn);
    }
  }
  if (coarsest) return;  // a smoothed coarsest level: the polynomial from zero only
  {
    Prof p(c->prof, s, lk(solve::K_RESID, l), spmv_bytes(A, TS, TS, TS, 1));
    VcOps<T>::resid(A, b, x, r, s);
  }
  Level& C = F.lv[l + 1];
  {
    const bool d0c = smoothed_level(F, l + 1) && C.cc.degree == 2;
    Prof p(c->prof, s, lk(solve::K_RESTRICT, l), spmv_bytes(L.R, TS, TS, TS, d0c ? 2 : 0));
    VcOps<T>::restrict_(L.R, r, B::b(C), d0c ? B::dinv(C) : nullptr, C.cc.c0, d0c ? B::d(C) : nullptr, s);
  }
  vcycle<T>(c, F, l + 1, tr, B::b(C), B::x(C), s);
  // coarse correction and the post-smoother's start: x += P xc, r = b - A x,
  // d = D^-1 r / theta, in one pass over [A P; P] from the residual r of
  // before the correction (r - A P xc = b - A (x + P xc))
  d = B::d(L);
  dn = B::dn(L);
  const DCsr& Q = tr ? L.QT : L.Q;
  if (Q.n) {
    Prof p(c->prof, s, lk(solve::K_CHEB_POST_A, l), spmv_bytes(Q, TS, TS, TS, 2));
    VcOps<T>::post_q(Q, dinv, cc, B::x(C), r, x, d, s);
  } else {
    {
      Prof p(c->prof, s, lk(solve::K_PROLONG, l), spmv_bytes(L.P, TS, TS, TS, 1));
      VcOps<T>::prolong(L.P, B::x(C), x, s);
    }
    Prof p(c->prof, s, lk(solve::K_CHEB_POST_A, l), spmv_bytes(A, TS, TS, 2 * TS, 2));
    VcOps<T>::post_start(A, dinv, cc, b, x, r, d, s);
  }
  if (cc.degree == 1) {
    Prof p(c->prof, s, lk(solve::K_CHEB_OTHER, l), 3.0 * n * TS);
    VcOps<T>::add(n, d, x, s);
  }
  for (int k = 1; k < cc.degree; ++k) {
    bool keep = k + 1 < cc.degree;
    Prof p(c->prof, s, lk(keep ? solve::K_CHEB_OTHER : solve::K_CHEB_POST_B, l), spmv_bytes(A, TS, TS, TS, 3));
    VcOps<T>::step(A, dinv, cc, k, k == 1, keep, r, d, dn, x, s);
    std::swap(d, dn);
  }
}

// z = M^-1 (v / vs) (tr = 0) or M^-T (v / vs) (tr = 1) over the fields of
// `plan`, in the permuted ordering shifted by `base` (field f's rows are
// v[F.lo - base ..]); z has type T; vs is a device scalar (null: 1)
template <class T>
static void sweep(hbgs_ctx* c, const SweepPlan& plan, int tr, const double* v, T* z, int base, const double* vs,
                  hipStream_t s0) {
  const int nl = (int)plan.order.size();
  const int TS = (int)sizeof(T);
  double plan_bytes = 0;
  for (int f : plan.order) plan_bytes += c->F[f].bytes[TS == 4 ? 1 : 0];
  Prof whole(c->prof, s0, solve::K_SWEEP, plan_bytes);
  HBGS_HIP(hipEventRecord(c->fork, s0));
  for (int k = 0; k < plan.nstreams; ++k) HBGS_HIP(hipStreamWaitEvent(c->fstream[k], c->fork, 0));
  std::vector<int> slot_of(c->nf, -1);
  for (int q = 0; q < nl; ++q) {
    Field& F = c->F[plan.order[q]];
    const int slot = plan.stream[q];
    hipStream_t s = c->fstream[slot];
    for (int k = 0; k < q; ++k) {
      int g = plan.order[k];
      if ((F.deps[tr] >> g & 1u) && slot_of[g] != slot) HBGS_HIP(hipStreamWaitEvent(s, c->fdone[g], 0));
    }
    slot_of[F.id] = slot;
    const DCsr& cpl = tr ? F.upperT : F.lower;
    const int off = F.lo - base;
    Level& L0 = F.lv[0];
    // the finest level's first Chebyshev direction is formed with its rhs
    const bool d0 = F.leaf == 0 && smoothed_level(F, 0) && L0.cc.degree == 2;
    const T* dinv0 = d0 ? Buf<T>::dinv(L0) : nullptr;
    T* d00 = d0 ? Buf<T>::d(L0) : nullptr;
    if (F.leaf == 1) {  // z = D^-1 t straight from the coupling / cast epilogue
      const T* dinv = Buf<T>::dinv(L0);
      T* zf = z + off;
      Prof p(c->prof, s, solve::K_COUPLE, (cpl.nnz ? spmv_bytes(cpl, TS, 0, TS, 2) : 0.0) + (8.0 + 2 * TS) * F.n());
      if (cpl.nnz > 0)
        VcOps<T>::couple(cpl, v + off, z, Buf<T>::t(F), dinv, 1.0, zf, vs, s);
      else if (sizeof(T) == sizeof(double) && !vs)
        VcOps<T>::make_d0(F.n(), reinterpret_cast<const T*>(v + off), dinv, 1.0, zf, s);
      else
        VcOps<T>::cast_in(F.n(), v + off, Buf<T>::t(F), dinv, 1.0, zf, vs, s);
      HBGS_HIP(hipEventRecord(c->fdone[F.id], s));
      continue;
    }
    const T* t;
    if (cpl.nnz > 0) {
      Prof p(c->prof, s, solve::K_COUPLE,
             spmv_bytes(cpl, TS, 0, TS, d0 ? 2 : 0) + 8.0 * F.n() + (double)std::min<int64_t>(cpl.nnz, c->n) * TS);
      VcOps<T>::couple(cpl, v + off, z, Buf<T>::t(F), dinv0, L0.cc.c0, d00, vs, s);
      t = Buf<T>::t(F);
    } else if (sizeof(T) == sizeof(double) && !vs) {
      t = reinterpret_cast<const T*>(v + off);
      if (d0) {
        Prof p(c->prof, s, solve::K_COUPLE, 3.0 * F.n() * TS);
        VcOps<T>::make_d0(F.n(), t, dinv0, L0.cc.c0, d00, s);
      }
    } else {
      Prof p(c->prof, s, solve::K_COUPLE, (8.0 + TS * (d0 ? 3 : 1)) * F.n());
      VcOps<T>::cast_in(F.n(), v + off, Buf<T>::t(F), dinv0, L0.cc.c0, d00, vs, s);
      t = Buf<T>::t(F);
    }
    if (F.leaf == 2) {
      Prof p(c->prof, s, solve::K_COARSE, 2.0 * spmv_bytes(F.ilu.F, TS, TS, TS, 1));
      VcOps<T>::ilu(F.ilu, tr, t, z + off, s);
    } else {
      vcycle<T>(c, F, 0, tr, t, z + off, s);
    }
    HBGS_HIP(hipEventRecord(c->fdone[F.id], s));
  }
  for (int q = 0; q < nl; ++q) HBGS_HIP(hipStreamWaitEvent(s0, c->fdone[plan.order[q]], 0));
}

// ------------------------------------------------------------------ GMRES
static void ensure_workspace(hbgs_ctx* c) {
  c->K.ensure(c->pool, c->n, c->m, c->precision);
  for (Group& g : c->G) {
    if (!g.K) g.K.reset(new Krylov());
    g.K->ensure(c->pool, g.n(), c->o.inner_restart, c->precision);
  }
}

static double norm2(hbgs_ctx* c, Krylov& K, const double* x, hipStream_t s) {
  int nb = solve::dot_blocks(K.n);
  {
    Prof p(c->prof, s, solve::K_REDUCE, 8.0 * K.n);
    solve::norm2_partial(K.n, x, K.part, s);
    solve::mdot_reduce(1, nb, K.part, K.hn2, s);
  }
  HBGS_HIP(hipMemcpyAsync(K.host, K.hn2, sizeof(double), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  return K.host[0];
}

// One Arnoldi step j of the flexible GMRES on A with workspace K:
// z_j = M(u_j) (written by prec into column j of K's Z), w = A z_j (into
// column j+1 of V), two classical Gram-Schmidt passes, Givens update.
// Column j+1 keeps the once-orthogonalised w' = w - V h1; its second
// correction and normalisation, v_{j+1} = (w' - V h2) / h_{j+1,j}, happen in
// the first pass of step j+1, which reads V anyway.  The preconditioner of
// step j+1 therefore reads u_{j+1} = w' / h_{j+1,j} = v_{j+1} + V h2 / h_{j+1,j}
// (the division is done as the sweep reads its input, with h_{j+1,j} from
// the device): a unit vector whose part in the span of the earlier basis
// vectors is of relative size ||h2|| / h_{j+1,j}.  That part lies in the
// span of the earlier directions z (the sweep is linear), so flexible GMRES
// is unaffected; ||h2|| is of the order of the rounding of w, and the
// breakdown test (h_{j+1,j} <= 1e-14 ||w||) ends the cycle before the ratio
// exceeds O(1).  Without the division the input would carry the scale
// prod_k h_{k+1,k}, which leaves FP32 range within a long cycle and costs
// accuracy in FP64 through the widely scaled least-squares columns.
template <class Prec>
static void iteration_body(hbgs_ctx* c, Krylov& K, const DCsr& A, Prec& prec, int j, hipStream_t s) {
  const int n = K.n, m = K.m;
  const size_t ld = K.ld;
  const int nb = solve::dot_blocks(n);
  double* vj = K.V + (size_t)j * ld;
  double* w = K.V + (size_t)(j + 1) * ld;
  prec(j, (const double*)vj, j > 0 ? K.scal + 1 : nullptr, s);
  {
    hipEvent_t e0, e1;  // stamped by the dispatch itself when this class is timed
    c->prof.stamp(solve::K_SPMV_OUTER, spmv_bytes(A, 8, c->precision ? 4 : 8, 8, 0), &e0, &e1);
    if (c->precision == 1)
      solve::spmv_outer_mixed(A, K.Zf + (size_t)j * ld, w, s, e0, e1);
    else
      solve::spmv_outer_f64(A, K.Zd + (size_t)j * ld, w, s, e0, e1);
  }
  {
    // column j holds the previous step's once-orthogonalised vector: this
    // pass finishes it (its second correction and normalisation) before
    // projecting w on it
    Prof p(c->prof, s, solve::K_DOT1, 8.0 * n * (j + (j > 0 ? 3 : 2)));
    if (j == 0)
      solve::cgs_dots(n, j, K.V, ld, w, K.part, s);
    else
      solve::cgs_finish_dots(n, j, K.V, ld, w, K.h2, K.scal, K.part, s);
  }
  {
    Prof p(c->prof, s, solve::K_REDUCE, 8.0 * nb * (j + 2));
    solve::mdot_reduce(j + 2, nb, K.part, K.h1, s);
  }
  {
    Prof p(c->prof, s, solve::K_UPD_DOT2, 8.0 * n * (j + 3));
    solve::cgs_update_dots(n, j, K.V, ld, w, K.h1, K.part, s);
  }
  {
    solve::GivensArgs ga;
    ga.j = j;
    ga.m = m;
    ga.h1 = K.h1;
    ga.H = K.H;
    ga.cs = K.cs;
    ga.sn = K.sn;
    ga.g = K.g;
    ga.scal = K.scal;
    ga.host_scal = K.host_dev;
    Prof p(c->prof, s, solve::K_GIVENS, 8.0 * nb * (j + 2));
    solve::reduce_givens(n, j, K.part, K.h2, ga, s);
  }
}

// Runs step j eagerly, or replays its captured graph (capturing it on first
// use; graphs are dropped when the hierarchy changes).  Kernel timing needs
// events around individual launches, which graph replays do not provide, so
// steps run eagerly while the profiler is on.  graph_key < 0: always eager.
template <class Prec>
static void run_iteration(hbgs_ctx* c, Krylov& K, const DCsr& A, Prec& prec, int j, int graph_key, hipStream_t s) {
  if (graph_key < 0 || !c->o.use_graphs || c->prof.on) {
    iteration_body(c, K, A, prec, j, s);
    return;
  }
  const int key = graph_key * 128 + j;
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    IterGraph ig;
    hipGraph_t g = nullptr;
    HBGS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
      iteration_body(c, K, A, prec, j, s);
    } catch (...) {
      (void)hipStreamEndCapture(s, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HBGS_HIP(hipStreamEndCapture(s, &g));
    hipError_t e = hipGraphInstantiate(&ig.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HBGS_HIP(e);
    it = c->graphs.emplace(key, std::move(ig)).first;
  }
  HBGS_HIP(hipGraphLaunch(it->second.exec, s));
}

// The Givens kernel stores ||w||, h_{j+1,j} and then, after a system-scope
// fence, the residual estimate into coherent pinned memory.  The host waits
// for the estimate slot to leave its sentinel instead of synchronising the
// stream, so it decides on the next step as soon as the store lands, while
// the Givens kernel's last wave and the stream's completion are still
// pending (enqueuing several steps ahead instead runs slower: the runtime
// handles a queue many steps deep worse than one a step deep).  Should the
// store not arrive, the stream's
// completion ends the wait (and an idle stream with the sentinel still in
// place is an error).
constexpr double kEstPending = -1.0;  // estimates are norms (>= 0, or NaN)
static void wait_estimate(const double* host, hipStream_t s) {
  const volatile double* slot = host;
  for (unsigned spins = 1;; ++spins) {
    if (*slot != kEstPending) return;
    if ((spins & 4095u) == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (*slot != kEstPending) return;
        HBGS_FAIL(HBGS_EHIP, "GMRES step ended without a residual estimate");
      }
      if (e != hipErrorNotReady) HBGS_HIP(e);
    }
    __builtin_ia32_pause();
  }
}

// Flexible GMRES(K.m) for A x = b with b in K.bp and x in K.xp (zero start
// unless use_x0); the relative residual target is rtol, at most max_iters
// Arnoldi steps.  hist (optional) receives the residual estimates, the true
// residual replacing the estimate at the end of every cycle.
template <class Prec>
static hbgs_status fgmres(hbgs_ctx* c, Krylov& K, const DCsr& A, Prec& prec, double rtol, int max_iters, int use_x0,
                          int32_t* iters, double* hist, int cap, int32_t* hlen, int graph_key, hipStream_t s) {
  const int n = K.n, m = K.m;
  const size_t ld = K.ld;
  *iters = 0;
  *hlen = 0;
  auto push = [&](double v) {
    if (hist && *hlen < cap) hist[*hlen] = v;
    (*hlen)++;
  };
  double bnorm = std::sqrt(norm2(c, K, K.bp, s));
  if (!std::isfinite(bnorm)) HBGS_FAIL(HBGS_EINVAL, "non-finite right-hand side");
  if (bnorm == 0.0) {
    HBGS_HIP(hipMemsetAsync(K.xp, 0, sizeof(double) * n, s));
    push(0.0);
    return HBGS_OK;
  }
  if (!use_x0) HBGS_HIP(hipMemsetAsync(K.xp, 0, sizeof(double) * n, s));
  auto true_resid = [&]() {
    {
      Prof p(c->prof, s, solve::K_SPMV_RESID, spmv_bytes(A, 8, 8, 8, 1));
      solve::spmv_resid_f64(A, K.xp, K.bp, K.r, s);
    }
    return std::sqrt(norm2(c, K, K.r, s));
  };
  double beta = true_resid();
  push(beta / bnorm);
  for (;;) {
    if (beta / bnorm <= rtol) return HBGS_OK;
    if (*iters >= max_iters) return HBGS_NOT_CONVERGED;
    {
      Prof p(c->prof, s, solve::K_SCALE, 16.0 * n);
      solve::scale_copy(n, K.r, K.hn2, K.V, s);  // hn2 holds ||r||^2 from true_resid
    }
    std::vector<double> g0(m + 1, 0.0);
    g0[0] = beta;
    HBGS_HIP(hipMemcpyAsync(K.g, g0.data(), sizeof(double) * (m + 1), hipMemcpyHostToDevice, s));
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      K.host[0] = kEstPending;
      run_iteration(c, K, A, prec, j, graph_key, s);  // its Givens step writes the estimate to K.host
      wait_estimate(K.host, s);
      (*iters)++;
      double est = K.host[0] / bnorm, hn = K.host[1], w0 = K.host[2];
      push(est);
      jend = j + 1;
      if (!(est == est)) HBGS_FAIL(HBGS_EHIP, "non-finite residual estimate");
      if (est <= rtol || hn <= 1e-14 * w0 || *iters >= max_iters) break;
    }
    solve::backsolve(jend, m, K.H, K.g, K.y, s);
    {
      Prof p(c->prof, s, solve::K_XUPDATE, (double)n * (16 + jend * (c->precision ? 4 : 8)));
      if (c->precision == 1)
        solve::xupdate<float>(n, jend, K.Zf, ld, K.y, K.xp, s);
      else
        solve::xupdate<double>(n, jend, K.Zd, ld, K.y, K.xp, s);
    }
    beta = true_resid();
    if (hist && *hlen - 1 < cap) hist[*hlen - 1] = beta / bnorm;
  }
}

static void nested_apply(hbgs_ctx* c, int tr, const double* v, int j, const double* vs, hipStream_t s);

// z_j = M^-1 (v / vs) (tr = 0) or M^-T (v / vs), permuted ordering, into
// column j of the outer Z (vs: device scalar or null)
static void apply_perm(hbgs_ctx* c, int tr, const double* v, int j, const double* vs, hipStream_t s) {
  Krylov& K = c->K;
  if (c->o.nested)
    nested_apply(c, tr, v, j, vs, s);
  else if (c->precision == 1)
    sweep<float>(c, c->plan[tr], tr, v, K.Zf + (size_t)j * K.ld, 0, vs, s);
  else
    sweep<double>(c, c->plan[tr], tr, v, K.Zd + (size_t)j * K.ld, 0, vs, s);
}

// Nested form (Sec. 3.2): the children of the outermost group are visited
// in order (reversed for the adjoint); child g receives v_g minus the
// couplings to the children already solved and is solved by an inner
// flexible GMRES from a zero start, preconditioned by its own sweep, to the
// inner tolerance.  Its result becomes block g of z_j (rounded to FP32 in the
// mixed mode, where Z is FP32).
static void nested_apply(hbgs_ctx* c, int tr, const double* v, int j, const double* vs, hipStream_t s) {
  Krylov& K = c->K;
  const int ng = (int)c->G.size();
  for (int q = 0; q < ng; ++q) {
    Group& g = c->G[tr ? ng - 1 - q : q];
    Krylov& KG = *g.K;
    const DCsr& cpl = tr ? g.upperT : g.lower;
    if (cpl.nnz > 0) {
      Prof p(c->prof, s, solve::K_COUPLE, spmv_bytes(cpl, 8, c->precision ? 4 : 8, 8, 1));
      if (c->precision == 1)
        solve::couple_f64<float>(cpl, v + g.lo, K.Zf + (size_t)j * K.ld, KG.bp, vs, s);
      else
        solve::couple_f64<double>(cpl, v + g.lo, K.Zd + (size_t)j * K.ld, KG.bp, vs, s);
    } else if (vs) {
      VcOps<double>::cast_in(g.n(), v + g.lo, KG.bp, nullptr, 0.0, nullptr, vs, s);
    } else {
      HBGS_HIP(hipMemcpyAsync(KG.bp, v + g.lo, sizeof(double) * g.n(), hipMemcpyDeviceToDevice, s));
    }
    auto prec = [&](int jj, const double* vv, const double* vvs, hipStream_t st) {
      if (c->precision == 1)
        sweep<float>(c, g.plan[tr], tr, vv, KG.Zf + (size_t)jj * KG.ld, g.lo, vvs, st);
      else
        sweep<double>(c, g.plan[tr], tr, vv, KG.Zd + (size_t)jj * KG.ld, g.lo, vvs, st);
    };
    int32_t it = 0, hl = 0;
    (void)fgmres(c, KG, tr ? g.AT : g.A, prec, c->o.inner_rtol, c->o.inner_max_iters, 0, &it, nullptr, 0, &hl, -1,
                 s);
    if (c->precision == 1)
      VcOps<float>::cast_in(g.n(), KG.xp, K.Zf + (size_t)j * K.ld + g.lo, nullptr, 0.0, nullptr, nullptr, s);
    else
      HBGS_HIP(hipMemcpyAsync(K.Zd + (size_t)j * K.ld + g.lo, KG.xp, sizeof(double) * g.n(),
                              hipMemcpyDeviceToDevice, s));
  }
}

static hbgs_status gmres(hbgs_ctx* c, int tr, int use_x0, int32_t* iters, double* hist, int cap, int32_t* hlen,
                         hipStream_t s) {
  auto prec = [&](int j, const double* v, const double* vs, hipStream_t st) { apply_perm(c, tr, v, j, vs, st); };
  const int graph_key = c->o.nested ? -1 : c->precision * 2 + tr;
  return fgmres(c, c->K, tr ? c->ApT : c->Ap, prec, c->o.rtol, c->o.max_iters, use_x0, iters, hist, cap, hlen,
                graph_key, s);
}

#define HBGS_FOR_ALL(k, n) \
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < (n); k += (int64_t)gridDim.x * blockDim.x)
__global__ void k_gather_vals(int64_t nnz, const double* v, const int* src, double* vp) {
  HBGS_FOR_ALL(k, nnz) vp[k] = v[src[k]];
}
__global__ void k_iota_f64(int64_t nnz, double* p) {
  HBGS_FOR_ALL(k, nnz) p[k] = (double)k;
}
__global__ void k_pos_int(int64_t nnz, const double* pos, int* posT) {
  HBGS_FOR_ALL(k, nnz) posT[k] = (int)pos[k];
}

// A_p^T's values from A_p's
static void gather_apt(hbgs_ctx* c, hipStream_t s) {
  k_gather_vals<<<grid_for(c->nnz, 256), 256, 0, s>>>(c->nnz, c->Ap.v, c->posT, c->ApT.v);
  HBGS_HIP(hipGetLastError());
  c->apt_fresh = true;
}

// Everything a transpose apply or solve reads, built on first use when the
// options defer it (build_transpose = 0), on the caller's stream.
static void ensure_transpose(hbgs_ctx* c, hipStream_t s) {
  if (!c->apt_fresh) gather_apt(c, s);
  if (c->hier_t) return;
  ScratchScope scratch(&c->scratch[HBGS_MAX_FIELDS]);
  StreamScope scope(s);
  for (Field& F : c->F) build_field_T(c, F, s);
  build_rest_T(c, s);
  HBGS_HIP(hipStreamSynchronize(s));
}
#undef HBGS_FOR_ALL

}  // namespace hbgs

// ===================================================================== C ABI
using namespace hbgs;

#define HBGS_API_BEGIN try {
#define HBGS_API_END                                 \
  }                                                  \
  catch (const hbgs::Error& e) {                     \
    return e.code;                                   \
  }                                                  \
  catch (const std::exception& e) {                  \
    hbgs::set_error(std::string("exception: ") + e.what()); \
    return HBGS_EHIP;                                \
  }

extern "C" {

void hbgs_default_options(hbgs_options* o) {
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
  o->coarse_max = 2000;
  o->max_levels = 10;
  o->seed = 0x2602ull;
  o->theta[0] = 0.04;
  o->use_graphs = 0;
  o->setup_concurrent = 1;
  o->block_jacobi = 0;
  o->nested = 0;
  o->inner_restart = 30;
  o->inner_max_iters = 300;
  o->inner_rtol = 1e-6;
  o->ilu_block = 4096;
  o->build_transpose = 1;
}

const char* hbgs_last_error(void) { return g_last_error.c_str(); }

hbgs_status hbgs_setup(hbgs_ctx** out, int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                       const double* val, int32_t n_fields, const int32_t* field_of_row, int32_t tree_len,
                       const int32_t* group_tree, const hbgs_options* opt, void* stream) {
  if (!out) {
    set_error("out is NULL");
    return HBGS_EINVAL;
  }
  *out = nullptr;
  hbgs_ctx* c = nullptr;
  HBGS_API_BEGIN
  hipStream_t s = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  if (n <= 0 || nnz <= 0 || nnz > INT32_MAX) HBGS_FAIL(HBGS_EINVAL, "n and nnz must be positive (nnz < 2^31)");
  if (n_fields < 1 || n_fields > HBGS_MAX_FIELDS) HBGS_FAIL(HBGS_EINVAL, "n_fields out of range");
  if (!rowptr || !col || !val || !field_of_row || !group_tree) HBGS_FAIL(HBGS_EINVAL, "NULL argument");
  {
    // the pattern phase's temporaries (before the build threads' scratch
    // stacks exist) come from HIP's default stream-ordered pool: let it keep
    // freed memory instead of returning it to the device
    int dev = 0;
    hipMemPool_t mp = nullptr;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&mp, dev) == hipSuccess && mp) {
      uint64_t keep = UINT64_MAX;
      (void)hipMemPoolSetAttribute(mp, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
  }
  c = new hbgs_ctx();
  c->noalloc_scratch = scratch_dev();
  if (opt)
    c->o = *opt;
  else
    hbgs_default_options(&c->o);
  validate_options(c->o);
  c->precision = c->o.precision;
  c->m = c->o.restart;
  c->n = n;
  c->nf = n_fields;
  c->nnz = nnz;
  parse_tree(c, group_tree, tree_len);
  // keep the caller's pattern and validate it
  c->rp0 = c->pool.make<int>(n + 1);
  c->ci0 = c->pool.make<int>(nnz);
  HBGS_HIP(hipMemcpyAsync(c->rp0, rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
  HBGS_HIP(hipMemcpyAsync(c->ci0, col, sizeof(int) * nnz, hipMemcpyDeviceToDevice, s));
  int64_t last = 0;
  HBGS_HIP(hipMemcpyAsync(&last, rowptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if ((int)last != nnz) HBGS_FAIL(HBGS_EINVAL, "rowptr[n] != nnz");
  {
    Tmp<int> flags(1);
    HBGS_HIP(hipMemsetAsync(flags.p, 0, sizeof(int), s));
    setup::validate(n, nnz, c->rp0, c->ci0, val, n_fields, field_of_row, flags.p, s);
    int f = 0;
    HBGS_HIP(hipMemcpyAsync(&f, flags.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    if (f & 1) HBGS_FAIL(HBGS_EINVAL, "invalid row pointers");
    if (f & 2) HBGS_FAIL(HBGS_EINVAL, "column index out of range");
    if (f & 4) HBGS_FAIL(HBGS_EINVAL, "columns not strictly increasing within a row");
    if (f & 8) HBGS_FAIL(HBGS_EINVAL, "missing or zero diagonal entry");
    if (f & 16) HBGS_FAIL(HBGS_EINVAL, "field id out of range");
    if (f & 32) HBGS_FAIL(HBGS_EINVAL, "non-finite matrix value");
  }
  // field-major permutation in depth-first leaf order
  std::vector<int> counts(n_fields);
  {
    Tmp<int> dc(n_fields);
    setup::field_histogram(n, field_of_row, n_fields, dc.p, s);
    HBGS_HIP(hipMemcpyAsync(counts.data(), dc.p, sizeof(int) * n_fields, hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
  }
  c->f_lo.assign(n_fields, 0);
  c->f_hi.assign(n_fields, 0);
  int off = 0;
  for (int f : c->leaf_order) {
    if (counts[f] == 0) HBGS_FAIL(HBGS_EINVAL, "a field has no rows");
    c->f_lo[f] = off;
    off += counts[f];
    c->f_hi[f] = off;
  }
  c->perm = c->pool.make<int>(n);
  c->iperm = c->pool.make<int>(n);
  setup::field_ranks_all(n, field_of_row, n_fields, c->f_lo.data(), c->perm, s);
  setup::invert_perm(n, c->perm, c->iperm, s);
  {
    Tmp<int> len(n);
    setup::permuted_lengths(n, c->rp0, c->perm, len.p, s);
    c->Ap.n = c->Ap.m = n;
    c->Ap.rp = c->pool.make<int>(n + 1);
    c->Ap.nnz = setup::counts_to_rowptr(len.p, c->Ap.rp, n, s);
    c->Ap.ci = c->pool.make<int>(nnz);
    c->Ap.v = c->pool.make<double>(nnz);
    c->src = c->pool.make<int>(nnz);
    setup::permute_fill(n, c->rp0, c->ci0, val, c->perm, c->iperm, c->Ap.rp, c->Ap.ci, c->Ap.v, c->src, s);
  }
  // A_p^T, and for each of its entries the caller's value index (so that a
  // value update is two gathers)
  {
    Tmp<double> pos(nnz);
    k_iota_f64<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, pos.p);
    HBGS_HIP(hipGetLastError());
    DCsr idx = c->Ap;
    idx.v = pos.p;
    c->ApT = transpose_new(c->pool, idx, s);
    c->posT = c->pool.make<int>(nnz);
    k_pos_int<<<grid_for(nnz, 256), 256, 0, s>>>(nnz, c->ApT.v, c->posT);
    HBGS_HIP(hipGetLastError());
    if (c->o.build_transpose) gather_apt(c, s);  // else on first use
  }
  setup::row_stats(c->Ap, s);
  setup::row_stats(c->ApT, s);
  setup::pack_columns(c->pool, c->Ap, s);
  setup::pack_columns(c->pool, c->ApT, s);
  for (DCsr* a : {&c->Ap, &c->ApT}) setup::build_tiles(c->pool, *a, solve::rows_per_block(*a, solve::ROWS_CAP_F64, true), s);
  build_values(c, s);
  c->stats.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = c;
  return HBGS_OK;
  }
  catch (const hbgs::Error& e) {
    delete c;
    return e.code;
  }
  catch (const std::exception& e) {
    delete c;
    hbgs::set_error(std::string("exception: ") + e.what());
    return HBGS_EHIP;
  }
}


hbgs_status hbgs_set_values(hbgs_ctx* c, const double* val, int32_t rebuild_hierarchy, void* stream) {
  if (!c || !val) {
    set_error("NULL argument");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  hipStream_t s = (hipStream_t)stream;
  auto t0 = std::chrono::steady_clock::now();
  // a kept hierarchy keeps its adjoint consistent with it: its transposed
  // parts are built from the old values before they change
  if (!rebuild_hierarchy && !c->hier_t) ensure_transpose(c, s);
  k_gather_vals<<<grid_for(c->nnz, 256), 256, 0, s>>>(c->nnz, val, c->src, c->Ap.v);
  HBGS_HIP(hipGetLastError());
  c->apt_fresh = false;
  if (c->o.build_transpose) gather_apt(c, s);
  if (rebuild_hierarchy) {
    build_values(c, s);
    c->stats.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  } else {
    HBGS_HIP(hipStreamSynchronize(s));
  }
  return HBGS_OK;
  HBGS_API_END
}

hbgs_status hbgs_set_precision(hbgs_ctx* c, int32_t precision) {
  if (!c || (precision != 0 && precision != 1)) {
    set_error("invalid precision");
    return HBGS_EINVAL;
  }
  c->precision = precision;
  return HBGS_OK;
}

hbgs_status hbgs_set_tolerance(hbgs_ctx* c, double rtol, int32_t max_iters) {
  if (!c || !(rtol >= 0.0) || max_iters < 0) {
    set_error("invalid tolerance");
    return HBGS_EINVAL;
  }
  c->o.rtol = rtol;
  c->o.max_iters = max_iters;
  return HBGS_OK;
}

hbgs_status hbgs_apply(hbgs_ctx* c, const double* r, double* z, int32_t transpose, void* stream) {
  if (!c || !r || !z) {
    set_error("NULL argument");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  hipStream_t s = (hipStream_t)stream;
  ensure_workspace(c);
  if (transpose) ensure_transpose(c, s);
  Krylov& K = c->K;
  solve::permute_in(c->n, c->perm, r, K.bp, s);
  apply_perm(c, transpose ? 1 : 0, K.bp, 0, nullptr, s);
  if (c->precision == 1)  // the FP32 result, widened as it is permuted back
    solve::permute_out_f32(c->n, c->perm, K.Zf, z, s);
  else
    solve::permute_out(c->n, c->perm, K.Zd, z, s);
  HBGS_HIP(hipStreamSynchronize(s));
  return HBGS_OK;
  HBGS_API_END
}

hbgs_status hbgs_apply_noalloc(hbgs_ctx* c, const double* r, double* z, int32_t transpose, void* stream) {
  if (!c || !r || !z) {
    set_error("NULL argument");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  hipStream_t s = (hipStream_t)stream;
  if ((int64_t)c->n > kNoAllocMaxRows)
    HBGS_FAIL(HBGS_EINVAL, "hbgs_apply_noalloc: " + std::to_string(c->n) + " rows exceed the fixed buffer's " +
                               std::to_string(kNoAllocMaxRows) + "; use hbgs_apply");
  if (c->o.nested) HBGS_FAIL(HBGS_EINVAL, "hbgs_apply_noalloc: the nested form needs the inner solvers' workspace");
  if (transpose && !(c->apt_fresh && c->hier_t))
    HBGS_FAIL(HBGS_EINVAL, "hbgs_apply_noalloc: the adjoint's operators are not built (build_transpose = 0 "
                           "and no transpose call since the last setup or value update)");
  if (!c->noalloc_scratch) HBGS_FAIL(HBGS_EHIP, "hbgs_apply_noalloc: no fixed scratch buffer");
  // [0, 8n): the permuted input; then the output column, 256-byte aligned;
  // both are written in full before they are read
  char* base = static_cast<char*>(c->noalloc_scratch);
  double* vp = reinterpret_cast<double*>(base);
  void* zp = base + ((size_t)c->n * sizeof(double) + 255) / 256 * 256;
  solve::permute_in(c->n, c->perm, r, vp, s);
  const int tr = transpose ? 1 : 0;
  if (c->precision == 1) {
    sweep<float>(c, c->plan[tr], tr, vp, static_cast<float*>(zp), 0, nullptr, s);
    solve::permute_out_f32(c->n, c->perm, static_cast<const float*>(zp), z, s);
  } else {
    sweep<double>(c, c->plan[tr], tr, vp, static_cast<double*>(zp), 0, nullptr, s);
    solve::permute_out(c->n, c->perm, static_cast<const double*>(zp), z, s);
  }
  return HBGS_OK;
  HBGS_API_END
}

hbgs_status hbgs_solve(hbgs_ctx* c, const double* b, double* x, int32_t use_x0, int32_t transpose, int32_t* iters,
                       double* hist, int32_t hist_cap, int32_t* hist_len, void* stream) {
  if (!c || !b || !x) {
    set_error("NULL argument");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  hipStream_t us = (hipStream_t)stream;
  ensure_workspace(c);
  int32_t it = 0, hl = 0;
  // work on the context's own stream, ordered after the caller's stream
  hipStream_t s = c->sm;
  HBGS_HIP(hipEventRecord(c->join_in, us));
  HBGS_HIP(hipStreamWaitEvent(s, c->join_in, 0));
  if (transpose) ensure_transpose(c, s);
  solve::permute_in(c->n, c->perm, b, c->K.bp, s);
  if (use_x0) solve::permute_in(c->n, c->perm, x, c->K.xp, s);
  hbgs_status st = gmres(c, transpose ? 1 : 0, use_x0, &it, hist, hist_cap, &hl, s);
  solve::permute_out(c->n, c->perm, c->K.xp, x, s);
  HBGS_HIP(hipEventRecord(c->join_out, s));
  HBGS_HIP(hipStreamWaitEvent(us, c->join_out, 0));
  HBGS_HIP(hipStreamSynchronize(us));
  if (c->prof.on) c->prof.flush();
  if (iters) *iters = it;
  if (hist_len) *hist_len = hl;
  return st;
  HBGS_API_END
}

hbgs_status hbgs_grad_values(hbgs_ctx* c, const double* lambda, const double* x, double* grad_val, void* stream) {
  if (!c || !lambda || !x || !grad_val) {
    set_error("NULL argument");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  solve::grad_values(c->n, c->rp0, c->ci0, lambda, x, grad_val, (hipStream_t)stream);
  return HBGS_OK;
  HBGS_API_END
}

hbgs_status hbgs_stats(hbgs_ctx* c, hbgs_stats_t* out) {
  if (!c || !out) {
    set_error("NULL argument");
    return HBGS_EINVAL;
  }
  *out = c->stats;
  return HBGS_OK;
}

hbgs_status hbgs_get_level(hbgs_ctx* c, int32_t field, int32_t level, int32_t which, int32_t* n_rows,
                           int32_t* n_cols, int64_t* nnz, int32_t* rowptr, int32_t* col, double* val) {
  if (!c || field < 0 || field >= c->nf || level < 0 || level >= (int)c->F[field].lv.size() || which < 0 ||
      which > 3) {
    set_error("invalid field/level/which");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  if (which == 3) ensure_transpose(c, nullptr);
  const Level& L = c->F[field].lv[level];
  bool coarsest = level + 1 == (int)c->F[field].lv.size();
  if ((which == 1 || which == 2) && coarsest) HBGS_FAIL(HBGS_EINVAL, "the coarsest level has no transfer operators");
  const DCsr& a = which == 0 ? L.A : which == 1 ? L.P : which == 2 ? L.R : L.AT;
  if (!a.rp || !a.v) HBGS_FAIL(HBGS_EINVAL, "this operator is not built for the field's leaf solver");
  if (n_rows) *n_rows = a.n;
  if (n_cols) *n_cols = a.m;
  if (nnz) *nnz = a.nnz;
  if (rowptr) HBGS_HIP(hipMemcpy(rowptr, a.rp, sizeof(int) * (a.n + 1), hipMemcpyDeviceToHost));
  if (col) HBGS_HIP(hipMemcpy(col, a.ci, sizeof(int) * a.nnz, hipMemcpyDeviceToHost));
  if (val) HBGS_HIP(hipMemcpy(val, a.v, sizeof(double) * a.nnz, hipMemcpyDeviceToHost));
  return HBGS_OK;
  HBGS_API_END
}

hbgs_status hbgs_get_aggregates(hbgs_ctx* c, int32_t field, int32_t level, int32_t* agg, double* out3) {
  if (!c || field < 0 || field >= c->nf || level < 0 || level >= (int)c->F[field].lv.size()) {
    set_error("invalid field/level");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  const Level& L = c->F[field].lv[level];
  if (agg) {
    if (!L.agg) HBGS_FAIL(HBGS_EINVAL, "the coarsest level has no aggregates");
    HBGS_HIP(hipMemcpy(agg, L.agg, sizeof(int) * L.A.n, hipMemcpyDeviceToHost));
  }
  if (out3) {
    out3[0] = L.lam_cheb;
    out3[1] = L.lam_p;
    out3[2] = L.omega;
  }
  return HBGS_OK;
  HBGS_API_END
}

hbgs_status hbgs_profile(hbgs_ctx* c, int32_t enable) {
  if (!c) {
    set_error("NULL context");
    return HBGS_EINVAL;
  }
  HBGS_API_BEGIN
  c->prof.flush();
  uint32_t mask = enable == -1 ? 0xFFFFFFFFu : (uint32_t)enable;
  c->prof.on = enable != 0;
  c->prof.mask = mask;
  if (enable) {
    std::fill(std::begin(c->prof.total_ms), std::end(c->prof.total_ms), 0.0);
    std::fill(std::begin(c->prof.launches), std::end(c->prof.launches), 0);
    std::fill(std::begin(c->prof.bytes), std::end(c->prof.bytes), 0.0);
  }
  return HBGS_OK;
  HBGS_API_END
}

int32_t hbgs_kernel_times(hbgs_ctx* c, char (*names)[48], double* total_ms, int64_t* launches, double* bytes,
                          int32_t cap) {
  if (!c) return 0;
  try {
    c->prof.flush();
  } catch (const hbgs::Error&) {
    return -1;
  }
  int k = 0;
  for (int q = 0; q < solve::K_COUNT && k < cap; ++q) {
    if (names) {
      std::strncpy(names[k], solve::kind_names[q], 47);
      names[k][47] = 0;
    }
    if (total_ms) total_ms[k] = c->prof.total_ms[q];
    if (launches) launches[k] = c->prof.launches[q];
    if (bytes) bytes[k] = c->prof.bytes[q];
    ++k;
  }
  return k;
}

hbgs_status hbgs_debug_spgemm_route(int32_t route) {
  if (route < 0 || route > 3) {
    set_error("spgemm route must be 0, 1, 2 or 3");
    return HBGS_EINVAL;
  }
  setup::set_spgemm_route(route);
  return HBGS_OK;
}

hbgs_status hbgs_debug_spmv_tiles(int32_t on) {
  if (on != 0 && on != 1) {
    set_error("spmv tiles switch must be 0 or 1");
    return HBGS_EINVAL;
  }
  solve::set_tiles(on != 0);
  return HBGS_OK;
}

hbgs_status hbgs_set_allocator(void* (*alloc)(size_t, void*), void (*free_fn)(void*, void*), void* user) {
  if ((alloc == nullptr) != (free_fn == nullptr)) {
    set_error("hbgs_set_allocator: give both functions or neither");
    return HBGS_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.free = free_fn;
  g_alloc.user = alloc ? user : nullptr;
  return HBGS_OK;
}

void hbgs_destroy(hbgs_ctx* c) { delete c; }

}  // extern "C"
