// Device setup of the block Gauss-Seidel / SA-AMG preconditioner (gfx950).
//
// Built with -ffp-contract=off: every floating-point value below is produced
// by the sequential, rounded-product-then-add evaluation that the method's
// definitions state (ascending column order within a row), so aggregates,
// sparsity patterns and hierarchy values are reproducible bit for bit.
// Parallelism comes from rows: a row has one thread, or a group of lanes
// that read its entries with coalesced loads and combine them with
// cross-lane shuffles, adding order-dependent sums in entry order.  Only
// integer decisions and order-independent max reductions use atomics.
#include <atomic>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hbgs_internal.h"

namespace hbgs {
namespace setup {

constexpr int BLK = 256;
constexpr int SCAN_PER_THREAD = 4;
constexpr int SCAN_TILE = BLK * SCAN_PER_THREAD;

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// aggregation priority: hash32(i ^ salt) << 32 | i (distinct per row)
__device__ __forceinline__ uint64_t agg_key(int i, uint64_t salt) {
  uint64_t h = splitmix64((uint64_t)(uint32_t)i ^ salt) >> 32;
  return (h << 32) | (uint64_t)(uint32_t)i;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------- row groups
// Rows of n handled by groups of L lanes (grid-stride over row groups); gl
// is the lane's index in its group.  Every lane of a group runs the same
// iterations, so the group's shuffles below always see their whole group.
#define ROW_GROUPS(L, i, gl, n)                                                       \
  const int gl = (int)(threadIdx.x % (L));                                             \
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / (L); i < (n); \
       i += (int64_t)gridDim.x * blockDim.x / (L))

template <int L, class T>
__device__ __forceinline__ T grp_max(T x) {
  for (int off = L >> 1; off > 0; off >>= 1) {
    const T o = __shfl_xor(x, off, L);
    x = o > x ? o : x;
  }
  return x;
}
template <int L, class T>
__device__ __forceinline__ T grp_min(T x) {
  for (int off = L >> 1; off > 0; off >>= 1) {
    const T o = __shfl_xor(x, off, L);
    x = o < x ? o : x;
  }
  return x;
}
template <int L>
__device__ __forceinline__ int grp_sum(int x) {
  for (int off = L >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, L);
  return x;
}
// s + (the x of the group's lanes with take set, added one by one in lane
// order): the sequential sum over a row's entries, L entries at a time
template <int L>
__device__ __forceinline__ double grp_ordered_add(double s, double x, bool take) {
  const uint64_t b = __ballot(take);
  const int lane = (int)(threadIdx.x & 63), base = lane & ~(L - 1);
  uint64_t g = L == 64 ? b : (b >> base) & ((1ull << (L & 63)) - 1);
  while (g) {  // the group's takers, lowest lane first
    const int j = __builtin_ctzll(g);
    s += __shfl(x, j, L);
    g &= g - 1;
  }
  return s;
}
// number of lanes below this one in the group with pred set; *total: in the group
template <int L>
__device__ __forceinline__ int grp_rank(bool pred, int* total) {
  const uint64_t b = __ballot(pred);
  const int lane = (int)(threadIdx.x & 63), base = lane & ~(L - 1);
  const uint64_t g = L == 64 ? b : (b >> base) & ((1ull << (L & 63)) - 1);
  *total = __popcll(g);
  return __popcll(g & ((1ull << (lane - base)) - 1));
}

// lanes per row from the mean row length
static int row_lanes(int64_t n, int64_t nnz) {
  const double avg = n ? (double)nnz / (double)n : 0.0;
  return avg <= 7.5 ? 8 : avg <= 15.0 ? 16 : 32;
}
#define LAUNCH_ROW_GROUPS(kern, L, nrows, s, ...) LAUNCH_ROW_GROUPS_CAP(kern, L, nrows, 1 << 20, s, __VA_ARGS__)
// cap: most blocks (kernels that end in one atomic per block use a small cap)
#define LAUNCH_ROW_GROUPS_CAP(kern, L, nrows, cap, s, ...)            \
  do {                                                                 \
    const unsigned g_ = grid_for((int64_t)(nrows) * (L), BLK, cap);    \
    switch (L) {                                                       \
      case 8: kern<8><<<g_, BLK, 0, s>>>(__VA_ARGS__); break;          \
      case 16: kern<16><<<g_, BLK, 0, s>>>(__VA_ARGS__); break;        \
      default: kern<32><<<g_, BLK, 0, s>>>(__VA_ARGS__); break;        \
    }                                                                  \
    HBGS_HIP(hipGetLastError());                                       \
  } while (0)

// ------------------------------------------------------------------ scans
// Exclusive scan in tiles of 1024: tile sums, scan of the tile sums
// (recursive), then a block-local scan with the tile offset.  Integers only.
template <class TI>
__global__ void k_tile_sums(const TI* in, int64_t n, int64_t* tsum) {
  __shared__ int64_t sh[BLK];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
  int64_t acc = 0;
  for (int q = 0; q < SCAN_PER_THREAD; ++q)
    if (base + q < n) acc += (int64_t)in[base + q];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = BLK / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) tsum[blockIdx.x] = sh[0];
}

template <class TI, class TO>
__global__ void k_tile_scan(const TI* in, int64_t n, const int64_t* toff, TO* out) {
  __shared__ int64_t sh[BLK];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PER_THREAD;
  int64_t v[SCAN_PER_THREAD];
  int64_t acc = 0;
  for (int q = 0; q < SCAN_PER_THREAD; ++q) {
    v[q] = base + q < n ? (int64_t)in[base + q] : 0;
    acc += v[q];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  // inclusive Hillis-Steele scan of the per-thread sums
  for (int s = 1; s < BLK; s <<= 1) {
    int64_t t = (int)threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = toff[blockIdx.x] + sh[threadIdx.x] - acc;
  for (int q = 0; q < SCAN_PER_THREAD; ++q) {
    if (base + q < n) out[base + q] = (TO)run;
    run += v[q];
  }
}

template <class TO>
__global__ void k_scan_total(const int64_t* toff, int64_t ntiles, int64_t n, TO* out) {
  out[n] = (TO)toff[ntiles];
}

// out[0..n] exclusive prefix of in[0..n-1] (out[n] = total); toff scratch
template <class TI, class TO>
static int64_t scan_impl(const TI* in, TO* out, int64_t n, hipStream_t s) {
  if (n == 0) {
    TO z = 0;
    HBGS_HIP(hipMemcpyAsync(out, &z, sizeof(TO), hipMemcpyHostToDevice, s));
    HBGS_HIP(hipStreamSynchronize(s));
    return 0;
  }
  int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  Tmp<int64_t> tsum(nt), toff(nt + 1);
  k_tile_sums<TI><<<(unsigned)nt, BLK, 0, s>>>(in, n, tsum.p);
  HBGS_HIP(hipGetLastError());
  if (nt == 1) {
    int64_t h[2] = {0, 0};
    HBGS_HIP(hipMemcpyAsync(&h[1], tsum.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    HBGS_HIP(hipMemcpyAsync(toff.p, h, 2 * sizeof(int64_t), hipMemcpyHostToDevice, s));
  } else {
    scan_impl<int64_t, int64_t>(tsum.p, toff.p, nt, s);
  }
  k_tile_scan<TI, TO><<<(unsigned)nt, BLK, 0, s>>>(in, n, toff.p, out);
  HBGS_HIP(hipGetLastError());
  k_scan_total<TO><<<1, 1, 0, s>>>(toff.p, nt, n, out);
  HBGS_HIP(hipGetLastError());
  int64_t total = 0;
  HBGS_HIP(hipMemcpyAsync(&total, toff.p + nt, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  return total;
}

int64_t scan_i32_to_i64(const int* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int, int64_t>(in, out, n, s);
}
int64_t scan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  return scan_impl<int64_t, int64_t>(in, out, n, s);
}
int64_t counts_to_rowptr(const int* counts, int* rp, int n, hipStream_t s) {
  return scan_impl<int, int>(counts, rp, n, s);
}

// --------------------------------------------------------------- validate
// flags bit 0: bad row pointers, 1: column out of range, 2: unsorted or
// duplicate columns, 3: missing or zero diagonal, 4: field id out of range,
// 5: non-finite value
__global__ void k_validate(int n, int64_t nnz, const int* rp, const int* ci, const double* v, int nf,
                           const int* field, int* flags) {
  GRID_STRIDE(i, n) {
    int f = 0;
    int s = rp[i], e = rp[i + 1];
    if (s < 0 || e < s || (int64_t)e > nnz) {
      atomicOr(flags, 1);
      continue;
    }
    bool diag = false;
    for (int k = s; k < e; ++k) {
      int c = ci[k];
      if (c < 0 || c >= n) f |= 2;
      if (k > s && c <= ci[k - 1]) f |= 4;
      if (c == i && v[k] != 0.0) diag = true;
      if (!isfinite(v[k])) f |= 32;
    }
    if (!diag) f |= 8;
    if (field[i] < 0 || field[i] >= nf) f |= 16;
    if (f) atomicOr(flags, f);
  }
}

void validate(int n, int64_t nnz, const int* rp, const int* ci, const double* v, int nf, const int* field,
              int* flags, hipStream_t s) {
  k_validate<<<grid_for(n, BLK, 65536), BLK, 0, s>>>(n, nnz, rp, ci, v, nf, field, flags);
  HBGS_HIP(hipGetLastError());
}

// ------------------------------------------------------------ permutation
__global__ void k_field_hist(int n, const int* field, int nf, int* counts) {
  __shared__ int sh[HBGS_MAX_FIELDS];
  if (threadIdx.x < HBGS_MAX_FIELDS) sh[threadIdx.x] = 0;
  __syncthreads();
  GRID_STRIDE(i, n) atomicAdd(&sh[field[i]], 1);
  __syncthreads();
  if ((int)threadIdx.x < nf) atomicAdd(&counts[threadIdx.x], sh[threadIdx.x]);
}

void field_histogram(int n, const int* field, int nf, int* counts, hipStream_t s) {
  HBGS_HIP(hipMemsetAsync(counts, 0, nf * sizeof(int), s));
  k_field_hist<<<grid_for(n, BLK, 4096), BLK, 0, s>>>(n, field, nf, counts);
  HBGS_HIP(hipGetLastError());
}

__global__ void k_flag_field(int n, const int* field, int f, int* flag) {
  GRID_STRIDE(i, n) flag[i] = field[i] == f ? 1 : 0;
}

__global__ void k_perm_from_rank(int n, const int* field, int f, int lo, const int64_t* rank, int* perm) {
  GRID_STRIDE(i, n) if (field[i] == f) perm[i] = lo + (int)rank[i];
}

void field_ranks_all(int n, const int* field, int nf, const int* f_lo_host, int* perm, hipStream_t s) {
  Tmp<int> flag(n);
  Tmp<int64_t> rank(n + 1);
  for (int f = 0; f < nf; ++f) {
    k_flag_field<<<grid_for(n, BLK), BLK, 0, s>>>(n, field, f, flag.p);
    HBGS_HIP(hipGetLastError());
    scan_i32_to_i64(flag.p, rank.p, n, s);
    k_perm_from_rank<<<grid_for(n, BLK), BLK, 0, s>>>(n, field, f, f_lo_host[f], rank.p, perm);
    HBGS_HIP(hipGetLastError());
  }
}

__global__ void k_invert_perm(int n, const int* perm, int* iperm) {
  GRID_STRIDE(i, n) iperm[perm[i]] = (int)i;
}
void invert_perm(int n, const int* perm, int* iperm, hipStream_t s) {
  k_invert_perm<<<grid_for(n, BLK), BLK, 0, s>>>(n, perm, iperm);
  HBGS_HIP(hipGetLastError());
}

__global__ void k_perm_len(int n, const int* rp, const int* perm, int* len) {
  GRID_STRIDE(i, n) len[perm[i]] = rp[i + 1] - rp[i];
}
void permuted_lengths(int n, const int* rp, const int* perm, int* len, hipStream_t s) {
  k_perm_len<<<grid_for(n, BLK), BLK, 0, s>>>(n, rp, perm, len);
  HBGS_HIP(hipGetLastError());
}

// row p of P A P^T: old row iperm[p] with columns mapped and re-sorted
// (insertion sort carrying value and source position)
__global__ void k_permute_fill(int n, const int* rp, const int* ci, const double* v, const int* perm,
                               const int* iperm, const int* rp_p, int* ci_p, double* v_p, int* pos_p) {
  GRID_STRIDE(p, n) {
    int i = iperm[p];
    int s = rp[i], e = rp[i + 1], o = rp_p[p];
    for (int k = s; k < e; ++k) {
      int c = perm[ci[k]];
      double x = v[k];
      int src = k;
      int q = o + (k - s) - 1;
      while (q >= o && ci_p[q] > c) {
        ci_p[q + 1] = ci_p[q];
        v_p[q + 1] = v_p[q];
        pos_p[q + 1] = pos_p[q];
        --q;
      }
      ci_p[q + 1] = c;
      v_p[q + 1] = x;
      pos_p[q + 1] = src;
    }
  }
}

// pos_p[q] holds the source entry of permuted entry q; invert it
__global__ void k_invert_pos(int64_t nnz, int* pos_p, int* tmp) {
  GRID_STRIDE(q, nnz) tmp[pos_p[q]] = (int)q;
}

void permute_fill(int n, const int* rp, const int* ci, const double* v, const int* perm, const int* iperm,
                  const int* rp_p, int* ci_p, double* v_p, int* pos_p, hipStream_t s) {
  k_permute_fill<<<grid_for(n, BLK), BLK, 0, s>>>(n, rp, ci, v, perm, iperm, rp_p, ci_p, v_p, pos_p);
  HBGS_HIP(hipGetLastError());
}

__global__ void k_scatter_values(int64_t nnz, const double* v, const int* pos, double* v_p) {
  GRID_STRIDE(k, nnz) v_p[pos[k]] = v[k];
}
void scatter_values(int64_t nnz, const double* v, const int* pos, double* v_p, hipStream_t s) {
  k_scatter_values<<<grid_for(nnz, BLK), BLK, 0, s>>>(nnz, v, pos, v_p);
  HBGS_HIP(hipGetLastError());
}

// --------------------------------------------------------------- transpose
__global__ void k_col_count(int64_t nnz, const int* ci, int* cnt) {
  GRID_STRIDE(k, nnz) atomicAdd(&cnt[ci[k]], 1);
}
template <int L>
__global__ void k_transpose_scatter(int n, const int* rp, const int* ci, const double* v, int* cursor,
                                    int* tci, double* tv) {
  ROW_GROUPS(L, i, gl, n) {
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L) {
      const int q = atomicAdd(&cursor[ci[k]], 1);
      tci[q] = (int)i;
      if (v) tv[q] = v[k];
    }
  }
}
// sort each row by column (entries are distinct, so the result is unique);
// rows of up to SORT_LDS entries are sorted in a per-thread LDS segment,
// longer rows are listed and sorted one block per row
constexpr int SORT_LDS = 32;
constexpr int SORT_BLK = 64;
constexpr int LONG_LDS = 2048;
__global__ __launch_bounds__(SORT_BLK) void k_sort_rows_lds(int n, const int* rp, int* ci, double* v,
                                                            int* n_long, int* long_rows) {
  __shared__ int sc[SORT_BLK][SORT_LDS + 1];
  __shared__ double sv[SORT_BLK][SORT_LDS + 1];
  int i = blockIdx.x * SORT_BLK + threadIdx.x;
  if (i >= n) return;
  int s = rp[i], e = rp[i + 1], len = e - s;
  if (len > SORT_LDS) {
    long_rows[atomicAdd(n_long, 1)] = i;
    return;
  }
  int* c = sc[threadIdx.x];
  double* x = sv[threadIdx.x];
  for (int k = 0; k < len; ++k) {
    int cc = ci[s + k];
    double xx = v ? v[s + k] : 0.0;
    int q = k - 1;
    while (q >= 0 && c[q] > cc) {
      c[q + 1] = c[q];
      x[q + 1] = x[q];
      --q;
    }
    c[q + 1] = cc;
    x[q + 1] = xx;
  }
  for (int k = 0; k < len; ++k) {
    ci[s + k] = c[k];
    if (v) v[s + k] = x[k];
  }
}

// one block per listed row of up to LONG_LDS entries: every entry's
// destination is its rank (the number of smaller columns in the row)
__global__ __launch_bounds__(BLK) void k_sort_long_rows(const int* rows, const int* rp, int* ci, double* v) {
  __shared__ int sc[LONG_LDS];
  __shared__ double sv[LONG_LDS];
  const int row = rows[blockIdx.x];
  const int s = rp[row], len = rp[row + 1] - s;
  if (len > LONG_LDS) return;
  for (int k = threadIdx.x; k < len; k += BLK) {
    sc[k] = ci[s + k];
    sv[k] = v ? v[s + k] : 0.0;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < len; k += BLK) {
    const int c = sc[k];
    int rank = 0;
    for (int q = 0; q < len; ++q) rank += sc[q] < c;
    ci[s + rank] = c;
    if (v) v[s + rank] = sv[k];
  }
}

// rows longer than LONG_LDS: insertion sort by one thread per listed row
__global__ void k_sort_huge_rows(int cnt, const int* rows, const int* rp, int* ci, double* v) {
  GRID_STRIDE(t, cnt) {
    const int i = rows[t];
    int s = rp[i], e = rp[i + 1];
    if (e - s <= LONG_LDS) continue;
    for (int k = s + 1; k < e; ++k) {
      int c = ci[k];
      double x = v ? v[k] : 0.0;
      int q = k - 1;
      while (q >= s && ci[q] > c) {
        ci[q + 1] = ci[q];
        if (v) v[q + 1] = v[q];
        --q;
      }
      ci[q + 1] = c;
      if (v) v[q + 1] = x;
    }
  }
}

void sort_rows(const DCsr& a, hipStream_t s) {
  if (a.n == 0) return;
  Tmp<int> n_long(1), long_rows(a.n);
  HBGS_HIP(hipMemsetAsync(n_long.p, 0, sizeof(int), s));
  k_sort_rows_lds<<<grid_for(a.n, SORT_BLK), SORT_BLK, 0, s>>>(a.n, a.rp, a.ci, a.v, n_long.p, long_rows.p);
  HBGS_HIP(hipGetLastError());
  int nl = 0;
  HBGS_HIP(hipMemcpyAsync(&nl, n_long.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (nl > 0) {
    k_sort_long_rows<<<nl, BLK, 0, s>>>(long_rows.p, a.rp, a.ci, a.v);
    HBGS_HIP(hipGetLastError());
    k_sort_huge_rows<<<grid_for(nl, BLK), BLK, 0, s>>>(nl, long_rows.p, a.rp, a.ci, a.v);
    HBGS_HIP(hipGetLastError());
  }
}

void transpose(const DCsr& a, DCsr& t, hipStream_t s) {
  t.n = a.m;
  t.m = a.n;
  t.nnz = a.nnz;
  Tmp<int> cnt(a.m);
  HBGS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * a.m, s));
  k_col_count<<<grid_for(a.nnz, BLK), BLK, 0, s>>>(a.nnz, a.ci, cnt.p);
  HBGS_HIP(hipGetLastError());
  counts_to_rowptr(cnt.p, t.rp, a.m, s);
  HBGS_HIP(hipMemcpyAsync(cnt.p, t.rp, sizeof(int) * a.m, hipMemcpyDeviceToDevice, s));
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_transpose_scatter, L, a.n, s, a.n, a.rp, a.ci, a.v, cnt.p, t.ci, t.v);
  sort_rows(t, s);
  HBGS_HIP(hipStreamSynchronize(s));
}

// ----------------------------------------------------------- block extract
template <int L>
__global__ void k_block_count(int r0, int r1, const int* rp, const int* ci, int c0, int c1, int* cnt) {
  const int64_t m = r1 - r0;
  ROW_GROUPS(L, t, gl, m) {
    const int i = r0 + (int)t;
    int c = 0;
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L) c += (ci[k] >= c0 && ci[k] < c1) ? 1 : 0;
    c = grp_sum<L>(c);
    if (gl == 0) cnt[t] = c;
  }
}
template <int L>
__global__ void k_block_fill(int r0, int r1, const int* rp, const int* ci, const double* v, int c0, int c1,
                             int coff, const int* rpo, int* cio, double* vo) {
  const int64_t m = r1 - r0;
  ROW_GROUPS(L, t, gl, m) {
    const int i = r0 + (int)t, e = rp[i + 1];
    int q = rpo[t];
    for (int b = rp[i]; b < e; b += L) {
      const int k = b + gl;
      const int c = k < e ? ci[k] : -1;
      const bool keep = k < e && c >= c0 && c < c1;
      int tot;
      const int r = grp_rank<L>(keep, &tot);
      if (keep) {
        cio[q + r] = c - coff;
        vo[q + r] = v[k];
      }
      q += tot;
    }
  }
}
void block_count(const DCsr& a, int r0, int r1, int c0, int c1, int* cnt, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_block_count, L, r1 - r0, s, r0, r1, a.rp, a.ci, c0, c1, cnt);
}
void block_fill(const DCsr& a, int r0, int r1, int c0, int c1, int coff, const int* rp_out, int* ci_out,
                double* v_out, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_block_fill, L, r1 - r0, s, r0, r1, a.rp, a.ci, a.v, c0, c1, coff, rp_out, ci_out, v_out);
}

// ---------------------------------------------------------------- strength
template <int L>
__global__ void k_diagonal(int n, const int* rp, const int* ci, const double* v, double* d, int* missing) {
  ROW_GROUPS(L, i, gl, n) {
    int pos = -1;
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L)
      if (ci[k] == (int)i) pos = k;
    pos = grp_max<L>(pos);
    if (gl == 0) {
      const double x = pos >= 0 ? v[pos] : 0.0;
      d[i] = x;
      if (pos < 0 || x == 0.0) atomicOr(missing, 1);
    }
  }
}
void diagonal(const DCsr& a, double* d, int* missing, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_diagonal, L, a.n, s, a.n, a.rp, a.ci, a.v, d, missing);
}

// (i,j) strong: a_ij*a_ij >= (theta^2 |a_ii|) |a_jj|, or the same test on the
// transposed entry (j,i); rows with no off-diagonal entry are excluded
template <int L>
__global__ void k_strength(int n, const int* rp, const int* ci, const double* v, const double* d, double th2,
                           char* strong, char* excluded) {
  ROW_GROUPS(L, i, gl, n) {
    int offd = 0;
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L) {
      const int j = ci[k];
      if (j == (int)i) {
        strong[k] = 0;
        continue;
      }
      offd = 1;
      bool st = v[k] * v[k] >= (th2 * fabs(d[i])) * fabs(d[j]);
      if (!st) {
        int lo = rp[j], hi = rp[j + 1] - 1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int cm = ci[mid];
          if (cm == (int)i) {
            st = v[mid] * v[mid] >= (th2 * fabs(d[j])) * fabs(d[i]);
            break;
          }
          if (cm < (int)i)
            lo = mid + 1;
          else
            hi = mid - 1;
        }
      }
      strong[k] = st ? 1 : 0;
    }
    offd = grp_max<L>(offd);
    if (gl == 0) excluded[i] = offd ? 0 : 1;
  }
}
void strength(const DCsr& a, const double* d, double theta, char* strong, char* excluded, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_strength, L, a.n, s, a.n, a.rp, a.ci, a.v, d, theta * theta, strong, excluded);
}

// ---------------------------------------------------------------- MIS-2
// Synchronous rounds: an undecided row becomes a root when its key is the
// largest among the undecided rows within strength distance 2 (the maxima
// propagate through all rows, decided or not); rows within distance 2 of a
// root leave.  This yields the greedy maximal distance-2 independent set
// taken in decreasing key order.
__global__ void k_mis2_init(int n, const char* excluded, char* state) {
  GRID_STRIDE(i, n) state[i] = excluded[i] ? 3 : 0;
}
template <int L>
__global__ void k_mis2_max1(int n, const int* rp, const int* ci, const char* strong, uint64_t salt,
                            const char* state, uint64_t* m1) {
  ROW_GROUPS(L, i, gl, n) {
    uint64_t m = (gl == 0 && state[i] == 0) ? agg_key((int)i, salt) : 0;
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L) {
      if (!strong[k]) continue;
      const int j = ci[k];
      if (state[j] == 0) {
        const uint64_t kj = agg_key(j, salt);
        m = kj > m ? kj : m;
      }
    }
    m = grp_max<L>(m);
    if (gl == 0) m1[i] = m;
  }
}
template <int L>
__global__ void k_mis2_max2(int n, const int* rp, const int* ci, const char* strong, uint64_t salt,
                            const uint64_t* m1, char* state) {
  ROW_GROUPS(L, i, gl, n) {
    if (state[i] != 0) continue;
    uint64_t m = m1[i];
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L)
      if (strong[k]) m = m1[ci[k]] > m ? m1[ci[k]] : m;
    m = grp_max<L>(m);
    if (gl == 0 && m == agg_key((int)i, salt)) state[i] = 1;
  }
}
template <int L>
__global__ void k_mis2_near1(int n, const int* rp, const int* ci, const char* strong, const char* state,
                             char* r1) {
  ROW_GROUPS(L, i, gl, n) {
    int r = state[i] == 1;
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L)
      if (strong[k] && state[ci[k]] == 1) r = 1;
    r = grp_max<L>(r);
    if (gl == 0) r1[i] = (char)r;
  }
}
template <int L>
__global__ void k_mis2_near2(int n, const int* rp, const int* ci, const char* strong, const char* r1,
                             char* state, int* undecided) {
  int local = 0;
  ROW_GROUPS(L, i, gl, n) {
    if (state[i] != 0) continue;
    int out = r1[i];
    for (int k = rp[i] + gl; k < rp[i + 1] && !out; k += L)
      if (strong[k] && r1[ci[k]]) out = 1;
    out = grp_max<L>(out);
    if (gl == 0) {
      if (out)
        state[i] = 2;
      else
        ++local;
    }
  }
  // one atomic per block (the grid is capped, so there are few)
  __shared__ int red[BLK / 64];
  for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BLK / 64; ++w) local += red[w];
    if (local) atomicAdd(undecided, local);
  }
}

void mis2_init(int n, const char* excluded, char* state, hipStream_t s) {
  k_mis2_init<<<grid_for(n, BLK), BLK, 0, s>>>(n, excluded, state);
  HBGS_HIP(hipGetLastError());
}

void mis2_round(const DCsr& a, const char* strong, uint64_t salt, char* state, uint64_t* m1, char* r1,
                int* undecided, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_mis2_max1, L, a.n, s, a.n, a.rp, a.ci, strong, salt, state, m1);
  LAUNCH_ROW_GROUPS(k_mis2_max2, L, a.n, s, a.n, a.rp, a.ci, strong, salt, m1, state);
  LAUNCH_ROW_GROUPS(k_mis2_near1, L, a.n, s, a.n, a.rp, a.ci, strong, state, r1);
  HBGS_HIP(hipMemsetAsync(undecided, 0, sizeof(int), s));
  LAUNCH_ROW_GROUPS_CAP(k_mis2_near2, L, a.n, 2048, s, a.n, a.rp, a.ci, strong, r1, state, undecided);
}

__global__ void k_agg_roots(int n, const char* state, int* flag) {
  GRID_STRIDE(i, n) flag[i] = state[i] == 1 ? 1 : 0;
}
void agg_roots(int n, const char* state, int* flag, hipStream_t s) {
  k_agg_roots<<<grid_for(n, BLK), BLK, 0, s>>>(n, state, flag);
  HBGS_HIP(hipGetLastError());
}

// phase 1: a row next to a root joins it (the root is unique: roots are at
// least 3 apart); phase 2: other rows join the phase-1 neighbour of largest
// key; rows left over are flagged for phase 3
template <int L>
__global__ void k_agg_phase1(int n, const int* rp, const int* ci, const char* strong, const char* state,
                             const int64_t* root_rank, int* p1) {
  ROW_GROUPS(L, i, gl, n) {
    int a = -1;
    if (state[i] == 1) {
      a = (int)root_rank[i];
    } else if (state[i] != 3) {
      for (int k = rp[i] + gl; k < rp[i + 1]; k += L)
        if (strong[k] && state[ci[k]] == 1) a = (int)root_rank[ci[k]];
      a = grp_max<L>(a);
    }
    if (gl == 0) p1[i] = a;
  }
}
// the phase-1 neighbour of largest key (keys are distinct, so the maximum
// is the row's unique choice)
template <int L>
__global__ void k_agg_phase2(int n, const int* rp, const int* ci, const char* strong, uint64_t salt,
                             const char* state, const int* p1, int* agg, int* single_flag) {
  ROW_GROUPS(L, i, gl, n) {
    int a = p1[i];
    int single = 0;
    if (state[i] != 3 && a < 0) {
      uint64_t best = 0;
      int bestu = -1;
      for (int k = rp[i] + gl; k < rp[i + 1]; k += L) {
        if (!strong[k]) continue;
        const int u = ci[k];
        if (p1[u] >= 0 && state[u] != 1) {
          const uint64_t ku = agg_key(u, salt);
          if (bestu < 0 || ku > best) {
            best = ku;
            bestu = u;
          }
        }
      }
      const uint64_t top = grp_max<L>(bestu < 0 ? 0ull : best + 1);  // 0: no candidate
      a = top ? p1[(int)(uint32_t)((top - 1) & 0xffffffffull)] : -1;
      single = top ? 0 : 1;
    }
    if (gl == 0) {
      agg[i] = a;
      single_flag[i] = single;
    }
  }
}
__global__ void k_agg_phase3(int n, const int* single_flag, const int64_t* single_rank, int nroot, int* agg) {
  GRID_STRIDE(i, n) if (single_flag[i]) agg[i] = nroot + (int)single_rank[i];
}

void agg_phase12(const DCsr& a, const char* strong, uint64_t salt, const char* state, const int64_t* root_rank,
                 int* agg, int* single_flag, hipStream_t s) {
  Tmp<int> p1(a.n);
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_agg_phase1, L, a.n, s, a.n, a.rp, a.ci, strong, state, root_rank, p1.p);
  LAUNCH_ROW_GROUPS(k_agg_phase2, L, a.n, s, a.n, a.rp, a.ci, strong, salt, state, p1.p, agg, single_flag);
  HBGS_HIP(hipStreamSynchronize(s));
}
void agg_phase3(int n, const int* single_flag, const int64_t* single_rank, int nroot, int* agg, hipStream_t s) {
  k_agg_phase3<<<grid_for(n, BLK), BLK, 0, s>>>(n, single_flag, single_rank, nroot, agg);
  HBGS_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ filter
// A_F: strong off-diagonal entries kept, dropped entries added to the
// diagonal in ascending column order; D_abs = sum |A_F| along the row
template <int L>
__global__ void k_filter_count(int n, const int* rp, const int* ci, const char* strong, int* cnt) {
  ROW_GROUPS(L, i, gl, n) {
    int c = 0;
    for (int k = rp[i] + gl; k < rp[i + 1]; k += L) c += (ci[k] == (int)i || strong[k]) ? 1 : 0;
    c = grp_sum<L>(c);
    if (gl == 0) cnt[i] = c;
  }
}
template <int L>
__global__ void k_filter_fill(int n, const int* rp, const int* ci, const double* v, const char* strong,
                              const int* rpf, int* cif, double* vf, double* dabs) {
  ROW_GROUPS(L, i, gl, n) {
    const int s = rp[i], e = rp[i + 1];
    int pos = -1;
    for (int k = s + gl; k < e; k += L)
      if (ci[k] == (int)i) pos = k;
    pos = grp_max<L>(pos);
    // diagonal of A_F: a_ii, then the dropped entries in column order
    double d = pos >= 0 ? v[pos] : 0.0;
    for (int b = s; b < e; b += L) {
      const int k = b + gl;
      const bool drop = k < e && ci[k] != (int)i && !strong[k];
      d = grp_ordered_add<L>(d, drop ? v[k] : 0.0, drop);
    }
    int q = rpf[i];
    double sa = 0.0;
    for (int b = s; b < e; b += L) {
      const int k = b + gl;
      const int c = k < e ? ci[k] : -1;
      const bool diag = c == (int)i;
      const bool keep = k < e && (diag || strong[k]);
      const double x = keep ? (diag ? d : v[k]) : 0.0;
      int tot;
      const int r = grp_rank<L>(keep, &tot);
      if (keep) {
        cif[q + r] = c;
        vf[q + r] = x;
      }
      q += tot;
      sa = grp_ordered_add<L>(sa, fabs(x), keep);
    }
    if (gl == 0) dabs[i] = sa;
  }
}
void filter_count(const DCsr& a, const char* strong, int* cnt, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_filter_count, L, a.n, s, a.n, a.rp, a.ci, strong, cnt);
}
void filter_fill(const DCsr& a, const char* strong, const int* rp_f, int* ci_f, double* v_f, double* dabs,
                 hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_filter_fill, L, a.n, s, a.n, a.rp, a.ci, a.v, strong, rp_f, ci_f, v_f, dabs);
}

// ------------------------------------------------------------ power method
__global__ void k_pw_init(int n, uint64_t salt, double* w) {
  GRID_STRIDE(i, n) {
    uint64_t h = splitmix64((uint64_t)(uint32_t)i ^ salt);
    w[i] = 2.0 * ((double)(h >> 11) * 0x1.0p-53) - 1.0;
  }
}
// y = D^-1 B w with every row summed in ascending column order; tracks max |y|.
// w is win, or (amax_in set) win scaled by 2^-e with max|win| = f * 2^e,
// f in [0.5, 1), as the power method normalises its iterate (zero if
// max|win| = 0); the scaling is exact, so folding it into the gather gives
// bitwise the products of the scaled vector.  A block of PW_BLK threads
// takes RB rows: its threads stage the products of PW_CH consecutive
// entries at a time in LDS with coalesced loads, then each row's thread
// (the first RB threads) adds its products in order.  Coarse levels (few
// rows of hundreds of entries) take small RB, so they spread over many
// blocks instead of walking many chunks in a few.
constexpr int PW_BLK = 256;
constexpr int PW_CH = 2048;
template <int RB>
__global__ __launch_bounds__(PW_BLK) void k_pw_apply(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ v, const double* __restrict__ d,
                                                     const double* __restrict__ win,
                                                     const unsigned long long* amax_in, double* __restrict__ y,
                                                     unsigned long long* amax) {
  static_assert(RB <= PW_BLK, "one thread per row in the sums");
  __shared__ double prod[PW_CH];
  __shared__ unsigned long long sh[PW_BLK / 64];
  bool scaled = amax_in != nullptr, zero = false;
  int e = 0;
  if (scaled) {
    const double mx = __longlong_as_double((long long)*amax_in);
    if (mx > 0.0)
      frexp(mx, &e);
    else
      zero = true;
  }
  unsigned long long m = 0;
  const int64_t nblk = ((int64_t)n + RB - 1) / RB;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int r0 = (int)(b * RB), r1 = min(r0 + RB, n);
    const int i = r0 + (int)threadIdx.x;
    const bool own = (int)threadIdx.x < RB && i < r1;
    const int e0 = rp[r0], e1 = rp[r1];
    const int my0 = own ? rp[i] : 0, my1 = own ? rp[i + 1] : 0;
    double s = 0.0;
    for (int c0 = e0; c0 < e1; c0 += PW_CH) {
      const int c1 = min(c0 + PW_CH, e1);
      for (int k = c0 + (int)threadIdx.x; k < c1; k += PW_BLK) {
        double w = win[ci[k]];
        if (scaled) w = zero ? 0.0 : ldexp(w, -e);
        prod[k - c0] = v[k] * w;
      }
      __syncthreads();
      const int a = max(my0, c0), z = min(my1, c1);
      for (int k = a; k < z; ++k) s += prod[k - c0];
      __syncthreads();
    }
    if (own) {
      const double yi = d[i] != 0.0 ? s / d[i] : 0.0;  // a zero weight only where the row is zero
      y[i] = yi;
      const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(yi));
      m = bits > m ? bits : m;
    }
  }
  if (!amax) return;
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < PW_BLK / 64; ++q) m = sh[q] > m ? sh[q] : m;
    atomicMax(amax, m);
  }
}
// rows per block: the largest of 256 ... 4 that still gives 1024 blocks
// (4 per CU), else 4; the grid is capped at 2048 blocks (8 per CU, one
// atomicMax each on a single address) that stride over the row blocks
static void pw_apply(const DCsr& b, const double* d, const double* win, const unsigned long long* amax_in,
                     double* y, unsigned long long* amax, hipStream_t s) {
  const int n = b.n;
  int rb = 4;
  for (int r = 256; r >= 4; r >>= 1)
    if (((int64_t)n + r - 1) / r >= 1024) {
      rb = r;
      break;
    }
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(((int64_t)n + rb - 1) / rb, 2048));
#define HBGS_PW(R)                                                                                   \
  case R:                                                                                            \
    k_pw_apply<R><<<g, PW_BLK, 0, s>>>(n, b.rp, b.ci, b.v, d, win, amax_in, y, amax);                \
    break;
  switch (rb) {
    HBGS_PW(256)
    HBGS_PW(128)
    HBGS_PW(64)
    HBGS_PW(32)
    HBGS_PW(16)
    HBGS_PW(8)
    HBGS_PW(4)
  }
#undef HBGS_PW
  HBGS_HIP(hipGetLastError());
}
// w = y * 2^-e with max|y| = f * 2^e, f in [0.5, 1)
__global__ void k_pw_scale(int n, const double* y, const unsigned long long* amax, double* w) {
  double mx = __longlong_as_double((long long)*amax);
  int e = 0;
  if (mx > 0.0) frexp(mx, &e);
  GRID_STRIDE(i, n) w[i] = mx > 0.0 ? ldexp(y[i], -e) : 0.0;
}
// fixed-association sum: consecutive runs of 256 terms summed in order ...
// A block of 256 threads takes 16 runs: it stages their 4096 products in
// LDS with coalesced loads (every load in flight at once), then 16 threads
// add one run each, in index order.  Terms beyond n are staged as +0.0,
// which leaves a sum that starts at +0.0 unchanged.
constexpr int DOT_RUNS = 16;
__global__ __launch_bounds__(256) void k_chunk_dot(int64_t n, const double* x, const double* y, double* part) {
  __shared__ double tile[DOT_RUNS][257];
  const int64_t m = (n + 255) / 256;
  const int t = (int)threadIdx.x;
  for (int64_t c0 = (int64_t)blockIdx.x * DOT_RUNS; c0 < m; c0 += (int64_t)gridDim.x * DOT_RUNS) {
#pragma unroll
    for (int r = 0; r < DOT_RUNS; ++r) {
      const int64_t i = (c0 + r) * 256 + t;
      tile[r][t] = i < n ? x[i] * y[i] : 0.0;
    }
    __syncthreads();
    if (t < DOT_RUNS && c0 + t < m) {
      double s = 0.0;
      for (int j = 0; j < 256; ++j) s += tile[t][j];
      part[c0 + t] = s;
    }
    __syncthreads();
  }
}
// ... then the m run sums added in order: the block stages 1024 of them in
// LDS at a time, one thread adds them
constexpr int RUN_STAGE = 1024;
__global__ void __launch_bounds__(256) k_chunk_total(int64_t m, const double* part, double* out) {
  __shared__ double sh[RUN_STAGE];
  double s = 0.0;
  for (int64_t c0 = 0; c0 < m; c0 += RUN_STAGE) {
    const int e = (int)(m - c0 < RUN_STAGE ? m - c0 : RUN_STAGE);
    for (int t = threadIdx.x; t < e; t += blockDim.x) sh[t] = part[c0 + t];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int t = 0; t < e; ++t) s += sh[t];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s;
}

static double chunked_dot(int64_t n, const double* x, const double* y, double* part, double* out,
                          hipStream_t s) {
  if (n == 0) return 0.0;
  const int64_t m = (n + 255) / 256;
  k_chunk_dot<<<grid_for(m, DOT_RUNS, 2048), 256, 0, s>>>(n, x, y, part);
  HBGS_HIP(hipGetLastError());
  k_chunk_total<<<1, 256, 0, s>>>(m, part, out);
  HBGS_HIP(hipGetLastError());
  double r = 0.0;
  HBGS_HIP(hipMemcpyAsync(&r, out, sizeof(double), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  return r;
}

double power_estimate(const DCsr& b, const double* d, int iters, uint64_t salt, hipStream_t s) {
  const int n = b.n;
  Tmp<double> w(n), y(n), pa((n + 255) / 256 + 1), pb(1);
  Tmp<unsigned long long> amax(iters > 0 ? iters : 1);
  const unsigned g = grid_for(n, BLK);
  k_pw_init<<<g, BLK, 0, s>>>(n, salt, w.p);
  HBGS_HIP(hipGetLastError());
  if (iters > 0) HBGS_HIP(hipMemsetAsync(amax.p, 0, sizeof(unsigned long long) * iters, s));
  // iterate it reads the previous one scaled on the fly: w -> y -> w -> ...
  double* buf[2] = {y.p, w.p};
  for (int it = 0; it < iters; ++it) {
    pw_apply(b, d, buf[(it + 1) & 1], it ? amax.p + it - 1 : nullptr, buf[it & 1], amax.p + it, s);
  }
  const double* wl = w.p;  // the normalised last iterate
  if (iters > 0) {
    unsigned long long mx = 0;
    HBGS_HIP(hipMemcpyAsync(&mx, amax.p + iters - 1, sizeof(mx), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    double m = 0.0;
    std::memcpy(&m, &mx, sizeof(m));
    if (m == 0.0) return 0.0;
    double* last = buf[(iters - 1) & 1];
    double* other = buf[iters & 1];
    k_pw_scale<<<g, BLK, 0, s>>>(n, last, amax.p + iters - 1, other);
    HBGS_HIP(hipGetLastError());
    wl = other;
    pw_apply(b, d, other, nullptr, last, nullptr, s);
    double wy = chunked_dot(n, wl, last, pa.p, pb.p, s);
    double ww = chunked_dot(n, wl, wl, pa.p, pb.p, s);
    return wy / ww;
  }
  pw_apply(b, d, w.p, nullptr, y.p, nullptr, s);
  double wy = chunked_dot(n, w.p, y.p, pa.p, pb.p, s);
  double ww = chunked_dot(n, w.p, w.p, pa.p, pb.p, s);
  return wy / ww;
}

// ------------------------------------------------------ smoothed prolongator
// Row i of P = P_tent - omega D_abs^-1 A_F P_tent: its columns are the
// aggregates met along row i of A_F (ascending); entry c is
// [agg(i)==c] - (omega / D_abs_i) * sum_{k: agg(k)==c} a_F(i,k).
template <int L>
__global__ void k_psmooth_count(int n, const int* rp, const int* ci, const int* agg, int* cnt) {
  ROW_GROUPS(L, i, gl, n) {
    int c = 0;
    if (agg[i] >= 0) {
      const int s = rp[i], e = rp[i + 1];
      int prev = -1;
      for (;;) {
        int next = INT32_MAX;
        for (int k = s + gl; k < e; k += L) {
          const int a = agg[ci[k]];
          if (a > prev && a < next) next = a;
        }
        next = grp_min<L>(next);
        if (next == INT32_MAX) break;
        ++c;
        prev = next;
      }
    }
    if (gl == 0) cnt[i] = c;
  }
}
template <int L>
__global__ void k_psmooth_fill(int n, const int* rp, const int* ci, const double* v, const int* agg,
                               const double* dabs, double omega, const int* rpp, int* cip, double* vp) {
  ROW_GROUPS(L, i, gl, n) {
    const int ai = agg[i];
    if (ai < 0) continue;
    const double q = dabs[i] != 0.0 ? omega / dabs[i] : 0.0;  // a zero row of A_F: no smoothing term
    const int s = rp[i], e = rp[i + 1];
    int o = rpp[i];
    int cur = INT32_MAX;
    for (int k = s + gl; k < e; k += L) {
      const int a = agg[ci[k]];
      if (a >= 0 && a < cur) cur = a;
    }
    cur = grp_min<L>(cur);
    // one pass per aggregate met: its entries summed in column order, and
    // the next larger aggregate
    while (cur != INT32_MAX) {
      double sum = 0.0;
      int next = INT32_MAX;
      for (int b = s; b < e; b += L) {
        const int k = b + gl;
        const int a = k < e ? agg[ci[k]] : -1;
        const bool hit = a == cur;
        sum = grp_ordered_add<L>(sum, hit ? v[k] : 0.0, hit);
        if (a > cur && a < next) next = a;
      }
      next = grp_min<L>(next);
      if (gl == 0) {
        const double tent = ai == cur ? 1.0 : 0.0;
        cip[o] = cur;
        vp[o] = tent - q * sum;
      }
      ++o;
      cur = next;
    }
  }
}
void psmooth_count(const DCsr& af, const int* agg, int* cnt, hipStream_t s) {
  const int L = row_lanes(af.n, af.nnz);
  LAUNCH_ROW_GROUPS(k_psmooth_count, L, af.n, s, af.n, af.rp, af.ci, agg, cnt);
}
void psmooth_fill(const DCsr& af, const int* agg, const double* dabs, double omega, const int* rp_p, int* ci_p,
                  double* v_p, hipStream_t s) {
  const int L = row_lanes(af.n, af.nnz);
  LAUNCH_ROW_GROUPS(k_psmooth_fill, L, af.n, s, af.n, af.rp, af.ci, af.v, agg, dabs, omega, rp_p, ci_p, v_p);
}

// ------------------------------------------------------------------ SpGEMM
// C = A B, Gustavson row by row.  Each row of C owns an open-addressing
// table whose slots accumulate the products a_ik b_kj in the order they are
// generated, i.e. ascending k, starting from 0.0; the occupied slots are
// then written out in column order.  The pattern is structural (entries
// that cancel to zero are kept).
//
// Rows whose tables fit in LDS are done by one wavefront each: the wave
// walks the row of A in order and its lanes take the entries of one row of
// B at a time.  The columns of one B row are distinct, so no two lanes
// update the same slot in one step, and a wave's LDS operations complete in
// program order, so each slot still sums its products in ascending k.  The
// remaining rows use one thread each and a table in global scratch memory.
__global__ void k_spgemm_ub(int n, const int* arp, const int* aci, const int* brp, int64_t* ub) {
  GRID_STRIDE(i, n) {
    int64_t u = 0;
    for (int k = arp[i]; k < arp[i + 1]; ++k) u += brp[aci[k] + 1] - brp[aci[k]];
    ub[i] = u;
  }
}
__host__ __device__ __forceinline__ int64_t table_size(int64_t ub) {
  if (ub == 0) return 0;
  int64_t t = 16;
  while (t < 2 * ub) t <<= 1;
  return t;
}
__device__ __forceinline__ uint32_t hslot(int c, uint32_t mask) { return ((uint32_t)c * 2654435761u) & mask; }

constexpr int SPG_WAVES = 4;          // rows (waves) per block
constexpr int SPG_SYM_SLOTS = 1024;   // symbolic: keys per wave (4 KB: 8 blocks of 4 waves per CU)
constexpr int SPG_NUM_SLOTS = 512;    // numeric: keys and values per wave (6 KB: 6 blocks per CU)
constexpr int SPG_BLK_SLOTS = 4096;  // numeric, one block per row: keys and values (48 KB)
// distinct columns of a product row are at most min(ub, columns of B)
__device__ __forceinline__ int64_t sym_need(int64_t ub, int m) { return ub < m ? ub : (int64_t)m; }

// slot holding key c (claimed if absent); -1 if the table is full, which
// the table sizes rule out (the caller reports it instead of looping);
// lds_claim_bounded gives up after max_probes slots
__device__ __forceinline__ int lds_claim_bounded(int* keys, uint32_t mask, int c, uint32_t max_probes, bool* fresh) {
  uint32_t h = hslot(c, mask);
  for (uint32_t probe = 0; probe < max_probes && probe <= mask; ++probe) {
    int prev = atomicCAS(&keys[h], -1, c);
    if (prev == -1 || prev == c) {
      *fresh = prev == -1;
      return (int)h;
    }
    h = (h + 1) & mask;
  }
  *fresh = false;
  return -1;
}
__device__ __forceinline__ int lds_claim(int* keys, uint32_t mask, int c, bool* fresh) {
  uint32_t h = hslot(c, mask);
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    int prev = atomicCAS(&keys[h], -1, c);
    if (prev == -1 || prev == c) {
      *fresh = prev == -1;
      return (int)h;
    }
    h = (h + 1) & mask;
  }
  *fresh = false;
  return -1;
}

// Groups of LPR lanes (64 / LPR rows per wavefront): a group walks its row
// of A in order and its lanes take the entries of one row of B at a time.
// Each row owns SLOTS / (64 / LPR) table slots.  The narrow kernels
// (LPR < 64) take the rows whose size measure is at most hi and append the
// others to a list for the one-row-per-wavefront kernels, which stride over
// that list (or over every row) with a device-side count (lanes of one
// wavefront stay in lockstep, so the per-slot order argument above holds
// group by group).
__device__ __forceinline__ int group_table(int64_t need) {  // power of two >= 2 need, at least 16
  int t = 16;
  while (t < 2 * need) t <<= 1;
  return t;
}
template <int LPR>
__global__ __launch_bounds__(64 * SPG_WAVES) void k_spgemm_sym_grp(int n, int bm, const int* arp, const int* aci,
                                                                  const int* brp, const int* bci, const int64_t* ub,
                                                                  int64_t hi, int* cnt, int* overflow) {
  constexpr int G = 64 / LPR, SLOTS = SPG_SYM_SLOTS / G;
  static_assert(LPR < 64, "the wide rows use k_spgemm_sym_wave");
  __shared__ int tab[SPG_WAVES][SPG_SYM_SLOTS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane / LPR, gl = lane % LPR;
  const int64_t i = ((int64_t)blockIdx.x * SPG_WAVES + wave) * G + grp;
  const int64_t need = i < n ? sym_need(ub[i], bm) : 0;
  const bool active = i < n && need <= hi && 2 * need <= SLOTS;
  int u = 0;
  if (active) {
    const int T = group_table(need);
    int* keys = tab[wave] + grp * SLOTS;
    for (int q = gl; q < T; q += LPR) keys[q] = -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t mask = (uint32_t)(T - 1);
    const int a0 = arp[i], a1 = arp[i + 1], gbase = grp * LPR;
    // A's row LPR entries at a time: the lanes load the entries' B row
    // bounds together, then take the B rows one after another (the distinct
    // count does not depend on the order)
    for (int c0 = a0; c0 < a1; c0 += LPR) {
      const int kl = c0 + gl;
      int bl0 = 0, bl1 = 0;
      if (kl < a1) {
        const int kk = aci[kl];
        bl0 = brp[kk];
        bl1 = brp[kk + 1];
      }
      const int nt = min(LPR, a1 - c0);
      if constexpr (LPR <= 16) {
        int pk[LPR];
#pragma unroll
        for (int t = 0; t < LPR; ++t) {
          const int q = __shfl(bl0, gbase + t) + gl;
          pk[t] = t < nt && q < __shfl(bl1, gbase + t) ? bci[q] : -1;
        }
#pragma unroll
        for (int t = 0; t < LPR; ++t) {
          if (pk[t] >= 0) {
            bool fresh;
            if (lds_claim(keys, mask, pk[t], &fresh) < 0) atomicOr(overflow, 1);
            u += fresh;
          }
        }
        // rows of B longer than LPR
        for (int t = 0; t < nt; ++t) {
          const int b1 = __shfl(bl1, gbase + t);
          for (int q = __shfl(bl0, gbase + t) + gl + LPR; q < b1; q += LPR) {
            bool fresh;
            if (lds_claim(keys, mask, bci[q], &fresh) < 0) atomicOr(overflow, 1);
            u += fresh;
          }
        }
      } else {
        for (int t = 0; t < nt; ++t) {
          const int b1 = __shfl(bl1, gbase + t);
          for (int q = __shfl(bl0, gbase + t) + gl; q < b1; q += LPR) {
            bool fresh;
            if (lds_claim(keys, mask, bci[q], &fresh) < 0) atomicOr(overflow, 1);
            u += fresh;
          }
        }
      }
    }
  }
  for (int off = LPR >> 1; off > 0; off >>= 1) u += __shfl_xor(u, off, LPR);
  if (active && gl == 0) cnt[i] = u;
}

// Symbolic product of one row per wavefront.  The distinct count does not
// depend on the order of insertion, so the row's products are flattened:
// 64 entries of A at a time are loaded together, a prefix sum of their B row
// lengths maps every lane to one product, and each step claims 64 products.
// Rows too large for a table of 2 * need slots (big) get the whole table
// with probing bounded by SPG_BIG_PROBES: the distinct count is usually far
// below the bound need, and a row whose claims fail is marked (cnt = -1) for
// the global-table pass.
constexpr uint32_t SPG_BIG_PROBES = 64;
__global__ __launch_bounds__(64 * SPG_WAVES) void k_spgemm_sym_wave(int n, int bm, const int* arp, const int* aci,
                                                                   const int* brp, const int* bci,
                                                                   const int64_t* ub, const int* rows,
                                                                   const int* nrows, int* cnt) {
  __shared__ int tab[SPG_WAVES][SPG_SYM_SLOTS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t count = rows ? *nrows : n;
  int* keys = tab[wave];
  for (int64_t w = (int64_t)blockIdx.x * SPG_WAVES + wave; w < count; w += (int64_t)gridDim.x * SPG_WAVES) {
    const int i = rows ? rows[w] : (int)w;
    const int64_t need = sym_need(ub[i], bm);
    const bool big = 2 * need > SPG_SYM_SLOTS;
    const int T = big ? SPG_SYM_SLOTS : group_table(need);
    const uint32_t mask = (uint32_t)(T - 1);
    for (int q = lane; q < T; q += 64) keys[q] = -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int u = 0, failed = 0;
    const int ae = arp[i + 1];
    for (int kb = arp[i]; kb < ae; kb += 64) {
      const int k = kb + lane;
      int beg = 0, len = 0;
      if (k < ae) {
        const int kk = aci[k];
        beg = brp[kk];
        len = brp[kk + 1] - beg;
      }
      int incl = len;
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      const int total = __shfl(incl, 63, 64);
      const int excl = incl - len;
      for (int t0 = 0; t0 < total; t0 += 64) {
        const int tp = t0 + lane;
        int j = 0;  // lanes whose products all come before tp
        for (int step = 32; step > 0; step >>= 1)
          if (__shfl(incl, j + step - 1, 64) <= tp) j += step;
        const int bj = __shfl(beg, j & 63, 64), ej = __shfl(excl, j & 63, 64);
        if (tp < total) {
          bool fresh;
          if (lds_claim_bounded(keys, mask, bci[bj + (tp - ej)], big ? SPG_BIG_PROBES : mask + 1, &fresh) < 0)
            failed = 1;
          u += fresh;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      u += __shfl_xor(u, off, 64);
      failed |= __shfl_xor(failed, off, 64);
    }
    if (lane == 0) cnt[i] = failed ? -1 : u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// rows whose size measure lies in (lo, hi]: min(ub, bm) with ub given, else
// the row length of crp; one atomic per block reserves the block's places
__global__ __launch_bounds__(BLK) void k_spgemm_list(int n, const int64_t* ub, int bm, const int* crp, int64_t lo,
                                                     int64_t hi, int* list, int* count) {
  __shared__ int nb, base;
  for (int64_t r0 = (int64_t)blockIdx.x * BLK; r0 < n; r0 += (int64_t)gridDim.x * BLK) {
    if (threadIdx.x == 0) nb = 0;
    __syncthreads();
    const int64_t i = r0 + threadIdx.x;
    bool in = false;
    if (i < n) {
      const int64_t m = ub ? sym_need(ub[i], bm) : (int64_t)(crp[i + 1] - crp[i]);
      in = m > lo && m <= hi;
    }
    const int slot = in ? atomicAdd(&nb, 1) : 0;
    __syncthreads();
    if (threadIdx.x == 0 && nb) base = atomicAdd(count, nb);
    __syncthreads();
    if (in) list[base + slot] = (int)i;
    __syncthreads();
  }
}

// numeric: rows is null for every row, else the listed rows (count *nrows)
template <int LPR>
__global__ __launch_bounds__(64 * SPG_WAVES) void k_spgemm_num_grp(int n, const int* arp, const int* aci,
                                                                  const double* av, const int* brp, const int* bci,
                                                                  const double* bv, const int* crp, int64_t hi,
                                                                  const int* rows, const int* nrows, int* cci,
                                                                  double* cv, int* overflow) {
  constexpr int G = 64 / LPR, SLOTS = SPG_NUM_SLOTS / G;
  __shared__ int tk[SPG_WAVES][SPG_NUM_SLOTS];
  __shared__ double tv[SPG_WAVES][SPG_NUM_SLOTS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane / LPR, gl = lane % LPR;
  const int64_t count = rows ? *nrows : n;
  for (int64_t w = ((int64_t)blockIdx.x * SPG_WAVES + wave) * G + grp; w < count;
       w += (int64_t)gridDim.x * SPG_WAVES * G) {
  const int i = rows ? rows[w] : (int)w;
  const int o = crp[i], cnt = crp[i + 1] - o;
  if (cnt > hi || 2 * cnt > SLOTS) continue;  // a wider kernel's row
  const int T = group_table(cnt);
  int* keys = tk[wave] + grp * SLOTS;
  double* vals = tv[wave] + grp * SLOTS;
  for (int q = gl; q < T; q += LPR) {
    keys[q] = -1;
    vals[q] = 0.0;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t mask = (uint32_t)(T - 1);
  const int a0 = arp[i], a1 = arp[i + 1], gbase = grp * LPR;
  // A's row LPR entries at a time: the group's lanes load the entries and
  // the bounds of their rows of B together, then the steps take the entries
  // in order (ascending k), each broadcast from its lane
  for (int c0 = a0; c0 < a1; c0 += LPR) {
    const int kl = c0 + gl;
    double al = 0.0;
    int bl0 = 0, bl1 = 0;
    if (kl < a1) {
      const int kk = aci[kl];
      al = av[kl];
      bl0 = brp[kk];
      bl1 = brp[kk + 1];
    }
    const int nt = min(LPR, a1 - c0);
    if constexpr (LPR <= 16) {
      // every step's first LPR entries of B, requested before the first step
      int pk[LPR];
      double pv[LPR];
#pragma unroll
      for (int t = 0; t < LPR; ++t) {
        const int q = __shfl(bl0, gbase + t) + gl;
        const bool ok = t < nt && q < __shfl(bl1, gbase + t);
        pk[t] = ok ? bci[q] : -1;
        pv[t] = ok ? bv[q] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < LPR; ++t) {
        if (t < nt) {
          const double a = __shfl(al, gbase + t);
          const int b1 = __shfl(bl1, gbase + t);
          int q = __shfl(bl0, gbase + t) + gl;
          if (q < b1) {
            bool fresh;
            const int h = lds_claim(keys, mask, pk[t], &fresh);
            if (h >= 0)
              vals[h] += a * pv[t];
            else
              atomicOr(overflow, 1);
          }
          for (q += LPR; q < b1; q += LPR) {
            bool fresh;
            const int h = lds_claim(keys, mask, bci[q], &fresh);
            if (h >= 0)
              vals[h] += a * bv[q];
            else
              atomicOr(overflow, 1);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
      }
    } else {
      for (int t = 0; t < nt; ++t) {
        const double a = __shfl(al, gbase + t);
        const int b0 = __shfl(bl0, gbase + t), b1 = __shfl(bl1, gbase + t);
        for (int q = b0 + gl; q < b1; q += LPR) {
          bool fresh;
          const int h = lds_claim(keys, mask, bci[q], &fresh);
          if (h >= 0)
            vals[h] += a * bv[q];
          else
            atomicOr(overflow, 1);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  // Compact the occupied slots to the front of the table, LPR slots at a
  // time (a round's slots are read before its writes, which land at or
  // before them), then each entry goes to its rank among the row's columns.
  int m = 0;
  for (int q0 = 0; q0 < T; q0 += LPR) {
    const bool in = q0 + gl < T;  // T < LPR for short rows of the wide groups
    const int c = in ? keys[q0 + gl] : -1;
    const double x = in ? vals[q0 + gl] : 0.0;
    int tot;
    const int r = grp_rank<LPR>(c >= 0, &tot);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (c >= 0) {
      keys[m + r] = c;
      vals[m + r] = x;
    }
    m += tot;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int q = gl; q < m; q += LPR) {
    const int c = keys[q];
    int rank = 0;
    for (int p = 0; p < m; ++p) rank += keys[p] < c;
    cci[o + rank] = c;
    cv[o + rank] = vals[q];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// one thread per row with its table in global scratch (rows with ts == 0
// are done by the wave kernels)
__global__ void k_spgemm_symbolic(int r0, int r1, const int* arp, const int* aci, const int* brp, const int* bci,
                                  const int64_t* toff, int64_t tbase, int* keys, int* cnt) {
  GRID_STRIDE(t, r1 - r0) {
    int i = r0 + (int)t;
    int64_t ts = toff[i + 1] - toff[i];
    if (ts == 0) continue;
    int* tk = keys + (toff[i] - tbase);
    for (int64_t q = 0; q < ts; ++q) tk[q] = -1;
    int u = 0;
    uint32_t mask = (uint32_t)(ts - 1);
    for (int k = arp[i]; k < arp[i + 1]; ++k) {
      int kk = aci[k];
      for (int q = brp[kk]; q < brp[kk + 1]; ++q) {
        int c = bci[q];
        uint32_t h = hslot(c, mask);
        while (tk[h] != -1 && tk[h] != c) h = (h + 1) & mask;
        if (tk[h] == -1) {
          tk[h] = c;
          ++u;
        }
      }
    }
    cnt[i] = u;
  }
}
__global__ void k_spgemm_numeric(int r0, int r1, const int* arp, const int* aci, const double* av, const int* brp,
                                 const int* bci, const double* bv, const int64_t* toff, int64_t tbase, int* keys,
                                 double* vals, const int* crp, int* cci, double* cv) {
  GRID_STRIDE(t, r1 - r0) {
    int i = r0 + (int)t;
    int64_t ts = toff[i + 1] - toff[i];
    if (ts == 0) continue;
    int* tk = keys + (toff[i] - tbase);
    double* tv = vals + (toff[i] - tbase);
    for (int64_t q = 0; q < ts; ++q) {
      tk[q] = -1;
      tv[q] = 0.0;
    }
    uint32_t mask = (uint32_t)(ts - 1);
    for (int k = arp[i]; k < arp[i + 1]; ++k) {
      int kk = aci[k];
      double a = av[k];
      for (int q = brp[kk]; q < brp[kk + 1]; ++q) {
        int c = bci[q];
        uint32_t h = hslot(c, mask);
        while (tk[h] != -1 && tk[h] != c) h = (h + 1) & mask;
        tk[h] = c;
        tv[h] += a * bv[q];
      }
    }
    int o = crp[i], e = crp[i + 1];
    for (int64_t q = 0; q < ts; ++q)
      if (tk[q] != -1) {
        cci[o] = tk[q];
        cv[o] = tv[q];
        ++o;
      }
    int s = crp[i];
    for (int k = s + 1; k < e; ++k) {
      int c = cci[k];
      double x = cv[k];
      int q = k - 1;
      while (q >= s && cci[q] > c) {
        cci[q + 1] = cci[q];
        cv[q + 1] = cv[q];
        --q;
      }
      cci[q + 1] = c;
      cv[q + 1] = x;
    }
  }
}
// every row with products goes to the global-table pass (route 3)
__global__ void k_spgemm_mark_all(int n, const int64_t* ub, int* cnt) {
  GRID_STRIDE(i, n) cnt[i] = ub[i] > 0 ? -1 : 0;
}
// global table sizes of the rows the group kernels marked (cnt < 0)
__global__ void k_spgemm_tsize_sym(int n, int bm, const int64_t* ub, const int* cnt, int64_t* ts) {
  GRID_STRIDE(i, n) ts[i] = cnt[i] < 0 ? table_size(sym_need(ub[i], bm)) : 0;
}
// rows beyond the wave kernels (more than wave_max entries) are listed for
// the one-block-per-row kernel; rows beyond it (block_max) get a global table
__global__ void k_spgemm_tsize_num(int n, const int* crp, int64_t wave_max, int64_t block_max, int64_t* ts,
                                   int* nmid, int* mid) {
  GRID_STRIDE(i, n) {
    const int64_t cnt = crp[i + 1] - crp[i];
    ts[i] = 0;
    if (cnt <= wave_max) continue;
    if (cnt <= block_max)
      mid[atomicAdd(nmid, 1)] = (int)i;
    else
      ts[i] = table_size(cnt);
  }
}

// numeric product of one listed row per block (rows of up to
// SPG_BLK_SLOTS / 2 entries): the threads take the entries of one B row at a
// time and the block synchronises between rows of B, so every slot sums its
// products in ascending k
__global__ __launch_bounds__(BLK) void k_spgemm_num_block(const int* rows, const int* arp, const int* aci,
                                                          const double* av, const int* brp, const int* bci,
                                                          const double* bv, const int* crp, int* cci, double* cv,
                                                          int* overflow) {
  __shared__ int keys[SPG_BLK_SLOTS];
  __shared__ double vals[SPG_BLK_SLOTS];
  const int i = rows[blockIdx.x];
  const int o = crp[i], cnt = crp[i + 1] - o;
  int T = 64;
  while (T < 2 * cnt) T <<= 1;
  for (int q = threadIdx.x; q < T; q += BLK) {
    keys[q] = -1;
    vals[q] = 0.0;
  }
  __syncthreads();
  const uint32_t mask = (uint32_t)(T - 1);
  for (int k = arp[i]; k < arp[i + 1]; ++k) {
    const int kk = aci[k];
    const double a = av[k];
    for (int q = brp[kk] + threadIdx.x; q < brp[kk + 1]; q += BLK) {
      bool fresh;
      const int h = lds_claim(keys, mask, bci[q], &fresh);
      if (h >= 0)
        vals[h] += a * bv[q];
      else
        atomicOr(overflow, 1);
    }
    __syncthreads();
  }
  for (int q = threadIdx.x; q < T; q += BLK) {
    const int c = keys[q];
    if (c < 0) continue;
    int rank = 0;
    for (int p = 0; p < T; ++p) {
      const int d = keys[p];
      rank += (d >= 0) & (d < c);
    }
    cci[o + rank] = c;
    cv[o + rank] = vals[q];
  }
}

// row batches whose global tables fit the scratch budget; returns the largest batch
static int64_t batch_rows(const std::vector<int64_t>& off, int n, std::vector<int>& cuts) {
  const int64_t budget = int64_t(64) << 20;  // table slots
  cuts.assign(1, 0);
  int64_t maxbatch = 0;
  while (cuts.back() < n) {
    int r0 = cuts.back();
    int r1 = (int)(std::upper_bound(off.begin() + r0 + 1, off.end(), off[r0] + budget) - off.begin()) - 1;
    if (r1 <= r0) r1 = r0 + 1;
    if (r1 > n) r1 = n;
    maxbatch = std::max(maxbatch, off[r1] - off[r0]);
    cuts.push_back(r1);
  }
  return maxbatch;
}

static std::atomic<int> g_spgemm_route{0};
void set_spgemm_route(int route) { g_spgemm_route.store(route); }

void spgemm(const DCsr& a, const DCsr& b, DCsr& c, Pool& pool, hipStream_t s) {
  const int n = a.n;
  // route: 0 by row size; 1 every row to the one-row-per-wavefront kernels;
  // 2 numeric rows to the one-block-per-row kernel; 3 every row to the
  // global-memory tables (the paths give bitwise the same product)
  const int route = g_spgemm_route.load();
  c.n = n;
  c.m = b.m;
  Tmp<int64_t> ub(n), ts(n), toff(n + 1);
  Tmp<int> cnt(n), overflow(1);
  HBGS_HIP(hipMemsetAsync(overflow.p, 0, sizeof(int), s));
  k_spgemm_ub<<<grid_for(n, BLK), BLK, 0, s>>>(n, a.rp, a.ci, b.rp, ub.p);
  HBGS_HIP(hipGetLastError());
  // lanes per row from the mean length of B's rows; rows too long for the
  // group tables go to the one-row-per-wavefront kernels
  const double bavg = b.n ? (double)b.nnz / b.n : 0.0;
  const int lpr = bavg <= 8.0 ? 8 : bavg <= 16.0 ? 16 : bavg <= 32.0 ? 32 : 64;
  const int64_t sym_g = route ? 0 : SPG_SYM_SLOTS / (64 / lpr) / 2;
  const int64_t num_g = route ? 0 : SPG_NUM_SLOTS / (64 / lpr) / 2;
  const int64_t num_w = route >= 2 ? 0 : SPG_NUM_SLOTS / 2;              // wave kernel's rows
  const int64_t num_b = route == 3 ? 0 : SPG_BLK_SLOTS / 2;              // block kernel's rows
  auto groups = [&](int l) { return (unsigned)(((int64_t)n + (int64_t)SPG_WAVES * (64 / l) - 1) / (SPG_WAVES * (64 / l))); };
  // the wide kernels stride over the listed rows (every row when lpr = 64)
  Tmp<int> wide(lpr < 64 ? n : 1), nwide(1);
  int* wl = lpr < 64 ? wide.p : nullptr;
  int* wn = lpr < 64 ? nwide.p : nullptr;
  const unsigned wgrid = lpr < 64 ? grid_for(n, SPG_WAVES, 8192) : grid_for(n, SPG_WAVES);
  // symbolic: distinct columns per row
  HBGS_HIP(hipMemsetAsync(nwide.p, 0, sizeof(int), s));
#define HBGS_SYM(L)                                                                                            \
  k_spgemm_sym_grp<L><<<groups(L), 64 * SPG_WAVES, 0, s>>>(n, b.m, a.rp, a.ci, b.rp, b.ci, ub.p, sym_g, cnt.p, \
                                                           overflow.p)
  if (route == 3) {
    k_spgemm_mark_all<<<grid_for(n, BLK), BLK, 0, s>>>(n, ub.p, cnt.p);
  } else {
    switch (lpr) {
      case 8: HBGS_SYM(8); break;
      case 16: HBGS_SYM(16); break;
      case 32: HBGS_SYM(32); break;
      default: break;
    }
    if (lpr < 64)
      k_spgemm_list<<<grid_for(n, BLK, 8192), BLK, 0, s>>>(n, ub.p, b.m, nullptr, sym_g, INT64_MAX, wide.p,
                                                           nwide.p);
    k_spgemm_sym_wave<<<wgrid, 64 * SPG_WAVES, 0, s>>>(n, b.m, a.rp, a.ci, b.rp, b.ci, ub.p, wl, wn, cnt.p);
  }
#undef HBGS_SYM
  HBGS_HIP(hipGetLastError());
  k_spgemm_tsize_sym<<<grid_for(n, BLK), BLK, 0, s>>>(n, b.m, ub.p, cnt.p, ts.p);
  HBGS_HIP(hipGetLastError());
  std::vector<int64_t> h_off;  // row offsets of the global tables, only when some row needs one
  std::vector<int> cuts;
  if (scan_i64(ts.p, toff.p, n, s) > 0) {
    h_off.resize(n + 1);
    HBGS_HIP(hipMemcpyAsync(h_off.data(), toff.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    Tmp<int> keys(batch_rows(h_off, n, cuts));
    for (size_t q = 0; q + 1 < cuts.size(); ++q) {
      int r0 = cuts[q], r1 = cuts[q + 1];
      if (h_off[r1] == h_off[r0]) continue;
      k_spgemm_symbolic<<<grid_for(r1 - r0, 64), 64, 0, s>>>(r0, r1, a.rp, a.ci, b.rp, b.ci, toff.p, h_off[r0],
                                                             keys.p, cnt.p);
      HBGS_HIP(hipGetLastError());
    }
  }
  c.rp = pool.make<int>(n + 1);
  c.nnz = counts_to_rowptr(cnt.p, c.rp, n, s);
  c.ci = pool.make<int>(c.nnz);
  c.v = pool.make<double>(c.nnz);
  // numeric
  HBGS_HIP(hipMemsetAsync(nwide.p, 0, sizeof(int), s));
#define HBGS_NUM(L)                                                                                            \
  k_spgemm_num_grp<L><<<groups(L), 64 * SPG_WAVES, 0, s>>>(n, a.rp, a.ci, a.v, b.rp, b.ci, b.v, c.rp, num_g,     \
                                                           nullptr, nullptr, c.ci, c.v, overflow.p)
  switch (lpr) {
    case 8: HBGS_NUM(8); break;
    case 16: HBGS_NUM(16); break;
    case 32: HBGS_NUM(32); break;
    default: break;
  }
#undef HBGS_NUM
  if (lpr < 64)
    k_spgemm_list<<<grid_for(n, BLK, 8192), BLK, 0, s>>>(n, nullptr, 0, c.rp, num_g, num_w, wide.p, nwide.p);
  k_spgemm_num_grp<64><<<wgrid, 64 * SPG_WAVES, 0, s>>>(n, a.rp, a.ci, a.v, b.rp, b.ci, b.v, c.rp, num_w, wl, wn,
                                                         c.ci, c.v, overflow.p);
  HBGS_HIP(hipGetLastError());
  Tmp<int> nmid(1), mid(n);
  HBGS_HIP(hipMemsetAsync(nmid.p, 0, sizeof(int), s));
  k_spgemm_tsize_num<<<grid_for(n, BLK), BLK, 0, s>>>(n, c.rp, num_w, num_b, ts.p, nmid.p, mid.p);
  HBGS_HIP(hipGetLastError());
  int h_nmid = 0;
  HBGS_HIP(hipMemcpyAsync(&h_nmid, nmid.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (h_nmid > 0) {
    k_spgemm_num_block<<<h_nmid, BLK, 0, s>>>(mid.p, a.rp, a.ci, a.v, b.rp, b.ci, b.v, c.rp, c.ci, c.v, overflow.p);
    HBGS_HIP(hipGetLastError());
  }
  if (scan_i64(ts.p, toff.p, n, s) > 0) {
    h_off.resize(n + 1);
    HBGS_HIP(hipMemcpyAsync(h_off.data(), toff.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    const int64_t maxbatch = batch_rows(h_off, n, cuts);
    Tmp<int> keys(maxbatch);
    Tmp<double> vals(maxbatch);
    for (size_t q = 0; q + 1 < cuts.size(); ++q) {
      int r0 = cuts[q], r1 = cuts[q + 1];
      if (h_off[r1] == h_off[r0]) continue;
      k_spgemm_numeric<<<grid_for(r1 - r0, 64), 64, 0, s>>>(r0, r1, a.rp, a.ci, a.v, b.rp, b.ci, b.v, toff.p,
                                                            h_off[r0], keys.p, vals.p, c.rp, c.ci, c.v);
      HBGS_HIP(hipGetLastError());
    }
  }
  int ovf = 0;
  HBGS_HIP(hipMemcpyAsync(&ovf, overflow.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (ovf) HBGS_FAIL(HBGS_ESETUP, "sparse product: accumulator table overflow");
}

// ------------------------------------------------------- dense coarsest LU
__global__ void k_dense_fill(int n, const int* rp, const int* ci, const double* v, double* m) {
  GRID_STRIDE(i, n) {
    for (int j = 0; j < n; ++j) m[i * (int64_t)n + j] = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) m[i * (int64_t)n + ci[k]] = v[k];
  }
}
// step k: pivot = first row with maximal |a_ik| (i >= k); swap rows; multipliers
__global__ void k_lu_pivot(int n, int k, double* m, int* piv, int* singular) {
  __shared__ double sv[BLK];
  __shared__ int si[BLK];
  double best = -1.0;
  int bi = n;
  for (int i = k + threadIdx.x; i < n; i += BLK) {
    double a = fabs(m[(int64_t)i * n + k]);
    if (a > best) {
      best = a;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int st = BLK / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      double a = sv[threadIdx.x + st];
      int ai = si[threadIdx.x + st];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  int p = si[0];
  if (threadIdx.x == 0) {
    piv[k] = p;
    if (!(sv[0] > 0.0)) *singular = 1;
  }
  if (!(sv[0] > 0.0)) return;
  if (p != k)
    for (int j = threadIdx.x; j < n; j += BLK) {
      double t = m[(int64_t)k * n + j];
      m[(int64_t)k * n + j] = m[(int64_t)p * n + j];
      m[(int64_t)p * n + j] = t;
    }
  __syncthreads();
  double akk = m[(int64_t)k * n + k];
  for (int i = k + 1 + threadIdx.x; i < n; i += BLK) m[(int64_t)i * n + k] = m[(int64_t)i * n + k] / akk;
}
__global__ void k_lu_update(int n, int k, double* m) {
  int64_t w = (int64_t)(n - k - 1);
  GRID_STRIDE(t, w * w) {
    int i = k + 1 + (int)(t / w), j = k + 1 + (int)(t % w);
    m[(int64_t)i * n + j] -= m[(int64_t)i * n + k] * m[(int64_t)k * n + j];
  }
}
// Blocked form of the same factorisation (partial pivoting, the first row
// of maximal |a_ik| as pivot, interchanges recorded as in the unblocked
// steps) for n <= LU_MAXN: panels of LU_NB columns are factored by one
// block holding the panel rows in registers; then the panel's interchanges
// are applied to the other columns together with U12 = L11^-1 A12, and the
// trailing matrix is updated by A22 -= L21 U12.
__global__ void k_iota_i32(int n, int* p) {
  GRID_STRIDE(i, n) p[i] = (int)i;
}
constexpr int LU_NB = 16;
constexpr int LU_PT = 1024;
constexpr int LU_R = 2;
constexpr int LU_MAXN = LU_PT * LU_R;

constexpr int LU_CH = 256;  // panel rows per staging pass through LDS

// Register-only (DPP) reductions within rows of 16 lanes; all 64 lanes must
// be active.  Every lane of a 16-lane row ends with the row's result: pairs
// within quads (quad_perm [1,0,3,2] and [2,3,0,1]), then quads (rotate right
// by 4 and by 8 lanes).  A lane whose source is unavailable keeps its own
// value (old = own).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = (int)bits, hi = (int)(bits >> 32);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)ohi << 32) | (unsigned int)olo);
}
__device__ __forceinline__ double max_row16(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));
  v = fmax(v, dpp_f64<0x4E>(v));
  v = fmax(v, dpp_f64<0x124>(v));
  return fmax(v, dpp_f64<0x128>(v));
}
__device__ __forceinline__ int min_row16(int r) {
  r = min(r, __builtin_amdgcn_update_dpp(r, r, 0xB1, 0xF, 0xF, false));
  r = min(r, __builtin_amdgcn_update_dpp(r, r, 0x4E, 0xF, 0xF, false));
  r = min(r, __builtin_amdgcn_update_dpp(r, r, 0x124, 0xF, 0xF, false));
  return min(r, __builtin_amdgcn_update_dpp(r, r, 0x128, 0xF, 0xF, false));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, lane), hi = __builtin_amdgcn_readlane((int)(bits >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// the wavefront's maximum (uniform); fmax passes over NaN
__device__ __forceinline__ double wave_max(double v) {
  v = max_row16(v);
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}
__device__ __forceinline__ int wave_min(int r) {
  r = min_row16(r);
  return min(min(__builtin_amdgcn_readlane(r, 0), __builtin_amdgcn_readlane(r, 16)),
             min(__builtin_amdgcn_readlane(r, 32), __builtin_amdgcn_readlane(r, 48)));
}

// The panel's rows move between memory and registers through LDS in passes
// of LU_CH rows, so that consecutive lanes touch consecutive columns of a row
// (a row's LU_NB values are one contiguous run) rather than one row each.
// Each column's pivot search runs in registers (DPP within 16-lane rows,
// lane reads across rows) and needs one barrier to combine the wavefronts.
__global__ __launch_bounds__(LU_PT) void k_lu_panel(int n, int k0, double* m, int* piv, int* singular) {
  static_assert(LU_PT / 64 <= 16, "the wavefronts' candidates are combined within one 16-lane row");
  const int PT = blockDim.x, NW = PT / 64;  // a multiple of 64, at least half the rows
  __shared__ double stage[LU_CH][LU_NB + 1];
  // per column: each wavefront's pivot candidate (|value|, row, the row's
  // values) and row j before the interchange; two sets, used by alternate
  // columns, so one barrier per column suffices
  __shared__ double cv[2][LU_PT / 64];
  __shared__ int cr[2][LU_PT / 64];
  __shared__ double crow[2][LU_PT / 64][LU_NB];
  __shared__ double xrow[2][LU_NB];
  const int rows = n - k0, nb = min(LU_NB, n - k0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double a[LU_R][LU_NB];
#pragma unroll
  for (int q = 0; q < LU_R; ++q)
#pragma unroll
    for (int t = 0; t < LU_NB; ++t) a[q][t] = 0.0;
  for (int c0 = 0; c0 < rows; c0 += LU_CH) {
    const int ce = min(LU_CH, rows - c0) * LU_NB;
    for (int e = tid; e < ce; e += PT) {
      const int i = e / LU_NB, t = e % LU_NB;
      stage[i][t] = t < nb ? m[(int64_t)(k0 + c0 + i) * n + k0 + t] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r >= c0 && r < c0 + LU_CH && r < rows)
#pragma unroll
        for (int t = 0; t < LU_NB; ++t) a[q][t] = stage[r - c0][t];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < LU_NB; ++j) {
    const int b = j & 1;
    if (j >= nb) break;  // uniform across the block
    // this wavefront's candidate: the largest |a_rj| over its rows r >= j,
    // then the first of its rows holding that value (two branch-free
    // reductions; NaN is never chosen)
    double best = -1.0;
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r >= j && r < rows) best = fmax(best, fabs(a[q][j]));
    }
    best = wave_max(best);
    int bi = INT32_MAX;
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r >= j && r < rows && fabs(a[q][j]) == best) bi = min(bi, r);
    }
    bi = wave_min(bi);
    if (lane == 0) {
      cv[b][wave] = best;
      cr[b][wave] = bi;
    }
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r == bi)
#pragma unroll
        for (int t = 0; t < LU_NB; ++t) crow[b][wave][t] = a[q][t];
    }
    if (tid == j)  // row j lives in a[0] of thread j (j < LU_NB <= PT)
#pragma unroll
      for (int t = 0; t < LU_NB; ++t) xrow[b][t] = a[0][t];
    __syncthreads();
    // lanes 0..NW-1 of every wavefront hold the wavefronts' candidates
    {
      const double cvl = lane < NW ? cv[b][lane] : -1.0;
      const int crl = lane < NW ? cr[b][lane] : INT32_MAX;
      best = readlane_f64(max_row16(cvl), 0);
      bi = __builtin_amdgcn_readlane(min_row16(cvl == best ? crl : INT32_MAX), 0);
    }
    if (!(best > 0.0)) {  // uniform: the factorisation has failed
      if (tid == 0) *singular = 1;
      return;
    }
    const int p = bi;
    if (tid == 0) piv[k0 + j] = k0 + p;
    const double* prow = crow[b][(p % PT) / 64];  // the pivot row (LDS)
    // interchange rows j and p
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r == j)
#pragma unroll
        for (int t = 0; t < LU_NB; ++t) a[q][t] = prow[t];
      else if (r == p)
#pragma unroll
        for (int t = 0; t < LU_NB; ++t) a[q][t] = xrow[b][t];
    }
    // multipliers and the update of the panel's remaining columns
    const double d = prow[j];
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r > j && r < rows) {
        const double l = a[q][j] / d;
        a[q][j] = l;
#pragma unroll
        for (int t = 0; t < LU_NB; ++t)
          if (t > j) a[q][t] -= l * prow[t];
      }
    }
  }
  for (int c0 = 0; c0 < rows; c0 += LU_CH) {
#pragma unroll
    for (int q = 0; q < LU_R; ++q) {
      const int r = tid + q * PT;
      if (r >= c0 && r < c0 + LU_CH && r < rows)
#pragma unroll
        for (int t = 0; t < LU_NB; ++t) stage[r - c0][t] = a[q][t];
    }
    __syncthreads();
    const int ce = min(LU_CH, rows - c0) * LU_NB;
    for (int e = tid; e < ce; e += PT) {
      const int i = e / LU_NB, t = e % LU_NB;
      if (t < nb) m[(int64_t)(k0 + c0 + i) * n + k0 + t] = stage[i][t];
    }
    __syncthreads();
  }
}

// every column outside the panel: the panel's interchanges; trailing
// columns also get U12 = L11^-1 A12 (L11 unit lower).  The interchanges,
// applied in order, move values among at most 2 LU_NB rows: one wavefront
// works out where each of those rows takes its value from, then every
// column gathers them at once (no chain of dependent swaps) and solves in
// registers with L11 from LDS.
__global__ __launch_bounds__(BLK) void k_lu_swap_trsm(int n, int k0, int nb, double* m, const int* piv) {
  __shared__ int dst[2 * LU_NB], src[2 * LU_NB];
  __shared__ int nrow;
  __shared__ double sl[LU_NB][LU_NB + 1];
  // The walk over the interchanges runs in the registers of wavefront 0
  // (all 64 lanes active): lane e holds slot e's (dst, src), the panel rows
  // first, then each other row as it is met; a row's slot is found by a
  // ballot and two slots' sources are swapped through lane reads.
  static_assert(2 * LU_NB <= 64, "one slot per lane");
  if (threadIdx.x < 64) {
    const int e = threadIdx.x;
    const int mp = e < nb ? piv[k0 + e] : 0;
    int d = e < nb ? k0 + e : -1, sr = d;
    int cnt = nb;
    for (int t = 0; t < nb; ++t) {
      const int p = __builtin_amdgcn_readlane(mp, t);
      if (p > k0 + t && p < n) {
        const unsigned long long hit = __ballot(d == p);  // at most one slot holds row p
        int q;
        if (hit) {
          q = __ffsll(hit) - 1;
        } else {
          q = cnt++;
          if (e == q) d = sr = p;
        }
        const int st = __builtin_amdgcn_readlane(sr, t), sq = __builtin_amdgcn_readlane(sr, q);
        if (e == t) sr = sq;
        if (e == q) sr = st;
      }
    }
    if (e < 2 * LU_NB) {
      dst[e] = d;
      src[e] = sr;
    }
    if (e == 0) nrow = cnt;
  }
  for (int e = threadIdx.x; e < LU_NB * LU_NB; e += BLK) {
    const int r = e / LU_NB, u = e % LU_NB;
    sl[r][u] = (r < nb && u < nb) ? m[(int64_t)(k0 + r) * n + k0 + u] : 0.0;
  }
  __syncthreads();
  const int cnt = nrow;
  const int64_t c = (int64_t)blockIdx.x * BLK + threadIdx.x;  // one column per thread
  if (c < n - nb) {
    const int j = c < k0 ? (int)c : (int)c + nb;
    double v[2 * LU_NB];
#pragma unroll
    for (int q = 0; q < 2 * LU_NB; ++q) v[q] = q < cnt ? m[(int64_t)src[q] * n + j] : 0.0;
    if (j >= k0 + nb) {
#pragma unroll
      for (int t = 1; t < LU_NB; ++t) {
        if (t < nb) {
          double s = v[t];
#pragma unroll
          for (int u = 0; u < t; ++u) s = fma(-sl[t][u], v[u], s);
          v[t] = s;
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the LDS reads row by row (registers)
      }
    }
#pragma unroll
    for (int q = 0; q < 2 * LU_NB; ++q)
      if (q < cnt) m[(int64_t)dst[q] * n + j] = v[q];
  }
}

// A22 -= L21 U12 in tiles of 32 rows x 64 columns (fused multiply-adds)
__global__ __launch_bounds__(BLK) void k_lu_gemm(int n, int k0, int nb, double* m) {
  __shared__ double sL[32][LU_NB];
  __shared__ double sU[LU_NB][64];
  const int r0 = k0 + nb + blockIdx.y * 32, c0 = k0 + nb + blockIdx.x * 64;
  for (int e = threadIdx.x; e < 32 * LU_NB; e += BLK) {
    const int i = e / LU_NB, t = e % LU_NB;
    sL[i][t] = (r0 + i < n && t < nb) ? m[(int64_t)(r0 + i) * n + k0 + t] : 0.0;
  }
  for (int e = threadIdx.x; e < LU_NB * 64; e += BLK) {
    const int t = e / 64, jj = e % 64;
    sU[t][jj] = (c0 + jj < n && t < nb) ? m[(int64_t)(k0 + t) * n + c0 + jj] : 0.0;
  }
  __syncthreads();
  const int jj = threadIdx.x & 63, ib = (threadIdx.x >> 6) * 8;
  if (c0 + jj >= n) return;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = r0 + ib + u;
    if (i >= n) break;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < LU_NB; ++t) acc = fma(sL[ib + u][t], sU[t][jj], acc);
    m[(int64_t)i * n + c0 + jj] -= acc;
  }
}

// Explicit inverse from the factors, X = U^-1 (L^-1 P), by blocks of
// INV_NB rows: each block row of X is finished by a small triangular solve
// (one thread per column) and then removed from the other block rows by a
// tiled update (forward: the rows below; backward: the rows above).
constexpr int INV_NB = 32;
// X = P: column c holds a 1 in row pinv[c]
__global__ void k_inv_init(int n, const int* pinv, double* x) {
  GRID_STRIDE(e, (int64_t)n * n) {
    const int i = (int)(e / n), c = (int)(e % n);
    x[e] = pinv[c] == i ? 1.0 : 0.0;
  }
}
// rows kb..kb+nb of X: unit lower (forward) or upper (backward) block solve,
// one thread per column with the block's rows in registers and the diagonal
// block of the factors in LDS (rows beyond nb: zero, with a unit diagonal)
template <bool UPPER>
__global__ __launch_bounds__(BLK) void k_inv_trsm(int n, int kb, int nb, const double* f, double* x) {
  // The unit lower solve is run as an upper solve on reversed indices
  // (position i holds row INV_NB-1-i, with unit diagonal), so both use the
  // one loop below.
  __shared__ double sf[INV_NB][INV_NB + 1];
  for (int e = threadIdx.x; e < INV_NB * INV_NB; e += BLK) {
    const int i = e / INV_NB, w = e % INV_NB;
    const int r = UPPER ? i : INV_NB - 1 - i, u = UPPER ? w : INV_NB - 1 - w;
    double val = r == u ? 1.0 : 0.0;
    if (r < nb && u < nb && (UPPER || r != u)) val = f[(int64_t)(kb + r) * n + kb + u];
    sf[i][w] = val;
  }
  __syncthreads();
  // one column per thread.  The terms are fused multiply-adds, so each row
  // is one dependent chain that stays in registers; the explicit inverse is
  // checked through the coarse solve's result, not bit for bit.
  const int64_t c = (int64_t)blockIdx.x * BLK + threadIdx.x;
  if (c >= n) return;
  double v[INV_NB];
#pragma unroll
  for (int i = 0; i < INV_NB; ++i) {
    const int r = UPPER ? i : INV_NB - 1 - i;
    v[i] = r < nb ? x[(int64_t)(kb + r) * n + c] : 0.0;
  }
#pragma unroll
  for (int i = INV_NB - 1; i >= 0; --i) {
    double s = v[i];
#pragma unroll
    for (int w = i + 1; w < INV_NB; ++w) s = fma(-sf[i][w], v[w], s);
    v[i] = s / sf[i][i];
  }
#pragma unroll
  for (int i = 0; i < INV_NB; ++i) {
    const int r = UPPER ? i : INV_NB - 1 - i;
    if (r < nb) x[(int64_t)(kb + r) * n + c] = v[i];
  }
}
// X[i, :] -= F[i, kb..kb+nb) X[kb..kb+nb, :] for rows i in [r_lo, r_hi), in
// tiles of 32 rows x 64 columns (fused multiply-adds, like the block solves)
__global__ __launch_bounds__(BLK) void k_inv_update(int n, int kb, int nb, int r_lo, int r_hi, const double* f,
                                                    double* x) {
  __shared__ double sF[32][INV_NB];
  __shared__ double sX[INV_NB][64];
  const int r0 = r_lo + blockIdx.y * 32, c0 = blockIdx.x * 64;
  for (int e = threadIdx.x; e < 32 * INV_NB; e += BLK) {
    const int i = e / INV_NB, t = e % INV_NB;
    sF[i][t] = (r0 + i < r_hi && t < nb) ? f[(int64_t)(r0 + i) * n + kb + t] : 0.0;
  }
  for (int e = threadIdx.x; e < INV_NB * 64; e += BLK) {
    const int t = e / 64, jj = e % 64;
    sX[t][jj] = (c0 + jj < n && t < nb) ? x[(int64_t)(kb + t) * n + c0 + jj] : 0.0;
  }
  __syncthreads();
  const int jj = threadIdx.x & 63, ib = (threadIdx.x >> 6) * 8;
  if (c0 + jj >= n) return;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int i = r0 + ib + u;
    if (i >= r_hi) break;
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < INV_NB; ++t) acc = fma(sF[ib + u][t], sX[t][jj], acc);
    x[(int64_t)i * n + c0 + jj] -= acc;
  }
}

int dense_inverse(const DCsr& a, double* inv, hipStream_t s) {
  const int n = a.n;
  Tmp<double> m((size_t)n * n);
  Tmp<int> piv(n), sing(1), pinv(n);
  HBGS_HIP(hipMemsetAsync(sing.p, 0, sizeof(int), s));
  k_dense_fill<<<grid_for(n, 64), 64, 0, s>>>(n, a.rp, a.ci, a.v, m.p);
  HBGS_HIP(hipGetLastError());
  if (n <= LU_MAXN) {
    k_iota_i32<<<grid_for(n, BLK), BLK, 0, s>>>(n, piv.p);  // no interchange unless a pivot is found
    HBGS_HIP(hipGetLastError());
    for (int k0 = 0; k0 < n; k0 += LU_NB) {
      const int nb = std::min(LU_NB, n - k0);
      // as many wavefronts as the panel's rows need (LU_R rows per thread):
      // every wavefront runs each column's pivot search, so fewer is faster
      const int pt = std::min(LU_PT, std::max(64, ((n - k0 + LU_R - 1) / LU_R + 63) / 64 * 64));
      k_lu_panel<<<1, pt, 0, s>>>(n, k0, m.p, piv.p, sing.p);
      if (n - nb > 0) k_lu_swap_trsm<<<(n - nb + BLK - 1) / BLK, BLK, 0, s>>>(n, k0, nb, m.p, piv.p);
      const int rest = n - k0 - nb;
      if (rest > 0) k_lu_gemm<<<dim3((rest + 63) / 64, (rest + 31) / 32), BLK, 0, s>>>(n, k0, nb, m.p);
    }
  } else {
    for (int k = 0; k < n; ++k) {
      k_lu_pivot<<<1, BLK, 0, s>>>(n, k, m.p, piv.p, sing.p);
      if (k + 1 < n)
        k_lu_update<<<grid_for((int64_t)(n - k - 1) * (n - k - 1), BLK, 8192), BLK, 0, s>>>(n, k, m.p);
    }
  }
  HBGS_HIP(hipGetLastError());
  int singular = 0;
  std::vector<int> hp(n);
  HBGS_HIP(hipMemcpyAsync(&singular, sing.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipMemcpyAsync(hp.data(), piv.p, sizeof(int) * n, hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (singular) return -4;
  // P e_c: apply the interchanges k <-> piv[k] in order to the identity row ids
  std::vector<int> rowof(n), where(n);
  for (int i = 0; i < n; ++i) rowof[i] = i;  // rowof[r] = original index now at position r
  for (int k = 0; k < n; ++k) std::swap(rowof[k], rowof[hp[k]]);
  for (int r = 0; r < n; ++r) where[rowof[r]] = r;
  HBGS_HIP(hipMemcpyAsync(pinv.p, where.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  k_inv_init<<<grid_for((int64_t)n * n, BLK), BLK, 0, s>>>(n, pinv.p, inv);
  HBGS_HIP(hipGetLastError());
  const unsigned cgrid = (unsigned)((n + 63) / 64);
  for (int kb = 0; kb < n; kb += INV_NB) {  // L Y = P
    const int nb = std::min(INV_NB, n - kb);
    k_inv_trsm<false><<<(n + BLK - 1) / BLK, BLK, 0, s>>>(n, kb, nb, m.p, inv);
    const int below = n - kb - nb;
    if (below > 0)
      k_inv_update<<<dim3(cgrid, (below + 31) / 32), BLK, 0, s>>>(n, kb, nb, kb + nb, n, m.p, inv);
  }
  for (int kb = (n - 1) / INV_NB * INV_NB; kb >= 0; kb -= INV_NB) {  // U X = Y
    const int nb = std::min(INV_NB, n - kb);
    k_inv_trsm<true><<<(n + BLK - 1) / BLK, BLK, 0, s>>>(n, kb, nb, m.p, inv);
    if (kb > 0) k_inv_update<<<dim3(cgrid, (kb + 31) / 32), BLK, 0, s>>>(n, kb, nb, 0, kb, m.p, inv);
  }
  HBGS_HIP(hipGetLastError());
  HBGS_HIP(hipStreamSynchronize(s));
  return 0;
}

// --------------------------------------------- transposes for the solve phase
// (A^T)_{ji} = A_{ij}: for a structurally symmetric A the pattern is A's own;
// each entry's value is found in the mirrored row by binary search
template <int L>
__global__ void k_transpose_sym(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                const double* __restrict__ v, double* __restrict__ vt) {
  ROW_GROUPS(L, j, gl, n) {
    for (int q = rp[j] + gl; q < rp[j + 1]; q += L) {
      const int i = ci[q];
      int lo = rp[i], hi = rp[i + 1] - 1;
      double x = 0.0;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        if (ci[mid] == (int)j) {
          x = v[mid];
          break;
        }
        if (ci[mid] < (int)j)
          lo = mid + 1;
        else
          hi = mid - 1;
      }
      vt[q] = x;
    }
  }
}
// Q with rows 2i = row i of a and 2i+1 = row i of b (same column count):
// one row-block pass over Q then forms both products with one operand
template <int L>
__global__ void k_interleave(int n, const int* arp, const int* aci, const double* av, const int* brp,
                             const int* bci, const double* bv, const int* qrp, int* qci, double* qv) {
  ROW_GROUPS(L, i, gl, n) {
    const int qa = qrp[2 * i], qb = qrp[2 * i + 1];
    for (int k = arp[i] + gl; k < arp[i + 1]; k += L) {
      qci[qa + k - arp[i]] = aci[k];
      qv[qa + k - arp[i]] = av[k];
    }
    for (int k = brp[i] + gl; k < brp[i + 1]; k += L) {
      qci[qb + k - brp[i]] = bci[k];
      qv[qb + k - brp[i]] = bv[k];
    }
  }
}
__global__ void k_interleave_rp(int n, const int* arp, const int* brp, int* qrp) {
  GRID_STRIDE(i, n + 1) {
    qrp[2 * i] = arp[i] + brp[i];
    if (i < n) qrp[2 * i + 1] = arp[i + 1] + brp[i];
  }
}
void interleave_rows(Pool& pool, const DCsr& a, const DCsr& b, DCsr& q, hipStream_t s) {
  q = DCsr{};
  q.n = 2 * a.n;
  q.m = a.m;
  q.nnz = a.nnz + b.nnz;
  q.rp = pool.make<int>(q.n + 1);
  q.ci = pool.make<int>(q.nnz);
  q.v = pool.make<double>(q.nnz);
  k_interleave_rp<<<grid_for(a.n + 1, BLK), BLK, 0, s>>>(a.n, a.rp, b.rp, q.rp);
  HBGS_HIP(hipGetLastError());
  const int L = row_lanes(a.n, a.nnz + b.nnz);
  LAUNCH_ROW_GROUPS(k_interleave, L, a.n, s, a.n, a.rp, a.ci, a.v, b.rp, b.ci, b.v, q.rp, q.ci, q.v);
}

void transpose_symmetric(const DCsr& a, double* vt, hipStream_t s) {
  const int L = row_lanes(a.n, a.nnz);
  LAUNCH_ROW_GROUPS(k_transpose_sym, L, a.n, s, a.n, a.rp, a.ci, a.v, vt);
}

// Per-block row statistics: part[9 b] = longest row, part[9 b + 1 + q] =
// entries of the fullest block of row_block(q) consecutive rows, over the
// units block b visits.  Unit u covers rows [4u, 4u + 4); the unit that
// starts a row block of each size also reads that block's end.  Wave maxima
// through shuffles, block maxima through LDS; the host takes the maximum
// over the blocks (no atomics: same-address atomics from every wave cost
// more than the kernel's loads).
__global__ __launch_bounds__(BLK) void k_row_stats(int n, const int* __restrict__ rp, int* __restrict__ part) {
  __shared__ int red[BLK / 64][1 + kRowBlocks];
  int m[1 + kRowBlocks] = {};
  const int64_t nu = ((int64_t)n + 3) / 4;
  GRID_STRIDE(u, nu) {
    const int r0 = (int)(4 * u), r1 = min(n, r0 + 4);
    const int base = rp[r0];
    int prev = base;
    for (int r = r0 + 1; r <= r1; ++r) {
      const int x = rp[r];
      m[0] = max(m[0], x - prev);
      prev = x;
    }
#pragma unroll
    for (int q = 0; q < kRowBlocks; ++q) {
      const int rb = row_block(q);
      if (r0 % rb == 0) m[1 + q] = max(m[1 + q], rp[min(n, r0 + rb)] - base);
    }
  }
  const int w = (int)threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q <= kRowBlocks; ++q) {
    int x = m[q];
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    if ((threadIdx.x & 63) == 0) red[w][q] = x;
  }
  __syncthreads();
  if (threadIdx.x <= kRowBlocks) {
    int x = 0;
    for (int k = 0; k < BLK / 64; ++k) x = max(x, red[k][threadIdx.x]);
    part[(size_t)blockIdx.x * (1 + kRowBlocks) + threadIdx.x] = x;
  }
}
void row_stats(DCsr& a, hipStream_t s) {
  a.maxlen = 0;
  for (int q = 0; q < kRowBlocks; ++q) a.blkmax[q] = 0;
  if (a.n <= 0) return;
  constexpr int S = 1 + kRowBlocks;
  const unsigned nb = grid_for(((int64_t)a.n + 3) / 4, BLK, 1024);
  Tmp<int> part((size_t)nb * S);
  std::vector<int> h((size_t)nb * S);
  k_row_stats<<<nb, BLK, 0, s>>>(a.n, a.rp, part.p);
  HBGS_HIP(hipGetLastError());
  HBGS_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(int) * h.size(), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  for (unsigned b = 0; b < nb; ++b) {
    a.maxlen = std::max(a.maxlen, h[(size_t)b * S]);
    for (int q = 0; q < kRowBlocks; ++q) a.blkmax[q] = std::max(a.blkmax[q], h[(size_t)b * S + 1 + q]);
  }
}

// Operand tiles of one row block per workgroup: the tile ids (col /
// TILE_W) of the block's entries go into an LDS hash set; each distinct id's
// slot is its rank among them (ascending), and each entry's slot is found by
// binary search in the ranked list.  A block with more than TILE_MAX tiles
// sets *too_many and writes nothing.
constexpr int TILE_ENTRIES = 4096;  // entries of one row block at most (the FP32 staging limit)
constexpr int TILE_HASH = 128;   // hash slots (> 2 TILE_MAX)
__global__ __launch_bounds__(256) void k_tiles(int n, int rb, const int* __restrict__ rp, const int* __restrict__ ci,
                                               int* __restrict__ tiles, uint16_t* __restrict__ lc,
                                               int* __restrict__ too_many, int* __restrict__ cnt_max) {
  __shared__ int tab[TILE_HASH];
  __shared__ int uniq[TILE_MAX];
  __shared__ int cnt, full;
  const int b = (int)blockIdx.x, t = (int)threadIdx.x;
  const int r0 = b * rb, r1 = min(n, r0 + rb);
  const int s0 = rp[r0], s1 = rp[r1];
  if (t < TILE_HASH) tab[t] = -1;
  if (t == 0) {
    cnt = 0;
    full = 0;
  }
  __syncthreads();
  for (int k = s0 + t; k < s1; k += 256) {
    const int id = ci[k] / TILE_W;
    uint32_t h = ((uint32_t)id * 2654435761u) & (TILE_HASH - 1);
    for (int probe = 0;; ++probe) {
      if (probe == TILE_HASH) {
        full = 1;
        break;
      }
      const int prev = atomicCAS(&tab[h], -1, id);
      if (prev == -1) {
        atomicAdd(&cnt, 1);
        break;
      }
      if (prev == id) break;
      h = (h + 1) & (TILE_HASH - 1);
    }
  }
  __syncthreads();
  const int nt = cnt;
  if (full || nt > TILE_MAX) {
    if (t == 0) atomicOr(too_many, 1);
    return;
  }
  if (t == 0 && nt) atomicMax(cnt_max, nt);
  if (t < TILE_HASH) {
    const int id = tab[t];
    if (id >= 0) {
      int rank = 0;
      for (int q = 0; q < TILE_HASH; ++q) rank += tab[q] >= 0 && tab[q] < id;
      uniq[rank] = id;
    }
  }
  __syncthreads();
  if (t < TILE_MAX) tiles[(size_t)b * TILE_MAX + t] = t < nt ? uniq[t] : -1;
  for (int k = s0 + t; k < s1; k += 256) {
    const int col = ci[k], id = col / TILE_W;
    int lo = 0, hi = nt - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (uniq[mid] < id)
        lo = mid + 1;
      else
        hi = mid;
    }
    lc[k] = (uint16_t)(lo * TILE_W + col % TILE_W);
  }
}
void build_tiles(Pool& pool, DCsr& a, int rb, hipStream_t s) {
  a.tile_rb = 0;
  a.tile_cnt = 0;
  a.tiles = nullptr;
  a.lc = nullptr;
  if (a.n <= 0 || a.nnz <= 0 || rb <= 0) return;
  int q = 0;
  while (q < kRowBlocks && row_block(q) != rb) ++q;
  if (q == kRowBlocks || a.blkmax[q] > TILE_ENTRIES) return;
  const int64_t nblk = ((int64_t)a.n + rb - 1) / rb;
  int* tiles = pool.make<int>((size_t)nblk * TILE_MAX);
  uint16_t* lc = pool.make<uint16_t>(a.nnz);
  Tmp<int> flags(2);
  HBGS_HIP(hipMemsetAsync(flags.p, 0, 2 * sizeof(int), s));
  k_tiles<<<(unsigned)nblk, 256, 0, s>>>(a.n, rb, a.rp, a.ci, tiles, lc, flags.p, flags.p + 1);
  HBGS_HIP(hipGetLastError());
  int h[2] = {0, 0};
  HBGS_HIP(hipMemcpyAsync(h, flags.p, sizeof(h), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (h[0] || h[1] <= 0) {
    pool.release(lc);
    pool.release(tiles);
    return;
  }
  a.tile_rb = rb;
  a.tile_cnt = h[1];
  a.tiles = tiles;
  a.lc = lc;
}

// ------------------------------------------------------- DD(0)-ILU(0) leaf
__global__ void k_sub_count(int n, const int* rp, const int* ci, int sub, int* cnt) {
  GRID_STRIDE(i, n) {
    const int b = (int)(i / sub);
    int c = 0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) c += ci[k] / sub == b;
    cnt[i] = c;
  }
}
__global__ void k_sub_fill(int n, const int* rp, const int* ci, const double* v, int sub, const int* orp, int* oci,
                           double* ov, int* dpos, int* missing) {
  GRID_STRIDE(i, n) {
    const int b = (int)(i / sub);
    int o = orp[i], d = -1;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] / sub == b) {
        if (ci[k] == (int)i) d = o;
        oci[o] = ci[k];
        ov[o] = v[k];
        ++o;
      }
    dpos[i] = d;
    if (d < 0) atomicOr(missing, 1);
  }
}
// one block per subdomain, level by level, one thread per row: the IKJ
// row update (each l_ik, then a_ij -= l_ik u_kj in ascending j), the rows it
// reads being final
__global__ __launch_bounds__(BLK) void k_ilu_factor(const int* ford, const int* flev, const int* fsub, const int* rp,
                                                    const int* ci, double* v, const int* dpos, int* zero_pivot) {
  const int b = blockIdx.x;
  for (int l = fsub[b]; l + 1 < fsub[b + 1]; ++l) {
    for (int t = flev[l] + threadIdx.x; t < flev[l + 1]; t += BLK) {
      const int i = ford[t];
      for (int p = rp[i]; p < dpos[i]; ++p) {
        const int k = ci[p];
        const double lik = v[p] / v[dpos[k]];
        v[p] = lik;
        int q = dpos[k] + 1;
        for (int r = p + 1; r < rp[i + 1]; ++r) {
          while (q < rp[k + 1] && ci[q] < ci[r]) ++q;
          if (q < rp[k + 1] && ci[q] == ci[r]) v[r] = v[r] - lik * v[q];
        }
      }
      if (v[dpos[i]] == 0.0) atomicOr(zero_pivot, 1);
    }
    __syncthreads();
  }
}

// level schedule of one direction on the host: level(i) = 1 + max level of
// the rows it reads (lower part for fwd, upper part for bwd), per subdomain
static void ilu_schedule(int n, int sub, const std::vector<int>& rp, const std::vector<int>& ci,
                         const std::vector<int>& dpos, bool fwd, std::vector<int>& order, std::vector<int>& lev,
                         std::vector<int>& subp) {
  std::vector<int> level(n, 0);
  if (fwd) {
    for (int i = 0; i < n; ++i)
      for (int k = rp[i]; k < dpos[i]; ++k) level[i] = std::max(level[i], level[ci[k]] + 1);
  } else {
    for (int i = n - 1; i >= 0; --i)
      for (int k = dpos[i] + 1; k < rp[i + 1]; ++k) level[i] = std::max(level[i], level[ci[k]] + 1);
  }
  const int nsub = (n + sub - 1) / sub;
  order.resize(n);
  lev.clear();
  subp.assign(nsub + 1, 0);
  for (int b = 0; b < nsub; ++b) {
    const int r0 = b * sub, r1 = std::min(n, r0 + sub);
    int nl = 0;
    for (int i = r0; i < r1; ++i) nl = std::max(nl, level[i] + 1);
    std::vector<int> cnt(nl + 1, 0);
    for (int i = r0; i < r1; ++i) cnt[level[i] + 1]++;
    for (int q = 0; q < nl; ++q) cnt[q + 1] += cnt[q];
    subp[b] = (int)lev.size();
    for (int q = 0; q <= nl; ++q) lev.push_back(r0 + cnt[q]);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int i = r0; i < r1; ++i) order[r0 + fill[level[i]]++] = i;
  }
  subp[nsub] = (int)lev.size();
}

int ilu_setup(Pool& pool, const DCsr& a, int sub, IluLeaf& out, hipStream_t s) {
  const int n = a.n;
  DCsr& F = out.F;
  F.n = F.m = n;
  {
    Tmp<int> cnt(n), missing(1);
    F.rp = pool.make<int>(n + 1);
    k_sub_count<<<grid_for(n, BLK), BLK, 0, s>>>(n, a.rp, a.ci, sub, cnt.p);
    HBGS_HIP(hipGetLastError());
    F.nnz = counts_to_rowptr(cnt.p, F.rp, n, s);
    F.ci = pool.make<int>(F.nnz);
    F.v = pool.make<double>(F.nnz);
    out.dpos = pool.make<int>(n);
    HBGS_HIP(hipMemsetAsync(missing.p, 0, sizeof(int), s));
    k_sub_fill<<<grid_for(n, BLK), BLK, 0, s>>>(n, a.rp, a.ci, a.v, sub, F.rp, F.ci, F.v, out.dpos, missing.p);
    HBGS_HIP(hipGetLastError());
    int h_missing = 0;
    HBGS_HIP(hipMemcpyAsync(&h_missing, missing.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HBGS_HIP(hipStreamSynchronize(s));
    if (h_missing) return -4;
  }
  // schedules (host)
  std::vector<int> rp(n + 1), ci(F.nnz), dp(n);
  HBGS_HIP(hipMemcpyAsync(rp.data(), F.rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipMemcpyAsync(ci.data(), F.ci, sizeof(int) * F.nnz, hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipMemcpyAsync(dp.data(), out.dpos, sizeof(int) * n, hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  out.nsub = (n + sub - 1) / sub;
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int> order, lev, subp;
    ilu_schedule(n, sub, rp, ci, dp, pass == 0, order, lev, subp);
    int* o = pool.make<int>(n);
    int* l = pool.make<int>(lev.size());
    int* sp = pool.make<int>(subp.size());
    HBGS_HIP(hipMemcpyAsync(o, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    HBGS_HIP(hipMemcpyAsync(l, lev.data(), sizeof(int) * lev.size(), hipMemcpyHostToDevice, s));
    HBGS_HIP(hipMemcpyAsync(sp, subp.data(), sizeof(int) * subp.size(), hipMemcpyHostToDevice, s));
    HBGS_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    if (pass == 0) {
      out.ford = o;
      out.flev = l;
      out.fsub = sp;
    } else {
      out.bord = o;
      out.blev = l;
      out.bsub = sp;
    }
  }
  // factorisation, transposed factors, FP32 copies, work vector
  Tmp<int> zp(1);
  HBGS_HIP(hipMemsetAsync(zp.p, 0, sizeof(int), s));
  k_ilu_factor<<<out.nsub, BLK, 0, s>>>(out.ford, out.flev, out.fsub, F.rp, F.ci, F.v, out.dpos, zp.p);
  HBGS_HIP(hipGetLastError());
  int h_zero = 0;
  HBGS_HIP(hipMemcpyAsync(&h_zero, zp.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (h_zero) return -4;
  F.vf = pool.make<float>(F.nnz);
  cast_f32(F.nnz, F.v, F.vf, s);
  out.yd = pool.make<double>(n);
  out.yf = pool.make<float>(n);
  HBGS_HIP(hipStreamSynchronize(s));
  return 0;
}

// the factors transposed (same pattern), for the adjoint sweep
void ilu_transpose(Pool& pool, IluLeaf& leaf, hipStream_t s) {
  const DCsr& F = leaf.F;
  leaf.vT = pool.make<double>(F.nnz);
  transpose_symmetric(F, leaf.vT, s);
  leaf.vTf = pool.make<float>(F.nnz);
  cast_f32(F.nnz, leaf.vT, leaf.vTf, s);
}

// One wavefront per chunk of COL_CHUNK entries.  k_col_base: the chunk's
// smallest column goes to cb; a chunk whose columns span 65536 or more sets
// bad.  k_col_pack: every entry's offset from its chunk's base.
static_assert(COL_CHUNK % 64 == 0, "chunks are whole wavefronts");
constexpr int COL_PER_LANE = COL_CHUNK / 64;
__global__ __launch_bounds__(256) void k_col_base(int64_t nnz, const int* __restrict__ ci, int* __restrict__ cb,
                                                  int* bad) {
  const int lane = threadIdx.x & 63;
  const int64_t nch = (nnz + COL_CHUNK - 1) / COL_CHUNK;
  int wide = 0;
  for (int64_t ch = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); ch < nch; ch += (int64_t)gridDim.x * 4) {
    if (*(volatile int*)bad) break;  // another wave already found a wide chunk
    const int64_t k0 = ch * COL_CHUNK + lane;
    int lo = INT32_MAX, hi = INT32_MIN;
#pragma unroll
    for (int q = 0; q < COL_PER_LANE; ++q) {
      const int64_t k = k0 + q * 64;
      if (k < nnz) {
        const int c = ci[k];
        lo = min(lo, c);
        hi = max(hi, c);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, __shfl_xor(lo, off, 64));
      hi = max(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) cb[ch] = lo;
    if ((int64_t)hi - (int64_t)lo > 65535) {
      wide = 1;
      break;
    }
  }
  if (lane == 0 && wide) atomicOr(bad, 1);
}
__global__ __launch_bounds__(256) void k_col_pack(int64_t nnz, const int* __restrict__ ci,
                                                  const int* __restrict__ cb, uint16_t* __restrict__ cd) {
  const int lane = threadIdx.x & 63;
  const int64_t nch = (nnz + COL_CHUNK - 1) / COL_CHUNK;
  for (int64_t ch = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); ch < nch; ch += (int64_t)gridDim.x * 4) {
    const int base = cb[ch];
    const int64_t k0 = ch * COL_CHUNK + lane;
#pragma unroll
    for (int q = 0; q < COL_PER_LANE; ++q) {
      const int64_t k = k0 + q * 64;
      if (k < nnz) cd[k] = (uint16_t)(ci[k] - base);
    }
  }
}
void pack_columns(Pool& pool, DCsr& a, hipStream_t s) {
  a.cd = nullptr;
  a.cb = nullptr;
  if (a.nnz == 0) return;
  const int64_t nch = (a.nnz + COL_CHUNK - 1) / COL_CHUNK;
  const unsigned g = grid_for((nch + 3) / 4, 1);
  int* cb = pool.make<int>(nch);
  Tmp<int> bad(1);
  HBGS_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  k_col_base<<<grid_for((nch + 3) / 4, 1, 8192), 256, 0, s>>>(a.nnz, a.ci, cb, bad.p);
  HBGS_HIP(hipGetLastError());
  int h_bad = 0;
  HBGS_HIP(hipMemcpyAsync(&h_bad, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HBGS_HIP(hipStreamSynchronize(s));
  if (h_bad) {
    pool.release(cb);
    return;
  }
  uint16_t* cd = pool.make<uint16_t>(a.nnz);
  k_col_pack<<<g, 256, 0, s>>>(a.nnz, a.ci, cb, cd);
  HBGS_HIP(hipGetLastError());
  a.cd = cd;
  a.cb = cb;
}

__global__ void k_dense_transpose(int n, const double* __restrict__ in, double* __restrict__ out) {
  GRID_STRIDE(t, (int64_t)n * n) {
    int i = (int)(t / n), j = (int)(t % n);
    out[(int64_t)j * n + i] = in[t];
  }
}
void dense_transpose(int n, const double* in, double* out, hipStream_t s) {
  k_dense_transpose<<<grid_for((int64_t)n * n, BLK), BLK, 0, s>>>(n, in, out);
  HBGS_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ casts
__global__ void k_cast_f32(int64_t n, const double* in, float* out) {
  GRID_STRIDE(i, n) out[i] = (float)in[i];
}
void cast_f32(int64_t n, const double* in, float* out, hipStream_t s) {
  if (n == 0) return;
  k_cast_f32<<<grid_for(n, BLK), BLK, 0, s>>>(n, in, out);
  HBGS_HIP(hipGetLastError());
}
__global__ void k_reciprocal(int n, const double* d, double* dinv, float* dinvf) {
  GRID_STRIDE(i, n) {
    double r = 1.0 / d[i];
    dinv[i] = r;
    dinvf[i] = (float)r;
  }
}
void reciprocal(int n, const double* d, double* dinv, float* dinvf, hipStream_t s) {
  k_reciprocal<<<grid_for(n, BLK), BLK, 0, s>>>(n, d, dinv, dinvf);
  HBGS_HIP(hipGetLastError());
}

}  // namespace setup
}  // namespace hbgs
