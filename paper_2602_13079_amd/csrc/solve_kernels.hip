// Solve-phase kernels (gfx950, wave64): everything here is sparse or
// vector work bound by HBM bandwidth, so no matrix cores are used.
//
// CSR kernels process one row per group of LPR lanes (LPR = 1..64 chosen
// from the mean row length): the value and column streams of consecutive
// rows are read by consecutive lanes, so a wavefront's loads are coalesced;
// the partial products are combined with cross-lane shuffles and the row's
// epilogue (residual, Chebyshev update, transfer accumulation) is fused into
// the same kernel, so each vector is read and written once per step.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "hbgs_internal.h"

namespace hbgs {
namespace solve {

constexpr int BLK = 256;

const char* kind_names[K_COUNT] = {
    "spmv_outer", "spmv_resid", "cheb_pre",  "cheb_post_a", "cheb_post_b", "cheb_other", "resid", "restrict",
    "prolong",    "coarse",     "couple",    "dot1",        "upd_dot2",    "reduce",
    "givens",     "scale",      "xupdate",   "permute",     "cheb_pre_c", "cheb_post_a_c", "cheb_post_b_c",
    "cheb_other_c", "resid_c",  "restrict_c", "prolong_c", "sweep"};

// ---------------------------------------------------------- CSR row engine
template <class T>
__device__ __forceinline__ T lanes_sum(T v, int lpr) {
  for (int off = lpr >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, lpr);
  return v;
}

// column index loaders: plain int32, or packed 16-bit offsets from a base
// per chunk of COL_CHUNK entries (2 bytes per entry instead of 4)
// load4(k, c): the columns of entries k..k+3, k a multiple of 4 (16-byte /
// 8-byte loads; the four share one packed base since 4 divides COL_CHUNK)
struct ColPlain {
  const int* __restrict__ ci;
  __device__ int operator()(int k) const { return ci[k]; }
  __device__ void load4(int k, int* c) const {
    const int4 t = *reinterpret_cast<const int4*>(ci + k);
    c[0] = t.x;
    c[1] = t.y;
    c[2] = t.z;
    c[3] = t.w;
  }
  bool aligned() const { return reinterpret_cast<uintptr_t>(ci) % 16 == 0; }
};
struct ColPacked {
  const uint16_t* __restrict__ cd;
  const int* __restrict__ cb;
  __device__ int operator()(int k) const { return cb[k / COL_CHUNK] + (int)cd[k]; }
  __device__ void load4(int k, int* c) const {
    const ushort4 t = *reinterpret_cast<const ushort4*>(cd + k);
    const int b = cb[k / COL_CHUNK];
    c[0] = b + (int)t.x;
    c[1] = b + (int)t.y;
    c[2] = b + (int)t.z;
    c[3] = b + (int)t.w;
  }
  bool aligned() const { return reinterpret_cast<uintptr_t>(cd) % 8 == 0; }
};
static_assert(COL_CHUNK % 4 == 0, "a group of four entries shares one packed base");
// values of entries k..k+3 (16-byte loads)
__device__ __forceinline__ void load4(const float* p, float* w) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  w[0] = t.x;
  w[1] = t.y;
  w[2] = t.z;
  w[3] = t.w;
}
__device__ __forceinline__ void load4(const double* p, double* w) {
  const double2 a = *reinterpret_cast<const double2*>(p), b = *reinterpret_cast<const double2*>(p + 2);
  w[0] = a.x;
  w[1] = a.y;
  w[2] = b.x;
  w[3] = b.y;
}

// acc = sum_k v[k] * X(ci[k]) over row `row`, then epi(row, acc)
template <int LPR, class TV, class TACC, class Col, class LoadX, class Epi>
__global__ __launch_bounds__(BLK) void k_csr(int n, const int* __restrict__ rp, Col ci, const TV* __restrict__ v,
                                             LoadX lx, Epi epi) {
  const int lane = threadIdx.x & (LPR - 1);
  const int row = (int)(((int64_t)blockIdx.x * BLK + threadIdx.x) / LPR);
  if (row >= n) return;
  const int s = rp[row], e = rp[row + 1];
  TACC acc = 0;
  for (int k = s + lane; k < e; k += LPR) acc += (TACC)v[k] * (TACC)lx(ci(k));
  if (LPR > 1) acc = lanes_sum<TACC>(acc, LPR);
  if (lane == 0) epi.store(row, acc, epi.load(row));
}

template <class TACC, class Epi>
__global__ void k_empty(int n, Epi epi) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) epi.store((int)i, TACC(0), epi.load((int)i));
}
// Row-block streaming form for short and medium rows (at most
// ROWS_LDS_BYTES / sizeof(TACC) entries in any block of RB rows).  Block b
// owns rows [RB b, RB (b+1)) and their entries: the
// row epilogues' vector loads and the rows' bounds are issued first, so they
// overlap the entry stream; the threads then stream the entries' values and column indices
// with unit-stride (coalesced) loads, gather the operand and stage the
// products in LDS; finally SBLK/RB lanes per row (or one thread per row when
// RB >= SBLK) sum each row's products from LDS and apply the epilogue.
constexpr int SBLK = 256;
constexpr int ROWS_LDS_BYTES = 16384;
static bool g_vec_entries = true;  // grouped entry loads where the arrays are aligned

// vec: the entry stream in groups of four (16-byte value and 16/8-byte
// column loads) over the block's 4-aligned entries, two groups per step,
// single entries at the two ends; else two single entries per step.  The
// products and their summation order are the same either way.
template <int RB, class TV, class TACC, class Col, class LoadX, class Epi>
__global__ __launch_bounds__(SBLK) void k_csr_rows(int n, const int* __restrict__ rp, Col ci,
                                                   const TV* __restrict__ v, LoadX lx, Epi epi, int vec) {
  constexpr int LPR = RB >= SBLK ? 1 : SBLK / RB;  // lanes per row in the row sums
  constexpr int RPT = RB >= SBLK ? RB / SBLK : 1;  // rows per thread
  __shared__ TACC prod[ROWS_LDS_BYTES / sizeof(TACC)];
  const int r0 = blockIdx.x * RB;
  const int r1 = min(n, r0 + RB);
  const int lane = threadIdx.x & (LPR - 1);
  const int rbase = r0 + (int)threadIdx.x / LPR;
  typename Epi::Pre pre[RPT];
  int rkb[RPT], rke[RPT];  // row bounds for the sums, requested before the barrier
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = rbase + q * SBLK;
    if (r < r1 && lane == 0) pre[q] = epi.load(r);
    rkb[q] = r < r1 ? rp[r] : 0;
    rke[q] = r < r1 ? rp[r + 1] : 0;
  }
  const int s0 = rp[r0], s1 = rp[r1];
  const int a0 = (s0 + 3) & ~3, a1 = s1 & ~3;  // the 4-aligned middle
  if (vec && a0 < a1) {
    const int t = (int)threadIdx.x;
    // the (at most 3 + 3) entries outside the 4-aligned middle: values and
    // columns requested first, operands gathered after the middle's, so
    // they add no round trip ahead of it (indices clamped into the block)
    const bool hh = s0 + t < a0, ht = a1 + t < s1;
    const int kh = hh ? s0 + t : a0, kt = ht ? a1 + t : a1 - 1;
    const TV vh = v[kh], vt = v[kt];
    const int ch = ci(kh), ct = ci(kt);
    // two groups of four per step, both requested before either is used
    // (a thread without a second group re-reads its first)
    for (int k4 = a0 + 4 * t; k4 < a1; k4 += 8 * SBLK) {
      const int k4b = k4 + 4 * SBLK;
      const bool two = k4b < a1;
      const int kb = two ? k4b : k4;
      TV w0[4], w1[4];
      int c0[4], c1[4];
      load4(v + k4, w0);
      ci.load4(k4, c0);
      load4(v + kb, w1);
      ci.load4(kb, c1);
      TACC x0[4], x1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x0[q] = (TACC)lx(c0[q]);
#pragma unroll
      for (int q = 0; q < 4; ++q) x1[q] = (TACC)lx(c1[q]);
#pragma unroll
      for (int q = 0; q < 4; ++q) prod[k4 + q - s0] = (TACC)w0[q] * x0[q];
      if (two)
#pragma unroll
        for (int q = 0; q < 4; ++q) prod[k4b + q - s0] = (TACC)w1[q] * x1[q];
    }
    const TACC xh = (TACC)lx(ch), xt = (TACC)lx(ct);
    if (hh) prod[kh - s0] = (TACC)vh * xh;
    if (ht) prod[kt - s0] = (TACC)vt * xt;
  } else {
    // two independent entries per step keep more gathers in flight
    int k = s0 + threadIdx.x;
    for (; k + SBLK < s1; k += 2 * SBLK) {
      const int c0 = ci(k), c1 = ci(k + SBLK);
      const TV w0 = v[k], w1 = v[k + SBLK];
      const TACC x0 = (TACC)lx(c0), x1 = (TACC)lx(c1);
      prod[k - s0] = (TACC)w0 * x0;
      prod[k + SBLK - s0] = (TACC)w1 * x1;
    }
    if (k < s1) prod[k - s0] = (TACC)v[k] * (TACC)lx(ci(k));
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = rbase + q * SBLK;
    TACC acc = 0;
    if (r < r1) {
      const int kb = rkb[q] - s0, ke = rke[q] - s0;
      for (int k = kb + lane; k < ke; k += LPR) acc += prod[k];
    }
    if (LPR > 1) acc = lanes_sum<TACC>(acc, LPR);
    if (r < r1 && lane == 0) epi.store(r, acc, pre[q]);
  }
}

// Row-block form with the operand staged in LDS (matrices with operand
// tiles): the block's tiles of TILE_W consecutive operand entries are
// loaded with coalesced loads at the same time as its entries, whose local
// columns (2 bytes each) then index the staged tiles, so no load waits on a
// column index.  The block's entries (at most 4 * SBLK * NG) are held in
// registers across the barrier that publishes the tiles.  Same products,
// LDS positions and row sums as k_csr_rows: bitwise the same result.
template <int RB, class TV, class TACC, class TX, class Epi>
__global__ __launch_bounds__(SBLK) void k_csr_rows_tiled(int n, int m, const int* __restrict__ rp,
                                                         const uint16_t* __restrict__ lc,
                                                         const int* __restrict__ tiles, int tcnt,
                                                         const TV* __restrict__ v, const TX* __restrict__ x,
                                                         Epi epi, int prod_bytes) {
  constexpr int LPR = RB >= SBLK ? 1 : SBLK / RB;
  constexpr int RPT = RB >= SBLK ? RB / SBLK : 1;
  constexpr int NG = (ROWS_LDS_BYTES / (int)sizeof(TACC)) / (4 * SBLK);  // groups of four per thread
  constexpr int TPP = SBLK / TILE_W;                                      // tiles per pass
  extern __shared__ __align__(16) unsigned char smem[];
  TACC* prod = reinterpret_cast<TACC*>(smem);
  TX* xs = reinterpret_cast<TX*>(smem + prod_bytes);
  const int t = (int)threadIdx.x;
  const int b = (int)blockIdx.x;
  const int r0 = b * RB, r1 = min(n, r0 + RB);
  const int lane = t & (LPR - 1);
  const int rbase = r0 + t / LPR;
  typename Epi::Pre pre[RPT];
  int rkb[RPT], rke[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = rbase + q * SBLK;
    if (r < r1 && lane == 0) pre[q] = epi.load(r);
    rkb[q] = r < r1 ? rp[r] : 0;
    rke[q] = r < r1 ? rp[r + 1] : 0;
  }
  // the tiles' ids, then their entries (thread t stages element t % TILE_W
  // of tiles t / TILE_W + TPP j)
  const int e = t % TILE_W, j0 = t / TILE_W;
  int id[TILE_MAX / TPP];
#pragma unroll
  for (int j = 0; j < TILE_MAX / TPP; ++j) {
    const int slot = j0 + TPP * j;
    id[j] = slot < tcnt ? tiles[(size_t)b * TILE_MAX + slot] : -1;
  }
  const int s0 = rp[r0], s1 = rp[r1];
  TX xv[TILE_MAX / TPP];
#pragma unroll
  for (int j = 0; j < TILE_MAX / TPP; ++j) {
    const int c = id[j] * TILE_W + e;
    xv[j] = id[j] >= 0 && c < m ? x[c] : TX(0);
  }
  // the entries: the 4-aligned middle [m0, m1) in groups of four, the at
  // most 3 + 3 entries at the ends singly
  const int m0 = min((s0 + 3) & ~3, s1), m1 = max(s1 & ~3, m0);
  const bool hh = s0 + t < m0, ht = m1 + t < s1;
  const int kh = s0 + t, kt = m1 + t;
  const TV vh = hh ? v[kh] : TV(0), vt = ht ? v[kt] : TV(0);
  const int lh = hh ? (int)lc[kh] : 0, lt = ht ? (int)lc[kt] : 0;
  TV w[NG][4];
  int c[NG][4];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int k4 = m0 + 4 * t + 4 * SBLK * g;
    if (k4 < m1) {
      load4(v + k4, w[g]);
      const ushort4 u = *reinterpret_cast<const ushort4*>(lc + k4);
      c[g][0] = u.x;
      c[g][1] = u.y;
      c[g][2] = u.z;
      c[g][3] = u.w;
    }
  }
#pragma unroll
  for (int j = 0; j < TILE_MAX / TPP; ++j)
    if (id[j] >= 0) xs[(j0 + TPP * j) * TILE_W + e] = xv[j];
  __syncthreads();
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int k4 = m0 + 4 * t + 4 * SBLK * g;
    if (k4 < m1)
#pragma unroll
      for (int q = 0; q < 4; ++q) prod[k4 + q - s0] = (TACC)w[g][q] * (TACC)xs[c[g][q]];
  }
  if (hh) prod[kh - s0] = (TACC)vh * (TACC)xs[lh];
  if (ht) prod[kt - s0] = (TACC)vt * (TACC)xs[lt];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = rbase + q * SBLK;
    TACC acc = 0;
    if (r < r1) {
      const int k0 = rkb[q] - s0, k1 = rke[q] - s0;
      for (int k = k0 + lane; k < k1; k += LPR) acc += prod[k];
    }
    if (LPR > 1) acc = lanes_sum<TACC>(acc, LPR);
    if (r < r1 && lane == 0) epi.store(r, acc, pre[q]);
  }
}

template <class T>
struct LoadArr;
template <class L>
struct load_arr_elem {
  using type = void;
};
template <class T>
struct load_arr_elem<LoadArr<T>> {
  using type = T;
};
static bool g_tiles_on = true;  // the LDS-staged operand where a matrix has tiles
void set_tiles(bool on) { g_tiles_on = on; }

int rows_per_block(const DCsr& a, int cap, bool vec) {
  // the largest RB whose every block's entries fit the LDS staging
  // (blkmax <= cap) and that still gives MIN_BLOCKS blocks, so a coarse
  // level (10^3 - 10^5 rows) spreads over every CU instead of a few hundred
  // blocks; where no RB gives that many, the smallest that fits.  With
  // grouped loads 256-row blocks beat 512-row ones (finest FP32 levels:
  // 13.7 vs 14.3 us at 1M rows); with single loads the larger wins.
  constexpr int64_t MIN_BLOCKS = 1024;  // 4 per CU
  int rb = 0;
  for (int q = vec ? 1 : 0; q < kRowBlocks; ++q) {
    const int r = row_block(q);
    if (a.blkmax[q] <= 0 || a.blkmax[q] > cap) continue;
    rb = r;
    if (((int64_t)a.n + r - 1) / r >= MIN_BLOCKS) break;
  }
  return rb;
}

// e0/e1 (optional): events that the dispatch itself stamps with the
// kernel's start and end (no extra packets in the stream), for timing one
// class of launches inside a timed run
template <class TV, class TACC, class Col, class LoadX, class Epi>
static void launch_csr_cols(const DCsr& a, Col col, const TV* v, LoadX lx, Epi epi, hipStream_t s,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  constexpr int cap = ROWS_LDS_BYTES / (int)sizeof(TACC);
  const int vec = g_vec_entries && reinterpret_cast<uintptr_t>(v) % 16 == 0 && col.aligned();
  const int rb = rows_per_block(a, cap, vec != 0);
  // the LDS-staged operand where the matrix has tiles for this block size
  // and the staging (products and tiles) takes at most 32 KiB, 5 blocks per
  // CU (at 4.2M DOF the outer SpMV's 21-27 KiB still run faster staged: 95
  // -> 83 us mixed, 102 -> 93 us FP64)
  using TX = typename load_arr_elem<LoadX>::type;
  if constexpr (!std::is_void<TX>::value) {
    if (g_tiles_on && vec && a.tile_rb == rb && a.lc && (rb == 256 || rb == 128 || rb == 64)) {
      int q = 0;
      while (row_block(q) != rb) ++q;
      const int pb = (a.blkmax[q] * (int)sizeof(TACC) + 15) / 16 * 16;
      const int lds = pb + a.tile_cnt * TILE_W * (int)sizeof(TX);
      if (lds <= 32768) {
        const unsigned grid = (unsigned)(((int64_t)a.n + rb - 1) / rb);
#define HBGS_TILED(RB)                                                                                     \
  if (rb == RB) {                                                                                          \
    if (e0)                                                                                                \
      hipExtLaunchKernelGGL(k_csr_rows_tiled<RB, TV, TACC, TX, Epi>, dim3(grid), dim3(SBLK), lds, s, e0, e1, 0, \
                            a.n, a.m, a.rp, a.lc, a.tiles, a.tile_cnt, v, lx.x, epi, pb);                  \
    else                                                                                                   \
      k_csr_rows_tiled<RB, TV, TACC, TX, Epi><<<grid, SBLK, lds, s>>>(a.n, a.m, a.rp, a.lc, a.tiles,       \
                                                                      a.tile_cnt, v, lx.x, epi, pb);       \
    HBGS_HIP(hipGetLastError());                                                                           \
    return;                                                                                                \
  }
        HBGS_TILED(256)
        HBGS_TILED(128)
        HBGS_TILED(64)
#undef HBGS_TILED
      }
    }
  }
#define HBGS_ROWS(RB)                                                                                      \
  case RB:                                                                                                 \
    if (e0)                                                                                                \
      hipExtLaunchKernelGGL(k_csr_rows<RB, TV, TACC, Col, LoadX, Epi>, dim3((a.n + RB - 1) / RB), dim3(SBLK), \
                            0, s, e0, e1, 0, a.n, a.rp, col, v, lx, epi, vec);                             \
    else                                                                                                   \
      k_csr_rows<RB, TV, TACC, Col, LoadX, Epi><<<(a.n + RB - 1) / RB, SBLK, 0, s>>>(a.n, a.rp, col, v, lx, epi, vec); \
    HBGS_HIP(hipGetLastError());                                                                           \
    return;
  switch (rb) {
    HBGS_ROWS(512)
    HBGS_ROWS(256)
    HBGS_ROWS(128)
    HBGS_ROWS(64)
    HBGS_ROWS(32)
    HBGS_ROWS(16)
    HBGS_ROWS(8)
    HBGS_ROWS(4)
    default: break;
  }
#undef HBGS_ROWS
  float avg = a.avg_row();
  int lpr = avg <= 1.5f ? 1 : avg <= 3.f ? 2 : avg <= 6.f ? 4 : avg <= 16.f ? 8 : avg <= 64.f ? 16 : avg <= 128.f ? 32 : 64;
  unsigned grid = (unsigned)(((int64_t)a.n * lpr + BLK - 1) / BLK);
#define HBGS_CASE(L)                                                                                       \
  case L:                                                                                                  \
    if (e0)                                                                                                \
      hipExtLaunchKernelGGL(k_csr<L, TV, TACC, Col, LoadX, Epi>, dim3(grid), dim3(BLK), 0, s, e0, e1, 0, a.n, \
                            a.rp, col, v, lx, epi);                                                        \
    else                                                                                                   \
      k_csr<L, TV, TACC, Col, LoadX, Epi><<<grid, BLK, 0, s>>>(a.n, a.rp, col, v, lx, epi);                \
    break;
  switch (lpr) {
    HBGS_CASE(1)
    HBGS_CASE(2)
    HBGS_CASE(4)
    HBGS_CASE(8)
    HBGS_CASE(16)
    HBGS_CASE(32)
    HBGS_CASE(64)
  }
#undef HBGS_CASE
  HBGS_HIP(hipGetLastError());
}

template <class TV, class TACC, class LoadX, class Epi>
static void launch_csr(const DCsr& a, const TV* v, LoadX lx, Epi epi, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr) {
  if (a.n == 0) return;
  if (a.nnz == 0) {  // rows without entries: epilogue of an empty sum
    if (e0) HBGS_HIP(hipEventRecord(e0, s));
    k_empty<TACC, Epi><<<grid_for(a.n, 256), 256, 0, s>>>(a.n, epi);
    HBGS_HIP(hipGetLastError());
    if (e1) HBGS_HIP(hipEventRecord(e1, s));
    return;
  }
  if (a.cd)
    launch_csr_cols<TV, TACC>(a, ColPacked{a.cd, a.cb}, v, lx, epi, s, e0, e1);
  else
    launch_csr_cols<TV, TACC>(a, ColPlain{a.ci}, v, lx, epi, s, e0, e1);
}

// operand loaders
template <class T>
struct LoadArr {
  const T* __restrict__ x;
  __device__ T operator()(int k) const { return x[k]; }
};

// Epilogues: load(i) issues the row's vector loads (before the row sum, so
// they overlap it); store(i, acc, pre) finishes the row.
template <class T, class TACC>
struct EpiStore {
  T* __restrict__ y;
  struct Pre {};
  __device__ Pre load(int) const { return {}; }
  __device__ void store(int i, TACC acc, Pre) const { y[i] = (T)acc; }
};
template <class T, class TACC>
struct EpiAdd {
  T* __restrict__ y;
  struct Pre {
    T y;
  };
  __device__ Pre load(int i) const { return {y[i]}; }
  __device__ void store(int i, TACC acc, Pre p) const { y[i] = p.y + (T)acc; }
};
// right-hand side of the next level: y = acc and, when the consumer level
// smooths with degree 2, its first Chebyshev direction d0 = (D^-1 y) / theta
template <class T>
struct EpiRhs {
  T* __restrict__ y;
  const T* __restrict__ dinv;
  T* __restrict__ d0;
  T c0;
  struct Pre {
    T dinv;
  };
  __device__ Pre load(int i) const { return {d0 ? dinv[i] : T(0)}; }
  __device__ void store(int i, T acc, Pre p) const {
    y[i] = acc;
    if (d0) d0[i] = p.dinv * acc * c0;
  }
};
template <class T>
struct EpiResid {
  const T* __restrict__ b;
  T* __restrict__ r;
  struct Pre {
    T b;
  };
  __device__ Pre load(int i) const { return {b[i]}; }
  __device__ void store(int i, T acc, Pre p) const { r[i] = p.b - acc; }
};
// degree-2 pre-smoothing from zero, d0 = (D^-1 b) / theta given:
// x = d0 + c1 d0 + c2 D^-1 (b - A d0)
template <class T>
struct EpiChebPre2 {
  const T* __restrict__ dinv;
  const T* __restrict__ b;
  const T* __restrict__ d0;
  T* __restrict__ x;
  T c1, c2;
  struct Pre {
    T dinv, b, d0;
  };
  __device__ Pre load(int i) const { return {dinv[i], b[i], d0[i]}; }
  __device__ void store(int i, T ad, Pre p) const {
    T r1 = p.b - ad;
    T d1 = c1 * p.d0 + c2 * (p.dinv * r1);
    x[i] = p.d0 + d1;
  }
};
// post-smoothing start from x: r = b - A x, d = D^-1 r / theta
template <class T>
struct EpiChebPostA {
  const T* __restrict__ dinv;
  const T* __restrict__ b;
  T* __restrict__ r;
  T* __restrict__ d;
  T c0;
  struct Pre {
    T dinv, b;
  };
  __device__ Pre load(int i) const { return {dinv[i], b[i]}; }
  __device__ void store(int i, T ax, Pre p) const {
    T ri = p.b - ax;
    r[i] = ri;
    d[i] = p.dinv * ri * c0;
  }
};
// Chebyshev step: r -= A d; dn = c1 d + c2 D^-1 r; x (+ d if pending) += dn
template <class T, bool ADD_D, bool KEEP>
struct EpiChebStep {
  const T* __restrict__ dinv;
  const T* __restrict__ d;
  T* __restrict__ r;
  T* __restrict__ dn;
  T* __restrict__ x;
  T c1, c2;
  struct Pre {
    T dinv, d, r, x;
  };
  __device__ Pre load(int i) const { return {dinv[i], d[i], r[i], x[i]}; }
  __device__ void store(int i, T ad, Pre p) const {
    T ri = p.r - ad;
    T di = c1 * p.d + c2 * (p.dinv * ri);
    T xi = ADD_D ? p.x + p.d : p.x;
    x[i] = xi + di;
    if (KEEP) {
      r[i] = ri;
      dn[i] = di;
    }
  }
};
// coupling: t = (T)v - sum a z, plus the fine level's d0 = (D^-1 t) / theta
template <class T>
struct EpiCouple {
  const double* __restrict__ v;
  T* __restrict__ t;
  const T* __restrict__ dinv;
  T* __restrict__ d0;
  T c0;
  const double* __restrict__ vs;  // divisor of v (null: none)
  struct Pre {
    double v;
    T dinv;
  };
  __device__ Pre load(int i) const { return {vs ? v[i] / *vs : v[i], d0 ? dinv[i] : T(0)}; }
  __device__ void store(int i, T acc, Pre p) const {
    T ti = (T)p.v - acc;
    t[i] = ti;
    if (d0) d0[i] = p.dinv * ti * c0;
  }
};

// rows of the interleaved [A P; P] operator: even row 2i gives
// r_i = r_i - (A P xc)_i and d_i = D^-1 r_i / theta, odd row 2i+1 gives
// x_i = x_i + (P xc)_i
template <class T>
struct EpiPostQ {
  const T* __restrict__ dinv;
  T* __restrict__ r;
  T* __restrict__ x;
  T* __restrict__ d;
  T c0;
  struct Pre {
    T a, b;
  };
  __device__ Pre load(int k) const {
    const int i = k >> 1;
    if (k & 1) return {x[i], T(0)};
    return {r[i], dinv[i]};
  }
  __device__ void store(int k, T acc, Pre p) const {
    const int i = k >> 1;
    if (k & 1) {
      x[i] = p.a + acc;
    } else {
      const T ri = p.a - acc;
      r[i] = ri;
      d[i] = p.b * ri * c0;
    }
  }
};

// group right-hand side of the nested form: t = v / vs - sum a z (FP64 out)
struct EpiSubFrom {
  const double* __restrict__ v;
  double* __restrict__ t;
  const double* __restrict__ vs;  // divisor of v (null: none)
  struct Pre {
    double v;
  };
  __device__ Pre load(int i) const { return {vs ? v[i] / *vs : v[i]}; }
  __device__ void store(int i, double acc, Pre p) const { t[i] = p.v - acc; }
};

// ---------------------------------------------------------- outer SpMV
void spmv_outer_f64(const DCsr& a, const double* x, double* y, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_csr<double, double>(a, a.v, LoadArr<double>{x}, EpiStore<double, double>{y}, s, e0, e1);
}
void spmv_outer_mixed(const DCsr& a, const float* x, double* y, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  launch_csr<double, double>(a, a.v, LoadArr<float>{x}, EpiStore<double, double>{y}, s, e0, e1);
}
template <class TZ>
void couple_f64(const DCsr& a, const double* v, const TZ* z, double* t, const double* vs, hipStream_t s) {
  launch_csr<double, double>(a, a.v, LoadArr<TZ>{z}, EpiSubFrom{v, t, vs}, s);
}
template void couple_f64<float>(const DCsr&, const double*, const float*, double*, const double*, hipStream_t);
template void couple_f64<double>(const DCsr&, const double*, const double*, double*, const double*, hipStream_t);
void spmv_resid_f64(const DCsr& a, const double* x, const double* b, double* r, hipStream_t s) {
  launch_csr<double, double>(a, a.v, LoadArr<double>{x}, EpiResid<double>{b, r}, s);
}

// ------------------------------------------------------- V-cycle pieces
template <class T>
static const T* vals_of(const DCsr& a);
template <>
const double* vals_of<double>(const DCsr& a) {
  return a.v;
}
template <>
const float* vals_of<float>(const DCsr& a) {
  return a.vf;
}

template <class T>
__global__ void k_cheb_init0(int n, const T* __restrict__ dinv, const T* __restrict__ b, T c0, T* __restrict__ r,
                             T* __restrict__ d, T* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
    T di = dinv[i] * b[i] * c0;
    r[i] = b[i];
    d[i] = di;
    x[i] = di;
  }
}

template <class T>
void VcOps<T>::pre2(const DCsr& a, const T* dinv, const ChebCoef& c, const T* b, const T* d0, T* x, hipStream_t s) {
  launch_csr<T, T>(a, vals_of<T>(a), LoadArr<T>{d0}, EpiChebPre2<T>{dinv, b, d0, x, (T)c.c1[1], (T)c.c2[1]}, s);
}

template <class T>
__global__ void k_make_d0(int n, const T* __restrict__ b, const T* __restrict__ dinv, T c0, T* __restrict__ d0) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) d0[i] = dinv[i] * b[i] * c0;
}
template <class T>
void VcOps<T>::make_d0(int n, const T* b, const T* dinv, double c0, T* d0, hipStream_t s) {
  k_make_d0<T><<<grid_for(n, BLK), BLK, 0, s>>>(n, b, dinv, (T)c0, d0);
  HBGS_HIP(hipGetLastError());
}

template <class T>
void VcOps<T>::init0(int n, const T* dinv, const ChebCoef& c, const T* b, T* r, T* d, T* x, hipStream_t s) {
  k_cheb_init0<T><<<grid_for(n, BLK), BLK, 0, s>>>(n, dinv, b, (T)c.c0, r, d, x);
  HBGS_HIP(hipGetLastError());
}

template <class T>
void VcOps<T>::post_start(const DCsr& a, const T* dinv, const ChebCoef& c, const T* b, const T* x, T* r, T* d,
                          hipStream_t s) {
  launch_csr<T, T>(a, vals_of<T>(a), LoadArr<T>{x}, EpiChebPostA<T>{dinv, b, r, d, (T)c.c0}, s);
}

template <class T>
__global__ void k_add(int n, const T* __restrict__ d, T* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) x[i] = x[i] + d[i];
}

template <class T>
void VcOps<T>::step(const DCsr& a, const T* dinv, const ChebCoef& c, int k, bool add_d, bool keep, T* r,
                    const T* d, T* dn, T* x, hipStream_t s) {
  const T* av = vals_of<T>(a);
  const T c1 = (T)c.c1[k], c2 = (T)c.c2[k];
  if (add_d && keep)
    launch_csr<T, T>(a, av, LoadArr<T>{d}, EpiChebStep<T, true, true>{dinv, d, r, dn, x, c1, c2}, s);
  else if (add_d)
    launch_csr<T, T>(a, av, LoadArr<T>{d}, EpiChebStep<T, true, false>{dinv, d, r, dn, x, c1, c2}, s);
  else if (keep)
    launch_csr<T, T>(a, av, LoadArr<T>{d}, EpiChebStep<T, false, true>{dinv, d, r, dn, x, c1, c2}, s);
  else
    launch_csr<T, T>(a, av, LoadArr<T>{d}, EpiChebStep<T, false, false>{dinv, d, r, dn, x, c1, c2}, s);
}

template <class T>
void VcOps<T>::add(int n, const T* d, T* x, hipStream_t s) {
  k_add<T><<<grid_for(n, BLK), BLK, 0, s>>>(n, d, x);
  HBGS_HIP(hipGetLastError());
}

template <class T>
void VcOps<T>::resid(const DCsr& a, const T* b, const T* x, T* r, hipStream_t s) {
  launch_csr<T, T>(a, vals_of<T>(a), LoadArr<T>{x}, EpiResid<T>{b, r}, s);
}
template <class T>
void VcOps<T>::restrict_(const DCsr& rmat, const T* r, T* bc, const T* dinv_c, double c0_c, T* d0_c,
                         hipStream_t s) {
  launch_csr<T, T>(rmat, vals_of<T>(rmat), LoadArr<T>{r}, EpiRhs<T>{bc, dinv_c, d0_c, (T)c0_c}, s);
}
template <class T>
void VcOps<T>::prolong(const DCsr& p, const T* xc, T* x, hipStream_t s) {
  launch_csr<T, T>(p, vals_of<T>(p), LoadArr<T>{xc}, EpiAdd<T, T>{x}, s);
}
template <class T>
void VcOps<T>::post_q(const DCsr& q, const T* dinv, const ChebCoef& c, const T* xc, T* r, T* x, T* d,
                      hipStream_t s) {
  launch_csr<T, T>(q, vals_of<T>(q), LoadArr<T>{xc}, EpiPostQ<T>{dinv, r, x, d, (T)c.c0}, s);
}
template <class T>
void VcOps<T>::couple(const DCsr& c, const double* v, const T* z, T* t, const T* dinv, double c0, T* d0,
                      const double* vs, hipStream_t s) {
  launch_csr<T, T>(c, vals_of<T>(c), LoadArr<T>{z}, EpiCouple<T>{v, t, dinv, d0, (T)c0, vs}, s);
}

template <class T>
__global__ void k_cast_in(int n, const double* __restrict__ v, T* __restrict__ t, const T* __restrict__ dinv, T c0,
                          T* __restrict__ d0, const double* __restrict__ vs) {
  const double h = vs ? *vs : 1.0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
    T ti = (T)(vs ? v[i] / h : v[i]);
    t[i] = ti;
    if (d0) d0[i] = dinv[i] * ti * c0;
  }
}
template <class T>
void VcOps<T>::cast_in(int n, const double* v, T* t, const T* dinv, double c0, T* d0, const double* vs,
                       hipStream_t s) {
  k_cast_in<T><<<grid_for(n, BLK), BLK, 0, s>>>(n, v, t, dinv, (T)c0, d0, vs);
  HBGS_HIP(hipGetLastError());
}

// coarsest level: x = A^-1 b with the dense FP64 inverse (row-major; the
// transposed solve passes the stored transpose).  One block per row: the
// row's 8 n bytes are streamed by 256 threads and reduced in fixed order.
template <class T>
__global__ __launch_bounds__(BLK) void k_gemv_block(int n, const double* __restrict__ inv, const T* __restrict__ b,
                                                    T* __restrict__ x) {
  __shared__ double sh[BLK / 64];
  const int row = blockIdx.x;
  const double* m = inv + (int64_t)row * n;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += BLK) acc += m[j] * (double)b[j];
  acc = lanes_sum<double>(acc, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < BLK / 64; ++q) t += sh[q];
    x[row] = (T)t;
  }
}
template <class T>
void VcOps<T>::coarse(int n, const double* inv, int transpose, const T* b, T* x, hipStream_t s) {
  (void)transpose;  // the caller passes the stored transpose of the inverse
  if (n <= 0) return;
  k_gemv_block<T><<<n, BLK, 0, s>>>(n, inv, b, x);
  HBGS_HIP(hipGetLastError());
}

// DD(0)-ILU(0) sweeps: one block per subdomain, level by level, one thread
// per row (each sum in ascending column)
template <class T, bool DIAG>
__global__ __launch_bounds__(BLK) void k_ilu_lower(const int* __restrict__ ord, const int* __restrict__ lev,
                                                   const int* __restrict__ sub, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ v,
                                                   const int* __restrict__ dpos, const T* __restrict__ t, T* y) {
  const int b = blockIdx.x;
  for (int l = sub[b]; l + 1 < sub[b + 1]; ++l) {
    for (int q = lev[l] + threadIdx.x; q < lev[l + 1]; q += BLK) {
      const int i = ord[q];
      T s = t[i];
      for (int k = rp[i]; k < dpos[i]; ++k) s -= v[k] * y[ci[k]];
      y[i] = DIAG ? s / v[dpos[i]] : s;
    }
    __syncthreads();
  }
}
template <class T, bool DIAG>
__global__ __launch_bounds__(BLK) void k_ilu_upper(const int* __restrict__ ord, const int* __restrict__ lev,
                                                   const int* __restrict__ sub, const int* __restrict__ rp,
                                                   const int* __restrict__ ci, const T* __restrict__ v,
                                                   const int* __restrict__ dpos, const T* __restrict__ y, T* z) {
  const int b = blockIdx.x;
  for (int l = sub[b]; l + 1 < sub[b + 1]; ++l) {
    for (int q = lev[l] + threadIdx.x; q < lev[l + 1]; q += BLK) {
      const int i = ord[q];
      T s = y[i];
      for (int k = dpos[i] + 1; k < rp[i + 1]; ++k) s -= v[k] * z[ci[k]];
      z[i] = DIAG ? s / v[dpos[i]] : s;
    }
    __syncthreads();
  }
}
template <class T>
static const T* ilu_vals(const IluLeaf& f, int transpose);
template <>
const double* ilu_vals<double>(const IluLeaf& f, int transpose) {
  return transpose ? f.vT : f.F.v;
}
template <>
const float* ilu_vals<float>(const IluLeaf& f, int transpose) {
  return transpose ? f.vTf : f.F.vf;
}
// z = U^-1 L^-1 t, or z = L^-T U^-T t (lower sweep on the transposed
// factors dividing by the diagonal, then the unit upper sweep)
template <class T>
void VcOps<T>::ilu(const IluLeaf& f, int transpose, const T* t, T* z, hipStream_t s) {
  const T* v = ilu_vals<T>(f, transpose);
  T* y = sizeof(T) == sizeof(double) ? reinterpret_cast<T*>(f.yd) : reinterpret_cast<T*>(f.yf);
  const DCsr& F = f.F;
  if (!transpose) {
    k_ilu_lower<T, false><<<f.nsub, BLK, 0, s>>>(f.ford, f.flev, f.fsub, F.rp, F.ci, v, f.dpos, t, y);
    k_ilu_upper<T, true><<<f.nsub, BLK, 0, s>>>(f.bord, f.blev, f.bsub, F.rp, F.ci, v, f.dpos, y, z);
  } else {
    k_ilu_lower<T, true><<<f.nsub, BLK, 0, s>>>(f.ford, f.flev, f.fsub, F.rp, F.ci, v, f.dpos, t, y);
    k_ilu_upper<T, false><<<f.nsub, BLK, 0, s>>>(f.bord, f.blev, f.bsub, F.rp, F.ci, v, f.dpos, y, z);
  }
  HBGS_HIP(hipGetLastError());
}

template struct VcOps<float>;
template struct VcOps<double>;

// --------------------------------------------------------------- GMRES
__global__ void k_permute_in(int n, const int* __restrict__ perm, const double* __restrict__ x,
                             double* __restrict__ xp) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) xp[perm[i]] = x[i];
}
__global__ void k_permute_out(int n, const int* __restrict__ perm, const double* __restrict__ xp,
                              double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) x[i] = xp[perm[i]];
}
void permute_in(int n, const int* perm, const double* x, double* xp, hipStream_t s) {
  k_permute_in<<<grid_for(n, BLK), BLK, 0, s>>>(n, perm, x, xp);
  HBGS_HIP(hipGetLastError());
}
void permute_out(int n, const int* perm, const double* xp, double* x, hipStream_t s) {
  k_permute_out<<<grid_for(n, BLK), BLK, 0, s>>>(n, perm, xp, x);
  HBGS_HIP(hipGetLastError());
}
__global__ void k_permute_out_f32(int n, const int* __restrict__ perm, const float* __restrict__ xp,
                                  double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK)
    x[i] = (double)xp[perm[i]];
}
void permute_out_f32(int n, const int* perm, const float* xp, double* x, hipStream_t s) {
  k_permute_out_f32<<<grid_for(n, BLK), BLK, 0, s>>>(n, perm, xp, x);
  HBGS_HIP(hipGetLastError());
}

constexpr int DOT_BLOCKS_MAX = 1024;
int dot_blocks(int n) {
  int64_t b = ((int64_t)n + BLK * 8 - 1) / (BLK * 8);
  if (b < 1) b = 1;
  if (b > DOT_BLOCKS_MAX) b = DOT_BLOCKS_MAX;
  return (int)b;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = lanes_sum<double>(v, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < BLK / 64; ++q) t += sh[q];
  return t;
}

// Givens rotation update of Hessenberg column j (H is (m+1) x m, row-major
// with leading dimension m) by one thread, on a copy of the column in LDS:
// col[k] = h1[k] + h2[k] (k <= j) on entry; the earlier rotations' cosines
// and sines in cs/sn (LDS).  h1/h2: first and second Gram-Schmidt
// coefficients; h2[j+1] = ||w||^2 after the first pass; ga.h1[j+1] = ||w||^2
// before orthogonalisation.  On exit col[0..j+1] is the rotated column;
// scal (device) and host_scal (pinned host memory) receive |g_{j+1}|,
// h_{j+1,j} and ||w||.
__device__ void givens_update(const GivensArgs& ga, const double* h2, double* col, const double* cs,
                              const double* sn) {
  const int j = ga.j;
  // ||w - V h2||^2 = ||w||^2 - ||h2||^2 for orthonormal V
  double ss = h2[j + 1];
  for (int k = 0; k <= j; ++k) ss -= h2[k] * h2[k];
  const double hn = ss > 0.0 ? sqrt(ss) : 0.0;
  col[j + 1] = hn;
  // the rotated entry k+1 is carried in a register to the next rotation
  double a = col[0];
  for (int k = 0; k < j; ++k) {
    const double b = col[k + 1];
    col[k] = cs[k] * a + sn[k] * b;
    a = -sn[k] * a + cs[k] * b;
  }
  const double b = hn;
  const double den = sqrt(a * a + b * b);
  const double c = a / den, sj = b / den;
  ga.cs[j] = c;
  ga.sn[j] = sj;
  col[j] = den;
  col[j + 1] = 0.0;
  const double gj = ga.g[j];
  ga.g[j + 1] = -sj * gj;
  ga.g[j] = c * gj;
  const double est = fabs(-sj * gj), w0 = sqrt(ga.h1[j + 1]);
  ga.scal[0] = est;
  ga.scal[1] = hn;
  ga.scal[2] = w0;
  if (ga.host_scal) {  // the estimate last: the host polls it
    ga.host_scal[1] = hn;
    ga.host_scal[2] = w0;
    __threadfence_system();  // orders the two values before the estimate
    ga.host_scal[0] = est;   // no wait for its arrival: the thread has nothing left to do
  }
}

// Classical Gram-Schmidt pass over rows: w holds column j+1 of V.
//   UPD:  w -= sum_k h_k V_k           (k <= j)
//   DOTS: part_k = sum V_k . w          (k <= j), after the update
//   FIN:  (with DOTS, not UPD) column j still holds the previous step's
//         once-orthogonalised vector u; it is finished first, in place, as
//         V_j = (u - sum_{k<j} hp_k V_k) / scal[1] (the previous step's
//         second-pass coefficients hp and h_{j,j-1}), then used in the dots
//   always: part_{j+1} = w . w
// (per-block partial sums; the reduction over blocks is a separate launch,
// since a grid-wide completion fence costs more than the launch)
template <int MAXV, bool UPD, bool DOTS, bool FIN>
__global__ __launch_bounds__(BLK) void k_cgs(int n, int nv, double* __restrict__ V, size_t ldv,
                                             double* __restrict__ w, const double* __restrict__ h,
                                             double* __restrict__ part, const double* __restrict__ hp,
                                             const double* __restrict__ scal) {
  static_assert(!(FIN && UPD) && (!FIN || DOTS), "FIN finishes a basis vector ahead of a dots-only pass");
  __shared__ double sh[BLK / 64];
  double acc[DOTS ? MAXV : 1];
  double hh[UPD ? MAXV : 1];
#pragma unroll
  for (int k = 0; k < (DOTS ? MAXV : 1); ++k) acc[k] = 0.0;
  if (UPD) {
#pragma unroll
    for (int k = 0; k < MAXV; ++k) hh[k] = k < nv ? h[k < nv ? k : 0] : 0.0;
  }
  const int nrd = FIN ? nv - 1 : nv;  // columns read as they stand
  const double hn = FIN ? scal[1] : 1.0;
  double hq[FIN ? MAXV : 1];  // in registers: zero beyond nrd, where vk is zero too
  if (FIN) {
#pragma unroll
    for (int k = 0; k < MAXV; ++k) hq[k] = k < nrd ? hp[k < nrd ? k : 0] : 0.0;
  }
  double ww = 0.0, accf = 0.0;
  // U rows per step (i, i + stride, ...), all their loads issued before any
  // use; the rows are accumulated in the order of a one-row loop
  constexpr int U = MAXV <= 16 ? 2 : 1;
  const int64_t stride = (int64_t)gridDim.x * BLK;
  for (int64_t i0 = (int64_t)blockIdx.x * BLK + threadIdx.x; i0 < n; i0 += U * stride) {
    double vk[U][MAXV], uu[U], wv[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t i = i0 + r * stride;
      const bool in = i < n;
#pragma unroll
      for (int k = 0; k < MAXV; ++k) vk[r][k] = in && k < nrd ? V[(size_t)(k < nrd ? k : 0) * ldv + i] : 0.0;
      uu[r] = FIN && in ? V[(size_t)nrd * ldv + i] : 0.0;
      wv[r] = in ? w[i] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t i = i0 + r * stride;
      if (i >= n) break;
      double vf = 0.0;
      if (FIN) {
        double u = uu[r];
#pragma unroll
        for (int k = 0; k < MAXV; ++k) u -= hq[k] * vk[r][k];
        vf = u / hn;
        V[(size_t)nrd * ldv + i] = vf;
      }
      double wi = wv[r];
      if (UPD) {
#pragma unroll
        for (int k = 0; k < MAXV; ++k) wi -= hh[k] * vk[r][k];
        w[i] = wi;
      }
      if (DOTS) {
#pragma unroll
        for (int k = 0; k < MAXV; ++k) acc[k] += vk[r][k] * wi;
        if (FIN) accf += vf * wi;  // the finished column's dot: acc[nrd] only saw zeros
      }
      ww += wi * wi;
    }
  }
  const int nb = gridDim.x;
  if (DOTS) {
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      if (k < nv) {
        double t = block_sum(FIN && k == nrd ? accf : acc[k], sh);
        if (threadIdx.x == 0) part[(size_t)k * nb + blockIdx.x] = t;
      }
    }
  }
  double t = block_sum(ww, sh);
  if (threadIdx.x == 0) part[(size_t)nv * nb + blockIdx.x] = t;
}

template <bool UPD, bool DOTS, bool FIN = false>
static void launch_cgs(int n, int nv, double* V, size_t ldv, double* w, const double* h, double* part,
                       const double* hp, const double* scal, hipStream_t s) {
  int nb = dot_blocks(n);
  if (nv <= 8)
    k_cgs<8, UPD, DOTS, FIN><<<nb, BLK, 0, s>>>(n, nv, V, ldv, w, h, part, hp, scal);
  else if (nv <= 16)
    k_cgs<16, UPD, DOTS, FIN><<<nb, BLK, 0, s>>>(n, nv, V, ldv, w, h, part, hp, scal);
  else if (nv <= 32)
    k_cgs<32, UPD, DOTS, FIN><<<nb, BLK, 0, s>>>(n, nv, V, ldv, w, h, part, hp, scal);
  else if (nv <= 48)  // 16-25% faster than the 64-vector form (one wave per SIMD) at 33-48 vectors
    k_cgs<48, UPD, DOTS, FIN><<<nb, BLK, 0, s>>>(n, nv, V, ldv, w, h, part, hp, scal);
  else
    k_cgs<64, UPD, DOTS, FIN><<<nb, BLK, 0, s>>>(n, nv, V, ldv, w, h, part, hp, scal);
  HBGS_HIP(hipGetLastError());
}

// out[k] = sum over blocks of part[k*nb + b] (fixed order per k)
__global__ __launch_bounds__(BLK) void k_reduce(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[BLK / 64];
  const double* p = part + (size_t)blockIdx.x * nb;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += BLK) acc += p[b];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}
void mdot_reduce(int nvec, int nblocks, const double* part, double* out, hipStream_t s) {
  k_reduce<<<nvec, BLK, 0, s>>>(nblocks, part, out);
  HBGS_HIP(hipGetLastError());
}

// one block: out[k] = sum over blocks of part[k*nb + b] for k < nvec (one
// wave per vector, fixed order), then the Givens update from out.  The
// column's first-pass coefficients and the earlier rotations are read by
// many threads at once into LDS, so the one thread's sequential update
// waits on no global loads.
constexpr int RG_BLK = 1024;
constexpr int RG_MAXV = 66;
__global__ __launch_bounds__(RG_BLK) void k_reduce_givens(int nvec, int nb, const double* __restrict__ part,
                                                          double* __restrict__ out, GivensArgs ga) {
  __shared__ double red[RG_MAXV], col[RG_MAXV], scs[RG_MAXV], ssn[RG_MAXV];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = ga.j;
  const double h1 = tid <= j ? ga.h1[tid] : 0.0;
  if (tid < j) {
    scs[tid] = ga.cs[tid];
    ssn[tid] = ga.sn[tid];
  }
  for (int k = wave; k < nvec; k += RG_BLK / 64) {
    const double* p = part + (size_t)k * nb;
    double a = 0.0;
    for (int b = lane; b < nb; b += 64) a += p[b];
    a = lanes_sum<double>(a, 64);
    if (lane == 0) red[k] = a;
  }
  __syncthreads();
  if (tid < nvec) out[tid] = red[tid];
  if (tid <= j) col[tid] = h1 + red[tid];
  __syncthreads();
  if (tid == 0) givens_update(ga, red, col, scs, ssn);
  __syncthreads();
  if (tid <= j + 1) ga.H[(size_t)tid * ga.m + j] = col[tid];
}

void cgs_dots(int n, int j, const double* V, size_t ldv, const double* w, double* part, hipStream_t s) {
  launch_cgs<false, true>(n, j + 1, const_cast<double*>(V), ldv, const_cast<double*>(w), nullptr, part, nullptr,
                          nullptr, s);
}
void cgs_finish_dots(int n, int j, double* V, size_t ldv, const double* w, const double* hp, const double* scal,
                     double* part, hipStream_t s) {
  launch_cgs<false, true, true>(n, j + 1, V, ldv, const_cast<double*>(w), nullptr, part, hp, scal, s);
}
void cgs_update_dots(int n, int j, const double* V, size_t ldv, double* w, const double* h1, double* part,
                     hipStream_t s) {
  launch_cgs<true, true>(n, j + 1, const_cast<double*>(V), ldv, w, h1, part, nullptr, nullptr, s);
}
void reduce_givens(int n, int j, const double* part, double* h2, const GivensArgs& ga, hipStream_t s) {
  if (j + 2 > RG_MAXV) HBGS_FAIL(HBGS_EINVAL, "Gram-Schmidt basis too large");
  k_reduce_givens<<<1, RG_BLK, 0, s>>>(j + 2, dot_blocks(n), part, h2, ga);
  HBGS_HIP(hipGetLastError());
}
// y = R^-1 g with R the leading jend x jend upper triangle of H: the block
// stages R and g in LDS, then one thread substitutes backwards (no global
// loads inside the dependent chain)
constexpr int BS_MAX = 64;
__global__ __launch_bounds__(BLK) void k_backsolve(int jend, int m, const double* __restrict__ H,
                                                   const double* __restrict__ g, double* __restrict__ y) {
  __shared__ double sr[BS_MAX][BS_MAX + 1];
  __shared__ double sy[BS_MAX], sg[BS_MAX];
  for (int e = threadIdx.x; e < jend * jend; e += BLK) {
    const int i = e / jend, k = e % jend;
    if (k >= i) sr[i][k] = H[(size_t)i * m + k];
  }
  if ((int)threadIdx.x < jend) sg[threadIdx.x] = g[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = jend - 1; i >= 0; --i) {
      double t = sg[i];
      for (int k = i + 1; k < jend; ++k) t -= sr[i][k] * sy[k];
      sy[i] = t / sr[i][i];
    }
  __syncthreads();
  if ((int)threadIdx.x < jend) y[threadIdx.x] = sy[threadIdx.x];
}
void backsolve(int jend, int m, const double* H, const double* g, double* y, hipStream_t s) {
  if (jend > BS_MAX) HBGS_FAIL(HBGS_EINVAL, "least-squares system too large");
  k_backsolve<<<1, BLK, 0, s>>>(jend, m, H, g, y);
  HBGS_HIP(hipGetLastError());
}

template <class TZ>
__global__ void k_xupdate(int n, int jend, const TZ* __restrict__ Z, size_t ldz, const double* __restrict__ y,
                          double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
    double xi = x[i];
    for (int k = 0; k < jend; ++k) xi += y[k] * (double)Z[(size_t)k * ldz + i];
    x[i] = xi;
  }
}
template <class TZ>
void xupdate(int n, int jend, const TZ* Z, size_t ldz, const double* y, double* x, hipStream_t s) {
  k_xupdate<TZ><<<grid_for(n, BLK), BLK, 0, s>>>(n, jend, Z, ldz, y, x);
  HBGS_HIP(hipGetLastError());
}
template void xupdate<float>(int, int, const float*, size_t, const double*, double*, hipStream_t);
template void xupdate<double>(int, int, const double*, size_t, const double*, double*, hipStream_t);

__global__ __launch_bounds__(BLK) void k_norm2_part(int n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[BLK / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK)
    acc += x[i] * x[i];
  double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
void norm2_partial(int n, const double* x, double* part, hipStream_t s) {
  k_norm2_part<<<dot_blocks(n), BLK, 0, s>>>(n, x, part);
  HBGS_HIP(hipGetLastError());
}

__global__ void k_scale_copy(int n, const double* __restrict__ r, const double* __restrict__ ss,
                             double* __restrict__ v) {
  const double nr = sqrt(*ss);
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) v[i] = r[i] / nr;
}
void scale_copy(int n, const double* r, const double* part_sum, double* v, hipStream_t s) {
  k_scale_copy<<<grid_for(n, BLK), BLK, 0, s>>>(n, r, part_sum, v);
  HBGS_HIP(hipGetLastError());
}

__global__ void k_grad(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ lam,
                       const double* __restrict__ x, double* __restrict__ g) {
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) {
    double li = lam[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) g[k] = -li * x[ci[k]];
  }
}
void grad_values(int n, const int* rp, const int* ci, const double* lam, const double* x, double* g,
                 hipStream_t s) {
  k_grad<<<grid_for(n, BLK), BLK, 0, s>>>(n, rp, ci, lam, x, g);
  HBGS_HIP(hipGetLastError());
}

__global__ void k_compare_int(int64_t n, const int* __restrict__ a, const int* __restrict__ b, int* diff) {
  int d = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLK) d |= a[i] != b[i];
  if (d) atomicOr(diff, 1);
}
void compare_int(int64_t n, const int* a, const int* b, int* diff, hipStream_t s) {
  if (n == 0) return;
  k_compare_int<<<grid_for(n, BLK, 65536), BLK, 0, s>>>(n, a, b, diff);
  HBGS_HIP(hipGetLastError());
}

struct FieldRanges {
  int nf;
  int lo[HBGS_MAX_FIELDS], hi[HBGS_MAX_FIELDS];
};
__global__ void k_column_fields(int64_t nnz, const int* __restrict__ ci, FieldRanges fr, int* mask) {
  int m = 0;
  for (int64_t k = (int64_t)blockIdx.x * BLK + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * BLK) {
    int c = ci[k];
    for (int f = 0; f < fr.nf; ++f)
      if (c >= fr.lo[f] && c < fr.hi[f]) m |= 1 << f;
  }
  if (m) atomicOr(mask, m);
}
void column_fields(const DCsr& c, int nf, const int* lo, const int* hi, int* mask, hipStream_t s) {
  if (c.nnz == 0) return;
  FieldRanges fr;
  fr.nf = nf;
  for (int f = 0; f < nf; ++f) {
    fr.lo[f] = lo[f];
    fr.hi[f] = hi[f];
  }
  k_column_fields<<<grid_for(c.nnz, BLK, 4096), BLK, 0, s>>>(c.nnz, c.ci, fr, mask);
  HBGS_HIP(hipGetLastError());
}

}  // namespace solve
}  // namespace hbgs
