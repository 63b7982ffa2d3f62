// Outer-iteration kernels of the CG-accelerated block Cimmino method
// (Algorithm 2 of the paper): the sparse products u = A p and psi = A^T y,
// and the fused vector updates with deterministic per-system reductions.
//
// Layout: all vectors are float64 over the concatenated index range of the
// (batched) system.  Row-space vectors (u, s, y, f) are in the block-permuted
// row order; column-space vectors (x, r, p, psi) in the original column
// order.  Both ranges are cut into the same tiles of TILE entries that never
// straddle a system; one workgroup handles one tile and writes one partial
// sum per reduced quantity, and every consumer re-adds a system's partials
// in the same fixed order, so all reductions are bitwise reproducible.
#include "common.h"

#include <cmath>

namespace {

__device__ __forceinline__ int tile_of_block() { return blockIdx.x; }

// Sum over the `lanes`-wide lane group of x (lanes a power of two <= 64); the
// group's first lane holds the result.
template <int L>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_down(v, o, L);
  return v;
}

template <int L>
__device__ __forceinline__ float group_sumf(float v) {
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) v += __shfl_down(v, o, L);
  return v;
}

// This lane's part of a row sum: entries e0 + l, e0 + l + L, ... in that
// order (so the rounding is that of the plain loop), in batches of U whose
// index and value loads, then gathers, are all issued before the arithmetic.
// Past the row's end a lane loads its last entry again and does not add it:
// loads under a per-entry condition let the compiler wait for each index
// before the next load is issued.
template <int L, typename V, typename ACC>
__device__ __forceinline__ ACC lane_row_sum(const int* __restrict__ col, const V* __restrict__ val,
                                            const double* __restrict__ x, int e0, int e1, int l) {
  constexpr int U = L <= 2 ? 8 : 4;
  ACC acc = (ACC)0;
  for (int e = e0 + l; e < e1; e += U * L) {
    int c[U];
    V v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int ek = min(e + k * L, e1 - 1);
      c[k] = col[ek];
      v[k] = val[ek];
    }
    ACC xv[U];
#pragma unroll
    for (int k = 0; k < U; ++k) xv[k] = (ACC)x[c[k]];
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (e + k * L < e1) acc += (ACC)v[k] * xv[k];
  }
  return acc;
}

// y[i] = sum_e val[e] * x[col[e]] for the rows of this tile (row-space tile).
template <int L, bool MIXED>
__global__ void __launch_bounds__(VEC_THREADS)
k_spmv(const int* __restrict__ rowptr, const int* __restrict__ col,
       const double* __restrict__ val, const float* __restrict__ val32,
       const double* __restrict__ x, double* __restrict__ y, OuterState S, int skip_done) {
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (skip_done && S.done[sys]) return;
  const int r0 = S.tile_start[t], r1 = S.tile_start[t + 1];
  const int g = threadIdx.x / L, l = threadIdx.x % L;
  constexpr int RPP = VEC_THREADS / L;  // rows per pass
  for (int i = r0 + g; i < r1; i += RPP) {
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    if constexpr (MIXED) {
      float acc = lane_row_sum<L, float, float>(col, val32, x, e0, e1, l);
      acc = group_sumf<L>(acc);
      if (l == 0) y[i] = (double)acc;
    } else {
      double acc = lane_row_sum<L, double, double>(col, val, x, e0, e1, l);
      acc = group_sum<L>(acc);
      if (l == 0) y[i] = acc;
    }
  }
}

// ---------------------------------------------------------- sliced ELL
// The same three products on the sliced-ELL copies (SellMat): one workgroup
// per tile, one wavefront per 64-row slice, one row per lane.  Every index
// and value load of a wavefront is a contiguous 256- or 512-byte line.  A
// lane sums its row's entries in their stored order, as the one-lane-per-row
// CSR kernels do, in batches of 8 whose loads, then gathers, are issued
// before the arithmetic; padding entries carry the value 0.
constexpr int SELL_THREADS = 64 * SELL_SLICES;

// Entries k0 .. k0 + N - 1 of a lane's slice row, N fixed: every index and
// value load, then every gather, then the sums in stored order.
template <int N, typename V, typename ACC>
__device__ __forceinline__ ACC sell_chunk(const int* __restrict__ col, const V* __restrict__ val,
                                          const double* __restrict__ x, long long e, int k0,
                                          ACC acc) {
  int c[N];
  V v[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    c[q] = col[e + (long long)(k0 + q) * 64];
    v[q] = val[e + (long long)(k0 + q) * 64];
  }
  ACC xv[N];
#pragma unroll
  for (int q = 0; q < N; ++q) xv[q] = (ACC)x[c[q]];
#pragma unroll
  for (int q = 0; q < N; ++q) acc += (ACC)v[q] * xv[q];
  return acc;
}

// The last nb < 8 entries of a slice whose width is the same on every lane
// of the wavefront: one fixed-size chunk per count.  (Loads under a per-entry
// condition let the compiler wait for each index before the next load is
// issued, one round trip per entry; loads repeated up to 8 entries cost
// issue slots on the narrow slices of five-point stencils.)
template <typename V, typename ACC>
__device__ __forceinline__ ACC sell_tail(const int* __restrict__ col, const V* __restrict__ val,
                                         const double* __restrict__ x, long long e, int k0, int nb,
                                         ACC acc) {
  switch (nb) {
    case 1: return sell_chunk<1, V, ACC>(col, val, x, e, k0, acc);
    case 2: return sell_chunk<2, V, ACC>(col, val, x, e, k0, acc);
    case 3: return sell_chunk<3, V, ACC>(col, val, x, e, k0, acc);
    case 4: return sell_chunk<4, V, ACC>(col, val, x, e, k0, acc);
    case 5: return sell_chunk<5, V, ACC>(col, val, x, e, k0, acc);
    case 6: return sell_chunk<6, V, ACC>(col, val, x, e, k0, acc);
    case 7: return sell_chunk<7, V, ACC>(col, val, x, e, k0, acc);
    default: return acc;
  }
}

template <typename V, typename ACC>
__device__ __forceinline__ ACC sell_row_sum(const int* __restrict__ col, const V* __restrict__ val,
                                            const double* __restrict__ x, long long e, int w) {
  w = __builtin_amdgcn_readfirstlane(w);
  ACC acc = (ACC)0;
  int k0 = 0;
  for (; k0 + 8 <= w; k0 += 8) acc = sell_chunk<8, V, ACC>(col, val, x, e, k0, acc);
  if (k0 < w) acc = sell_tail<V, ACC>(col, val, x, e, k0, w - k0, acc);
  return acc;
}

template <bool MIXED>
__global__ void __launch_bounds__(SELL_THREADS)
k_spmv_sell(SellMat A, const double* __restrict__ x, double* __restrict__ y, OuterState S,
            int skip_done) {
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (skip_done && S.done[sys]) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sl = t * SELL_SLICES + wave;
  const int i = S.tile_start[t] + wave * 64 + lane;
  const long long e = A.ptr[sl] + lane;
  const int w = A.wid[sl];
  if constexpr (MIXED) {
    const float acc = sell_row_sum<float, float>(A.col, A.val32, x, e, w);
    if (i < S.tile_start[t + 1]) y[i] = (double)acc;
  } else {
    const double acc = sell_row_sum<double, double>(A.col, A.val, x, e, w);
    if (i < S.tile_start[t + 1]) y[i] = acc;
  }
}

template <bool MIXED>
__global__ void __launch_bounds__(SELL_THREADS)
k_spmvT_dot_sell(SellMat AT, const double* __restrict__ y, double* __restrict__ psi,
                 const double* __restrict__ p, OuterState S) {
  __shared__ double sh[SELL_SLICES];
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (S.done[sys]) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sl = t * SELL_SLICES + wave;
  const int j = S.tile_start[t] + wave * 64 + lane;
  const long long e = AT.ptr[sl] + lane;
  const int w = AT.wid[sl];
  // p is loaded before the product, not after it
  const bool own = j < S.tile_start[t + 1];
  const double pj = own ? p[j] : 0.0;
  double acc;
  if constexpr (MIXED)
    acc = (double)sell_row_sum<float, float>(AT.col, AT.val32, y, e, w);
  else
    acc = sell_row_sum<double, double>(AT.col, AT.val, y, e, w);
  double dot = 0.0;
  if (own) {
    psi[j] = acc;
    dot = pj * acc;
  }
  dot = block_sum(dot, sh);
  if (threadIdx.x == 0) S.part_a[t] = dot;
}

__global__ void __launch_bounds__(SELL_THREADS)
k_residual_sell(SellMat A, const double* __restrict__ x, const double* __restrict__ f,
                double* __restrict__ s, OuterState S, const int* __restrict__ mask) {
  __shared__ double sh[SELL_SLICES];
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (mask && !mask[sys]) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sl = t * SELL_SLICES + wave;
  const int i = S.tile_start[t] + wave * 64 + lane;
  const double acc = sell_row_sum<double, double>(A.col, A.val, x, A.ptr[sl] + lane, A.wid[sl]);
  double ss = 0.0;
  if (i < S.tile_start[t + 1]) {
    const double v = f[i] - acc;
    s[i] = v;
    ss = v * v;
  }
  ss = block_sum(ss, sh);
  if (threadIdx.x == 0) S.part_c[t] = ss;
}

// The three sliced-ELL products for nrhs vectors at once (multiple right-hand
// sides).  The vectors are concatenated, vector j at offset j * n1, and the
// per-vector state in S is that of nrhs systems of ntiles1 tiles each (tile t
// of vector j is j * ntiles1 + t).  Grid: ntiles1 x chunks of NR vectors.  The
// index and value loads of a batch of entries serve the chunk's vectors, and
// each vector sums its row in the stored order, so it gets the bits of the
// one-vector kernels above.  The gathered vectors are read either where they
// are (sell_rows_multi: NR gathers per index) or, when the matrix copy's
// columns are scattered (SellMat::il), from a copy made first into M.il with
// the chunk's NR values of index c side by side (sell_rows_multi_il: one
// 64-byte gather per index).
// N entries (fixed) from k0 of a lane's slice row for the chunk's active
// vectors: the index and value loads, then per vector the gathers and sums.
template <int N, typename V, typename ACC, int NR>
__device__ __forceinline__ void multi_chunk(const int* __restrict__ col, const V* __restrict__ val,
                                            const double* __restrict__ x, long long n1, int j0,
                                            const bool (&act)[NR], long long e, int k0,
                                            ACC (&acc)[NR]) {
  int c[N];
  V v[N];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    c[r] = col[e + (long long)(k0 + r) * 64];
    v[r] = val[e + (long long)(k0 + r) * 64];
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    if (!act[q]) continue;
    const double* xq = x + (long long)(j0 + q) * n1;
    ACC xv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) xv[r] = (ACC)xq[c[r]];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[q] += (ACC)v[r] * xv[r];
  }
}

template <typename V, typename ACC, int NR>
__device__ __forceinline__ void sell_rows_multi(const int* __restrict__ col,
                                                const V* __restrict__ val,
                                                const double* __restrict__ x, long long n1,
                                                int j0, const bool (&act)[NR], long long e, int w,
                                                ACC (&acc)[NR]) {
  w = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = (ACC)0;
  int k0 = 0;
  for (; k0 + 8 <= w; k0 += 8) multi_chunk<8, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc);
  // the rest as one fixed-size batch (see sell_tail)
  switch (w - k0) {
    case 1: multi_chunk<1, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    case 2: multi_chunk<2, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    case 3: multi_chunk<3, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    case 4: multi_chunk<4, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    case 5: multi_chunk<5, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    case 6: multi_chunk<6, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    case 7: multi_chunk<7, V, ACC, NR>(col, val, x, n1, j0, act, e, k0, acc); break;
    default: break;
  }
}

typedef double dbl4m __attribute__((ext_vector_type(4)));
// N entries (fixed) from k0, gathered from the interleaved copy: one 32-byte
// vector per 4 right-hand sides and index.
template <int N, typename V, typename ACC, int NR>
__device__ __forceinline__ void multi_chunk_il(const int* __restrict__ col,
                                               const V* __restrict__ val,
                                               const double* __restrict__ xil, long long e, int k0,
                                               ACC (&acc)[NR]) {
  V v[N];
  dbl4m xv[N][NR / 4];
#pragma unroll
  for (int r = 0; r < N; ++r) {
    const int c = col[e + (long long)(k0 + r) * 64];
    v[r] = val[e + (long long)(k0 + r) * 64];
#pragma unroll
    for (int h = 0; h < NR / 4; ++h) xv[r][h] = *(const dbl4m*)(xil + (long long)c * NR + 4 * h);
  }
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] += (ACC)v[r] * (ACC)xv[r][q / 4][q % 4];
}

template <typename V, typename ACC, int NR>
__device__ __forceinline__ void sell_rows_multi_il(const int* __restrict__ col,
                                                   const V* __restrict__ val,
                                                   const double* __restrict__ xil, long long e,
                                                   int w, ACC (&acc)[NR]) {
  static_assert(NR % 4 == 0, "whole 32-byte vectors per index");
  constexpr int B = 4;  // entries per batch: B * NR gathered doubles in flight
  w = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] = (ACC)0;
  int k0 = 0;
  for (; k0 + B <= w; k0 += B) multi_chunk_il<B, V, ACC, NR>(col, val, xil, e, k0, acc);
  switch (w - k0) {
    case 1: multi_chunk_il<1, V, ACC, NR>(col, val, xil, e, k0, acc); break;
    case 2: multi_chunk_il<2, V, ACC, NR>(col, val, xil, e, k0, acc); break;
    case 3: multi_chunk_il<3, V, ACC, NR>(col, val, xil, e, k0, acc); break;
    default: break;
  }
}

// dst[(chunk * n1 + i) * NR + q] = src[(chunk * NR + q) * n1 + i] (zero past
// nrhs): the chunks' vectors interleaved for the gathers above.
template <int NR>
__global__ void __launch_bounds__(256)
k_interleave(const double* __restrict__ src, double* __restrict__ dst, int n1, int nrhs) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int ch = blockIdx.y;
  if (i >= n1) return;
  double v[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int j = ch * NR + q;
    v[q] = j < nrhs ? src[(long long)j * n1 + i] : 0.0;
  }
  dbl4m* d = (dbl4m*)(dst + ((long long)ch * n1 + i) * NR);
#pragma unroll
  for (int h = 0; h < NR / 4; ++h) d[h] = dbl4m{v[4 * h], v[4 * h + 1], v[4 * h + 2], v[4 * h + 3]};
}

// Per-vector block sums of NR values, each summed like block_sum.
template <int NR>
__device__ __forceinline__ void block_sum_multi(double (&v)[NR], double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NR; ++q) v[q] = wave_sum_lane0(v[q]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NR; ++q) sh[q * nw + w] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    double t = 0.0;
    for (int i = 0; i < nw; ++i) t += sh[q * nw + i];
    v[q] = t;
  }
}

template <int NR>
__device__ __forceinline__ bool chunk_active(int j0, int nrhs, const int* flags, bool skip_if_set,
                                             bool (&act)[NR]) {
  bool any = false;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    act[q] = j0 + q < nrhs && !(flags && (flags[j0 + q] != 0) == skip_if_set);
    any = any || act[q];
  }
  return any;
}

template <bool MIXED, bool IL, int NR>
__global__ void __launch_bounds__(SELL_THREADS)
k_spmv_sell_multi(SellMat A, MultiRhs M, const double* __restrict__ x, double* __restrict__ y,
                  OuterState S, int skip_done) {
  const int t = blockIdx.x, j0 = blockIdx.y * NR;
  bool act[NR];
  if (!chunk_active<NR>(j0, M.nrhs, skip_done ? S.done : nullptr, true, act)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sl = t * SELL_SLICES + wave;
  const int i = M.tile_start[t] + wave * 64 + lane;
  const long long e = A.ptr[sl] + lane;
  const int w = A.wid[sl];
  const bool row = i < M.tile_start[t + 1];
  const double* xil = M.il + (long long)blockIdx.y * M.n1 * NR;
  if constexpr (MIXED) {
    float acc[NR];
    if constexpr (IL) sell_rows_multi_il<float, float, NR>(A.col, A.val32, xil, e, w, acc);
    else sell_rows_multi<float, float, NR>(A.col, A.val32, x, M.n1, j0, act, e, w, acc);
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (act[q] && row) y[(long long)(j0 + q) * M.n1 + i] = (double)acc[q];
  } else {
    double acc[NR];
    if constexpr (IL) sell_rows_multi_il<double, double, NR>(A.col, A.val, xil, e, w, acc);
    else sell_rows_multi<double, double, NR>(A.col, A.val, x, M.n1, j0, act, e, w, acc);
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (act[q] && row) y[(long long)(j0 + q) * M.n1 + i] = acc[q];
  }
}

template <bool MIXED, bool IL, int NR>
__global__ void __launch_bounds__(SELL_THREADS)
k_spmvT_dot_sell_multi(SellMat AT, MultiRhs M, const double* __restrict__ y,
                       double* __restrict__ psi, const double* __restrict__ p, OuterState S) {
  __shared__ double sh[NR * SELL_SLICES];
  const int t = blockIdx.x, j0 = blockIdx.y * NR;
  bool act[NR];
  if (!chunk_active<NR>(j0, M.nrhs, S.done, true, act)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sl = t * SELL_SLICES + wave;
  const int j = M.tile_start[t] + wave * 64 + lane;
  const long long e = AT.ptr[sl] + lane;
  const int w = AT.wid[sl];
  const bool row = j < M.tile_start[t + 1];
  double acc[NR];
  const double* yil = M.il + (long long)blockIdx.y * M.n1 * NR;
  if constexpr (MIXED) {
    float a32[NR];
    if constexpr (IL) sell_rows_multi_il<float, float, NR>(AT.col, AT.val32, yil, e, w, a32);
    else sell_rows_multi<float, float, NR>(AT.col, AT.val32, y, M.n1, j0, act, e, w, a32);
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = (double)a32[q];
  } else {
    if constexpr (IL) sell_rows_multi_il<double, double, NR>(AT.col, AT.val, yil, e, w, acc);
    else sell_rows_multi<double, double, NR>(AT.col, AT.val, y, M.n1, j0, act, e, w, acc);
  }
  double dot[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    dot[q] = 0.0;
    const long long o = (long long)(j0 + q) * M.n1 + j;
    if (act[q] && row) {
      psi[o] = acc[q];
      dot[q] = p[o] * acc[q];
    }
  }
  block_sum_multi<NR>(dot, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (act[q]) S.part_a[(j0 + q) * M.ntiles1 + t] = dot[q];
}

template <bool IL, int NR>
__global__ void __launch_bounds__(SELL_THREADS)
k_residual_sell_multi(SellMat A, MultiRhs M, const double* __restrict__ x,
                      const double* __restrict__ f, double* __restrict__ s, OuterState S,
                      const int* __restrict__ mask) {
  __shared__ double sh[NR * SELL_SLICES];
  const int t = blockIdx.x, j0 = blockIdx.y * NR;
  bool act[NR];
  if (!chunk_active<NR>(j0, M.nrhs, mask, false, act)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int sl = t * SELL_SLICES + wave;
  const int i = M.tile_start[t] + wave * 64 + lane;
  const bool row = i < M.tile_start[t + 1];
  double acc[NR];
  if constexpr (IL)
    sell_rows_multi_il<double, double, NR>(A.col, A.val, M.il + (long long)blockIdx.y * M.n1 * NR,
                                           A.ptr[sl] + lane, A.wid[sl], acc);
  else
    sell_rows_multi<double, double, NR>(A.col, A.val, x, M.n1, j0, act, A.ptr[sl] + lane,
                                        A.wid[sl], acc);
  double ss[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    ss[q] = 0.0;
    const long long o = (long long)(j0 + q) * M.n1 + i;
    if (act[q] && row) {
      const double v = f[o] - acc[q];
      s[o] = v;
      ss[q] = v * v;
    }
  }
  block_sum_multi<NR>(ss, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NR; ++q)
      if (act[q]) S.part_c[(j0 + q) * M.ntiles1 + t] = ss[q];
}

// ---- block CG on H: tall-skinny products of a few vectors of length n.
// Gram: G[a][b] = V1_a . V2_b for the columns of two lists.  A fixed number
// of workgroups walk the 128-row tiles (tile t by workgroup t mod groups);
// each stages the tile's columns in LDS, and wave w accumulates the 16x16
// block (w / 2, w % 2) of G over the tile's rows on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: A[i][k] = V1_i at row k from lane i + 16k, B[k][j]
// = V2_j at row k from lane j + 16k, D[i][j] in register r of lane j + 16g
// with i = 4r + g), K = 4 rows per step.  Each workgroup writes one partial
// per entry; k_block_gram_reduce adds the partials in workgroup order.  The
// order of every sum is fixed by n and the list sizes, so the result is
// reproducible.
typedef double dbl4v __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(BG_THREADS)
k_block_gram(ColList L1, ColList L2, int n, double* __restrict__ part) {
  extern __shared__ double gsh[];  // c1 + c2 columns of BG_LD (odd: no bank conflicts)
  const int c1 = L1.c, c2 = L2.c, np = c1 * c2;
  const int tid = threadIdx.x, r = tid % BG_ROWS, h = tid / BG_ROWS;
  static_assert(BG_THREADS == 2 * BG_ROWS, "two columns per staging pass");
  static_assert(BG_THREADS == 4 * 64 && BG_MAX == 32, "four waves, one 16x16 block each");
  // h is uniform per wave (waves 0-1: h = 0, waves 2-3: h = 1)
  const int w = tid >> 6, l = tid & 63;
  const int bi = w >> 1, bj = w & 1;
  const int i = bi * 16 + (l & 15), j = bj * 16 + (l & 15), kq = l >> 4;
  const bool live = bi * 16 < c1 && bj * 16 < c2;   // this wave's block holds entries
  dbl4v acc = {0.0, 0.0, 0.0, 0.0};
  const int ntl = (n + BG_ROWS - 1) / BG_ROWS;
  // Thread (r, h) stages row r of the columns 2q + h of both lists.  The
  // values of a tile are loaded into registers one tile ahead, so the loads
  // of the next tile are in flight while the matrix cores work on this one.
  double va[BG_MAX / 2], vb[BG_MAX / 2];
  auto load = [&](int tl) {
    const int row = tl * BG_ROWS + r;
    const bool in = tl < ntl && row < n;
#pragma unroll
    for (int q = 0; q < BG_MAX / 2; ++q) {
      const int col = 2 * q + h;
      const double* v1 = h ? L1.v[2 * q + 1] : L1.v[2 * q];
      const double* v2 = h ? L2.v[2 * q + 1] : L2.v[2 * q];
      va[q] = (in && col < c1) ? v1[row] : 0.0;
      vb[q] = (in && col < c2) ? v2[row] : 0.0;
    }
  };
  load(blockIdx.x);
  for (int tl = blockIdx.x; tl < ntl; tl += gridDim.x) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BG_MAX / 2; ++q) {
      const int col = 2 * q + h;
      if (col < c1) gsh[col * BG_LD + r] = va[q];
      if (col < c2) gsh[(c1 + col) * BG_LD + r] = vb[q];
    }
    __syncthreads();
    load(tl + gridDim.x);
    if (live) {
      const double* xa = gsh + (i < c1 ? i : 0) * BG_LD;
      const double* xb = gsh + (c1 + (j < c2 ? j : 0)) * BG_LD;
#pragma unroll 8
      for (int k0 = 0; k0 < BG_ROWS; k0 += 4) {
        const double a = i < c1 ? xa[k0 + kq] : 0.0;
        const double b = j < c2 ? xb[k0 + kq] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
    }
  }
  if (live)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ii = bi * 16 + 4 * q + kq;
      if (ii < c1 && j < c2) part[(size_t)blockIdx.x * np + ii * c2 + j] = acc[q];
    }
}

__global__ void __launch_bounds__(256)
k_block_gram_reduce(const double* __restrict__ part, int groups, int np, double* __restrict__ out) {
  __shared__ double sh[4];
  const int pr = blockIdx.x;
  double sum = 0.0;
  for (int g = threadIdx.x; g < groups; g += blockDim.x) sum += part[(size_t)g * np + pr];
  sum = block_sum(sum, sh);
  if (threadIdx.x == 0) out[pr] = sum;
}

// out_j = base_j + sum_k in_k * coef[k][j] (coef row-major, ci x co; base may
// be the output itself, or absent), one row per thread, k in order.
__global__ void __launch_bounds__(256)
k_block_combine(ColList in, ColList outl, ColList base, const double* __restrict__ coef, int n) {
  __shared__ double cs[BG_MAX * BG_MAX / 2];
  const int ci = in.c, co = outl.c;
  for (int e = threadIdx.x; e < ci * co; e += blockDim.x) cs[e] = coef[e];
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double v[BG_MAX];
#pragma unroll
  for (int k = 0; k < BG_MAX; ++k) v[k] = k < ci ? in.v[k][row] : 0.0;
#pragma unroll
  for (int j = 0; j < BG_MAX / 2; ++j) {
    if (j < co) {
      double sum = base.c > j ? base.v[j][row] : 0.0;
#pragma unroll
      for (int k = 0; k < BG_MAX; ++k)
        if (k < ci) sum += v[k] * cs[k * co + j];
      outl.v[j][row] = sum;
    }
  }
}

// psi[j] = sum over column j of A of a_ij * y[i] (stored A^T), plus the
// tile's partial of p . psi.
template <int L, bool MIXED>
__global__ void __launch_bounds__(VEC_THREADS)
k_spmvT_dot(const int* __restrict__ tptr, const int* __restrict__ trow,
            const double* __restrict__ tval, const float* __restrict__ tval32,
            const double* __restrict__ y, double* __restrict__ psi,
            const double* __restrict__ p, OuterState S) {
  __shared__ double sh[VEC_THREADS / 64];
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (S.done[sys]) return;
  const int c0 = S.tile_start[t], c1 = S.tile_start[t + 1];
  const int g = threadIdx.x / L, l = threadIdx.x % L;
  constexpr int RPP = VEC_THREADS / L;
  double dot = 0.0;
  for (int j = c0 + g; j < c1; j += RPP) {
    const int e0 = tptr[j], e1 = tptr[j + 1];
    double acc;
    if constexpr (MIXED) {
      const float a = lane_row_sum<L, float, float>(trow, tval32, y, e0, e1, l);
      acc = (double)group_sumf<L>(a);
    } else {
      const double a = lane_row_sum<L, double, double>(trow, tval, y, e0, e1, l);
      acc = group_sum<L>(a);
    }
    if (l == 0) {
      psi[j] = acc;
      dot += p[j] * acc;
    }
  }
  dot = block_sum(dot, sh);
  if (threadIdx.x == 0) S.part_a[t] = dot;
}

// s[i] = f[i] - (A x)[i] in FP64 for the systems with mask[sys] != 0 (all
// systems if mask is null); tile partial of s.s into part_c.
template <int L>
__global__ void __launch_bounds__(VEC_THREADS)
k_residual(const int* __restrict__ rowptr, const int* __restrict__ col,
           const double* __restrict__ val, const double* __restrict__ x,
           const double* __restrict__ f, double* __restrict__ s, OuterState S,
           const int* __restrict__ mask) {
  __shared__ double sh[VEC_THREADS / 64];
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (mask && !mask[sys]) return;
  const int r0 = S.tile_start[t], r1 = S.tile_start[t + 1];
  const int g = threadIdx.x / L, l = threadIdx.x % L;
  constexpr int RPP = VEC_THREADS / L;
  double ss = 0.0;
  for (int i = r0 + g; i < r1; i += RPP) {
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    double acc = lane_row_sum<L, double, double>(col, val, x, e0, e1, l);
    acc = group_sum<L>(acc);
    if (l == 0) {
      const double v = f[i] - acc;
      s[i] = v;
      ss += v * v;
    }
  }
  ss = block_sum(ss, sh);
  if (threadIdx.x == 0) S.part_c[t] = ss;
}

// alpha = rr / (p.psi); x += alpha p; r -= alpha psi; s -= alpha u (the true
// residual f - A x moves by -alpha A p, and A p = u is already at hand);
// tile partials of r.r (part_b) and s.s (part_c).
__global__ void __launch_bounds__(VEC_THREADS)
k_update_xrs(double* __restrict__ x, double* __restrict__ r, double* __restrict__ s,
             const double* __restrict__ p, const double* __restrict__ psi,
             const double* __restrict__ u, OuterState S) {
  __shared__ double sh[VEC_THREADS / 64];
  __shared__ double alpha_sh;
  __shared__ int bad_sh;
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (S.done[sys]) return;
  const int it = S.iters[sys] + 1;  // this iteration of the system (k_book advances the count)
  // The tile's vector entries do not depend on alpha: they are loaded first,
  // so that their latency overlaps the reduction of p.psi below.
  constexpr int PER = TILE / VEC_THREADS;
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  double xv[PER], pv[PER], rv[PER], qv[PER], sv[PER], uv[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = i0 + threadIdx.x + k * VEC_THREADS;
    const bool in = i < i1;
    xv[k] = in ? x[i] : 0.0;
    pv[k] = in ? p[i] : 0.0;
    rv[k] = in ? r[i] : 0.0;
    qv[k] = in ? psi[i] : 0.0;
    sv[k] = in ? s[i] : 0.0;
    uv[k] = in ? u[i] : 0.0;
  }
  if (threadIdx.x < 64) {
    const double ppsi = sys_sum_wave(S.part_a, S.sys_tile[sys], S.sys_tile[sys + 1]);
    if (threadIdx.x == 0) {
      const double rr = S.rr[2 * sys + ((it - 1) & 1)];
      const bool bad = !(ppsi > 0.0) || !isfinite(ppsi) || !isfinite(rr);
      bad_sh = bad;
      alpha_sh = bad ? 0.0 : rr / ppsi;
    }
  }
  __syncthreads();
  if (bad_sh) {
    if (t == S.sys_tile[sys] && threadIdx.x == 0) {
      S.status[sys] = BC_ERR_BREAKDOWN;
      S.iters[sys] = it - 1;
      S.done[sys] = 1;
    }
    return;
  }
  const double alpha = alpha_sh;
  double rr = 0.0, ss = 0.0, smax = 0.0, xsum = 0.0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = i0 + threadIdx.x + k * VEC_THREADS;
    if (i < i1) {
      const double xi = xv[k] + alpha * pv[k];
      x[i] = xi;
      xsum += fabs(xi);
      const double ri = rv[k] - alpha * qv[k];
      r[i] = ri;
      rr += ri * ri;
      const double si = sv[k] - alpha * uv[k];
      s[i] = si;
      ss += si * si;
      smax = fmax(smax, fabs(si));
    }
  }
  rr = block_sum(rr, sh);
  ss = block_sum(ss, sh);
  if (S.use_backward) {
    xsum = block_sum(xsum, sh);
    smax = block_max(smax, sh);
  }
  if (threadIdx.x == 0) {
    S.part_b[t] = rr;
    S.part_c[t] = ss;
    if (S.use_backward) {
      S.part_d[t] = smax;
      S.part_e[t] = xsum;
    }
  }
}

// Stop test on ||s||^2 for iteration `it`, then beta = rr_new / rr and
// p = r + beta p.  The first tile of a system records rr, the iteration count
// and the stop decision in `pending`; `done` itself is only changed by
// k_book after this kernel, so every tile of a system sees the same flags.
__global__ void __launch_bounds__(VEC_THREADS)
k_update_p(double* __restrict__ p, const double* __restrict__ r, OuterState S) {
  __shared__ double beta_sh;
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (S.done[sys]) return;
  const int it = S.iters[sys] + 1;
  // entries first (they do not depend on beta), as in k_update_xrs
  constexpr int PER = TILE / VEC_THREADS;
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  double rv[PER], pv[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = i0 + threadIdx.x + k * VEC_THREADS;
    rv[k] = i < i1 ? r[i] : 0.0;
    pv[k] = i < i1 ? p[i] : 0.0;
  }
  if (threadIdx.x < 64) {
    const int a = S.sys_tile[sys], b = S.sys_tile[sys + 1];
    const double rrn = sys_sum_wave(S.part_b, a, b);
    const double ss = sys_sum_wave(S.part_c, a, b);
    if (threadIdx.x == 0) {
      const double rro = S.rr[2 * sys + ((it - 1) & 1)];
      beta_sh = rrn / rro;
      if (t == a) {
        S.rr[2 * sys + (it & 1)] = rrn;
        if (S.hist) S.hist[sys] = ss;
        bool conv;
        if (S.use_backward) {
          const double smax = sys_max_serial(S.part_d, a, b);
          const double xsum = sys_sum_serial(S.part_e, a, b);
          const double den = S.normA[sys] * xsum + S.finf[sys];
          conv = den > 0.0 ? (smax / den < S.tol_bw) : true;
        } else {
          conv = S.rec_stop && ss <= S.thr[sys];
        }
        S.pending[sys] = conv ? 1 : (it >= S.maxit ? 2 : 0);
      }
    }
  }
  __syncthreads();
  const double beta = beta_sh;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = i0 + threadIdx.x + k * VEC_THREADS;
    if (i < i1) p[i] = rv[k] + beta * pv[k];
  }
}

// Stop test on the FP64 true residual (partials of s.s in part_c from
// k_residual), used where the recursively updated s is not accurate enough.
__global__ void k_true_check(OuterState S) {
  const int sys = blockIdx.x;
  const double ss = sys_sum_wave(S.part_c, S.sys_tile[sys], S.sys_tile[sys + 1]);
  if (threadIdx.x == 0 && !S.done[sys] && ss <= S.thr[sys]) {
    S.status[sys] = BC_OK;
    S.done[sys] = 1;
  }
}

// Per-system bookkeeping after k_update_p: apply the stop decision.
__global__ void k_book(OuterState S) {
  const int sys = blockIdx.x * blockDim.x + threadIdx.x;
  if (sys >= S.nsys || S.done[sys]) return;
  S.iters[sys] += 1;  // the iteration every kernel of this system just ran
  const int pend = S.pending[sys];
  if (pend) {
    S.status[sys] = pend == 1 ? BC_OK : BC_NOT_CONVERGED;
    S.done[sys] = 1;
  }
}

// p = r and the tile partial of r.r (CG start).
__global__ void __launch_bounds__(VEC_THREADS)
k_init_cg(double* __restrict__ p, const double* __restrict__ r, OuterState S) {
  __shared__ double sh[VEC_THREADS / 64];
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (S.done[sys]) return;
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  double rr = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
    const double v = r[i];
    p[i] = v;
    rr += v * v;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) S.part_b[t] = rr;
}

// Per system: r.r from the partials in part_b into the slot the next
// iteration reads (iteration iters+1 reads slot iters & 1).
__global__ void k_rr_from_partials(OuterState S) {
  const int sys = blockIdx.x;
  const double rr = sys_sum_wave(S.part_b, S.sys_tile[sys], S.sys_tile[sys + 1]);
  if (threadIdx.x == 0 && !S.done[sys]) S.rr[2 * sys + (S.iters[sys] & 1)] = rr;
}

// Residual replacement with factor-based projections, per system: the new
// r.r (partials in part_b) replaces the slot the next iteration reads; when it
// exceeds 4x the recursive value it replaces (the recursion had drifted away
// from the true residual) the system restarts CG (flag set for
// k_restart_where), otherwise the search direction is kept.
__global__ void k_replace_decide(OuterState S, int* __restrict__ restart) {
  const int sys = blockIdx.x;
  const int slot = S.iters[sys] & 1;
  const double rr = sys_sum_wave(S.part_b, S.sys_tile[sys], S.sys_tile[sys + 1]);
  if (threadIdx.x == 0 && !S.done[sys]) {
    const double old = S.rr[2 * sys + slot];
    restart[sys] = !(rr <= 4.0 * old);
    S.rr[2 * sys + slot] = rr;
  }
}

__global__ void __launch_bounds__(VEC_THREADS)
k_restart_where(double* __restrict__ p, const double* __restrict__ r,
                const int* __restrict__ restart, OuterState S) {
  const int t = tile_of_block();
  const int sys = S.tile_sys[t];
  if (S.done[sys] || !restart[sys]) return;
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  for (int i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) p[i] = r[i];
}

// Tile partials at the start of a solve: f.f (part_f), max|f| (part_g),
// max|s| (part_d) and sum|x| (part_e).
__global__ void __launch_bounds__(VEC_THREADS)
k_init_norms(const double* __restrict__ f, const double* __restrict__ s,
             const double* __restrict__ x, double* __restrict__ part_f, OuterState S) {
  __shared__ double sh[VEC_THREADS / 64];
  const int t = tile_of_block();
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  double ff = 0.0, fm = 0.0, sm = 0.0, xs = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) {
    ff += f[i] * f[i];
    fm = fmax(fm, fabs(f[i]));
    sm = fmax(sm, fabs(s[i]));
    xs += fabs(x[i]);
  }
  ff = block_sum(ff, sh);
  fm = block_max(fm, sh);
  sm = block_max(sm, sh);
  xs = block_sum(xs, sh);
  if (threadIdx.x == 0) {
    part_f[t] = ff;
    S.part_g[t] = fm;
    S.part_d[t] = sm;
    S.part_e[t] = xs;
  }
}

// Per system, from the tile partials (fixed order): ||s||^2, ||f||^2, max|s|,
// max|f| and sum|x|, into out[5 sys + 0..4] (the figures the solve reports:
// relative residual and the normwise backward error of eq. (stopping)).
__global__ void k_final_stats(const double* __restrict__ part_f, OuterState S,
                              double* __restrict__ out) {
  const int sys = blockIdx.x;
  const int a = S.sys_tile[sys], b = S.sys_tile[sys + 1];
  const double ss = sys_sum_wave(S.part_c, a, b);
  const double ff = sys_sum_wave(part_f, a, b);
  const double xs = sys_sum_wave(S.part_e, a, b);
  if (threadIdx.x == 0) {
    out[5 * sys + 0] = ss;
    out[5 * sys + 1] = ff;
    out[5 * sys + 2] = sys_max_serial(S.part_d, a, b);
    out[5 * sys + 3] = sys_max_serial(S.part_g, a, b);
    out[5 * sys + 4] = xs;
  }
}

// Algorithm 1, per system: the stop test on ||s||^2 of the current iterate
// (tile partials part_c, fixed order), then the count of the update this
// iteration makes; a system at maxit updates, or whose residual is not
// finite, is finished.
__global__ void k_cimmino_check(OuterState S) {
  const int sys = blockIdx.x;
  if (S.done[sys]) return;
  const int a = S.sys_tile[sys], b = S.sys_tile[sys + 1];
  const double ss = sys_sum_wave(S.part_c, a, b);
  if (threadIdx.x == 0) {
    if (ss <= S.thr[sys]) {
      S.done[sys] = 1;
      S.status[sys] = BC_OK;
    } else if (!isfinite(ss)) {
      S.done[sys] = 1;
      S.status[sys] = BC_ERR_BREAKDOWN;
    } else if (S.iters[sys] >= S.maxit) {
      S.done[sys] = 1;
      S.status[sys] = BC_NOT_CONVERGED;
    } else {
      S.iters[sys] += 1;
    }
  }
}

// Algorithm 1: x += omega psi (psi = sum_i A_i^+ s_i) on the systems not done.
__global__ void __launch_bounds__(VEC_THREADS)
k_cimmino_update(double* __restrict__ x, const double* __restrict__ psi, double omega,
                 OuterState S) {
  const int t = tile_of_block();
  if (S.done[S.tile_sys[t]]) return;
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  for (int i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) x[i] += omega * psi[i];
}

// Tile partials of v.v (into part).
__global__ void __launch_bounds__(VEC_THREADS)
k_sqnorm_tiles(const double* __restrict__ v, double* __restrict__ part, OuterState S) {
  __shared__ double sh[VEC_THREADS / 64];
  const int t = tile_of_block();
  const int i0 = S.tile_start[t], i1 = S.tile_start[t + 1];
  double a = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += VEC_THREADS) a += v[i] * v[i];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) part[t] = a;
}

// Per system: thr = tol^2 ||f||^2 from the partials of f.f and ||f||_inf; a
// system whose initial residual already meets the stop rule, or with f = 0,
// is done at iteration 0.
__global__ void k_set_thresholds(const double* __restrict__ part_f, double tol2, OuterState S) {
  const int sys = blockIdx.x;
  const int a = S.sys_tile[sys], b = S.sys_tile[sys + 1];
  const double ff = sys_sum_wave(part_f, a, b);
  const double ss = sys_sum_wave(S.part_c, a, b);
  if (threadIdx.x == 0) {
    const double thr = tol2 * ff;
    const double fm = sys_max_serial(S.part_g, a, b);
    S.finf[sys] = fm;
    S.thr[sys] = thr;
    S.iters[sys] = 0;
    S.status[sys] = BC_NOT_CONVERGED;
    S.done[sys] = 0;
    S.pending[sys] = 0;
    bool conv = ss <= thr;
    if (S.use_backward) {
      const double den = S.normA[sys] * sys_sum_serial(S.part_e, a, b) + fm;
      conv = den > 0.0 ? (sys_max_serial(S.part_d, a, b) / den < S.tol_bw) : true;
    }
    if (ff == 0.0 || conv) {
      S.done[sys] = 1;
      S.status[sys] = BC_OK;
    }
  }
}

__global__ void k_gather(const double* __restrict__ src, const int* __restrict__ idx,
                         double* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_copy(const double* __restrict__ src, double* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_zero(double* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = 0.0;
}

}  // namespace

#define LANE_SWITCH(lanes, MACRO) \
  switch (lanes) {                \
    case 1: MACRO(1); break;      \
    case 2: MACRO(2); break;      \
    case 4: MACRO(4); break;      \
    case 8: MACRO(8); break;      \
    case 16: MACRO(16); break;    \
    case 32: MACRO(32); break;    \
    default: MACRO(64); break;    \
  }

hipError_t launch_spmv(int lanes, hipStream_t st, const int* rowptr, const int* col,
                       const double* val, const float* val32, bool mixed, const double* x,
                       double* y, const OuterState& S, bool skip_done) {
  if (S.ntiles == 0) return hipSuccess;
#define L_SPMV(L)                                                                          \
  if (mixed)                                                                               \
    hipLaunchKernelGGL((k_spmv<L, true>), dim3(S.ntiles), dim3(VEC_THREADS), 0, st, rowptr, \
                       col, val, val32, x, y, S, (int)skip_done);                          \
  else                                                                                     \
    hipLaunchKernelGGL((k_spmv<L, false>), dim3(S.ntiles), dim3(VEC_THREADS), 0, st, rowptr,\
                       col, val, val32, x, y, S, (int)skip_done);
  LANE_SWITCH(lanes, L_SPMV)
#undef L_SPMV
  return hipGetLastError();
}

hipError_t launch_spmvT_dot(int lanes, hipStream_t st, const int* tptr, const int* trow,
                            const double* tval, const float* tval32, bool mixed, const double* y,
                            double* psi, const double* p, const OuterState& S) {
  if (S.ntiles == 0) return hipSuccess;
#define L_SPMVT(L)                                                                           \
  if (mixed)                                                                                 \
    hipLaunchKernelGGL((k_spmvT_dot<L, true>), dim3(S.ntiles), dim3(VEC_THREADS), 0, st, tptr,\
                       trow, tval, tval32, y, psi, p, S);                                    \
  else                                                                                       \
    hipLaunchKernelGGL((k_spmvT_dot<L, false>), dim3(S.ntiles), dim3(VEC_THREADS), 0, st,     \
                       tptr, trow, tval, tval32, y, psi, p, S);
  LANE_SWITCH(lanes, L_SPMVT)
#undef L_SPMVT
  return hipGetLastError();
}

hipError_t launch_residual(int lanes, hipStream_t st, const int* rowptr, const int* col,
                           const double* val, const double* x, const double* fperm, double* s,
                           const OuterState& S, const int* mask) {
  if (S.ntiles == 0) return hipSuccess;
#define L_RES(L)                                                                             \
  hipLaunchKernelGGL((k_residual<L>), dim3(S.ntiles), dim3(VEC_THREADS), 0, st, rowptr, col, \
                     val, x, fperm, s, S, mask);
  LANE_SWITCH(lanes, L_RES)
#undef L_RES
  return hipGetLastError();
}

hipError_t launch_update_xrs(hipStream_t st, double* x, double* r, double* s, const double* p,
                             const double* psi, const double* u, const OuterState& S) {
  if (S.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_xrs, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, x, r, s, p, psi, u,
                     S);
  return hipGetLastError();
}

hipError_t launch_update_p(hipStream_t st, double* p, const double* r, const OuterState& S) {
  if (S.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_p, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, p, r, S);
  hipLaunchKernelGGL(k_book, dim3((S.nsys + 63) / 64), dim3(64), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_init_cg(hipStream_t st, double* p, const double* r, const OuterState& S) {
  if (S.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_cg, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, p, r, S);
  hipLaunchKernelGGL(k_rr_from_partials, dim3(S.nsys), dim3(64), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_true_check(hipStream_t st, const OuterState& S) {
  hipLaunchKernelGGL(k_true_check, dim3(S.nsys), dim3(64), 0, st, S);
  return hipGetLastError();
}

// Device wall-clock stamp (constant-rate counter) for timing inside graphs.
__global__ void k_stamp(unsigned long long* __restrict__ t, int i) {
  if (threadIdx.x == 0) t[i] = wall_clock64();
}

hipError_t launch_stamp(hipStream_t st, unsigned long long* t, int i) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, st, t, i);
  return hipGetLastError();
}

hipError_t launch_replace_decide(hipStream_t st, const OuterState& S, int* restart, double* p,
                                 const double* r) {
  hipLaunchKernelGGL(k_replace_decide, dim3(S.nsys), dim3(64), 0, st, S, restart);
  hipLaunchKernelGGL(k_restart_where, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, p, r, restart, S);
  return hipGetLastError();
}

hipError_t launch_rr_from_partials(hipStream_t st, const OuterState& S) {
  hipLaunchKernelGGL(k_rr_from_partials, dim3(S.nsys), dim3(64), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_init_norms(hipStream_t st, const double* f, const double* s, const double* x,
                             double* part_f, const OuterState& S) {
  if (S.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_norms, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, f, s, x, part_f, S);
  return hipGetLastError();
}

hipError_t launch_sqnorm_tiles(hipStream_t st, const double* v, double* part, const OuterState& S) {
  if (S.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sqnorm_tiles, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, v, part, S);
  return hipGetLastError();
}

hipError_t launch_set_thresholds(hipStream_t st, const double* part_f, double tol,
                                 const OuterState& S) {
  hipLaunchKernelGGL(k_set_thresholds, dim3(S.nsys), dim3(64), 0, st, part_f, tol * tol, S);
  return hipGetLastError();
}

hipError_t launch_spmv_sell(hipStream_t st, const SellMat& A, bool mixed, const double* x,
                            double* y, const OuterState& S, bool skip_done) {
  if (mixed)
    hipLaunchKernelGGL(k_spmv_sell<true>, dim3(S.ntiles), dim3(SELL_THREADS), 0, st, A, x, y, S,
                       (int)skip_done);
  else
    hipLaunchKernelGGL(k_spmv_sell<false>, dim3(S.ntiles), dim3(SELL_THREADS), 0, st, A, x, y, S,
                       (int)skip_done);
  return hipGetLastError();
}

hipError_t launch_spmvT_dot_sell(hipStream_t st, const SellMat& AT, bool mixed, const double* y,
                                 double* psi, const double* p, const OuterState& S) {
  if (mixed)
    hipLaunchKernelGGL(k_spmvT_dot_sell<true>, dim3(S.ntiles), dim3(SELL_THREADS), 0, st, AT, y,
                       psi, p, S);
  else
    hipLaunchKernelGGL(k_spmvT_dot_sell<false>, dim3(S.ntiles), dim3(SELL_THREADS), 0, st, AT, y,
                       psi, p, S);
  return hipGetLastError();
}

hipError_t launch_residual_sell(hipStream_t st, const SellMat& A, const double* x, const double* f,
                                double* s, const OuterState& S, const int* mask) {
  hipLaunchKernelGGL(k_residual_sell, dim3(S.ntiles), dim3(SELL_THREADS), 0, st, A, x, f, s, S,
                     mask);
  return hipGetLastError();
}

hipError_t launch_cimmino_check(hipStream_t st, const OuterState& S) {
  hipLaunchKernelGGL(k_cimmino_check, dim3(S.nsys), dim3(64), 0, st, S);
  return hipGetLastError();
}

hipError_t launch_cimmino_update(hipStream_t st, double* x, const double* psi, double omega,
                                 const OuterState& S) {
  hipLaunchKernelGGL(k_cimmino_update, dim3(S.ntiles), dim3(VEC_THREADS), 0, st, x, psi, omega, S);
  return hipGetLastError();
}

hipError_t launch_final_stats(hipStream_t st, const double* part_f, const OuterState& S,
                              double* out) {
  hipLaunchKernelGGL(k_final_stats, dim3(S.nsys), dim3(64), 0, st, part_f, S, out);
  return hipGetLastError();
}

hipError_t launch_gather(hipStream_t st, const double* src, const int* idx, double* dst, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, st, src, idx, dst, n);
  return hipGetLastError();
}

hipError_t launch_copy(hipStream_t st, const double* src, double* dst, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_zero(hipStream_t st, double* dst, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, st, dst, n);
  return hipGetLastError();
}

// Chunk width of the multi-vector sparse products: 8 vectors (8 entries'
// indices and values plus 8 accumulators stay within 76 VGPRs at 1024
// threads, without spills).

// The gathered input of a multi-vector product, interleaved per chunk.
hipError_t interleave_input(hipStream_t st, const MultiRhs& M, const double* src) {
  const dim3 grid((M.n1 + 255) / 256, (M.nrhs + SELL_MULTI_NR - 1) / SELL_MULTI_NR);
  hipLaunchKernelGGL(k_interleave<SELL_MULTI_NR>, grid, dim3(256), 0, st, src, M.il, M.n1, M.nrhs);
  return hipGetLastError();
}

template <bool MIXED, bool IL>
void spmv_multi_t(hipStream_t st, const SellMat& A, const MultiRhs& M, const double* x, double* y,
                  const OuterState& S, bool skip_done) {
  const dim3 grid(M.ntiles1, (M.nrhs + SELL_MULTI_NR - 1) / SELL_MULTI_NR);
  hipLaunchKernelGGL((k_spmv_sell_multi<MIXED, IL, SELL_MULTI_NR>), grid, dim3(SELL_THREADS), 0,
                     st, A, M, x, y, S, (int)skip_done);
}

hipError_t launch_spmv_sell_multi(hipStream_t st, const SellMat& A, const MultiRhs& M, bool mixed,
                                  const double* x, double* y, const OuterState& S, bool skip_done) {
  if (A.il) {
    const hipError_t ei = interleave_input(st, M, x);
    if (ei != hipSuccess) return ei;
    if (mixed) spmv_multi_t<true, true>(st, A, M, x, y, S, skip_done);
    else spmv_multi_t<false, true>(st, A, M, x, y, S, skip_done);
  } else {
    if (mixed) spmv_multi_t<true, false>(st, A, M, x, y, S, skip_done);
    else spmv_multi_t<false, false>(st, A, M, x, y, S, skip_done);
  }
  return hipGetLastError();
}

template <bool MIXED, bool IL>
void spmvT_multi_t(hipStream_t st, const SellMat& AT, const MultiRhs& M, const double* y,
                   double* psi, const double* p, const OuterState& S) {
  const dim3 grid(M.ntiles1, (M.nrhs + SELL_MULTI_NR - 1) / SELL_MULTI_NR);
  hipLaunchKernelGGL((k_spmvT_dot_sell_multi<MIXED, IL, SELL_MULTI_NR>), grid, dim3(SELL_THREADS),
                     0, st, AT, M, y, psi, p, S);
}

hipError_t launch_spmvT_dot_sell_multi(hipStream_t st, const SellMat& AT, const MultiRhs& M,
                                       bool mixed, const double* y, double* psi, const double* p,
                                       const OuterState& S) {
  if (AT.il) {
    const hipError_t ei = interleave_input(st, M, y);
    if (ei != hipSuccess) return ei;
    if (mixed) spmvT_multi_t<true, true>(st, AT, M, y, psi, p, S);
    else spmvT_multi_t<false, true>(st, AT, M, y, psi, p, S);
  } else {
    if (mixed) spmvT_multi_t<true, false>(st, AT, M, y, psi, p, S);
    else spmvT_multi_t<false, false>(st, AT, M, y, psi, p, S);
  }
  return hipGetLastError();
}

hipError_t launch_residual_sell_multi(hipStream_t st, const SellMat& A, const MultiRhs& M,
                                      const double* x, const double* f, double* s,
                                      const OuterState& S, const int* mask) {
  const dim3 grid(M.ntiles1, (M.nrhs + SELL_MULTI_NR - 1) / SELL_MULTI_NR);
  if (A.il) {
    const hipError_t ei = interleave_input(st, M, x);
    if (ei != hipSuccess) return ei;
    hipLaunchKernelGGL((k_residual_sell_multi<true, SELL_MULTI_NR>), grid, dim3(SELL_THREADS), 0,
                       st, A, M, x, f, s, S, mask);
  } else {
    hipLaunchKernelGGL((k_residual_sell_multi<false, SELL_MULTI_NR>), grid, dim3(SELL_THREADS), 0,
                       st, A, M, x, f, s, S, mask);
  }
  return hipGetLastError();
}

hipError_t prepare_block_gram() {
  return hipFuncSetAttribute((const void*)k_block_gram, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(BG_LD * 2 * BG_MAX * sizeof(double)));
}

hipError_t launch_block_gram(hipStream_t st, const ColList& L1, const ColList& L2, int n,
                             double* part, double* out) {
  const int np = L1.c * L2.c;
  if (np == 0) return hipSuccess;
  if (L1.c > BG_MAX || L2.c > BG_MAX || np > BG_PAIRS) return hipErrorInvalidValue;
  const int ntl = (n + BG_ROWS - 1) / BG_ROWS;
  const int groups = ntl < BG_GROUPS ? ntl : BG_GROUPS;
  const size_t lds = (size_t)BG_LD * (L1.c + L2.c) * sizeof(double);
  hipLaunchKernelGGL(k_block_gram, dim3(groups), dim3(BG_THREADS), lds, st, L1, L2, n, part);
  hipLaunchKernelGGL(k_block_gram_reduce, dim3(np), dim3(256), 0, st, part, groups, np, out);
  return hipGetLastError();
}

hipError_t launch_block_combine(hipStream_t st, const ColList& in, const ColList& out,
                                const ColList& base, const double* coef, int n) {
  if (out.c == 0) return hipSuccess;
  if (in.c > BG_MAX || out.c > BG_MAX / 2 || base.c > BG_MAX / 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_block_combine, dim3((n + 255) / 256), dim3(256), 0, st, in, out, base, coef,
                     n);
  return hipGetLastError();
}
