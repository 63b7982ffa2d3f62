// Dense projections for small blocks: G_i = A_i A_i^T = L_i L_i^T in FP64,
// then y_i = G_i^{-1} u_i by two triangular sweeps (the normal-equation form
// of the block projection, Section 1; the factor is computed once, like the
// paper's one-time factorisation of the augmented systems in Section 3.5).
//
// Storage of a block with m rows, nt = ceil(m / 64) tiles per side, padded
// with an identity block so the factor of the padding is the identity:
//   L    packed lower tiles (i >= j), tile (i,j) at (i(i+1)/2 + j) * 4096,
//        each tile column-major (element (r,c) at c*64 + r);
//   LT   packed upper tiles (j >= i) of L^T: tile (i,j) = (L_ji)^T, at
//        (i*nt - i(i-1)/2 + j - i) * 4096, column-major (the backward sweep
//        then reads contiguous columns, like the forward sweep);
//   Dinv the inverted diagonal tiles L_kk^{-1} followed by their transposes,
//        2*nt tiles per block.
// The sweeps are GEMV-shaped (one right-hand side) and bounded by the bytes of
// L; a factor copy in FP32 halves them in mixed precision.
#include "common.h"

#include <cmath>

namespace {

constexpr int GEMM_THREADS = 256;
constexpr int APPLY_THREADS = 256;
constexpr long long TSZ = (long long)DT * DT;

__device__ __forceinline__ long long ltile(int i, int j) { return (long long)(i * (i + 1) / 2 + j) * TSZ; }
__device__ __forceinline__ long long uttile(int nt, int i, int j) {
  return (long long)(i * nt - i * (i - 1) / 2 + (j - i)) * TSZ;
}

// ---------------------------------------------------------------- Gram tiles
// One wavefront per (block, i, j) tile, lane r builds row i*64+r of the tile:
// G[row][col] = sum over the row's entries (ascending column k) of
// a_row,k * a_col,k, with the rows of column k found in the stored A^T.
__global__ void __launch_bounds__(64)
k_gram(DenseBlocks D, const int4* __restrict__ tiles, const int* __restrict__ rowptr,
       const int* __restrict__ col, const double* __restrict__ val,
       const int* __restrict__ tptr, const int* __restrict__ trow,
       const double* __restrict__ tval) {
  __shared__ double acc[DT * DT];
  const int4 tl = tiles[blockIdx.x];
  const int b = tl.x, ti = tl.y, tj = tl.z;
  const int r = threadIdx.x;
  for (int c = 0; c < DT; ++c) acc[c * DT + r] = 0.0;
  const int m = D.m[b], row0 = D.row0[b];
  const int lr = ti * DT + r;  // local row
  const int clo = row0 + tj * DT, chi = row0 + min(m, tj * DT + DT);
  if (lr < m) {
    const int grow = row0 + lr;
    const double dr = D.dsc[grow];
    for (int e = rowptr[grow]; e < rowptr[grow + 1]; ++e) {
      const int k = col[e];
      const double a = val[e] * dr;
      // rows of column k are sorted: find the first >= clo
      int lo = tptr[k], hi = tptr[k + 1];
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (trow[mid] < clo) lo = mid + 1; else hi = mid;
      }
      for (int f = lo; f < tptr[k + 1] && trow[f] < chi; ++f)
        acc[(trow[f] - clo) * DT + r] += a * (tval[f] * D.dsc[trow[f]]);
    }
  } else if (ti == tj) {
    acc[r * DT + r] = 1.0;  // identity padding
  }
  if (ti == tj && lr < m) D.gdiag[row0 + lr] = acc[r * DT + r];
  double* dst = D.L + D.loff[b] + ltile(ti, tj);
  for (int c = 0; c < DT; ++c) dst[c * DT + r] = acc[c * DT + r];
}

// C (64x64, LDS, column-major) = X Y^T (SUB: C -= X Y^T) with X, Y 64x64
// column-major LDS tiles, on the FP64 matrix cores: v_mfma_f64_16x16x4f64
// takes A[i][k] from lane i + 16k and B[k][j] from lane j + 16k, and leaves
// D[i][j] in register r of lane j + 16g with i = 4r + g.  Wave w of the four
// owns the 32x32 quadrant (rows 32 (w & 1), columns 32 (w >> 1)) as 2x2 such
// tiles and runs 16 k-steps of 4.  The caller separates reads of an aliased
// operand from the writes with a barrier (SUB = false writes C only after
// all of the wave's products are in registers).
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <bool SUB>
__device__ __forceinline__ void tile_mfma_nt(double* C, const double* X, const double* Y,
                                             bool sync_before_store) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w & 1), c0 = 32 * (w >> 1);
  const int li = l & 15, lk = l >> 4;
  dbl4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int p0 = 0; p0 < DT; p0 += 4) {
    const int p = p0 + lk;
    const double a0 = X[p * DT + r0 + li], a1 = X[p * DT + r0 + 16 + li];
    const double b0 = Y[p * DT + c0 + li], b1 = Y[p * DT + c0 + 16 + li];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  if (sync_before_store) __syncthreads();
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 16 * ti + 4 * r + lk, col = c0 + 16 * tj + li;
        if constexpr (SUB) C[col * DT + row] -= acc[ti][tj][r];
        else C[col * DT + row] = acc[ti][tj][r];
      }
}

__device__ __forceinline__ void load_tile(double* dst, const double* src) {
  for (int e = threadIdx.x; e < DT * DT; e += blockDim.x) dst[e] = src[e];
}
__device__ __forceinline__ void store_tile(double* dst, const double* src) {
  for (int e = threadIdx.x; e < DT * DT; e += blockDim.x) dst[e] = src[e];
}

// ------------------------------------------------------------- Cholesky
// Blocked right-looking Cholesky of every block, in place on the packed lower
// tiles, one panel of CHOL_PW tile columns (kb .. kb + kw - 1) per step:
//   k_chol_diag   one workgroup per block: the kw x kw tiles of the diagonal
//                 block, tile by tile (factor the diagonal tile, invert it,
//                 form the panel tiles below it inside the diagonal block,
//                 update the rest of the diagonal block);
//   k_chol_panel  one workgroup per (block, tile row i below the diagonal
//                 block): L_ik = (A_ik - sum_{kb <= c < k} L_ic L_kc^T) L_kk^{-T}
//                 for k = kb .. kb + kw - 1;
//   k_chol_update one workgroup per (block, i, j), kb + kw <= j <= i:
//                 A_ij -= sum_{kb <= k < kb + kw} L_ik L_jk^T.
// The panel and trailing products read their operand tiles straight from
// global memory into the FP64 matrix cores (v_mfma_f64_16x16x4f64, lane
// layout as in tile_mfma_nt: wave w owns the 32x32 quadrant at rows
// 32 (w & 1), columns 32 (w >> 1)), and accumulate a whole panel of kw tile
// columns in registers before the result tile is written once.

// unblocked Cholesky, inverse and transposed inverse of diagonal tile k
// (in T0, T1 = scratch); returns false (bad set) on a failed pivot
__device__ bool chol_diag_tile(const DenseBlocks& D, int b, int k, int nt, int m, int row0,
                               double* L, double* Dv, double* T0, double* T1, int& bad,
                               double rel_piv) {
  __syncthreads();
  load_tile(T0, L + ltile(k, k));
  __syncthreads();
  for (int c = 0; c < DT; ++c) {
    if (threadIdx.x == 0) {
      const double d = T0[c * DT + c];
      const int gr = k * DT + c;
      const double g0 = gr < m ? D.gdiag[row0 + gr] : 1.0;
      if (!(d > rel_piv * g0) || !isfinite(d)) {
        bad = k * DT + c + 1;
      } else {
        T0[c * DT + c] = sqrt(d);
      }
    }
    __syncthreads();
    if (bad) return false;
    const double piv = T0[c * DT + c];
    for (int rr = c + 1 + threadIdx.x; rr < DT; rr += blockDim.x) T0[c * DT + rr] /= piv;
    __syncthreads();
    // rank-1 update of the remaining lower part of the tile
    const int rem = DT - c - 1;
    for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
      const int c2 = c + 1 + e / rem, rr = c + 1 + e % rem;
      if (rr >= c2) T0[c2 * DT + rr] -= T0[c * DT + rr] * T0[c * DT + c2];
    }
    __syncthreads();
  }
  // zero the strict upper part, write L_kk
  for (int e = threadIdx.x; e < DT * DT; e += blockDim.x) {
    const int c = e / DT, rr = e % DT;
    if (rr < c) T0[e] = 0.0;
  }
  __syncthreads();
  store_tile(L + ltile(k, k), T0);
  // inverse of the lower-triangular tile: thread c solves L x = e_c
  if (threadIdx.x < DT) {
    const int c = threadIdx.x;
    for (int rr = 0; rr < DT; ++rr) T1[c * DT + rr] = 0.0;
    for (int rr = c; rr < DT; ++rr) {
      double s = (rr == c) ? 1.0 : 0.0;
      for (int j = c; j < rr; ++j) s -= T0[j * DT + rr] * T1[c * DT + j];
      T1[c * DT + rr] = s / T0[rr * DT + rr];
    }
  }
  __syncthreads();
  store_tile(Dv + (long long)k * TSZ, T1);
  // transposed inverse for the backward sweep
  for (int e = threadIdx.x; e < DT * DT; e += blockDim.x) {
    const int c = e / DT, rr = e % DT;
    Dv[(long long)(nt + k) * TSZ + e] = T1[rr * DT + c];
  }
  return true;
}

__global__ void __launch_bounds__(GEMM_THREADS)
k_chol_diag(DenseBlocks D, int kb) {
  extern __shared__ double lds[];
  double* T0 = lds;             // diagonal tile / C tile
  double* T1 = lds + TSZ;       // inverse of the diagonal tile
  double* T2 = lds + 2 * TSZ;   // panel tile X
  double* T3 = lds + 3 * TSZ;   // panel tile Y
  __shared__ int bad;
  const int b = blockIdx.x;
  const int nt = D.nt[b], m = D.m[b], row0 = D.row0[b];
  if (kb >= nt || D.info[b] != 0) return;
  const int ke = min(nt, kb + CHOL_PW);
  double* L = D.L + D.loff[b];
  double* Dv = D.Dinv + D.doff[b];
  // a pivot at or below m * eps * G_jj means A_i A_i^T is numerically singular
  const double rel_piv = (double)m * 2.220446049250313e-16;
  if (threadIdx.x == 0) bad = 0;
  for (int k = kb; k < ke; ++k) {
    if (!chol_diag_tile(D, b, k, nt, m, row0, L, Dv, T0, T1, bad, rel_piv)) break;
    // panel and trailing update inside the diagonal block
    for (int i = k + 1; i < ke; ++i) {
      __syncthreads();
      load_tile(T2, L + ltile(i, k));
      __syncthreads();
      // X = A_ik * Linv^T:  X[r][c] = sum_p A_ik[r][p] * Linv[c][p] (in place)
      tile_mfma_nt<false>(T2, T2, T1, true);
      __syncthreads();
      store_tile(L + ltile(i, k), T2);
      // A_ij -= L_ik L_jk^T for k < j <= i
      for (int j = k + 1; j <= i; ++j) {
        __syncthreads();
        if (j == i) {
          load_tile(T3, T2);
        } else {
          load_tile(T3, L + ltile(j, k));
        }
        load_tile(T0, L + ltile(i, j));
        __syncthreads();
        tile_mfma_nt<true>(T0, T2, T3, false);
        __syncthreads();
        store_tile(L + ltile(i, j), T0);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad) D.info[b] = bad;
}

// acc (this wave's quadrant, MFMA output layout) -= X Y^T for 64x64
// column-major tiles X, Y in global memory
__device__ __forceinline__ void quad_sub_xyt(dbl4 (&acc)[2][2], const double* __restrict__ X,
                                             const double* __restrict__ Y, int r0, int c0, int li,
                                             int lk) {
#pragma unroll 4
  for (int p0 = 0; p0 < DT; p0 += 4) {
    const int p = p0 + lk;
    const double a0 = -X[p * DT + r0 + li], a1 = -X[p * DT + r0 + 16 + li];
    const double b0 = Y[p * DT + c0 + li], b1 = Y[p * DT + c0 + 16 + li];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

// the wave's quadrant of a 64x64 column-major tile <-> MFMA output layout
// (element (i, j) of a 16x16 result in register r of lane j + 16 g, i = 4 r + g)
__device__ __forceinline__ void quad_load(dbl4 (&acc)[2][2], const double* C, int r0, int c0,
                                          int li, int lk) {
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[ti][tj][r] = C[(c0 + 16 * tj + li) * DT + r0 + 16 * ti + 4 * r + lk];
}
__device__ __forceinline__ void quad_store(double* C, const dbl4 (&acc)[2][2], int r0, int c0,
                                           int li, int lk) {
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        C[(c0 + 16 * tj + li) * DT + r0 + 16 * ti + 4 * r + lk] = acc[ti][tj][r];
}

__global__ void __launch_bounds__(GEMM_THREADS)
k_chol_panel(DenseBlocks D, int kb, const int2* __restrict__ list) {
  extern __shared__ double lds[];
  double* T0 = lds;         // the tile being formed
  double* T1 = lds + TSZ;   // L_kk^{-1}
  const int2 e = list[blockIdx.x];
  const int b = e.x, i = e.y;
  if (D.info[b] != 0) return;
  const int nt = D.nt[b], ke = min(nt, kb + CHOL_PW);
  double* L = D.L + D.loff[b];
  const double* Dv = D.Dinv + D.doff[b];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w & 1), c0 = 32 * (w >> 1), li = l & 15, lk = l >> 4;
  for (int k = kb; k < ke; ++k) {
    dbl4 acc[2][2];
    quad_load(acc, L + ltile(i, k), r0, c0, li, lk);
    for (int c = kb; c < k; ++c) quad_sub_xyt(acc, L + ltile(i, c), L + ltile(k, c), r0, c0, li, lk);
    __syncthreads();
    quad_store(T0, acc, r0, c0, li, lk);
    load_tile(T1, Dv + (long long)k * TSZ);
    __syncthreads();
    tile_mfma_nt<false>(T0, T0, T1, true);
    __syncthreads();
    store_tile(L + ltile(i, k), T0);
    // the next tiles of this row read L_ik back from global memory, each
    // wave its own quadrant's rows of all of it
    __threadfence_block();
    __syncthreads();
  }
}

__global__ void __launch_bounds__(GEMM_THREADS)
k_chol_update(DenseBlocks D, int kb, const int4* __restrict__ list) {
  const int4 e = list[blockIdx.x];
  const int b = e.x, i = e.y, j = e.z;
  if (D.info[b] != 0) return;
  const int nt = D.nt[b], ke = min(nt, kb + CHOL_PW);
  double* L = D.L + D.loff[b];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = 32 * (w & 1), c0 = 32 * (w >> 1), li = l & 15, lk = l >> 4;
  dbl4 acc[2][2];
  quad_load(acc, L + ltile(i, j), r0, c0, li, lk);
  for (int k = kb; k < ke; ++k) quad_sub_xyt(acc, L + ltile(i, k), L + ltile(j, k), r0, c0, li, lk);
  quad_store(L + ltile(i, j), acc, r0, c0, li, lk);
}

// Transposed copy for the backward sweep and FP32 copies of everything.
__global__ void k_dense_finish(DenseBlocks D, int mixed) {
  const int b = blockIdx.y;
  const int nt = D.nt[b];
  const long long ntiles = (long long)nt * (nt + 1) / 2;
  const double* L = D.L + D.loff[b];
  double* LT = D.LT + D.loff[b];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < ntiles * TSZ;
       e += (long long)gridDim.x * blockDim.x) {
    const long long tile = e / TSZ;
    const int off = (int)(e % TSZ);
    // tile index -> (i, j) of the packed lower layout
    int i = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
    while ((long long)(i + 1) * (i + 2) / 2 <= tile) ++i;
    while ((long long)i * (i + 1) / 2 > tile) --i;
    const int j = (int)(tile - (long long)i * (i + 1) / 2);
    const int c = off / DT, r = off % DT;
    // LT tile (j, i) holds (L_ij)^T: element (r, c) = L_ij(c, r)
    const double v = L[tile * TSZ + r * DT + c];
    LT[uttile(nt, j, i) + c * DT + r] = v;
    if (mixed) {
      D.L32[D.loff[b] + tile * TSZ + off] = (float)L[tile * TSZ + off];
      D.LT32[D.loff[b] + uttile(nt, j, i) + c * DT + r] = (float)v;
    }
  }
  if (mixed) {
    const double* Dv = D.Dinv + D.doff[b];
    float* Dv32 = D.Dinv32 + D.doff[b];
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 2LL * nt * TSZ;
         e += (long long)gridDim.x * blockDim.x)
      Dv32[e] = (float)Dv[e];
  }
}

// ------------------------------------------------------------- apply
// y = D L^{-T} L^{-1} D u (D: the row scaling dsc, L L^T the Cholesky
// factorization of the scaled Gram matrix) for one block per workgroup and up to NR vectors
// at once (grid.y walks chunks of NR of the nrhs vectors, vector j at offset
// j * n1).  Forward sweep over tile rows: acc_i = D u_i - sum_{j<i} L_ij z_j,
// z_i = L_ii^{-1} acc_i; backward sweep with the transposed tiles and
// L_ii^{-T}; z of the chunk's vectors stays in LDS.  Every tile product
// (64x64 factor tile times 64 x NR vectors) runs on the matrix cores as
// 16x16x4 MFMAs with the vectors as the N dimension (columns n >= NR are
// zero).  Lane l loads a 4-vector of rows 4 (l % 16) .. + 3 of column
// c0 + l / 16 of the factor tile (64 lanes read 4 whole columns); component
// e of it is the A operand of the MFMA for the rows 4 i' + e, so the 4
// MFMAs of a k-step cover the 64 rows and each factor element is read once.
// Wave w takes the off-diagonal tiles j = w mod 4 of a tile row, the
// partials are summed in wave order with the right-hand side, and wave w
// computes the rows 4 i' + w of the diagonal-tile product.  Every output
// element of an MFMA depends only on its own row and column, so a vector
// gets the same bits whatever the chunk holds.
typedef float flt4 __attribute__((ext_vector_type(4)));
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = flt4; };
template <> struct Vec4<double> { using type = dbl4; };

template <typename T>
__device__ __forceinline__ typename Vec4<T>::type mfma16(T a, T b, typename Vec4<T>::type c) {
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row (0..15) of a 16x16x4 MFMA result held in register v of lane l: the
// FP32 form keeps rows 4 (l / 16) .. + 3 in a lane, the FP64 form rows
// v * 4 + l / 16.  The column is l % 16 in both.
template <typename T>
__device__ __forceinline__ int mfma_row(int l, int v) {
  return sizeof(T) == 4 ? 4 * (l >> 4) + v : 4 * v + (l >> 4);
}

// k-steps whose factor loads are issued together: the whole 64-column tile
// (16 KiB per wave) in FP32, half of it in FP64
template <typename T>
constexpr int multi_u() { return sizeof(T) == 4 ? 16 : 8; }

// acc[e] += tile (64x64, column-major) * Z (64 x NR, rows z[c * NR + n]) for
// the rows 4 i' + e.  Lane l loads the 4-vector of rows 4 (l % 16) .. + 3 of
// column c0 + 4 u + l / 16; the loads of a batch of U k-steps are issued
// before its MFMAs.
template <typename T, int NR>
__device__ __forceinline__ void tile_prod_mfma(const T* __restrict__ tile, const T* z,
                                               typename Vec4<T>::type (&acc)[4], int l) {
  using V = typename Vec4<T>::type;
  constexpr int MULTI_U = multi_u<T>();
  const int li = l & 15, lk = l >> 4;
  const bool bn = li < NR;
  for (int c0 = 0; c0 < DT; c0 += 4 * MULTI_U) {
    V a[MULTI_U];
    T b[MULTI_U];
#pragma unroll
    for (int u = 0; u < MULTI_U; ++u)
      a[u] = *(const V*)(tile + (c0 + 4 * u + lk) * DT + 4 * li);
#pragma unroll
    for (int u = 0; u < MULTI_U; ++u) b[u] = bn ? z[(c0 + 4 * u + lk) * NR + li] : (T)0;
#pragma unroll
    for (int u = 0; u < MULTI_U; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = mfma16<T>(a[u][e], b[u], acc[e]);
  }
}

template <typename T, int NR>
__global__ void __launch_bounds__(APPLY_THREADS)
k_dense_apply(DenseBlocks D, const double* __restrict__ u, double* __restrict__ y,
                    const int* __restrict__ done, int nrhs, int n1, int sys_done) {
  using V = typename Vec4<T>::type;
  extern __shared__ __align__(16) unsigned char dyn[];
  constexpr int NW = APPLY_THREADS / 64;
  static_assert(NW == 4, "one wave per MFMA row interleave");
  const int b = blockIdx.x;
  const int m = D.m[b], nt = D.nt[b], row0 = D.row0[b];
  const int j0 = blockIdx.y * NR;
  // sys_done: one vector (of a batch of systems), stopped with the block's system
  if (sys_done && done && done[D.sys[b]]) return;
  if (sys_done) done = nullptr;
  bool any = false;
  for (int q = 0; q < NR; ++q) any = any || (j0 + q < nrhs && !(done && done[j0 + q]));
  if (!any) return;
  T* zs = (T*)dyn;                                  // nt * DT rows of NR
  T* part = zs + (size_t)nt * DT * NR;              // [NW][DT][NR]
  T* accs = part + (size_t)NW * DT * NR;            // [DT][NR]
  const T* L;
  const T* LT;
  const T* Dv;
  if constexpr (sizeof(T) == 8) {
    L = (const T*)(D.L + D.loff[b]);
    LT = (const T*)(D.LT + D.loff[b]);
    Dv = (const T*)(D.Dinv + D.doff[b]);
  } else {
    L = (const T*)(D.L32 + D.loff[b]);
    LT = (const T*)(D.LT32 + D.loff[b]);
    Dv = (const T*)(D.Dinv32 + D.doff[b]);
  }
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4;
  if (threadIdx.x == 0) atomicAdd(&D.applies[b], 1ull);
  // The right-hand-side step of a tile row: thread t handles the entries
  // q = t + 256 k (k < NR/4) of the 64 x NR tile, always of vector n = t % NR.
  constexpr int QK = DT * NR / APPLY_THREADS;
  static_assert(QK >= 1 && APPLY_THREADS % NR == 0, "entries per thread");
  const int qn = threadIdx.x % NR;
  const bool qon = j0 + qn < nrhs && !(done && done[j0 + qn]);
  // the output rows of lane l in the diagonal-tile product, and whether
  // its vector is written
  const bool non = li < NR && j0 + li < nrhs && !(done && done[j0 + li]);
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    for (int s = 0; s < nt; ++s) {
      const int i = fwd ? s : nt - 1 - s;
      // Loads of this step that depend on nothing computed here are issued
      // first, so that they arrive during the off-diagonal products: the A
      // operands of the diagonal-tile product, the scaled right-hand side
      // (forward) and the output scales (backward).
      const T* inv = Dv + (long long)(fwd ? i : nt + i) * TSZ;
      T ainv[DT / 4];
#pragma unroll
      for (int c = 0; c < DT / 4; ++c) ainv[c] = inv[(4 * c + lk) * DT + 4 * li + w];
      T upre[QK];
      if (fwd) {
#pragma unroll
        for (int k = 0; k < QK; ++k) {
          const int gi = i * DT + (threadIdx.x + APPLY_THREADS * k) / NR;
          upre[k] = (qon && gi < m) ? (T)(u[(size_t)(j0 + qn) * n1 + row0 + gi] * D.dsc[row0 + gi])
                                    : (T)0;
        }
      }
      double osc[4];
      if (!fwd) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = i * DT + 4 * mfma_row<T>(l, v) + w;
          osc[v] = gi < m ? D.dsc[row0 + gi] : 0.0;
        }
      }
      // off-diagonal part of tile row i: tiles j = w mod 4 (j < i forward,
      // j > i backward)
      V acc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = V{};
      if (fwd) {
        for (int j = w; j < i; j += NW)
          tile_prod_mfma<T, NR>(L + ltile(i, j), zs + (size_t)j * DT * NR, acc, l);
      } else {
        for (int j = i + 1 + w; j < nt; j += NW)
          tile_prod_mfma<T, NR>(LT + uttile(nt, i, j), zs + (size_t)j * DT * NR, acc, l);
      }
      if (li < NR)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            part[((size_t)w * DT + 4 * mfma_row<T>(l, v) + e) * NR + li] = acc[e][v];
      __syncthreads();
      // right-hand side of the diagonal tile: (scaled u or z) minus the partials
#pragma unroll
      for (int k = 0; k < QK; ++k) {
        const int q = threadIdx.x + APPLY_THREADS * k;
        const int r = q / NR;
        T a = fwd ? upre[k] : zs[(size_t)(i * DT + r) * NR + qn];
        for (int ww = 0; ww < NW; ++ww) a -= part[((size_t)ww * DT + r) * NR + qn];
        accs[q] = a;
      }
      __syncthreads();
      // diagonal tile: rows 4 i' + w of (L_ii^{-1} or its transpose) * accs
      V d = V{};
#pragma unroll
      for (int c = 0; c < DT / 4; ++c) {
        const T bb = li < NR ? accs[(4 * c + lk) * NR + li] : (T)0;
        d = mfma16<T>(ainv[c], bb, d);
      }
      if (li < NR) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * mfma_row<T>(l, v) + w;
          const int gi = i * DT + r;
          zs[(size_t)gi * NR + li] = d[v];
          if (!fwd && non && gi < m) y[(size_t)(j0 + li) * n1 + row0 + gi] = (double)d[v] * osc[v];
        }
      }
      __syncthreads();
    }
  }
}

// FP32 factors applied in FP64 arithmetic (the mixed-precision projections):
// the same lockstep sweeps, chunks of NR = 4 or 8 vectors, with every tile product on
// v_mfma_f64_4x4x4_4b_f64.  That instruction computes four 4x4x4 blocks;
// block b takes A[i][k] from lane 16 k + 4 b + i and B[k][j] from lane
// 16 k + 4 b + j, and leaves D[i][j] in lane 16 i + 4 b + j (checked on
// gfx950 with an in-bounds one-wave probe).  Lane l loads the 4-vector of
// rows 4 (l % 16) .. + 3 of column c0 + l / 16, as in the FP32 kernel; its
// component g is the A operand of the instruction for the rows 4 m + g, m =
// 4 b + i, so the four instructions of a k-step cover the 64 rows, and each
// group of 4 of the chunk's vectors is the columns j of one instruction.  Every product and sum is FP64 (the
// factor values are the FP32 ones, converted exactly), so the operator is the
// fixed inverse of the rounded factor; an output element depends only on its
// own row and vector.
__device__ __forceinline__ int x_row(int l, int g) { return 16 * ((l & 15) >> 2) + 4 * (l >> 4) + g; }

template <int NR>
__device__ __forceinline__ void tile_prod_x(const float* __restrict__ tile, const double* z,
                                            double (&acc)[NR / 4][4], int l) {
  constexpr int NQ = NR / 4;  // groups of 4 vectors (the columns of one instruction)
  const int li = l & 15, lk = l >> 4, lj = l & 3;
  constexpr int MU = 16;  // the whole 64-column tile's loads issued together
  flt4 a[MU];
  double bz[MU][NQ];
#pragma unroll
  for (int u = 0; u < MU; ++u) a[u] = *(const flt4*)(tile + (4 * u + lk) * DT + 4 * li);
#pragma unroll
  for (int u = 0; u < MU; ++u)
#pragma unroll
    for (int q = 0; q < NQ; ++q) bz[u][q] = z[(4 * u + lk) * NR + 4 * q + lj];
#pragma unroll
  for (int u = 0; u < MU; ++u)
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        acc[q][g] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)a[u][g], bz[u][q], acc[q][g], 0, 0, 0);
}

template <int NR>
__global__ void __launch_bounds__(APPLY_THREADS)
k_dense_apply_x(DenseBlocks D, const double* __restrict__ u, double* __restrict__ y,
                const int* __restrict__ done, int nrhs, int n1, int sys_done) {
  constexpr int NQ = NR / 4;
  extern __shared__ __align__(16) unsigned char dyn[];
  constexpr int NW = APPLY_THREADS / 64;
  static_assert(NW == 4, "one wave per row interleave");
  const int b = blockIdx.x;
  const int m = D.m[b], nt = D.nt[b], row0 = D.row0[b];
  const int j0 = blockIdx.y * NR;
  if (sys_done && done && done[D.sys[b]]) return;
  if (sys_done) done = nullptr;
  bool any = false;
  for (int q = 0; q < NR; ++q) any = any || (j0 + q < nrhs && !(done && done[j0 + q]));
  if (!any) return;
  double* zs = (double*)dyn;                             // nt * DT rows of NR
  double* part = zs + (size_t)nt * DT * NR;              // [NW][DT][NR]
  double* accs = part + (size_t)NW * DT * NR;            // [DT][NR]
  const float* L = D.L32 + D.loff[b];
  const float* LT = D.LT32 + D.loff[b];
  const float* Dv = D.Dinv32 + D.doff[b];
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4, lj = l & 3;
  if (threadIdx.x == 0) atomicAdd(&D.applies[b], 1ull);
  // right-hand-side step: thread t handles the entries t + 256 k of the
  // 64 x NR tile, always of vector t % NR
  constexpr int QK = DT * NR / APPLY_THREADS;
  const int qn = threadIdx.x % NR;
  const bool qon = j0 + qn < nrhs && !(done && done[j0 + qn]);
  // the vectors of this lane's outputs, and whether they are written
  bool non[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) non[q] = j0 + 4 * q + lj < nrhs && !(done && done[j0 + 4 * q + lj]);
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    for (int s = 0; s < nt; ++s) {
      const int i = fwd ? s : nt - 1 - s;
      const float* inv = Dv + (long long)(fwd ? i : nt + i) * TSZ;
      float ainv[DT / 4];
#pragma unroll
      for (int c = 0; c < DT / 4; ++c) ainv[c] = inv[(4 * c + lk) * DT + 4 * li + w];
      double upre[QK];
      if (fwd) {
#pragma unroll
        for (int k = 0; k < QK; ++k) {
          const int gi = i * DT + (threadIdx.x + APPLY_THREADS * k) / NR;
          upre[k] = (qon && gi < m) ? u[(size_t)(j0 + qn) * n1 + row0 + gi] * D.dsc[row0 + gi] : 0.0;
        }
      }
      const int orow = x_row(l, w);  // this lane's output row of the diagonal product
      double osc = 0.0;
      if (!fwd) {
        const int gi = i * DT + orow;
        osc = gi < m ? D.dsc[row0 + gi] : 0.0;
      }
      double acc[NQ][4];
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[q][g] = 0.0;
      if (fwd) {
        for (int j = w; j < i; j += NW)
          tile_prod_x<NR>(L + ltile(i, j), zs + (size_t)j * DT * NR, acc, l);
      } else {
        for (int j = i + 1 + w; j < nt; j += NW)
          tile_prod_x<NR>(LT + uttile(nt, i, j), zs + (size_t)j * DT * NR, acc, l);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int g = 0; g < 4; ++g)
          part[((size_t)w * DT + x_row(l, g)) * NR + 4 * q + lj] = acc[q][g];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < QK; ++k) {
        const int e = threadIdx.x + APPLY_THREADS * k;
        const int r = e / NR;
        double a = fwd ? upre[k] : zs[(size_t)(i * DT + r) * NR + qn];
        for (int ww = 0; ww < NW; ++ww) a -= part[((size_t)ww * DT + r) * NR + qn];
        accs[e] = a;
      }
      __syncthreads();
      // diagonal tile: rows 4 m + w of (L_ii^{-1} or its transpose) * accs
      double d[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) d[q] = 0.0;
#pragma unroll
      for (int c = 0; c < DT / 4; ++c)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          d[q] = __builtin_amdgcn_mfma_f64_4x4x4f64((double)ainv[c],
                                                    accs[(4 * c + lk) * NR + 4 * q + lj], d[q], 0,
                                                    0, 0);
      const int gi = i * DT + orow;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        zs[(size_t)gi * NR + 4 * q + lj] = d[q];
        if (!fwd && non[q] && gi < m) y[(size_t)(j0 + 4 * q + lj) * n1 + row0 + gi] = d[q] * osc;
      }
      __syncthreads();
    }
  }
}

// The same sweeps with tile rows owned by waves, for chunks whose LDS leaves
// room for one workgroup per CU only (where the lockstep sweep above would
// leave the CU idle at every barrier).  Wave w computes the rows k = w mod 4
// from start to end (its off-diagonal tiles in order, then the diagonal-tile
// product for all 64 rows) and publishes each finished row with an LDS flag.
// A wave reading z_j (y_j) first waits for that flag; since every row needs
// the one before it, rows finish in order, and the loads of a tile are issued
// before the wait for the row they multiply, so one wave streams its factor
// tiles while another finishes its diagonal product.  The waits are bounded
// by the wall clock (D.wait_ticks); a wave that gives up sets *D.err (the
// result is then invalid).

// Orders the LDS accesses of the lanes of one wave (they execute in program
// order; the fences keep the compiler from moving accesses across).
__device__ __forceinline__ void dense_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Waits until a row of the current sweep is published (its flag >= 1).
__device__ __forceinline__ void wait_row(const int* flag, unsigned long long t0, int* err,
                                         unsigned long long ticks, bool& ok) {
  // ticks == 0 gives up at the first check
  while (ok && (ticks == 0 ||
                __hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < 1)) {
    if (wall_clock64() - t0 > ticks) {
      if ((threadIdx.x & 63) == 0) atomicExch(err, 1);
      ok = false;
    } else {
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

// Publishes a row of the current sweep after the LDS writes of every lane of
// the wave.
__device__ __forceinline__ void publish_row(int* flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  if ((threadIdx.x & 63) == 0)
    __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename T, int NR>
__global__ void __launch_bounds__(APPLY_THREADS)
k_dense_apply_rows(DenseBlocks D, const double* __restrict__ u, double* __restrict__ y,
              const int* __restrict__ done, int nrhs, int n1, int sys_done) {
  using V = typename Vec4<T>::type;
  extern __shared__ __align__(16) unsigned char dyn[];
  constexpr int NW = APPLY_THREADS / 64;
  constexpr int U = multi_u<T>();
  const unsigned long long t0 = wall_clock64();
  const int b = blockIdx.x;
  const int m = D.m[b], nt = D.nt[b], row0 = D.row0[b];
  const int j0 = blockIdx.y * NR;
  // sys_done: one vector (of a batch of systems), stopped with the block's system
  if (sys_done && done && done[D.sys[b]]) return;
  if (sys_done) done = nullptr;
  bool any = false;
  for (int q = 0; q < NR; ++q) any = any || (j0 + q < nrhs && !(done && done[j0 + q]));
  if (!any) return;
  T* zs = (T*)dyn;                                  // nt * DT rows of NR
  T* wsc = zs + (size_t)nt * DT * NR;               // per wave: DT rows of NR
  int* flags = (int*)(wsc + (size_t)NW * DT * NR);  // 2 * nt: forward, backward
  const T* L;
  const T* LT;
  const T* Dv;
  if constexpr (sizeof(T) == 8) {
    L = (const T*)(D.L + D.loff[b]);
    LT = (const T*)(D.LT + D.loff[b]);
    Dv = (const T*)(D.Dinv + D.doff[b]);
  } else {
    L = (const T*)(D.L32 + D.loff[b]);
    LT = (const T*)(D.LT32 + D.loff[b]);
    Dv = (const T*)(D.Dinv32 + D.doff[b]);
  }
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = l & 15, lk = l >> 4;
  const bool bn = li < NR;                                           // column holds a vector
  const bool on = bn && j0 + li < nrhs && !(done && done[j0 + li]);  // ... that is written
  T* my = wsc + (size_t)w * DT * NR;
  for (int e = threadIdx.x; e < 2 * nt; e += APPLY_THREADS) flags[e] = 0;
  if (threadIdx.x == 0) atomicAdd(&D.applies[b], 1ull);
  __syncthreads();
  bool ok = true;
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = pass == 0;
    int* fl = flags + (fwd ? 0 : nt);
    // rows known to be finished: forward j <= ready, backward j >= ready
    int ready = fwd ? -1 : nt;
    const int nown = (nt - w + NW - 1) / NW;  // rows owned by this wave
    for (int s = 0; s < nown; ++s) {
      const int k = fwd ? w + NW * s : w + NW * (nown - 1 - s);
      const int gk = k * DT;
      // loads that depend on nothing of this sweep: the right-hand side of
      // the row (forward) and the output scales, issued first in FP32 (in
      // FP64 their registers would cost occupancy; they are loaded at use)
      constexpr bool PRE = sizeof(T) == 4;
      double ru[16], rd[16];
      auto load_rhs = [&]() {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gi = gk + 4 * mfma_row<T>(l, v) + e;
            const bool in = gi < m;
            rd[4 * e + v] = in ? D.dsc[row0 + gi] : 0.0;
            ru[4 * e + v] = (fwd && in && on) ? u[(size_t)(j0 + li) * n1 + row0 + gi] : 0.0;
          }
      };
      if constexpr (PRE) load_rhs();
      // off-diagonal tiles: forward j = 0 .. k-1, backward j = nt-1 .. k+1,
      // in the order their rows finish
      V acc[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = V{};
      const int nj = fwd ? k : nt - 1 - k;
      for (int q = 0; q < nj; ++q) {
        const int j = fwd ? q : nt - 1 - q;
        const T* tile = fwd ? L + ltile(k, j) : LT + uttile(nt, k, j);
        const T* zj = zs + (size_t)j * DT * NR;
        for (int c0 = 0; c0 < DT; c0 += 4 * U) {
          V a[U];
#pragma unroll
          for (int uu = 0; uu < U; ++uu)
            a[uu] = *(const V*)(tile + (c0 + 4 * uu + lk) * DT + 4 * li);
          if (c0 == 0 && (fwd ? j > ready : j < ready)) {
            wait_row(fl + j, t0, D.err, D.wait_ticks, ok);
            ready = j;
          }
          T bz[U];
#pragma unroll
          for (int uu = 0; uu < U; ++uu) bz[uu] = bn ? zj[(c0 + 4 * uu + lk) * NR + li] : (T)0;
#pragma unroll
          for (int uu = 0; uu < U; ++uu)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = mfma16<T>(a[uu][e], bz[uu], acc[e]);
        }
      }
      // a = (D u_k, or z_k) - acc; its rows are re-read as B operands
      // through the wave's LDS scratch
      if constexpr (!PRE) load_rhs();
      if (bn) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 4 * mfma_row<T>(l, v) + e;
            const T base = fwd ? (T)(ru[4 * e + v] * rd[4 * e + v]) : zs[(size_t)(gk + r) * NR + li];
            my[r * NR + li] = base - acc[e][v];
          }
      }
      dense_wave_sync();
      // diagonal tile: (L_kk^{-1} or its transpose) times a, all 64 rows
      const T* inv = Dv + (long long)(fwd ? k : nt + k) * TSZ;
      T bq[DT / 4];
#pragma unroll
      for (int c = 0; c < DT / 4; ++c) bq[c] = bn ? my[(4 * c + lk) * NR + li] : (T)0;
      V d[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) d[e] = V{};
#pragma unroll
      for (int c = 0; c < DT / 4; ++c) {
        const V iv = *(const V*)(inv + (4 * c + lk) * DT + 4 * li);
#pragma unroll
        for (int e = 0; e < 4; ++e) d[e] = mfma16<T>(iv[e], bq[c], d[e]);
      }
      if (bn) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 4 * mfma_row<T>(l, v) + e;
            const int gi = gk + r;
            zs[(size_t)gi * NR + li] = d[e][v];
            if (!fwd && on && gi < m)
              y[(size_t)(j0 + li) * n1 + row0 + gi] = (double)d[e][v] * rd[4 * e + v];
          }
      }
      publish_row(fl + k);
      dense_wave_sync();  // the scratch is reused by the next row
    }
    __syncthreads();  // every forward row is in before the backward sweep
  }
}

}  // namespace

hipError_t launch_gram(hipStream_t st, const DenseBlocks& D, const int4* tiles, int ntiles,
                       const int* rowptr, const int* col, const double* val, const int* tptr,
                       const int* trow, const double* tval) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram, dim3(ntiles), dim3(64), 0, st, D, tiles, rowptr, col, val, tptr,
                     trow, tval);
  return hipGetLastError();
}

hipError_t launch_cholesky(hipStream_t st, const DenseBlocks& D, const CholPlan& P) {
  if (D.nblk == 0) return hipSuccess;
  const size_t lds = 4 * TSZ * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_chol_diag,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  for (int s = 0; s < P.steps; ++s) {
    const int kb = s * CHOL_PW;
    hipLaunchKernelGGL(k_chol_diag, dim3(D.nblk), dim3(GEMM_THREADS), lds, st, D, kb);
    const long long np = P.panel_off[s + 1] - P.panel_off[s];
    if (np > 0)
      hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)np), dim3(GEMM_THREADS),
                         2 * TSZ * sizeof(double), st, D, kb, P.panel + P.panel_off[s]);
    const long long nu = P.upd_off[s + 1] - P.upd_off[s];
    if (nu > 0)
      hipLaunchKernelGGL(k_chol_update, dim3((unsigned)nu), dim3(GEMM_THREADS), 0, st, D, kb,
                         P.upd + P.upd_off[s]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_dense_finish(hipStream_t st, const DenseBlocks& D, bool mixed) {
  if (D.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_finish, dim3(64, D.nblk), dim3(256), 0, st, D, (int)mixed);
  return hipGetLastError();
}

// Dynamic LDS of k_dense_apply for NR vectors and blocks of up to
// max_nt tiles (z, the partials of the 4 waves and the diagonal right-hand
// side), and of k_dense_apply_rows (z, one 64-row scratch per wave and
// 2 * max_nt row flags).
size_t dense_multi_lds(int nr, int max_nt, bool mixed) {
  return (size_t)(max_nt + 5) * DT * nr * (mixed ? sizeof(float) : sizeof(double));
}
size_t dense_rows_lds(int nr, int max_nt, bool mixed) {
  return (size_t)(max_nt + APPLY_THREADS / 64) * DT * nr * (mixed ? sizeof(float) : sizeof(double)) +
         2 * (size_t)max_nt * sizeof(int);
}

// The lockstep sweep while two workgroups fit on a CU; the row-owned sweep
// when only one does (measured on the 27-point 100^3 blocks: 16 FP32
// vectors per chunk 2.51 -> 1.54 ms, while with two workgroups per CU the
// lockstep sweep stays 4% ahead).
template <typename T, int NR>
hipError_t launch_dense_multi_nr(hipStream_t st, const DenseBlocks& D, const double* u, double* y,
                                 const int* done, int nrhs, int n1, int max_nt, int sys_done) {
  const bool f32 = sizeof(T) == 4;
  const dim3 grid(D.nblk, (nrhs + NR - 1) / NR);
  const size_t lds = dense_multi_lds(NR, max_nt, f32);
  if (lds <= DENSE_MULTI_LDS / 2)
    hipLaunchKernelGGL((k_dense_apply<T, NR>), grid, dim3(APPLY_THREADS), lds, st, D, u, y, done,
                       nrhs, n1, sys_done);
  else
    hipLaunchKernelGGL((k_dense_apply_rows<T, NR>), grid, dim3(APPLY_THREADS),
                       dense_rows_lds(NR, max_nt, f32), st, D, u, y, done, nrhs, n1, sys_done);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_multi_t(hipStream_t st, const DenseBlocks& D, const double* u, double* y,
                                const int* done, int nrhs, int n1, int max_nt, int sys_done) {
  // chunk width: the widest of 16, 8 and 4 vectors (no wider than nrhs
  // needs) whose LDS fits in one workgroup, so each factor is read as few
  // times as possible (a narrower chunk at higher occupancy reads it more
  // often and was measured slower)
  const bool f32 = sizeof(T) == 4;
  int nr = 16;
  while (nr > 4 && (nr / 2 >= nrhs || dense_multi_lds(nr, max_nt, f32) > DENSE_MULTI_LDS)) nr /= 2;
  switch (nr) {
    case 16: return launch_dense_multi_nr<T, 16>(st, D, u, y, done, nrhs, n1, max_nt, sys_done);
    case 8: return launch_dense_multi_nr<T, 8>(st, D, u, y, done, nrhs, n1, max_nt, sys_done);
    default: return launch_dense_multi_nr<T, 4>(st, D, u, y, done, nrhs, n1, max_nt, sys_done);
  }
}

// Allows every variant of the apply the full LDS of a workgroup (once per
// process and device, outside any stream capture).
hipError_t prepare_dense_apply() {
  const void* fns[] = {(const void*)k_dense_apply_x<4>, (const void*)k_dense_apply_x<8>,
                       (const void*)k_dense_apply<double, 4>,      (const void*)k_dense_apply<double, 8>,
                       (const void*)k_dense_apply<double, 16>,     (const void*)k_dense_apply_rows<double, 4>,
                       (const void*)k_dense_apply_rows<double, 8>, (const void*)k_dense_apply_rows<double, 16>};
  for (const void* fn : fns) {
    const hipError_t e =
        hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)DENSE_MULTI_LDS);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// FP32 factors with FP64 arithmetic: chunks of 4 vectors
// (chunks of 8 when more than 4 vectors and their LDS fits: one read of each
// factor per 8 vectors)
hipError_t launch_dense_x(hipStream_t st, const DenseBlocks& D, const double* u, double* y,
                          const int* done, int nrhs, int n1, int max_nt, int sys_done) {
  if (nrhs > 4 && dense_multi_lds(8, max_nt, false) <= DENSE_MULTI_LDS) {
    hipLaunchKernelGGL(k_dense_apply_x<8>, dim3(D.nblk, (nrhs + 7) / 8), dim3(APPLY_THREADS),
                       dense_multi_lds(8, max_nt, false), st, D, u, y, done, nrhs, n1, sys_done);
  } else {
    hipLaunchKernelGGL(k_dense_apply_x<4>, dim3(D.nblk, (nrhs + 3) / 4), dim3(APPLY_THREADS),
                       dense_multi_lds(4, max_nt, false), st, D, u, y, done, nrhs, n1, sys_done);
  }
  return hipGetLastError();
}

hipError_t launch_dense_apply_multi(hipStream_t st, const DenseBlocks& D, bool mixed,
                                    const double* u, double* y, const int* done, int nrhs, int n1,
                                    int max_nt) {
  if (D.nblk == 0 || nrhs <= 0) return hipSuccess;
  if (dense_multi_lds(4, max_nt, false) > DENSE_MULTI_LDS) return hipErrorInvalidValue;
  return mixed ? launch_dense_x(st, D, u, y, done, nrhs, n1, max_nt, 0)
               : launch_dense_multi_t<double>(st, D, u, y, done, nrhs, n1, max_nt, 0);
}

hipError_t launch_dense_apply(hipStream_t st, const DenseBlocks& D, bool mixed, const double* u,
                              double* y, const int* done, int max_nt) {
  if (D.nblk == 0) return hipSuccess;
  if (dense_multi_lds(4, max_nt, false) > DENSE_MULTI_LDS) return hipErrorInvalidValue;
  return mixed ? launch_dense_x(st, D, u, y, done, 1, 0, max_nt, 1)
               : launch_dense_multi_t<double>(st, D, u, y, done, 1, 0, max_nt, 1);
}
