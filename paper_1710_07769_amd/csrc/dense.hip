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
// Right-looking blocked Cholesky of one block per workgroup, in place on the
// packed lower tiles: factor the diagonal tile, invert it, form the panel
// L_ik = A_ik L_kk^{-T}, update the trailing tiles A_ij -= L_ik L_jk^T.
__global__ void __launch_bounds__(GEMM_THREADS)
k_cholesky(DenseBlocks D) {
  extern __shared__ double lds[];
  double* T0 = lds;             // diagonal tile / C tile
  double* T1 = lds + TSZ;       // inverse of the diagonal tile
  double* T2 = lds + 2 * TSZ;   // panel tile X
  double* T3 = lds + 3 * TSZ;   // panel tile Y
  __shared__ int bad;
  const int b = blockIdx.x;
  const int nt = D.nt[b], m = D.m[b], row0 = D.row0[b];
  double* L = D.L + D.loff[b];
  double* Dv = D.Dinv + D.doff[b];
  // a pivot at or below m * eps * G_jj means A_i A_i^T is numerically singular
  const double rel_piv = (double)m * 2.220446049250313e-16;
  if (threadIdx.x == 0) bad = 0;
  for (int k = 0; k < nt; ++k) {
    __syncthreads();
    load_tile(T0, L + ltile(k, k));
    __syncthreads();
    // unblocked Cholesky of the diagonal tile (column by column)
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
      if (bad) break;
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
    if (bad) break;
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
    // panel and trailing update
    for (int i = k + 1; i < nt; ++i) {
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
  if (threadIdx.x == 0) D.info[b] = bad;
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
// y = L^{-T} L^{-1} u for one block per workgroup.  Forward sweep over tile
// rows: acc_i = u_i - sum_{j<i} L_ij z_j (the j tiles are split over the
// wavefronts; lane r owns row r, so each load reads one 512-byte column),
// then z_i = Linv_i acc_i.  Backward sweep with the LT tiles and Linv_i^T.
template <typename T>
__global__ void __launch_bounds__(APPLY_THREADS)
k_dense_apply(DenseBlocks D, const double* __restrict__ u, double* __restrict__ y,
              const int* __restrict__ done) {
  __shared__ T zs[4096 + DT];
  __shared__ T part[APPLY_THREADS / 64][DT];
  __shared__ T accs[DT];
  const int b = blockIdx.x;
  if (done && done[D.sys[b]]) return;
  const int m = D.m[b], nt = D.nt[b], row0 = D.row0[b];
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
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = APPLY_THREADS / 64;
  if (threadIdx.x == 0) atomicAdd(&D.applies[b], 1ull);
  // forward: z = L^{-1} u
  for (int i = 0; i < nt; ++i) {
    T acc = (T)0;
    for (int j = w; j < i; j += NW) {
      const T* tile = L + ltile(i, j);
      const T* zj = zs + j * DT;
#pragma unroll 8
      for (int c = 0; c < DT; ++c) acc += tile[c * DT + lane] * zj[c];
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
      const int gi = i * DT + lane;
      T a = gi < m ? (T)(u[row0 + gi] * D.dsc[row0 + gi]) : (T)0;
      for (int q = 0; q < NW; ++q) a -= part[q][lane];
      accs[lane] = a;
    }
    __syncthreads();
    if (w == 0) {
      const T* inv = Dv + (long long)i * TSZ;
      T s = (T)0;
#pragma unroll 8
      for (int c = 0; c < DT; ++c) s += inv[c * DT + lane] * accs[c];
      zs[i * DT + lane] = s;
    }
    __syncthreads();
  }
  // backward: y = L^{-T} z, overwriting zs tile by tile from the end
  for (int i = nt - 1; i >= 0; --i) {
    T acc = (T)0;
    for (int j = i + 1 + w; j < nt; j += NW) {
      const T* tile = LT + uttile(nt, i, j);
      const T* yj = zs + j * DT;
#pragma unroll 8
      for (int c = 0; c < DT; ++c) acc += tile[c * DT + lane] * yj[c];
    }
    part[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
      T a = zs[i * DT + lane];
      for (int q = 0; q < NW; ++q) a -= part[q][lane];
      accs[lane] = a;
    }
    __syncthreads();
    if (w == 0) {
      const T* invT = Dv + (long long)(nt + i) * TSZ;
      T s = (T)0;
#pragma unroll 8
      for (int c = 0; c < DT; ++c) s += invT[c * DT + lane] * accs[c];
      zs[i * DT + lane] = s;
      const int gi = i * DT + lane;
      if (gi < m) y[row0 + gi] = (double)s * D.dsc[row0 + gi];
    }
    __syncthreads();
  }
}

// The same sweeps for NR right-hand sides at once (grid.y walks chunks of NR
// of the nrhs vectors, vector j at offset j * n1).  Each L, LT and inverse
// element is loaded once and used for the NR vectors, whose sums run in the
// order of k_dense_apply, so every vector gets the bits of a one-vector
// apply.  z of the NR vectors sits in dynamic LDS as zs[row][NR]; the
// diagonal-tile steps of vector q run on wavefront q % NW.
template <typename T, int NR>
__global__ void __launch_bounds__(APPLY_THREADS)
k_dense_apply_multi(DenseBlocks D, const double* __restrict__ u, double* __restrict__ y,
                    const int* __restrict__ done, int nrhs, int n1) {
  extern __shared__ __align__(16) unsigned char dyn[];
  constexpr int NW = APPLY_THREADS / 64;
  const int b = blockIdx.x;
  const int m = D.m[b], nt = D.nt[b], row0 = D.row0[b];
  const int j0 = blockIdx.y * NR;
  bool act[NR];
  bool any = false;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    act[q] = j0 + q < nrhs && !(done && done[j0 + q]);
    any = any || act[q];
  }
  if (!any) return;
  T* zs = (T*)dyn;                                  // nt * DT rows of NR
  T* part = zs + (size_t)nt * DT * NR;              // [NW][NR][DT]
  T* accs = part + (size_t)NW * NR * DT;            // [NR][DT]
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
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) atomicAdd(&D.applies[b], 1ull);
  // forward: z = L^{-1} u
  for (int i = 0; i < nt; ++i) {
    T acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = (T)0;
    for (int j = w; j < i; j += NW) {
      const T* tile = L + ltile(i, j);
      const T* zj = zs + (size_t)j * DT * NR;
#pragma unroll 4
      for (int c = 0; c < DT; ++c) {
        const T l = tile[c * DT + lane];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] += l * zj[c * NR + q];
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) part[(w * NR + q) * DT + lane] = acc[q];
    __syncthreads();
    const int gi = i * DT + lane;
    for (int q = w; q < NR; q += NW) {
      const int jr = j0 + q;
      T a = (gi < m && act[q]) ? (T)(u[(size_t)jr * n1 + row0 + gi] * D.dsc[row0 + gi]) : (T)0;
      for (int qq = 0; qq < NW; ++qq) a -= part[(qq * NR + q) * DT + lane];
      accs[q * DT + lane] = a;
    }
    __syncthreads();
    for (int q = w; q < NR; q += NW) {
      const T* inv = Dv + (long long)i * TSZ;
      const T* aq = accs + q * DT;
      T s = (T)0;
#pragma unroll 8
      for (int c = 0; c < DT; ++c) s += inv[c * DT + lane] * aq[c];
      zs[(size_t)gi * NR + q] = s;
    }
    __syncthreads();
  }
  // backward: y = L^{-T} z, overwriting zs tile by tile from the end
  for (int i = nt - 1; i >= 0; --i) {
    T acc[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) acc[q] = (T)0;
    for (int j = i + 1 + w; j < nt; j += NW) {
      const T* tile = LT + uttile(nt, i, j);
      const T* yj = zs + (size_t)j * DT * NR;
#pragma unroll 4
      for (int c = 0; c < DT; ++c) {
        const T l = tile[c * DT + lane];
#pragma unroll
        for (int q = 0; q < NR; ++q) acc[q] += l * yj[c * NR + q];
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) part[(w * NR + q) * DT + lane] = acc[q];
    __syncthreads();
    const int gi = i * DT + lane;
    for (int q = w; q < NR; q += NW) {
      T a = zs[(size_t)gi * NR + q];
      for (int qq = 0; qq < NW; ++qq) a -= part[(qq * NR + q) * DT + lane];
      accs[q * DT + lane] = a;
    }
    __syncthreads();
    for (int q = w; q < NR; q += NW) {
      const T* invT = Dv + (long long)(nt + i) * TSZ;
      const T* aq = accs + q * DT;
      T s = (T)0;
#pragma unroll 8
      for (int c = 0; c < DT; ++c) s += invT[c * DT + lane] * aq[c];
      zs[(size_t)gi * NR + q] = s;
      if (gi < m && act[q]) y[(size_t)(j0 + q) * n1 + row0 + gi] = (double)s * D.dsc[row0 + gi];
    }
    __syncthreads();
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

hipError_t launch_cholesky(hipStream_t st, const DenseBlocks& D) {
  if (D.nblk == 0) return hipSuccess;
  const size_t lds = 4 * TSZ * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_cholesky,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cholesky, dim3(D.nblk), dim3(GEMM_THREADS), lds, st, D);
  return hipGetLastError();
}

hipError_t launch_dense_finish(hipStream_t st, const DenseBlocks& D, bool mixed) {
  if (D.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_finish, dim3(64, D.nblk), dim3(256), 0, st, D, (int)mixed);
  return hipGetLastError();
}

// Dynamic LDS of k_dense_apply_multi for NR vectors and blocks of up to
// max_nt tiles.
size_t dense_multi_lds(int nr, int max_nt, bool mixed) {
  return (size_t)(max_nt + 5) * DT * nr * (mixed ? sizeof(float) : sizeof(double));
}

template <typename T, int NR>
hipError_t launch_dense_multi_nr(hipStream_t st, const DenseBlocks& D, const double* u, double* y,
                                 const int* done, int nrhs, int n1, size_t lds) {
  const void* fn = (const void*)k_dense_apply_multi<T, NR>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_dense_apply_multi<T, NR>), dim3(D.nblk, (nrhs + NR - 1) / NR),
                     dim3(APPLY_THREADS), lds, st, D, u, y, done, nrhs, n1);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dense_multi_t(hipStream_t st, const DenseBlocks& D, const double* u, double* y,
                                const int* done, int nrhs, int n1, int max_nt) {
  // the widest chunk (at most 8, and at most the next power of two of nrhs)
  // whose LDS fits in one workgroup
  int nr = 8;
  while (nr > 1 && (nr / 2 >= nrhs || dense_multi_lds(nr, max_nt, sizeof(T) == 4) > DENSE_MULTI_LDS))
    nr /= 2;
  const size_t lds = dense_multi_lds(nr, max_nt, sizeof(T) == 4);
  switch (nr) {
    case 8: return launch_dense_multi_nr<T, 8>(st, D, u, y, done, nrhs, n1, lds);
    case 4: return launch_dense_multi_nr<T, 4>(st, D, u, y, done, nrhs, n1, lds);
    case 2: return launch_dense_multi_nr<T, 2>(st, D, u, y, done, nrhs, n1, lds);
    default: return launch_dense_multi_nr<T, 1>(st, D, u, y, done, nrhs, n1, lds);
  }
}

hipError_t launch_dense_apply_multi(hipStream_t st, const DenseBlocks& D, bool mixed,
                                    const double* u, double* y, const int* done, int nrhs, int n1,
                                    int max_nt) {
  if (D.nblk == 0 || nrhs <= 0) return hipSuccess;
  if (dense_multi_lds(1, max_nt, mixed) > DENSE_MULTI_LDS) return hipErrorInvalidValue;
  return mixed ? launch_dense_multi_t<float>(st, D, u, y, done, nrhs, n1, max_nt)
               : launch_dense_multi_t<double>(st, D, u, y, done, nrhs, n1, max_nt);
}

hipError_t launch_dense_apply(hipStream_t st, const DenseBlocks& D, bool mixed, const double* u,
                              double* y, const int* done) {
  if (D.nblk == 0) return hipSuccess;
  if (mixed)
    hipLaunchKernelGGL(k_dense_apply<float>, dim3(D.nblk), dim3(APPLY_THREADS), 0, st, D, u, y,
                       done);
  else
    hipLaunchKernelGGL(k_dense_apply<double>, dim3(D.nblk), dim3(APPLY_THREADS), 0, st, D, u, y,
                       done);
  return hipGetLastError();
}
