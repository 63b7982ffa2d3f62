// Banded Cholesky projections.
//
// For a block whose rows are in reverse Cuthill-McKee order, the scaled
// normal-equation matrix G = D A_i A_i^T D (D = unit-row scaling; Section 1,
// eq. (H): y_i = (A_i A_i^T)^{-1} u_i) is banded with a small half-bandwidth
// bw, and so is its Cholesky factor (a banded matrix factors without fill
// outside its band).  Setup forms G in the band storage (k_band_gram),
// factors it in FP64 in place (k_band_chol) and derives the reversed
// transpose and the FP32 copies (k_band_finish).  Each projection then runs
// two banded triangular sweeps (k_band_apply): L z = D u and L^T w = z, y = D w.
//
// Storage (see BandBlocks): per 64-row tile, diagonal-major, entry d of local
// row p at tile*64*ld + d*64 + p%64, column p - bw + d (ld = bw+1 rounded up
// to a multiple of 4).  Lanes of a wave own consecutive rows, so every band
// access of the sweeps is coalesced, and a tile is one contiguous chunk.
#include "common.h"

#include <cmath>
#include <utility>
#include <vector>

std::vector<int> band_nvp_buckets(const BandBlocks& B, size_t elem);

namespace {

__device__ __forceinline__ long long band_at(int p, int d, int ld) {
  return (long long)(p >> 6) * 64 * ld + (long long)d * 64 + (p & 63);
}

// ------------------------------------------------------------------ Gram
// One workgroup per block; thread-per-row.  Row p of G: for every entry
// (c, a_pc) of row p and every row s of column c with p - bw <= s <= p,
// G[p][s] += (a_pc d_p)(a_sc d_s), accumulated in the fixed order (entries of
// row p by ascending column, rows of a column ascending).
__global__ void __launch_bounds__(256)
k_band_gram(BandBlocks B, const int* __restrict__ rowptr, const int* __restrict__ col,
            const double* __restrict__ val, const int* __restrict__ tptr,
            const int* __restrict__ trow, const double* __restrict__ tval) {
  const int blk = blockIdx.x;
  const int m = B.m[blk], bw = B.bw[blk], ld = B.ld[blk], row0 = B.row0[blk];
  const int nt = (m + 63) >> 6;
  double* G = B.L + B.off[blk];
  for (int p = threadIdx.x; p < nt * 64; p += blockDim.x) {
    for (int d = 0; d < ld; ++d) G[band_at(p, d, ld)] = 0.0;
    if (p >= m) continue;
    const int i = row0 + p;
    const double di = B.dsc[i];
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int c = col[e];
      const double a = val[e] * di;
      for (int q = tptr[c]; q < tptr[c + 1]; ++q) {
        const int s = trow[q] - row0;
        if (s < p - bw) continue;
        if (s > p) break;  // rows of a column are ascending
        const double gs = a * (tval[q] * B.dsc[row0 + s]);
        G[band_at(p, s - p + bw, ld)] += gs;
      }
    }
  }
}

// -------------------------------------------------------------- Cholesky
// Right-looking banded Cholesky, one workgroup per block, with the active
// window (rows j..j+bw, each with its bw+1 band entries) held in LDS as a
// circular buffer of rows.  Step j: pivot L_jj = sqrt(G_jj) with the relative
// test G_jj > m eps G_jj(original); multipliers l_i = G_ij / L_jj for the
// rows i <= j+bw below it; rank-1 update of the trailing window; row j is
// final and goes back to global memory, and row j+bw+1 enters its slot.
__global__ void __launch_bounds__(256)
k_band_chol(BandBlocks B) {
  extern __shared__ double lds[];
  const int blk = blockIdx.x;
  const int m = B.m[blk], bw = B.bw[blk], W = bw + 1, ld = B.ld[blk];
  double* win = lds;            // W x W
  double* gd = lds + W * W;     // original diagonal of the row in each slot
  double* G = B.L + B.off[blk];
  const int tid = threadIdx.x;
  const double rel_piv = (double)m * 2.220446049250313e-16;
  for (int e = tid; e < W * W; e += blockDim.x) {
    const int r = e / W, d = e - r * W;
    win[e] = r < m ? G[band_at(r, d, ld)] : 0.0;
  }
  for (int r = tid; r < W; r += blockDim.x) gd[r] = r < m ? G[band_at(r, bw, ld)] : 1.0;
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    const int sj = j % W;
    const double a = win[sj * W + bw];
    if (!(a > rel_piv * gd[sj])) {  // uniform: every thread reads the same value
      if (tid == 0) B.info[blk] = j + 1;
      return;
    }
    const double ljj = sqrt(a);
    const double inv = 1.0 / ljj;
    const int nb = min(bw, m - 1 - j);
    // multipliers: row i = j+1+t holds column j at d = bw-1-t
    if (tid < nb) {
      const int si = (j + 1 + tid) % W;
      win[si * W + (bw - 1 - tid)] *= inv;
    }
    __syncthreads();
    // trailing update over pairs (i, k), j < k <= i <= j + nb
    const int npairs = nb * (nb + 1) / 2;
    for (int q = tid; q < npairs; q += blockDim.x) {
      int ii = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
      while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
      while (ii * (ii + 1) / 2 > q) --ii;
      const int kk = q - ii * (ii + 1) / 2;
      const int si = (j + 1 + ii) % W, sk = (j + 1 + kk) % W;
      const double li = win[si * W + (bw - 1 - ii)];
      const double lk = win[sk * W + (bw - 1 - kk)];
      win[si * W + (kk - ii + bw)] -= li * lk;
    }
    // row j is final (its slot is not touched by the update above): write it
    // out and bring in row j + W
    for (int d = tid; d < W; d += blockDim.x) {
      G[band_at(j, d, ld)] = d == bw ? ljj : win[sj * W + d];
      const int nr = j + W;
      const double v = nr < m ? G[band_at(nr, d, ld)] : 0.0;
      win[sj * W + d] = v;
      if (d == bw) gd[sj] = nr < m ? v : 1.0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- finish
// Reversed transpose R[p][d] = L[m-1-p+bw-d][d] (zero outside the matrix and
// for d >= bw), 1/L_pp, and the FP32 copies (diagonal zero).  Grid: (tiles,
// blocks).  k_band_zero_diag then clears the diagonal of the FP64 factor, so
// that every copy the sweeps read has a zero diagonal.
__global__ void __launch_bounds__(256)
k_band_finish(BandBlocks B, int mixed) {
  const int blk = blockIdx.y;
  const int m = B.m[blk], bw = B.bw[blk], ld = B.ld[blk], row0 = B.row0[blk];
  const int nt = (m + 63) >> 6;
  const long long off = B.off[blk];
  const double* L = B.L + off;
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    for (int e = threadIdx.x; e < 64 * ld; e += blockDim.x) {
      const int d = e >> 6, p = t * 64 + (e & 63);
      const long long at = band_at(p, d, ld);
      double r = 0.0;
      const int k = p - bw + d;          // column of R, reversed row of L
      const int src = m - 1 - k;         // row of L holding R[p][k]
      if (d < bw && p < m && k >= 0 && src < m) r = L[band_at(src, d, ld)];
      // the sweeps take 1/L_pp from dinv; their copies keep a zero diagonal
      if (mixed) {
        B.L32[off + at] = d == bw ? 0.f : (float)L[at];
        B.R32[off + at] = (float)r;
      } else {
        B.R[off + at] = r;
      }
      if (d == bw && p < m) {
        const double iv = 1.0 / L[at];
        B.dinv[row0 + p] = iv;
        if (mixed) B.dinv32[row0 + p] = (float)iv;
      }
    }
  }
}

__global__ void __launch_bounds__(256)
k_band_zero_diag(BandBlocks B) {
  const int blk = blockIdx.y;
  const int m = B.m[blk], bw = B.bw[blk], ld = B.ld[blk];
  double* L = B.L + B.off[blk];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < m; p += gridDim.x * blockDim.x)
    L[band_at(p, bw, ld)] = 0.0;
}

// ----------------------------------------------------------------- apply
template <typename T>
__device__ __forceinline__ T lane_bcast(T v, int lane);
template <>
__device__ __forceinline__ float lane_bcast<float>(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
template <>
__device__ __forceinline__ double lane_bcast<double>(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The computation of one tile of a sweep for lane l (row p) and NR vectors
// (window q at yw + 256 q): the off-tile part against the window, then the
// in-tile column sweep; leaves w_p of each vector in acc.  The band entries
// are read once for the NR vectors, whose independent broadcast-and-FMA
// chains of the column sweep interleave.
// The window slots of the tile's rows are zero (they held rows 256 back, no
// longer referenced) and slots of rows below 0 are zero from the start of the
// sweep, so in-tile and out-of-matrix columns contribute nothing and the
// batches of 8 need no mask; only the tail batch is masked.  All LDS reads
// of a batch are issued before its arithmetic.  In the column sweep, entries
// outside the band of row p (including j >= l) are read from the zero
// diagonal slot, so a step is a multiply, a broadcast and an FMA; lane l's
// value stops changing after step l, and rows past m have a zero pivot
// reciprocal.
template <typename T, int NR>
__device__ __forceinline__ void band_tile(const T* buf, const T* yw, T (&acc)[NR], T dp, int p,
                                          int l, int bw, int ld) {
  // The entry indices of the column sweep are the same for every tile; an
  // opaque copy of the lane index keeps the compiler from holding all 64 of
  // them in registers across the tile loop (recomputing them is cheap).
  asm volatile("" : "+v"(l));
  const int kb = p - bw;
  int d0 = 0;
  for (; d0 + 8 <= bw; d0 += 8) {
    T v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = buf[(d0 + i) * 64 + l];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      T yk[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) yk[i] = yw[q * 256 + ((kb + d0 + i) & 255)];
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[q] -= v[i] * yk[i];
    }
  }
  if (d0 < bw) {
    T v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = buf[min(d0 + i, ld - 1) * 64 + l];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      T yk[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) yk[i] = yw[q * 256 + ((kb + d0 + i) & 255)];
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[q] -= (d0 + i < bw) ? v[i] * yk[i] : (T)0;
    }
  }
#pragma unroll
  for (int j0 = 0; j0 < 64; j0 += 8) {
    T e[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int dd = bw - l + j0 + i;  // entry of row p for column i0 + j
      e[i] = buf[((unsigned)dd <= (unsigned)bw ? dd : bw) * 64 + l];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const T s = lane_bcast<T>(acc[q] * dp, j0 + i);
        acc[q] -= e[i] * s;
      }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) acc[q] *= dp;
}

// One wave per block; lane l owns row p = i0 + l of the current 64-row tile.
// The tiles of the forward sweep (factor L, right-hand side D u) and then of
// the backward sweep (factor R, right-hand side the reversed forward result)
// are processed in one sequence.  The band of a tile (64*ld contiguous
// values) and its right-hand side are loaded two tiles ahead into one of two
// named register sets and written to the (single) LDS stage at the end of the
// tile before their use, so each load has two tiles of compute to arrive
// (the first two backward tiles need the forward result and load their
// right-hand side after the forward sweep instead).  Per tile: the off-tile
// part acc -= sum_{k < i0} F[p][k] w[k] reads the stage against the solved
// values kept in a 256-entry circular window (bw <= BAND_MAX < 192, so rows
// i0-bw..i0-1 are all still there); the in-tile triangle is a column sweep:
// at step j, w_j = acc_j / F_jj is broadcast from lane j and the lanes below
// it subtract F[p][i0+j] w_j.

// Ordering point for the one-wave workgroup of k_band_apply: LDS operations
// of a wave execute in program order, so a compiler barrier with
// wavefront-scope fences orders the lanes' LDS accesses without the
// memory-counter waits of a workgroup barrier (which would also wait for the
// prefetch loads in flight and for the global stores of the last tile).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define BC_LIST(M, S)                                                                   \
  M(S, 0) M(S, 1) M(S, 2) M(S, 3) M(S, 4) M(S, 5) M(S, 6) M(S, 7) M(S, 8) M(S, 9)        \
  M(S, 10) M(S, 11) M(S, 12) M(S, 13) M(S, 14) M(S, 15) M(S, 16) M(S, 17) M(S, 18)       \
  M(S, 19) M(S, 20) M(S, 21) M(S, 22) M(S, 23) M(S, 24) M(S, 25) M(S, 26) M(S, 27)       \
  M(S, 28) M(S, 29) M(S, 30) M(S, 31)
#define BC_DECL(S, q) float4 S##q;
// vectors q >= npre re-read / re-write vector 0 (in bounds, idempotent), so
// the loads and stores of a set carry no predicate
#define BC_LOAD(S, q) if constexpr (NVP > q) S##q = src_[((q) < npre ? (q) : 0) * 64 + l];
#define BC_STORE(S, q) if constexpr (NVP > q) dst_[((q) < npre ? (q) : 0) * 64 + l] = S##q;

template <typename T, int NVP, int NR>
__global__ void __launch_bounds__(64)
k_band_apply(BandBlocks B, const double* __restrict__ u, double* __restrict__ y,
             const int* __restrict__ done, int nrhs, int n1, int sys_done) {
  extern __shared__ float4 lds4[];
  const int blk = blockIdx.x;
  // vectors j0 .. j0 + NR - 1 of the nrhs at offsets j * n1; sys_done: one
  // vector of a batch of systems, stopped with the block's system
  const int j0 = blockIdx.y * NR;
  if (sys_done && done && done[B.sys[blk]]) return;
  bool act[NR];
  bool any = false;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    act[q] = j0 + q < nrhs && !(!sys_done && done && done[j0 + q]);
    any = any || act[q];
  }
  if (!any) return;
  const int m = B.m[blk], bw = B.bw[blk], ld = B.ld[blk], row0 = B.row0[blk];
  const int nt = (m + 63) >> 6;
  const int l = threadIdx.x;
  T* stage = (T*)lds4;                         // band of the current tile, 64*ld
  T* yw = stage + 64 * B.ldmax;                // solved values, circular, 256 per vector
  double* ra = (double*)(yw + 256 * NR);       // staged right-hand sides of the tile, 64 per vector
  double* rs = ra + 64 * NR;                   // staged output scale
  T* rd = (T*)(rs + 64);                       // staged pivot reciprocal
  constexpr int VT = 16 / (int)sizeof(T);
  const int nv = ld / VT;          // 16-byte vectors per lane per tile
  const int npre = min(nv, NVP);   // of which prefetched
  if (l == 0) atomicAdd(&B.applies[blk], 1ull);
  const T* Fl;
  const T* Fr;
  const T* dv;
  if constexpr (sizeof(T) == 8) {
    Fl = (const T*)(B.L + B.off[blk]);
    Fr = (const T*)(B.R + B.off[blk]);
    dv = (const T*)(B.dinv + row0);
  } else {
    Fl = (const T*)(B.L32 + B.off[blk]);
    Fr = (const T*)(B.R32 + B.off[blk]);
    dv = (const T*)(B.dinv32 + row0);
  }
  const double* dsc = B.dsc + row0;
  const int total = 2 * nt;
  // vector q's right-hand side and output (vectors past nrhs read vector j0;
  // inactive vectors write nothing)
  auto ub = [&](int q) -> const double* {
    return u + (size_t)(j0 + q < nrhs ? j0 + q : j0) * n1 + row0;
  };
  auto yb = [&](int q) -> double* { return y + (size_t)(j0 + q < nrhs ? j0 + q : j0) * n1 + row0; };
  // band of tile idx (clamped into the sequence, so any idx is in bounds)
  auto chunk = [&](int idx) -> const float4* {
    idx = min(idx, total - 1);
    const bool bwd = idx >= nt;
    const int t = bwd ? idx - nt : idx;
    return (const float4*)((bwd ? Fr : Fl) + (long long)t * 64 * ld);
  };
  // row whose right-hand side, output scale and pivot lane l loads for tile
  // idx, clamped into the block so the loads carry no predicate
  auto rhs_row = [&](int idx) -> int {
    idx = min(idx, total - 1);
    const int bwd = idx >= nt;
    const int pc = min((bwd ? idx - nt : idx) * 64 + l, m - 1);
    return bwd ? m - 1 - pc : pc;
  };
  auto rhs_src = [&](int idx, int q, int r) -> const double* {
    return min(idx, total - 1) >= nt ? yb(q) + r : ub(q) + r;
  };
  // prologue: tile 0 staged, tile 1 in set A
  {
    const float4* src = chunk(0);
    float4* dst = (float4*)stage;
    for (int q = 0; q < nv; ++q) dst[q * 64 + l] = src[q * 64 + l];
    const int r = rhs_row(0);
#pragma unroll
    for (int q = 0; q < NR; ++q) ra[q * 64 + l] = ub(q)[r] * dsc[r];
    rd[l] = dv[r];
  }
  BC_LIST(BC_DECL, pa)
  BC_LIST(BC_DECL, pb)
  double xa_a[NR], xb_a[NR], xa_s, xb_s;
  T xa_d, xb_d;
  {
    const int r = rhs_row(1);
#pragma unroll
    for (int q = 0; q < NR; ++q) xa_a[q] = *rhs_src(1, q, r);
    xa_s = dsc[r];
    xa_d = dv[r];
    const float4* src_ = chunk(1);
    BC_LIST(BC_LOAD, pa)
  }
  wave_sync();

  // One tile: CUR holds tile idx+1 (loaded one tile ago), NXT receives tile
  // idx+2.
#define BC_TILE(CUR, XC, NXT, XN)                                                         \
  {                                                                                      \
    const bool bwd = idx >= nt;                                                          \
    const int t = bwd ? idx - nt : idx;                                                  \
    const int i0 = t * 64, p = i0 + l;                                                   \
    if (idx == nt || idx == nt + 1) {                                                    \
      /* the first backward tiles start from the forward result of all lanes */         \
      if (idx == nt) {                                                                   \
        __threadfence_block();                                                           \
        __syncthreads();                                                                 \
      }                                                                                  \
      const int r = rhs_row(idx);                                                        \
      _Pragma("unroll") for (int q = 0; q < NR; ++q) ra[q * 64 + l] = yb(q)[r];          \
      rs[l] = dsc[r];                                                                    \
      rd[l] = dv[r];                                                                     \
    }                                                                                    \
    if (t == 0) {                                                                        \
      _Pragma("unroll") for (int q = 0; q < 4 * NR; ++q) yw[q * 64 + l] = (T)0;          \
    }                                                                                    \
    _Pragma("unroll") for (int q = 0; q < NR; ++q) yw[q * 256 + (p & 255)] = (T)0;       \
    wave_sync();                                                                         \
    T acc[NR];                                                                           \
    _Pragma("unroll") for (int q = 0; q < NR; ++q) acc[q] = p < m ? (T)ra[q * 64 + l] : (T)0; \
    const T dp = p < m ? rd[l] : (T)0;                                                   \
    const double sc = rs[l];                                                             \
    /* prefetch tile idx+2: right-hand side first, then band */                         \
    {                                                                                    \
      const int r = rhs_row(idx + 2);                                                    \
      _Pragma("unroll") for (int q = 0; q < NR; ++q) XN##_a[q] = *rhs_src(idx + 2, q, r); \
      XN##_s = dsc[r];                                                                   \
      XN##_d = dv[r];                                                                    \
      const float4* src_ = chunk(idx + 2);                                               \
      BC_LIST(BC_LOAD, NXT)                                                              \
    }                                                                                    \
    band_tile<T, NR>(stage, yw, acc, dp, p, l, bw, ld);                                  \
    wave_sync(); /* every lane is done with the stage and the window */                 \
    _Pragma("unroll") for (int q = 0; q < NR; ++q) yw[q * 256 + (p & 255)] = acc[q];     \
    if (idx + 1 < total) {                                                               \
      /* stage tile idx+1 (the one wait for HBM per tile) */                            \
      float4* dst_ = (float4*)stage;                                                     \
      BC_LIST(BC_STORE, CUR)                                                             \
      const float4* nsrc = chunk(idx + 1);                                               \
      for (int q = npre; q < nv; ++q) dst_[q * 64 + l] = nsrc[q * 64 + l];               \
      _Pragma("unroll") for (int q = 0; q < NR; ++q)                                     \
        ra[q * 64 + l] = (idx + 1 >= nt) ? XC##_a[q] : XC##_a[q] * XC##_s;              \
      rs[l] = XC##_s;                                                                    \
      rd[l] = XC##_d;                                                                    \
    }                                                                                    \
    if (p < m) {                                                                         \
      _Pragma("unroll") for (int q = 0; q < NR; ++q) {                                   \
        if (act[q]) {                                                                    \
          if (!bwd) yb(q)[p] = (double)acc[q];                                           \
          else yb(q)[m - 1 - p] = (double)acc[q] * sc;                                   \
        }                                                                                \
      }                                                                                  \
    }                                                                                    \
    wave_sync();                                                                         \
  }

  for (int idx = 0; idx < total; ++idx) {
    BC_TILE(pa, xa, pb, xb)
    if (++idx >= total) break;
    BC_TILE(pb, xb, pa, xa)
  }
#undef BC_TILE
}
#undef BC_LIST
#undef BC_DECL
#undef BC_LOAD
#undef BC_STORE

// Compute units of the current device (read once).
int device_cus() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    return n;
  }();
  return cus;
}

// Dynamic LDS of the sweep for NR vectors: stage, NR windows, NR staged
// right-hand sides, output scales and pivot reciprocals.
template <typename T>
size_t band_apply_lds(const BandBlocks& B, int nr) {
  return (size_t)(64 * B.ldmax + 256 * nr) * sizeof(T) + 64 * nr * sizeof(double) +
         64 * (sizeof(double) + sizeof(T));
}

template <typename T, int NR>
hipError_t launch_apply_nr(hipStream_t st, const BandBlocks& B, const double* u, double* y,
                           const int* done, int nrhs, int n1, int sys_done, int nvp) {
  const size_t lds = band_apply_lds<T>(B, NR);
  const dim3 grid(B.nblk, (nrhs + NR - 1) / NR);
#define BC_LAUNCH(V)                                                                       \
  hipLaunchKernelGGL((k_band_apply<T, V, NR>), grid, dim3(64), lds, st, B, u, y, done, nrhs, \
                     n1, sys_done)
  if constexpr (NR == 1) {
    if (nvp == 4) BC_LAUNCH(4);
    else if (nvp == 8) BC_LAUNCH(8);
    else if (nvp == 12) BC_LAUNCH(12);
    else if (nvp == 20) BC_LAUNCH(20);
    else if (nvp == 16) BC_LAUNCH(16);
    else if (nvp == 24) BC_LAUNCH(24);
    else BC_LAUNCH(32);
  } else {
    // the multi-vector sweeps use register sets of at most BAND_MULTI_NVP
    if (nvp <= 4) BC_LAUNCH(4);
    else if (nvp <= 8) BC_LAUNCH(8);
    else BC_LAUNCH(BAND_MULTI_NVP);
  }
#undef BC_LAUNCH
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_t(hipStream_t st, const BandBlocks& B, const double* u, double* y,
                          const int* done, int nrhs, int n1, int sys_done) {
  const int nvp = B.nvp > 0 ? B.nvp : band_nvp_buckets(B, sizeof(T)).back();
  if (nrhs == 1) return launch_apply_nr<T, 1>(st, B, u, y, done, nrhs, n1, sys_done, nvp);
  // Several vectors: one wave per block and chunk of 1, 4 or 8 vectors.  A
  // wave is bound by the latency of its column sweeps, and a second wave on
  // a SIMD slows both about as much as running after it, so the time is
  // about (rounds of one wave per SIMD) x (the chunk's cost), the chunks of
  // 1, 4 and 8 vectors costing about 1 : 2.6 : 3.7 (measured on the 27-point
  // 100^3 blocks).  The cheapest is taken (the narrower on a tie).
  const long long simds = 4LL * device_cus();
  auto cost = [&](int nr, double w) {
    const long long waves = (long long)B.nblk * ((nrhs + nr - 1) / nr);
    return (double)((waves + simds - 1) / simds) * w;
  };
  const double c1 = cost(1, 1.0), c4 = cost(4, 2.6), c8 = cost(8, 3.7);
  if (c1 <= c4 && c1 <= c8) return launch_apply_nr<T, 1>(st, B, u, y, done, nrhs, n1, sys_done, nvp);
  if (c4 <= c8) return launch_apply_nr<T, 4>(st, B, u, y, done, nrhs, n1, sys_done, nvp);
  return launch_apply_nr<T, 8>(st, B, u, y, done, nrhs, n1, sys_done, nvp);
}

}  // namespace

hipError_t launch_band_gram(hipStream_t st, const BandBlocks& B, const int* rowptr, const int* col,
                            const double* val, const int* tptr, const int* trow, const double* tval) {
  if (B.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_gram, dim3(B.nblk), dim3(256), 0, st, B, rowptr, col, val, tptr, trow,
                     tval);
  return hipGetLastError();
}

hipError_t launch_band_cholesky(hipStream_t st, const BandBlocks& B) {
  if (B.nblk == 0) return hipSuccess;
  const size_t lds = (size_t)(BAND_MAX + 1) * (BAND_MAX + 2) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)k_band_chol,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_chol, dim3(B.nblk), dim3(256), lds, st, B);
  return hipGetLastError();
}

hipError_t launch_band_finish(hipStream_t st, const BandBlocks& B, bool mixed) {
  if (B.nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_finish, dim3(32, B.nblk), dim3(256), 0, st, B, (int)mixed);
  if (!mixed) hipLaunchKernelGGL(k_band_zero_diag, dim3(4, B.nblk), dim3(256), 0, st, B);
  return hipGetLastError();
}

// Register-set sizes (16-byte vectors per lane and tile) worth trying for
// these blocks: every instantiated size up to the first one that holds a
// whole tile of the widest band.
std::vector<int> band_nvp_buckets(const BandBlocks& B, size_t elem) {
  static const int sizes[] = {4, 8, 12, 16, 20, 24, 32};
  const int nvmax = B.ldmax * (int)elem / 16;
  std::vector<int> out;
  for (int v : sizes) {
    out.push_back(v);
    if (v >= nvmax) break;
  }
  return out;
}

// Raises the dynamic LDS limit of every sweep instantiation to what the
// widest band needs (set once at setup, so that a launch inside a stream
// capture is a plain kernel launch).
template <typename T>
hipError_t prepare_apply_t(const BandBlocks& B) {
  const int l1 = (int)band_apply_lds<T>(B, 1), l4 = (int)band_apply_lds<T>(B, 4);
  const int l8 = (int)band_apply_lds<T>(B, 8);
  const std::pair<const void*, int> fns[] = {
      {(const void*)k_band_apply<T, 4, 1>, l1},  {(const void*)k_band_apply<T, 8, 1>, l1},
      {(const void*)k_band_apply<T, 12, 1>, l1}, {(const void*)k_band_apply<T, 16, 1>, l1},
      {(const void*)k_band_apply<T, 20, 1>, l1}, {(const void*)k_band_apply<T, 24, 1>, l1},
      {(const void*)k_band_apply<T, 32, 1>, l1}, {(const void*)k_band_apply<T, 4, 4>, l4},
      {(const void*)k_band_apply<T, 8, 4>, l4},  {(const void*)k_band_apply<T, 12, 4>, l4},
      {(const void*)k_band_apply<T, 4, 8>, l8},  {(const void*)k_band_apply<T, 8, 8>, l8},
      {(const void*)k_band_apply<T, 12, 8>, l8}};
  for (const auto& f : fns) {
    hipError_t e = hipFuncSetAttribute(f.first, hipFuncAttributeMaxDynamicSharedMemorySize, f.second);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t prepare_band_apply(const BandBlocks& B, bool mixed) {
  if (B.nblk == 0) return hipSuccess;
  return mixed ? prepare_apply_t<float>(B) : prepare_apply_t<double>(B);
}

hipError_t launch_band_apply(hipStream_t st, const BandBlocks& B, bool mixed, const double* u,
                             double* y, const int* done) {
  if (B.nblk == 0) return hipSuccess;
  return mixed ? launch_apply_t<float>(st, B, u, y, done, 1, 0, 1)
               : launch_apply_t<double>(st, B, u, y, done, 1, 0, 1);
}

hipError_t launch_band_apply_multi(hipStream_t st, const BandBlocks& B, bool mixed,
                                   const double* u, double* y, const int* done, int nrhs, int n1) {
  if (B.nblk == 0 || nrhs <= 0) return hipSuccess;
  return mixed ? launch_apply_t<float>(st, B, u, y, done, nrhs, n1, 0)
               : launch_apply_t<double>(st, B, u, y, done, nrhs, n1, 0);
}

std::vector<int> band_apply_candidates(const BandBlocks& B, bool mixed) {
  return band_nvp_buckets(B, mixed ? sizeof(float) : sizeof(double));
}
