// Banded Cholesky projections.
//
// For a block whose rows are in reverse Cuthill-McKee order, the scaled
// normal-equation matrix G = D A_i A_i^T D (D = unit-row scaling; Section 1,
// eq. (H): y_i = (A_i A_i^T)^{-1} u_i) is banded with a small half-bandwidth
// bw, and so is its Cholesky factor (a banded matrix factors without fill
// outside its band).  Setup forms G in the band storage (k_band_gram),
// factors it in FP64 in place (k_band_chol) and writes the factor and its
// reversed transpose in the slot layout of the sweeps (k_band_slots), FP64 or
// rounded once to FP32.  Each projection then runs two banded triangular
// sweeps (k_band_sweep): L z = D u and L^T w = z, y = D w.
//
// Band storage (see BandBlocks): per 64-row tile, diagonal-major, entry d of
// local row p at tile*64*ld + d*64 + p%64, column p - bw + d (ld = bw+1
// rounded up to a multiple of 4).  Lanes of a wave own consecutive rows, so
// every access is coalesced, and a tile is one contiguous chunk.
#include "common.h"

#include <cmath>
#include <utility>
#include <vector>

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

// ------------------------------------------------------------ slot layout
// The sweeps read each factor F (L, or its reversed transpose R) in a slot
// layout.  A 64-row tile is cut into sub-tiles of q rows, q the largest power
// of two with q <= min(ld, 64) (q = 64 once bw >= 63).  Slot s of local row p
// (lane l = p % 64, l' = l % q) holds the coefficient of the value of row
// p - s:
//   s <= l':  X[l'][l'-s], X the inverse of the sub-tile's lower-triangular
//             q x q diagonal block of F (rows past m: X = I);
//   s >  l':  F[p][p-s], an entry left of the sub-tile (zero outside the band).
// One sub-tile of the sweep F z = b is then
//   a_p = b_p - sum_{s > l'} F[p][p-s] z_{p-s}   (rows already solved)
//   z_p = sum_{s <= l'} X[l'][l'-s] a_{p-s}       (the sub-tile's block inverse)
// and both are the same loop over slots against values indexed by p - s.  In
// the band layout row p keeps l'+1 entries of F inside its sub-tile (diagonal
// included); in the slot layout it keeps the l'+1 entries of row l' of X, so
// the two layouts hold the same number of entries (q <= ld keeps every entry
// of X inside the row's ld slots).
//
// Slots are grouped in 16-byte vectors of VT = 16 / sizeof(element) slots:
// slot s of lane l sits at tile*64*ld + (s/VT)*64*VT + l*VT + s%VT, so a wave
// loads VT slots of its 64 rows with one coalesced 1 KiB access.
//
// Reversed transpose: R[p][k] = L[m-1-k][m-1-p], so the backward sweep
// L^T w = z is the forward sweep R w' = z' on reversed vectors.

// Sub-tile height of a block's sweeps.
__device__ __forceinline__ int band_subtile(int ld) {
  int q = 64;
  while (q > ld) q >>= 1;
  return q;
}

// One 64-thread workgroup per (tile, block, factor): the tile's block-diagonal
// of sub-tile blocks is inverted in FP64 by forward substitution, one column
// per thread, and every slot of the tile is written (FP64, or rounded once to
// FP32).
template <typename TF>
__global__ void __launch_bounds__(64)
k_band_slots(BandBlocks B, TF* __restrict__ outL, TF* __restrict__ outR) {
  __shared__ double Tb[64][65];
  __shared__ double Xb[64][65];
  const int blk = blockIdx.y, rev = blockIdx.z;
  const int m = B.m[blk], bw = B.bw[blk], ld = B.ld[blk], sld = B.sld[blk];
  const int nt = (m + 63) >> 6;
  const double* L = B.L + B.off[blk];
  TF* out = (rev ? outR : outL) + B.soff[blk];
  const int l = threadIdx.x, q = band_subtile(sld);
  for (int t = blockIdx.x; t < nt; t += gridDim.x) {
    const int i0 = t * 64;
    // row l of the block diagonal of sub-tile blocks
    for (int b = 0; b < 64; ++b) {
      double v = 0.0;
      if (i0 + l >= m) {
        v = l == b ? 1.0 : 0.0;
      } else if (b <= l && l - b <= bw && l / q == b / q) {
        v = rev ? L[band_at(m - 1 - i0 - b, bw - (l - b), ld)] : L[band_at(i0 + l, bw - (l - b), ld)];
      }
      Tb[l][b] = v;
    }
    __syncthreads();
    // column l of X: T x = e_l
    double x[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      double s = i == l ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) s -= Tb[i][k] * x[k];
      x[i] = s / Tb[i][i];
    }
#pragma unroll
    for (int i = 0; i < 64; ++i) Xb[i][l] = x[i];
    __syncthreads();
    const int p = i0 + l;
    constexpr int VT = 16 / (int)sizeof(TF);
    TF* o = out + (long long)t * 64 * sld + l * VT;
    for (int s = 0; s < sld; ++s) {
      double v = 0.0;
      if (s <= l % q) {
        v = Xb[l][l - s];
      } else if (p < m && s <= bw && p - s >= 0) {
        v = rev ? L[band_at(m - 1 - p + s, bw - s, ld)] : L[band_at(p, bw - s, ld)];
      }
      o[(s / VT) * 64 * VT + s % VT] = (TF)v;
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- apply
// k_band_sweep: one workgroup of four waves per block (and chunk of NR
// vectors); lane l owns row p = i0 + l of the current tile, and wave w owns
// the slot vectors 4i + w (i < NV).  Per sub-tile, with the waves' partial
// sums exchanged through LDS:
//   phase 1: each wave sums its slots against its window of solved values
//            (z of rows p - s; rows of the tile not yet solved read 0);
//            barrier; every wave forms a = b - (sum of the four partials), in
//            wave order, on the sub-tile's rows (0 elsewhere);
//   phase 2: each wave sums its slots s < q against [0 x 64 | a] (a of row
//            p - s, zero outside the sub-tile); barrier; every wave forms z,
//            in wave order, and writes the sub-tile's rows to its own window;
//            wave 0 stores them.
// Every wave thus holds the same z, and the only cross-wave traffic is the
// two partial-sum exchanges.  The window keeps each value twice, 256 rows
// apart, so that the reads of rows p - s need no wrap-around.  The slots and
// right-hand sides of the next tiles are loaded into registers while tile t
// is computed (register sets in rotation, issued in tile order).  The
// forward sweep (slots of L,
// right-hand side D u) and the backward sweep (slots of R, right-hand side
// the reversed forward result, output scaled by D) run one after the other.
// Blocks are taken in decreasing order of work (B.order), so the long chains
// of the largest blocks start first.
constexpr int SWEEP_WAVES = 4;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename TF, int NV, int NR>
struct SweepSet {
  TF cf[NV * (16 / sizeof(TF))];
  double ra[NR];
  double sc;
};

// Barrier that orders only LDS: the global loads of the prefetch stay in
// flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Ordering point for one wave's own LDS accesses (LDS operations of a wave
// execute in program order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename TA>
constexpr size_t sweep_lds(int nr) {
  // per wave and vector: window 2 x 256 + [zeros | a] 128; per vector and wave: two partials 64
  return (size_t)SWEEP_WAVES * nr * (512 + 128 + 2 * 64) * sizeof(TA);
}

// The tiles of one sweep (BWD: the backward sweep, slots of R, right-hand
// side the reversed forward result, output scaled by D).
template <bool BWD, typename TF, typename TA, int NV, int NR>
__device__ __forceinline__ void band_sweep_run(const TF* __restrict__ F0, const double* __restrict__ dsc,
                                               const double* const (&src)[NR], double* const (&dst)[NR],
                                               const bool (&act)[NR], TA* win, TA* za, TA* p1, TA* p2,
                                               int m, int ld, int w, int l) {
  constexpr int VT = 16 / (int)sizeof(TF);
  constexpr int SMAX = 4 * NV * VT;  // bound of the slots a wave holds
  constexpr int GI = 4;  // one vector: slot vectors whose LDS reads issue together
  const int nt = (m + 63) >> 6;
  const int qh = band_subtile(ld), qlog = __builtin_ctz(qh), nsub = 64 >> qlog;
  using Set = SweepSet<TF, NV, NR>;
  auto load = [&](Set& S, int t) {
    // A buffer resource over exactly the tile's slots: vectors past its ld
    // are out of range and read as zero, so every wave multiplies all NV of
    // its vectors, in and past the block's band alike, with no mask.  A tile
    // past the last one has an empty range (its set is never used).
    const int nrec = t < nt ? 64 * ld * (int)sizeof(TF) : 0;
    t = min(t, nt - 1);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(F0 + (long long)t * 64 * ld), (short)0, nrec, 0x00020000);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (w * 64 + l) * 16, i * 4096, 0);
      __builtin_memcpy(&S.cf[i * VT], &v, 16);
    }
    const int pc = min(t * 64 + l, m - 1);
    const int r = BWD ? m - 1 - pc : pc;
#pragma unroll
    for (int q = 0; q < NR; ++q) S.ra[q] = src[q][r];
    S.sc = dsc[r];
    // The sets are issued in tile order and never reordered: the compiler's
    // wait counts take a set as complete only once every set issued before
    // it is, so a later set issued first would make every tile wait for the
    // set of the tile after it.
    __builtin_amdgcn_sched_barrier(0);
  };
  // one sub-tile: the rows with mine set take a and z (q = 64: every row)
  auto substep = [&](const Set& S, const TA (&b)[NR], TA (&zp)[NR], int p, bool mine) {
    wave_sync();
    // phase 1: this wave's slots against the solved values; win1 points at
    // row p - SMAX of the doubled window
    const TA* win1 = win + (p & 255) + 256 - SMAX;
    TA part[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) part[q] = (TA)0;
    // (the reads of a group of GI vectors are issued together, then
    // multiplied in slot order)
    if constexpr (NR == 1) {
#pragma unroll
      for (int g = 0; g < NV; g += GI) {
        TA wv[GI * VT][NR];
#pragma unroll
        for (int i = g; i < g + GI && i < NV; ++i)
#pragma unroll
          for (int e = 0; e < VT; ++e)
#pragma unroll
            for (int q = 0; q < NR; ++q)
              wv[(i - g) * VT + e][q] = win1[q * 512 + SMAX - ((4 * i + w) * VT + e)];
#pragma unroll
        for (int i = g; i < g + GI && i < NV; ++i)
#pragma unroll
          for (int e = 0; e < VT; ++e)
#pragma unroll
            for (int q = 0; q < NR; ++q) part[q] += (TA)S.cf[i * VT + e] * wv[(i - g) * VT + e][q];
      }
    } else {
      // several vectors: the NR values of one slot at a time (NR independent sums)
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int e = 0; e < VT; ++e) {
          TA wv[NR];
#pragma unroll
          for (int q = 0; q < NR; ++q) wv[q] = win1[q * 512 + SMAX - ((4 * i + w) * VT + e)];
          const TA c = (TA)S.cf[i * VT + e];
#pragma unroll
          for (int q = 0; q < NR; ++q) part[q] += c * wv[q];
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) p1[(w * NR + q) * 64 + l] = part[q];
    lds_barrier();
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const TA* P = p1 + q * 64 + l;
      const TA sum = ((P[0] + P[NR * 64]) + P[2 * NR * 64]) + P[3 * NR * 64];
      za[q * 128 + 64 + l] = mine && p < m ? b[q] - sum : (TA)0;
    }
    wave_sync();
    // phase 2: this wave's slots inside the sub-tile against a
#pragma unroll
    for (int q = 0; q < NR; ++q) part[q] = (TA)0;
    // (vectors i < 16 / VT hold every slot below 64; a slot at or past q
    // reads a row before the sub-tile, which is 0 in [0 x 64 | a])
    constexpr int NV2 = NV < 16 / VT ? NV : 16 / VT;
    if constexpr (NR == 1) {
#pragma unroll
      for (int g = 0; g < NV2; g += GI) {
        TA wv[GI * VT][NR];
#pragma unroll
        for (int i = g; i < g + GI && i < NV2; ++i)
#pragma unroll
          for (int e = 0; e < VT; ++e)
#pragma unroll
            for (int q = 0; q < NR; ++q)
              wv[(i - g) * VT + e][q] = za[q * 128 + 64 + l - ((4 * i + w) * VT + e)];
#pragma unroll
        for (int i = g; i < g + GI && i < NV2; ++i)
#pragma unroll
          for (int e = 0; e < VT; ++e)
#pragma unroll
            for (int q = 0; q < NR; ++q) part[q] += (TA)S.cf[i * VT + e] * wv[(i - g) * VT + e][q];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NV2; ++i)
#pragma unroll
        for (int e = 0; e < VT; ++e) {
          TA wv[NR];
#pragma unroll
          for (int q = 0; q < NR; ++q) wv[q] = za[q * 128 + 64 + l - ((4 * i + w) * VT + e)];
          const TA c = (TA)S.cf[i * VT + e];
#pragma unroll
          for (int q = 0; q < NR; ++q) part[q] += c * wv[q];
        }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) p2[(w * NR + q) * 64 + l] = part[q];
    lds_barrier();
    if (mine) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const TA* P = p2 + q * 64 + l;
        zp[q] = ((P[0] + P[NR * 64]) + P[2 * NR * 64]) + P[3 * NR * 64];
        win[q * 512 + (p & 255)] = zp[q];
        win[q * 512 + (p & 255) + 256] = zp[q];
      }
    }
  };
  auto tile = [&](int t, const Set& S) {
    const int p = t * 64 + l;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      win[q * 512 + (p & 255)] = (TA)0;
      win[q * 512 + (p & 255) + 256] = (TA)0;
    }
    TA b[NR], zp[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) b[q] = BWD ? (TA)S.ra[q] : (TA)(S.ra[q] * S.sc);
    // The first sub-tile is outside the loop, so every path through the tile
    // has used the set; the loop holds no global store (a loop with stores
    // and no loads makes the compiler wait for every load in flight, the
    // prefetch included, before entering it).
    substep(S, b, zp, p, (l >> qlog) == 0);
    for (int k = 1; k < nsub; ++k) substep(S, b, zp, p, (l >> qlog) == k);
    if (w == 0 && p < m) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (act[q]) {
          if (!BWD) dst[q][p] = (double)zp[q];
          else dst[q][m - 1 - p] = (double)zp[q] * S.sc;
        }
      }
    }
  };
  // rows before the first tile read 0
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int k = 0; k < 8; ++k) win[q * 512 + k * 64 + l] = (TA)0;
  // One vector: three register sets in rotation, tile t computed while the
  // sets of tiles t+1 and t+2 are in flight.  Several vectors (larger sets):
  // two, so that the wide bands fit the registers without spilling.
  if constexpr (NR == 1) {
    Set S0, S1, S2;
    load(S0, 0);
    load(S1, 1);
    for (int t = 0; t < nt; t += 3) {
      load(S2, t + 2);
      tile(t, S0);
      if (t + 1 >= nt) break;
      load(S0, t + 3);
      tile(t + 1, S1);
      if (t + 2 >= nt) break;
      load(S1, t + 4);
      tile(t + 2, S2);
    }
  } else {
    Set S0, S1;
    load(S0, 0);
    for (int t = 0; t < nt; t += 2) {
      load(S1, t + 1);
      tile(t, S0);
      if (t + 1 >= nt) break;
      load(S0, t + 2);
      tile(t + 1, S1);
    }
  }
}

// The sweep bodies inside one kernel: a block whose band needs fewer slot
// vectors per wave (nvb) than the kernel's NV runs the smallest body from
// about NV/3, NV/2, 2NV/3 and NV that holds it, so narrow bands do not load
// and multiply the zero slots of the widest one.  The sums are the same bits
// either way: a slot past a block's band only adds zero products, in the same
// wave and order.  (The chunks of several vectors keep the one body.)
template <int NV, int K>
constexpr int body_nv() {
  return K == 0 ? (NV + 2) / 3 : K == 1 ? (NV + 1) / 2 : K == 2 ? (2 * NV + 2) / 3 : NV;
}

template <bool BWD, typename TF, typename TA, int NV, int NR, int K = 0>
__device__ __forceinline__ void sweep_body(int nvb, const TF* __restrict__ F0,
                                           const double* __restrict__ dsc,
                                           const double* const (&src)[NR],
                                           double* const (&dst)[NR], const bool (&act)[NR],
                                           TA* win, TA* za, TA* p1, TA* p2, int m, int ld, int w,
                                           int l) {
  if constexpr (K < 3 && NR == 1) {
    constexpr int C = body_nv<NV, K>(), Cn = body_nv<NV, K + 1>();
    if constexpr (C < Cn) {
      if (nvb <= C) {
        band_sweep_run<BWD, TF, TA, C, NR>(F0, dsc, src, dst, act, win, za, p1, p2, m, ld, w, l);
        return;
      }
    }
    sweep_body<BWD, TF, TA, NV, NR, K + 1>(nvb, F0, dsc, src, dst, act, win, za, p1, p2, m, ld, w,
                                           l);
  } else {
    band_sweep_run<BWD, TF, TA, NV, NR>(F0, dsc, src, dst, act, win, za, p1, p2, m, ld, w, l);
  }
}

template <typename TF, typename TA, int NV, int NR>
__global__ void __launch_bounds__(256, 2)
k_band_sweep(BandBlocks B, const TF* __restrict__ FL, const TF* __restrict__ FR,
             const double* __restrict__ u, double* __restrict__ y, const int* __restrict__ done,
             int nrhs, int n1, int sys_done) {
  extern __shared__ double sweep_lds_mem[];
  // the wave index is uniform: slot bounds and branches on it stay scalar
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
  TA* lbase = (TA*)sweep_lds_mem;
  TA* win = lbase + w * NR * 512;                                   // own windows, 2 x 256 per vector
  TA* za = lbase + SWEEP_WAVES * NR * 512 + w * NR * 128;           // own [0 x 64 | a], per vector
  TA* p1 = lbase + SWEEP_WAVES * NR * 640;                          // [wave][vector][64]
  TA* p2 = p1 + SWEEP_WAVES * NR * 64;
  const int blk = B.order[blockIdx.x];
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
  const int m = B.m[blk], ld = B.sld[blk], row0 = B.row0[blk];
  if (threadIdx.x == 0) atomicAdd(&B.applies[blk], 1ull);
  // vectors past nrhs read vector j0; inactive vectors write nothing
  const double* ub[NR];
  double* yb[NR];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const size_t o = (size_t)(j0 + q < nrhs ? j0 + q : j0) * n1 + row0;
    ub[q] = u + o;
    yb[q] = y + o;
  }
  // [0 x 64 | a]: the zero half is written once
#pragma unroll
  for (int q = 0; q < NR; ++q) za[q * 128 + l] = (TA)0;
  // slot vectors per wave this block's band needs (uniform)
  const int nvb = __builtin_amdgcn_readfirstlane((ld * (int)sizeof(TF) / 16 + 3) / 4);
  sweep_body<false, TF, TA, NV, NR>(nvb, FL + B.soff[blk], B.dsc + row0, ub, yb, act, win, za, p1,
                                    p2, m, ld, w, l);
  // the backward sweep starts from the forward result of every row
  __threadfence_block();
  __syncthreads();
  sweep_body<true, TF, TA, NV, NR>(nvb, FR + B.soff[blk], B.dsc + row0, yb, yb, act, win, za, p1,
                                   p2, m, ld, w, l);
}

// Register-set sizes (16-byte slot vectors per wave) the sweeps are built
// for: the widest band (ld = 128) takes 16 vectors in FP64, 8 in FP32.
constexpr int SWEEP_NV[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16};

template <typename TF, typename TA, int NR, int K = 0>
const void* sweep_kernel(int nv) {
  if constexpr (K + 1 < (int)(sizeof(SWEEP_NV) / sizeof(int)) &&
                (sizeof(TF) == 8 || SWEEP_NV[K] < 8)) {
    if (nv > SWEEP_NV[K]) return sweep_kernel<TF, TA, NR, K + 1>(nv);
  }
  return (const void*)k_band_sweep<TF, TA, SWEEP_NV[K], NR>;
}

template <typename TF, typename TA, int NR>
hipError_t launch_sweep_nr(hipStream_t st, const BandBlocks& B, const TF* FL, const TF* FR,
                           const double* u, double* y, const int* done, int nrhs, int n1,
                           int sys_done) {
  const size_t lds = sweep_lds<TA>(NR);
  const dim3 grid(B.nblk, (nrhs + NR - 1) / NR);
  // slot vectors per wave: the widest block's slots / VT over four waves
  const int nv = (B.sldmax * (int)sizeof(TF) / 16 + 3) / 4;
  void* args[] = {(void*)&B, (void*)&FL, (void*)&FR, (void*)&u, (void*)&y, (void*)&done,
                  (void*)&nrhs, (void*)&n1, (void*)&sys_done};
  return hipLaunchKernel(sweep_kernel<TF, TA, NR>(nv), grid, dim3(64 * SWEEP_WAVES), args, lds, st);
}

template <typename TF, typename TA>
hipError_t launch_sweep_t(hipStream_t st, const BandBlocks& B, const TF* FL, const TF* FR,
                          const double* u, double* y, const int* done, int nrhs, int n1,
                          int sys_done) {
  // several vectors: chunks of 4 read each factor once per chunk
  if (nrhs == 1) return launch_sweep_nr<TF, TA, 1>(st, B, FL, FR, u, y, done, nrhs, n1, sys_done);
  return launch_sweep_nr<TF, TA, 4>(st, B, FL, FR, u, y, done, nrhs, n1, sys_done);
}

hipError_t launch_sweep(hipStream_t st, const BandBlocks& B, bool mixed, const double* u, double* y,
                        const int* done, int nrhs, int n1, int sys_done) {
  // FP32 projections read the FP32 slot copies and compute in FP64: the
  // operator applied is then the exact inverse (to FP64 rounding) of the
  // factor rounded once, a fixed SPD operator for the outer CG (config 4:
  // 2,858 outer iterations against 3,379 with FP32 arithmetic and 2,746 in
  // FP64), for the same bytes
  return mixed ? launch_sweep_t<float, double>(st, B, B.SL32, B.SR32, u, y, done, nrhs, n1, sys_done)
               : launch_sweep_t<double, double>(st, B, B.SL, B.SR, u, y, done, nrhs, n1, sys_done);
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
  const dim3 grid(64, B.nblk, 2);
  if (mixed)
    hipLaunchKernelGGL(k_band_slots<float>, grid, dim3(64), 0, st, B, B.SL32, B.SR32);
  else
    hipLaunchKernelGGL(k_band_slots<double>, grid, dim3(64), 0, st, B, B.SL, B.SR);
  return hipGetLastError();
}

// Raises the dynamic LDS limit of the multi-vector sweeps (set once at setup,
// so that a launch inside a stream capture is a plain kernel launch).
hipError_t prepare_band_apply(const BandBlocks& B, bool mixed) {
  if (B.nblk == 0) return hipSuccess;
  const int l4 = (int)sweep_lds<double>(4);
  for (int nv : SWEEP_NV) {
    const void* f = mixed ? sweep_kernel<float, double, 4>(nv) : sweep_kernel<double, double, 4>(nv);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, l4);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_band_apply(hipStream_t st, const BandBlocks& B, bool mixed, const double* u,
                             double* y, const int* done) {
  if (B.nblk == 0) return hipSuccess;
  return launch_sweep(st, B, mixed, u, y, done, 1, 0, 1);
}

hipError_t launch_band_apply_multi(hipStream_t st, const BandBlocks& B, bool mixed,
                                   const double* u, double* y, const int* done, int nrhs, int n1) {
  if (B.nblk == 0 || nrhs <= 0) return hipSuccess;
  return launch_sweep(st, B, mixed, u, y, done, nrhs, n1, 0);
}
