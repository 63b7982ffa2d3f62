// Matrix-free inner CG on the block normal equations (A_i A_i^T) y_i = u_i.
//
// The block projection of eq. (H) needs y_i = (A_i A_i^T)^{-1} u_i for every
// block (the paper obtains the same minimum-norm solution through the
// augmented system, Section 1; the normal-equation form is the one named in
// Section 1 as an alternative).  For blocks too large for a dense factor this
// runs classical CG on G_i = A_i A_i^T without forming G_i: each iteration
// computes t = A_i^T q over the block's column support, then z = A_i t.
//
// Work decomposition: a block is owned by `groups` workgroups that split its
// rows (for z and the vector updates) and its support columns (for t).  The
// workgroups of a block meet at a barrier in global memory after t, after the
// reduction of q.z and after the reduction of r.r.  Blocks are placed so that
// the workgroups of one block share an XCD (workgroup ids are dispatched to the
// 8 XCDs round robin), which keeps the block's vectors in one L2.  Every wait
// is bounded by a wall-clock limit; a timeout sets an error flag and ends the
// kernel instead of spinning forever.
#include "common.h"

#include <cmath>

namespace {

constexpr int IN_THREADS = 512;
constexpr int NXCD = 8;

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  static __device__ double* q(const InnerBlocks& B) { return B.q; }
  static __device__ double* z(const InnerBlocks& B) { return B.z; }
  static __device__ double* r(const InnerBlocks& B) { return B.ri; }
  static __device__ double* t(const InnerBlocks& B) { return B.t; }
};
template <>
struct Vec<float> {
  static __device__ float* q(const InnerBlocks& B) { return B.q32; }
  static __device__ float* z(const InnerBlocks& B) { return B.z32; }
  static __device__ float* r(const InnerBlocks& B) { return B.ri32; }
  static __device__ float* t(const InnerBlocks& B) { return B.t32; }
};

constexpr int WG_THREADS = 1024;

// Same single-workgroup inner CG on the sliced ELL copies: for a slice
// every load address is known without reading a row pointer, so a wavefront
// issues the eight index and eight value loads of a chunk at once.
template <typename T>
__device__ __forceinline__ const T* sel_val(const double* d, const float* f);
template <>
__device__ __forceinline__ const double* sel_val<double>(const double* d, const float*) { return d; }
template <>
__device__ __forceinline__ const float* sel_val<float>(const double*, const float* f) { return f; }

// N entries (fixed) from k0 of a lane's slice row, summed in stored order
// after all their loads and gathers are issued; gx(i) reads the gathered
// vector at i.
template <int N, typename T, typename TV, typename IX, class Gx>
__device__ __forceinline__ T inner_chunk(const IX* __restrict__ idx, const TV* __restrict__ val,
                                         long long e, int k0, Gx gx, T acc) {
  IX ix[N];
  TV vv[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    ix[k] = idx[e + (long long)(k0 + k) * 64];
    vv[k] = val[e + (long long)(k0 + k) * 64];
  }
  T xv[N];
#pragma unroll
  for (int k = 0; k < N; ++k) xv[k] = gx(ix[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) acc += (T)vv[k] * xv[k];
  return acc;
}

// The last nb < 8 entries of a slice (widths under 5 are not padded to 8):
// one fixed-size chunk per count, instead of one round trip per entry.
template <typename T, typename TV, typename IX, class Gx>
__device__ __forceinline__ T inner_tail(const IX* __restrict__ idx, const TV* __restrict__ val,
                                        long long e, int k0, int nb, Gx gx, T acc) {
  switch (nb) {
    case 1: return inner_chunk<1, T, TV, IX>(idx, val, e, k0, gx, acc);
    case 2: return inner_chunk<2, T, TV, IX>(idx, val, e, k0, gx, acc);
    case 3: return inner_chunk<3, T, TV, IX>(idx, val, e, k0, gx, acc);
    case 4: return inner_chunk<4, T, TV, IX>(idx, val, e, k0, gx, acc);
    case 5: return inner_chunk<5, T, TV, IX>(idx, val, e, k0, gx, acc);
    case 6: return inner_chunk<6, T, TV, IX>(idx, val, e, k0, gx, acc);
    case 7: return inner_chunk<7, T, TV, IX>(idx, val, e, k0, gx, acc);
    default: return acc;
  }
}

template <typename T>
struct PlainGx {
  const T* __restrict__ x;
  template <typename IX>
  __device__ __forceinline__ T operator()(IX i) const { return x[i]; }
};

// T: vector and arithmetic type; TV: stored matrix values (float values with
// double arithmetic are converted exactly before each product).  w is the
// same on every lane of the wavefront.  BT: the rest of the slice after its
// whole chunks of 8 as one batch (else entry by entry: fewer registers).
template <typename T, typename TV, typename IX, bool BT = true>
__device__ __forceinline__ T sell_row(const IX* __restrict__ idx, const TV* __restrict__ val,
                                      long long e, int w, const T* __restrict__ x, T acc = (T)0) {
  w = __builtin_amdgcn_readfirstlane(w);
  int k0 = 0;
  for (; k0 + 8 <= w; k0 += 8) {
    IX ix[8];
    TV vv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ix[k] = idx[e + (long long)(k0 + k) * 64];
      vv[k] = val[e + (long long)(k0 + k) * 64];
    }
    T xv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) xv[k] = x[ix[k]];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += (T)vv[k] * xv[k];
  }
  if constexpr (BT) {
    if (k0 < w) acc = inner_tail<T, TV, IX>(idx, val, e, k0, w - k0, PlainGx<T>{x}, acc);
  } else {
    for (; k0 < w; ++k0) acc += (T)val[e + (long long)k0 * 64] * x[idx[e + (long long)k0 * 64]];
  }
  return acc;
}

// Two 8-wide slices at once: 32 independent loads per lane in flight.
template <typename T, typename TV, typename IX>
__device__ __forceinline__ void two_slices8(const IX* __restrict__ idx, const TV* __restrict__ val,
                                            long long e1, long long e2, const T* __restrict__ x,
                                            T& a1, T& a2) {
  IX i1[8], i2[8];
  TV v1[8], v2[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    i1[k] = idx[e1 + k * 64];
    v1[k] = val[e1 + k * 64];
    i2[k] = idx[e2 + k * 64];
    v2[k] = val[e2 + k * 64];
  }
  T s1 = (T)0, s2 = (T)0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    s1 += (T)v1[k] * x[i1[k]];
    s2 += (T)v2[k] * x[i2[k]];
  }
  a1 = s1;
  a2 = s2;
}

// LDS layout: q (qcap), t (tcap, if resident), then the slice descriptors
// (offset of every row slice and column slice, and their widths).
// Several right-hand sides of a one-system context: blockIdx.y = j picks
// vector j, whose u, y and residual scratch sit at offset j * vs and whose
// support scratch (when t is not in LDS) at j * tstr; done[sys + j] is its
// flag.  One vector: gridDim.y = 1, vs = tstr = 0.
template <typename T, typename TV, typename IX, int RPT, bool TLDS>
__global__ void __launch_bounds__(WG_THREADS)
k_inner_sell(InnerBlocks B, const double* __restrict__ u, double* __restrict__ y,
             const int* __restrict__ done, int qcap, int tcap, int dcap, long long vs,
             long long tstr) {
  extern __shared__ double lds_d[];
  __shared__ double sh[WG_THREADS / 64];
  const int b = blockIdx.x;
  const int j = blockIdx.y;
  if (done && done[B.sys[b] + j]) return;
  const int row0 = B.row0[b], m = B.m[b];
  const int sup0 = B.sup0[b], ns = B.nsup[b];
  u += (long long)j * vs;
  y += (long long)j * vs;
  T* qs = reinterpret_cast<T*>(lds_d);
  T* ts = TLDS ? qs + qcap : Vec<T>::t(B) + (long long)j * tstr + sup0;
  long long* dptr = reinterpret_cast<long long*>(qs + qcap + (TLDS ? tcap : 0));
  int* dw = reinterpret_cast<int*>(dptr + dcap);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const IX* __restrict__ aidx = reinterpret_cast<const IX*>(B.a_idx);
  const IX* __restrict__ tidx = reinterpret_cast<const IX*>(B.t_idx);
  const TV* __restrict__ aval = sel_val<TV>(B.a_val, B.a_val32);
  const TV* __restrict__ tval = sel_val<TV>(B.t_val, B.t_val32);
  const int nsa = (m + 63) >> 6, nst = (ns + 63) >> 6;
  constexpr int NW = WG_THREADS / 64;
  T* __restrict__ rg = Vec<T>::r(B) + (long long)j * vs + row0;   // residual of the block
  double* __restrict__ yg = y + row0;          // iterate of the block
  // slice descriptors: row slices at [0, nsa), column slices at [nsa, nsa + nst)
  for (int s = threadIdx.x; s < nsa + nst; s += WG_THREADS) {
    if (s < nsa) {
      dptr[s] = B.a_ptr[B.a_s0[b] + s];
      dw[s] = B.a_w[B.a_s0[b] + s];
    } else {
      dptr[s] = B.t_ptr[B.t_s0[b] + s - nsa];
      dw[s] = B.t_w[B.t_s0[b] + s - nsa];
    }
  }
  T zz[RPT];
  double part = 0.0;
  const double* __restrict__ dsc = B.dsc + row0;  // row scaling: solve on D A_i A_i^T D
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int i = (wave + k * NW) * 64 + lane;
    zz[k] = (T)0;
    if (i < m) {
      const T v = (T)(u[row0 + i] * dsc[i]);
      rg[i] = v;
      qs[i] = v;
      yg[i] = 0.0;
      part += (double)v * (double)v;
    }
  }
  const double gamma0 = block_sum(part, sh);
  int it = 0;
  if (gamma0 > 0.0) {
    const double thr = B.tol * B.tol * gamma0;
    double gamma = gamma0;
    while (it < B.maxit) {
      ++it;
      __syncthreads();
      // t = A_i^T q: column slices, two per wavefront round when both are 8 wide
      for (int s = wave; s < nst; s += 2 * NW) {
        const int s2 = s + NW;
        const long long e1 = dptr[nsa + s] + lane;
        const int w1 = dw[nsa + s];
        if (s2 < nst && w1 == 8 && dw[nsa + s2] == 8) {
          T a1, a2;
          two_slices8<T, TV, IX>(tidx, tval, e1, dptr[nsa + s2] + lane, qs, a1, a2);
          if (s * 64 + lane < ns) ts[s * 64 + lane] = a1;
          if (s2 * 64 + lane < ns) ts[s2 * 64 + lane] = a2;
        } else {
          const T a1 = sell_row<T, TV, IX>(tidx, tval, e1, w1, qs);
          if (s * 64 + lane < ns) ts[s * 64 + lane] = a1;
          if (s2 < nst) {
            const T a2 = sell_row<T, TV, IX>(tidx, tval, dptr[nsa + s2] + lane, dw[nsa + s2], qs);
            if (s2 * 64 + lane < ns) ts[s2 * 64 + lane] = a2;
          }
        }
      }
      __syncthreads();
      // z = A_i t on the own rows (two row slices per round), and q.z
      part = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; k += 2) {
        const int s = wave + k * NW, s2 = s + NW;
        if (s < nsa) {
          T a1 = (T)0, a2 = (T)0;
          if (k + 1 < RPT && s2 < nsa && dw[s] == 8 && dw[s2] == 8) {
            two_slices8<T, TV, IX>(aidx, aval, dptr[s] + lane, dptr[s2] + lane, ts, a1, a2);
          } else {
            a1 = sell_row<T, TV, IX>(aidx, aval, dptr[s] + lane, dw[s], ts);
            if (k + 1 < RPT && s2 < nsa) a2 = sell_row<T, TV, IX>(aidx, aval, dptr[s2] + lane, dw[s2], ts);
          }
          const int i1 = s * 64 + lane, i2 = s2 * 64 + lane;
          if (i1 < m) {
            zz[k] = a1;
            part += (double)qs[i1] * (double)a1;
          }
          if (k + 1 < RPT && i2 < m) {
            zz[k + 1] = a2;
            part += (double)qs[i2] * (double)a2;
          }
        }
        __asm__ __volatile__("" ::: "memory");
      }
      const double delta = block_sum(part, sh);
      if (!(delta > 0.0) || !isfinite(delta)) break;
      const double alpha = gamma / delta;
      part = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = (wave + k * NW) * 64 + lane;
        if (i < m) {
          yg[i] += alpha * (double)qs[i];
          const T rn = rg[i] - (T)alpha * zz[k];
          rg[i] = rn;
          part += (double)rn * (double)rn;
        }
      }
      const double gnew = block_sum(part, sh);
      if (gnew <= thr) break;
      const T beta = (T)(gnew / gamma);
      gamma = gnew;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int i = (wave + k * NW) * 64 + lane;
        if (i < m) qs[i] = rg[i] + beta * qs[i];
      }
    }
  }
  // y_i = D z~ where z~ solved the scaled system
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += WG_THREADS) yg[i] *= dsc[i];
  if (threadIdx.x == 0) {
    if (j == 0) B.iters[b] = it;
    atomicAdd(B.total, (unsigned long long)it);
    atomicAdd(&B.blk_total[b], (unsigned long long)it);
  }
}

// Vectors of one launch of the single-workgroup kernel: nv, at strides vs
// (rows) and tstr (support positions).
struct VecSet {
  int nv;
  long long vs, tstr;
};

template <typename T, typename TV, typename IX, int RPT>
hipError_t launch_sell(hipStream_t st, const InnerBlocks& B, const double* u, double* y,
                       const int* done, int qcap, int tcap, int dcap, bool tlds, size_t lds,
                       const VecSet& V) {
  const void* fn = tlds ? (const void*)k_inner_sell<T, TV, IX, RPT, true>
                        : (const void*)k_inner_sell<T, TV, IX, RPT, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid(B.nblk, V.nv);
  if (tlds)
    hipLaunchKernelGGL((k_inner_sell<T, TV, IX, RPT, true>), grid, dim3(WG_THREADS), lds, st, B, u, y,
                       done, qcap, tcap, dcap, V.vs, V.tstr);
  else
    hipLaunchKernelGGL((k_inner_sell<T, TV, IX, RPT, false>), grid, dim3(WG_THREADS), lds, st, B, u,
                       y, done, qcap, tcap, dcap, V.vs, V.tstr);
  return hipGetLastError();
}

template <typename T, typename TV, typename IX>
hipError_t launch_sell_rows(hipStream_t st, const InnerBlocks& B, const double* u, double* y,
                            const int* done, const VecSet& V = VecSet{1, 0, 0}) {
  const int rpt = (B.max_m + WG_THREADS - 1) / WG_THREADS;
  // element counts rounded so that the descriptor array stays 8-byte aligned
  const int qcap = (B.max_m + 1) / 2 * 2;
  const int tcap = (B.max_nsup + 1) / 2 * 2;
  const int dcap = (B.max_m + 63) / 64 + (B.max_nsup + 63) / 64;
  const size_t dbytes = (size_t)dcap * (sizeof(long long) + sizeof(int));
  const size_t lds_budget = 160 * 1024 - (WG_THREADS / 64) * sizeof(double) - 256;
  const bool tlds = (size_t)(qcap + tcap) * sizeof(T) + dbytes <= lds_budget;
  const size_t lds = (size_t)(qcap + (tlds ? tcap : 0)) * sizeof(T) + dbytes;
  if (rpt <= 4) return launch_sell<T, TV, IX, 4>(st, B, u, y, done, qcap, tcap, dcap, tlds, lds, V);
  if (rpt <= 8) return launch_sell<T, TV, IX, 8>(st, B, u, y, done, qcap, tcap, dcap, tlds, lds, V);
  if (rpt <= 9) return launch_sell<T, TV, IX, 9>(st, B, u, y, done, qcap, tcap, dcap, tlds, lds, V);
  if (rpt <= 10) return launch_sell<T, TV, IX, 10>(st, B, u, y, done, qcap, tcap, dcap, tlds, lds, V);
  if (rpt <= 12) return launch_sell<T, TV, IX, 12>(st, B, u, y, done, qcap, tcap, dcap, tlds, lds, V);
  return launch_sell<T, TV, IX, 16>(st, B, u, y, done, qcap, tcap, dcap, tlds, lds, V);
}

// ------------------------------------------------------------------------
// Several workgroups per block (`groups`, all on the block's XCD), running CG
// in the Chronopoulos-Gear arrangement.  Every workgroup keeps the block's
// whole r and s = G q in LDS (updated redundantly); t and w = G r are
// exchanged through global memory.  Per inner iteration:
//   t = A_i^T r on the own column slices -> barrier
//   w = A_i t on the own row slices (t gathered from global), (r,r), (w,r)
//     -> each workgroup publishes its two partials, tagged with the epoch
//   alpha, beta from the G partials; q and y on the own rows, s and r on all
//   rows (w read from global).
//
// The barrier is a flag array: each workgroup stores its epoch with an
// agent-scope store after its stores have completed, and polls the block's
// flags with agent-scope loads; exchanged data is read with agent-scope loads.
// The partials need no barrier of their own: each is stored, once the
// workgroup's w stores have completed, as two 64-bit words {half, epoch}
// (an aligned 64-bit atomic store is seen whole), and a reader that finds the
// current epoch in both words of every workgroup has the partials and, by
// that ordering, all of w.  This relies on the workgroups of a block sharing
// one L2: the kernel checks the XCC id of every workgroup at entry and, if any
// is misplaced, the whole group adds full agent-scope fences.
constexpr int GRP_THREADS = 1024;

__device__ __forceinline__ unsigned xcc_id() {
  return __builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xf;
}

template <typename T>
__device__ __forceinline__ T agent_load(const T* p);
template <>
__device__ __forceinline__ double agent_load<double>(const double* p) {
  return __builtin_bit_cast(double, __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
template <>
__device__ __forceinline__ float agent_load<float>(const float* p) {
  return __builtin_bit_cast(float, __hip_atomic_load(reinterpret_cast<const unsigned*>(p),
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

struct FlagBar {
  unsigned* flags;   // this block's `groups` epoch slots
  unsigned epoch;
  int g, groups;
  bool fenced;       // full agent-scope fences (workgroups not on one XCC)
  unsigned long long ticks;  // wait bound (0: give up at the first check)
};

__device__ __forceinline__ bool flag_barrier(FlagBar& fb, int* err) {
  __shared__ int ok_sh;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  fb.epoch += 1;
  if (threadIdx.x == 0) {
    if (fb.fenced) __threadfence();
    __hip_atomic_store(&fb.flags[fb.g], fb.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  int ok = 1;
  if (threadIdx.x < 64) {
    const unsigned long long t0 = wall_clock64();
    while (true) {
      const unsigned v = threadIdx.x < fb.groups
                             ? __hip_atomic_load(&fb.flags[threadIdx.x], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                             : fb.epoch;
      if (fb.ticks != 0 && __all((int)(v - fb.epoch) >= 0)) break;
      if (wall_clock64() - t0 > fb.ticks) {
        ok = 0;
        if (threadIdx.x == 0) atomicExch(err, 1);
        break;
      }
    }
    if (fb.fenced) __threadfence();
  }
  if (threadIdx.x == 0) ok_sh = ok;
  __syncthreads();
  return ok_sh != 0;
}

// A wavefront-uniform double moved to scalar registers (frees vector
// registers for loop-carried scalars).
__device__ __forceinline__ double uniform_f64(double v) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)bits);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(bits >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// A value published as two words {low or high half, epoch}.
__device__ __forceinline__ void put_tagged(unsigned long long* p, double v, unsigned ep) {
  const unsigned long long bits = __builtin_bit_cast(unsigned long long, v);
  const unsigned long long tag = (unsigned long long)ep << 32;
  __hip_atomic_store(p, tag | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, tag | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits (bounded) for the two tagged values at p and p + 2 of epoch ep on
// every lane of the wavefront where `active` (the others pass).
__device__ __forceinline__ bool get_tagged2(const unsigned long long* p, bool active, unsigned ep,
                                            double& a, double& b, int* err,
                                            unsigned long long ticks) {
  const unsigned long long idle = (unsigned long long)ep << 32;
  const unsigned long long t0 = wall_clock64();
  while (true) {
    unsigned long long v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      v[q] = active ? __hip_atomic_load(p + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : idle;
    const bool here = (unsigned)(v[0] >> 32) == ep && (unsigned)(v[1] >> 32) == ep &&
                      (unsigned)(v[2] >> 32) == ep && (unsigned)(v[3] >> 32) == ep;
    if (ticks != 0 && __all(here)) {
      a = __builtin_bit_cast(double, (v[1] << 32) | (v[0] & 0xffffffffull));
      b = __builtin_bit_cast(double, (v[3] << 32) | (v[2] & 0xffffffffull));
      return true;
    }
    if (wall_clock64() - t0 > ticks) {
      if ((threadIdx.x & 63) == 0) atomicExch(err, 1);
      return false;
    }
  }
}

template <typename T, typename TV, typename IX, int RPT>
__global__ void __launch_bounds__(GRP_THREADS)
k_inner_grp(InnerBlocks B, const double* __restrict__ u, double* __restrict__ y,
            const int* __restrict__ done, int rcap, int* err) {
  extern __shared__ double lds_d[];
  __shared__ double sh[GRP_THREADS / 64];
  __shared__ double sh2[2 * (GRP_THREADS / 64)];
  __shared__ int fenced_sh;
  const int G = B.groups;
  const int w = blockIdx.x;
  const int xcd = w % NXCD, kk = w / NXCD;
  const int lb = kk / G, g = kk % G;
  const int b = lb * NXCD + xcd;
  if (b >= B.nblk) return;
  if (done && done[B.sys[b]]) return;
  const int row0 = B.row0[b], m = B.m[b];
  const int sup0 = B.sup0[b], ns = B.nsup[b];
  const int nsa = (m + 63) >> 6, nst = (ns + 63) >> 6;
  // own slices
  const int sa0 = nsa * g / G, sa1 = nsa * (g + 1) / G;
  const int st0 = nst * g / G, st1 = nst * (g + 1) / G;
  T* qs = reinterpret_cast<T*>(lds_d);
  T* rs = qs + rcap;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  constexpr int NW = GRP_THREADS / 64;
  const IX* __restrict__ aidx = reinterpret_cast<const IX*>(B.a_idx);
  const IX* __restrict__ tidx = reinterpret_cast<const IX*>(B.t_idx);
  const TV* __restrict__ aval = sel_val<TV>(B.a_val, B.a_val32);
  const TV* __restrict__ tval = sel_val<TV>(B.t_val, B.t_val32);
  const long long* __restrict__ aptr = B.a_ptr + B.a_s0[b];
  const int* __restrict__ aw = B.a_w + B.a_s0[b];
  const long long* __restrict__ tptr = B.t_ptr + B.t_s0[b];
  const int* __restrict__ tw = B.t_w + B.t_s0[b];
  T* tg = Vec<T>::t(B) + sup0;     // exchanged t of the block
  T* zg = Vec<T>::z(B) + row0;     // exchanged z of the block
  unsigned long long* const xp = B.xp + (size_t)b * 2 * 64;  // tagged partials, 2 parities
  // entry offsets (relative to the block's first slice, 32 bit) and widths
  // of the own slices, loop invariant: the first RPT own column slices of a
  // wavefront and all its own row slices
  const long long abase = aptr[0], tbase = tptr[0];
  const IX* __restrict__ aidxb = aidx + abase;
  const TV* __restrict__ avalb = aval + abase;
  const IX* __restrict__ tidxb = tidx + tbase;
  const TV* __restrict__ tvalb = tval + tbase;
  int ea[RPT], et[RPT];
  int wa[RPT], wt[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int s = sa0 + wave + k * NW;
    ea[k] = s < sa1 ? (int)(aptr[s] - abase) + lane : 0;
    wa[k] = s < sa1 ? aw[s] : 0;
    const int c = st0 + wave + k * NW;
    et[k] = c < st1 ? (int)(tptr[c] - tbase) + lane : 0;
    wt[k] = c < st1 ? tw[c] : 0;
  }
  const int nown = sa1 - sa0;
  // stores of t and w held back to the end of their phase (registers allow
  // it for up to two slices per wavefront)
  constexpr bool DEFER = RPT <= 2;
  __shared__ double gd_sh[2];
  __shared__ int fail_sh;
  FlagBar fb{B.bar + (size_t)b * 32, 0u, g, G, false, B.wait_ticks};
  if (threadIdx.x == 0) {
    fb.epoch = __hip_atomic_load(&fb.flags[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // placement check: publish this workgroup's XCC and whether it matches
    __hip_atomic_store(&fb.flags[16 + g], (unsigned)(xcc_id() == (unsigned)xcd ? 1 : 2),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
  fb.epoch = __shfl(fb.epoch, 0, 64);
  __shared__ unsigned epoch_sh;
  if (threadIdx.x == 0) epoch_sh = fb.epoch;
  __syncthreads();
  fb.epoch = epoch_sh;
  // first barrier with fences; then every workgroup reads the placement flags
  fb.fenced = true;
  bool ok = flag_barrier(fb, err);
  if (threadIdx.x == 0) {
    int bad = 0;
    for (int q = 0; q < G; ++q)
      bad |= __hip_atomic_load(&fb.flags[16 + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 1;
    fenced_sh = bad;
  }
  __syncthreads();
  fb.fenced = fenced_sh != 0;

  // CG in the Chronopoulos-Gear arrangement: one product w = G r and one
  // fused reduction of (r, r) and (w, r) per iteration, with
  //   beta = gamma / gamma_old,  alpha = gamma / (delta - beta gamma / alpha_old),
  //   q = r + beta q,  s = w + beta s (= G q),  y += alpha q,  r -= alpha s.
  // r and s are kept whole in every workgroup's LDS (updated redundantly;
  // w is exchanged through global memory), q and y only on the own rows.
  // Full r = D u in LDS (row scaling), s = 0.
  const double* __restrict__ dsc = B.dsc + row0;
  T* ss = qs;  // the first LDS vector holds s
  for (int i = threadIdx.x; i < m; i += GRP_THREADS) {
    rs[i] = (T)(u[row0 + i] * dsc[i]);
    ss[i] = (T)0;
  }
  double yy[RPT];
  T qq[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    yy[k] = 0.0;
    qq[k] = (T)0;
  }
  __syncthreads();
  int it = 0;
  T* wg = zg;  // exchanged w of the block
  unsigned long long* tr = (B.trace && b == 0 && threadIdx.x == 0) ? B.trace + (size_t)g * 8 * 64 : nullptr;
#define TRACE_AT(slot) do { if (tr && it <= 64) tr[(it - 1) * 8 + (slot)] = wall_clock64(); } while (0)
  if (ok) {
    double thr = -1.0, gamma_old = 0.0, alpha_old = 0.0;
    while (it < B.maxit) {
      ++it;
      TRACE_AT(0);
      // t = A_i^T r on the own column slices (r from LDS).  With few slices
      // per wavefront the stores come after all the loads: a load issued
      // after a store is not complete before the store is.
      T tacc[RPT];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int c = st0 + wave + k * NW;
        tacc[k] = (T)0;
        if (c < st1) {
          // opaque to the compiler, so that the entry addresses are formed
          // here rather than held across the whole loop
          int e = et[k];
          asm volatile("" : "+v"(e));
          tacc[k] = sell_row<T, TV, IX, (RPT <= 4)>(tidxb, tvalb, e, wt[k], rs);
          if (!DEFER && c * 64 + lane < ns) tg[c * 64 + lane] = tacc[k];
        }
      }
      for (int c = st0 + wave + RPT * NW; c < st1; c += NW) {
        const T acc = sell_row<T, TV, IX, (RPT <= 4)>(tidx, tval, tptr[c] + lane, tw[c], rs);
        if (c * 64 + lane < ns) tg[c * 64 + lane] = acc;
      }
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int c = st0 + wave + k * NW;
        if (DEFER && c < st1 && c * 64 + lane < ns) tg[c * 64 + lane] = tacc[k];
      }
      TRACE_AT(1);
      if (!flag_barrier(fb, err)) { ok = false; break; }
      TRACE_AT(2);
      const unsigned E = fb.epoch;
      // w = A_i t on the own row slices, t gathered from global; (r,r), (w,r)
      double pg = 0.0, pd = 0.0;
      T wacc[RPT];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int s = sa0 + wave + k * NW;
        if (s < sa1) {
          int e = ea[k];
          asm volatile("" : "+v"(e));
          const int ww = wa[k];
          T acc = (T)0;
          int k0 = 0;
          for (; k0 + 8 <= ww; k0 += 8) {
            IX ix[8];
            TV vv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
              ix[q] = aidxb[e + (k0 + q) * 64];
              vv[q] = avalb[e + (k0 + q) * 64];
            }
            T tv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) tv[q] = agent_load<T>(&tg[ix[q]]);
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += (T)vv[q] * tv[q];
          }
          for (; k0 < ww; ++k0) acc += (T)avalb[e + k0 * 64] * agent_load<T>(&tg[aidxb[e + k0 * 64]]);
          const int i = s * 64 + lane;
          if (DEFER)
            wacc[k] = acc;
          else if (i < m)
            wg[i] = acc;
          if (i < m) {
            const double ri = (double)rs[i];
            pg += ri * ri;
            pd += (double)acc * ri;
          }
        }
      }
      // (stores after all the loads, as in the t phase)
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int s = sa0 + wave + k * NW;
        if (DEFER && s < sa1 && s * 64 + lane < m) wg[s * 64 + lane] = wacc[k];
      }
      TRACE_AT(3);
      // workgroup partials (wave sums, then the waves in order), published by
      // thread 0 once every wavefront's w stores have completed
      pg = wave_sum_lane0(pg);
      pd = wave_sum_lane0(pd);
      __builtin_amdgcn_s_waitcnt(0);
      if (lane == 0) {
        sh2[wave] = pg;
        sh2[NW + wave] = pd;
      }
      __syncthreads();
      TRACE_AT(6);
      unsigned long long* const xpe = xp + (E & 1u) * 64;
      if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
        for (int q = 0; q < NW; ++q) {
          ta += sh2[q];
          tb += sh2[NW + q];
        }
        if (fb.fenced) __threadfence();
        put_tagged(xpe + g * 4, ta, E);
        put_tagged(xpe + g * 4 + 2, tb, E);
      }
      // the G partials, summed in group order by wavefront 0
      if (wave == 0) {
        double pgq = 0.0, pdq = 0.0;
        bool okp = true;
        okp = get_tagged2(xpe + (lane < G ? lane : 0) * 4, lane < G, E, pgq, pdq, err, B.wait_ticks);
        if (lane >= G) pgq = pdq = 0.0;
        if (fb.fenced) __threadfence();
        double gsum = 0.0, dsum = 0.0;
        for (int q = 0; q < G; ++q) {
          gsum += __shfl(pgq, q, 64);
          dsum += __shfl(pdq, q, 64);
        }
        if (lane == 0) {
          gd_sh[0] = gsum;
          gd_sh[1] = dsum;
          fail_sh = 0;
        }
        TRACE_AT(7);
        if (__any(!okp) && lane == 0) fail_sh = 1;
      }
      __syncthreads();
      TRACE_AT(4);
      if (fail_sh) {
        ok = false;
        break;
      }
      const double gamma = uniform_f64(gd_sh[0]), delta = uniform_f64(gd_sh[1]);
      if (thr < 0.0) {
        if (!(gamma > 0.0)) break;  // u_i = 0: y_i = 0
        thr = B.tol * B.tol * gamma;
      }
      if (gamma <= thr) break;
      double beta = 0.0, alpha;
      if (it == 1) {
        alpha = gamma / delta;
      } else {
        beta = gamma / gamma_old;
        alpha = gamma / (delta - beta * gamma / alpha_old);
      }
      alpha = uniform_f64(alpha);
      beta = uniform_f64(beta);
      if (!(alpha > 0.0) || !isfinite(alpha)) break;
      gamma_old = gamma;
      alpha_old = alpha;
      // s = w + beta s, r -= alpha s on all rows, and on the own rows first
      // q = r + beta q, y += alpha q.  Slice j = wave + c NW of this
      // wavefront is slice sa0 + j (mod nsa): the own slices come first and
      // stay with the thread that holds their q and y.  The w loads of UB
      // slices are issued before their use.
      constexpr int UB = 8;  // slices per batch of loads
      // (lane index opaque: the row indices are formed here, not kept live)
      int ln = lane;
      asm volatile("" : "+v"(ln));
#pragma unroll
      for (int c0 = 0; c0 < 16; c0 += UB) {
        if (wave + c0 * NW >= nsa) break;
        int ri[UB];
        T wv[UB];
#pragma unroll
        for (int c = 0; c < UB; ++c) {
          const int j = wave + (c0 + c) * NW;
          int sl = sa0 + j;
          if (sl >= nsa) sl -= nsa;
          ri[c] = j < nsa ? sl * 64 + ln : m;
          wv[c] = ri[c] < m ? agent_load<T>(&wg[ri[c]]) : (T)0;
        }
#pragma unroll
        for (int c = 0; c < UB; ++c) {
          const int i = ri[c];
          if (i < m) {
            if (c0 + c < RPT && wave + (c0 + c) * NW < nown) {
              qq[(c0 + c) % RPT] = rs[i] + (T)beta * qq[(c0 + c) % RPT];
              yy[(c0 + c) % RPT] += alpha * (double)qq[(c0 + c) % RPT];
            }
            const T si = wv[c] + (T)beta * ss[i];
            ss[i] = si;
            rs[i] = rs[i] - (T)alpha * si;
          }
        }
      }
      __syncthreads();
      TRACE_AT(5);
    }
  }
#undef TRACE_AT
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int s = sa0 + wave + k * NW;
    const int i = s * 64 + lane;
    if (s < sa1 && i < m) y[row0 + i] = yy[k] * dsc[i];
  }
  if (g == 0 && threadIdx.x == 0) {
    B.iters[b] = ok ? it : -1;
    atomicAdd(B.total, (unsigned long long)it);
    atomicAdd(&B.blk_total[b], (unsigned long long)it);
  }
}

template <typename T, typename TV, typename IX, int RPT>
hipError_t launch_grp_t(hipStream_t st, const InnerBlocks& B, const double* u, double* y,
                        const int* done, int* err) {
  const int rcap = (B.max_m + 1) / 2 * 2;
  const size_t lds = (size_t)2 * rcap * sizeof(T);
  const void* fn = (const void*)k_inner_grp<T, TV, IX, RPT>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int per_xcd = (B.nblk + NXCD - 1) / NXCD;
  const int grid = per_xcd * B.groups * NXCD;
  InnerBlocks Bc = B;
  int rc = rcap;
  void* args[] = {&Bc, (void*)&u, (void*)&y, (void*)&done, &rc, &err};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(GRP_THREADS), args, lds, st);
}

template <typename T, typename TV, typename IX>
hipError_t launch_grp(hipStream_t st, const InnerBlocks& B, const double* u, double* y,
                      const int* done, int* err) {
  // own row slices per workgroup, spread over the 16 wavefronts
  const int nsa_max = (B.max_m + 63) / 64;
  const int own = (nsa_max + B.groups - 1) / B.groups;
  const int rpt = (own + 15) / 16;
  if (rpt <= 1) return launch_grp_t<T, TV, IX, 1>(st, B, u, y, done, err);
  if (rpt <= 2) return launch_grp_t<T, TV, IX, 2>(st, B, u, y, done, err);
  if (rpt <= 4) return launch_grp_t<T, TV, IX, 4>(st, B, u, y, done, err);
  return launch_grp_t<T, TV, IX, 8>(st, B, u, y, done, err);
}

}  // namespace

// The kernel pair for the context's precision and index width.
template <typename IX>
hipError_t launch_inner_ix(hipStream_t st, const InnerBlocks& B, InnerPrec prec, const double* u,
                           double* y, const int* done) {
  if (B.groups > 1) {
    int* err = B.err;
    if (prec == INNER_F32) return launch_grp<float, float, IX>(st, B, u, y, done, err);
    if (prec == INNER_F64_V32) return launch_grp<double, float, IX>(st, B, u, y, done, err);
    return launch_grp<double, double, IX>(st, B, u, y, done, err);
  }
  if (prec == INNER_F32) return launch_sell_rows<float, float, IX>(st, B, u, y, done);
  if (prec == INNER_F64_V32) return launch_sell_rows<double, float, IX>(st, B, u, y, done);
  return launch_sell_rows<double, double, IX>(st, B, u, y, done);
}

hipError_t launch_inner_cg(hipStream_t st, const InnerBlocks& B, InnerPrec prec, const double* u,
                           double* y, const int* done) {
  if (B.nblk == 0) return hipSuccess;
  return B.idx16 ? launch_inner_ix<uint16_t>(st, B, prec, u, y, done)
                 : launch_inner_ix<int>(st, B, prec, u, y, done);
}

// nrhs vectors of a one-system context in one launch of the single-workgroup
// kernel (grid blocks x vectors), with per-vector residual scratch rs
// (nrhs * n1 values) and support scratch ts (nrhs * sup_total values), both
// of the inner precision.  Taken when the blocks use that kernel anyway
// (groups = 1: the same bits as one vector at a time) or when blocks x
// vectors reach the CUs, where concurrent single-workgroup solves beat the
// grouped ones run one vector after another; *taken = false leaves the
// vectors to the caller.
hipError_t launch_inner_cg_multi(hipStream_t st, const InnerBlocks& B, InnerPrec prec,
                                 const double* u, double* y, const int* done, int nrhs, int n1,
                                 int sup_total, void* rs, void* ts, bool* taken) {
  *taken = false;
  if (B.nblk == 0) {
    *taken = true;
    return hipSuccess;
  }
  static const int ncu = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    return n;
  }();
  if (!rs || !ts || nrhs < 1 || nrhs > 65535) return hipSuccess;
  if (B.groups > 1 && (long long)nrhs * B.nblk < ncu) return hipSuccess;
  InnerBlocks Bm = B;
  if (prec == INNER_F32) {
    Bm.ri32 = static_cast<float*>(rs);
    Bm.t32 = static_cast<float*>(ts);
  } else {
    Bm.ri = static_cast<double*>(rs);
    Bm.t = static_cast<double*>(ts);
  }
  const VecSet V{nrhs, (long long)n1, (long long)sup_total};
  *taken = true;
  if (B.idx16) {
    if (prec == INNER_F32) return launch_sell_rows<float, float, uint16_t>(st, Bm, u, y, done, V);
    if (prec == INNER_F64_V32) return launch_sell_rows<double, float, uint16_t>(st, Bm, u, y, done, V);
    return launch_sell_rows<double, double, uint16_t>(st, Bm, u, y, done, V);
  }
  if (prec == INNER_F32) return launch_sell_rows<float, float, int>(st, Bm, u, y, done, V);
  if (prec == INNER_F64_V32) return launch_sell_rows<double, float, int>(st, Bm, u, y, done, V);
  return launch_sell_rows<double, double, int>(st, Bm, u, y, done, V);
}

int inner_grp_max_resident(bool f32_vectors, int max_m) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const int rcap = (max_m + 1) / 2 * 2;
  const size_t lds = (size_t)2 * rcap * (f32_vectors ? sizeof(float) : sizeof(double));
  const void* fn = f32_vectors ? (const void*)k_inner_grp<float, float, uint16_t, 2>
                               : (const void*)k_inner_grp<double, double, uint16_t, 2>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, GRP_THREADS, lds) != hipSuccess)
    return 0;
  return per_cu * ncu;
}

