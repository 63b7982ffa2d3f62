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
// about 2 s of the 100 MHz constant clock
constexpr unsigned long long WAIT_LIMIT = 200000000ull;

struct GroupCtx {
  unsigned* bar;      // [0] arrival count, [1] generation
  unsigned gen;       // generation this workgroup waits to leave
  int groups;
};

__device__ __forceinline__ bool group_barrier(GroupCtx& gc, int* err) {
  __shared__ int ok_sh;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    __threadfence();
    const unsigned arrived = atomicAdd(&gc.bar[0], 1u);
    if (arrived == (unsigned)(gc.groups - 1)) {
      atomicExch(&gc.bar[0], 0u);
      __threadfence();
      atomicAdd(&gc.bar[1], 1u);
    } else {
      const unsigned long long t0 = wall_clock64();
      while (__hip_atomic_load(&gc.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gc.gen) {
        __builtin_amdgcn_s_sleep(2);
        if (wall_clock64() - t0 > WAIT_LIMIT) {
          ok = 0;
          atomicExch(err, 1);
          break;
        }
      }
    }
    __threadfence();
    gc.gen += 1;
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  static __device__ double* q(const InnerBlocks& B) { return B.q; }
  static __device__ double* z(const InnerBlocks& B) { return B.z; }
  static __device__ double* r(const InnerBlocks& B) { return B.ri; }
  static __device__ double* t(const InnerBlocks& B) { return B.t; }
  static __device__ const double* v(const InnerBlocks& B) { return B.val; }
  static __device__ const double* bv(const InnerBlocks& B) { return B.btval; }
};
template <>
struct Vec<float> {
  static __device__ float* q(const InnerBlocks& B) { return B.q32; }
  static __device__ float* z(const InnerBlocks& B) { return B.z32; }
  static __device__ float* r(const InnerBlocks& B) { return B.ri32; }
  static __device__ float* t(const InnerBlocks& B) { return B.t32; }
  static __device__ const float* v(const InnerBlocks& B) { return B.val32; }
  static __device__ const float* bv(const InnerBlocks& B) { return B.btval32; }
};

// Sum of a workgroup-local partial over the `groups` workgroups of a block,
// in a fixed order.  slots: this block's `groups` doubles.
template <bool MULTI>
__device__ __forceinline__ double group_allreduce(double v, double* sh, double* slots, int g,
                                                  GroupCtx& gc, int* err, bool& ok) {
  v = block_sum(v, sh);
  if constexpr (!MULTI) {
    return v;
  } else {
    if (threadIdx.x == 0) slots[g] = v;
    ok = group_barrier(gc, err) && ok;
    double s = 0.0;
    for (int i = 0; i < gc.groups; ++i) s += slots[i];
    return s;
  }
}

template <typename T, bool MULTI>
__global__ void __launch_bounds__(IN_THREADS)
k_inner_cg(InnerBlocks B, const double* __restrict__ u, double* __restrict__ y,
           const int* __restrict__ done, int nslots_per_xcd, int* err) {
  __shared__ double sh[IN_THREADS / 64];
  const int G = MULTI ? B.groups : 1;
  // XCD-aware placement: workgroup w runs on XCD w % 8; block b lives on XCD
  // b % 8 and uses that XCD's workgroup slots [lb*G, lb*G+G), lb = b / 8.
  const int w = blockIdx.x;
  const int xcd = w % NXCD, k = w / NXCD;
  const int lb = k / G, g = k % G;
  const int b = lb * NXCD + xcd;
  if (b >= B.nblk) return;
  if (done && done[B.sys[b]]) return;

  const int row0 = B.row0[b], m = B.m[b];
  const int sup0 = B.sup0[b], ns = B.nsup[b];
  const int lo = (int)((long long)m * g / G), hi = (int)((long long)m * (g + 1) / G);
  const int slo = (int)((long long)ns * g / G), shi = (int)((long long)ns * (g + 1) / G);
  T* q = Vec<T>::q(B) + row0;
  T* z = Vec<T>::z(B) + row0;
  T* r = Vec<T>::r(B) + row0;
  T* t = Vec<T>::t(B) + sup0;
  const T* av = Vec<T>::v(B);
  const T* bv = Vec<T>::bv(B);
  const int* __restrict__ rowptr = B.rowptr + row0;
  const int* __restrict__ btptr = B.btptr + sup0;
  double* slots_a = B.red + (size_t)b * 2 * G;
  double* slots_b = slots_a + G;
  GroupCtx gc{B.bar + 2 * b, 0u, G};
  if (MULTI && threadIdx.x == 0)
    gc.gen = __hip_atomic_load(&gc.bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  bool ok = true;

  // r = u, q = u, y = 0 on this workgroup's rows; gamma0 = ||u_i||^2
  double part = 0.0;
  for (int i = lo + threadIdx.x; i < hi; i += IN_THREADS) {
    const double ui = u[row0 + i];
    const T uv = (T)ui;
    r[i] = uv;
    q[i] = uv;
    y[row0 + i] = 0.0;
    part += (double)uv * (double)uv;
  }
  const double gamma0 = group_allreduce<MULTI>(part, sh, slots_a, g, gc, err, ok);
  if (gamma0 == 0.0 || !ok) {
    if (g == 0 && threadIdx.x == 0) B.iters[b] = 0;
    return;
  }
  const double thr = B.tol * B.tol * gamma0;
  double gamma = gamma0;
  // y accumulates in registers? No: rows per thread vary; keep y in memory.
  int it = 0;
  while (it < B.maxit) {
    ++it;
    // t = A_i^T q on this workgroup's support columns
    for (int c = slo + threadIdx.x; c < shi; c += IN_THREADS) {
      const int e0 = btptr[c], e1 = btptr[c + 1];
      T acc = (T)0;
      for (int e = e0; e < e1; ++e) acc += bv[e] * q[B.btrow[e]];
      t[c] = acc;
    }
    if constexpr (MULTI) {
      if (!group_barrier(gc, err)) { ok = false; break; }
    } else {
      __syncthreads();
    }
    // z = A_i t on this workgroup's rows; q.z
    part = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += IN_THREADS) {
      const int e0 = rowptr[i], e1 = rowptr[i + 1];
      T acc = (T)0;
      for (int e = e0; e < e1; ++e) acc += av[e] * t[B.loc[e]];
      z[i] = acc;
      part += (double)q[i] * (double)acc;
    }
    const double delta = group_allreduce<MULTI>(part, sh, slots_a, g, gc, err, ok);
    if (!ok) break;
    if (!(delta > 0.0) || !isfinite(delta)) break;
    const double alpha = gamma / delta;
    part = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += IN_THREADS) {
      y[row0 + i] += alpha * (double)q[i];
      const T ri = r[i] - (T)alpha * z[i];
      r[i] = ri;
      part += (double)ri * (double)ri;
    }
    const double gnew = group_allreduce<MULTI>(part, sh, slots_b, g, gc, err, ok);
    if (!ok) break;
    if (gnew <= thr) break;
    const T beta = (T)(gnew / gamma);
    gamma = gnew;
    for (int i = lo + threadIdx.x; i < hi; i += IN_THREADS) q[i] = r[i] + beta * q[i];
    if constexpr (MULTI) {
      if (!group_barrier(gc, err)) { ok = false; break; }
    } else {
      __syncthreads();
    }
  }
  if (g == 0 && threadIdx.x == 0) {
    B.iters[b] = ok ? it : -1;
    atomicAdd(B.total, (unsigned long long)it);
  }
}

}  // namespace

// Device-side error flag of the inner CG (wait timeouts); allocated once per process.
static int* g_inner_err = nullptr;

int* inner_err_flag() {
  if (!g_inner_err) {
    if (hipMalloc(&g_inner_err, sizeof(int)) != hipSuccess) return nullptr;
    if (hipMemset(g_inner_err, 0, sizeof(int)) != hipSuccess) return nullptr;
  }
  return g_inner_err;
}

hipError_t launch_inner_cg(hipStream_t st, const InnerBlocks& B, bool mixed, const double* u,
                           double* y, const int* done) {
  if (B.nblk == 0) return hipSuccess;
  int* err = inner_err_flag();
  if (!err) return hipErrorOutOfMemory;
  const int G = B.groups < 1 ? 1 : B.groups;
  const int per_xcd = (B.nblk + NXCD - 1) / NXCD;
  const int grid = per_xcd * G * NXCD;
  if (G == 1) {
    if (mixed)
      hipLaunchKernelGGL((k_inner_cg<float, false>), dim3(grid), dim3(IN_THREADS), 0, st, B, u, y,
                         done, per_xcd, err);
    else
      hipLaunchKernelGGL((k_inner_cg<double, false>), dim3(grid), dim3(IN_THREADS), 0, st, B, u,
                         y, done, per_xcd, err);
    return hipGetLastError();
  }
  // Workgroups of a block wait for each other: launch cooperatively so that
  // the whole grid is resident.
  InnerBlocks Bc = B;
  int nsl = per_xcd;
  void* args[] = {&Bc, (void*)&u, (void*)&y, (void*)&done, &nsl, &err};
  if (mixed)
    return hipLaunchCooperativeKernel((const void*)k_inner_cg<float, true>, dim3(grid),
                                      dim3(IN_THREADS), args, 0, st);
  return hipLaunchCooperativeKernel((const void*)k_inner_cg<double, true>, dim3(grid),
                                    dim3(IN_THREADS), args, 0, st);
}

int inner_max_resident_groups(bool mixed) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  hipError_t e = mixed ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &per_cu, (const void*)k_inner_cg<float, true>, IN_THREADS, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                             &per_cu, (const void*)k_inner_cg<double, true>, IN_THREADS, 0);
  if (e != hipSuccess) return 0;
  return per_cu * ncu;
}
