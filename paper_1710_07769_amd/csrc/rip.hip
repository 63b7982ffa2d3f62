// Row inner-product graph G_RIP(A) (Sections 2.1 and 2.3 of the paper).
//
// Edges are the nonzero off-diagonal entries of C = A~ A~^T and costs their
// absolute values, where A~ is A with rows scaled to unit 2-norm and every
// dense column (more than isqrt(n) entries) cut down to its isqrt(n) largest
// entries.  C is built row by row (Gustavson): row i of C accumulates
// a~_ik * a~_jk over the entries k of row i (ascending) and the entries j of
// column k.  Bit-exactness: row norms sum the squares in ascending column
// order; each product is rounded before it is added (fp contraction is off in
// this file), and c_ij receives its products in ascending k, because the
// wavefront owning row i walks k in order and, for one k, every j is distinct.
#pragma clang fp contract(off)

#include "common.h"

#include <cmath>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace {

constexpr int RIP_WAVES = 4;                 // wavefronts per workgroup (one row each)
constexpr int TBL = 1024;                    // LDS hash slots per wavefront
constexpr int SHORT_MAX = 768;               // rows with at most this many products use LDS

__device__ __forceinline__ unsigned hash_key(int j) { return (unsigned)j * 2654435761u; }

// ---------------------------------------------------------------- prescale
// norm_i = sqrt(sum_k a_ik^2) in ascending k; a~ = a / norm (row CSR and
// transposed copy).  zero_row is set if some row has norm 0.
__global__ void k_rownorm(int n, const int* __restrict__ rowptr, const double* __restrict__ val,
                          double* __restrict__ nrm, int* __restrict__ zero_row) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const double a = val[e];
    const double sq = a * a;
    s = s + sq;
  }
  const double r = sqrt(s);
  nrm[i] = r;
  if (r == 0.0) atomicExch(zero_row, 1);
}

__global__ void k_scale_rows(int n, const int* __restrict__ rowptr, double* __restrict__ val,
                             const double* __restrict__ nrm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = nrm[i];
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) val[e] = val[e] / d;
}

// ------------------------------------------------------------- transpose
// A^T by a stable sort of the entries by column: within a column the entries
// keep the row-major order of A, i.e. ascending rows.
__global__ void k_entry_rows(int n, const int* __restrict__ rowptr, int* __restrict__ erow) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) erow[e] = i;
}

__global__ void k_col_count(long long nnz, const int* __restrict__ col, int* __restrict__ cnt) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  atomicAdd(&cnt[col[e]], 1);
}

__global__ void k_iota(long long nnz, int* __restrict__ v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) v[e] = (int)e;
}

// transposed entry f is A's entry tpos[f]: its row and (scaled) value
__global__ void k_transpose_gather(long long nnz, const int* __restrict__ tpos,
                                   const int* __restrict__ erow, const double* __restrict__ aval,
                                   int* __restrict__ trow, double* __restrict__ tval) {
  const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nnz) return;
  const int e = tpos[f];
  trow[f] = erow[e];
  tval[f] = aval[e];
}

// columns with more than t entries, appended in any order (each is sparsified
// on its own)
__global__ void k_dense_cols(int n, const int* __restrict__ tptr, int t, int* __restrict__ dense,
                             int* __restrict__ ndense) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (tptr[k + 1] - tptr[k] > t) dense[atomicAdd(ndense, 1)] = k;
}

// counts widened to 64 bits with a zero appended (input of the offsets scan)
__global__ void k_widen(int n, const int* __restrict__ c, long long* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = c[i];
  if (i == n) w[i] = 0;
}

// --------------------------------------------------------------- sparsify
// For column k with more than t entries: entry f is kept iff fewer than t
// entries precede it in the order (|a| descending, row ascending).  Dropped
// entries are zeroed in both copies (a zero entry contributes nothing to any
// sum; the transposed lists are then compacted).
__global__ void k_sparsify(const int* __restrict__ dense_cols, int t, const int* __restrict__ tptr,
                           const int* __restrict__ trow, double* __restrict__ tval,
                           const int* __restrict__ tpos, double* __restrict__ aval) {
  const int k = dense_cols[blockIdx.x];
  const int f0 = tptr[k], f1 = tptr[k + 1];
  for (int f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
    const double mine = fabs(tval[f]);
    const int myrow = trow[f];
    int before = 0;
    for (int g = f0; g < f1; ++g) {
      const double o = fabs(tval[g]);
      before += (o > mine) || (o == mine && trow[g] < myrow);
    }
    if (before >= t) aval[tpos[f]] = 0.0;
  }
  __syncthreads();
  for (int f = f0 + threadIdx.x; f < f1; f += blockDim.x)
    if (aval[tpos[f]] == 0.0) tval[f] = 0.0;
}

// count of nonzero entries per column (for compaction), cnt[n] = 0
__global__ void k_col_nonzeros(int n, const int* __restrict__ tptr, const double* __restrict__ tval,
                               int* __restrict__ cnt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == n) cnt[n] = 0;
  if (k >= n) return;
  int c = 0;
  for (int f = tptr[k]; f < tptr[k + 1]; ++f) c += tval[f] != 0.0;
  cnt[k] = c;
}

__global__ void k_compact_cols(int n, const int* __restrict__ tptr, const int* __restrict__ trow,
                               const double* __restrict__ tval, const int* __restrict__ cptr,
                               int* __restrict__ crow, double* __restrict__ cval) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int o = cptr[k];
  for (int f = tptr[k]; f < tptr[k + 1]; ++f)
    if (tval[f] != 0.0) {
      crow[o] = trow[f];
      cval[o] = tval[f];
      ++o;
    }
}

// number of products of each row (upper bound of its distinct columns)
__global__ void k_row_products(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                               const double* __restrict__ aval, const int* __restrict__ cptr,
                               long long* __restrict__ ub) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  long long s = 0;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e)
    if (aval[e] != 0.0) s += cptr[col[e] + 1] - cptr[col[e]];
  ub[i] = s;
}

// --------------------------------------------------------------- products
// Accumulate row i of C into the hash table (keys -1 = empty) by one wavefront.
__device__ __forceinline__ void accumulate_row(int i, const int* __restrict__ rowptr,
                                               const int* __restrict__ col,
                                               const double* __restrict__ aval,
                                               const int* __restrict__ cptr,
                                               const int* __restrict__ crow,
                                               const double* __restrict__ cval, int* keys,
                                               double* vals, unsigned mask) {
  const int lane = threadIdx.x & 63;
  for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const double a = aval[e];
    if (a == 0.0) continue;
    const int k = col[e];
    for (int f = cptr[k] + lane; f < cptr[k + 1]; f += 64) {
      const int j = crow[f];
      const double prod = a * cval[f];
      unsigned h = hash_key(j) & mask;
      while (true) {
        const int old = atomicCAS(&keys[h], -1, j);
        if (old == -1 || old == j) break;
        h = (h + 1) & mask;
      }
      vals[h] = vals[h] + prod;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }
}

__device__ __forceinline__ bool is_edge(int key, int i, double v) { return key >= 0 && key != i && v != 0.0; }

// Pass 1 (count) or pass 2 (emit sorted) for rows whose products fit the LDS table.
template <bool EMIT>
__global__ void __launch_bounds__(64 * RIP_WAVES)
k_rip_short(const int* __restrict__ rows, int nrows, const int* __restrict__ rowptr,
            const int* __restrict__ col, const double* __restrict__ aval,
            const int* __restrict__ cptr, const int* __restrict__ crow,
            const double* __restrict__ cval, int* __restrict__ cnt,
            const long long* __restrict__ optr, int* __restrict__ ocol, double* __restrict__ ocost,
            long long* __restrict__ owgt, double alpha, int* __restrict__ overflow) {
  __shared__ int keys_sh[RIP_WAVES][TBL];
  __shared__ double vals_sh[RIP_WAVES][TBL];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int idx = blockIdx.x * RIP_WAVES + w;
  if (idx >= nrows) return;
  const int i = rows[idx];
  int* keys = keys_sh[w];
  double* vals = vals_sh[w];
  for (int s = lane; s < TBL; s += 64) {
    keys[s] = -1;
    vals[s] = 0.0;
  }
  __builtin_amdgcn_wave_barrier();
  accumulate_row(i, rowptr, col, aval, cptr, crow, cval, keys, vals, TBL - 1);
  __builtin_amdgcn_wave_barrier();
  if (!EMIT) {
    int c = 0;
    for (int s = lane; s < TBL; s += 64) c += is_edge(keys[s], i, vals[s]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if (lane == 0) cnt[i] = c;
    return;
  }
  // compact the edges to the front of the table (order by slot), then sort by key
  int myc = 0;
  int mk[TBL / 64];
  double mv[TBL / 64];
#pragma unroll
  for (int q = 0; q < TBL / 64; ++q) {
    const int s = q * 64 + lane;
    mk[q] = keys[s];
    mv[q] = vals[s];
    myc += is_edge(mk[q], i, mv[q]);
  }
  // exclusive prefix over lanes
  int incl = myc;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const int total = __shfl(incl, 63, 64);
  int pos = incl - myc;
  __builtin_amdgcn_wave_barrier();
  for (int s = lane; s < TBL; s += 64) keys[s] = 0x7fffffff;
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < TBL / 64; ++q)
    if (is_edge(mk[q], i, mv[q])) {
      keys[pos] = mk[q];
      vals[pos] = mv[q];
      ++pos;
    }
  __builtin_amdgcn_wave_barrier();
  int sz = 1;
  while (sz < total) sz <<= 1;
  // bitonic sort of keys[0..sz) (padding keys are INT_MAX)
  for (int k2 = 2; k2 <= sz; k2 <<= 1) {
    for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
      for (int a = lane; a < sz; a += 64) {
        const int bidx = a ^ j2;
        if (bidx > a) {
          const bool up = (a & k2) == 0;
          const int ka = keys[a], kb = keys[bidx];
          if ((ka > kb) == up) {
            keys[a] = kb;
            keys[bidx] = ka;
            const double t = vals[a];
            vals[a] = vals[bidx];
            vals[bidx] = t;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
  }
  const long long o0 = optr[i];
  for (int a = lane; a < total; a += 64) {
    const double c = fabs(vals[a]);
    const double sc = c * alpha;
    ocol[o0 + a] = keys[a];
    ocost[o0 + a] = c;
    if (!(sc < 4611686018427387904.0)) atomicExch(overflow, 1);
    owgt[o0 + a] = (long long)ceil(sc);
  }
}

// Long rows: one workgroup per row with a table in global memory
// (size a power of two >= 2 * products), then a bitonic sort there.
template <bool EMIT>
__global__ void __launch_bounds__(256)
k_rip_long(const int* __restrict__ rows, const long long* __restrict__ toff,
           const int* __restrict__ tsize, const int* __restrict__ rowptr,
           const int* __restrict__ col, const double* __restrict__ aval,
           const int* __restrict__ cptr, const int* __restrict__ crow,
           const double* __restrict__ cval, int* __restrict__ gkeys, double* __restrict__ gvals,
           int* __restrict__ cnt, const long long* __restrict__ optr, int* __restrict__ ocol,
           double* __restrict__ ocost, long long* __restrict__ owgt, double alpha,
           int* __restrict__ overflow) {
  __shared__ int total_sh;
  const int i = rows[blockIdx.x];
  const int T = tsize[blockIdx.x];
  int* keys = gkeys + toff[blockIdx.x];
  double* vals = gvals + toff[blockIdx.x];
  for (int s = threadIdx.x; s < T; s += blockDim.x) {
    keys[s] = -1;
    vals[s] = 0.0;
  }
  __threadfence_block();
  __syncthreads();
  // the whole accumulation by wavefront 0 keeps the ascending-k order simple
  if (threadIdx.x < 64) accumulate_row(i, rowptr, col, aval, cptr, crow, cval, keys, vals, T - 1);
  __threadfence_block();
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int s = 0; s < T; ++s) {
      if (is_edge(keys[s], i, vals[s])) {
        keys[c] = keys[s];
        vals[c] = vals[s];
        ++c;
      }
    }
    for (int s = c; s < T; ++s) keys[s] = 0x7fffffff;
    total_sh = c;
    if (!EMIT) cnt[i] = c;
  }
  __threadfence_block();
  __syncthreads();
  if (!EMIT) return;
  const int total = total_sh;
  int sz = 1;
  while (sz < total) sz <<= 1;
  for (int k2 = 2; k2 <= sz; k2 <<= 1) {
    for (int j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
      for (int a = threadIdx.x; a < sz; a += blockDim.x) {
        const int bidx = a ^ j2;
        if (bidx > a) {
          const bool up = (a & k2) == 0;
          const int ka = keys[a], kb = keys[bidx];
          if ((ka > kb) == up) {
            keys[a] = kb;
            keys[bidx] = ka;
            const double t = vals[a];
            vals[a] = vals[bidx];
            vals[bidx] = t;
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
  }
  const long long o0 = optr[i];
  for (int a = threadIdx.x; a < total; a += blockDim.x) {
    const double c = fabs(vals[a]);
    const double sc = c * alpha;
    ocol[o0 + a] = keys[a];
    ocost[o0 + a] = c;
    if (!(sc < 4611686018427387904.0)) atomicExch(overflow, 1);
    owgt[o0 + a] = (long long)ceil(sc);
  }
}

}  // namespace

// ------------------------------------------------------------ launchers

hipError_t rip_launch_prescale(hipStream_t st, int n, const int* rowptr, double* aval,
                               double* nrm, int* zero_row) {
  hipLaunchKernelGGL(k_rownorm, dim3((n + 255) / 256), dim3(256), 0, st, n, rowptr, aval, nrm,
                     zero_row);
  hipLaunchKernelGGL(k_scale_rows, dim3((n + 255) / 256), dim3(256), 0, st, n, rowptr, aval, nrm);
  return hipGetLastError();
}

// Temporary bytes of rip_launch_transpose's column sort and of the scans.
size_t rip_transpose_temp_bytes(int n, long long nnz) {
  size_t sort = 0, scan = 0;
  (void)rocprim::radix_sort_pairs(nullptr, sort, (const unsigned*)nullptr, (unsigned*)nullptr,
                                  (const int*)nullptr, (int*)nullptr, (size_t)nnz, 0, 32);
  (void)rocprim::exclusive_scan(nullptr, scan, (const int*)nullptr, (int*)nullptr, 0,
                                (size_t)n + 1, rocprim::plus<int>());
  return std::max<size_t>(std::max(sort, scan), 256);
}

size_t rip_offsets_temp_bytes(int n) {
  size_t scan = 0;
  (void)rocprim::exclusive_scan(nullptr, scan, (const long long*)nullptr, (long long*)nullptr,
                                0LL, (size_t)n + 1, rocprim::plus<long long>());
  return std::max<size_t>(scan, 256);
}

// A^T of the n x n CSR matrix on the device: tptr (n+1), and per transposed
// entry its row trow, value tval and position tpos in A.  Scratch: erow,
// tkey, iota (nnz each), tcnt (n+1, zeroed here), temp (temp_bytes).
hipError_t rip_launch_transpose(hipStream_t st, int n, long long nnz, const int* rowptr,
                                const int* col, const double* aval, int* erow, unsigned* tkey,
                                int* iota, int* tcnt, int* tptr, int* trow, double* tval,
                                int* tpos, void* temp, size_t temp_bytes) {
  const unsigned gn = (unsigned)((nnz + 255) / 256);
  hipError_t e = hipMemsetAsync(tcnt, 0, ((size_t)n + 1) * sizeof(int), st);
  if (e != hipSuccess) return e;
  if (nnz > 0) {
    hipLaunchKernelGGL(k_entry_rows, dim3((n + 255) / 256), dim3(256), 0, st, n, rowptr, erow);
    hipLaunchKernelGGL(k_col_count, dim3(gn), dim3(256), 0, st, nnz, col, tcnt);
    hipLaunchKernelGGL(k_iota, dim3(gn), dim3(256), 0, st, nnz, iota);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned bits = 1;
    while (bits < 32 && (1u << bits) < (unsigned)n) ++bits;
    size_t tb = temp_bytes;
    e = rocprim::radix_sort_pairs(temp, tb, (const unsigned*)col, tkey, (const int*)iota, tpos,
                                  (size_t)nnz, 0, bits, st);
    if (e != hipSuccess) return e;
  }
  size_t tb = temp_bytes;
  e = rocprim::exclusive_scan(temp, tb, (const int*)tcnt, tptr, 0, (size_t)n + 1,
                              rocprim::plus<int>(), st);
  if (e != hipSuccess) return e;
  if (nnz > 0)
    hipLaunchKernelGGL(k_transpose_gather, dim3(gn), dim3(256), 0, st, nnz, tpos, erow, aval, trow,
                       tval);
  return hipGetLastError();
}

hipError_t rip_launch_dense_cols(hipStream_t st, int n, const int* tptr, int t, int* dense,
                                 int* ndense) {
  hipLaunchKernelGGL(k_dense_cols, dim3((n + 255) / 256), dim3(256), 0, st, n, tptr, t, dense,
                     ndense);
  return hipGetLastError();
}

hipError_t rip_launch_sparsify(hipStream_t st, const int* dense_cols, int ndense, int t,
                               const int* tptr, const int* trow, double* tval, const int* tpos,
                               double* aval) {
  if (ndense == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sparsify, dim3(ndense), dim3(256), 0, st, dense_cols, t, tptr, trow, tval,
                     tpos, aval);
  return hipGetLastError();
}

// cptr = exclusive scan of the n+1 counts (the last one zero)
hipError_t rip_launch_scan_int(hipStream_t st, const int* cnt, int* out, int n, void* temp,
                               size_t temp_bytes) {
  size_t tb = temp_bytes;
  return rocprim::exclusive_scan(temp, tb, cnt, out, 0, (size_t)n + 1, rocprim::plus<int>(), st);
}

// row offsets of the graph: exclusive scan of the per-row edge counts in 64 bits
hipError_t rip_launch_offsets(hipStream_t st, const int* cnt, long long* wide, long long* optr,
                              int n, void* temp, size_t temp_bytes) {
  hipLaunchKernelGGL(k_widen, dim3((n + 256) / 256), dim3(256), 0, st, n, cnt, wide);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t tb = temp_bytes;
  return rocprim::exclusive_scan(temp, tb, (const long long*)wide, optr, 0LL, (size_t)n + 1,
                                 rocprim::plus<long long>(), st);
}

hipError_t rip_launch_col_nonzeros(hipStream_t st, int n, const int* tptr, const double* tval,
                                   int* cnt) {
  hipLaunchKernelGGL(k_col_nonzeros, dim3((n + 256) / 256), dim3(256), 0, st, n, tptr, tval, cnt);
  return hipGetLastError();
}

hipError_t rip_launch_compact(hipStream_t st, int n, const int* tptr, const int* trow,
                              const double* tval, const int* cptr, int* crow, double* cval) {
  hipLaunchKernelGGL(k_compact_cols, dim3((n + 255) / 256), dim3(256), 0, st, n, tptr, trow, tval,
                     cptr, crow, cval);
  return hipGetLastError();
}

hipError_t rip_launch_row_products(hipStream_t st, int n, const int* rowptr, const int* col,
                                   const double* aval, const int* cptr, long long* ub) {
  hipLaunchKernelGGL(k_row_products, dim3((n + 255) / 256), dim3(256), 0, st, n, rowptr, col,
                     aval, cptr, ub);
  return hipGetLastError();
}

hipError_t rip_launch_short(hipStream_t st, bool emit, const int* rows, int nrows,
                            const int* rowptr, const int* col, const double* aval,
                            const int* cptr, const int* crow, const double* cval, int* cnt,
                            const long long* optr, int* ocol, double* ocost, long long* owgt,
                            double alpha, int* overflow) {
  if (nrows == 0) return hipSuccess;
  const int grid = (nrows + RIP_WAVES - 1) / RIP_WAVES;
  if (emit)
    hipLaunchKernelGGL(k_rip_short<true>, dim3(grid), dim3(64 * RIP_WAVES), 0, st, rows, nrows,
                       rowptr, col, aval, cptr, crow, cval, cnt, optr, ocol, ocost, owgt, alpha,
                       overflow);
  else
    hipLaunchKernelGGL(k_rip_short<false>, dim3(grid), dim3(64 * RIP_WAVES), 0, st, rows, nrows,
                       rowptr, col, aval, cptr, crow, cval, cnt, optr, ocol, ocost, owgt, alpha,
                       overflow);
  return hipGetLastError();
}

hipError_t rip_launch_long(hipStream_t st, bool emit, const int* rows, int nrows,
                           const long long* toff, const int* tsize, const int* rowptr,
                           const int* col, const double* aval, const int* cptr, const int* crow,
                           const double* cval, int* gkeys, double* gvals, int* cnt,
                           const long long* optr, int* ocol, double* ocost, long long* owgt,
                           double alpha, int* overflow) {
  if (nrows == 0) return hipSuccess;
  if (emit)
    hipLaunchKernelGGL(k_rip_long<true>, dim3(nrows), dim3(256), 0, st, rows, toff, tsize, rowptr,
                       col, aval, cptr, crow, cval, gkeys, gvals, cnt, optr, ocol, ocost, owgt,
                       alpha, overflow);
  else
    hipLaunchKernelGGL(k_rip_long<false>, dim3(nrows), dim3(256), 0, st, rows, toff, tsize,
                       rowptr, col, aval, cptr, crow, cval, gkeys, gvals, cnt, optr, ocol, ocost,
                       owgt, alpha, overflow);
  return hipGetLastError();
}

int rip_short_max() { return SHORT_MAX; }
