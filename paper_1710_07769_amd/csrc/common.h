// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bc.h"
#include "host.h"

// ------------------------------------------------------------------ errors

#define BC_HIP(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      bc_set_error(std::string(#call " failed: ") + hipGetErrorString(e_));            \
      return BC_ERR_DEVICE;                                                            \
    }                                                                                  \
  } while (0)

// ------------------------------------------------------------ device memory

// Owning device buffer; released with the context.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// ------------------------------------------------------------------ layout
constexpr int VEC_THREADS = 256;
static_assert(TILE % VEC_THREADS == 0, "a tile is a whole number of rows per thread");
// Dense projection tile edge (tiles of the packed lower-triangular factor).
constexpr int DT = 64;

// Per-solve device state shared by the outer-iteration kernels.
struct OuterState {
  int nsys;
  int ntiles;
  const int* tile_start;   // ntiles + 1 row/column offsets
  const int* tile_sys;     // system of each tile
  const int* sys_tile;     // nsys + 1 tile offsets
  int* done;               // per system: 1 once finished (converged, maxit, breakdown)
  int* iters;              // per system: outer iterations done
  int* status;             // per system: bc_status
  double* thr;             // per system: stop threshold on ||s||^2 (tol^2 ||f||^2)
  int maxit;
  double* part_a;          // ntiles partial sums (p.psi)
  double* part_b;          // ntiles partial sums (r.r)
  double* part_c;          // ntiles partial sums (s.s)
  double* rr;              // per system r.r of the current iterate
  double* hist;            // per system ||s||^2 of the last iteration (may be null)
  int* pending;            // per system stop decision of the last k_update_p (1 conv, 2 maxit)
  int use_backward;        // 1: stop when gamma < tol_bw (eq. (stopping)) instead of ||s||^2 <= thr
  double tol_bw;
  double* part_d;          // ntiles partial max |s|
  double* part_e;          // ntiles partial sum |x|
  double* part_g;          // ntiles partial max |f|
  const double* normA;     // per system ||A||_inf
  double* finf;            // per system ||f||_inf
  int rec_stop;            // 1: k_update_p may stop on the recursively updated s
};

// Sliced-ELL copy of a sparse matrix for the sparse products (built when
// its padding is modest; layout as build_sell in host.h).
struct SellMat {
  const long long* ptr;   // ntiles * SELL_SLICES entry offsets
  const int* wid;         // ntiles * SELL_SLICES widths
  const int* col;
  const double* val;
  const float* val32;     // FP32 copy for FP32 products, else null
  int il;                 // multi-vector products gather an interleaved copy
};

// ---------------------------------------------------------- device helpers
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

__device__ __forceinline__ double wave_sum_lane0(double v) {
  // Butterfly over the 64 lanes; lane 0's association order is the same in
  // every wavefront, so taking lane 0 makes the result deterministic.
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return __shfl(v, 0, 64);
}

// Sum of the partials of one system, in a fixed order, computed by one
// wavefront (every lane returns the same value).
__device__ __forceinline__ double sys_sum_wave(const double* part, int t0, int t1) {
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  // each lane adds part[t0 + lane + 64 k] for k = 0, 1, ... in that order; the
  // loads of 8 consecutive k are issued together (past t1 a lane reloads the
  // last partial and does not add it), not one round trip per partial
  for (int t = t0 + lane; t < t1; t += 64 * 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = part[min(t + 64 * q, t1 - 1)];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (t + 64 * q < t1) acc += v[q];
  }
  return wave_sum_lane0(acc);
}

// Serial fixed-order sum / max of a system's partials (one thread).
__device__ __forceinline__ double sys_sum_serial(const double* part, int t0, int t1) {
  double a = 0.0;
  for (int t = t0; t < t1; ++t) a += part[t];
  return a;
}
__device__ __forceinline__ double sys_max_serial(const double* part, int t0, int t1) {
  double a = 0.0;
  for (int t = t0; t < t1; ++t) a = fmax(a, part[t]);
  return a;
}

// Workgroup max of non-negative values; all threads get the result.
__device__ __forceinline__ double block_max(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t = fmax(t, sh[i]);
  return t;
}

// Workgroup sum (blockDim.x a multiple of 64, at most 1024); all threads get
// the result.  `sh` must hold blockDim.x/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum_lane0(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  return t;
}

// Two block sums at the cost of one (sh holds 2 * waves doubles).
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  a = wave_sum_lane0(a);
  b = wave_sum_lane0(b);
  __syncthreads();
  if (lane == 0) {
    sh[w] = a;
    sh[nw + w] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int i = 0; i < nw; ++i) {
    ta += sh[i];
    tb += sh[nw + i];
  }
  a = ta;
  b = tb;
}

#endif

// ------------------------------------------------------- kernel launchers
// (defined in the .hip files; all return hipError_t of the launch)

hipError_t launch_spmv(int lanes, hipStream_t st, const int* rowptr, const int* col,
                       const double* val, const float* val32, bool mixed, const double* x,
                       double* y, const OuterState& S, bool skip_done);
hipError_t launch_spmvT_dot(int lanes, hipStream_t st, const int* tptr, const int* trow,
                            const double* tval, const float* tval32, bool mixed, const double* y,
                            double* psi, const double* p, const OuterState& S);
hipError_t launch_residual(int lanes, hipStream_t st, const int* rowptr, const int* col,
                           const double* val, const double* x, const double* fperm, double* s,
                           const OuterState& S, const int* mask);
hipError_t launch_update_xrs(hipStream_t st, double* x, double* r, double* s, const double* p,
                             const double* psi, const double* u, const OuterState& S);
hipError_t launch_update_p(hipStream_t st, double* p, const double* r, const OuterState& S);
hipError_t launch_init_cg(hipStream_t st, double* p, const double* r, const OuterState& S);
hipError_t launch_rr_from_partials(hipStream_t st, const OuterState& S);
hipError_t launch_stamp(hipStream_t st, unsigned long long* t, int i);
hipError_t launch_replace_decide(hipStream_t st, const OuterState& S, int* restart, double* p,
                                 const double* r);
hipError_t launch_true_check(hipStream_t st, const OuterState& S);
hipError_t launch_init_norms(hipStream_t st, const double* f, const double* s, const double* x,
                             double* part_f, const OuterState& S);
hipError_t launch_final_stats(hipStream_t st, const double* part_f, const OuterState& S,
                              double* out);
hipError_t launch_cimmino_check(hipStream_t st, const OuterState& S);
hipError_t launch_cimmino_update(hipStream_t st, double* x, const double* psi, double omega,
                                 const OuterState& S);
hipError_t launch_spmv_sell(hipStream_t st, const SellMat& A, bool mixed, const double* x,
                            double* y, const OuterState& S, bool skip_done);
hipError_t launch_spmvT_dot_sell(hipStream_t st, const SellMat& AT, bool mixed, const double* y,
                                 double* psi, const double* p, const OuterState& S);
hipError_t launch_residual_sell(hipStream_t st, const SellMat& A, const double* x, const double* f,
                                double* s, const OuterState& S, const int* mask);
// Multiple right-hand sides of one system: nrhs vectors of n1 entries,
// concatenated; the one-vector tiling is tile_start (ntiles1 + 1 offsets).
// The OuterState passed with it is that of nrhs systems of ntiles1 tiles.
struct MultiRhs {
  int nrhs;
  int n1;
  int ntiles1;
  const int* tile_start;
  double* il;  // scratch for the gathered input, interleaved per chunk of vectors
};
// Vectors per chunk of the multi-vector sparse products: one 64-byte gather
// per index of the interleaved input; il holds ceil(nrhs / 8) * 8 * n1 doubles.
constexpr int SELL_MULTI_NR = 8;
// Block CG on H: products of short lists of n-vectors (column k at v[k]).
constexpr int BG_MAX = 32;       // columns per list (16 for combine outputs)
constexpr int BG_ROWS = 128;     // rows per Gram tile
constexpr int BG_LD = BG_ROWS + 1;  // LDS column stride of a Gram tile
constexpr int BG_THREADS = 256;
constexpr int BG_PAIRS = 1024;   // c1 * c2 at most
constexpr int BG_GROUPS = 512;   // Gram workgroups (partials per pair)
struct ColList {
  double* v[BG_MAX];
  int c;
};
// Lets the Gram kernel stage two full lists (once, before its first use).
hipError_t prepare_block_gram();
// out[a * c2 + b] = L1_a . L2_b (device, c1*c2 doubles); part: BG_GROUPS * c1 * c2.
hipError_t launch_block_gram(hipStream_t st, const ColList& L1, const ColList& L2, int n,
                             double* part, double* out);
// out_j = base_j + sum_k in_k coef[k * out.c + j] (base.c = 0: no base term;
// base may list the output vectors themselves).
hipError_t launch_block_combine(hipStream_t st, const ColList& in, const ColList& out,
                                const ColList& base, const double* coef, int n);
hipError_t launch_spmv_sell_multi(hipStream_t st, const SellMat& A, const MultiRhs& M, bool mixed,
                                  const double* x, double* y, const OuterState& S, bool skip_done);
hipError_t launch_spmvT_dot_sell_multi(hipStream_t st, const SellMat& AT, const MultiRhs& M,
                                       bool mixed, const double* y, double* psi, const double* p,
                                       const OuterState& S);
hipError_t launch_residual_sell_multi(hipStream_t st, const SellMat& A, const MultiRhs& M,
                                      const double* x, const double* f, double* s,
                                      const OuterState& S, const int* mask);
hipError_t launch_gather(hipStream_t st, const double* src, const int* idx, double* dst, int n);
hipError_t launch_sqnorm_tiles(hipStream_t st, const double* v, double* part, const OuterState& S);
hipError_t launch_set_thresholds(hipStream_t st, const double* part_f, double tol, const OuterState& S);
hipError_t launch_copy(hipStream_t st, const double* src, double* dst, int n);
hipError_t launch_zero(hipStream_t st, double* dst, int n);

// Inner CG on the normal equations of the inner-CG blocks.
struct InnerBlocks {
  int nblk;                // number of inner-CG blocks
  const int* row0;         // first permuted row
  const int* m;            // rows
  const int* sup0;         // first support position
  const int* nsup;         // support size
  const int* sys;          // system of the block
  double* q; double* z; double* ri; double* t;   // scratch (rows / support)
  float* q32; float* z32; float* ri32; float* t32;
  unsigned long long* xp;  // per block 2 x 16 groups x 4 words: the (r,r), (w,r) partials
                           // of each workgroup as words {payload32, epoch32}
  unsigned* bar;           // per block barrier flags (epochs) and placement words
  int* iters;              // per block inner iterations of the last call
  unsigned long long* total; // running sum of inner iterations over blocks and calls
  unsigned long long* blk_total; // per block running sum of inner iterations
  double tol;
  int maxit;
  int groups;              // workgroups per block
  int max_m;               // largest block
  int max_nsup;            // largest support
  unsigned long long* trace; // optional phase timestamps (block 0), null when off
  int* err;                // the context's wait-error word: set to 1 when a workgroup gave up
                           // waiting for the others of its block (the result is then invalid)
  unsigned long long wait_ticks;  // bound of a wait, 100 MHz wall-clock ticks (0: give up at once)
  const double* dsc;       // per permuted row 1/||a_r||_2: the projections solve the
                           // scaled normal equations (D A_i A_i^T D) z = D u, y = D z
  // Sliced ELL copies of the scaled block rows (slices of 64 rows) and of
  // their transposes (slices of 64 support columns); entry k of lane l of
  // slice s at ptr[s] + 64 k + l; padding has index 0, value 0
  int idx16;               // indices stored as uint16 (else int32)
  const int* a_s0;         // per block first row slice
  const long long* a_ptr;  // per row slice entry offset
  const int* a_w;          // per row slice width
  const void* a_idx;       // support position of each entry
  const double* a_val;
  const float* a_val32;
  const int* t_s0;         // per block first column slice
  const long long* t_ptr;
  const int* t_w;
  const void* t_idx;       // local row of each entry
  const double* t_val;
  const float* t_val32;
};
// Precision of the inner CG: FP64 throughout; FP32 throughout (vectors,
// values, arithmetic); or FP64 vectors and arithmetic on the FP32 copies of
// the block matrix values.
enum InnerPrec { INNER_F64 = 0, INNER_F32 = 1, INNER_F64_V32 = 2 };
hipError_t launch_inner_cg(hipStream_t st, const InnerBlocks& B, InnerPrec prec, const double* u,
                           double* y, const int* done);
hipError_t launch_inner_cg_multi(hipStream_t st, const InnerBlocks& B, InnerPrec prec,
                                 const double* u, double* y, const int* done, int nrhs, int n1,
                                 int sup_total, void* rs, void* ts, bool* taken);

// Dense blocks: packed lower-triangular tiles of L (column-major 64x64 tiles)
struct DenseBlocks {
  int nblk;
  const int* row0;
  const int* m;
  const int* nt;           // tiles per side
  const long long* loff;   // offset (elements) of the block's packed L tiles
  const long long* doff;   // offset (elements) of the block's inverted diagonal tiles
  const int* sys;
  double* L;               // packed lower tiles, tile (i,j), i>=j, at loff + (i(i+1)/2+j)*DT*DT
  double* LT;              // packed transposed copy for the backward sweep: tile (i,j), j>=i
                           // holds (L_ji)^T at loff + (i*nt - i(i-1)/2 + (j-i))*DT*DT
  double* Dinv;            // inverted diagonal tiles L_kk^{-1}
  float* L32; float* LT32; float* Dinv32;
  int* info;               // per block: 0 ok, j+1 = first pivot at or below m*eps*G_jj
  double* gdiag;           // diagonal of every block's Gram matrix (permuted row index)
  unsigned long long* applies; // per block running count of applications
  const double* dsc;       // per permuted row 1/||a_r||_2 (see InnerBlocks)
  int* err;                // the context's wait-error word: set to 1 when a wave of a sweep
                           // gave up waiting (the result is then invalid)
  unsigned long long wait_ticks;  // bound of a wait, 100 MHz wall-clock ticks (0: give up at once)
};
// Blocked Cholesky: panels of CHOL_PW tile columns; per panel step s the
// (block, tile row) pairs of the panel solves and the (block, i, j) tiles of
// the trailing update, concatenated over the steps (offsets on the host).
constexpr int CHOL_PW = 4;
struct CholPlan {
  int steps;
  const int2* panel;
  const int4* upd;
  std::vector<long long> panel_off, upd_off;  // steps + 1 each
};
hipError_t launch_cholesky(hipStream_t st, const DenseBlocks& D, const CholPlan& P);
hipError_t launch_dense_finish(hipStream_t st, const DenseBlocks& D, bool mixed);
// Lets the apply kernels use the full LDS of a workgroup; call before the
// first apply (and outside stream capture).
hipError_t prepare_dense_apply();
// y_i = D L^{-T} L^{-1} D u_i on every dense block (done indexed by the
// block's system); max_nt: the largest tiles-per-side of the dense blocks.
hipError_t launch_dense_apply(hipStream_t st, const DenseBlocks& D, bool mixed, const double* u,
                              double* y, const int* done, int max_nt);
// The same apply to nrhs vectors of a one-system context at once (vector j at
// u + j*n1, y + j*n1; done indexed by j), in chunks whose z fits the LDS of
// one workgroup.  Every vector gets the bits it gets alone.
constexpr size_t DENSE_MULTI_LDS = 160 * 1024;
hipError_t launch_dense_apply_multi(hipStream_t st, const DenseBlocks& D, bool mixed,
                                    const double* u, double* y, const int* done, int nrhs, int n1,
                                    int max_nt);

// Banded blocks: rows of the block in reverse Cuthill-McKee order, so that the
// scaled normal-equation matrix G = D A_i A_i^T D has half-bandwidth bw.  The
// factor is stored per 64-row tile in diagonal-major order: entry d (0..bw)
// of local row p, i.e. L[p][p - bw + d], is at off + (p/64)*64*ld + d*64 +
// p%64, with ld = bw+1 rounded up to a multiple of 4 (entries left of column
// 0, entries d > bw and rows past m are zero; a tile is 64*ld contiguous
// values, a multiple of 16 bytes).  The sweeps read L and its reversed
// transpose R[p][k] = L[m-1-k][m-1-p] (the backward sweep with L^T is a
// forward sweep with R on reversed vectors) in a slot layout of the same size
// that puts the inverse of each tile's diagonal block in place of the
// in-tile entries (band.hip).
constexpr int BAND_MAX = 127;  // largest half-bandwidth (LDS window of the factorization)

struct BandBlocks {
  int nblk;
  const int* row0;
  const int* m;
  const int* bw;           // half-bandwidth per block
  const int* ld;           // stored entries per row (bw+1 rounded up to a multiple of 4)
  int ldmax;               // largest ld
  const int* order;        // blocks by decreasing m * sld: launch order of the sweeps
  const int* sys;
  const long long* off;    // element offset of the block's tiles in the band layout
  const int* sld;          // slots per row in the slot layout of the sweeps (>= ld)
  const long long* soff;   // element offset of the block's tiles in the slot layout
  int sldmax;              // largest sld
  double* L;               // Gram matrix on entry to the factorization, FP64 factor after (band layout)
  double* SL; double* SR;  // slot layout of L and of its reversed transpose (FP64 projections)
  float* SL32; float* SR32;// the same rounded to FP32 (FP32 projections)
  int* info;               // per block: 0 ok, j+1 = first pivot at or below m*eps*G_jj
  unsigned long long* applies; // per block running count of applications
  const double* dsc;       // per permuted row 1/||a_r||_2 (see InnerBlocks)
};
hipError_t launch_band_gram(hipStream_t st, const BandBlocks& B, const int* rowptr, const int* col,
                            const double* val, const int* tptr, const int* trow, const double* tval);
hipError_t launch_band_cholesky(hipStream_t st, const BandBlocks& B);
hipError_t launch_band_finish(hipStream_t st, const BandBlocks& B, bool mixed);
hipError_t launch_band_apply(hipStream_t st, const BandBlocks& B, bool mixed, const double* u,
                             double* y, const int* done);
hipError_t prepare_band_apply(const BandBlocks& B, bool mixed);
// The same sweeps for nrhs vectors of a one-system context at once (vector j
// at u + j*n1, y + j*n1; done indexed by j): chunks of 4 vectors per
// workgroup read each factor once.  Every vector gets the bits of
// launch_band_apply.
hipError_t launch_band_apply_multi(hipStream_t st, const BandBlocks& B, bool mixed,
                                   const double* u, double* y, const int* done, int nrhs, int n1);
