// C-ABI entry points: setup (validation, block permutation, transposes,
// per-block metadata, dense factorisation), projection and solve drivers,
// and the row inner-product graph builder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <cstdio>
#include <string>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "common.h"

// launchers defined in the other translation units
hipError_t launch_gram(hipStream_t st, const DenseBlocks& D, const int4* tiles, int ntiles,
                       const int* rowptr, const int* col, const double* val, const int* tptr,
                       const int* trow, const double* tval);
int inner_max_resident_groups(bool mixed);
int inner_grp_max_resident(bool f32_vectors, int max_m);
hipError_t rip_launch_prescale(hipStream_t st, int n, const int* rowptr, double* aval,
                               double* nrm, int* zero_row);
size_t rip_transpose_temp_bytes(int n, long long nnz);
size_t rip_offsets_temp_bytes(int n);
hipError_t rip_launch_transpose(hipStream_t st, int n, long long nnz, const int* rowptr,
                                const int* col, const double* aval, int* erow, unsigned* tkey,
                                int* iota, int* tcnt, int* tptr, int* trow, double* tval,
                                int* tpos, void* temp, size_t temp_bytes);
hipError_t rip_launch_dense_cols(hipStream_t st, int n, const int* tptr, int t, int* dense,
                                 int* ndense);
hipError_t rip_launch_sparsify(hipStream_t st, const int* dense_cols, int ndense, int t,
                               const int* tptr, const int* trow, double* tval, const int* tpos,
                               double* aval);
hipError_t rip_launch_col_nonzeros(hipStream_t st, int n, const int* tptr, const double* tval,
                                   int* cnt);
hipError_t rip_launch_scan_int(hipStream_t st, const int* cnt, int* out, int n, void* temp,
                               size_t temp_bytes);
hipError_t rip_launch_offsets(hipStream_t st, const int* cnt, long long* wide, long long* optr,
                              int n, void* temp, size_t temp_bytes);
hipError_t rip_launch_compact(hipStream_t st, int n, const int* tptr, const int* trow,
                              const double* tval, const int* cptr, int* crow, double* cval);
hipError_t rip_launch_row_products(hipStream_t st, int n, const int* rowptr, const int* col,
                                   const double* aval, const int* cptr, long long* ub);
hipError_t rip_launch_short(hipStream_t st, bool emit, const int* rows, int nrows,
                            const int* rowptr, const int* col, const double* aval,
                            const int* cptr, const int* crow, const double* cval, int* cnt,
                            const long long* optr, int* ocol, double* ocost, long long* owgt,
                            double alpha, int* overflow);
hipError_t rip_launch_long(hipStream_t st, bool emit, const int* rows, int nrows,
                           const long long* toff, const int* tsize, const int* rowptr,
                           const int* col, const double* aval, const int* cptr, const int* crow,
                           const double* cval, int* gkeys, double* gvals, int* cnt,
                           const long long* optr, int* ocol, double* ocost, long long* owgt,
                           double alpha, int* overflow);
int rip_short_max();


// ------------------------------------------------------------- helpers

namespace {

// Device allocations of one owner, released together.
struct Arena {
  std::vector<void*> ptrs;
  ~Arena() { release(); }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
  template <typename T>
  bc_status alloc(T** out, size_t count) {
    *out = nullptr;
    if (count == 0) count = 1;
    void* p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      bc_set_error("hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
      return BC_ERR_NOMEM;
    }
    ptrs.push_back(p);
    *out = (T*)p;
    return BC_OK;
  }
  template <typename T>
  bc_status upload(T** out, const std::vector<T>& v, hipStream_t st) {
    bc_status s = alloc(out, v.size());
    if (s != BC_OK) return s;
    if (!v.empty() &&
        hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess) {
      bc_set_error("host-to-device copy failed");
      return BC_ERR_DEVICE;
    }
    return BC_OK;
  }
};

#define BC_TRY(expr)             \
  do {                           \
    bc_status s_ = (expr);       \
    if (s_ != BC_OK) return s_;  \
  } while (0)

bool is_gfx950_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

bc_status check_device() {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    bc_set_error("no HIP device available");
    return BC_ERR_DEVICE;
  }
  if (!is_gfx950_device()) {
    bc_set_error("this library is built for gfx950 (MI355X) only");
    return BC_ERR_DEVICE;
  }
  return BC_OK;
}

struct SysIn {
  int32_t n;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  int32_t K;
  const int32_t* part;
};

// Per-vector state of a solve with several right-hand sides of a one-system
// context: the context's per-system arrays, tiles and work vectors for nrhs
// copies of its system.  swap_view exchanges them with the context's own for
// the duration of the solve, so the outer iteration runs unchanged on nrhs
// "systems" that share one matrix and one set of block factors.
struct MultiView {
  Arena arena;
  int nrhs = 0;
  int nsys = 0;
  int n_total = 0;
  std::vector<int> sys_off;
  std::vector<double> normA_inf;
  int* d_perm = nullptr;
  int ntiles = 0;
  int *d_tile_start = nullptr, *d_tile_sys = nullptr, *d_sys_tile = nullptr;
  int *d_done = nullptr, *d_zero_flags = nullptr, *d_iters = nullptr, *d_status = nullptr;
  int *d_pending = nullptr, *d_mask = nullptr, *d_restart = nullptr;
  double *d_thr = nullptr, *d_rr = nullptr, *d_hist = nullptr;
  double *d_part_a = nullptr, *d_part_b = nullptr, *d_part_c = nullptr, *d_part_f = nullptr;
  double *d_part_d = nullptr, *d_part_e = nullptr, *d_part_g = nullptr;
  double *d_final = nullptr, *d_normA = nullptr, *d_finf = nullptr;
  double *d_r = nullptr, *d_p = nullptr, *d_psi = nullptr;
  double *d_s = nullptr, *d_u = nullptr, *d_y = nullptr, *d_f = nullptr;
  // the sparse products' input, interleaved per chunk of 8 vectors
  double* d_il = nullptr;
  // inner CG of all vectors in one launch: residual and support scratch
  double *d_inner_r = nullptr, *d_inner_t = nullptr;
  // block CG only (allocated on its first call): the next directions Z,
  // Gram partials and results, and the coefficient matrices of the updates
  double *d_z = nullptr, *d_gpart = nullptr, *d_gout = nullptr, *d_coef = nullptr;
};

}  // namespace

// ------------------------------------------------------------------ context

struct bc_ctx {
  Arena arena;
  bc_opts opts;
  hipStream_t stream = nullptr;
  hipEvent_t ev_sync = nullptr;
  std::vector<hipEvent_t> ev_proj;  // pairs around projection launches
  int ev_used = 0;                  // pairs recorded since the last harvest
  double t_proj_ms = 0.0;           // harvested projection time of the current solve
  int proj_launches = 0;
  bool timing = false;
  bool noalloc = false;  // solve without any allocation (bc_solve_noalloc): no graphs, no events
  bool mixed = false;     // FP32 projections (BC_MIXED or BC_MIXED_PROJ)
  InnerPrec inner_prec = INNER_F64;
  bool spmv32 = false;    // FP32 sparse products (BC_MIXED)
  int nsys = 0;
  int n_total = 0;
  long long nnz_total = 0;
  int lanes = 4;      // lanes per row of A in the sparse products (u = A p, residuals)
  int lanesT = 4;     // lanes per row of A^T (psi = A^T y)
  std::vector<int> sys_off;        // nsys + 1
  std::vector<double> normA_inf;   // per system
  // permuted A and A^T
  int* d_perm = nullptr;           // permuted row -> original (global) row
  int* d_rowptr = nullptr;
  int* d_col = nullptr;
  double* d_val = nullptr;
  float* d_val32 = nullptr;
  int* d_tptr = nullptr;
  int* d_trow = nullptr;
  double* d_tval = nullptr;
  float* d_tval32 = nullptr;
  bool have_sell = false;          // sliced-ELL copies of A and A^T built
  SellMat sellA{}, sellT{};
  MultiRhs mrhs{};                 // nrhs > 0 while a multi-right-hand-side solve runs
  std::unique_ptr<MultiView> mview;
  // tiles
  int ntiles = 0;
  int* d_tile_start = nullptr;
  int* d_tile_sys = nullptr;
  int* d_sys_tile = nullptr;
  // per-system state
  int* d_done = nullptr;
  int* d_zero_flags = nullptr;
  int* d_iters = nullptr;
  int* d_status = nullptr;
  int* d_pending = nullptr;
  int* d_mask = nullptr;
  int* d_restart = nullptr;
  double* d_thr = nullptr;
  double* d_rr = nullptr;
  double* d_hist = nullptr;
  double *d_part_a = nullptr, *d_part_b = nullptr, *d_part_c = nullptr, *d_part_f = nullptr;
  double *d_part_d = nullptr, *d_part_e = nullptr, *d_part_g = nullptr;
  double* d_final = nullptr;  // per system 5 figures of the final residual (k_final_stats)
  double* d_normA = nullptr;
  double* d_finf = nullptr;
  // vectors
  double *d_r = nullptr, *d_p = nullptr, *d_psi = nullptr;
  double *d_s = nullptr, *d_u = nullptr, *d_y = nullptr, *d_f = nullptr;
  // blocks
  int nblk = 0;
  InnerBlocks inner{};
  int inner_sup_total = 0;         // support positions over the inner-CG blocks
  DenseBlocks dense{};
  BandBlocks band{};
  std::vector<long long> bd_m_h, bd_bw_h;  // per banded block rows and half-bandwidth
  std::vector<int> blk_kind, blk_bw;       // per block: 0 dense, 1 inner CG, 2 banded; bandwidth or -1
  unsigned long long* d_inner_total = nullptr;
  std::vector<int> blk_m;
  std::vector<long long> in_nnz, in_m_h, dn_m_h;  // per inner / dense block sizes
  int dense_max_nt = 0;                             // largest tiles per side of a dense block

  // Wait-error word of the bounded device waits (inner-CG workgroups, dense
  // sweep waves): cleared at the start of each call, read at its end.
  int* d_err = nullptr;
  unsigned long long wait_ticks = 0;  // bound of a wait in device wall-clock ticks (set at setup)

  // captured group of outer iterations (factor-based projections only)
  hipGraphExec_t gexec = nullptr;
  unsigned long long* d_stamps = nullptr;  // wall-clock stamps around the sweeps of a replay
  double wall_khz = 0.0;                    // rate of the device wall clock
  OuterState gS{};                 // state the graph was captured with
  double* gx = nullptr;            // solution vector the graph was captured with
  int gG = 0;                      // iterations per replay
  bool graph_off = false;          // capture failed once: plain launches from then on
  int graph_pending = 0;           // event pairs of the last replay not yet harvested

  ~bc_ctx() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (hipEvent_t e : ev_proj) (void)hipEventDestroy(e);
    if (ev_sync) (void)hipEventDestroy(ev_sync);
    if (stream) (void)hipStreamDestroy(stream);
  }

  OuterState outer(int maxit, int use_backward) const {
    OuterState S;
    S.nsys = nsys;
    S.ntiles = ntiles;
    S.tile_start = d_tile_start;
    S.tile_sys = d_tile_sys;
    S.sys_tile = d_sys_tile;
    S.done = d_done;
    S.iters = d_iters;
    S.status = d_status;
    S.thr = d_thr;
    S.maxit = maxit;
    S.part_a = d_part_a;
    S.part_b = d_part_b;
    S.part_c = d_part_c;
    S.rr = d_rr;
    S.hist = d_hist;
    S.pending = d_pending;
    S.use_backward = use_backward;
    S.tol_bw = 0.0;
    S.part_d = d_part_d;
    S.part_e = d_part_e;
    S.part_g = d_part_g;
    S.normA = d_normA;
    S.finf = d_finf;
    S.rec_stop = spmv32 ? 0 : 1;
    return S;
  }
};

namespace {

// Enter/leave the library stream in the order of the caller's stream.
bc_status enter(bc_ctx* c, void* user_stream) {
  BC_HIP(hipEventRecord(c->ev_sync, (hipStream_t)user_stream));
  BC_HIP(hipStreamWaitEvent(c->stream, c->ev_sync, 0));
  return BC_OK;
}
bc_status leave(bc_ctx* c, void* user_stream) {
  BC_HIP(hipEventRecord(c->ev_sync, c->stream));
  BC_HIP(hipStreamWaitEvent((hipStream_t)user_stream, c->ev_sync, 0));
  BC_HIP(hipStreamSynchronize(c->stream));
  return BC_OK;
}

// ---- rows-per-wavefront autotuner for the two sparse products.  Each
// candidate lane count L (lanes of a wave sharing one row, so 64/L rows per
// wavefront) is timed with HIP events on the library stream on the actual
// permuted matrix; the fastest L is kept for A and for A^T separately.  The
// choice is cached per sparsity pattern so that a matrix set up twice in a
// process gets the same schedule (and the same rounding).
struct LaneChoice {
  int a, t;
};
std::mutex g_tune_mu;
std::unordered_map<unsigned long long, LaneChoice> g_tune;

unsigned long long pattern_key(const std::vector<int>& rowptr, const std::vector<int>& col, int n,
                               bool fp32) {
  // every row pointer and column index, two 32-bit entries per 64-bit mix
  unsigned long long h = 0x243F6A8885A308D3ULL;
  auto mix = [&](unsigned long long v) {
    h ^= v + 0x9E3779B97F4A7C15ULL + (h << 6) + (h >> 2);
    h *= 0xBF58476D1CE4E5B9ULL;
    h ^= h >> 31;
  };
  mix((unsigned long long)n);
  mix((unsigned long long)col.size());
  mix(fp32 ? 1 : 0);
  auto mix_all = [&](const std::vector<int>& a) {
    size_t i = 0;
    for (; i + 1 < a.size(); i += 2)
      mix((unsigned long long)(unsigned)a[i] | ((unsigned long long)(unsigned)a[i + 1] << 32));
    if (i < a.size()) mix((unsigned long long)(unsigned)a[i]);
  };
  mix_all(rowptr);
  mix_all(col);
  return h;
}

// The three sparse products, on the CSR arrays with `lanes` lanes per row or
// on the sliced-ELL copies (lanes == LANES_SELL); during a solve with several
// right-hand sides, on the sliced-ELL copies for all vectors at once.
hipError_t spmv_a(const bc_ctx* c, hipStream_t st, int lanes, const double* x, double* y,
                  const OuterState& S, bool skip_done) {
  if (c->mrhs.nrhs > 0)
    return launch_spmv_sell_multi(st, c->sellA, c->mrhs, c->spmv32, x, y, S, skip_done);
  if (lanes == LANES_SELL) return launch_spmv_sell(st, c->sellA, c->spmv32, x, y, S, skip_done);
  return launch_spmv(lanes, st, c->d_rowptr, c->d_col, c->d_val, c->d_val32, c->spmv32, x, y, S,
                     skip_done);
}
hipError_t spmv_t(const bc_ctx* c, hipStream_t st, int lanes, const double* y, double* psi,
                  const double* p, const OuterState& S) {
  if (c->mrhs.nrhs > 0)
    return launch_spmvT_dot_sell_multi(st, c->sellT, c->mrhs, c->spmv32, y, psi, p, S);
  if (lanes == LANES_SELL) return launch_spmvT_dot_sell(st, c->sellT, c->spmv32, y, psi, p, S);
  return launch_spmvT_dot(lanes, st, c->d_tptr, c->d_trow, c->d_tval, c->d_tval32, c->spmv32, y,
                          psi, p, S);
}
hipError_t residual_a(const bc_ctx* c, hipStream_t st, int lanes, const double* x, const double* f,
                      double* s, const OuterState& S, const int* mask) {
  if (c->mrhs.nrhs > 0) return launch_residual_sell_multi(st, c->sellA, c->mrhs, x, f, s, S, mask);
  if (lanes == LANES_SELL) return launch_residual_sell(st, c->sellA, x, f, s, S, mask);
  return launch_residual(lanes, st, c->d_rowptr, c->d_col, c->d_val, x, f, s, S, mask);
}

bc_status autotune_lanes(bc_ctx* c, unsigned long long key) {
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      c->lanes = it->second.a;
      c->lanesT = it->second.t;
      return BC_OK;
    }
  }
  hipStream_t st = c->stream;
  const int n = c->n_total;
  BC_HIP(hipMemsetAsync(c->d_p, 0, (size_t)n * sizeof(double), st));
  BC_HIP(hipMemsetAsync(c->d_y, 0, (size_t)n * sizeof(double), st));
  OuterState S = c->outer(0, 0);
  S.done = c->d_zero_flags;
  hipEvent_t e0, e1;
  BC_HIP(hipEventCreate(&e0));
  BC_HIP(hipEventCreate(&e1));
  float best_a = 1e30f, best_t = 1e30f;
  int la = c->lanes, lt = c->lanesT;
  bc_status rc = BC_OK;
  std::vector<int> cand;
  for (int L = 1; L <= 64; L *= 2) cand.push_back(L);
  if (c->have_sell) cand.push_back(LANES_SELL);
  for (size_t ci = 0; ci < cand.size() && rc == BC_OK; ++ci) {
    const int L = cand[ci];
    for (int which = 0; which < 2 && rc == BC_OK; ++which) {
      float ms = 0.f;
      for (int rep = 0; rep < 4; ++rep) {
        if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = BC_ERR_DEVICE;
        hipError_t e = which == 0 ? spmv_a(c, st, L, c->d_p, c->d_u, S, false)
                                  : spmv_t(c, st, L, c->d_y, c->d_psi, c->d_p, S);
        if (e != hipSuccess) rc = BC_ERR_DEVICE;
      }
      if (rc != BC_OK || hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = BC_ERR_DEVICE;
        break;
      }
      if (which == 0 && ms < best_a) {
        best_a = ms;
        la = L;
      }
      if (which == 1 && ms < best_t) {
        best_t = ms;
        lt = L;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != BC_OK) {
    bc_set_error("sparse-product autotuning failed");
    return rc;
  }
  c->lanes = la;
  c->lanesT = lt;
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune[key] = LaneChoice{la, lt};
  return BC_OK;
}

enum { KIND_DENSE = 0, KIND_INNER = 1, KIND_BAND = 2 };
constexpr int BAND_MAX_ROWS = 65536;  // largest block considered for the banded form

// Reverse Cuthill-McKee order of the m rows rows[0..m) (global ids of system
// S, offset off) on the graph of A_i A_i^T (rows sharing a column).  Returns
// the half-bandwidth under that order and order[new] = old local index, or -1
// without an order when a row has more than 2 BAND_MAX neighbours (then no
// order can bring the bandwidth within BAND_MAX).  cid: scratch of size >= n
// filled with -1, restored on return.
int block_rcm(const SysIn& S, int off, const int* rows, int m, std::vector<int>& cid,
              std::vector<int>& order) {
  std::vector<int> touched;
  for (int l = 0; l < m; ++l) {
    const int r = rows[l] - off;
    for (int q = S.rowptr[r]; q < S.rowptr[r + 1]; ++q) {
      const int cc = S.col[q];
      if (cid[cc] < 0) {
        cid[cc] = (int)touched.size();
        touched.push_back(cc);
      }
    }
  }
  const int nc = (int)touched.size();
  std::vector<int> cptr(nc + 1, 0);
  for (int l = 0; l < m; ++l) {
    const int r = rows[l] - off;
    for (int q = S.rowptr[r]; q < S.rowptr[r + 1]; ++q) cptr[cid[S.col[q]] + 1]++;
  }
  for (int k = 0; k < nc; ++k) cptr[k + 1] += cptr[k];
  std::vector<int> crow(cptr[nc]);
  {
    std::vector<int> cur(cptr.begin(), cptr.end() - 1);
    for (int l = 0; l < m; ++l) {
      const int r = rows[l] - off;
      for (int q = S.rowptr[r]; q < S.rowptr[r + 1]; ++q) crow[cur[cid[S.col[q]]]++] = l;
    }
  }
  std::vector<int> xadj(m + 1, 0), adj, stamp(m, -1);
  bool too_wide = false;
  for (int l = 0; l < m && !too_wide; ++l) {
    const int r = rows[l] - off;
    for (int q = S.rowptr[r]; q < S.rowptr[r + 1]; ++q) {
      const int k = cid[S.col[q]];
      for (int e = cptr[k]; e < cptr[k + 1]; ++e) {
        const int l2 = crow[e];
        if (l2 != l && stamp[l2] != l) {
          stamp[l2] = l;
          adj.push_back(l2);
        }
      }
    }
    xadj[l + 1] = (int)adj.size();
    if (xadj[l + 1] - xadj[l] > 2 * BAND_MAX) too_wide = true;
  }
  for (int cc : touched) cid[cc] = -1;
  if (too_wide) return -1;
  order.resize(m);
  return bc_rcm_order(m, xadj.data(), adj.data(), order.data());
}

bc_status setup_impl(bc_ctx* c, const std::vector<SysIn>& sys) {
  const bc_opts& o = c->opts;
  c->mixed = o.precision == BC_MIXED || o.precision == BC_MIXED_PROJ;
  // inner CG: FP32 throughout with FP32 sparse products; with FP64 products
  // FP64 vectors and arithmetic on FP32 copies of the block matrices
  c->inner_prec = o.precision == BC_MIXED        ? INNER_F32
                  : o.precision == BC_MIXED_PROJ ? INNER_F64_V32
                                                 : INNER_F64;
  c->spmv32 = o.precision == BC_MIXED;
  c->nsys = (int)sys.size();
  // ---- sizes
  c->sys_off.assign(c->nsys + 1, 0);
  long long ntot = 0, nnz = 0;
  for (int s = 0; s < c->nsys; ++s) {
    ntot += sys[s].n;
    nnz += sys[s].rowptr[sys[s].n];
    c->sys_off[s + 1] = (int)std::min<long long>(ntot, INT32_MAX);
  }
  if (ntot > INT32_MAX / 2 || nnz > INT32_MAX) {
    bc_set_error("problem too large for 32-bit indices");
    return BC_ERR_INVALID;
  }
  c->n_total = (int)ntot;
  c->nnz_total = nnz;
  const int n = c->n_total;
  // ---- permutation and blocks
  std::vector<int> perm(n);
  std::vector<int> blk_row0, blk_m, blk_sys;
  for (int s = 0; s < c->nsys; ++s) {
    const SysIn& S = sys[s];
    std::vector<int> cnt(S.K + 1, 0);
    for (int r = 0; r < S.n; ++r) cnt[S.part[r] + 1]++;
    for (int k = 0; k < S.K; ++k) {
      if (cnt[k + 1] == 0) {
        bc_set_error("empty block " + std::to_string(k) + " in system " + std::to_string(s));
        return BC_ERR_INVALID;
      }
    }
    std::vector<int> start(S.K + 1, 0);
    for (int k = 0; k < S.K; ++k) start[k + 1] = start[k] + cnt[k + 1];
    for (int k = 0; k < S.K; ++k) {
      blk_row0.push_back(c->sys_off[s] + start[k]);
      blk_m.push_back(cnt[k + 1]);
      blk_sys.push_back(s);
    }
    std::vector<int> cur(start.begin(), start.end() - 1);
    for (int r = 0; r < S.n; ++r) perm[c->sys_off[s] + cur[S.part[r]]++] = c->sys_off[s] + r;
  }
  c->nblk = (int)blk_m.size();
  c->blk_m = blk_m;
  // ---- block kinds.  Every kind computes y_i = (A_i A_i^T)^{-1} u_i
  // (Section 1, eq. (H)); they differ in how.  Banded blocks get their rows
  // in reverse Cuthill-McKee order (the order of rows inside a block does not
  // change its projection, Section 2.2).
  const int dmax = std::min(o.dense_max_m, 4096);
  std::vector<int> kind(c->nblk, KIND_INNER), bandw(c->nblk, -1);
  {
    int maxn = 0;
    for (int s = 0; s < c->nsys; ++s) maxn = std::max(maxn, sys[s].n);
    std::vector<int> cid(maxn, -1);
    for (int b = 0; b < c->nblk; ++b) {
      const int m = blk_m[b];
      if (o.projection == BC_PROJ_DENSE_CHOL) {
        if (m > 4096) {
          bc_set_error("dense Cholesky projection needs blocks of at most 4096 rows");
          return BC_ERR_INVALID;
        }
        kind[b] = KIND_DENSE;
        continue;
      }
      if (o.projection == BC_PROJ_INNER_CG) continue;
      std::vector<int> order;
      const int bwid = m <= BAND_MAX_ROWS
                           ? block_rcm(sys[blk_sys[b]], c->sys_off[blk_sys[b]], perm.data() + blk_row0[b], m,
                                       cid, order)
                           : -1;
      const bool band_ok = bwid >= 0 && bwid <= BAND_MAX;
      if (o.projection == BC_PROJ_BAND_CHOL) {
        if (!band_ok) {
          bc_set_error("block " + std::to_string(b) + " (" + std::to_string(m) +
                       " rows) has no banded form within half-bandwidth " + std::to_string(BAND_MAX) +
                       (bwid >= 0 ? " (reverse Cuthill-McKee gives " + std::to_string(bwid) + ")" : ""));
          return BC_ERR_INVALID;
        }
        kind[b] = KIND_BAND;
      } else {
        // bytes per application: band 2 m (bw+1), dense m (m+1), inner CG
        // (thousands of sparse products) the most; band wins by a margin
        kind[b] = band_ok && (m > dmax || 8LL * (bwid + 1) <= (long long)m + 1)
                      ? KIND_BAND
                      : (m <= dmax ? KIND_DENSE : KIND_INNER);
      }
      if (kind[b] == KIND_BAND) {
        bandw[b] = bwid;
        std::vector<int> idx(perm.begin() + blk_row0[b], perm.begin() + blk_row0[b] + m);
        for (int l = 0; l < m; ++l) perm[blk_row0[b] + l] = idx[order[l]];
      }
    }
  }
  c->blk_kind = kind;
  c->blk_bw = bandw;
  // Rows of an inner-CG block are ordered by decreasing length (stable) when
  // their 64-row slices would otherwise be padded by more than 25%.
  for (int b = 0; b < c->nblk; ++b) {
    if (kind[b] != KIND_INNER) continue;
    const int r0 = blk_row0[b], m = blk_m[b];
    auto len = [&](int i) {
      const int g = perm[i];
      const int s = (int)(std::upper_bound(c->sys_off.begin(), c->sys_off.end(), g) - c->sys_off.begin()) - 1;
      const int r = g - c->sys_off[s];
      return sys[s].rowptr[r + 1] - sys[s].rowptr[r];
    };
    long long used = 0, padded = 0;
    for (int s0 = 0; s0 < m; s0 += 64) {
      int w = 0;
      for (int l = s0; l < std::min(m, s0 + 64); ++l) {
        const int L = len(r0 + l);
        used += L;
        w = std::max(w, L);
      }
      padded += (long long)64 * w;
    }
    if (padded > used + used / 4) {
      std::vector<int> idx(perm.begin() + r0, perm.begin() + r0 + m);
      std::vector<int> L(m);
      for (int l = 0; l < m; ++l) L[l] = len(r0 + l);
      std::vector<int> ord(m);
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return L[x] > L[y]; });
      for (int l = 0; l < m; ++l) perm[r0 + l] = idx[ord[l]];
    }
  }
  // ---- permuted CSR (global columns)
  std::vector<int> rowptr(n + 1, 0), col(nnz);
  std::vector<double> val(nnz);
  std::vector<int> row_sys(n);
  c->normA_inf.assign(c->nsys, 0.0);
  {
    int e = 0;
    for (int i = 0; i < n; ++i) {
      const int g = perm[i];
      const int s = (int)(std::upper_bound(c->sys_off.begin(), c->sys_off.end(), g) - c->sys_off.begin()) - 1;
      row_sys[i] = s;
      const int r = g - c->sys_off[s];
      const SysIn& S = sys[s];
      double rs = 0.0;
      for (int q = S.rowptr[r]; q < S.rowptr[r + 1]; ++q) {
        col[e] = S.col[q] + c->sys_off[s];
        val[e] = S.val[q];
        rs += std::fabs(S.val[q]);
        ++e;
      }
      c->normA_inf[s] = std::max(c->normA_inf[s], rs);
      rowptr[i + 1] = e;
    }
  }
  // ---- row scales 1/||a_r||_2 of the permuted rows (the projections work on
  // rows of unit 2-norm, which leaves every P_i unchanged; Section 3.1)
  std::vector<double> dsc(n);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) s += val[e] * val[e];
    if (!(s > 0.0)) {
      bc_set_error("row " + std::to_string(perm[i]) + " of A is zero: A is singular");
      return BC_ERR_SINGULAR_BLOCK;
    }
    dsc[i] = 1.0 / std::sqrt(s);
  }
  // ---- A^T: per column, permuted rows ascending
  std::vector<int> tptr(n + 1, 0), trow(nnz);
  std::vector<double> tval(nnz);
  for (long long e = 0; e < nnz; ++e) tptr[col[e] + 1]++;
  for (int j = 0; j < n; ++j) tptr[j + 1] += tptr[j];
  {
    std::vector<int> cur(tptr.begin(), tptr.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int q = cur[col[e]]++;
        trow[q] = i;
        tval[q] = val[e];
      }
  }
  // ---- tiles
  std::vector<int> tile_start, tile_sys, sys_tile(c->nsys + 1, 0);
  for (int s = 0; s < c->nsys; ++s) {
    for (int a = c->sys_off[s]; a < c->sys_off[s + 1]; a += TILE) {
      tile_start.push_back(a);
      tile_sys.push_back(s);
    }
    sys_tile[s + 1] = (int)tile_start.size();
  }
  c->ntiles = (int)tile_start.size();
  tile_start.push_back(n);
  c->lanes = c->lanesT = o.spmv_lanes != 0 ? o.spmv_lanes : choose_lanes(nnz, n);
  std::vector<int> is_dense(c->nblk, 0);
  for (int b = 0; b < c->nblk; ++b) is_dense[b] = kind[b] == KIND_DENSE;
  // ---- inner-CG block data
  std::vector<int> in_row0, in_m, in_sup0, in_nsup, in_sys;
  std::vector<int> loc(nnz, 0), btptr(1, 0), btrow;
  std::vector<double> btval;
  {
    std::vector<int> mark(n, -1);
    int sup_total = 0;
    for (int b = 0; b < c->nblk; ++b) {
      if (kind[b] != KIND_INNER) continue;
      const int r0 = blk_row0[b], m = blk_m[b];
      std::vector<int> sup;
      for (int i = r0; i < r0 + m; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) sup.push_back(col[e]);
      std::sort(sup.begin(), sup.end());
      sup.erase(std::unique(sup.begin(), sup.end()), sup.end());
      {
        // support columns by decreasing count (stable) when 64-column slices
        // would be padded by more than 25%
        for (size_t q = 0; q < sup.size(); ++q) mark[sup[q]] = 0;
        for (int i = r0; i < r0 + m; ++i)
          for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) mark[col[e]]++;
        long long used = 0, padded = 0;
        for (size_t s0 = 0; s0 < sup.size(); s0 += 64) {
          int w = 0;
          for (size_t l = s0; l < std::min(sup.size(), s0 + 64); ++l) {
            used += mark[sup[l]];
            w = std::max(w, mark[sup[l]]);
          }
          padded += 64LL * w;
        }
        if (padded > used + used / 4) {
          std::stable_sort(sup.begin(), sup.end(), [&](int x, int y) { return mark[x] > mark[y]; });
        }
      }
      for (size_t q = 0; q < sup.size(); ++q) mark[sup[q]] = (int)q;
      for (int i = r0; i < r0 + m; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) loc[e] = mark[col[e]];
      // transposed block CSR: support columns ascending, rows ascending
      std::vector<int> cnt(sup.size() + 1, 0);
      for (int i = r0; i < r0 + m; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) cnt[mark[col[e]] + 1]++;
      for (size_t q = 0; q < sup.size(); ++q) cnt[q + 1] += cnt[q];
      const int base = (int)btrow.size();
      btrow.resize(base + cnt[sup.size()]);
      btval.resize(base + cnt[sup.size()]);
      std::vector<int> cur(cnt.begin(), cnt.end() - 1);
      for (int i = r0; i < r0 + m; ++i)
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
          const int q = base + cur[mark[col[e]]]++;
          btrow[q] = i - r0;
          btval[q] = val[e];
        }
      for (size_t q = 0; q < sup.size(); ++q) btptr.push_back(base + cnt[q + 1]);
      for (int cc : sup) mark[cc] = -1;
      in_row0.push_back(r0);
      in_m.push_back(m);
      c->in_nnz.push_back(rowptr[r0 + m] - rowptr[r0]);
      c->in_m_h.push_back(m);
      in_sup0.push_back(sup_total);
      in_nsup.push_back((int)sup.size());
      in_sys.push_back(blk_sys[b]);
      sup_total += (int)sup.size();
    }
  }
  // ---- dense block data
  std::vector<int> dn_row0, dn_m, dn_nt, dn_sys;
  std::vector<long long> dn_loff, dn_doff;
  std::vector<int4> gram_tiles;
  long long ltot = 0, dtot = 0;
  for (int b = 0; b < c->nblk; ++b) {
    if (!is_dense[b]) continue;
    const int m = blk_m[b], nt = (m + DT - 1) / DT;
    const int db = (int)dn_m.size();
    dn_row0.push_back(blk_row0[b]);
    dn_m.push_back(m);
    c->dn_m_h.push_back(m);
    c->dense_max_nt = std::max(c->dense_max_nt, nt);
    dn_nt.push_back(nt);
    dn_sys.push_back(blk_sys[b]);
    dn_loff.push_back(ltot);
    dn_doff.push_back(dtot);
    ltot += (long long)nt * (nt + 1) / 2 * DT * DT;
    dtot += 2LL * nt * DT * DT;
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j <= i; ++j) gram_tiles.push_back(make_int4(db, i, j, 0));
  }
  // ---- device state
  hipStream_t st = c->stream;
  Arena& A = c->arena;
  {
    std::vector<int> ez(1, 0);
    BC_TRY(A.upload(&c->d_err, ez, st));
    int dev = 0, khz = 0;
    BC_HIP(hipGetDevice(&dev));
    BC_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    c->wall_khz = khz > 0 ? khz : 100000;
    c->wait_ticks = (unsigned long long)(2.0 * c->wall_khz * 1e3);  // 2 s
  }
  BC_TRY(A.upload(&c->d_perm, perm, st));
  BC_TRY(A.upload(&c->d_rowptr, rowptr, st));
  BC_TRY(A.upload(&c->d_col, col, st));
  BC_TRY(A.upload(&c->d_val, val, st));
  BC_TRY(A.upload(&c->d_tptr, tptr, st));
  BC_TRY(A.upload(&c->d_trow, trow, st));
  BC_TRY(A.upload(&c->d_tval, tval, st));
  if (c->mixed) {
    std::vector<float> v32(val.begin(), val.end()), t32(tval.begin(), tval.end());
    BC_TRY(A.upload(&c->d_val32, v32, st));
    BC_TRY(A.upload(&c->d_tval32, t32, st));
  }
  // sliced-ELL copies for the sparse products (a candidate of the autotuner,
  // or requested with spmv_lanes = -1)
  {
    const bool force = o.spmv_lanes == LANES_SELL;
    if (force || o.spmv_lanes == 0) {
      std::vector<long long> pa, pt;
      std::vector<int> wa, wt, ca, ct;
      std::vector<double> va, vt;
      if (build_sell(rowptr, col, val, tile_start, force, pa, wa, ca, va) &&
          build_sell(tptr, trow, tval, tile_start, force, pt, wt, ct, vt)) {
        long long *ppa, *ppt;
        int *pwa, *pwt, *pca, *pct;
        double *pva, *pvt;
        BC_TRY(A.upload(&ppa, pa, st));
        BC_TRY(A.upload(&pwa, wa, st));
        BC_TRY(A.upload(&pca, ca, st));
        BC_TRY(A.upload(&pva, va, st));
        BC_TRY(A.upload(&ppt, pt, st));
        BC_TRY(A.upload(&pwt, wt, st));
        BC_TRY(A.upload(&pct, ct, st));
        BC_TRY(A.upload(&pvt, vt, st));
        c->sellA = SellMat{ppa, pwa, pca, pva, nullptr, gather_interleaved(pa, wa, ca, o)};
        c->sellT = SellMat{ppt, pwt, pct, pvt, nullptr, gather_interleaved(pt, wt, ct, o)};
        if (c->spmv32) {
          std::vector<float> a32(va.begin(), va.end()), t32(vt.begin(), vt.end());
          float *pa32, *pt32;
          BC_TRY(A.upload(&pa32, a32, st));
          BC_TRY(A.upload(&pt32, t32, st));
          c->sellA.val32 = pa32;
          c->sellT.val32 = pt32;
        }
        c->have_sell = true;
        BC_HIP(hipStreamSynchronize(st));  // host staging vectors go out of scope
      }
    }
  }
  double* d_dsc;
  BC_TRY(A.upload(&d_dsc, dsc, st));
  BC_TRY(A.upload(&c->d_tile_start, tile_start, st));
  BC_TRY(A.upload(&c->d_tile_sys, tile_sys, st));
  BC_TRY(A.upload(&c->d_sys_tile, sys_tile, st));
  const int ns = c->nsys;
  std::vector<int> zeros_ns(ns, 0);
  BC_TRY(A.upload(&c->d_done, zeros_ns, st));
  BC_TRY(A.upload(&c->d_zero_flags, zeros_ns, st));
  BC_TRY(A.upload(&c->d_iters, zeros_ns, st));
  BC_TRY(A.upload(&c->d_status, zeros_ns, st));
  BC_TRY(A.upload(&c->d_pending, zeros_ns, st));
  BC_TRY(A.upload(&c->d_mask, zeros_ns, st));
  BC_TRY(A.upload(&c->d_restart, zeros_ns, st));
  BC_TRY(A.alloc(&c->d_thr, ns));
  BC_TRY(A.alloc(&c->d_rr, 2 * ns));
  BC_TRY(A.alloc(&c->d_hist, ns));
  BC_TRY(A.alloc(&c->d_part_a, c->ntiles));
  BC_TRY(A.alloc(&c->d_part_b, c->ntiles));
  BC_TRY(A.alloc(&c->d_part_c, c->ntiles));
  BC_TRY(A.alloc(&c->d_part_f, c->ntiles));
  BC_TRY(A.alloc(&c->d_part_d, c->ntiles));
  BC_TRY(A.alloc(&c->d_part_e, c->ntiles));
  BC_TRY(A.alloc(&c->d_part_g, c->ntiles));
  BC_TRY(A.alloc(&c->d_final, (size_t)5 * c->nsys));
  BC_TRY(A.upload(&c->d_normA, c->normA_inf, st));
  BC_TRY(A.alloc(&c->d_finf, ns));
  BC_TRY(A.alloc(&c->d_r, n));
  BC_TRY(A.alloc(&c->d_p, n));
  BC_TRY(A.alloc(&c->d_psi, n));
  BC_TRY(A.alloc(&c->d_s, n));
  BC_TRY(A.alloc(&c->d_u, n));
  BC_TRY(A.alloc(&c->d_y, n));
  BC_TRY(A.alloc(&c->d_f, n));
  BC_TRY(A.alloc(&c->d_inner_total, 1));
  // inner blocks
  InnerBlocks& B = c->inner;
  B = InnerBlocks{};
  B.nblk = (int)in_m.size();
  if (B.nblk > 0) {
    int *p0, *p1, *p2, *p3, *p4;
    BC_TRY(A.upload(&p0, in_row0, st));
    BC_TRY(A.upload(&p1, in_m, st));
    BC_TRY(A.upload(&p2, in_sup0, st));
    BC_TRY(A.upload(&p3, in_nsup, st));
    BC_TRY(A.upload(&p4, in_sys, st));
    B.row0 = p0; B.m = p1; B.sup0 = p2; B.nsup = p3; B.sys = p4;
    B.dsc = d_dsc;
    const int sup_total = (int)btptr.size() - 1;
    c->inner_sup_total = sup_total;
    if (c->inner_prec == INNER_F32) {
      BC_TRY(A.alloc(&B.q32, n));
      BC_TRY(A.alloc(&B.z32, n));
      BC_TRY(A.alloc(&B.ri32, n));
      BC_TRY(A.alloc(&B.t32, sup_total));
    } else {
      BC_TRY(A.alloc(&B.q, n));
      BC_TRY(A.alloc(&B.z, n));
      BC_TRY(A.alloc(&B.ri, n));
      BC_TRY(A.alloc(&B.t, sup_total));
    }
    B.max_m = *std::max_element(in_m.begin(), in_m.end());
    B.max_nsup = *std::max_element(in_nsup.begin(), in_nsup.end());
    if (B.max_m > 16384) {
      bc_set_error("inner-CG blocks are limited to 16384 rows (largest block has " +
                   std::to_string(B.max_m) + ")");
      return BC_ERR_INVALID;
    }
    // Sliced ELL copies of every inner block (slices of 64 rows and of 64
    // support columns, widths padded to a multiple of 8).
    {
      const bool i16 = B.max_m < 65536 && B.max_nsup < 65536;
      std::vector<int> a_s0, a_w, t_s0, t_w;
      std::vector<long long> a_ptr, t_ptr;
      std::vector<int> a_ix, t_ix;
      std::vector<double> a_v, t_v;
      for (int q = 0; q < B.nblk; ++q) {
        const int r0 = in_row0[q], m = in_m[q], s0 = in_sup0[q], ns2 = in_nsup[q];
        a_s0.push_back((int)a_w.size());
        for (int s = 0; s * 64 < m; ++s) {
          int w = 0;
          for (int l = 0; l < 64 && s * 64 + l < m; ++l) {
            const int i = r0 + s * 64 + l;
            w = std::max(w, rowptr[i + 1] - rowptr[i]);
          }
          if (w >= 5) w = (w + 7) / 8 * 8;
          const long long base = (long long)a_ix.size();
          a_ptr.push_back(base);
          a_w.push_back(w);
          a_ix.resize(base + (long long)w * 64, 0);
          a_v.resize(base + (long long)w * 64, 0.0);
          for (int l = 0; l < 64 && s * 64 + l < m; ++l) {
            const int i = r0 + s * 64 + l;
            for (int e = rowptr[i], k = 0; e < rowptr[i + 1]; ++e, ++k) {
              a_ix[base + (long long)k * 64 + l] = loc[e];
              a_v[base + (long long)k * 64 + l] = val[e] * dsc[i];
            }
          }
        }
        t_s0.push_back((int)t_w.size());
        for (int s = 0; s * 64 < ns2; ++s) {
          int w = 0;
          for (int l = 0; l < 64 && s * 64 + l < ns2; ++l) {
            const int cc = s0 + s * 64 + l;
            w = std::max(w, btptr[cc + 1] - btptr[cc]);
          }
          if (w >= 5) w = (w + 7) / 8 * 8;
          const long long base = (long long)t_ix.size();
          t_ptr.push_back(base);
          t_w.push_back(w);
          t_ix.resize(base + (long long)w * 64, 0);
          t_v.resize(base + (long long)w * 64, 0.0);
          for (int l = 0; l < 64 && s * 64 + l < ns2; ++l) {
            const int cc = s0 + s * 64 + l;
            for (int e = btptr[cc], k = 0; e < btptr[cc + 1]; ++e, ++k) {
              t_ix[base + (long long)k * 64 + l] = btrow[e];
              t_v[base + (long long)k * 64 + l] = btval[e] * dsc[r0 + btrow[e]];
            }
          }
        }
      }
      int *pas0, *paw, *pts0, *ptw;
      long long *pap, *ptp;
      double *pav = nullptr, *ptv = nullptr;
      BC_TRY(A.upload(&pas0, a_s0, st));
      BC_TRY(A.upload(&paw, a_w, st));
      BC_TRY(A.upload(&pap, a_ptr, st));
      BC_TRY(A.upload(&pts0, t_s0, st));
      BC_TRY(A.upload(&ptw, t_w, st));
      BC_TRY(A.upload(&ptp, t_ptr, st));
      if (c->inner_prec == INNER_F64) {  // (the other precisions read the FP32 copies)
        BC_TRY(A.upload(&pav, a_v, st));
        BC_TRY(A.upload(&ptv, t_v, st));
      }
      if (i16) {
        std::vector<uint16_t> a16(a_ix.begin(), a_ix.end()), t16(t_ix.begin(), t_ix.end());
        uint16_t *pa16, *pt16;
        BC_TRY(A.upload(&pa16, a16, st));
        BC_TRY(A.upload(&pt16, t16, st));
        B.a_idx = pa16;
        B.t_idx = pt16;
      } else {
        int *pa32, *pt32;
        BC_TRY(A.upload(&pa32, a_ix, st));
        BC_TRY(A.upload(&pt32, t_ix, st));
        B.a_idx = pa32;
        B.t_idx = pt32;
      }
      if (c->inner_prec != INNER_F64) {
        std::vector<float> a32(a_v.begin(), a_v.end()), t32(t_v.begin(), t_v.end());
        float *pa32f, *pt32f;
        BC_TRY(A.upload(&pa32f, a32, st));
        BC_TRY(A.upload(&pt32f, t32, st));
        B.a_val32 = pa32f;
        B.t_val32 = pt32f;
      }
      B.a_s0 = pas0; B.a_w = paw; B.a_ptr = pap; B.a_val = pav;
      B.t_s0 = pts0; B.t_w = ptw; B.t_ptr = ptp; B.t_val = ptv;
      B.idx16 = i16 ? 1 : 0;
      BC_HIP(hipStreamSynchronize(st));  // host staging vectors go out of scope
    }
    // workgroups per block: spread the blocks over the CUs (at most 16 per
    // block, each owning at least 4 row slices), limited by co-residency
    int G = o.inner_groups;
    if (G <= 0) {
      G = std::max(1, 256 / std::max(1, B.nblk));
      const int minm = *std::min_element(in_m.begin(), in_m.end());
      G = std::min(G, std::max(1, minm / 256));
    }
    G = std::min(G, 16);
    // the group kernel keeps two full block vectors in LDS
    if ((size_t)2 * ((B.max_m + 1) / 2 * 2) * (c->inner_prec == INNER_F32 ? 4 : 8) > 150 * 1024) G = 1;
    if (G > 1) {
      const int per_xcd = (B.nblk + 7) / 8;
      const int cap = inner_grp_max_resident(c->inner_prec == INNER_F32, B.max_m);
      while (G > 1 && per_xcd * G * 8 > cap) --G;
    }
    B.groups = G;
    B.trace = nullptr;
    if (std::getenv("BC_INNER_TRACE")) {
      unsigned long long* ptr;
      BC_TRY(A.alloc(&ptr, 16 * 8 * 64));
      BC_HIP(hipMemsetAsync(ptr, 0, 16 * 8 * 64 * sizeof(unsigned long long), st));
      B.trace = ptr;
    }
    BC_TRY(A.alloc(&B.xp, (size_t)B.nblk * 2 * 64));
    BC_HIP(hipMemsetAsync(B.xp, 0, (size_t)B.nblk * 2 * 64 * sizeof(unsigned long long), st));
    std::vector<unsigned> bz(32 * B.nblk, 0u);
    unsigned* pbar;
    BC_TRY(A.upload(&pbar, bz, st));
    B.bar = pbar;
    B.err = c->d_err;
    B.wait_ticks = c->wait_ticks;
    std::vector<int> iz(B.nblk, 0);
    int* pit;
    BC_TRY(A.upload(&pit, iz, st));
    B.iters = pit;
    B.total = c->d_inner_total;
    unsigned long long* pbt;
    BC_TRY(A.alloc(&pbt, B.nblk));
    BC_HIP(hipMemsetAsync(pbt, 0, B.nblk * sizeof(unsigned long long), st));
    B.blk_total = pbt;
    // FP32 inner CG cannot resolve residuals far below its unit roundoff
    B.tol = (c->inner_prec == INNER_F32 && o.inner_tol < 1e-6) ? 1e-6 : o.inner_tol;
    B.maxit = o.inner_maxit;
  }
  // dense blocks
  DenseBlocks& D = c->dense;
  D = DenseBlocks{};
  D.nblk = (int)dn_m.size();
  if (D.nblk > 0) {
    int *p0, *p1, *p2, *p3, *pinfo;
    long long *pl, *pd;
    int4* ptiles;
    BC_TRY(A.upload(&p0, dn_row0, st));
    BC_TRY(A.upload(&p1, dn_m, st));
    BC_TRY(A.upload(&p2, dn_nt, st));
    BC_TRY(A.upload(&p3, dn_sys, st));
    BC_TRY(A.upload(&pl, dn_loff, st));
    BC_TRY(A.upload(&pd, dn_doff, st));
    BC_TRY(A.upload(&ptiles, gram_tiles, st));
    std::vector<int> iz(D.nblk, 0);
    BC_TRY(A.upload(&pinfo, iz, st));
    D.row0 = p0; D.m = p1; D.nt = p2; D.sys = p3; D.loff = pl; D.doff = pd; D.info = pinfo;
    D.dsc = d_dsc;
    unsigned long long* pap;
    BC_TRY(A.alloc(&pap, D.nblk));
    BC_HIP(hipMemsetAsync(pap, 0, D.nblk * sizeof(unsigned long long), st));
    D.applies = pap;
    BC_TRY(A.alloc(&D.gdiag, n));
    BC_TRY(A.alloc(&D.L, ltot));
    BC_TRY(A.alloc(&D.LT, ltot));
    BC_TRY(A.alloc(&D.Dinv, dtot));
    if (c->mixed) {
      BC_TRY(A.alloc(&D.L32, ltot));
      BC_TRY(A.alloc(&D.LT32, ltot));
      BC_TRY(A.alloc(&D.Dinv32, dtot));
    }
    BC_HIP(launch_gram(st, D, ptiles, (int)gram_tiles.size(), c->d_rowptr, c->d_col, c->d_val,
                       c->d_tptr, c->d_trow, c->d_tval));
    // blocked Cholesky plan: per panel step, the panel rows and trailing tiles
    CholPlan P;
    {
      int maxnt = 0;
      for (int b = 0; b < D.nblk; ++b) maxnt = std::max(maxnt, dn_nt[b]);
      P.steps = (maxnt + CHOL_PW - 1) / CHOL_PW;
      std::vector<int2> pl_h;
      std::vector<int4> up_h;
      P.panel_off.assign(1, 0);
      P.upd_off.assign(1, 0);
      for (int s = 0; s < P.steps; ++s) {
        const int kb = s * CHOL_PW;
        for (int b = 0; b < D.nblk; ++b) {
          const int ntb = dn_nt[b], ke = std::min(ntb, kb + CHOL_PW);
          if (kb >= ntb) continue;
          for (int i = ke; i < ntb; ++i) pl_h.push_back(make_int2(b, i));
          for (int i = ke; i < ntb; ++i)
            for (int j = ke; j <= i; ++j) up_h.push_back(make_int4(b, i, j, 0));
        }
        P.panel_off.push_back((long long)pl_h.size());
        P.upd_off.push_back((long long)up_h.size());
      }
      int2* ppl;
      int4* pup;
      BC_TRY(A.upload(&ppl, pl_h, st));
      BC_TRY(A.upload(&pup, up_h, st));
      P.panel = ppl;
      P.upd = pup;
    }
    BC_HIP(launch_cholesky(st, D, P));
    BC_HIP(launch_dense_finish(st, D, c->mixed));
    BC_HIP(prepare_dense_apply());
    D.err = c->d_err;
    D.wait_ticks = c->wait_ticks;
    std::vector<int> info(D.nblk);
    BC_HIP(hipMemcpyAsync(info.data(), pinfo, D.nblk * sizeof(int), hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < D.nblk; ++b)
      if (info[b] != 0) {
        bc_set_error("block " + std::to_string(b) + " of the dense projections has a non-positive "
                     "pivot at row " + std::to_string(info[b] - 1) + ": A_i A_i^T is numerically singular");
        return BC_ERR_SINGULAR_BLOCK;
      }
  }
  // banded blocks
  BandBlocks& Bd = c->band;
  Bd = BandBlocks{};
  {
    std::vector<int> bd_row0, bd_m, bd_bw, bd_ld, bd_sys, bd_sld;
    std::vector<long long> bd_off, bd_soff;
    long long btot = 0, stot = 0;
    int ldmax = 0, sldmax = 0;
    for (int b = 0; b < c->nblk; ++b) {
      if (kind[b] != KIND_BAND) continue;
      const int m = blk_m[b], W = (bandw[b] + 1 + 3) / 4 * 4;
      ldmax = std::max(ldmax, W);
      bd_row0.push_back(blk_row0[b]);
      bd_m.push_back(m);
      bd_bw.push_back(bandw[b]);
      bd_ld.push_back(W);
      bd_sys.push_back(blk_sys[b]);
      bd_off.push_back(btot);
      c->bd_m_h.push_back(m);
      c->bd_bw_h.push_back(bandw[b]);
      btot += (long long)((m + 63) / 64) * 64 * W;
      // slot layout: as many slots per row as the band layout
      const int S = W;
      sldmax = std::max(sldmax, S);
      bd_sld.push_back(S);
      bd_soff.push_back(stot);
      stot += (long long)((m + 63) / 64) * 64 * S;
    }
    Bd.nblk = (int)bd_m.size();
    if (Bd.nblk > 0) {
      int *p0, *p1, *p2, *p3, *p4, *pinfo;
      long long* po;
      BC_TRY(A.upload(&p0, bd_row0, st));
      BC_TRY(A.upload(&p1, bd_m, st));
      BC_TRY(A.upload(&p2, bd_bw, st));
      BC_TRY(A.upload(&p4, bd_ld, st));
      BC_TRY(A.upload(&p3, bd_sys, st));
      BC_TRY(A.upload(&po, bd_off, st));
      std::vector<int> iz(Bd.nblk, 0);
      BC_TRY(A.upload(&pinfo, iz, st));
      Bd.row0 = p0; Bd.m = p1; Bd.bw = p2; Bd.ld = p4; Bd.sys = p3; Bd.off = po; Bd.info = pinfo;
      Bd.ldmax = ldmax;
      {
        int* ps;
        long long* pso;
        BC_TRY(A.upload(&ps, bd_sld, st));
        BC_TRY(A.upload(&pso, bd_soff, st));
        Bd.sld = ps;
        Bd.soff = pso;
        Bd.sldmax = sldmax;
      }
      Bd.dsc = d_dsc;
      unsigned long long* pap;
      BC_TRY(A.alloc(&pap, Bd.nblk));
      BC_HIP(hipMemsetAsync(pap, 0, Bd.nblk * sizeof(unsigned long long), st));
      Bd.applies = pap;
      BC_TRY(A.alloc(&Bd.L, btot));
      if (c->mixed) {
        BC_TRY(A.alloc(&Bd.SL32, stot));
        BC_TRY(A.alloc(&Bd.SR32, stot));
      } else {
        BC_TRY(A.alloc(&Bd.SL, stot));
        BC_TRY(A.alloc(&Bd.SR, stot));
      }
      {
        // sweeps of the blocks with the most work are launched first
        std::vector<int> ord(Bd.nblk);
        for (int b = 0; b < Bd.nblk; ++b) ord[b] = b;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
          return (long long)bd_m[x] * bd_sld[x] > (long long)bd_m[y] * bd_sld[y];
        });
        int* pord;
        BC_TRY(A.upload(&pord, ord, st));
        Bd.order = pord;
      }
      BC_HIP(launch_band_gram(st, Bd, c->d_rowptr, c->d_col, c->d_val, c->d_tptr, c->d_trow, c->d_tval));
      BC_HIP(launch_band_cholesky(st, Bd));
      std::vector<int> info(Bd.nblk);
      BC_HIP(hipMemcpyAsync(info.data(), pinfo, Bd.nblk * sizeof(int), hipMemcpyDeviceToHost, st));
      BC_HIP(hipStreamSynchronize(st));
      for (int b = 0; b < Bd.nblk; ++b)
        if (info[b] != 0) {
          bc_set_error("banded block " + std::to_string(b) + " has a non-positive pivot at row " +
                       std::to_string(info[b] - 1) + ": A_i A_i^T is numerically singular");
          return BC_ERR_SINGULAR_BLOCK;
        }
      BC_HIP(launch_band_finish(st, Bd, c->mixed));
      BC_HIP(prepare_band_apply(Bd, c->mixed));
    }
  }
  if (o.spmv_lanes == 0) BC_TRY(autotune_lanes(c, pattern_key(rowptr, col, n, c->spmv32)));
  BC_HIP(hipStreamSynchronize(st));
  return BC_OK;
}

bc_status new_ctx(bc_ctx** out, const bc_opts* opts) {
  *out = nullptr;
  BC_TRY(check_device());
  bc_ctx* c = new (std::nothrow) bc_ctx();
  if (!c) {
    bc_set_error("host allocation failed");
    return BC_ERR_NOMEM;
  }
  if (opts) c->opts = *opts; else bc_opts_default(&c->opts);
  if (c->opts.check_every < 1) c->opts.check_every = 1;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_sync, hipEventDisableTiming) != hipSuccess) {
    delete c;
    bc_set_error("stream/event creation failed");
    return BC_ERR_DEVICE;
  }
  *out = c;
  return BC_OK;
}

}  // namespace

extern "C" bc_status bc_setup_batched(bc_ctx** ctx, int32_t nsys, const int32_t* n,
                                      const int32_t* const* rowptr, const int32_t* const* colidx,
                                      const double* const* vals, const int32_t* K,
                                      const int32_t* const* part, const bc_opts* opts) {
  if (!ctx) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  *ctx = nullptr;
  if (nsys < 1 || !n || !rowptr || !colidx || !vals || !K || !part) {
    bc_set_error("bc_setup_batched: null argument or nsys < 1");
    return BC_ERR_INVALID;
  }
  if (opts) BC_TRY(validate_opts(*opts));
  std::vector<SysIn> sys(nsys);
  for (int s = 0; s < nsys; ++s) {
    BC_TRY(validate_system(s, n[s], rowptr[s], colidx[s], vals[s], K[s], part[s]));
    sys[s] = SysIn{n[s], rowptr[s], colidx[s], vals[s], K[s], part[s]};
  }
  bc_ctx* c = nullptr;
  BC_TRY(new_ctx(&c, opts));
  bc_status st = setup_impl(c, sys);
  if (st != BC_OK) {
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return st;
  }
  *ctx = c;
  return BC_OK;
}

extern "C" bc_status bc_setup(bc_ctx** ctx, int32_t n, const int32_t* rowptr,
                              const int32_t* colidx, const double* vals, int32_t K,
                              const int32_t* part, const bc_opts* opts) {
  return bc_setup_batched(ctx, 1, &n, &rowptr, &colidx, &vals, &K, &part, opts);
}

extern "C" void bc_destroy(bc_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->inner.trace && std::getenv("BC_INNER_TRACE")) {
    std::vector<unsigned long long> h(16 * 8 * 64);
    if (hipMemcpy(h.data(), ctx->inner.trace, h.size() * 8, hipMemcpyDeviceToHost) == hipSuccess) {
      FILE* fp = std::fopen(std::getenv("BC_INNER_TRACE"), "w");
      if (fp) {
        for (size_t q = 0; q < h.size(); ++q) std::fprintf(fp, "%llu\n", h[q]);
        std::fclose(fp);
      }
    }
  }
  delete ctx;
}

extern "C" bc_status bc_info(const bc_ctx* c, int64_t* n_total, int32_t* nsys, int32_t* nblocks,
                             int32_t* ndense) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  if (n_total) *n_total = c->n_total;
  if (nsys) *nsys = c->nsys;
  if (nblocks) *nblocks = c->nblk;
  if (ndense) *ndense = c->dense.nblk;
  return BC_OK;
}

extern "C" bc_status bc_schedule(const bc_ctx* c, int32_t* lanes_a, int32_t* lanes_at) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  if (lanes_a) *lanes_a = c->lanes;
  if (lanes_at) *lanes_at = c->lanesT;
  return BC_OK;
}

extern "C" bc_status bc_set_wait_limit(bc_ctx* c, double seconds) {
  if (!c || !(seconds >= 0.0) || !std::isfinite(seconds) || seconds > 1e9) {
    bc_set_error("bc_set_wait_limit: null context or seconds not in [0, 1e9]");
    return BC_ERR_INVALID;
  }
  c->wait_ticks = (unsigned long long)(seconds * c->wall_khz * 1e3);
  c->inner.wait_ticks = c->wait_ticks;
  c->dense.wait_ticks = c->wait_ticks;
  if (c->gexec) {  // the captured iterations hold the old bound
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  return BC_OK;
}

extern "C" bc_status bc_block_info(const bc_ctx* c, int32_t* kind, int32_t* bandwidth) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  for (int b = 0; b < c->nblk; ++b) {
    if (kind) kind[b] = c->blk_kind[b];
    if (bandwidth) bandwidth[b] = c->blk_bw[b];
  }
  return BC_OK;
}

// ------------------------------------------------------------- projections

namespace {

// y = D^{-1} u block by block (dense sweeps and inner CG).
bc_status block_solves(bc_ctx* c, const double* u, double* y, const int* done) {
  hipStream_t st = c->stream;
  if (c->timing) {
    if (2 * c->ev_used + 2 > (int)c->ev_proj.size()) {
      for (int q = 0; q < 16; ++q) {
        hipEvent_t e;
        BC_HIP(hipEventCreate(&e));
        c->ev_proj.push_back(e);
      }
    }
    BC_HIP(hipEventRecord(c->ev_proj[2 * c->ev_used], st));
  }
  if (c->mrhs.nrhs > 0) {
    // several right-hand sides: each dense or banded factor is read once
    // for a chunk of vectors; inner-CG blocks take all vectors in one launch
    // of the single-workgroup kernel, or else one vector after another
    const int nr = c->mrhs.nrhs, n1 = c->mrhs.n1;
    BC_HIP(launch_dense_apply_multi(st, c->dense, c->mixed, u, y, done, nr, n1, c->dense_max_nt));
    BC_HIP(launch_band_apply_multi(st, c->band, c->mixed, u, y, done, nr, n1));
    bool taken = false;
    MultiView* mv = c->mview.get();
    BC_HIP(launch_inner_cg_multi(st, c->inner, c->inner_prec, u, y, done, nr, n1, c->inner_sup_total,
                                 mv ? mv->d_inner_r : nullptr, mv ? mv->d_inner_t : nullptr,
                                 &taken));
    for (int j = 0; j < nr && !taken; ++j) {
      const size_t o = (size_t)j * n1;
      BC_HIP(launch_inner_cg(st, c->inner, c->inner_prec, u + o, y + o, done ? done + j : nullptr));
    }
  } else {
    BC_HIP(launch_dense_apply(st, c->dense, c->mixed, u, y, done, c->dense_max_nt));
    BC_HIP(launch_band_apply(st, c->band, c->mixed, u, y, done));
    BC_HIP(launch_inner_cg(st, c->inner, c->inner_prec, u, y, done));
  }
  if (c->timing) {
    BC_HIP(hipEventRecord(c->ev_proj[2 * c->ev_used + 1], st));
    ++c->ev_used;
  }
  return BC_OK;
}

// Adds the elapsed times of the recorded projection event pairs (the stream
// must have been synchronised).
void harvest_proj_events(bc_ctx* c) {
  for (int q = 0; q < c->ev_used; ++q) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_proj[2 * q], c->ev_proj[2 * q + 1]) == hipSuccess) {
      c->t_proj_ms += ms;
      ++c->proj_launches;
    } else {
      (void)hipGetLastError();  // leave no sticky error for the next launch check
    }
  }
  c->ev_used = 0;
}

__global__ void k_zero_words(unsigned* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Clears the context's wait-error word at the start of a call (a kernel, not
// a memset: the caller's stream may be under capture).
bc_status clear_wait_error(bc_ctx* c) {
  hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, c->stream, (unsigned*)c->d_err, 1LL);
  BC_HIP(hipGetLastError());
  return BC_OK;
}

// BC_ERR_DEVICE if a bounded device wait gave up during the call.  The
// inner-CG barrier epochs and tagged partials then start again from zero, so
// that workgroups that stopped at different barriers meet again at the next
// call.
bc_status check_wait_error(bc_ctx* c) {
  int h = 0;
  BC_HIP(hipMemcpyAsync(&h, c->d_err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  BC_HIP(hipStreamSynchronize(c->stream));
  if (!h) return BC_OK;
  if (c->inner.nblk) {
    hipLaunchKernelGGL(k_zero_words, dim3(64), dim3(256), 0, c->stream, c->inner.bar,
                       32LL * c->inner.nblk);
    hipLaunchKernelGGL(k_zero_words, dim3(64), dim3(256), 0, c->stream, (unsigned*)c->inner.xp,
                       2LL * 2 * 64 * c->inner.nblk);
    BC_HIP(hipGetLastError());
    BC_HIP(hipStreamSynchronize(c->stream));
  }
  bc_set_error("a device wait gave up (inner-CG workgroups of a block or dense sweep waves did "
               "not meet within the wait limit); the result is invalid");
  return BC_ERR_DEVICE;
}

// Algorithmic bytes of all projection launches counted by the device counters.
bc_status proj_bytes(bc_ctx* c, double* out) {
  const double w = c->mixed ? 4.0 : 8.0;
  double bytes = 0.0;
  if (c->inner.nblk) {
    std::vector<unsigned long long> it(c->inner.nblk);
    BC_HIP(hipMemcpy(it.data(), c->inner.blk_total, it.size() * sizeof(it[0]), hipMemcpyDeviceToHost));
    // stored values w bytes; vectors FP32 only in the FP32 inner CG
    const double wx = c->inner_prec == INNER_F32 ? 4.0 : 8.0;
    for (int b = 0; b < c->inner.nblk; ++b)
      bytes += (double)it[b] * (2.0 * (w + 4.0) * (double)c->in_nnz[b] + 6.0 * wx * (double)c->in_m_h[b]);
  }
  if (c->dense.nblk) {
    std::vector<unsigned long long> ap(c->dense.nblk);
    BC_HIP(hipMemcpy(ap.data(), c->dense.applies, ap.size() * sizeof(ap[0]), hipMemcpyDeviceToHost));
    for (int b = 0; b < c->dense.nblk; ++b) {
      const double m = (double)c->dn_m_h[b];
      bytes += (double)ap[b] * m * (m + 1.0) * w;
    }
  }
  if (c->band.nblk) {
    std::vector<unsigned long long> ap(c->band.nblk);
    BC_HIP(hipMemcpy(ap.data(), c->band.applies, ap.size() * sizeof(ap[0]), hipMemcpyDeviceToHost));
    for (int b = 0; b < c->band.nblk; ++b)
      bytes += (double)ap[b] * 2.0 * (double)c->bd_m_h[b] * (double)(c->bd_bw_h[b] + 1) * w;
  }
  *out = bytes;
  return BC_OK;
}

bc_status reset_proj_counters(bc_ctx* c) {
  if (c->inner.nblk)
    BC_HIP(hipMemsetAsync(c->inner.blk_total, 0, c->inner.nblk * sizeof(unsigned long long), c->stream));
  if (c->dense.nblk)
    BC_HIP(hipMemsetAsync(c->dense.applies, 0, c->dense.nblk * sizeof(unsigned long long), c->stream));
  if (c->band.nblk)
    BC_HIP(hipMemsetAsync(c->band.applies, 0, c->band.nblk * sizeof(unsigned long long), c->stream));
  c->ev_used = 0;
  c->t_proj_ms = 0.0;
  c->proj_launches = 0;
  return BC_OK;
}


}  // namespace

extern "C" bc_status bc_project(bc_ctx* c, const double* v, double* Hv) {
  if (!c || !v || !Hv) {
    bc_set_error("bc_project: null argument");
    return BC_ERR_INVALID;
  }
  BC_TRY(enter(c, c->opts.stream));
  BC_TRY(clear_wait_error(c));
  OuterState S = c->outer(0, 0);
  S.done = c->d_zero_flags;
  hipStream_t st = c->stream;
  BC_HIP(spmv_a(c, st, c->lanes, v, c->d_u, S, false));
  BC_TRY(block_solves(c, c->d_u, c->d_y, nullptr));
  BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, Hv, v, S));
  const bc_status werr = check_wait_error(c);
  BC_TRY(leave(c, c->opts.stream));
  return werr;
}

// ------------------------------------------------------------------- solve

namespace {

// One outer iteration of Algorithm 2 on every system not yet done: u = A p,
// y_i = (A_i A_i^T)^{-1} u_i, psi = A^T y with p.psi, then alpha, x, r, s,
// beta, p and the per-system bookkeeping.
bc_status outer_iteration(bc_ctx* c, double* x, const OuterState& S, bool timed) {
  hipStream_t st = c->stream;
  BC_HIP(spmv_a(c, st, c->lanes, c->d_p, c->d_u, S, true));
  const bool keep = c->timing;
  c->timing = timed && keep;
  const bc_status rs = block_solves(c, c->d_u, c->d_y, c->d_done);
  c->timing = keep;
  BC_TRY(rs);
  BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_psi, c->d_p, S));
  BC_HIP(launch_update_xrs(st, x, c->d_r, c->d_s, c->d_p, c->d_psi, c->d_u, S));
  BC_HIP(launch_update_p(st, c->d_p, c->d_r, S));
  return BC_OK;
}

// Runs G outer iterations as one replay of a captured hipGraph.  The graph
// is captured on first use and again whenever the solve state or x changes
// (every kernel argument is fixed; each system's iteration number lives on
// the device).  Projection times come from event pairs captured around each
// factor sweep and are harvested once the stream has been synchronised.
// *ran is false when capture is not available (then the caller launches the
// iterations itself, and this context stops trying).
bc_status group_graph(bc_ctx* c, double* x, const OuterState& S, int G, bool* ran) {
  *ran = false;
  hipStream_t st = c->stream;
  // everything else in S is fixed for the context
  const bool same_state = c->gS.maxit == S.maxit && c->gS.use_backward == S.use_backward &&
                          c->gS.tol_bw == S.tol_bw && c->gS.rec_stop == S.rec_stop &&
                          c->gS.done == S.done;
  if (!c->gexec || c->gx != x || c->gG != G || !same_state) {
    if (c->gexec) {
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
    if (!c->d_stamps) {
      BC_TRY(c->arena.alloc(&c->d_stamps, 2 * 64));
      int dev = 0, khz = 0;
      BC_HIP(hipGetDevice(&dev));
      BC_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
      c->wall_khz = khz;
    }
    if (G > 64) {
      c->graph_off = true;
      return BC_OK;
    }
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      c->graph_off = true;
      return BC_OK;
    }
    bool ok = true;
    for (int q = 0; q < G && ok; ++q) {
      ok = spmv_a(c, st, c->lanes, c->d_p, c->d_u, S, true) == hipSuccess &&
           launch_stamp(st, c->d_stamps, 2 * q) == hipSuccess &&
           launch_dense_apply(st, c->dense, c->mixed, c->d_u, c->d_y, c->d_done, c->dense_max_nt) == hipSuccess &&
           launch_band_apply(st, c->band, c->mixed, c->d_u, c->d_y, c->d_done) == hipSuccess &&
           launch_stamp(st, c->d_stamps, 2 * q + 1) == hipSuccess &&
           spmv_t(c, st, c->lanesT, c->d_y, c->d_psi, c->d_p, S) == hipSuccess &&
           launch_update_xrs(st, x, c->d_r, c->d_s, c->d_p, c->d_psi, c->d_u, S) == hipSuccess &&
           launch_update_p(st, c->d_p, c->d_r, S) == hipSuccess;
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    hipGraphExec_t ex = nullptr;
    if (ok && ec == hipSuccess && g && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) {
      c->gexec = ex;
    } else {
      (void)hipGetLastError();
      c->graph_off = true;
    }
    if (g) (void)hipGraphDestroy(g);
    if (!c->gexec) return BC_OK;
    c->gS = S;
    c->gx = x;
    c->gG = G;
  }
  BC_HIP(hipGraphLaunch(c->gexec, st));
  *ran = true;
  c->graph_pending = G;
  return BC_OK;
}

// Adds the projection times of the last graph replay (stream synchronised):
// wall-clock stamps written by the device right before and after each sweep.
bc_status harvest_graph_events(bc_ctx* c) {
  if (c->graph_pending == 0) return BC_OK;
  std::vector<unsigned long long> t(2 * c->graph_pending);
  BC_HIP(hipMemcpy(t.data(), c->d_stamps, t.size() * sizeof(t[0]), hipMemcpyDeviceToHost));
  if (c->wall_khz > 0.0)
    for (int q = 0; q < c->graph_pending; ++q) {
      c->t_proj_ms += (double)(t[2 * q + 1] - t[2 * q]) / c->wall_khz;
      ++c->proj_launches;
    }
  c->graph_pending = 0;
  return BC_OK;
}

// Per-system statistics of a finished solve: the FP64 true residual of x and
// the normwise backward error of eq. (stopping), reduced on the device.
bc_status fill_stats(bc_ctx* c, double* x, const OuterState& S, const std::vector<int>& iters,
                     const std::vector<int>& status, const std::vector<int>& replacements,
                     double t_ms, double pbytes, unsigned long long inner_total, bc_stats* stats) {
  hipStream_t st = c->stream;
  const int ns = c->nsys;
  BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, S, nullptr));
  BC_HIP(launch_init_norms(st, c->d_f, c->d_s, x, c->d_part_f, S));
  BC_HIP(launch_final_stats(st, c->d_part_f, S, c->d_final));
  std::vector<double> fin((size_t)5 * ns);
  BC_HIP(hipMemcpyAsync(fin.data(), c->d_final, fin.size() * sizeof(double), hipMemcpyDeviceToHost,
                        st));
  BC_HIP(hipStreamSynchronize(st));
  for (int s2 = 0; s2 < ns; ++s2) {
    const double ss = fin[5 * s2], ff = fin[5 * s2 + 1], smax = fin[5 * s2 + 2];
    const double fmax = fin[5 * s2 + 3], x1 = fin[5 * s2 + 4];
    bc_stats& q = stats[s2];
    q.iterations = iters[s2];
    q.status = status[s2];
    q.rel_residual = ff > 0 ? std::sqrt(ss / ff) : 0.0;
    const double den = c->normA_inf[s2] * x1 + fmax;
    q.backward_err = den > 0 ? smax / den : 0.0;
    q.t_solve_ms = t_ms;
    q.t_proj_ms = c->t_proj_ms;
    q.proj_launches = c->proj_launches;
    q.proj_bytes = pbytes;
    q.replacements = replacements[s2];
    q.inner_iterations = (int64_t)inner_total;
  }
  return BC_OK;
}

bc_status solve_impl(bc_ctx* c, const double* f, const double* x0, double tol, int maxit,
                     double* x, bc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!f || !x || !(tol >= 0.0) || maxit < 0) {
    bc_set_error("bc_solve: null f/x, negative tol or maxit");
    return BC_ERR_INVALID;
  }
  const bc_opts& o = c->opts;
  hipStream_t st = c->stream;
  const int n = c->n_total, ns = c->nsys;
  const bool backward = o.stop_rule == BC_STOP_BACKWARD_ERR;
  const bool verbose = std::getenv("BC_VERBOSE") != nullptr;
  if (backward && c->spmv32) {
    bc_set_error("the backward-error stop rule needs FP64 sparse products (not BC_MIXED)");
    return BC_ERR_INVALID;
  }
  BC_TRY(enter(c, o.stream));
  BC_TRY(clear_wait_error(c));
  OuterState S = c->outer(maxit, backward ? 1 : 0);
  S.tol_bw = tol;
  // f in block order, x = x0 (or 0), s = f - A x
  BC_HIP(launch_gather(st, f, c->d_perm, c->d_f, n));
  if (x0) BC_HIP(launch_copy(st, x0, x, n)); else BC_HIP(launch_zero(st, x, n));
  BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, S, nullptr));
  BC_HIP(launch_init_norms(st, c->d_f, c->d_s, x, c->d_part_f, S));
  BC_HIP(launch_set_thresholds(st, c->d_part_f, backward ? 0.0 : tol, S));
  BC_HIP(hipMemsetAsync(c->d_inner_total, 0, sizeof(unsigned long long), st));
  BC_TRY(reset_proj_counters(c));
  c->timing = !c->noalloc;
  // r = sum_i A_i^+ (f_i - A_i x0) = A^T D^{-1} s ; p = r
  BC_TRY(block_solves(c, c->d_s, c->d_y, c->d_done));
  BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_r, c->d_p, S));
  BC_HIP(launch_init_cg(st, c->d_p, c->d_r, S));

  // Outer iterations run in groups of G between host checks; with FP32
  // sparse products and inner CG (BC_MIXED) G divides replace_every, so
  // replacements fall between groups.  BC_MIXED_PROJ applies its FP32 operator
  // copies in FP64 arithmetic: the operator is the same at every application
  // and the FP64 recursion needs no replacement.
  int G = std::max(1, o.check_every);
  if (c->spmv32 && o.replace_every > 0) G = std::gcd(G, o.replace_every);
  const bool graphs = o.use_graph && c->inner.nblk == 0 && !c->graph_off && c->mrhs.nrhs == 0 &&
                      !c->noalloc;
  std::vector<int> done(ns, 0), status(ns, 0), iters(ns, 0);
  std::vector<int> verified(ns, 0), replacements(ns, 0);
  int it = 0;
  BC_HIP(hipMemcpyAsync(done.data(), c->d_done, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  bool all_done = std::all_of(done.begin(), done.end(), [](int d) { return d != 0; });
  while (!all_done && it < maxit) {
    const int steps = std::min(G, maxit - it);
    bool replayed = false;
    if (graphs && steps == G && !c->graph_off) {
      BC_TRY(group_graph(c, x, S, G, &replayed));
      if (replayed) it += G;
    }
    if (!replayed) {
      for (int q = 0; q < steps; ++q) {
        ++it;
        BC_TRY(outer_iteration(c, x, S, true));
      }
    }
    if (c->spmv32 && o.replace_every > 0 && it % o.replace_every == 0) {
      // FP64 true residual s = f - A x (and, with FP32 sparse products, the
      // stop test on it), then r = A^T D^{-1} s through the working-precision
      // projections.  With factor-based projections the FP32 operator is the
      // same at every application: r and r.r are replaced and the search
      // direction is kept (a reliable update), unless the new residual is
      // more than twice the recursive one (the recursion had drifted: near
      // the attainable accuracy of the FP32 operator), where CG restarts.
      // With (FP32) inner-CG projections the operator changes from one
      // application to the next, and CG always restarts with p = r: each
      // cycle is then a defect correction of x by replace_every CG steps.
      BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, S, nullptr));
      if (c->spmv32) BC_HIP(launch_true_check(st, S));
      BC_TRY(block_solves(c, c->d_s, c->d_y, c->d_done));
      BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_r, c->d_p, S));
      if (c->inner.nblk > 0) {
        BC_HIP(launch_init_cg(st, c->d_p, c->d_r, S));
      } else {
        BC_HIP(launch_sqnorm_tiles(st, c->d_r, c->d_part_b, S));
        BC_HIP(launch_replace_decide(st, S, c->d_restart, c->d_p, c->d_r));
      }
      for (int s2 = 0; s2 < ns; ++s2) replacements[s2]++;
    }
    BC_HIP(hipMemcpyAsync(done.data(), c->d_done, ns * sizeof(int), hipMemcpyDeviceToHost, st));
    BC_HIP(hipMemcpyAsync(status.data(), c->d_status, ns * sizeof(int), hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    harvest_proj_events(c);
    BC_TRY(harvest_graph_events(c));
    if (verbose) {
      std::vector<double> hs(ns), th(ns);
      BC_HIP(hipMemcpy(hs.data(), c->d_hist, ns * sizeof(double), hipMemcpyDeviceToHost));
      BC_HIP(hipMemcpy(th.data(), c->d_thr, ns * sizeof(double), hipMemcpyDeviceToHost));
      int nd = 0;
      double worst = 0.0;
      for (int s2 = 0; s2 < ns; ++s2) {
        nd += done[s2] != 0;
        if (!done[s2] && th[s2] > 0) worst = std::max(worst, std::sqrt(hs[s2] / th[s2]) * tol);
      }
      std::fprintf(stderr, "[bc] it=%d done=%d/%d max_rel_res(recursive)=%.3e proj_ms=%.1f\n", it,
                   nd, ns, worst, c->t_proj_ms);
      std::fflush(stderr);
    }
    // verify newly converged systems on the true residual; resume those that fail
    std::vector<int> mask(ns, 0);
    bool any = false;
    for (int s2 = 0; s2 < ns; ++s2)
      if (done[s2] && status[s2] == BC_OK && !verified[s2] && !backward) {
        mask[s2] = 1;
        any = true;
      }
    if (any) {
      BC_HIP(hipMemcpyAsync(c->d_mask, mask.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
      BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, S, c->d_mask));
      std::vector<double> pc(c->ntiles), thr(ns);
      std::vector<int> st_h(c->ntiles + 1);
      BC_HIP(hipMemcpyAsync(pc.data(), c->d_part_c, c->ntiles * sizeof(double), hipMemcpyDeviceToHost, st));
      BC_HIP(hipMemcpyAsync(thr.data(), c->d_thr, ns * sizeof(double), hipMemcpyDeviceToHost, st));
      BC_HIP(hipStreamSynchronize(st));
      std::vector<int> sys_tile(ns + 1);
      BC_HIP(hipMemcpy(sys_tile.data(), c->d_sys_tile, (ns + 1) * sizeof(int), hipMemcpyDeviceToHost));
      bool resume = false;
      for (int s2 = 0; s2 < ns; ++s2) {
        if (!mask[s2]) continue;
        double ss = 0.0;
        for (int tt = sys_tile[s2]; tt < sys_tile[s2 + 1]; ++tt) ss += pc[tt];
        if (ss <= thr[s2]) {
          verified[s2] = 1;
        } else {
          done[s2] = 0;
          resume = true;
          replacements[s2]++;
        }
      }
      if (resume) {
        BC_HIP(hipMemcpyAsync(c->d_done, done.data(), ns * sizeof(int), hipMemcpyHostToDevice, st));
        BC_HIP(hipStreamSynchronize(st));
      }
    }
    all_done = std::all_of(done.begin(), done.end(), [](int d) { return d != 0; });
  }
  // final bookkeeping
  BC_HIP(hipMemcpyAsync(iters.data(), c->d_iters, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  BC_HIP(hipMemcpyAsync(status.data(), c->d_status, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  unsigned long long inner_total = 0;
  BC_HIP(hipMemcpyAsync(&inner_total, c->d_inner_total, sizeof(inner_total), hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  harvest_proj_events(c);
  c->timing = false;
  double pbytes = 0.0;
  BC_TRY(proj_bytes(c, &pbytes));
  for (int s2 = 0; s2 < ns; ++s2)
    if (!done[s2]) status[s2] = BC_NOT_CONVERGED;
  // a wait that gave up invalidates the result; the stats and the stream
  // order are still completed before the error is returned
  const bc_status werr = check_wait_error(c);
  const double t_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    BC_TRY(fill_stats(c, x, S, iters, status, replacements, t_ms, pbytes, inner_total, stats));
  BC_TRY(leave(c, o.stream));
  if (werr != BC_OK) return werr;
  int worst = BC_OK;
  for (int s2 = 0; s2 < ns; ++s2) {
    const int v = status[s2];
    if (v < 0 && (worst >= 0 || v < worst)) worst = v;
    else if (v > 0 && worst == BC_OK) worst = v;
  }
  return (bc_status)worst;
}

// Algorithm 1 (plain block Cimmino): per iteration s = f - A x in FP64, the
// stop test on it, y_i = (A_i A_i^T)^{-1} s_i through the block projections,
// and x += omega A^T y, i.e. x += omega sum_i A_i^+ (f_i - A_i x).  The
// iteration count is the number of updates made (as for Algorithm 2).
bc_status cimmino_impl(bc_ctx* c, const double* f, const double* x0, double omega, double tol,
                       int maxit, double* x, bc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!f || !x || !(tol >= 0.0) || maxit < 0 || !(omega > 0.0) || !std::isfinite(omega)) {
    bc_set_error("bc_cimmino: null f/x, negative tol or maxit, or omega not positive");
    return BC_ERR_INVALID;
  }
  const bc_opts& o = c->opts;
  if (o.stop_rule != BC_STOP_REL2) {
    bc_set_error("bc_cimmino stops on the relative residual only (stop_rule BC_STOP_REL2)");
    return BC_ERR_INVALID;
  }
  hipStream_t st = c->stream;
  const int n = c->n_total, ns = c->nsys;
  BC_TRY(enter(c, o.stream));
  BC_TRY(clear_wait_error(c));
  OuterState S = c->outer(maxit, 0);
  BC_HIP(launch_gather(st, f, c->d_perm, c->d_f, n));
  if (x0) BC_HIP(launch_copy(st, x0, x, n)); else BC_HIP(launch_zero(st, x, n));
  BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, S, nullptr));
  BC_HIP(launch_init_norms(st, c->d_f, c->d_s, x, c->d_part_f, S));
  BC_HIP(launch_set_thresholds(st, c->d_part_f, tol, S));
  BC_HIP(hipMemsetAsync(c->d_inner_total, 0, sizeof(unsigned long long), st));
  BC_TRY(reset_proj_counters(c));
  c->timing = true;
  const int G = std::max(1, o.check_every);
  std::vector<int> done(ns, 0), status(ns, 0), iters(ns, 0), replacements(ns, 0);
  int passes = 0;
  bool all_done = false;
  while (!all_done) {
    // one pass more than maxit updates: the last pass only tests the stop rule
    for (int q = 0; q < G && passes <= maxit; ++q, ++passes) {
      if (passes > 0) BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, S, nullptr));
      BC_HIP(launch_cimmino_check(st, S));
      BC_TRY(block_solves(c, c->d_s, c->d_y, c->d_done));
      BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_psi, c->d_p, S));
      BC_HIP(launch_cimmino_update(st, x, c->d_psi, omega, S));
    }
    BC_HIP(hipMemcpyAsync(done.data(), c->d_done, ns * sizeof(int), hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    harvest_proj_events(c);
    all_done = passes > maxit || std::all_of(done.begin(), done.end(), [](int d) { return d != 0; });
  }
  BC_HIP(hipMemcpyAsync(iters.data(), c->d_iters, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  BC_HIP(hipMemcpyAsync(status.data(), c->d_status, ns * sizeof(int), hipMemcpyDeviceToHost, st));
  unsigned long long inner_total = 0;
  BC_HIP(hipMemcpyAsync(&inner_total, c->d_inner_total, sizeof(inner_total), hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  harvest_proj_events(c);
  c->timing = false;
  double pbytes = 0.0;
  BC_TRY(proj_bytes(c, &pbytes));
  for (int s2 = 0; s2 < ns; ++s2)
    if (!done[s2]) status[s2] = BC_NOT_CONVERGED;
  // a wait that gave up invalidates the result; the stats and the stream
  // order are still completed before the error is returned
  const bc_status werr = check_wait_error(c);
  const double t_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    BC_TRY(fill_stats(c, x, S, iters, status, replacements, t_ms, pbytes, inner_total, stats));
  BC_TRY(leave(c, o.stream));
  if (werr != BC_OK) return werr;
  int worst = BC_OK;
  for (int s2 = 0; s2 < ns; ++s2) {
    const int v = status[s2];
    if (v < 0 && (worst >= 0 || v < worst)) worst = v;
    else if (v > 0 && worst == BC_OK) worst = v;
  }
  return (bc_status)worst;
}

}  // namespace

extern "C" bc_status bc_solve(bc_ctx* c, const double* f, const double* x0, double tol,
                              int32_t maxit, double* x, bc_stats* stats) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  if (c->nsys != 1) {
    bc_set_error("bc_solve on a batched context: use bc_solve_batched");
    return BC_ERR_INVALID;
  }
  return solve_impl(c, f, x0, tol, maxit, x, stats);
}

// ------------------------------------------------ solve without allocation
// The seven work vectors of the outer iteration (f in block order, r, p, psi,
// s, u = A p, y) live in this file-scope array during bc_solve_noalloc
// instead of the context's own vectors; every GPU the library runs on holds
// its copy until the process ends.  Host code takes its address per device
// with hipGetSymbolAddress (the name itself is not a device address on the
// host).
constexpr size_t SCRATCH_BYTES = 256ull << 20;
constexpr int SCRATCH_VECTORS = 7;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::unordered_map<int, double*> g_scratch_ptr;  // device id -> address of its scratch

bc_status scratch_of_device(double** out) {
  int dev = 0;
  BC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      bc_set_error(std::string("bc_solve_noalloc: address of the static scratch: ") +
                   hipGetErrorString(e));
      return BC_ERR_DEVICE;
    }
    it = g_scratch_ptr.emplace(dev, (double*)ptr).first;
  }
  *out = it->second;
  return BC_OK;
}

}  // namespace

extern "C" bc_status bc_solve_noalloc(bc_ctx* c, const double* f, const double* x0, double tol,
                                      int32_t maxit, double* x, bc_stats* stats) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  if (c->mrhs.nrhs > 0) {
    bc_set_error("bc_solve_noalloc: context is inside a solve with several right-hand sides");
    return BC_ERR_INVALID;
  }
  const size_t need = (size_t)SCRATCH_VECTORS * (size_t)c->n_total * sizeof(double);
  if (need > SCRATCH_BYTES) {
    bc_set_error("bc_solve_noalloc: " + std::to_string(SCRATCH_VECTORS) + " vectors of " +
                 std::to_string(c->n_total) + " rows need " + std::to_string(need) +
                 " bytes, more than the " + std::to_string(SCRATCH_BYTES) +
                 "-byte static scratch (at most " +
                 std::to_string(SCRATCH_BYTES / (SCRATCH_VECTORS * sizeof(double))) + " rows)");
    return BC_ERR_INVALID;
  }
  double* base = nullptr;
  BC_TRY(scratch_of_device(&base));
  const size_t n = (size_t)c->n_total;
  // what the solve reads before writing must start at zero: clear the whole
  // part it uses (a kernel, no memset)
  {
    const long long words = (long long)(need / sizeof(unsigned));
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<long long>((words + 255) / 256, 4096)),
                       dim3(256), 0, c->stream, (unsigned*)base, words);
    BC_HIP(hipGetLastError());
  }
  double** vecs[SCRATCH_VECTORS] = {&c->d_f, &c->d_r, &c->d_p, &c->d_psi, &c->d_s, &c->d_u, &c->d_y};
  double* saved[SCRATCH_VECTORS];
  for (int q = 0; q < SCRATCH_VECTORS; ++q) {
    saved[q] = *vecs[q];
    *vecs[q] = base + q * n;
  }
  c->noalloc = true;
  const bc_status rc = solve_impl(c, f, x0, tol, maxit, x, stats);
  c->noalloc = false;
  for (int q = 0; q < SCRATCH_VECTORS; ++q) *vecs[q] = saved[q];
  return rc;
}

extern "C" bc_status bc_solve_batched(bc_ctx* c, const double* f, const double* x0, double tol,
                                      int32_t maxit, double* x, bc_stats* stats) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  return solve_impl(c, f, x0, tol, maxit, x, stats);
}

namespace {

// Exchanges the per-system state of the context with that of the view.
void swap_view(bc_ctx* c, MultiView& v) {
  using std::swap;
  swap(c->nsys, v.nsys);
  swap(c->n_total, v.n_total);
  swap(c->sys_off, v.sys_off);
  swap(c->normA_inf, v.normA_inf);
  swap(c->d_perm, v.d_perm);
  swap(c->ntiles, v.ntiles);
  swap(c->d_tile_start, v.d_tile_start);
  swap(c->d_tile_sys, v.d_tile_sys);
  swap(c->d_sys_tile, v.d_sys_tile);
  swap(c->d_done, v.d_done);
  swap(c->d_zero_flags, v.d_zero_flags);
  swap(c->d_iters, v.d_iters);
  swap(c->d_status, v.d_status);
  swap(c->d_pending, v.d_pending);
  swap(c->d_mask, v.d_mask);
  swap(c->d_restart, v.d_restart);
  swap(c->d_thr, v.d_thr);
  swap(c->d_rr, v.d_rr);
  swap(c->d_hist, v.d_hist);
  swap(c->d_part_a, v.d_part_a);
  swap(c->d_part_b, v.d_part_b);
  swap(c->d_part_c, v.d_part_c);
  swap(c->d_part_d, v.d_part_d);
  swap(c->d_part_e, v.d_part_e);
  swap(c->d_part_f, v.d_part_f);
  swap(c->d_part_g, v.d_part_g);
  swap(c->d_final, v.d_final);
  swap(c->d_normA, v.d_normA);
  swap(c->d_finf, v.d_finf);
  swap(c->d_r, v.d_r);
  swap(c->d_p, v.d_p);
  swap(c->d_psi, v.d_psi);
  swap(c->d_s, v.d_s);
  swap(c->d_u, v.d_u);
  swap(c->d_y, v.d_y);
  swap(c->d_f, v.d_f);
}

// The per-vector state of nrhs right-hand sides of the context's one system
// (kept for the next call with the same nrhs).
bc_status build_view(bc_ctx* c, int nrhs) {
  if (!c->mview) c->mview.reset(new MultiView());
  MultiView& v = *c->mview;
  if (v.nrhs == nrhs) return BC_OK;
  BC_HIP(hipStreamSynchronize(c->stream));
  v.arena.release();
  v.nrhs = 0;
  v.d_z = v.d_gpart = v.d_gout = v.d_coef = v.d_il = v.d_inner_r = v.d_inner_t = nullptr;
  hipStream_t st = c->stream;
  const int n1 = c->n_total, T1 = c->ntiles;
  std::vector<int> ts1(T1 + 1), perm1(n1);
  BC_HIP(hipMemcpy(ts1.data(), c->d_tile_start, ts1.size() * sizeof(int), hipMemcpyDeviceToHost));
  BC_HIP(hipMemcpy(perm1.data(), c->d_perm, perm1.size() * sizeof(int), hipMemcpyDeviceToHost));
  const size_t n = (size_t)n1 * nrhs, T = (size_t)T1 * nrhs;
  std::vector<int> tile_start(T + 1), tile_sys(T), sys_tile(nrhs + 1), perm(n), zeros(nrhs, 0);
  for (int j = 0; j < nrhs; ++j) {
    for (int t = 0; t < T1; ++t) {
      tile_start[(size_t)j * T1 + t] = j * n1 + ts1[t];
      tile_sys[(size_t)j * T1 + t] = j;
    }
    sys_tile[j] = j * T1;
    for (int i = 0; i < n1; ++i) perm[(size_t)j * n1 + i] = perm1[i] + j * n1;
  }
  tile_start[T] = (int)n;
  sys_tile[nrhs] = (int)T;
  v.nsys = nrhs;
  v.n_total = (int)n;
  v.ntiles = (int)T;
  v.sys_off.resize(nrhs + 1);
  for (int j = 0; j <= nrhs; ++j) v.sys_off[j] = j * n1;
  v.normA_inf.assign(nrhs, c->normA_inf[0]);
  Arena& A = v.arena;
  BC_TRY(A.upload(&v.d_perm, perm, st));
  BC_TRY(A.upload(&v.d_tile_start, tile_start, st));
  BC_TRY(A.upload(&v.d_tile_sys, tile_sys, st));
  BC_TRY(A.upload(&v.d_sys_tile, sys_tile, st));
  BC_TRY(A.upload(&v.d_done, zeros, st));
  BC_TRY(A.upload(&v.d_zero_flags, zeros, st));
  BC_TRY(A.upload(&v.d_iters, zeros, st));
  BC_TRY(A.upload(&v.d_status, zeros, st));
  BC_TRY(A.upload(&v.d_pending, zeros, st));
  BC_TRY(A.upload(&v.d_mask, zeros, st));
  BC_TRY(A.upload(&v.d_restart, zeros, st));
  BC_TRY(A.alloc(&v.d_thr, nrhs));
  BC_TRY(A.alloc(&v.d_rr, 2 * (size_t)nrhs));
  BC_TRY(A.alloc(&v.d_hist, nrhs));
  for (double** q : {&v.d_part_a, &v.d_part_b, &v.d_part_c, &v.d_part_d, &v.d_part_e, &v.d_part_f,
                     &v.d_part_g})
    BC_TRY(A.alloc(q, T));
  BC_TRY(A.alloc(&v.d_final, 5 * (size_t)nrhs));
  BC_TRY(A.upload(&v.d_normA, v.normA_inf, st));
  BC_TRY(A.alloc(&v.d_finf, nrhs));
  for (double** q : {&v.d_r, &v.d_p, &v.d_psi, &v.d_s, &v.d_u, &v.d_y, &v.d_f})
    BC_TRY(A.alloc(q, n));
  if (c->inner.nblk > 0) {
    BC_TRY(A.alloc(&v.d_inner_r, (size_t)nrhs * n1));
    BC_TRY(A.alloc(&v.d_inner_t, (size_t)nrhs * std::max(1, c->inner_sup_total)));
  }
  if (c->sellA.il || c->sellT.il) {
    const size_t nch = (size_t)(nrhs + SELL_MULTI_NR - 1) / SELL_MULTI_NR;
    BC_TRY(A.alloc(&v.d_il, nch * SELL_MULTI_NR * n1));
  }
  BC_HIP(hipStreamSynchronize(st));  // host staging vectors go out of scope
  v.nrhs = nrhs;
  return BC_OK;
}

}  // namespace

namespace {

// Checks shared by the entry points for several right-hand sides of one
// system, then the per-vector state for nrhs of them.
bc_status multi_begin(bc_ctx* c, int32_t nrhs, const char* who, int max_nrhs) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  if (c->nsys != 1) {
    bc_set_error(std::string(who) + " needs a one-system context (bc_setup)");
    return BC_ERR_INVALID;
  }
  if (nrhs < 1 || nrhs > max_nrhs || (long long)nrhs * c->n_total > INT32_MAX) {
    bc_set_error(std::string(who) + ": nrhs must be in [1, " + std::to_string(max_nrhs) +
                 "] and nrhs * n below 2^31");
    return BC_ERR_INVALID;
  }
  if (!c->have_sell) {
    bc_set_error(std::string(who) +
                 " needs the sliced-ELL copies of A (bc_opts.spmv_lanes = -1 builds them "
                 "whatever their padding)");
    return BC_ERR_INVALID;
  }
  return build_view(c, nrhs);
}

}  // namespace

extern "C" bc_status bc_solve_multi(bc_ctx* c, int32_t nrhs, const double* f, const double* x0,
                                    double tol, int32_t maxit, double* x, bc_stats* stats) {
  // the multi-vector kernels take one grid row per chunk of vectors, the
  // narrowest chunk being 4 (dense sweeps of the largest blocks)
  BC_TRY(multi_begin(c, nrhs, "bc_solve_multi", 65535 * 4));
  const MultiRhs m{nrhs, c->n_total, c->ntiles, c->d_tile_start, c->mview->d_il};
  swap_view(c, *c->mview);
  c->mrhs = m;
  const bc_status rc = solve_impl(c, f, x0, tol, maxit, x, stats);
  c->mrhs = MultiRhs{};
  swap_view(c, *c->mview);
  return rc;
}

namespace {

// ---- block CG on H (several right-hand sides, one Krylov space).  The small
// dense algebra runs on the host in FP64; matrices are row-major.

// M = L L^T from the lower triangle of the p x p matrix M; false if a pivot
// is not positive and finite.
bool chol_lower(const std::vector<double>& M, int p, std::vector<double>& L) {
  L.assign((size_t)p * p, 0.0);
  for (int j = 0; j < p; ++j) {
    double d = M[(size_t)j * p + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * p + k] * L[(size_t)j * p + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double ljj = std::sqrt(d);
    L[(size_t)j * p + j] = ljj;
    for (int i = j + 1; i < p; ++i) {
      double sum = M[(size_t)i * p + j];
      for (int k = 0; k < j; ++k) sum -= L[(size_t)i * p + k] * L[(size_t)j * p + k];
      L[(size_t)i * p + j] = sum / ljj;
    }
  }
  return true;
}

// B <- (L L^T)^{-1} B for B of p rows and a columns.
void chol_solve(const std::vector<double>& L, int p, std::vector<double>& B, int a) {
  for (int c = 0; c < a; ++c) {
    for (int i = 0; i < p; ++i) {
      double sum = B[(size_t)i * a + c];
      for (int k = 0; k < i; ++k) sum -= L[(size_t)i * p + k] * B[(size_t)k * a + c];
      B[(size_t)i * a + c] = sum / L[(size_t)i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {
      double sum = B[(size_t)i * a + c];
      for (int k = i + 1; k < p; ++k) sum -= L[(size_t)k * p + i] * B[(size_t)k * a + c];
      B[(size_t)i * a + c] = sum / L[(size_t)i * p + i];
    }
  }
}

// Orthonormal directions from the Gram matrix G (a x a) of the columns of Z:
// the columns scaled to unit norm, a Cholesky factorization of their Gram
// matrix column by column, a column whose pivot is at most drop left out.
// Returns r and T (a x r) with Z T = Zn[:, kept] L^{-T}, orthonormal columns.
int orth_from_gram(const std::vector<double>& G, int a, double drop, std::vector<double>& T) {
  std::vector<double> d(a);
  std::vector<int> kept;
  for (int j = 0; j < a; ++j) {
    d[j] = std::sqrt(std::max(G[(size_t)j * a + j], 0.0));
    if (d[j] > 0.0) kept.push_back(j);
  }
  const int k = (int)kept.size();
  auto gn = [&](int x, int y) {
    return G[(size_t)kept[x] * a + kept[y]] / (d[kept[x]] * d[kept[y]]);
  };
  std::vector<double> L((size_t)k * k, 0.0), l;
  std::vector<int> keep2;
  for (int q = 0; q < k; ++q) {
    const int r = (int)keep2.size();
    l.assign(r, 0.0);
    for (int i = 0; i < r; ++i) {
      double sum = gn(keep2[i], q);
      for (int m = 0; m < i; ++m) sum -= L[(size_t)i * k + m] * l[m];
      l[i] = sum / L[(size_t)i * k + i];
    }
    double piv = gn(q, q);
    for (int i = 0; i < r; ++i) piv -= l[i] * l[i];
    if (piv > drop) {
      for (int i = 0; i < r; ++i) L[(size_t)r * k + i] = l[i];
      L[(size_t)r * k + r] = std::sqrt(piv);
      keep2.push_back(q);
    }
  }
  const int r = (int)keep2.size();
  std::vector<double> Li((size_t)r * r, 0.0);  // L^{-1}, lower
  for (int c = 0; c < r; ++c)
    for (int i = c; i < r; ++i) {
      double sum = i == c ? 1.0 : 0.0;
      for (int m = c; m < i; ++m) sum -= L[(size_t)i * k + m] * Li[(size_t)m * r + c];
      Li[(size_t)i * r + c] = sum / L[(size_t)i * k + i];
    }
  T.assign((size_t)a * r, 0.0);
  for (int i = 0; i < r; ++i) {
    const int col = kept[keep2[i]];
    for (int c = 0; c < r; ++c) T[(size_t)col * r + c] = Li[(size_t)c * r + i] / d[col];
  }
  return r;
}

ColList cols(double* base, long long n1, const std::vector<int>& idx) {
  ColList L{};
  L.c = (int)idx.size();
  for (size_t q = 0; q < idx.size(); ++q) L.v[q] = base + idx[q] * n1;
  return L;
}
ColList cols_first(double* base, long long n1, int count) {
  ColList L{};
  L.c = count;
  for (int q = 0; q < count; ++q) L.v[q] = base + q * n1;
  return L;
}
ColList cat(const ColList& a, const ColList& b) {
  ColList L = a;
  for (int q = 0; q < b.c; ++q) L.v[a.c + q] = b.v[q];
  L.c = a.c + b.c;
  return L;
}

// Squared 2-norm of each of the nr vectors from per-(vector, tile) partials,
// summed in tile order.
bc_status vector_sq_norms(bc_ctx* c, const double* part, int nr, int T1, std::vector<double>& out) {
  std::vector<double> h((size_t)nr * T1);
  BC_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  BC_HIP(hipStreamSynchronize(c->stream));
  out.assign(nr, 0.0);
  for (int j = 0; j < nr; ++j)
    for (int t = 0; t < T1; ++t) out[j] += h[(size_t)j * T1 + t];
  return BC_OK;
}

// The block CG iteration of the oracle's block_cimmino_block_cg, on the view
// of nrhs right-hand sides (context state swapped in; c->mrhs set).
bc_status block_cg_impl(bc_ctx* c, const double* f, const double* x0, double tol, int maxit,
                        double* x, bc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!f || !x || !(tol >= 0.0) || maxit < 0) {
    bc_set_error("bc_solve_block: null f/x, negative tol or maxit");
    return BC_ERR_INVALID;
  }
  const bc_opts& o = c->opts;
  if (o.stop_rule != BC_STOP_REL2) {
    bc_set_error("bc_solve_block stops on the relative residual only (stop_rule BC_STOP_REL2)");
    return BC_ERR_INVALID;
  }
  MultiView& v = *c->mview;
  hipStream_t st = c->stream;
  const int nr = c->nsys, n = c->n_total;
  const int n1 = c->mrhs.n1, T1 = c->mrhs.ntiles1;
  const double drop = 1e-10;
  if (!v.d_z) {
    BC_TRY(v.arena.alloc(&v.d_z, (size_t)n));
    BC_TRY(v.arena.alloc(&v.d_gpart, (size_t)BG_GROUPS * BG_PAIRS));
    BC_TRY(v.arena.alloc(&v.d_gout, (size_t)BG_PAIRS));
    BC_TRY(v.arena.alloc(&v.d_coef, (size_t)4 * BG_MAX * BG_MAX));
    BC_HIP(prepare_block_gram());
  }
  double* coef_a = v.d_coef;
  double* coef_ma = v.d_coef + BG_MAX * BG_MAX;
  double* coef_b = v.d_coef + 2 * BG_MAX * BG_MAX;
  double* coef_t = v.d_coef + 3 * BG_MAX * BG_MAX;
  // the coefficient uploads come from host vectors that live until the
  // stream is synchronised at the next readback
  auto upload = [&](double* dst, const std::vector<double>& h) -> bc_status {
    if (!h.empty())
      BC_HIP(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st));
    return BC_OK;
  };
  auto gram = [&](const ColList& L1, const ColList& L2, std::vector<double>& out) -> bc_status {
    BC_HIP(launch_block_gram(st, L1, L2, n1, v.d_gpart, v.d_gout));
    out.resize((size_t)L1.c * L2.c);
    BC_HIP(hipMemcpyAsync(out.data(), v.d_gout, out.size() * sizeof(double), hipMemcpyDeviceToHost,
                          st));
    BC_HIP(hipStreamSynchronize(st));
    return BC_OK;
  };
  BC_TRY(enter(c, o.stream));
  BC_TRY(clear_wait_error(c));
  OuterState S = c->outer(maxit, 0);
  OuterState Sall = S;
  Sall.done = c->d_zero_flags;
  // f in block order, x = x0 (or 0), s = f - A x, ||f||^2 and ||s||^2 per vector
  BC_HIP(launch_gather(st, f, c->d_perm, c->d_f, n));
  if (x0) BC_HIP(launch_copy(st, x0, x, n)); else BC_HIP(launch_zero(st, x, n));
  BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, Sall, nullptr));
  BC_HIP(launch_sqnorm_tiles(st, c->d_f, c->d_part_f, Sall));
  std::vector<double> ff, ss;
  BC_TRY(vector_sq_norms(c, c->d_part_f, nr, T1, ff));
  BC_TRY(vector_sq_norms(c, c->d_part_c, nr, T1, ss));
  BC_HIP(hipMemsetAsync(c->d_inner_total, 0, sizeof(unsigned long long), st));
  BC_TRY(reset_proj_counters(c));
  c->timing = true;
  std::vector<int> iters(nr, 0), status(nr, BC_NOT_CONVERGED), replacements(nr, 0), act;
  for (int j = 0; j < nr; ++j) {
    if (ff[j] == 0.0 || std::sqrt(ss[j]) <= tol * std::sqrt(ff[j])) status[j] = BC_OK;
    else act.push_back(j);
  }
  std::vector<int> flags(nr);
  // device flags per vector: 1 for the active vectors (or for the others)
  auto set_flags = [&](int* dev, bool mark_active) -> bc_status {
    for (int j = 0; j < nr; ++j) flags[j] = mark_active ? 0 : 1;
    for (int j : act) flags[j] = mark_active ? 1 : 0;
    BC_HIP(hipMemcpyAsync(dev, flags.data(), nr * sizeof(int), hipMemcpyHostToDevice, st));
    BC_HIP(hipStreamSynchronize(st));  // flags is reused
    return BC_OK;
  };
  std::vector<double> G, T, M, Lm, PQ, alpha, malpha, beta, QRn;
  if (!act.empty()) {
    // R = Xi - H X = A^T D^{-1} s for the active vectors (done marks the others)
    BC_TRY(set_flags(c->d_done, false));
    OuterState Sact = S;
    Sact.done = c->d_done;
    BC_TRY(block_solves(c, c->d_s, c->d_y, c->d_done));
    BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_r, c->d_p, Sact));
    // first directions: an orthonormal basis of the active columns of R
    ColList Ract = cols(c->d_r, n1, act);
    BC_TRY(gram(Ract, Ract, G));
    int p = orth_from_gram(G, (int)act.size(), drop, T);
    BC_TRY(upload(coef_t, T));
    BC_HIP(launch_block_combine(st, Ract, cols_first(c->d_p, n1, p), ColList{}, coef_t, n1));
    for (int t = 1; t <= maxit; ++t) {
      if (p == 0) {
        for (int j : act) status[j] = BC_ERR_BREAKDOWN;
        break;
      }
      const int a = (int)act.size();
      // Q = H P for the p directions
      c->mrhs.nrhs = p;
      BC_HIP(spmv_a(c, st, c->lanes, c->d_p, c->d_u, Sall, false));
      const bc_status rs = block_solves(c, c->d_u, c->d_y, nullptr);
      if (rs == BC_OK) BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_psi, c->d_p, Sall));
      c->mrhs.nrhs = nr;
      BC_TRY(rs);
      const ColList P = cols_first(c->d_p, n1, p), Q = cols_first(c->d_psi, n1, p);
      Ract = cols(c->d_r, n1, act);
      // [P Q]^T [Q R_act]: M = P^T Q, P^T R, Q^T Q, Q^T R
      BC_TRY(gram(cat(P, Q), cat(Q, Ract), PQ));
      const int c2 = p + a;
      M.assign((size_t)p * p, 0.0);
      alpha.assign((size_t)p * a, 0.0);
      for (int i = 0; i < p; ++i) {
        for (int k = 0; k < p; ++k) M[(size_t)i * p + k] = PQ[(size_t)i * c2 + k];
        for (int j = 0; j < a; ++j) alpha[(size_t)i * a + j] = PQ[(size_t)i * c2 + p + j];
      }
      if (!chol_lower(M, p, Lm)) {
        for (int j : act) status[j] = BC_ERR_BREAKDOWN;
        break;
      }
      chol_solve(Lm, p, alpha, a);
      malpha.resize(alpha.size());
      for (size_t e = 0; e < alpha.size(); ++e) malpha[e] = -alpha[e];
      BC_TRY(upload(coef_a, alpha));
      BC_TRY(upload(coef_ma, malpha));
      const ColList Xact = cols(x, n1, act);
      BC_HIP(launch_block_combine(st, P, Xact, Xact, coef_a, n1));
      BC_HIP(launch_block_combine(st, Q, Ract, Ract, coef_ma, n1));
      // true residuals of the active vectors and the stop test
      BC_TRY(set_flags(c->d_mask, true));
      BC_HIP(residual_a(c, st, c->lanes, x, c->d_f, c->d_s, Sall, c->d_mask));
      BC_TRY(vector_sq_norms(c, c->d_part_c, nr, T1, ss));
      harvest_proj_events(c);
      std::vector<int> still, pos;  // pos: index of each remaining vector in act
      for (int q = 0; q < a; ++q) {
        const int j = act[q];
        iters[j] = t;
        if (std::sqrt(ss[j]) <= tol * std::sqrt(ff[j])) {
          status[j] = BC_OK;
        } else {
          still.push_back(j);
          pos.push_back(q);
        }
      }
      act = still;
      if (act.empty()) break;
      const int a2 = (int)act.size();
      if (c->spmv32 && o.replace_every > 0 && t % o.replace_every == 0) {
        // FP32 projections: the recursive R drifts from Xi - H X by the
        // rounding of the FP32 operator, so every replace_every iterations R
        // is recomputed from the true residual, R = A^T D^{-1} s, and the
        // iteration restarts with directions from it
        BC_TRY(set_flags(c->d_done, false));
        OuterState Sact = S;
        Sact.done = c->d_done;
        BC_TRY(block_solves(c, c->d_s, c->d_y, c->d_done));
        BC_HIP(spmv_t(c, st, c->lanesT, c->d_y, c->d_r, c->d_psi, Sact));
        Ract = cols(c->d_r, n1, act);
        BC_TRY(gram(Ract, Ract, G));
        p = orth_from_gram(G, a2, drop, T);
        BC_TRY(upload(coef_t, T));
        BC_HIP(launch_block_combine(st, Ract, cols_first(c->d_p, n1, p), ColList{}, coef_t, n1));
        for (int j : act) replacements[j]++;
        continue;
      }
      // Q^T R after the update = Q^T R - (Q^T Q) alpha; beta = -M^{-1} Q^T R
      QRn.assign((size_t)p * a2, 0.0);
      for (int i = 0; i < p; ++i)
        for (int q = 0; q < a2; ++q) {
          double sum = PQ[(size_t)(p + i) * c2 + p + pos[q]];
          for (int k = 0; k < p; ++k)
            sum -= PQ[(size_t)(p + i) * c2 + k] * alpha[(size_t)k * a + pos[q]];
          QRn[(size_t)i * a2 + q] = sum;
        }
      chol_solve(Lm, p, QRn, a2);
      beta.resize(QRn.size());
      for (size_t e = 0; e < QRn.size(); ++e) beta[e] = -QRn[e];
      // Z = R_act + P beta, then its orthonormal basis as the next directions
      Ract = cols(c->d_r, n1, act);
      const ColList Z = cols_first(v.d_z, n1, a2);
      BC_TRY(upload(coef_b, beta));
      BC_HIP(launch_block_combine(st, P, Z, Ract, coef_b, n1));
      BC_TRY(gram(Z, Z, G));
      p = orth_from_gram(G, a2, drop, T);
      BC_TRY(upload(coef_t, T));
      BC_HIP(launch_block_combine(st, Z, cols_first(c->d_p, n1, p), ColList{}, coef_t, n1));
    }
  }
  unsigned long long inner_total = 0;
  BC_HIP(hipMemcpyAsync(&inner_total, c->d_inner_total, sizeof(inner_total), hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  harvest_proj_events(c);
  c->timing = false;
  double pbytes = 0.0;
  BC_TRY(proj_bytes(c, &pbytes));
  // a wait that gave up invalidates the result; the stats and the stream
  // order are still completed before the error is returned
  const bc_status werr = check_wait_error(c);
  const double t_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    BC_TRY(fill_stats(c, x, Sall, iters, status, replacements, t_ms, pbytes, inner_total, stats));
  BC_TRY(leave(c, o.stream));
  if (werr != BC_OK) return werr;
  int worst = BC_OK;
  for (int j = 0; j < nr; ++j) {
    const int sv = status[j];
    if (sv < 0 && (worst >= 0 || sv < worst)) worst = sv;
    else if (sv > 0 && worst == BC_OK) worst = sv;
  }
  return (bc_status)worst;
}

}  // namespace

extern "C" bc_status bc_solve_block(bc_ctx* c, int32_t nrhs, const double* f, const double* x0,
                                    double tol, int32_t maxit, double* x, bc_stats* stats) {
  BC_TRY(multi_begin(c, nrhs, "bc_solve_block", BG_MAX / 2));
  const MultiRhs m{nrhs, c->n_total, c->ntiles, c->d_tile_start, c->mview->d_il};
  swap_view(c, *c->mview);
  c->mrhs = m;
  const bc_status rc = block_cg_impl(c, f, x0, tol, maxit, x, stats);
  c->mrhs = MultiRhs{};
  swap_view(c, *c->mview);
  return rc;
}

extern "C" bc_status bc_cimmino(bc_ctx* c, const double* f, const double* x0, double omega,
                                double tol, int32_t maxit, double* x, bc_stats* stats) {
  if (!c) {
    bc_set_error("ctx is null");
    return BC_ERR_INVALID;
  }
  return cimmino_impl(c, f, x0, omega, tol, maxit, x, stats);
}

// ------------------------------------------------------- row inner-product graph

namespace {
thread_local double g_rip_spgemm_ms = 0.0, g_rip_total_ms = 0.0;

template <typename T>
bc_status d2h(std::vector<T>& h, const T* d, size_t count, hipStream_t st) {
  h.resize(count);
  if (count) BC_HIP(hipMemcpyAsync(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost, st));
  return BC_OK;
}

bc_status rip_impl(int32_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                   const rip_opts& o, rip_graph_t* out, hipStream_t st, Arena& A) {
  const auto t0 = std::chrono::steady_clock::now();
  const long long nnz = rowptr[n];
  // A straight from the caller's arrays; A^T, dense columns and the
  // compacted column lists are built on the device
  int *d_rowptr, *d_col, *d_flag;
  double *d_aval, *d_nrm;
  BC_TRY(A.alloc(&d_rowptr, (size_t)n + 1));
  BC_TRY(A.alloc(&d_col, (size_t)nnz));
  BC_TRY(A.alloc(&d_aval, (size_t)nnz));
  BC_HIP(hipMemcpyAsync(d_rowptr, rowptr, ((size_t)n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  if (nnz > 0) {
    BC_HIP(hipMemcpyAsync(d_col, colidx, (size_t)nnz * sizeof(int), hipMemcpyHostToDevice, st));
    BC_HIP(hipMemcpyAsync(d_aval, vals, (size_t)nnz * sizeof(double), hipMemcpyHostToDevice, st));
  }
  std::vector<int> flags(3, 0);
  BC_TRY(A.upload(&d_flag, flags, st));  // [0] zero row, [1] weight overflow, [2] dense columns
  BC_TRY(A.alloc(&d_nrm, n));
  if (o.prescale) BC_HIP(rip_launch_prescale(st, n, d_rowptr, d_aval, d_nrm, d_flag));
  int *d_erow, *d_iota, *d_tcnt, *d_tptr, *d_trow, *d_tpos;
  unsigned* d_tkey;
  double* d_tval;
  void* d_temp;
  const size_t temp_bytes = std::max(rip_transpose_temp_bytes(n, nnz), rip_offsets_temp_bytes(n));
  BC_TRY(A.alloc(&d_erow, (size_t)nnz));
  BC_TRY(A.alloc(&d_iota, (size_t)nnz));
  BC_TRY(A.alloc(&d_tkey, (size_t)nnz));
  BC_TRY(A.alloc(&d_tcnt, (size_t)n + 1));
  BC_TRY(A.alloc(&d_tptr, (size_t)n + 1));
  BC_TRY(A.alloc(&d_trow, (size_t)nnz));
  BC_TRY(A.alloc(&d_tpos, (size_t)nnz));
  BC_TRY(A.alloc(&d_tval, (size_t)nnz));
  BC_TRY(A.alloc((char**)&d_temp, temp_bytes));
  BC_HIP(rip_launch_transpose(st, n, nnz, d_rowptr, d_col, d_aval, d_erow, d_tkey, d_iota, d_tcnt,
                              d_tptr, d_trow, d_tval, d_tpos, d_temp, temp_bytes));
  if (o.sparsify) {
    int t = (int)std::sqrt((double)n);
    while ((long long)(t + 1) * (t + 1) <= n) ++t;
    while ((long long)t * t > n) --t;
    int* d_dense;
    BC_TRY(A.alloc(&d_dense, n));
    BC_HIP(rip_launch_dense_cols(st, n, d_tptr, t, d_dense, d_flag + 2));
    int ndense = 0;
    BC_HIP(hipMemcpyAsync(&ndense, d_flag + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    BC_HIP(rip_launch_sparsify(st, d_dense, ndense, t, d_tptr, d_trow, d_tval, d_tpos, d_aval));
  }
  // compact the column lists (drop zero entries)
  int *d_ccnt, *d_cptr, *d_crow;
  double* d_cval;
  BC_TRY(A.alloc(&d_ccnt, (size_t)n + 1));
  BC_TRY(A.alloc(&d_cptr, (size_t)n + 1));
  BC_TRY(A.alloc(&d_crow, (size_t)nnz));
  BC_TRY(A.alloc(&d_cval, (size_t)nnz));
  BC_HIP(rip_launch_col_nonzeros(st, n, d_tptr, d_tval, d_ccnt));
  BC_HIP(rip_launch_scan_int(st, d_ccnt, d_cptr, n, d_temp, temp_bytes));
  BC_HIP(rip_launch_compact(st, n, d_tptr, d_trow, d_tval, d_cptr, d_crow, d_cval));
  // products per row -> short (LDS table) and long (global table) rows
  long long* d_ub;
  BC_TRY(A.alloc(&d_ub, n));
  BC_HIP(rip_launch_row_products(st, n, d_rowptr, d_col, d_aval, d_cptr, d_ub));
  std::vector<long long> ub;
  BC_TRY(d2h(ub, d_ub, n, st));
  std::vector<int> flags_h(2);
  BC_HIP(hipMemcpyAsync(flags_h.data(), d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  if (flags_h[0]) {
    bc_set_error("rip_graph: a row of A is zero, cannot prescale");
    return BC_ERR_INVALID;
  }
  std::vector<int> short_rows, long_rows, tsize;
  std::vector<long long> toff;
  long long ttot = 0;
  for (int i = 0; i < n; ++i) {
    if (ub[i] <= rip_short_max()) {
      short_rows.push_back(i);
    } else {
      long long s = 64;
      while (s < 2 * ub[i]) s <<= 1;
      if (s > (1LL << 30)) {
        bc_set_error("rip_graph: row " + std::to_string(i) + " has too many products");
        return BC_ERR_INVALID;
      }
      long_rows.push_back(i);
      tsize.push_back((int)s);
      toff.push_back(ttot);
      ttot += s;
    }
  }
  int *d_srows = nullptr, *d_lrows = nullptr, *d_tsize = nullptr, *d_gkeys = nullptr, *d_cnt;
  long long* d_toff = nullptr;
  double* d_gvals = nullptr;
  BC_TRY(A.upload(&d_srows, short_rows, st));
  BC_TRY(A.upload(&d_lrows, long_rows, st));
  BC_TRY(A.upload(&d_tsize, tsize, st));
  BC_TRY(A.upload(&d_toff, toff, st));
  BC_TRY(A.alloc(&d_gkeys, ttot));
  BC_TRY(A.alloc(&d_gvals, ttot));
  BC_TRY(A.alloc(&d_cnt, n));
  hipEvent_t e0, e1, e2, e3;
  BC_HIP(hipEventCreate(&e0));
  BC_HIP(hipEventCreate(&e1));
  BC_HIP(hipEventCreate(&e2));
  BC_HIP(hipEventCreate(&e3));
  const double alpha = (double)o.alpha;
  BC_HIP(hipEventRecord(e0, st));
  BC_HIP(rip_launch_short(st, false, d_srows, (int)short_rows.size(), d_rowptr, d_col, d_aval,
                          d_cptr, d_crow, d_cval, d_cnt, nullptr, nullptr, nullptr, nullptr, alpha,
                          d_flag + 1));
  BC_HIP(rip_launch_long(st, false, d_lrows, (int)long_rows.size(), d_toff, d_tsize, d_rowptr,
                         d_col, d_aval, d_cptr, d_crow, d_cval, d_gkeys, d_gvals, d_cnt, nullptr,
                         nullptr, nullptr, nullptr, alpha, d_flag + 1));
  BC_HIP(hipEventRecord(e1, st));
  long long *d_wide, *d_optr;
  BC_TRY(A.alloc(&d_wide, (size_t)n + 1));
  BC_TRY(A.alloc(&d_optr, (size_t)n + 1));
  BC_HIP(rip_launch_offsets(st, d_cnt, d_wide, d_optr, n, d_temp, temp_bytes));
  // the result lives in pinned host memory: the copies below go straight
  // into it (released by rip_graph_free)
  out->n = n;
  if (hipHostMalloc((void**)&out->rowptr, ((size_t)n + 1) * sizeof(int64_t), hipHostMallocDefault) !=
      hipSuccess) {
    (void)hipGetLastError();
    out->rowptr = nullptr;
    bc_set_error("rip_graph: pinned host allocation failed");
    return BC_ERR_NOMEM;
  }
  BC_HIP(hipMemcpyAsync(out->rowptr, d_optr, ((size_t)n + 1) * sizeof(int64_t),
                        hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  const long long ne = out->rowptr[n];
  out->nnz = ne;
  int* d_ocol;
  double* d_ocost;
  long long* d_owgt;
  BC_TRY(A.alloc(&d_ocol, ne));
  BC_TRY(A.alloc(&d_ocost, ne));
  BC_TRY(A.alloc(&d_owgt, ne));
  BC_HIP(hipEventRecord(e2, st));
  BC_HIP(rip_launch_short(st, true, d_srows, (int)short_rows.size(), d_rowptr, d_col, d_aval,
                          d_cptr, d_crow, d_cval, nullptr, d_optr, d_ocol, d_ocost, d_owgt, alpha,
                          d_flag + 1));
  BC_HIP(rip_launch_long(st, true, d_lrows, (int)long_rows.size(), d_toff, d_tsize, d_rowptr,
                         d_col, d_aval, d_cptr, d_crow, d_cval, d_gkeys, d_gvals, nullptr, d_optr,
                         d_ocol, d_ocost, d_owgt, alpha, d_flag + 1));
  BC_HIP(hipEventRecord(e3, st));
  const size_t ne1 = (size_t)std::max<long long>(ne, 1);
  if (hipHostMalloc((void**)&out->col, ne1 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&out->cost, ne1 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&out->wgt, ne1 * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    BC_HIP(hipStreamSynchronize(st));
    bc_set_error("rip_graph: pinned host allocation failed");
    return BC_ERR_NOMEM;
  }
  if (ne) {
    BC_HIP(hipMemcpyAsync(out->col, d_ocol, ne * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    BC_HIP(hipMemcpyAsync(out->cost, d_ocost, ne * sizeof(double), hipMemcpyDeviceToHost, st));
    BC_HIP(hipMemcpyAsync(out->wgt, d_owgt, ne * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  }
  BC_HIP(hipMemcpyAsync(flags_h.data(), d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  BC_HIP(hipStreamSynchronize(st));
  float ms1 = 0.f, ms2 = 0.f;
  (void)hipEventElapsedTime(&ms1, e0, e1);
  (void)hipEventElapsedTime(&ms2, e2, e3);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  (void)hipEventDestroy(e3);
  g_rip_spgemm_ms = (double)ms1 + (double)ms2;
  g_rip_total_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (flags_h[1]) {
    bc_set_error("rip_graph: alpha * cost does not fit below 2^62");
    return BC_ERR_INVALID;
  }
  return BC_OK;
}

}  // namespace

extern "C" void rip_graph_free(rip_graph_t* g) {
  if (!g) return;
  if (g->rowptr) (void)hipHostFree(g->rowptr);
  if (g->col) (void)hipHostFree(g->col);
  if (g->cost) (void)hipHostFree(g->cost);
  if (g->wgt) (void)hipHostFree(g->wgt);
  g->rowptr = nullptr;
  g->col = nullptr;
  g->cost = nullptr;
  g->wgt = nullptr;
  g->n = 0;
  g->nnz = 0;
}

extern "C" bc_status rip_graph(int32_t n, const int32_t* rowptr, const int32_t* colidx,
                               const double* vals, const rip_opts* opts, rip_graph_t* out) {
  if (!out) {
    bc_set_error("rip_graph: out is null");
    return BC_ERR_INVALID;
  }
  std::memset(out, 0, sizeof(*out));
  BC_TRY(validate_csr(n, rowptr, colidx, vals, "rip_graph"));
  rip_opts o;
  if (opts) o = *opts; else rip_opts_default(&o);
  if (o.alpha < 1) {
    bc_set_error("rip_graph: alpha must be >= 1");
    return BC_ERR_INVALID;
  }
  BC_TRY(check_device());
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  BC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(ev, (hipStream_t)o.stream) != hipSuccess ||
      hipStreamWaitEvent(st, ev, 0) != hipSuccess) {
    (void)hipStreamDestroy(st);
    bc_set_error("rip_graph: stream ordering failed");
    return BC_ERR_DEVICE;
  }
  bc_status s;
  {
    Arena A;
    s = rip_impl(n, rowptr, colidx, vals, o, out, st, A);
    (void)hipStreamSynchronize(st);
  }
  (void)hipEventDestroy(ev);
  (void)hipStreamDestroy(st);
  if (s != BC_OK) rip_graph_free(out);
  return s;
}

extern "C" bc_status rip_graph_timing(double* spgemm_ms, double* total_ms) {
  if (spgemm_ms) *spgemm_ms = g_rip_spgemm_ms;
  if (total_ms) *total_ms = g_rip_total_ms;
  return BC_OK;
}
