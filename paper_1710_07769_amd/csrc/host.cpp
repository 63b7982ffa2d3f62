// Host-only parts of the library (declared in host.h): argument validation
// and the sliced-ELL layout.
#include "host.h"

#include <algorithm>
#include <cmath>

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;
void bc_set_error(const std::string& msg) { g_last_error = msg; }

extern "C" const char* bc_last_error(void) { return g_last_error.c_str(); }

extern "C" const char* bc_status_str(bc_status s) {
  switch (s) {
    case BC_OK: return "ok";
    case BC_NOT_CONVERGED: return "not converged";
    case BC_ERR_INVALID: return "invalid argument";
    case BC_ERR_SINGULAR_BLOCK: return "singular block";
    case BC_ERR_BREAKDOWN: return "CG breakdown";
    case BC_ERR_DEVICE: return "device error";
    case BC_ERR_NOMEM: return "out of memory";
  }
  return "unknown status";
}

extern "C" void bc_opts_default(bc_opts* o) {
  if (!o) return;
  o->precision = BC_FP64;
  o->projection = BC_PROJ_AUTO;
  o->dense_max_m = 4096;
  o->inner_tol = 1e-12;
  o->inner_maxit = 20000;
  o->inner_groups = 0;
  o->replace_every = 20;
  o->stop_rule = BC_STOP_REL2;
  o->check_every = 8;
  o->spmv_lanes = 0;
  o->use_graph = 1;
  o->multi_gather = BC_GATHER_AUTO;
  o->stream = nullptr;
}

extern "C" void rip_opts_default(rip_opts* o) {
  if (!o) return;
  o->prescale = 1;
  o->sparsify = 1;
  o->alpha = (int64_t)1 << 20;
  o->stream = nullptr;
}

bc_status validate_csr(int32_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                       const char* who) {
  if (n < 1 || !rowptr) {
    bc_set_error(std::string(who) + ": n must be >= 1 and rowptr non-null");
    return BC_ERR_INVALID;
  }
  if (rowptr[0] != 0) {
    bc_set_error(std::string(who) + ": rowptr[0] != 0");
    return BC_ERR_INVALID;
  }
  for (int32_t i = 0; i < n; ++i) {
    if (rowptr[i + 1] < rowptr[i]) {
      bc_set_error(std::string(who) + ": rowptr decreases at row " + std::to_string(i));
      return BC_ERR_INVALID;
    }
  }
  const int64_t nnz = rowptr[n];
  if (nnz > 0 && (!colidx || !vals)) {
    bc_set_error(std::string(who) + ": null colidx/vals");
    return BC_ERR_INVALID;
  }
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int32_t c = colidx[e];
      if (c < 0 || c >= n) {
        bc_set_error(std::string(who) + ": column index out of range in row " + std::to_string(i));
        return BC_ERR_INVALID;
      }
      if (e > rowptr[i] && colidx[e - 1] >= c) {
        bc_set_error(std::string(who) + ": columns not strictly ascending in row " + std::to_string(i));
        return BC_ERR_INVALID;
      }
      if (!std::isfinite(vals[e])) {
        bc_set_error(std::string(who) + ": non-finite value in row " + std::to_string(i));
        return BC_ERR_INVALID;
      }
    }
  }
  return BC_OK;
}

int choose_lanes(int64_t nnz, int64_t rows) {
  const double avg = rows ? (double)nnz / (double)rows : 1.0;
  int l = 1;
  while (l < 64 && l * 2 <= avg) l <<= 1;
  return std::max(1, std::min(64, l));
}

// Sliced-ELL copy (SellMat) of the CSR matrix (rp, ci, v) over the tiles.
// Without `force` nothing is built (false) when padding would add more than
// a quarter to the stored entries.
bool build_sell(const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<double>& v,
                const std::vector<int>& tile_start, bool force, std::vector<long long>& ptr,
                std::vector<int>& wid, std::vector<int>& col, std::vector<double>& val) {
  const int ntiles = (int)tile_start.size() - 1;
  ptr.assign((size_t)ntiles * SELL_SLICES, 0);
  wid.assign((size_t)ntiles * SELL_SLICES, 0);
  long long total = 0;
  for (int t = 0; t < ntiles; ++t)
    for (int j = 0; j < SELL_SLICES; ++j) {
      const int ra = tile_start[t] + 64 * j, rb = std::min(ra + 64, tile_start[t + 1]);
      int w = 0;
      for (int i = ra; i < rb; ++i) w = std::max(w, rp[i + 1] - rp[i]);
      ptr[(size_t)t * SELL_SLICES + j] = total;
      wid[(size_t)t * SELL_SLICES + j] = w;
      total += 64LL * w;
    }
  const long long nnz = rp.back();
  if (!force && (double)total > 1.25 * (double)nnz) return false;
  col.assign((size_t)total, 0);
  val.assign((size_t)total, 0.0);
  for (int t = 0; t < ntiles; ++t)
    for (int j = 0; j < SELL_SLICES; ++j) {
      const int ra = tile_start[t] + 64 * j;
      const long long base = ptr[(size_t)t * SELL_SLICES + j];
      const int w = wid[(size_t)t * SELL_SLICES + j];
      for (int l = 0; l < 64; ++l) {
        const int i = ra + l;
        const bool row = i < tile_start[t + 1];
        const int e0 = row ? rp[i] : 0, len = row ? rp[i + 1] - rp[i] : 0;
        const int pad = len > 0 ? ci[e0 + len - 1] : tile_start[t];
        for (int k = 0; k < w; ++k) {
          const size_t q = (size_t)(base + 64LL * k + l);
          col[q] = k < len ? ci[e0 + k] : pad;
          val[q] = k < len ? v[e0 + k] : 0.0;
        }
      }
    }
  return true;
}

// Gather layout of the multi-vector products over one sliced-ELL copy.  A
// chunk of 8 vectors gathered separately reads, per entry column of a slice,
// 8 x (distinct 64-byte segments among the 64 column indices); interleaved it
// reads one 64-byte segment per distinct index, after a copy of 128 bytes per
// row.  With contiguous neighbours the ratio is about 1.3 and the copy would
// be pure overhead.  Measured on a 27-point stencil in reverse Cuthill-McKee
// order inside blocks of about 1950 rows: at a ratio of 3.7 (A) interleaving
// lost 16% and at 6.3 (A^T) it gained 36%, so it is taken from 4.5 up.
int gather_interleaved(const std::vector<long long>& ptr, const std::vector<int>& wid,
                       const std::vector<int>& col, const bc_opts& o) {
  if (o.multi_gather != BC_GATHER_AUTO) return o.multi_gather == BC_GATHER_INTERLEAVED;
  long long seg = 0, idx = 0;
  int c[64], g[64];
  const size_t stride = std::max<size_t>(1, ptr.size() / 4096);  // a sample of slices
  for (size_t sl = 0; sl < ptr.size(); sl += stride)
    for (int k = 0; k < wid[sl]; ++k) {
      for (int l = 0; l < 64; ++l) {
        c[l] = col[(size_t)(ptr[sl] + 64LL * k + l)];
        g[l] = c[l] >> 3;
      }
      std::sort(c, c + 64);
      std::sort(g, g + 64);
      idx += std::unique(c, c + 64) - c;
      seg += std::unique(g, g + 64) - g;
    }
  return 16 * seg >= 9 * idx;  // 8 seg / idx >= 4.5
}

bc_status validate_system(int s, int32_t n, const int32_t* rowptr, const int32_t* colidx,
                          const double* vals, int32_t K, const int32_t* part) {
  const bc_status st = validate_csr(n, rowptr, colidx, vals, "bc_setup");
  if (st != BC_OK) return st;
  if (K < 1 || K > n || !part) {
    bc_set_error("K must satisfy 1 <= K <= n and part must be non-null");
    return BC_ERR_INVALID;
  }
  std::vector<int> used(K, 0);
  for (int32_t r = 0; r < n; ++r) {
    if (part[r] < 0 || part[r] >= K) {
      bc_set_error("part[" + std::to_string(r) + "] outside [0, K)");
      return BC_ERR_INVALID;
    }
    used[part[r]] = 1;
  }
  for (int32_t k = 0; k < K; ++k)
    if (!used[k]) {
      bc_set_error("empty block " + std::to_string(k) + " in system " + std::to_string(s));
      return BC_ERR_INVALID;
    }
  return BC_OK;
}

bc_status validate_opts(const bc_opts& o) {
  if (o.precision != BC_FP64 && o.precision != BC_MIXED && o.precision != BC_MIXED_PROJ) {
    bc_set_error("unknown precision");
    return BC_ERR_INVALID;
  }
  if (o.projection < BC_PROJ_AUTO || o.projection > BC_PROJ_BAND_CHOL || !(o.inner_tol >= 0.0) ||
      o.inner_maxit < 1 || o.dense_max_m < 0 || o.stop_rule < 0 || o.stop_rule > 1 ||
      o.spmv_lanes < LANES_SELL || o.use_graph < 0 || o.use_graph > 1 ||
      o.multi_gather < BC_GATHER_AUTO || o.multi_gather > BC_GATHER_INTERLEAVED ||
      (o.spmv_lanes > 0 && (o.spmv_lanes & (o.spmv_lanes - 1))) || o.spmv_lanes > 64) {
    bc_set_error("invalid option value");
    return BC_ERR_INVALID;
  }
  return BC_OK;
}
