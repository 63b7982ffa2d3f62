// Host-only parts of the library: argument validation and the sliced-ELL
// layout of the sparse products.  Nothing here touches HIP, so these sources
// also build on their own with the host sanitizers (tests/native/).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bc.h"

void bc_set_error(const std::string& msg);

// Elements per reduction tile of the vector kernels.  A tile never straddles
// two systems of a batch, so per-system sums are sums over a tile range.
constexpr int TILE = 1024;
// Sliced-ELL slices of 64 rows per tile.
constexpr int SELL_SLICES = TILE / 64;
// `lanes` value that selects the sliced-ELL kernels
constexpr int LANES_SELL = -1;

// CSR checks of a matrix argument (n >= 1, rowptr from 0 and non-decreasing,
// columns in [0, n) strictly ascending per row, finite values).
bc_status validate_csr(int32_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                       const char* who);
// validate_csr plus 1 <= K <= n and a partition with every block in [0, K) used.
bc_status validate_system(int s, int32_t n, const int32_t* rowptr, const int32_t* colidx,
                          const double* vals, int32_t K, const int32_t* part);
// Range checks of every option field.
bc_status validate_opts(const bc_opts& o);

// Reverse Cuthill-McKee order of an m-vertex graph (order.cpp).
int bc_rcm_order(int m, const int* xadj, const int* adj, int* order);

// Lanes per row of the CSR sparse products for an average row length.
int choose_lanes(int64_t nnz, int64_t rows);

// Sliced-ELL copy of the CSR matrix (rp, ci, v) over the tiles: the rows of
// tile t are cut into SELL_SLICES slices of 64 rows (slice t * SELL_SLICES + j
// starts at row tile_start[t] + 64 j; slices past the tile's end have width
// 0); entry k of lane l of slice s is at ptr[s] + 64 k + l, in the row's
// stored order; padding entries repeat the row's last column (or the tile's
// first index for absent rows) with value 0.  Without `force` nothing is
// built (false) when padding would add more than a quarter to the entries.
bool build_sell(const std::vector<int>& rp, const std::vector<int>& ci, const std::vector<double>& v,
                const std::vector<int>& tile_start, bool force, std::vector<long long>& ptr,
                std::vector<int>& wid, std::vector<int>& col, std::vector<double>& val);

// Whether the multi-vector products should gather an interleaved copy of
// their input (1) or the vectors separately (0), from a sample of slices.
int gather_interleaved(const std::vector<long long>& ptr, const std::vector<int>& wid,
                       const std::vector<int>& col, const bc_opts& o);
