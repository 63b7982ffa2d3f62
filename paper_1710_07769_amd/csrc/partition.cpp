// Deterministic greedy K-way partitioner on integer edge weights, used in
// place of METIS to partition the row inner-product graph (Sections 2.3 and
// 3.1 of the paper: k-way, 10% imbalance, unit vertex weights), and the
// cutsize of eq. (partcut).  The algorithm is specified in include/bc.h.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bc.h"

void bc_set_error(const std::string& msg);

namespace {

bool check_graph(int32_t n, const int64_t* rowptr, const int32_t* col, const int64_t* wgt) {
  if (n < 1 || !rowptr || (!col && rowptr[n] > 0)) return false;
  if (rowptr[0] != 0) return false;
  for (int32_t v = 0; v < n; ++v) {
    if (rowptr[v + 1] < rowptr[v]) return false;
    for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n || col[e] == v) return false;
      if (wgt && wgt[e] < 1) return false;
    }
  }
  return true;
}

}  // namespace

extern "C" bc_status bc_partition_greedy(int32_t n, const int64_t* rowptr, const int32_t* col,
                                         const int64_t* wgt, int32_t K, int32_t passes,
                                         int32_t* part) {
  if (!part || K < 1 || K > n || passes < 0 || !check_graph(n, rowptr, col, wgt) || !wgt) {
    bc_set_error("bc_partition_greedy: invalid graph, K or output");
    return BC_ERR_INVALID;
  }
  std::vector<int32_t> p(n, -1);
  std::vector<int64_t> conn(n, 0);
  std::vector<int32_t> touched;
  int32_t lowest = 0;
  int64_t remaining = n;
  // max-heap on (connection, -vertex): largest weight first, ties to the lower index
  using Item = std::pair<int64_t, int32_t>;
  auto cmp = [](const Item& a, const Item& b) {
    if (a.first != b.first) return a.first < b.first;
    return a.second > b.second;
  };
  for (int32_t k = 0; k < K - 1; ++k) {
    const int64_t target = (remaining + (K - k) - 1) / (K - k);
    std::priority_queue<Item, std::vector<Item>, decltype(cmp)> heap(cmp);
    touched.clear();
    for (int64_t c = 0; c < target; ++c) {
      int32_t v = -1;
      while (!heap.empty()) {
        const Item it = heap.top();
        heap.pop();
        if (p[it.second] == -1 && conn[it.second] == it.first) {
          v = it.second;
          break;
        }
      }
      if (v == -1) {
        while (p[lowest] != -1) ++lowest;
        v = lowest;
      }
      p[v] = k;
      --remaining;
      for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int32_t u = col[e];
        if (p[u] == -1) {
          if (conn[u] == 0) touched.push_back(u);
          conn[u] += wgt[e];
          heap.push(Item(conn[u], u));
        }
      }
    }
    for (int32_t u : touched) conn[u] = 0;
  }
  for (int32_t v = 0; v < n; ++v)
    if (p[v] == -1) p[v] = K - 1;

  const int64_t wmax = std::max<int64_t>((int64_t)std::floor(1.1 * n / K), ((int64_t)n + K - 1) / K);
  std::vector<int64_t> W(K, 0);
  for (int32_t v = 0; v < n; ++v) W[p[v]]++;
  std::vector<int64_t> to(K, 0);
  std::vector<int32_t> seen;
  for (int32_t pass = 0; pass < passes; ++pass) {
    for (int32_t v = 0; v < n; ++v) {
      const int32_t a = p[v];
      if (W[a] <= 1) continue;
      seen.clear();
      for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        const int32_t q = p[col[e]];
        if (to[q] == 0) seen.push_back(q);
        to[q] += wgt[e];
      }
      std::sort(seen.begin(), seen.end());
      const int64_t inside = to[a];
      int32_t best = -1;
      int64_t best_gain = 0;
      for (int32_t q : seen) {
        if (q == a || W[q] + 1 > wmax) continue;
        const int64_t gain = to[q] - inside;
        if (gain > best_gain) {
          best = q;
          best_gain = gain;
        }
      }
      for (int32_t q : seen) to[q] = 0;
      if (best >= 0) {
        p[v] = best;
        W[a]--;
        W[best]++;
      }
    }
  }
  std::copy(p.begin(), p.end(), part);
  return BC_OK;
}

extern "C" bc_status bc_partition_cut(int32_t n, const int64_t* rowptr, const int32_t* col,
                                      const double* cost, const int64_t* wgt, const int32_t* part,
                                      double* cutsize, int64_t* int_cut) {
  if (!part || !check_graph(n, rowptr, col, nullptr)) {
    bc_set_error("bc_partition_cut: invalid graph or partition");
    return BC_ERR_INVALID;
  }
  double cs = 0.0;
  int64_t ic = 0;
  for (int32_t v = 0; v < n; ++v)
    for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
      const int32_t u = col[e];
      if (v < u && part[v] != part[u]) {
        if (cost) cs += cost[e];
        if (wgt) ic += wgt[e];
      }
    }
  if (cutsize) *cutsize = cs;
  if (int_cut) *int_cut = ic;
  return BC_OK;
}
