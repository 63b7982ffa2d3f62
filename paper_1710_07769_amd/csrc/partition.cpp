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
  if (!part || K < 1 || K > n || passes < 0 || !check_graph(n, rowptr, col, wgt) ||
      (!wgt && rowptr[n] > 0)) {
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

// ---------------------------------------------------------------- multilevel
// Multilevel K-way partitioner on the same integer edge weights (coarsen by
// heavy-edge matching, grow K parts on the coarsest graph, project back and
// refine at every level).  The algorithm is specified in include/bc.h next to
// bc_partition_multilevel; every choice is deterministic.
namespace {

struct Level {
  int32_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<int64_t> wgt;
  std::vector<int64_t> vw;     // vertex weights
  std::vector<int32_t> cmap;   // fine vertex -> coarse vertex (set on the finer level)
};

// heavy-edge matching and contraction of L into C (sets L.cmap)
void coarsen(Level& L, Level& C, int64_t maxvw) {
  const int32_t n = L.n;
  std::vector<int32_t> match(n, -1);
  for (int32_t v = 0; v < n; ++v) {
    if (match[v] != -1) continue;
    int32_t best = -1;
    int64_t bw = 0;
    for (int64_t e = L.rowptr[v]; e < L.rowptr[v + 1]; ++e) {
      const int32_t u = L.col[e];
      if (match[u] != -1 || L.vw[v] + L.vw[u] > maxvw) continue;
      if (L.wgt[e] > bw || (L.wgt[e] == bw && best >= 0 && u < best)) {
        best = u;
        bw = L.wgt[e];
      }
    }
    match[v] = best >= 0 ? best : v;
    if (best >= 0) match[best] = v;
  }
  L.cmap.assign(n, -1);
  int32_t nc = 0;
  std::vector<int32_t> first;  // coarse vertex -> its lower fine vertex
  for (int32_t v = 0; v < n; ++v) {
    if (L.cmap[v] != -1) continue;
    L.cmap[v] = nc;
    L.cmap[match[v]] = nc;
    first.push_back(v);
    ++nc;
  }
  C.n = nc;
  C.vw.assign(nc, 0);
  C.rowptr.assign(1, 0);
  C.col.clear();
  C.wgt.clear();
  std::vector<int64_t> acc(nc, 0);
  std::vector<int32_t> seen;
  for (int32_t c = 0; c < nc; ++c) {
    const int32_t a = first[c], b = match[a];
    C.vw[c] = L.vw[a] + (b != a ? L.vw[b] : 0);
    seen.clear();
    const int32_t members[2] = {a, b};
    for (int t = 0; t < (b != a ? 2 : 1); ++t) {
      const int32_t x = members[t];
      for (int64_t e = L.rowptr[x]; e < L.rowptr[x + 1]; ++e) {
        const int32_t d = L.cmap[L.col[e]];
        if (d == c) continue;
        if (acc[d] == 0) seen.push_back(d);
        acc[d] += L.wgt[e];
      }
    }
    std::sort(seen.begin(), seen.end());
    for (int32_t d : seen) {
      C.col.push_back(d);
      C.wgt.push_back(acc[d]);
      acc[d] = 0;
    }
    C.rowptr.push_back((int64_t)C.col.size());
  }
}

// greedy growth of K parts by weight on L (the rule of bc_partition_greedy
// with vertex weights)
void grow(const Level& L, int32_t K, std::vector<int32_t>& p) {
  const int32_t n = L.n;
  p.assign(n, -1);
  std::vector<int64_t> conn(n, 0);
  std::vector<int32_t> touched;
  int32_t lowest = 0;
  int64_t rem_w = 0;
  for (int32_t v = 0; v < n; ++v) rem_w += L.vw[v];
  int32_t rem_v = n;
  using Item = std::pair<int64_t, int32_t>;
  auto cmp = [](const Item& a, const Item& b) {
    if (a.first != b.first) return a.first < b.first;
    return a.second > b.second;
  };
  for (int32_t k = 0; k < K - 1; ++k) {
    const int64_t target = (rem_w + (K - k) - 1) / (K - k);
    std::priority_queue<Item, std::vector<Item>, decltype(cmp)> heap(cmp);
    touched.clear();
    int64_t wk = 0;
    while (wk < target && rem_v > K - 1 - k) {
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
      wk += L.vw[v];
      --rem_v;
      for (int64_t e = L.rowptr[v]; e < L.rowptr[v + 1]; ++e) {
        const int32_t u = L.col[e];
        if (p[u] == -1) {
          if (conn[u] == 0) touched.push_back(u);
          conn[u] += L.wgt[e];
          heap.push(Item(conn[u], u));
        }
      }
    }
    rem_w -= wk;
    for (int32_t u : touched) conn[u] = 0;
  }
  for (int32_t v = 0; v < n; ++v)
    if (p[v] == -1) p[v] = K - 1;
}

// Fiduccia-Mattheyses refinement with vertex weights (the rule is stated in
// include/bc.h under bc_partition_multilevel, step 3).
constexpr int FM_STALL = 64;

struct FmState {
  const Level& L;
  const std::vector<int32_t>& p;
  std::vector<int64_t> to;      // conn(v, q), cleared after use
  std::vector<int32_t> seen;    // parts v touches, ascending after conn()
  FmState(const Level& L_, const std::vector<int32_t>& p_, int32_t K) : L(L_), p(p_), to(K, 0) {}
  // fills to[]/seen for v; returns whether v touches another part and sets key
  bool conn(int32_t v, int64_t& key) {
    seen.clear();
    for (int64_t e = L.rowptr[v]; e < L.rowptr[v + 1]; ++e) {
      const int32_t q = p[L.col[e]];
      if (to[q] == 0) seen.push_back(q);
      to[q] += L.wgt[e];
    }
    std::sort(seen.begin(), seen.end());
    const int32_t a = p[v];
    bool any = false;
    for (int32_t q : seen) {
      if (q == a) continue;
      const int64_t g = to[q] - to[a];
      if (!any || g > key) key = g;
      any = true;
    }
    return any;
  }
  void clear() {
    for (int32_t q : seen) to[q] = 0;
  }
};

void refine(const Level& L, int32_t K, int64_t wmax, int32_t passes, std::vector<int32_t>& p) {
  const int32_t n = L.n;
  std::vector<int64_t> W(K, 0);
  for (int32_t v = 0; v < n; ++v) W[p[v]] += L.vw[v];
  FmState st(L, p, K);
  // (key, vertex): larger key first, then lower vertex
  using Item = std::pair<int64_t, int32_t>;
  auto cmp = [](const Item& x, const Item& y) {
    if (x.first != y.first) return x.first < y.first;
    return x.second > y.second;
  };
  std::vector<uint8_t> locked(n);
  std::vector<std::pair<int32_t, int32_t>> log;  // (vertex, part it left)
  for (int32_t pass = 0; pass < passes; ++pass) {
    std::fill(locked.begin(), locked.end(), 0);
    std::vector<Item> init;
    for (int32_t v = 0; v < n; ++v) {
      int64_t key = 0;
      if (st.conn(v, key)) init.emplace_back(key, v);
      st.clear();
    }
    std::priority_queue<Item, std::vector<Item>, decltype(cmp)> heap(cmp, std::move(init));
    log.clear();
    int64_t cum = 0, best = 0;
    size_t best_len = 0;
    int stall = 0;
    while (!heap.empty() && stall < FM_STALL) {
      const Item it = heap.top();
      heap.pop();
      const int32_t v = it.second;
      if (locked[v]) continue;
      int64_t key = 0;
      const bool any = st.conn(v, key);
      const int32_t a = p[v];
      int32_t q_best = -1;
      int64_t g_best = 0;
      if (any && key == it.first && W[a] > L.vw[v]) {
        for (int32_t q : st.seen) {
          if (q == a || W[q] + L.vw[v] > wmax) continue;
          const int64_t g = st.to[q] - st.to[a];
          if (q_best < 0 || g > g_best) {
            q_best = q;
            g_best = g;
          }
        }
      }
      st.clear();
      if (q_best < 0) continue;
      p[v] = q_best;
      W[a] -= L.vw[v];
      W[q_best] += L.vw[v];
      locked[v] = 1;
      log.emplace_back(v, a);
      cum += g_best;
      if (cum > best) {
        best = cum;
        best_len = log.size();
        stall = 0;
      } else {
        ++stall;
      }
      for (int64_t e = L.rowptr[v]; e < L.rowptr[v + 1]; ++e) {
        const int32_t u = L.col[e];
        if (locked[u]) continue;
        int64_t ku = 0;
        if (st.conn(u, ku)) heap.push(Item(ku, u));
        st.clear();
      }
    }
    for (size_t i = log.size(); i > best_len; --i) {
      const int32_t v = log[i - 1].first, a = log[i - 1].second;
      W[p[v]] -= L.vw[v];
      W[a] += L.vw[v];
      p[v] = a;
    }
    if (best == 0) break;
  }
}

}  // namespace

extern "C" bc_status bc_partition_multilevel(int32_t n, const int64_t* rowptr, const int32_t* col,
                                             const int64_t* wgt, int32_t K, int32_t passes,
                                             int32_t* part) {
  if (!part || K < 1 || K > n || passes < 0 || !check_graph(n, rowptr, col, wgt) ||
      (!wgt && rowptr[n] > 0)) {
    bc_set_error("bc_partition_multilevel: invalid graph, K or output");
    return BC_ERR_INVALID;
  }
  const int64_t wmax = std::max<int64_t>((int64_t)std::floor(1.1 * n / K), ((int64_t)n + K - 1) / K);
  const int64_t coarse_to = std::max<int64_t>(30LL * K, K);
  const int64_t maxvw = std::max<int64_t>(1, ((int64_t)n + 20LL * K - 1) / (20LL * K));
  std::vector<Level> lv(1);
  lv[0].n = n;
  lv[0].rowptr.assign(rowptr, rowptr + n + 1);
  lv[0].col.assign(col, col + rowptr[n]);
  lv[0].wgt.assign(wgt, wgt + rowptr[n]);
  lv[0].vw.assign(n, 1);
  while ((int64_t)lv.back().n > coarse_to && lv.size() < 30) {
    Level C;
    coarsen(lv.back(), C, maxvw);
    if ((double)C.n > 0.9 * (double)lv.back().n) {
      lv.back().cmap.clear();
      break;
    }
    lv.push_back(std::move(C));
  }
  std::vector<int32_t> p;
  grow(lv.back(), K, p);
  refine(lv.back(), K, wmax, passes, p);
  for (int l = (int)lv.size() - 2; l >= 0; --l) {
    std::vector<int32_t> fine(lv[l].n);
    for (int32_t v = 0; v < lv[l].n; ++v) fine[v] = p[lv[l].cmap[v]];
    p.swap(fine);
    refine(lv[l], K, wmax, passes, p);
  }
  std::copy(p.begin(), p.end(), part);
  return BC_OK;
}
