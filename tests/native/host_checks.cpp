// Checks of the library's host-only code, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py: the greedy and
// multilevel partitioners and the cutsize (partition.cpp), the reverse
// Cuthill-McKee order (order.cpp), and the argument validation and
// sliced-ELL layout (host.cpp).  Seeded random inputs of many shapes, plus
// the invalid arguments each entry point must refuse.  Prints one line per
// group and exits non-zero at the first failed check.
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

#include "../../include/bc.h"
#include "../../paper_1710_07769_amd/csrc/host.h"

namespace {

int g_checks = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    ++g_checks;                                                            \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      std::exit(1);                                                        \
    }                                                                      \
  } while (0)

// splitmix64
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
  }
  int below(int n) { return (int)(next() % (uint64_t)n); }
  double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct Graph {
  int32_t n = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<int64_t> wgt;
  std::vector<double> cost;
};

// symmetric graph without loops: each pair joined with probability p
Graph random_graph(int32_t n, double p, Rng& r) {
  std::vector<std::vector<std::pair<int32_t, int64_t>>> adj(n);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t j = i + 1; j < n; ++j)
      if (r.unit() < p) {
        const int64_t w = 1 + r.below(9);
        adj[i].push_back({j, w});
        adj[j].push_back({i, w});
      }
  Graph g;
  g.n = n;
  g.rowptr.assign(1, 0);
  for (int32_t i = 0; i < n; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    for (auto& e : adj[i]) {
      g.col.push_back(e.first);
      g.wgt.push_back(e.second);
      g.cost.push_back(0.125 * (double)e.second);
    }
    g.rowptr.push_back((int64_t)g.col.size());
  }
  return g;
}

int64_t int_cut(const Graph& g, const std::vector<int32_t>& part) {
  int64_t c = 0;
  for (int32_t v = 0; v < g.n; ++v)
    for (int64_t e = g.rowptr[v]; e < g.rowptr[v + 1]; ++e)
      if (v < g.col[e] && part[v] != part[g.col[e]]) c += g.wgt[e];
  return c;
}

void check_partition(const Graph& g, int32_t K, const std::vector<int32_t>& part, bool capped) {
  std::vector<int64_t> W(K, 0);
  for (int32_t v = 0; v < g.n; ++v) {
    CHECK(part[v] >= 0 && part[v] < K);
    W[part[v]]++;
  }
  const int64_t wmax = std::max<int64_t>((int64_t)std::floor(1.1 * g.n / K), ((int64_t)g.n + K - 1) / K);
  for (int32_t k = 0; k < K; ++k) {
    CHECK(W[k] >= 1);
    if (capped) CHECK(W[k] <= wmax);
  }
  double cs = -1.0;
  int64_t ic = -1;
  CHECK(bc_partition_cut(g.n, g.rowptr.data(), g.col.data(), g.cost.data(), g.wgt.data(),
                         part.data(), &cs, &ic) == BC_OK);
  CHECK(ic == int_cut(g, part));
  CHECK(std::fabs(cs - 0.125 * (double)ic) <= 1e-9 * (1.0 + cs));
}

void partitioners() {
  Rng r(7);
  const int32_t sizes[] = {1, 2, 3, 5, 17, 64, 65, 200, 700};
  for (int32_t n : sizes)
    for (double p : {0.0, 0.05, 0.3})
      for (int32_t K : {1, 2, 3, 7, 61, n}) {
        if (K > n) continue;
        const Graph g = random_graph(n, p, r);
        std::vector<int32_t> part(n, -1);
        for (int32_t passes : {0, 1, 3}) {
          CHECK(bc_partition_greedy(n, g.rowptr.data(), g.col.data(), g.wgt.data(), K, passes,
                                    part.data()) == BC_OK);
          check_partition(g, K, part, true);
          CHECK(bc_partition_multilevel(n, g.rowptr.data(), g.col.data(), g.wgt.data(), K,
                                        passes, part.data()) == BC_OK);
          check_partition(g, K, part, false);
        }
      }
  // a graph large enough for several coarsening levels
  {
    const Graph g = random_graph(3000, 0.004, r);
    std::vector<int32_t> part(g.n);
    CHECK(bc_partition_multilevel(g.n, g.rowptr.data(), g.col.data(), g.wgt.data(), 8, 4,
                                  part.data()) == BC_OK);
    check_partition(g, 8, part, false);
  }
  // invalid arguments
  Graph g = random_graph(20, 0.3, r);
  std::vector<int32_t> part(g.n);
  auto greedy = [&](const Graph& h, int32_t K, int32_t* out) {
    return bc_partition_greedy(h.n, h.rowptr.data(), h.col.data(), h.wgt.data(), K, 1, out);
  };
  auto multi = [&](const Graph& h, int32_t K, int32_t* out) {
    return bc_partition_multilevel(h.n, h.rowptr.data(), h.col.data(), h.wgt.data(), K, 1, out);
  };
  for (int32_t K : {0, -1, g.n + 1}) {
    CHECK(greedy(g, K, part.data()) == BC_ERR_INVALID);
    CHECK(multi(g, K, part.data()) == BC_ERR_INVALID);
  }
  CHECK(greedy(g, 2, nullptr) == BC_ERR_INVALID);
  CHECK(multi(g, 2, nullptr) == BC_ERR_INVALID);
  CHECK(bc_partition_multilevel(g.n, g.rowptr.data(), g.col.data(), g.wgt.data(), 2, -1,
                                part.data()) == BC_ERR_INVALID);
  {
    Graph h = g;
    h.col[0] = h.n;  // out of range
    CHECK(greedy(h, 2, part.data()) == BC_ERR_INVALID);
    CHECK(multi(h, 2, part.data()) == BC_ERR_INVALID);
    h = g;
    h.col[0] = 0;  // a loop on vertex 0
    CHECK(greedy(h, 2, part.data()) == BC_ERR_INVALID);
    h = g;
    h.wgt[0] = 0;
    CHECK(greedy(h, 2, part.data()) == BC_ERR_INVALID);
    CHECK(multi(h, 2, part.data()) == BC_ERR_INVALID);
    h = g;
    h.rowptr[3] = h.rowptr[4] + 1;  // decreasing
    CHECK(greedy(h, 2, part.data()) == BC_ERR_INVALID);
  }
  double cs;
  int64_t ic;
  CHECK(bc_partition_cut(g.n, g.rowptr.data(), g.col.data(), g.cost.data(), g.wgt.data(), nullptr,
                         &cs, &ic) == BC_ERR_INVALID);
  std::printf("partitioners: ok\n");
}

void rcm() {
  Rng r(11);
  for (int m : {1, 2, 3, 10, 64, 300}) {
    for (double p : {0.0, 0.02, 0.2}) {
      const Graph g = random_graph(m, p, r);
      std::vector<int> xadj(g.rowptr.begin(), g.rowptr.end());
      std::vector<int> adj(g.col.begin(), g.col.end());
      std::vector<int> order(m, -1);
      const int bw = bc_rcm_order(m, xadj.data(), adj.data(), order.data());
      std::vector<int> pos(m, -1);
      for (int i = 0; i < m; ++i) {
        CHECK(order[i] >= 0 && order[i] < m);
        CHECK(pos[order[i]] == -1);
        pos[order[i]] = i;
      }
      int want = 0;
      for (int v = 0; v < m; ++v)
        for (int e = xadj[v]; e < xadj[v + 1]; ++e) want = std::max(want, std::abs(pos[v] - pos[adj[e]]));
      CHECK(bw == want);
    }
  }
  // a path in scrambled numbering gets half-bandwidth 1
  {
    const int m = 50;
    std::vector<int> label(m);
    for (int i = 0; i < m; ++i) label[i] = (i * 17) % m;
    std::vector<std::vector<int>> nb(m);
    for (int i = 0; i + 1 < m; ++i) {
      nb[label[i]].push_back(label[i + 1]);
      nb[label[i + 1]].push_back(label[i]);
    }
    std::vector<int> xadj(1, 0), adj;
    for (int v = 0; v < m; ++v) {
      std::sort(nb[v].begin(), nb[v].end());
      adj.insert(adj.end(), nb[v].begin(), nb[v].end());
      xadj.push_back((int)adj.size());
    }
    std::vector<int> order(m);
    CHECK(bc_rcm_order(m, xadj.data(), adj.data(), order.data()) == 1);
  }
  std::printf("rcm: ok\n");
}

struct Csr {
  int32_t n = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
};

Csr random_csr(int32_t n, int maxlen, Rng& r) {
  Csr a;
  a.n = n;
  a.rowptr.assign(1, 0);
  std::vector<int32_t> cols;
  for (int32_t i = 0; i < n; ++i) {
    cols.clear();
    const int len = r.below(maxlen + 1);
    for (int k = 0; k < len; ++k) cols.push_back(r.below(n));
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int32_t c : cols) {
      a.col.push_back(c);
      a.val.push_back(r.unit() - 0.5);
    }
    a.rowptr.push_back((int32_t)a.col.size());
  }
  return a;
}

void validation() {
  Rng r(5);
  const Csr a = random_csr(100, 6, r);
  auto v = [](const Csr& m) {
    return validate_csr(m.n, m.rowptr.data(), m.col.data(), m.val.data(), "check");
  };
  CHECK(v(a) == BC_OK);
  CHECK(validate_csr(0, a.rowptr.data(), a.col.data(), a.val.data(), "check") == BC_ERR_INVALID);
  CHECK(validate_csr(a.n, nullptr, a.col.data(), a.val.data(), "check") == BC_ERR_INVALID);
  CHECK(validate_csr(a.n, a.rowptr.data(), nullptr, a.val.data(), "check") == BC_ERR_INVALID);
  CHECK(validate_csr(a.n, a.rowptr.data(), a.col.data(), nullptr, "check") == BC_ERR_INVALID);
  int row = 0;
  while (a.rowptr[row + 1] - a.rowptr[row] < 2) ++row;
  {
    Csr b = a;
    b.rowptr[0] = 1;
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    b.rowptr[row + 1] = b.rowptr[row] - 1;
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    b.col[b.rowptr[row]] = -1;
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    b.col[b.rowptr[row]] = b.n;
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    std::swap(b.col[b.rowptr[row]], b.col[b.rowptr[row] + 1]);  // descending
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    b.col[b.rowptr[row] + 1] = b.col[b.rowptr[row]];  // repeated column
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    b.val[3] = std::numeric_limits<double>::quiet_NaN();
    CHECK(v(b) == BC_ERR_INVALID);
    b = a;
    b.val[3] = std::numeric_limits<double>::infinity();
    CHECK(v(b) == BC_ERR_INVALID);
  }
  // partitions
  std::vector<int32_t> part(a.n);
  for (int32_t i = 0; i < a.n; ++i) part[i] = i % 4;
  auto sys = [&](int32_t K, const int32_t* p) {
    return validate_system(0, a.n, a.rowptr.data(), a.col.data(), a.val.data(), K, p);
  };
  CHECK(sys(4, part.data()) == BC_OK);
  CHECK(sys(0, part.data()) == BC_ERR_INVALID);
  CHECK(sys(a.n + 1, part.data()) == BC_ERR_INVALID);
  CHECK(sys(4, nullptr) == BC_ERR_INVALID);
  CHECK(sys(5, part.data()) == BC_ERR_INVALID);  // block 4 empty
  part[7] = 4;
  CHECK(sys(4, part.data()) == BC_ERR_INVALID);  // outside [0, K)
  part[7] = -1;
  CHECK(sys(4, part.data()) == BC_ERR_INVALID);
  // options
  bc_opts o;
  bc_opts_default(&o);
  CHECK(validate_opts(o) == BC_OK);
  auto bad = [&](void (*f)(bc_opts&)) {
    bc_opts q;
    bc_opts_default(&q);
    f(q);
    return validate_opts(q) == BC_ERR_INVALID;
  };
  CHECK(bad([](bc_opts& q) { q.precision = 7; }));
  CHECK(bad([](bc_opts& q) { q.projection = BC_PROJ_BAND_CHOL + 1; }));
  CHECK(bad([](bc_opts& q) { q.projection = BC_PROJ_AUTO - 1; }));
  CHECK(bad([](bc_opts& q) { q.inner_tol = -1.0; }));
  CHECK(bad([](bc_opts& q) { q.inner_tol = std::numeric_limits<double>::quiet_NaN(); }));
  CHECK(bad([](bc_opts& q) { q.inner_maxit = 0; }));
  CHECK(bad([](bc_opts& q) { q.dense_max_m = -1; }));
  CHECK(bad([](bc_opts& q) { q.stop_rule = 2; }));
  CHECK(bad([](bc_opts& q) { q.spmv_lanes = 3; }));
  CHECK(bad([](bc_opts& q) { q.spmv_lanes = 128; }));
  CHECK(bad([](bc_opts& q) { q.spmv_lanes = -2; }));
  CHECK(bad([](bc_opts& q) { q.use_graph = 2; }));
  CHECK(bad([](bc_opts& q) { q.multi_gather = BC_GATHER_INTERLEAVED + 1; }));
  for (int lanes : {-1, 0, 1, 2, 4, 8, 16, 32, 64}) {
    bc_opts q;
    bc_opts_default(&q);
    q.spmv_lanes = lanes;
    CHECK(validate_opts(q) == BC_OK);
  }
  std::printf("validation: ok\n");
}

void sell_layout() {
  Rng r(3);
  for (int32_t n : {1, 63, 64, 65, 1024, 2500}) {
    for (int maxlen : {0, 3, 12}) {
      const Csr a = random_csr(n, maxlen, r);
      // tiles of TILE rows with a ragged last tile
      std::vector<int> ts;
      for (int32_t t = 0; t < n; t += TILE) ts.push_back(t);
      ts.push_back(n);
      const std::vector<int> rp(a.rowptr.begin(), a.rowptr.end());
      const std::vector<int> ci(a.col.begin(), a.col.end());
      std::vector<long long> ptr;
      std::vector<int> wid, col;
      std::vector<double> val;
      CHECK(build_sell(rp, ci, a.val, ts, true, ptr, wid, col, val));
      const int ntiles = (int)ts.size() - 1;
      CHECK(ptr.size() == (size_t)ntiles * SELL_SLICES && wid.size() == ptr.size());
      for (int t = 0; t < ntiles; ++t)
        for (int j = 0; j < SELL_SLICES; ++j) {
          const size_t s = (size_t)t * SELL_SLICES + j;
          for (int l = 0; l < 64; ++l) {
            const int i = ts[t] + 64 * j + l;
            const bool present = i < ts[t + 1];
            const int len = present ? rp[i + 1] - rp[i] : 0;
            CHECK(len <= wid[s]);
            for (int k = 0; k < wid[s]; ++k) {
              const size_t q = (size_t)(ptr[s] + 64LL * k + l);
              CHECK(q < col.size());
              if (k < len) {
                CHECK(col[q] == ci[rp[i] + k] && val[q] == a.val[rp[i] + k]);
              } else {
                CHECK(val[q] == 0.0 && col[q] >= 0 && col[q] < n);
              }
            }
          }
        }
      bc_opts o;
      bc_opts_default(&o);
      const int il = gather_interleaved(ptr, wid, col, o);
      CHECK(il == 0 || il == 1);
      o.multi_gather = BC_GATHER_SEPARATE;
      CHECK(gather_interleaved(ptr, wid, col, o) == 0);
      o.multi_gather = BC_GATHER_INTERLEAVED;
      CHECK(gather_interleaved(ptr, wid, col, o) == 1);
      CHECK(choose_lanes((int64_t)a.col.size(), n) >= 1 && choose_lanes((int64_t)a.col.size(), n) <= 64);
    }
  }
  // one long row among short ones: the padding is refused without force
  {
    Csr a;
    a.n = 128;
    a.rowptr.assign(1, 0);
    for (int32_t i = 0; i < a.n; ++i) {
      const int len = i == 5 ? 100 : 1;
      for (int k = 0; k < len; ++k) {
        a.col.push_back(len == 1 ? i : k);
        a.val.push_back(1.0);
      }
      a.rowptr.push_back((int32_t)a.col.size());
    }
    const std::vector<int> rp(a.rowptr.begin(), a.rowptr.end());
    const std::vector<int> ci(a.col.begin(), a.col.end());
    std::vector<long long> ptr;
    std::vector<int> wid, col;
    std::vector<double> val;
    CHECK(!build_sell(rp, ci, a.val, {0, a.n}, false, ptr, wid, col, val));
  }
  std::printf("sell layout: ok\n");
}

}  // namespace

int main() {
  partitioners();
  rcm();
  validation();
  sell_layout();
  std::printf("all %d checks passed\n", g_checks);
  return 0;
}
