// Reverse Cuthill-McKee ordering of the rows of one block (host side).
//
// The graph has one vertex per row of the block and an edge wherever two rows
// share a column, i.e. the pattern of A_i A_i^T.  Reordering the rows inside a
// block leaves its projection unchanged (Section 2.2), and a small bandwidth
// of A_i A_i^T lets the projections use a banded Cholesky factor.
//
// Cuthill-McKee: per connected component, start from a pseudo-peripheral
// vertex (repeated breadth-first search from the lowest-degree vertex of the
// last level while the eccentricity grows), then number vertices in
// breadth-first order, visiting the neighbours of each vertex by increasing
// degree (ties: lower index).  The reverse of that numbering is returned.
// Everything is deterministic.
#include <algorithm>
#include <cstdlib>
#include <vector>

namespace {

struct Bfs {
  std::vector<int> level;
  std::vector<int> touched;
  explicit Bfs(int m) : level(m, -1) {}
  // Breadth-first levels from s over unvisited vertices; returns the depth and
  // the lowest-degree vertex (ties: lower index) of the deepest level.
  int run(int s, const int* xadj, const int* adj, const std::vector<char>& vis,
          const std::vector<int>& deg, int* far) {
    for (int v : touched) level[v] = -1;
    touched.clear();
    level[s] = 0;
    touched.push_back(s);
    size_t head = 0;
    int depth = 0;
    while (head < touched.size()) {
      const int v = touched[head++];
      depth = std::max(depth, level[v]);
      for (int e = xadj[v]; e < xadj[v + 1]; ++e) {
        const int w = adj[e];
        if (vis[w] || level[w] >= 0) continue;
        level[w] = level[v] + 1;
        touched.push_back(w);
      }
    }
    int best = -1;
    for (int v : touched)
      if (level[v] == depth && (best < 0 || deg[v] < deg[best] || (deg[v] == deg[best] && v < best)))
        best = v;
    *far = best;
    return depth;
  }
};

}  // namespace

// order[new] = old.  Returns the half-bandwidth max |pos(u) - pos(v)| over the
// edges under the new order (0 for a graph without edges).
int bc_rcm_order(int m, const int* xadj, const int* adj, int* order) {
  std::vector<int> deg(m);
  for (int v = 0; v < m; ++v) deg[v] = xadj[v + 1] - xadj[v];
  std::vector<int> seeds(m);
  for (int v = 0; v < m; ++v) seeds[v] = v;
  std::stable_sort(seeds.begin(), seeds.end(), [&](int a, int b) { return deg[a] < deg[b]; });
  std::vector<char> vis(m, 0);
  std::vector<int> out;
  out.reserve(m);
  Bfs bfs(m);
  std::vector<int> nb;
  size_t sp = 0;
  while ((int)out.size() < m) {
    while (vis[seeds[sp]]) ++sp;
    int start = seeds[sp];
    int far = start;
    int ecc = bfs.run(start, xadj, adj, vis, deg, &far);
    for (int round = 0; round < 8 && far != start; ++round) {
      int far2 = far;
      const int e2 = bfs.run(far, xadj, adj, vis, deg, &far2);
      if (e2 <= ecc) break;
      start = far;
      ecc = e2;
      far = far2;
    }
    // Cuthill-McKee numbering of this component
    size_t head = out.size();
    vis[start] = 1;
    out.push_back(start);
    while (head < out.size()) {
      const int v = out[head++];
      nb.clear();
      for (int e = xadj[v]; e < xadj[v + 1]; ++e)
        if (!vis[adj[e]]) {
          vis[adj[e]] = 1;
          nb.push_back(adj[e]);
        }
      std::sort(nb.begin(), nb.end(), [&](int a, int b) {
        return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
      });
      out.insert(out.end(), nb.begin(), nb.end());
    }
  }
  std::vector<int> pos(m);
  for (int k = 0; k < m; ++k) {
    order[k] = out[m - 1 - k];
    pos[order[k]] = k;
  }
  int bw = 0;
  for (int v = 0; v < m; ++v)
    for (int e = xadj[v]; e < xadj[v + 1]; ++e) bw = std::max(bw, std::abs(pos[v] - pos[adj[e]]));
  return bw;
}
