// Minimum weighted vertex cover of a bipartite graph by a minimum s-t cut
// (the solution of Sec. 5.3): s -> left vertex i with capacity w_left[i],
// left -> right along every edge with a capacity no cut can afford, right
// vertex j -> t with capacity w_right[j].  Max flow by Dinic's algorithm;
// the cover is the left vertices cut off from s plus the right vertices
// still reachable from s in the residual graph.  Host-only C++ (no HIP), so
// it can also be built on its own, for instance with the host sanitizers.
#pragma once

#include <algorithm>
#include <cstdint>
#include <limits>
#include <vector>

namespace shiro {
namespace mvc {

class MaxFlow {
 public:
  explicit MaxFlow(int n) : n_(n), first_(n + 1, 0) {}

  // Edges are added in two passes: count(), then build(), then add().
  void count(int u, int v) {
    ++deg_[u];
    ++deg_[v];
  }
  void reserve_counts() { deg_.assign(n_, 0); }
  void build() {
    for (int u = 0; u < n_; ++u) first_[u + 1] = first_[u] + deg_[u];
    to_.resize(first_[n_]);
    cap_.resize(first_[n_]);
    rev_.resize(first_[n_]);
    fill_ = std::vector<int64_t>(first_.begin(), first_.end() - 1);
  }
  void add(int u, int v, int64_t c) {
    const int64_t a = fill_[u]++, b = fill_[v]++;
    to_[a] = v;
    cap_[a] = c;
    rev_[a] = b;
    to_[b] = u;
    cap_[b] = 0;
    rev_[b] = a;
  }

  int64_t run(int s, int t) {
    int64_t flow = 0;
    level_.resize(n_);
    it_.resize(n_);
    std::vector<int> queue(n_);
    while (true) {
      // BFS levels from s over residual edges
      std::fill(level_.begin(), level_.end(), -1);
      int qh = 0, qt = 0;
      level_[s] = 0;
      queue[qt++] = s;
      while (qh < qt) {
        const int u = queue[qh++];
        for (int64_t e = first_[u]; e < first_[u + 1]; ++e)
          if (cap_[e] > 0 && level_[to_[e]] < 0) {
            level_[to_[e]] = level_[u] + 1;
            queue[qt++] = to_[e];
          }
      }
      if (level_[t] < 0) break;
      for (int u = 0; u < n_; ++u) it_[u] = first_[u];
      // blocking flow by iterative depth-first search along the levels
      while (true) {
        const int64_t f = augment(s, t);
        if (f == 0) break;
        flow += f;
      }
    }
    return flow;
  }

  // Vertices reachable from s in the residual graph (after run()).
  std::vector<char> reachable(int s) const {
    std::vector<char> seen(n_, 0);
    std::vector<int> stack{s};
    seen[s] = 1;
    while (!stack.empty()) {
      const int u = stack.back();
      stack.pop_back();
      for (int64_t e = first_[u]; e < first_[u + 1]; ++e)
        if (cap_[e] > 0 && !seen[to_[e]]) {
          seen[to_[e]] = 1;
          stack.push_back(to_[e]);
        }
    }
    return seen;
  }

 private:
  // One augmenting path in the level graph (iterative DFS with per-vertex
  // edge cursors); returns its bottleneck, 0 when none is left.
  int64_t augment(int s, int t) {
    path_.clear();
    int u = s;
    while (true) {
      if (u == t) {
        int64_t f = std::numeric_limits<int64_t>::max();
        for (int64_t e : path_) f = std::min(f, cap_[e]);
        for (int64_t e : path_) {
          cap_[e] -= f;
          cap_[rev_[e]] += f;
        }
        return f;
      }
      bool advanced = false;
      for (int64_t& e = it_[u]; e < first_[u + 1]; ++e) {
        const int v = to_[e];
        if (cap_[e] > 0 && level_[v] == level_[u] + 1) {
          path_.push_back(e);
          u = v;
          advanced = true;
          break;
        }
      }
      if (advanced) continue;
      // dead end: retreat and never try this vertex again in this phase
      level_[u] = -1;
      if (path_.empty()) return 0;
      const int64_t e = path_.back();
      path_.pop_back();
      u = to_[rev_[e]];
      ++it_[u];
    }
  }

  int n_;
  std::vector<int64_t> first_, fill_;
  std::vector<int> deg_;
  std::vector<int> to_;
  std::vector<int64_t> cap_, rev_;
  std::vector<int> level_;
  std::vector<int64_t> it_;
  std::vector<int64_t> path_;
};

// Text of what is wrong with the arguments of a cover problem, or nullptr
// when they are valid (sizes, endpoints in range, non-negative costs).
inline const char* arg_error(int64_t n_left, int64_t n_right, int64_t n_edges, const int32_t* left,
                             const int32_t* right, const int64_t* w_left, const int64_t* w_right,
                             const uint8_t* cover_left, const uint8_t* cover_right, const int64_t* weight) {
  if (n_left < 0 || n_right < 0 || n_edges < 0 || n_left + n_right > (1 << 30)) return "bad sizes";
  if (!weight || (n_left > 0 && !cover_left) || (n_right > 0 && !cover_right) ||
      (n_edges > 0 && (!left || !right)))
    return "NULL pointer";
  for (int64_t e = 0; e < n_edges; ++e)
    if (left[e] < 0 || left[e] >= n_left || right[e] < 0 || right[e] >= n_right)
      return "edge endpoint out of range";
  for (int64_t i = 0; w_left && i < n_left; ++i)
    if (w_left[i] < 0) return "negative weight";
  for (int64_t j = 0; w_right && j < n_right; ++j)
    if (w_right[j] < 0) return "negative weight";
  return nullptr;
}

// Writes cover_left[i], cover_right[j] (1 = in the cover) and returns the
// cover's cost.  w_left / w_right may be NULL (unit costs).  Arguments must
// pass arg_error.
inline int64_t min_weight_cover(int64_t n_left, int64_t n_right, int64_t n_edges, const int32_t* left,
                                const int32_t* right, const int64_t* w_left, const int64_t* w_right,
                                uint8_t* cover_left, uint8_t* cover_right) {
  const int L = (int)n_left, Rn = (int)n_right;
  const int s = L + Rn, t = s + 1;
  int64_t total = 1;
  for (int i = 0; i < L; ++i) total += w_left ? w_left[i] : 1;
  for (int j = 0; j < Rn; ++j) total += w_right ? w_right[j] : 1;
  MaxFlow g(L + Rn + 2);
  g.reserve_counts();
  for (int i = 0; i < L; ++i) g.count(s, i);
  for (int j = 0; j < Rn; ++j) g.count(L + j, t);
  for (int64_t e = 0; e < n_edges; ++e) g.count(left[e], L + right[e]);
  g.build();
  for (int i = 0; i < L; ++i) g.add(s, i, w_left ? w_left[i] : 1);
  for (int j = 0; j < Rn; ++j) g.add(L + j, t, w_right ? w_right[j] : 1);
  for (int64_t e = 0; e < n_edges; ++e) g.add(left[e], L + right[e], total);  // never cut
  g.run(s, t);
  const std::vector<char> S = g.reachable(s);
  int64_t w = 0;
  for (int i = 0; i < L; ++i) {
    cover_left[i] = !S[i];
    if (cover_left[i]) w += w_left ? w_left[i] : 1;
  }
  for (int j = 0; j < Rn; ++j) {
    cover_right[j] = S[L + j] ? 1 : 0;
    if (cover_right[j]) w += w_right ? w_right[j] : 1;
  }
  return w;
}

}  // namespace mvc
}  // namespace shiro
