// Joint row-column strategy (Sec. 5.2 problem; Sec. 5.3 solution): for each
// off-diagonal block A^(p,q), choose which rows of C (row-based) and which
// rows of B (column-based) to communicate so that every nonzero is covered
// at minimum total cost.  This is a minimum weighted vertex cover of the
// bipartite graph (rows of the block | columns of the block, one edge per
// nonzero), found as a minimum s-t cut: s -> row i with capacity w_row[i],
// row -> column with a capacity no cut can afford, column j -> t with
// capacity w_col[j].  Max flow by Dinic's algorithm (which the paper uses;
// on unit costs it runs like Hopcroft-Karp); the cover is the rows cut off
// from s plus the columns still reachable from s in the residual graph.
//
// Host code: the paper runs this offline on the CPU, once per sparsity
// pattern, with the blocks solved independently in parallel.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "mvc.hpp"
#include "plan.hpp"

namespace shiro {

int solve_mvc(int64_t n_left, int64_t n_right, int64_t n_edges, const int32_t* left,
              const int32_t* right, const int64_t* w_left, const int64_t* w_right,
              uint8_t* cover_left, uint8_t* cover_right, int64_t* weight) {
  *weight = mvc::min_weight_cover(n_left, n_right, n_edges, left, right, w_left, w_right, cover_left,
                                  cover_right);
  return SHIRO_OK;
}

// Per-panel plan: every off-diagonal block solved independently (threads
// take blocks from a shared counter).  A nonzero whose row is in its
// block's cover is computed row-based (assign = 1); every other nonzero,
// and all of the diagonal block, column-based (assign = 0).
int joint_plan(shiro_plan plan, const int64_t* w_row, const int64_t* w_col, uint8_t* assign,
               int64_t* stats, int32_t n_threads, hipStream_t s) {
  const int64_t rows = plan->rows, nnz = plan->nnz, K = plan->K;
  const int32_t P = plan->P, p = plan->p;
  std::vector<int64_t> rp((size_t)rows + 1);
  std::vector<int32_t> col((size_t)std::max<int64_t>(nnz, 1));
  SHIRO_HIP(hipMemcpyAsync(rp.data(), plan->row_ptr, (size_t)(rows + 1) * 8, hipMemcpyDeviceToHost, s));
  if (nnz > 0) SHIRO_HIP(hipMemcpyAsync(col.data(), plan->col, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  // bucket the nonzeros by block, keeping CSR order inside each block
  std::vector<int64_t> boff((size_t)P + 1, 0);
  for (int64_t k = 0; k < nnz; ++k) ++boff[col[k] / K + 1];
  for (int32_t q = 0; q < P; ++q) boff[q + 1] += boff[q];
  std::vector<int64_t> order((size_t)std::max<int64_t>(nnz, 1)), fill(boff.begin(), boff.end() - 1);
  std::vector<int32_t> row_of((size_t)std::max<int64_t>(nnz, 1));
  for (int64_t i = 0; i < rows; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      row_of[k] = (int32_t)i;
      order[fill[col[k] / K]++] = k;
    }
  if (assign) std::memset(assign, 0, (size_t)nnz);
  if (stats) std::memset(stats, 0, sizeof(int64_t) * 5 * (size_t)P);
  std::atomic<int32_t> next{0};
  std::atomic<int> failed{0};
  auto worker = [&]() {
    std::vector<int32_t> lrow, lcol, left, right;
    std::vector<int64_t> wl, wr;
    std::vector<uint8_t> cl, cr;
    for (int32_t q = next++; q < P; q = next++) {
      const int64_t b = boff[q], e = boff[q + 1];
      // local ids: rows ascending by first appearance (CSR order), columns sorted
      lrow.clear();
      lcol.clear();
      left.resize((size_t)(e - b));
      right.resize((size_t)(e - b));
      for (int64_t x = b; x < e; ++x) {
        const int32_t r = row_of[order[x]];
        if (lrow.empty() || lrow.back() != r) lrow.push_back(r);
        left[x - b] = (int32_t)lrow.size() - 1;
        lcol.push_back(col[order[x]]);
      }
      std::sort(lcol.begin(), lcol.end());
      lcol.erase(std::unique(lcol.begin(), lcol.end()), lcol.end());
      for (int64_t x = b; x < e; ++x)
        right[x - b] = (int32_t)(std::lower_bound(lcol.begin(), lcol.end(), col[order[x]]) - lcol.begin());
      if (stats) {
        stats[5 * q + 1] = (int64_t)lrow.size();
        stats[5 * q + 2] = (int64_t)lcol.size();
      }
      if (q == p || e == b) continue;
      wl.resize(lrow.size());
      wr.resize(lcol.size());
      for (size_t i = 0; i < lrow.size(); ++i) wl[i] = w_row ? w_row[lrow[i]] : 1;
      for (size_t j = 0; j < lcol.size(); ++j) wr[j] = w_col ? w_col[lcol[j]] : 1;
      cl.assign(lrow.size(), 0);
      cr.assign(lcol.size(), 0);
      int64_t mu = 0;
      if (solve_mvc((int64_t)lrow.size(), (int64_t)lcol.size(), e - b, left.data(), right.data(), wl.data(),
                    wr.data(), cl.data(), cr.data(), &mu) != SHIRO_OK) {
        failed = 1;
        return;
      }
      if (stats) {
        stats[5 * q + 0] = mu;
        int64_t nr = 0, nc = 0;
        for (uint8_t v : cl) nr += v;
        for (uint8_t v : cr) nc += v;
        stats[5 * q + 3] = nr;
        stats[5 * q + 4] = nc;
      }
      if (assign)
        for (int64_t x = b; x < e; ++x) assign[order[x]] = cl[left[x - b]];
    }
  };
  int nt = n_threads > 0 ? n_threads : (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  nt = std::min<int>(nt, std::max(1, P));
  std::vector<std::thread> pool;
  for (int i = 1; i < nt; ++i) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  if (failed) return set_error(SHIRO_ERR_HIP, "joint_plan: a block failed");
  return SHIRO_OK;
}

}  // namespace shiro
