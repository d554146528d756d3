// Host driver of the cover solver (csrc/mvc.hpp), built with the address and
// undefined-behaviour sanitizers by tests/test_sanitizers.py.  Random
// bipartite graphs: the cover must cover every edge, its cost must equal the
// exhaustive minimum on small graphs, and invalid arguments must be named.
// Exit status 0 = every check passed.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2512_20178_amd/csrc/mvc.hpp"

using shiro::mvc::arg_error;
using shiro::mvc::min_weight_cover;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                     \
    }                                                              \
  } while (0)

int main() {
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 400; ++trial) {
    const int L = (int)(rng() % 7), R = (int)(rng() % 7);
    const int E = (L && R) ? (int)(rng() % (L * R + 1)) : 0;
    std::vector<int32_t> le(E), ri(E);
    for (int e = 0; e < E; ++e) {
      le[e] = (int32_t)(rng() % L);
      ri[e] = (int32_t)(rng() % R);
    }
    const bool unit = trial % 2 == 0;
    std::vector<int64_t> wl(L), wr(R);
    for (auto& w : wl) w = unit ? 1 : (int64_t)(rng() % 5);
    for (auto& w : wr) w = unit ? 1 : (int64_t)(rng() % 5);
    std::vector<uint8_t> cl(L + 1), cr(R + 1);
    int64_t weight = -1;
    CHECK(arg_error(L, R, E, le.data(), ri.data(), wl.data(), wr.data(), cl.data(), cr.data(), &weight) == nullptr);
    weight = min_weight_cover(L, R, E, le.data(), ri.data(), unit ? nullptr : wl.data(),
                              unit ? nullptr : wr.data(), cl.data(), cr.data());
    int64_t w = 0;
    for (int i = 0; i < L; ++i) w += cl[i] ? wl[i] : 0;
    for (int j = 0; j < R; ++j) w += cr[j] ? wr[j] : 0;
    CHECK(w == weight);
    for (int e = 0; e < E; ++e) CHECK(cl[le[e]] || cr[ri[e]]);
    // exhaustive minimum over all vertex subsets
    int64_t best = -1;
    for (uint32_t m = 0; m < (1u << (L + R)); ++m) {
      bool ok = true;
      for (int e = 0; e < E && ok; ++e) ok = ((m >> le[e]) & 1u) || ((m >> (L + ri[e])) & 1u);
      if (!ok) continue;
      int64_t c = 0;
      for (int i = 0; i < L; ++i) c += ((m >> i) & 1u) ? wl[i] : 0;
      for (int j = 0; j < R; ++j) c += ((m >> (L + j)) & 1u) ? wr[j] : 0;
      if (best < 0 || c < best) best = c;
    }
    CHECK(best == weight);
  }
  // a larger random graph: the cover is valid
  {
    const int L = 3000, R = 2500, E = 40000;
    std::vector<int32_t> le(E), ri(E);
    for (int e = 0; e < E; ++e) {
      le[e] = (int32_t)(rng() % L);
      ri[e] = (int32_t)(rng() % R);
    }
    std::vector<uint8_t> cl(L), cr(R);
    const int64_t w = min_weight_cover(L, R, E, le.data(), ri.data(), nullptr, nullptr, cl.data(), cr.data());
    for (int e = 0; e < E; ++e) CHECK(cl[le[e]] || cr[ri[e]]);
    CHECK(w <= (L < R ? L : R));
  }
  // invalid arguments are named, nothing is read out of range
  {
    int32_t le[2] = {0, 3}, ri[2] = {0, 0};
    int64_t wl[2] = {1, -1};
    uint8_t cl[2], cr[1];
    int64_t w;
    CHECK(arg_error(2, 1, 2, le, ri, nullptr, nullptr, cl, cr, &w) != nullptr);  // endpoint 3 >= 2
    le[1] = 1;
    CHECK(arg_error(2, 1, 2, le, ri, nullptr, nullptr, cl, cr, &w) == nullptr);
    CHECK(arg_error(2, 1, 2, le, ri, wl, nullptr, cl, cr, &w) != nullptr);  // negative cost
    CHECK(arg_error(-1, 1, 0, nullptr, nullptr, nullptr, nullptr, cl, cr, &w) != nullptr);
    CHECK(arg_error(2, 1, 2, nullptr, ri, nullptr, nullptr, cl, cr, &w) != nullptr);
    CHECK(arg_error(2, 1, 2, le, ri, nullptr, nullptr, cl, cr, nullptr) != nullptr);
  }
  std::printf("mvc driver: %d failed checks\n", fails);
  return fails ? 1 : 0;
}
