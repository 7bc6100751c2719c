// A stand-in for qpg::parallel_chunks (csrc/host_parallel.cpp) for tests: QPG_TEST_THREADS
// threads (1 when unset) take the chunks in a scrambled order, so that a result that depended on
// the number of threads or on the order in which chunks run would differ between builds.
#include <atomic>
#include <cstdlib>
#include <functional>
#include <thread>
#include <vector>

#include "qpg_internal.hpp"

namespace qpg {

void parallel_chunks(int64_t n, int64_t chunk, const std::function<void(int64_t, int64_t, int64_t)>& f) {
  if (n <= 0) return;
  const int64_t nc = (n + chunk - 1) / chunk;
  const char* env = std::getenv("QPG_TEST_THREADS");
  const int64_t T = std::max<int64_t>(1, std::min<int64_t>(env ? std::atoi(env) : 1, 64));
  // chunk order: a multiplicative scramble of 0..nc−1 (a stride coprime to nc)
  int64_t stride = 1;
  for (int64_t s : {7919, 104729, 15485863, 3, 5})
    if (nc % s != 0) {
      stride = s % nc == 0 ? 1 : s;
      break;
    }
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    for (int64_t i; (i = next.fetch_add(1)) < nc;) {
      const int64_t c = (i * stride) % nc;
      f(c, c * chunk, std::min(n, (c + 1) * chunk));
    }
  };
  std::vector<std::thread> th;
  for (int64_t t = 1; t < T; ++t) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
}

}  // namespace qpg
