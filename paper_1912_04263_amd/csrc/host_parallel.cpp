// Host threads for setup work (validation, format conversion, equilibration, work lists).
#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

#include "qpg_internal.hpp"

namespace qpg {

void parallel_chunks(int64_t n, int64_t chunk, const std::function<void(int64_t, int64_t, int64_t)>& f) {
  if (n <= 0) return;
  const int64_t nc = (n + chunk - 1) / chunk;
  const int64_t hw = std::max(1u, std::thread::hardware_concurrency());
  const int64_t T = std::min<int64_t>(std::min<int64_t>(hw, 16), nc);
  auto body = [&](int64_t c) { f(c, c * chunk, std::min(n, (c + 1) * chunk)); };
  if (T <= 1) {
    for (int64_t c = 0; c < nc; ++c) body(c);
    return;
  }
  // an exception in a worker (an allocation failure) stops the remaining chunks and is
  // rethrown here, in the calling thread
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&]() {
    try {
      for (int64_t c; (c = next.fetch_add(1)) < nc;) body(c);
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!err) err = std::current_exception();
      next.store(nc);
    }
  };
  std::vector<std::thread> th;
  th.reserve((size_t)T - 1);
  for (int64_t t = 1; t < T; ++t) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace qpg
