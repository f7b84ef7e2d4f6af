// Host worker threads for the per-problem host work of the batched form
// (plans, Ritz values and restarts of many problems at once).  Plain C++ (no
// HIP), so it can be built alone under the thread sanitizer.
#pragma once
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace riga {

// Host worker threads kept for the life of the process (up to 15 besides the
// caller): run(n, f) calls f(i) for every i in [0, n) on the workers and the
// caller, handing indices out one at a time (problems differ in cost), and
// returns when all are done.  Calls are serialised.
class HostPool {
 public:
  static HostPool& get() {
    static HostPool pool;
    return pool;
  }
  void run(int n, const std::function<void(int)>& f) {
    std::lock_guard<std::mutex> serial(run_mu_);
    if (th_.empty() || n <= 1) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &f;
      n_ = n;
      next_.store(0);
      busy_ = (int)th_.size();
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return busy_ == 0; });
    job_ = nullptr;
    std::exception_ptr e;
    {
      std::lock_guard<std::mutex> ek(err_mu_);
      std::swap(e, err_);
    }
    if (e) std::rethrow_exception(e);
  }

 private:
  HostPool() {
    const int nt = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
    for (int t = 1; t < nt; ++t) th_.emplace_back([this] { loop(); });
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  // A job that throws stops nothing else: the first exception is kept and
  // rethrown on the calling thread once every worker is idle.
  void work() {
    for (int i = next_.fetch_add(1); i < n_; i = next_.fetch_add(1)) {
      try {
        (*job_)(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(err_mu_);
        if (!err_) err_ = std::current_exception();
      }
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
      std::lock_guard<std::mutex> lk(mu_);
      if (--busy_ == 0) done_cv_.notify_one();
    }
  }
  std::vector<std::thread> th_;
  std::mutex run_mu_, mu_, err_mu_;
  std::exception_ptr err_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* job_ = nullptr;
  int n_ = 0, busy_ = 0;
  std::atomic<int> next_{0};
  uint64_t gen_ = 0;
  bool stop_ = false;
};

}  // namespace riga
