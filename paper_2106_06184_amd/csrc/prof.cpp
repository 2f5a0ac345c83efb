// Opt-in kernel timing (see prof.h).
#include "prof.h"

#include <thread>
#include <unordered_map>

namespace bem {

namespace {
// begin/end pairs are matched per calling thread (launches from different threads interleave)
thread_local std::vector<hipEvent_t> t_open;
}  // namespace

Profiler& Profiler::get() {
  static Profiler p;
  return p;
}

void Profiler::enable(bool on) {
  std::lock_guard<std::mutex> g(mu_);
  on_ = on;
  if (on)
    for (auto& s : stats_) s = ClassStats{};
}

hipEvent_t Profiler::take() {
  if (!pool_.empty()) {
    hipEvent_t e = pool_.back();
    pool_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void Profiler::begin(hipStream_t st) {
  hipEvent_t a;
  {
    std::lock_guard<std::mutex> g(mu_);
    a = take();
  }
  (void)hipEventRecord(a, st);
  t_open.push_back(a);
}

void Profiler::end(hipStream_t st, int cls, double bytes, double work) {
  if (t_open.empty()) return;
  hipEvent_t a = t_open.back();
  t_open.pop_back();
  hipEvent_t b;
  {
    std::lock_guard<std::mutex> g(mu_);
    b = take();
  }
  (void)hipEventRecord(b, st);
  std::lock_guard<std::mutex> g(mu_);
  pending_.push_back({a, b, cls, bytes, work});
  if (pending_.size() > 4096) {
    // keep the pool bounded: harvest what has completed
    std::vector<Pending> keep;
    for (auto& p : pending_) {
      if (hipEventQuery(p.b) == hipSuccess) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
          auto& s = stats_[p.cls];
          s.launches++;
          s.ms += ms;
          s.bytes += p.bytes;
          s.work += p.work;
        }
        pool_.push_back(p.a);
        pool_.push_back(p.b);
      } else {
        keep.push_back(p);
      }
    }
    pending_.swap(keep);
  }
}

void Profiler::harvest(bool wait) {
  std::lock_guard<std::mutex> g(mu_);
  std::vector<Pending> keep;
  for (auto& p : pending_) {
    if (wait) (void)hipEventSynchronize(p.b);
    if (hipEventQuery(p.b) == hipSuccess) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        auto& s = stats_[p.cls];
        s.launches++;
        s.ms += ms;
        s.bytes += p.bytes;
        s.work += p.work;
      }
      pool_.push_back(p.a);
      pool_.push_back(p.b);
    } else {
      keep.push_back(p);
    }
  }
  pending_.swap(keep);
  (void)hipGetLastError();
}

ClassStats Profiler::read(int cls) {
  harvest(true);
  std::lock_guard<std::mutex> g(mu_);
  return (cls >= 0 && cls < KC_COUNT) ? stats_[cls] : ClassStats{};
}

}  // namespace bem
