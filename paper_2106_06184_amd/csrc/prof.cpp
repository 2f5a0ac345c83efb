// Opt-in kernel timing (see prof.h).
#include "prof.h"

#include <thread>
#include <unordered_map>

namespace bem {

namespace {
// begin/end pairs are matched per calling thread (launches from different threads interleave)
thread_local std::vector<hipEvent_t> t_open;
thread_local bool t_opted_out = false;
}  // namespace

void Profiler::opt_out_this_thread() { t_opted_out = true; }

bool Profiler::enabled() const { return on_ && !t_opted_out; }

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
  Pending oldest{};
  bool wait_oldest = false;
  {
    std::lock_guard<std::mutex> g(mu_);
    pending_.push_back({a, b, cls, bytes, work});
    // harvest the oldest pairs that have completed (a few per launch, oldest first: O(1) per
    // launch however deep the device queues of the streams are)
    for (int n = 0; n < 8 && !pending_.empty(); ++n) {
      const Pending& p = pending_.front();
      if (hipEventQuery(p.b) != hipSuccess) break;
      account(p);
      pending_.pop_front();
    }
    (void)hipGetLastError();
    // bound the events in flight: beyond kMaxOutstanding the calling thread waits for the oldest
    // pair (outside the lock), so timing never holds an unbounded number of device signals
    if (pending_.size() > kMaxOutstanding) {
      oldest = pending_.front();
      pending_.pop_front();
      wait_oldest = true;
    }
  }
  if (wait_oldest) {
    (void)hipEventSynchronize(oldest.b);
    std::lock_guard<std::mutex> g(mu_);
    account(oldest);
  }
}

void Profiler::account(const Pending& p) {
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
}

void Profiler::harvest(bool wait) {
  std::lock_guard<std::mutex> g(mu_);
  std::deque<Pending> keep;
  for (auto& p : pending_) {
    if (wait) (void)hipEventSynchronize(p.b);
    if (hipEventQuery(p.b) == hipSuccess) account(p);
    else keep.push_back(p);
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
