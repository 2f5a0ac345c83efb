// Online launch-variant selection (see tune.h).
#include "tune.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace bem {

namespace {
constexpr int kTrials = 3;  // timed launches per candidate; the fastest counts
// another candidate replaces the first only when it is faster by this factor (launches that
// overlap other work, as in serving, time noisily)
constexpr float kMargin = 0.97f;

bool verbose_env() {
  const char* v = std::getenv("BEM_VERBOSE");
  return v && std::strcmp(v, "0") != 0;
}
}  // namespace

Tuner& Tuner::get() {
  static Tuner t;
  return t;
}

hipEvent_t Tuner::take_event() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  {
    std::lock_guard<std::mutex> g(mu_);
    auto& pool = pool_[dev];
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void Tuner::harvest_locked() {
  while (!pending_.empty()) {
    const Trial& t = pending_.front();
    if (hipEventQuery(t.b) != hipSuccess) {
      (void)hipGetLastError();
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      Entry& e = map_[t.key];
      if (t.cand < e.n) {
        e.best[t.cand] = e.done[t.cand] == 0 ? ms : std::min(e.best[t.cand], ms);
        e.done[t.cand]++;
      }
    } else {
      (void)hipGetLastError();
    }
    pool_[t.dev].push_back(t.a);
    pool_[t.dev].push_back(t.b);
    pending_.pop_front();
  }
}

int Tuner::pick(uint64_t key, int n, hipStream_t st, bool* trial) {
  *trial = false;
  if (n <= 1) return 0;
  std::lock_guard<std::mutex> g(mu_);
  if (enabled_ < 0) {
    const char* v = std::getenv("BEM_TUNE");
    enabled_ = (v && std::strcmp(v, "0") == 0) ? 0 : 1;
  }
  if (!enabled_) return 0;
  {
    auto it = map_.find(key);
    if (it != map_.end() && it->second.choice >= 0) return it->second.choice;
  }
  // a launch being captured into a graph is not timed (and no event is queried meanwhile)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  if (cs != hipStreamCaptureStatusNone) return 0;
  harvest_locked();  // (may add entries: take the reference after it)
  Entry& e = map_[key];
  if (e.n == 0) {
    e.n = n;
    e.best.assign(n, 0.f);
    e.done.assign(n, 0);
  }
  bool all = true;
  for (int c = 0; c < e.n; ++c) all = all && e.done[c] >= kTrials;
  if (all) {
    int best = 0;
    for (int c = 1; c < e.n; ++c)
      if (e.best[c] < e.best[best]) best = c;
    if (best != 0 && !(e.best[best] < kMargin * e.best[0])) best = 0;
    e.choice = best;
    if (verbose_env()) {
      std::fprintf(stderr, "[bem] tuned class %016llx: candidate %d of %d (", (unsigned long long)key, best, e.n);
      for (int c = 0; c < e.n; ++c) std::fprintf(stderr, "%s%.4f ms", c ? ", " : "", e.best[c]);
      std::fprintf(stderr, ")\n");
    }
    return best;
  }
  if (e.issued < e.n * kTrials) {
    const int c = e.issued % e.n;
    ++e.issued;
    *trial = true;
    return c;
  }
  // every trial is in flight: the first candidate until they complete
  return 0;
}

void Tuner::submit(uint64_t key, int cand, hipEvent_t a, hipEvent_t b) {
  int dev = int((key >> 56) & 0xff);
  std::lock_guard<std::mutex> g(mu_);
  pending_.push_back({key, cand, dev, a, b});
}

void Tuner::give_back(hipEvent_t e) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> g(mu_);
  pool_[dev].push_back(e);
}

int Tuner::decided(uint64_t key) {
  std::lock_guard<std::mutex> g(mu_);
  harvest_locked();
  auto it = map_.find(key);
  return it == map_.end() ? -1 : it->second.choice;
}

TuneScope::TuneScope(uint64_t key, int n, hipStream_t st) : key_(key), st_(st) {
  // classes are per device (its events time its own launches)
  int dev = 0;
  if (n > 1 && hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  key_ = key ^ (uint64_t(dev & 0xff) << 56);
  cand_ = Tuner::get().pick(key_, n, st, &trial_);
  if (trial_) {
    a_ = Tuner::get().take_event();
    if (!a_ || hipEventRecord(a_, st_) != hipSuccess) {
      (void)hipGetLastError();
      trial_ = false;
    }
  }
}

TuneScope::~TuneScope() {
  if (!trial_) return;
  hipEvent_t b = Tuner::get().take_event();
  if (!b || hipEventRecord(b, st_) != hipSuccess) {
    (void)hipGetLastError();
    Tuner::get().give_back(a_);
    if (b) Tuner::get().give_back(b);
    return;
  }
  Tuner::get().submit(key_, cand_, a_, b);
}

}  // namespace bem
