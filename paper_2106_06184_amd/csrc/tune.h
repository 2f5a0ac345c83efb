// Online launch-variant selection (one tuner per process, classes kept per device).  Some kernels come in variants that compute bitwise the same
// result (the same products summed in the same order; only the workgroup tile shape, the rows
// per workgroup or the tile-to-XCD mapping differ).  For every problem class (a key built from
// the shape) the first launches try each candidate three times, timed with HIP events on the
// launch stream; once every trial has completed, the fastest candidate (by its fastest trial,
// and by at least 3% over the first candidate) is used for that class for the rest of the
// process.  Because the candidates agree bitwise, results do not depend on which
// one runs.  Launches into a capturing stream never time (they take the decided candidate, or
// the first).  BEM_TUNE=0 in the environment always takes the first candidate.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <deque>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace bem {

class Tuner {
 public:
  static Tuner& get();
  // Candidate for a launch of class `key` among n; *trial is set when the launch is to be timed.
  int pick(uint64_t key, int n, hipStream_t st, bool* trial);
  // Register a timed trial (events recorded around the launch on its stream).
  void submit(uint64_t key, int cand, hipEvent_t a, hipEvent_t b);
  hipEvent_t take_event();
  void give_back(hipEvent_t e);
  // Decided candidate of a class, or -1 (tests and reports).
  int decided(uint64_t key);

 private:
  struct Entry {
    int n = 0, choice = -1, issued = 0;
    std::vector<float> best;
    std::vector<int> done;
  };
  struct Trial {
    uint64_t key;
    int cand, dev;
    hipEvent_t a, b;
  };
  void harvest_locked();
  std::mutex mu_;
  std::unordered_map<uint64_t, Entry> map_;
  std::deque<Trial> pending_;
  std::unordered_map<int, std::vector<hipEvent_t>> pool_;  // per device
  int enabled_ = -1;
};

// RAII use around one launch: picks the candidate, records the trial's events.
class TuneScope {
 public:
  TuneScope(uint64_t key, int n, hipStream_t st);
  ~TuneScope();
  int variant() const { return cand_; }

 private:
  uint64_t key_;
  int cand_ = 0;
  bool trial_ = false;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
};

// Key helpers: a class id and up to six fields packed 8 bits each (log2 buckets for sizes); the
// top byte is the device's.
inline int log2_bucket(int64_t v) {
  int b = 0;
  while (v > 1 && b < 62) {
    v >>= 1;
    ++b;
  }
  return b;
}
inline uint64_t tune_key(uint32_t cls, std::initializer_list<int64_t> fields) {
  uint64_t k = cls & 0xff;
  int sh = 8;
  for (int64_t f : fields) {
    k |= (uint64_t(f) & 0xff) << sh;
    sh += 8;
    if (sh >= 56) break;
  }
  return k;
}

}  // namespace bem
