// Opt-in per-kernel-class timing: HIP events recorded around launches on their own stream,
// with the algorithmic bytes (or work units) of every launch.  Disabled by default; the events
// are harvested at the library's own stream synchronisation points.
#pragma once

#include <hip/hip_runtime.h>

#include <deque>
#include <mutex>
#include <vector>

namespace bem {

enum KernelClass : int {
  KC_GEMV_F64 = 0,   // dense complex products, float64 storage (bytes = matrix bytes read)
  KC_GEMV_F32 = 1,   // dense complex products, float32 storage
  KC_FILL_L = 2,     // far L^A/L^phi fill (work = Green's-function evaluations, bytes = written)
  KC_FILL_K = 3,     // far K~ fill (work = gradient evaluations, bytes = written)
  KC_FILL_NEAR = 4,  // near-pair singular corrections
  KC_GATHER = 5,     // half-RWG / cell to edge gathers (bytes = read + written)
  KC_GEMM_F32 = 6,   // multi-excitation products on matrix cores (work = real flops)
  KC_DENSE_INV = 7,  // Gauss-Jordan panel updates of the dense inversions (work = real flops)
  KC_GEMM_F64 = 8,   // multi-excitation products, float64 matrix cores (work = real flops)
  KC_COUNT = 9
};

struct ClassStats {
  long long launches = 0;
  double ms = 0, bytes = 0, work = 0;
};

class Profiler {
 public:
  static Profiler& get();
  // Launches from threads that opted out (the serving loop's workers) are not timed: requests
  // that overlap on the device would time each other, and a timing event waited for on one
  // worker can depend on launches another worker has still to make.
  static void opt_out_this_thread();
  bool enabled() const;
  void enable(bool on);
  // Record an event pair around a launch issued between begin() and end().
  void begin(hipStream_t st);
  void end(hipStream_t st, int cls, double bytes, double work);
  void harvest(bool wait);
  ClassStats read(int cls);

 private:
  struct Pending {
    hipEvent_t a, b;
    int cls;
    double bytes, work;
  };
  hipEvent_t take();
  void account(const Pending& p);  // with mu_ held
  static constexpr size_t kMaxOutstanding = 1024;
  std::mutex mu_;
  bool on_ = false;
  std::vector<hipEvent_t> pool_;
  std::deque<Pending> pending_;
  ClassStats stats_[KC_COUNT];
};

// RAII helper for a single launch.
struct ProfScope {
  hipStream_t st;
  int cls;
  double bytes, work;
  bool on;
  ProfScope(hipStream_t s, int c, double b, double w) : st(s), cls(c), bytes(b), work(w) {
    on = Profiler::get().enabled();
    if (on) Profiler::get().begin(st);
  }
  ~ProfScope() {
    if (on) Profiler::get().end(st, cls, bytes, work);
  }
};

}  // namespace bem
