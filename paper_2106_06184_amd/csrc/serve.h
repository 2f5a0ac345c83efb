// Serving loop for bem_submit / bem_poll: requests are admitted while their estimated device
// footprint fits the context budget and a slot is free; every admitted request runs on its own
// HIP stream (own operator, own Krylov state), so the work of requests admitted at different
// times overlaps on the device.  While requests solve, their small dense products (those that
// would not fill the GPU alone) are gathered by a combiner into shared grouped launches.
// Results do not depend on the mix: every product row and every reduction is computed in a
// fixed order whatever launch it runs in.
#pragma once

#include <condition_variable>
#include <deque>
#include <thread>

#include "ctx.h"

namespace bem {

struct Request;

// Leader-based combiner: a request that needs a small product enqueues its descriptors and
// waits; when every solving request has a product waiting, or the oldest waiter's window has
// passed, the waiting thread that notices launches all waiting descriptors as one grouped
// launch on the combiner's stream (after each requester's stream, via events) and every
// requester's stream then waits for it.
class Combiner : public ProductCombiner {
 public:
  explicit Combiner(int device);
  ~Combiner() override;
  void run(const std::vector<GemvDesc>& ds, hipStream_t st) override;
  void join();   // a request enters its solve phase
  void leave();  // ... and leaves it
  long long launches() {
    std::lock_guard<std::mutex> g(mu_);
    return launches_;
  }
  long long requests() {
    std::lock_guard<std::mutex> g(mu_);
    return served_;
  }

 private:
  struct Pending {
    const std::vector<GemvDesc>* ds;
    hipEvent_t ready, done;
    bool finished;
  };
  void launch_all();  // with mu_ held
  std::mutex mu_;
  std::condition_variable cv_;
  std::vector<Pending*> pending_;
  int solving_ = 0;
  hipStream_t stream_ = nullptr;
  long long launches_ = 0, served_ = 0;
};

class Server {
 public:
  explicit Server(Ctx* ctx);
  ~Server();
  bem_ticket submit(const bem_request& r);
  int poll(bem_ticket t, bem_solve_info* info, std::string* msg);
  void drain();
  static size_t estimate_bytes(int64_t nt, int64_t ne, int64_t nobj, int precision, int restart);
  void combiner_stats(int64_t* launches, int64_t* products) {
    *launches = comb_.launches();
    *products = comb_.requests();
  }

 private:
  void worker(int slot);
  void release_slots();
  Ctx* ctx_;
  std::vector<hipStream_t> slot_stream_;
  std::vector<double*> slot_pinned_;
  Combiner comb_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<std::shared_ptr<Request>> queue_;
  std::map<bem_ticket, std::shared_ptr<Request>> all_;
  std::vector<std::thread> threads_;
  size_t reserved_ = 0;
  int active_ = 0;
  bool exclusive_ = false;  // a request rerun after running out of device memory is solving alone
  bool stop_ = false;
  bem_ticket next_ = 1;
};

}  // namespace bem
