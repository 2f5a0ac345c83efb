// Serving loop for bem_submit / bem_poll: requests are admitted while their estimated device
// footprint fits the context budget and a slot is free; every admitted request runs on its own
// HIP stream (own operator, own Krylov state), so the work of requests admitted at different
// times overlaps on the device.  Results do not depend on the mix: every kernel reduces in a
// fixed order.
#pragma once

#include <condition_variable>
#include <deque>
#include <thread>

#include "ctx.h"

namespace bem {

struct Request;

class Server {
 public:
  explicit Server(Ctx* ctx);
  ~Server();
  bem_ticket submit(const bem_request& r);
  int poll(bem_ticket t, bem_solve_info* info, std::string* msg);
  void drain();
  static size_t estimate_bytes(int64_t nt, int64_t ne, int64_t nobj, int precision, int restart);

 private:
  void worker(int slot);
  Ctx* ctx_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<std::shared_ptr<Request>> queue_;
  std::map<bem_ticket, std::shared_ptr<Request>> all_;
  std::vector<std::thread> threads_;
  size_t reserved_ = 0;
  int active_ = 0;
  bool stop_ = false;
  bem_ticket next_ = 1;
};

}  // namespace bem
