// Serving loop (see serve.h).
#include "serve.h"

#include "prof.h"

#include <chrono>

namespace bem {

constexpr int kSlots = 4;
constexpr int kNomemRetries = 2;  // reruns of a request that ran out of device memory beside others

struct Request {
  // owned copies of the caller's inputs
  std::vector<double> xyz;
  std::vector<int32_t> tri, obj;
  std::vector<bem_material> mats;
  bem_problem prob{};
  std::vector<bem_excitation> exc;
  std::vector<std::vector<int32_t>> gaps;
  bem_solve_opts opts{};
  bem_c64 *H = nullptr, *E = nullptr, *rho = nullptr;
  // state
  size_t bytes = 0;   // admitted reservation (the estimate, plus what the solve added)
  size_t bytes0 = 0;  // the estimate
  int nomem_retries = 0;
  int status = BEM_PENDING;
  std::string msg;
  bem_solve_info info{};
  std::chrono::steady_clock::time_point t_submit;
};

// ---------------------------------------------------------------- combiner

namespace {
// Time a waiting product gives the other solving requests to join its launch.
constexpr auto kCombineWindow = std::chrono::microseconds(100);
thread_local hipEvent_t tl_ready = nullptr, tl_done = nullptr;
}  // namespace

Combiner::Combiner(int device) {
  (void)device;
  BEM_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
}

Combiner::~Combiner() {
  if (stream_) (void)hipStreamDestroy(stream_);
}

void Combiner::join() {
  std::lock_guard<std::mutex> g(mu_);
  ++solving_;
}

void Combiner::leave() {
  std::lock_guard<std::mutex> g(mu_);
  --solving_;
  cv_.notify_all();  // a waiter may now complete the group
}

void Combiner::launch_all() {
  std::vector<GemvDesc> all;
  for (Pending* p : pending_) {
    BEM_HIP(hipStreamWaitEvent(stream_, p->ready, 0));
    all.insert(all.end(), p->ds->begin(), p->ds->end());
  }
  launch_gemv_grouped(all.data(), int(all.size()), stream_);
  for (Pending* p : pending_) {
    BEM_HIP(hipEventRecord(p->done, stream_));
    p->finished = true;
  }
  ++launches_;
  served_ += (long long)pending_.size();
  pending_.clear();
  cv_.notify_all();
}

void Combiner::run(const std::vector<GemvDesc>& ds, hipStream_t st) {
  if (!tl_ready) {
    BEM_HIP(hipEventCreateWithFlags(&tl_ready, hipEventDisableTiming));
    BEM_HIP(hipEventCreateWithFlags(&tl_done, hipEventDisableTiming));
  }
  BEM_HIP(hipEventRecord(tl_ready, st));
  Pending me{&ds, tl_ready, tl_done, false};
  {
    std::unique_lock<std::mutex> lk(mu_);
    pending_.push_back(&me);
    const auto deadline = std::chrono::steady_clock::now() + kCombineWindow;
    while (!me.finished) {
      if (int(pending_.size()) >= solving_ || std::chrono::steady_clock::now() >= deadline) {
        launch_all();
        break;
      }
      cv_.wait_until(lk, deadline);
    }
  }
  BEM_HIP(hipStreamWaitEvent(st, tl_done, 0));
}

// ---------------------------------------------------------------- server

size_t Server::estimate_bytes(int64_t nt, int64_t ne, int64_t nobj, int precision, int restart) {
  (void)ne;
  return estimate_request_bytes(nt, nobj, precision, restart, 1);
}

// Every slot's stream and pinned staging are made here, on the caller's thread, so that a
// failure reaches the caller (bem_submit) instead of leaving a slot silently dead.
Server::Server(Ctx* ctx) : ctx_(ctx), comb_(ctx->device) {
  slot_stream_.assign(kSlots, nullptr);
  slot_pinned_.assign(kSlots, nullptr);
  for (int s = 0; s < kSlots; ++s) {
    hipError_t e = hipStreamCreateWithFlags(&slot_stream_[s], hipStreamNonBlocking);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&slot_pinned_[s]), kPinnedBytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release_slots();
      throw Error(BEM_E_DEVICE, std::string("serving slot set-up failed: ") + hipGetErrorString(e));
    }
  }
  for (int s = 0; s < kSlots; ++s) threads_.emplace_back(&Server::worker, this, s);
}

void Server::release_slots() {
  for (auto& p : slot_pinned_)
    if (p) (void)hipHostFree(p), p = nullptr;
  for (auto& st : slot_stream_)
    if (st) (void)hipStreamDestroy(st), st = nullptr;
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto& t : threads_) t.join();
  release_slots();
}

bem_ticket Server::submit(const bem_request& r) {
  if (!r.xyz || !r.tri || r.nv <= 0 || r.nt <= 0 || !r.exc || r.nexc <= 0)
    throw Error(BEM_E_INVALID, "incomplete request");
  if (r.prob.n_obj <= 0 || !r.prob.obj) throw Error(BEM_E_INVALID, "request without materials");
  auto q = std::make_shared<Request>();
  q->xyz.assign(r.xyz, r.xyz + 3 * r.nv);
  q->tri.assign(r.tri, r.tri + 3 * r.nt);
  if (r.obj) q->obj.assign(r.obj, r.obj + r.nt);
  q->mats.assign(r.prob.obj, r.prob.obj + r.prob.n_obj);
  q->prob = r.prob;
  q->prob.obj = q->mats.data();
  q->exc.assign(r.exc, r.exc + r.nexc);
  for (auto& e : q->exc) {
    if (e.kind == BEM_EXC_DELTA_GAP && e.gap_edges && e.n_gap > 0) {
      q->gaps.emplace_back(e.gap_edges, e.gap_edges + 2 * e.n_gap);
      e.gap_edges = q->gaps.back().data();
    }
  }
  q->opts = r.opts;
  q->H = r.H;
  q->E = r.E;
  q->rho = r.rho;
  const int64_t ne = 3 * r.nt / 2;
  (void)ne;
  const int64_t nunk = 4 * r.nt - 2 * r.prob.n_obj;  // upper bound of 2 NE + NT - n_obj
  q->bytes = estimate_request_bytes(r.nt, r.prob.n_obj, r.prob.precision,
                                    r.opts.restart > 0 ? r.opts.restart : auto_restart(nunk, r.nexc),
                                    r.nexc, r.prob.formulation);
  if (q->bytes > ctx_->budget) throw Error(BEM_E_NOMEM, "request can never fit the device budget");
  q->bytes0 = q->bytes;
  q->t_submit = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> g(mu_);
  const bem_ticket t = next_++;
  all_[t] = q;
  queue_.push_back(q);
  cv_.notify_all();
  return t;
}

int Server::poll(bem_ticket t, bem_solve_info* info, std::string* msg) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = all_.find(t);
  if (it == all_.end()) throw Error(BEM_E_INVALID, "unknown ticket");
  auto& q = it->second;
  if (q->status == BEM_PENDING) return BEM_PENDING;
  if (info) *info = q->info;
  if (msg) *msg = q->msg;
  const int st = q->status;
  all_.erase(it);
  return st;
}

void Server::drain() {
  std::unique_lock<std::mutex> lk(mu_);
  done_cv_.wait(lk, [&] { return queue_.empty() && active_ == 0; });
}

void Server::worker(int slot) {
  Profiler::opt_out_this_thread();
  hipStream_t st = slot_stream_[slot];
  double* pinned = slot_pinned_[slot];
  const bool device_ok = hipSetDevice(ctx_->device) == hipSuccess;
  while (true) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(mu_);
      // admit the oldest request whose estimate fits next to the running ones (first-fit
      // from the head keeps small requests moving while a large one waits for memory); a
      // request that ran out of device memory beside others runs alone, and nothing queued
      // behind it starts before it
      auto pick = [&]() {
        if (exclusive_) return queue_.end();
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
          if ((*it)->nomem_retries > 0) return active_ == 0 ? it : queue_.end();
          if (reserved_ + (*it)->bytes <= ctx_->budget) return it;
        }
        return queue_.end();
      };
      cv_.wait(lk, [&] { return stop_ || pick() != queue_.end(); });
      if (stop_) break;
      const auto it = pick();
      q = *it;
      queue_.erase(it);
      if (q->nomem_retries > 0) exclusive_ = true;
      reserved_ += q->bytes;
      ++active_;
    }
    int status = BEM_OK;
    std::string msg;
    bem_solve_info info{};
    try {
      if (!device_ok) throw Error(BEM_E_DEVICE, "serving slot could not select the device");
      auto mo = std::make_unique<MeshObj>();
      mo->mesh = build_mesh(q->xyz.data(), int64_t(q->xyz.size() / 3), q->tri.data(), int64_t(q->tri.size() / 3),
                            q->obj.empty() ? nullptr : q->obj.data());
      OpObj op(ctx_);
      op.stream = st;
      op.pinned = pinned;
      assemble_op(op, *mo, q->prob);
      // solve phase: small products go through the combiner
      struct Joined {
        Combiner& c;
        explicit Joined(Combiner& cc) : c(cc) { c.join(); }
        ~Joined() { c.leave(); }
      } joined(comb_);
      op.comb = &comb_;
      op.reserve = [this, &q](size_t extra) {
        std::lock_guard<std::mutex> g(mu_);
        if (reserved_ + extra > ctx_->budget) return false;
        reserved_ += extra;
        q->bytes += extra;  // released with the rest of the request's reservation
        return true;
      };
      status = solve_op(op, q->exc.data(), int64_t(q->exc.size()), q->opts, q->H, q->E, q->rho, &info, st);
      op.comb = nullptr;
      op.reserve = nullptr;
      info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - q->t_submit).count();
    } catch (const Error& e) {
      status = e.code;
      msg = e.what();
    } catch (const std::exception& e) {
      status = BEM_E_INVALID;
      msg = e.what();
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      reserved_ -= q->bytes;
      --active_;
      if (q->nomem_retries > 0) exclusive_ = false;
      if (status == BEM_E_NOMEM && active_ > 0 && q->nomem_retries < kNomemRetries) {
        // the estimates let the device fill beyond what was free: the request waits at the
        // head of the queue and runs again alone
        ++q->nomem_retries;
        q->bytes = q->bytes0;
        queue_.push_front(q);
      } else {
        q->status = status;
        q->msg = msg;
        q->info = info;
      }
    }
    cv_.notify_all();
    done_cv_.notify_all();
  }
  if (tl_ready) (void)hipEventDestroy(tl_ready);
  if (tl_done) (void)hipEventDestroy(tl_done);
  tl_ready = tl_done = nullptr;
}

}  // namespace bem
