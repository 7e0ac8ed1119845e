// Serving loop: window solves of many systems on one GPU with continuous batching.
//
// Not part of the paper's method (which solves one system at a time); it is the
// request loop around it:
//  * submit copies a request's inputs to host memory and queues it;
//  * a scheduler thread admits queued requests in arrival order while their device
//    footprint (context_footprint + window_solve_bytes, an upper bound of what the
//    request allocates) fits the budget and a solve slot is free;
//  * one worker thread per admitted request sets its system up on the request's own
//    stream (overlapping with the passes of the requests already solving), reserves
//    its product workspace and runs the window solve;
//  * every product request of every solving request goes to one GroupBatcher: a pass
//    starts when all solving requests have a request pending (or the oldest pending
//    one has waited 'linger'), and runs sigma_group on the pass stream, so each
//    contraction step of the product is one grouped launch over all requests in the
//    pass;
//  * a request retires when its solve returns; its context is freed, the scheduler
//    admits what now fits, and the result waits for poll/wait.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ppwin.h"
#include "abi.h"
#include "context.h"
#include "solver.h"

namespace ppw {
namespace {

using Clock = std::chrono::steady_clock;

double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

// Product requests of the solving requests, merged into grouped passes.
class GroupBatcher : public ProductSink {
 public:
  GroupBatcher(hipStream_t s, std::chrono::microseconds linger) : s_(s), linger_(linger) {}
  ~GroupBatcher() override {
    for (auto& t : timed_) {
      (void)hipEventDestroy(t.first);
      (void)hipEventDestroy(t.second);
    }
  }
  void join() {
    std::lock_guard<std::mutex> lk(mu_);
    ++active_;
  }
  void leave() {
    std::lock_guard<std::mutex> lk(mu_);
    --active_;
    if (!pending_.empty() && (int)pending_.size() >= active_) serve();
  }
  void multiply(ProductRequest& r) override {
    std::unique_lock<std::mutex> lk(mu_);
    r.served = false;
    pending_.push_back(&r);
    if ((int)pending_.size() >= active_) {
      serve();
    } else {
      const auto deadline = Clock::now() + linger_;
      while (!r.served) {
        if (cv_.wait_until(lk, deadline) == std::cv_status::timeout && !r.served) serve();
      }
    }
    if (r.err) std::rethrow_exception(r.err);
  }
  // passes, requests over all passes, flops, device seconds (synchronizes on the pass events)
  void counters(long* passes, long* jobs, double* flops, double* seconds, long* grouped) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& t : timed_) {
      PPW_HIP(hipEventSynchronize(t.second));
      float ms = 0.f;
      PPW_HIP(hipEventElapsedTime(&ms, t.first, t.second));
      seconds_ += 1e-3 * ms;
      (void)hipEventDestroy(t.first);
      (void)hipEventDestroy(t.second);
    }
    timed_.clear();
    *passes = passes_;
    *jobs = jobs_;
    *flops = flops_;
    *seconds = seconds_;
    *grouped = grouped_;
  }
  void reset() {
    long p, j, g;
    double f, s;
    counters(&p, &j, &f, &s, &g);
    std::lock_guard<std::mutex> lk(mu_);
    passes_ = jobs_ = grouped_ = 0;
    flops_ = seconds_ = 0.0;
  }

 private:
  void serve() {
    std::exception_ptr err;
    try {
      std::vector<PassJob> jobs;
      double flops = 0.0;
      for (auto* r : pending_) {
        PPW_HIP(hipStreamWaitEvent(s_, r->ready, 0));
        PassJob j;
        j.c = r->ctx;
        j.order = r->ctx->order;
        j.k = r->k;
        j.prec = r->prec;
        j.V = r->V;
        j.AV = r->AV;
        j.BV = r->BV;
        j.SV = r->SV;
        jobs.push_back(j);
        flops += sigma_flops(*r->ctx, r->ctx->order, r->k, r->prec);
      }
      hipEvent_t a, b;
      PPW_HIP(hipEventCreate(&a));
      PPW_HIP(hipEventCreate(&b));
      timed_.push_back({a, b});
      PPW_HIP(hipEventRecord(a, s_));
      grouped_ += sigma_group(jobs, s_);
      PPW_HIP(hipEventRecord(b, s_));
      for (auto* r : pending_) PPW_HIP(hipEventRecord(r->done, s_));
      ++passes_;
      jobs_ += (long)pending_.size();
      flops_ += flops;
    } catch (...) {
      err = std::current_exception();
    }
    for (auto* r : pending_) {
      r->err = err;
      r->served = true;
    }
    pending_.clear();
    cv_.notify_all();
  }

  hipStream_t s_;
  std::chrono::microseconds linger_;
  std::mutex mu_;
  std::condition_variable cv_;
  std::vector<ProductRequest*> pending_;
  int active_ = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> timed_;
  long passes_ = 0, jobs_ = 0, grouped_ = 0;
  double flops_ = 0.0, seconds_ = 0.0;
};

struct Request {
  uint64_t id = 0;
  int o = 0, v = 0, naux = 0, order = 2;
  std::vector<double> eps, Boo, Bov, Bvv, dip;
  bool has_dip = false;
  double omega = 0.0;
  int n_roots = 0;
  size_t bytes = 0;
  bool store = false;
  int strip_rows = 0;
  enum State { kQueued, kRunning, kDone } state = kQueued;
  pp_status status = PP_OK;
  std::string error;
  std::vector<double> energies, vectors, osc;
  pp_solve_info info{};
  Clock::time_point t_submit, t_admit, t_done;
};

double percentile(std::vector<double> x, double q) {
  if (x.empty()) return 0.0;
  std::sort(x.begin(), x.end());
  const double pos = q * (double)(x.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < x.size() ? x[i] * (1.0 - f) + x[i + 1] * f : x[i];
}

}  // namespace

class Server {
 public:
  Server(const pp_options& opt, uint64_t budget, int max_active) : opt_(opt), so_(solve_options(opt)) {
    PPW_HIP(hipSetDevice(opt_.device));
    size_t freeb = 0, totalb = 0;
    PPW_HIP(hipMemGetInfo(&freeb, &totalb));
    budget_ = budget ? budget : (size_t)(0.85 * (double)freeb);
    max_active_ = max_active > 0 ? max_active : 8;
    PPW_HIP(hipStreamCreateWithFlags(&pass_stream_, hipStreamNonBlocking));
    gb_.reset(new GroupBatcher(pass_stream_, std::chrono::microseconds(1000)));
    sched_ = std::thread(&Server::scheduler, this);
  }
  ~Server() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
      for (auto& r : queue_) {
        r->state = Request::kDone;
        r->status = PP_EINVAL;
        r->error = "server destroyed before the request was admitted";
      }
      queue_.clear();
    }
    cv_.notify_all();
    if (sched_.joinable()) sched_.join();
    for (auto& w : workers_)
      if (w.joinable()) w.join();
    gb_.reset();
    (void)hipStreamSynchronize(pass_stream_);
    (void)hipStreamDestroy(pass_stream_);
  }

  // device bytes a request may hold, and the amplitude policy it gets
  void plan(Request& r) const {
    const size_t N = (size_t)r.o * r.v;
    const bool f32 = opt_.precision != PP_FP64;
    const double tau_bytes = (double)N * N * (f32 ? 12.0 : 8.0);
    r.store = r.order >= 2 && (opt_.store_amplitudes == 1 ||
                               (opt_.store_amplitudes < 0 && tau_bytes <= (double)budget_ / 16.0));
    if (opt_.strip_rows > 0) {
      r.strip_rows = std::min(opt_.strip_rows, r.o);
    } else {
      const double cap = std::min<double>(2.0 * (1 << 30), (double)budget_ / 32.0);
      r.strip_rows = (int)std::max<double>(1.0, std::min<double>(r.o, cap / (5.0 * r.v * (double)N * 8.0)));
    }
    const int k = window_block_vectors((long)N, r.n_roots, so_);
    const Footprint fp = context_footprint(r.o, r.v, r.naux, r.order, r.has_dip, r.store, r.strip_rows, f32, k,
                                           opt_.precision == PP_SPLIT_BF16);
    r.bytes = std::max(fp.setup_peak, fp.steady + window_solve_bytes((long)N, r.n_roots, so_)) + ((size_t)1 << 20);
  }

  size_t request_bytes(const pp_system& sys, int n_roots) const {
    if (sys.n_occ < 1 || sys.n_vir < 1 || sys.n_aux < 1 || sys.order < 1 || sys.order > 2 || n_roots < 1) return 0;
    Request r;
    r.o = sys.n_occ;
    r.v = sys.n_vir;
    r.naux = sys.n_aux;
    r.order = sys.order;
    r.n_roots = n_roots;
    r.has_dip = sys.dip != nullptr;
    plan(r);
    return r.bytes;
  }

  uint64_t submit(const pp_system& sys, double omega, int n_roots) {
    if (sys.device_ptrs) throw InvalidArg("server requests take host arrays");
    const int o = sys.n_occ, v = sys.n_vir, X = sys.n_aux;
    if (o < 1 || v < 1 || X < 1) throw InvalidArg("n_occ, n_vir and n_aux must be positive");
    if (sys.order < 1 || sys.order > 2) throw InvalidArg("server requests are of order 1 or 2");
    if (!sys.eps || !sys.B_oo || !sys.B_ov || !sys.B_vv) throw InvalidArg("NULL input array");
    const size_t N = (size_t)o * v;
    if (n_roots < 1 || n_roots > PP_MAX_ROOTS || (size_t)n_roots > N) throw InvalidArg("n_roots out of range");
    if (!std::isfinite(omega)) throw InvalidArg("omega0 must be finite");
    check_host_system(sys);
    auto r = std::make_shared<Request>();
    r->o = o;
    r->v = v;
    r->naux = X;
    r->order = sys.order;
    r->omega = omega;
    r->n_roots = n_roots;
    r->has_dip = sys.dip != nullptr;
    plan(*r);
    if (r->bytes > budget_)
      throw OutOfBudget("request needs " + std::to_string(r->bytes) + " B of device memory; the server budget is " +
                        std::to_string(budget_) + " B");
    r->eps.assign(sys.eps, sys.eps + o + v);
    r->Boo.assign(sys.B_oo, sys.B_oo + (size_t)X * o * o);
    r->Bov.assign(sys.B_ov, sys.B_ov + (size_t)X * N);
    r->Bvv.assign(sys.B_vv, sys.B_vv + (size_t)X * v * v);
    if (sys.dip) r->dip.assign(sys.dip, sys.dip + 3 * N);
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) throw InvalidArg("server is shutting down");
    r->id = next_id_++;
    r->t_submit = Clock::now();
    if (submitted_ == 0) first_submit_ = r->t_submit;
    ++submitted_;
    reqs_[r->id] = r;
    queue_.push_back(r);
    cv_.notify_all();
    return r->id;
  }

  pp_status take(uint64_t id, pp_result* res, bool block) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) throw InvalidArg("unknown request id (already delivered?)");
    std::shared_ptr<Request> r = it->second;
    if (block)
      done_cv_.wait(lk, [&] { return r->state == Request::kDone; });
    else if (r->state != Request::kDone)
      return PP_EPENDING;
    reqs_.erase(it);
    lk.unlock();
    if (res) {
      const int n = (int)r->energies.size();
      if (res->energies && n) std::copy(r->energies.begin(), r->energies.end(), res->energies);
      if (res->vectors && !r->vectors.empty()) std::copy(r->vectors.begin(), r->vectors.end(), res->vectors);
      if (res->osc && n) {
        if (r->osc.empty())
          std::fill(res->osc, res->osc + n, 0.0);
        else
          std::copy(r->osc.begin(), r->osc.end(), res->osc);
      }
      res->n_roots = n;
      res->status = r->status;
      res->info = r->info;
      res->queued_seconds = r->t_admit > r->t_submit ? secs(r->t_submit, r->t_admit) : 0.0;
      res->run_seconds = r->t_done > r->t_admit ? secs(r->t_admit, r->t_done) : 0.0;
      res->latency_seconds = secs(r->t_submit, r->t_done);
    }
    if (r->status != PP_OK && r->status != PP_ENOTCONV) {
      std::lock_guard<std::mutex> g(err_mu_);
      err_ = r->error;
    }
    return r->status;
  }

  void stats(pp_server_stats* st) {
    long passes = 0, jobs = 0, grouped = 0;
    double flops = 0.0, seconds = 0.0;
    gb_->counters(&passes, &jobs, &flops, &seconds, &grouped);
    std::lock_guard<std::mutex> lk(mu_);
    *st = pp_server_stats{};
    st->submitted = submitted_;
    st->completed = completed_;
    st->failed = failed_;
    st->queued = (long)queue_.size();
    st->running = running_;
    st->peak_running = peak_running_;
    st->latency_p50 = percentile(latency_, 0.50);
    st->latency_p99 = percentile(latency_, 0.99);
    st->queued_p50 = percentile(queued_, 0.50);
    st->queued_p99 = percentile(queued_, 0.99);
    const double span = completed_ ? secs(first_submit_, last_done_) : 0.0;
    st->solves_per_second = span > 0 ? completed_ / span : 0.0;
    st->passes = passes;
    st->mean_requests_per_pass = passes ? (double)jobs / passes : 0.0;
    st->product_flops = flops;
    st->product_seconds = seconds;
    st->budget_bytes = budget_;
    st->reserved_bytes = reserved_;
    st->peak_reserved_bytes = peak_reserved_;
    st->grouped_launches = grouped;
  }
  void reset_stats() {
    gb_->reset();
    std::lock_guard<std::mutex> lk(mu_);
    submitted_ = completed_ = failed_ = 0;
    latency_.clear();
    queued_.clear();
    peak_running_ = running_;
    peak_reserved_ = reserved_;
  }
  std::string last_error() {
    std::lock_guard<std::mutex> g(err_mu_);
    return err_;
  }
  void set_error(const std::string& e) {
    std::lock_guard<std::mutex> g(err_mu_);
    err_ = e;
  }

 private:
  bool can_admit(const Request& r) const { return running_ < max_active_ && reserved_ + r.bytes <= budget_; }

  void scheduler() {
    (void)hipSetDevice(opt_.device);
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || (!queue_.empty() && can_admit(*queue_.front())); });
      if (stop_) return;
      std::shared_ptr<Request> r = queue_.front();
      queue_.pop_front();
      r->state = Request::kRunning;
      r->t_admit = Clock::now();
      reserved_ += r->bytes;
      ++running_;
      peak_running_ = std::max(peak_running_, running_);
      peak_reserved_ = std::max(peak_reserved_, reserved_);
      workers_.emplace_back(&Server::work, this, r);
    }
  }

  void work(std::shared_ptr<Request> r) {
    std::string err;
    Context* c = nullptr;
    bool joined = false;
    pp_status st = guarded(&err, [&] {
      PPW_HIP(hipSetDevice(opt_.device));
      SetupParams p;
      p.o = r->o;
      p.v = r->v;
      p.naux = r->naux;
      p.order = r->order;
      p.eps = r->eps.data();
      p.Boo = r->Boo.data();
      p.Bov = r->Bov.data();
      p.Bvv = r->Bvv.data();
      p.dip = r->has_dip ? r->dip.data() : nullptr;
      p.store_amplitudes = r->store ? 1 : 0;
      p.strip_rows = r->strip_rows;
      p.want_f32 = opt_.precision != PP_FP64;
      p.split_bf16 = opt_.precision == PP_SPLIT_BF16;
      p.tda = opt_.tda != 0;
      p.budget = r->bytes;
      p.device = opt_.device;
      c = setup_context(p);
      // inputs now live on the device
      std::vector<double>().swap(r->Boo);
      std::vector<double>().swap(r->Bov);
      std::vector<double>().swap(r->Bvv);
      const int k = window_block_vectors(c->N, r->n_roots, so_);
      sigma_reserve(*c, k, 0);
      if (opt_.precision != PP_FP64) sigma_reserve(*c, k, 1);
      r->energies.assign(r->n_roots, 0.0);
      r->vectors.assign((size_t)r->n_roots * 2 * c->N, 0.0);
      if (r->has_dip) r->osc.assign(r->n_roots, 0.0);
      gb_->join();
      joined = true;
      window_solve_shared(*c, so_, r->omega, r->n_roots, *gb_, (int)(r->id & 0x7fffffff), r->energies.data(),
                          r->vectors.data(), r->has_dip ? r->osc.data() : nullptr, &r->info);
    });
    if (joined) gb_->leave();
    if (c) {
      (void)hipSetDevice(opt_.device);
      delete c;
    }
    std::lock_guard<std::mutex> lk(mu_);
    r->status = st;
    r->error = err;
    r->t_done = Clock::now();
    r->state = Request::kDone;
    std::vector<double>().swap(r->eps);
    std::vector<double>().swap(r->dip);
    reserved_ -= r->bytes;
    --running_;
    if (st == PP_OK) {
      ++completed_;
      latency_.push_back(secs(r->t_submit, r->t_done));
      queued_.push_back(secs(r->t_submit, r->t_admit));
      last_done_ = r->t_done;
    } else {
      ++failed_;
    }
    cv_.notify_all();
    done_cv_.notify_all();
  }

  pp_options opt_;
  SolveOptions so_;
  size_t budget_ = 0;
  int max_active_ = 8;
  hipStream_t pass_stream_ = nullptr;
  std::unique_ptr<GroupBatcher> gb_;
  std::thread sched_;
  std::vector<std::thread> workers_;
  std::mutex mu_;
  std::condition_variable cv_, done_cv_;
  std::deque<std::shared_ptr<Request>> queue_;
  std::map<uint64_t, std::shared_ptr<Request>> reqs_;
  uint64_t next_id_ = 1;
  bool stop_ = false;
  size_t reserved_ = 0, peak_reserved_ = 0;
  int running_ = 0, peak_running_ = 0;
  long submitted_ = 0, completed_ = 0, failed_ = 0;
  std::vector<double> latency_, queued_;
  Clock::time_point first_submit_, last_done_;
  std::mutex err_mu_;
  std::string err_;
};

}  // namespace ppw

struct pp_server {
  std::unique_ptr<ppw::Server> s;
  std::string err;  // creation errors
};

namespace {
thread_local std::string g_server_error;
}

extern "C" {

pp_status pp_server_create(const pp_options* opt_in, uint64_t hbm_budget, int32_t max_active, pp_server** out) {
  if (out) *out = nullptr;
  g_server_error.clear();
  pp_server* srv = nullptr;
  pp_status st = ppw::guarded(&g_server_error, [&] {
    if (!out) throw ppw::InvalidArg("out must not be NULL");
    if (max_active < 0 || max_active > 8) throw ppw::InvalidArg("max_active must be in 0..8");
    pp_options opt;
    pp_default_options(&opt);
    if (opt_in) opt = *opt_in;
    ppw::check_options(opt);
    srv = new pp_server();
    srv->s.reset(new ppw::Server(opt, hbm_budget, max_active));
    *out = srv;
  });
  if (st != PP_OK && srv) {
    delete srv;
    if (out) *out = nullptr;
  }
  return st;
}

pp_status pp_server_submit(pp_server* srv, const pp_system* sys, double omega0, int32_t n_roots, uint64_t* req_id) {
  if (!srv || !srv->s || !sys || !req_id) return PP_EINVAL;
  std::string err;
  pp_status st = ppw::guarded(&err, [&] { *req_id = srv->s->submit(*sys, omega0, n_roots); });
  if (st != PP_OK) srv->s->set_error(err);
  return st;
}

uint64_t pp_server_request_bytes(const pp_server* srv, const pp_system* sys, int32_t n_roots) {
  if (!srv || !srv->s || !sys) return 0;
  try {
    return srv->s->request_bytes(*sys, n_roots);
  } catch (...) {
    return 0;
  }
}

pp_status pp_server_poll(pp_server* srv, uint64_t req_id, pp_result* res) {
  if (!srv || !srv->s) return PP_EINVAL;
  pp_status out = PP_OK;
  std::string err;
  pp_status st = ppw::guarded(&err, [&] { out = srv->s->take(req_id, res, false); });
  if (st != PP_OK) {
    srv->s->set_error(err);
    return st;
  }
  return out;
}

pp_status pp_server_wait(pp_server* srv, uint64_t req_id, pp_result* res) {
  if (!srv || !srv->s) return PP_EINVAL;
  pp_status out = PP_OK;
  std::string err;
  pp_status st = ppw::guarded(&err, [&] { out = srv->s->take(req_id, res, true); });
  if (st != PP_OK) {
    srv->s->set_error(err);
    return st;
  }
  return out;
}

pp_status pp_server_stats_get(pp_server* srv, pp_server_stats* st) {
  if (!srv || !srv->s || !st) return PP_EINVAL;
  std::string err;
  return ppw::guarded(&err, [&] { srv->s->stats(st); });
}

pp_status pp_server_stats_reset(pp_server* srv) {
  if (!srv || !srv->s) return PP_EINVAL;
  std::string err;
  return ppw::guarded(&err, [&] { srv->s->reset_stats(); });
}

pp_status pp_server_destroy(pp_server* srv) {
  if (!srv) return PP_OK;
  std::string err;
  pp_status st = ppw::guarded(&err, [&] { srv->s.reset(); });
  delete srv;
  return st;
}

const char* pp_server_last_error(const pp_server* srv) {
  if (!srv || !srv->s) return g_server_error.c_str();
  thread_local std::string copy;
  copy = srv->s->last_error();
  return copy.c_str();
}

}  // extern "C"
