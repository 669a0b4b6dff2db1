// vh_server.hip -- persistent request loop with admission by HBM footprint.
//
// Requests (grid, medium, frequency, sources) are copied at submission and queued.
// Up to max_slots worker threads, each with its own HIP stream (default priority),
// take requests as soon as a slot is free and the request's device footprint fits in
// the remaining budget: requests arriving while others run are admitted as slots and
// memory free up, and their kernels overlap on the device.  Each request runs
// vh_setup + vh_solve on its own handle, so its result does not depend on what else
// is running.  Results are held until fetched.
#include <hip/hip_runtime.h>

#include <chrono>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vh.h"

namespace {

using clk = std::chrono::steady_clock;

enum ReqState { QUEUED = 0, RUNNING = 1, DONE = 2 };

struct Req {
  uint64_t ticket = 0;
  int dim = 2, n[3] = {1, 1, 1}, levels = 1, patch = 0, nsrc = 1;
  double h = 0, omega = 0, shift = 0, tol = 1e-6;
  vh_options opt{};
  std::vector<double> kappa, gamma;
  std::vector<std::complex<double>> q, u;
  std::vector<vh_solve_stats> stats;
  size_t footprint = 0;
  size_t N = 0;
  vh_status status = VH_OK;
  std::string error;
  ReqState state = QUEUED;
  clk::time_point t_submit, t_start, t_done;
};

}  // namespace

void vh_internal_set_error(const std::string& msg);  // vh_runtime.hip

namespace {

vh_status serr(vh_status st, const std::string& m) {
  vh_internal_set_error(m);
  return st;
}

}  // namespace

struct vh_server {
  size_t budget = 0, in_use = 0, peak = 0;
  int max_slots = 1, running = 0, peak_running = 0, device = 0;
  uint64_t next_ticket = 1, completed = 0;
  int head_skips = 0;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  std::vector<std::thread> workers;
};

namespace {

constexpr int MAX_HEAD_SKIPS = 4;  // later requests may overtake the head this often

// device bytes of one request: the handle (hierarchy + FGMRES workspace) plus the
// caller-side arrays the worker allocates (kappa, gamma, q, u)
size_t request_footprint(const Req& r) {
  const size_t lib = vh_footprint_bytes(r.dim, r.n, r.levels, r.patch, r.nsrc, &r.opt);
  return lib + r.N * 2 * sizeof(double) + r.N * (size_t)r.nsrc * 2 * 16;
}

// under the lock: pick the next admissible request (first fit, bounded overtaking)
Req* pick(vh_server* S) {
  if (S->running >= S->max_slots || S->queue.empty()) return nullptr;
  for (size_t k = 0; k < S->queue.size(); ++k) {
    Req* r = S->queue[k];
    if (S->in_use + r->footprint <= S->budget) {
      if (k == 0)
        S->head_skips = 0;
      else
        ++S->head_skips;
      S->queue.erase(S->queue.begin() + k);
      return r;
    }
    if (k == 0 && S->head_skips >= MAX_HEAD_SKIPS) return nullptr;  // let the head drain in
  }
  return nullptr;
}

void run_request(Req* r, hipStream_t stream) {
  const size_t N = r->N;
  double *dk = nullptr, *dg = nullptr;
  void *dq = nullptr, *du = nullptr;
  vh_handle* hd = nullptr;
  vh_status st = VH_OK;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    st = (e == hipErrorOutOfMemory) ? VH_ENOMEM : VH_EDEVICE;
    r->error = std::string(what) + ": " + hipGetErrorString(e);
    return false;
  };
  const size_t qb = N * (size_t)r->nsrc * 16;
  if (hip_ok(hipMalloc((void**)&dk, N * sizeof(double)), "hipMalloc") &&
      hip_ok(hipMalloc(&dq, qb), "hipMalloc") && hip_ok(hipMalloc(&du, qb), "hipMalloc") &&
      (r->gamma.empty() || hip_ok(hipMalloc((void**)&dg, N * sizeof(double)), "hipMalloc")) &&
      hip_ok(hipMemcpyAsync(dk, r->kappa.data(), N * sizeof(double), hipMemcpyHostToDevice, stream),
             "copy") &&
      (r->gamma.empty() ||
       hip_ok(hipMemcpyAsync(dg, r->gamma.data(), N * sizeof(double), hipMemcpyHostToDevice, stream),
              "copy")) &&
      hip_ok(hipMemcpyAsync(dq, r->q.data(), qb, hipMemcpyHostToDevice, stream), "copy")) {
    vh_options o = r->opt;
    o.stream = stream;
    st = vh_setup(&hd, r->dim, r->n, r->h, r->omega, dk, dg, r->shift, r->levels, r->patch, &o);
    if (st != VH_OK) {
      r->error = vh_last_error();
    } else {
      r->stats.assign(r->nsrc, vh_solve_stats{});
      st = vh_solve(hd, dq, r->nsrc, r->tol, du, r->stats.data());
      if (st != VH_OK) r->error = vh_last_error();
      if (st == VH_OK || st == VH_ENOCONV) {
        r->u.resize(N * (size_t)r->nsrc);
        hipError_t e = hipMemcpyAsync(r->u.data(), du, qb, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
          st = VH_EDEVICE;
          r->error = hipGetErrorString(e);
        }
      }
      vh_destroy(hd);
    }
  }
  (void)hipStreamSynchronize(stream);
  if (dk) (void)hipFree(dk);
  if (dg) (void)hipFree(dg);
  if (dq) (void)hipFree(dq);
  if (du) (void)hipFree(du);
  r->status = st;
}

void worker(vh_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = nullptr;
  (void)hipStreamCreate(&stream);  // default priority
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    Req* r = nullptr;
    S->cv_work.wait(lk, [&] { return S->stop || (r = pick(S)) != nullptr; });
    if (!r) break;  // stopping
    S->in_use += r->footprint;
    S->peak = std::max(S->peak, S->in_use);
    ++S->running;
    S->peak_running = std::max(S->peak_running, S->running);
    r->state = RUNNING;
    r->t_start = clk::now();
    lk.unlock();
    run_request(r, stream);
    lk.lock();
    r->t_done = clk::now();
    r->state = DONE;
    r->kappa.clear();
    r->kappa.shrink_to_fit();
    r->gamma.clear();
    r->gamma.shrink_to_fit();
    r->q.clear();
    r->q.shrink_to_fit();
    S->in_use -= r->footprint;
    --S->running;
    ++S->completed;
    S->cv_done.notify_all();
    S->cv_work.notify_all();  // memory and a slot were freed: admit the next ones
  }
  lk.unlock();
  (void)hipStreamSynchronize(stream);
  (void)hipStreamDestroy(stream);
}

double ms_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

extern "C" {

vh_status vh_server_create(vh_server** out, size_t hbm_budget, int max_slots) {
  if (!out) return serr(VH_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 64) return serr(VH_EINVAL, "max_slots must be in [1, 64]");
  if (hbm_budget == 0) return serr(VH_EINVAL, "hbm_budget must be > 0");
  vh_server* S = new (std::nothrow) vh_server();
  if (!S) return serr(VH_ENOMEM, "host allocation failed");
  S->budget = hbm_budget;
  S->max_slots = max_slots;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return serr(VH_EDEVICE, "hipGetDevice failed");
  }
  for (int k = 0; k < max_slots; ++k) S->workers.emplace_back(worker, S);
  *out = S;
  return VH_OK;
}

vh_status vh_server_submit(vh_server* S, const vh_request* q, uint64_t* ticket) {
  if (!S || !q || !ticket) return serr(VH_EINVAL, "NULL argument");
  if ((q->dim != 2 && q->dim != 3) || q->nsrc < 1 || !q->kappa || !q->q || !(q->tol > 0))
    return serr(VH_EINVAL, "invalid request");
  Req* r = new (std::nothrow) Req();
  if (!r) return serr(VH_ENOMEM, "host allocation failed");
  r->dim = q->dim;
  r->N = 1;
  for (int d = 0; d < 3; ++d) r->n[d] = (d < q->dim) ? q->n[d] : 1;
  for (int d = 0; d < q->dim; ++d) {
    if (q->n[d] < 3) {
      delete r;
      return serr(VH_EINVAL, "every dimension needs >= 3 nodes");
    }
    r->N *= (size_t)q->n[d];
  }
  r->h = q->h;
  r->omega = q->omega;
  r->shift = q->shift;
  r->levels = q->levels;
  r->patch = q->patch;
  r->nsrc = q->nsrc;
  r->tol = q->tol;
  if (q->opt)
    r->opt = *q->opt;
  else
    vh_options_default(&r->opt);
  r->opt.stream = nullptr;
  r->kappa.assign(q->kappa, q->kappa + r->N);
  if (q->gamma) r->gamma.assign(q->gamma, q->gamma + r->N);
  const std::complex<double>* qp = static_cast<const std::complex<double>*>(q->q);
  r->q.assign(qp, qp + r->N * (size_t)r->nsrc);
  r->footprint = request_footprint(*r);
  if (r->footprint == 0) {
    delete r;
    return serr(VH_EINVAL, "invalid grid for the footprint");
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (r->footprint > S->budget) {
    delete r;
    return serr(VH_ENOMEM, "request footprint exceeds the server's HBM budget");
  }
  r->ticket = S->next_ticket++;
  r->t_submit = clk::now();
  S->reqs[r->ticket] = r;
  S->queue.push_back(r);
  *ticket = r->ticket;
  S->cv_work.notify_all();
  return VH_OK;
}

vh_status vh_server_poll(vh_server* S, uint64_t ticket, int* done) {
  if (!S || !done) return serr(VH_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return serr(VH_EINVAL, "unknown ticket");
  *done = it->second->state == DONE ? 1 : 0;
  return VH_OK;
}

vh_status vh_server_wait(vh_server* S, uint64_t ticket) {
  if (!S) return serr(VH_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return serr(VH_EINVAL, "unknown ticket");
  Req* r = it->second;
  S->cv_done.wait(lk, [&] { return r->state == DONE; });
  return VH_OK;
}

vh_status vh_server_result(vh_server* S, uint64_t ticket, void* u, vh_solve_stats* stats,
                           double* latency_ms, double* queue_ms) {
  if (!S) return serr(VH_EINVAL, "NULL argument");
  Req* r = nullptr;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return serr(VH_EINVAL, "unknown ticket");
    r = it->second;
    S->cv_done.wait(lk, [&] { return r->state == DONE; });
    S->reqs.erase(it);
  }
  if (u && !r->u.empty()) std::memcpy(u, r->u.data(), r->u.size() * sizeof(std::complex<double>));
  if (stats)
    for (int k = 0; k < r->nsrc; ++k) stats[k] = k < (int)r->stats.size() ? r->stats[k] : vh_solve_stats{};
  if (latency_ms) *latency_ms = ms_between(r->t_submit, r->t_done);
  if (queue_ms) *queue_ms = ms_between(r->t_submit, r->t_start);
  const vh_status st = r->status;
  if (st != VH_OK) vh_internal_set_error(r->error);
  delete r;
  return st;
}

vh_status vh_server_get_info(vh_server* S, vh_server_info* info) {
  if (!S || !info) return serr(VH_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  info->budget = S->budget;
  info->in_use = S->in_use;
  info->peak_in_use = S->peak;
  info->running = S->running;
  info->peak_running = S->peak_running;
  info->queued = (int)S->queue.size();
  info->completed = S->completed;
  return VH_OK;
}

vh_status vh_server_destroy(vh_server* S) {
  if (!S) return VH_OK;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // finish everything that was submitted
    S->cv_done.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
    S->stop = true;
    S->cv_work.notify_all();
  }
  for (auto& t : S->workers) t.join();
  for (auto& kv : S->reqs) delete kv.second;
  delete S;
  return VH_OK;
}

}  // extern "C"
