// vh_server.hip -- persistent request loop with admission by HBM footprint.
//
// Requests (grid, medium, frequency, sources) are copied at submission and queued.
// Up to max_slots worker threads, each with its own HIP stream (default priority),
// take requests as soon as a slot is free and a contiguous region of the request's
// device footprint is free in the server's arena: requests arriving while others run
// are admitted as slots and memory free up, and their kernels overlap on the device.
// The arena is one device allocation made when the server is created; a request's
// medium, sources, solution and whole handle (hierarchy and Krylov workspaces) are
// carved out of its region, and the pinned status buffers belong to the worker, so no
// request calls hipMalloc, hipFree or the pinned-memory allocator (each of which can
// wait for the whole device and stall the other requests).  Each request runs
// vh_setup + vh_solve on its own handle, so its result does not depend on what else
// is running.  Results are held until fetched.
#include <hip/hip_runtime.h>

#include <chrono>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vh.h"
#include "vh_internal.h"

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
  size_t footprint = 0;    // bytes of the request's region
  size_t region_off = 0;   // offset of its region in the arena while it runs
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

namespace {

// First-fit allocator of byte ranges of one device allocation (host bookkeeping only,
// callers hold the server lock).  Ranges are 256-byte aligned; freed ranges coalesce.
struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(char* b, size_t n) {
    base = b;
    bytes = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t* off) {
    n = (n + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n;
      const size_t roff = it->first + n;
      free_.erase(it);
      if (rest) free_[roff] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) / 256 * 256;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct vh_server {
  Arena arena;
  double* pinned = nullptr;  // one 4 + 256 double status buffer per worker
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

constexpr size_t PINNED_DOUBLES = 4 + 256;  // per worker: one- and multi-source status

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// device bytes of one request's region: its arrays (kappa, gamma, q, u) and the handle
// (hierarchy + FGMRES workspaces at their peak, with alignment)
size_t request_footprint(const Req& r) {
  const size_t lib = vh_region_bytes(r.dim, r.n, r.levels, r.patch, r.nsrc, &r.opt);
  if (lib == 0) return 0;
  return lib + 2 * align256(r.N * sizeof(double)) + 2 * align256(r.N * (size_t)r.nsrc * 16);
}

// under the lock: pick the next admissible request (first fit, bounded overtaking)
Req* pick(vh_server* S) {
  if (S->running >= S->max_slots || S->queue.empty()) return nullptr;
  for (size_t k = 0; k < S->queue.size(); ++k) {
    Req* r = S->queue[k];
    if (S->arena.alloc(r->footprint, &r->region_off)) {
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

void run_request(Req* r, char* region, double* pinned, hipStream_t stream) {
  const size_t N = r->N;
  vh_handle* hd = nullptr;
  vh_status st = VH_OK;
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    st = VH_EDEVICE;
    r->error = std::string(what) + ": " + hipGetErrorString(e);
    return false;
  };
  const size_t qb = N * (size_t)r->nsrc * 16;
  // region layout: kappa | gamma | q | u | handle
  char* p = region;
  double* dk = (double*)p;
  p += align256(N * sizeof(double));
  double* dg = r->gamma.empty() ? nullptr : (double*)p;
  p += align256(N * sizeof(double));
  void* dq = p;
  p += align256(qb);
  void* du = p;
  p += align256(qb);
  const size_t hbytes = r->footprint - (size_t)(p - region);
  if (hip_ok(hipMemcpyAsync(dk, r->kappa.data(), N * sizeof(double), hipMemcpyHostToDevice, stream),
             "copy") &&
      (r->gamma.empty() ||
       hip_ok(hipMemcpyAsync(dg, r->gamma.data(), N * sizeof(double), hipMemcpyHostToDevice, stream),
              "copy")) &&
      hip_ok(hipMemcpyAsync(dq, r->q.data(), qb, hipMemcpyHostToDevice, stream), "copy")) {
    vh_options o = r->opt;
    o.stream = stream;
    st = vh_setup_region(&hd, r->dim, r->n, r->h, r->omega, dk, dg, r->shift, r->levels,
                         r->patch, &o, p, hbytes, pinned);
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
      vh_destroy(hd);  // a region handle returns nothing to the device allocator
    }
  }
  (void)hipStreamSynchronize(stream);
  r->status = st;
}

void worker(vh_server* S, int slot) {
  (void)hipSetDevice(S->device);
  double* pinned = S->pinned + (size_t)slot * PINNED_DOUBLES;
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
    char* region = S->arena.base + r->region_off;
    lk.unlock();
    run_request(r, region, pinned, stream);
    lk.lock();
    r->t_done = clk::now();
    r->state = DONE;
    r->kappa.clear();
    r->kappa.shrink_to_fit();
    r->gamma.clear();
    r->gamma.shrink_to_fit();
    r->q.clear();
    r->q.shrink_to_fit();
    S->arena.release(r->region_off, r->footprint);
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
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, hbm_budget);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return serr(VH_ENOMEM, std::string("the server arena of the HBM budget: ") + hipGetErrorString(e));
  }
  e = hipHostMalloc((void**)&S->pinned, (size_t)max_slots * PINNED_DOUBLES * sizeof(double),
                    hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(base);
    delete S;
    return serr(VH_ENOMEM, std::string("pinned status buffers: ") + hipGetErrorString(e));
  }
  S->arena.init((char*)base, hbm_budget);
  for (int k = 0; k < max_slots; ++k) S->workers.emplace_back(worker, S, k);
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
  if (S->arena.base) (void)hipFree(S->arena.base);
  if (S->pinned) (void)hipHostFree(S->pinned);
  delete S;
  return VH_OK;
}

}  // extern "C"
