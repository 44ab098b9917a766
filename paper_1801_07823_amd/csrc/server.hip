// Solver service: a stream of solve requests over device-resident
// configurations, continuously batched.
//
// Each registered configuration is a hierarchy built once (null vectors and
// prolongators, Sec. 4 setup).  A request names a configuration, a mass and a
// device rhs.  Worker threads, each with its own HIP stream, take requests in
// arrival order as soon as a worker is free and the request's device
// footprint fits the memory budget, so requests that arrive while others run
// join the device immediately and their kernels overlap.  A request runs on a
// pooled per-shape hierarchy moved onto its configuration and mass with
// kdmg_hierarchy_set_mass (coarse operators re-Galerkined at the request's
// mass, no allocation), or on a new one from kdmg_hierarchy_at_mass when no
// pooled one is idle; idle pooled hierarchies of other shapes are released
// when memory is needed.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "api_guard.h"
#include "internal.h"

using namespace kdmg;

namespace {

using Clock = std::chrono::steady_clock;

// what makes two requests able to share a pooled hierarchy
struct ShapeKey {
  std::vector<long> v;
  bool operator<(const ShapeKey& o) const { return v < o.v; }
};

ShapeKey shape_of(const kdmg_hierarchy& h, int nrhs, kdmg_prec prec) {
  ShapeKey k;
  for (int mu = 0; mu < 4; ++mu) k.v.push_back(h.lat->dims[mu]);
  k.v.push_back(h.lat->nd);
  k.v.push_back(h.lat->nc);
  k.v.push_back(h.nlevels);
  for (int l = 0; l < h.nlevels - 1; ++l) {
    for (int mu = 0; mu < 4; ++mu) k.v.push_back(h.params.lvl[l].agg[mu]);
    k.v.push_back(h.params.lvl[l].nvec);
  }
  k.v.push_back(nrhs);
  k.v.push_back((long)prec);
  return k;
}

struct Request {
  long long id = 0;
  int cfg = 0;
  double mass = 0.0;
  const void* b = nullptr;
  void* x = nullptr;
  int nrhs = 1;
  double tol = 1e-10;
  kdmg_prec prec = KDMG_MIXED;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  ShapeKey key;
  size_t bytes = 0;
  Clock::time_point t_sub, t_start, t_end;
  bool done = false;
  kdmg_status status = KDMG_OK;
  std::string err;
  std::vector<kdmg_solve_info> info;
};

struct Pooled {
  kdmg_hierarchy* h = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct kdmg_server {
  int device = 0;
  size_t budget = 0;
  std::vector<const kdmg_hierarchy*> cfgs;
  std::deque<Request*> queue;
  std::map<long long, std::unique_ptr<Request>> reqs;
  std::multimap<ShapeKey, Pooled> idle;
  size_t allocated = 0, peak_allocated = 0;  // in use + pooled idle
  int running = 0, peak_running = 0;
  long long completed = 0, next_id = 1;
  bool stop = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::vector<std::unique_ptr<std::mutex>> tune_mu;  // per configuration
};

namespace {

// Under s.mu: take the queue head if it can run now.  On success `slot` holds
// a pooled hierarchy (reuse) or is empty with the head's bytes reserved; idle
// hierarchies released to make room are appended to `evict`.
bool try_admit(kdmg_server& s, Request*& r, Pooled& slot, std::vector<kdmg_hierarchy*>& evict) {
  if (s.queue.empty()) return false;
  Request* q = s.queue.front();
  auto it = s.idle.find(q->key);
  if (it != s.idle.end()) {
    slot = it->second;
    s.idle.erase(it);
  } else {
    while (s.allocated + q->bytes > s.budget && !s.idle.empty()) {
      auto v = s.idle.begin();
      s.allocated -= v->second.bytes;
      evict.push_back(v->second.h);
      s.idle.erase(v);
    }
    if (s.allocated + q->bytes > s.budget) return false;
    s.allocated += q->bytes;
    s.peak_allocated = std::max(s.peak_allocated, s.allocated);
    slot = Pooled{nullptr, q->bytes};
  }
  s.queue.pop_front();
  r = q;
  return true;
}

std::string last_error_copy() {
  const char* e = kdmg_last_error();
  return e ? std::string(e) : std::string();
}

// Runs one request on the worker's stream; returns the hierarchy it used
// (to be pooled) or null if none survived.
kdmg_hierarchy* run_request(kdmg_server& s, Request& r, Pooled slot, hipStream_t st) {
  const kdmg_hierarchy* base = s.cfgs[r.cfg];
  kdmg_status rc = KDMG_OK;
  {
    // tune the configuration's launch shapes once per (nrhs, prec), so every
    // hierarchy derived from it uses the same shapes
    std::lock_guard<std::mutex> g(*s.tune_mu[r.cfg]);
    if (autotune_enabled())
      rc = kdmg_hierarchy_autotune(const_cast<kdmg_hierarchy*>(base), r.nrhs, r.prec, st);
  }
  kdmg_hierarchy* h = slot.h;
  // the caller's work on b and x that was queued before the submit comes first
  if (rc == KDMG_OK && hipStreamWaitEvent(st, r.ready, 0) != hipSuccess) {
    rc = KDMG_EHIP;
    set_last_error("kdmg_server: hipStreamWaitEvent on the submit event failed");
  }
  if (rc == KDMG_OK) {
    if (h) rc = kdmg_hierarchy_set_mass(h, base, r.mass, st);
    else rc = kdmg_hierarchy_at_mass(base, r.mass, st, &h);
  }
  // Served solves launch plainly, without graph capture: a request rebinds
  // its hierarchy (new mass, often a new configuration), which would recapture
  // every graph anyway, and a capture in one worker overlapping another
  // worker's first-use calls (the autotuner's timing launches, allocations)
  // gave HIP errors on the first requests of a configuration.
  if (rc == KDMG_OK && h) h->use_graphs = false;
  if (rc == KDMG_OK) rc = kdmg_solve(h, r.b, r.x, r.nrhs, r.tol, r.prec, r.info.data(), st);
  r.status = rc;
  if (rc != KDMG_OK) r.err = last_error_copy();
  if (rc != KDMG_OK && rc != KDMG_ENOCONV && h) {
    kdmg_hierarchy_destroy(h);  // do not pool a hierarchy in an unknown state
    h = nullptr;
  }
  return h;
}

void worker_main(kdmg_server* sp, int w) {
  kdmg_server& s = *sp;
  (void)hipSetDevice(s.device);
  hipStream_t st = s.streams[w];
  std::unique_lock<std::mutex> lk(s.mu);
  for (;;) {
    Request* r = nullptr;
    Pooled slot;
    std::vector<kdmg_hierarchy*> evict;
    while (!s.stop && !try_admit(s, r, slot, evict)) s.cv_work.wait(lk);
    if (!r) break;  // stopping
    ++s.running;
    s.peak_running = std::max(s.peak_running, s.running);
    r->t_start = Clock::now();
    lk.unlock();
    for (kdmg_hierarchy* e : evict) kdmg_hierarchy_destroy(e);
    kdmg_hierarchy* h = run_request(s, *r, slot, st);
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
    lk.lock();
    r->t_end = Clock::now();
    if (h) s.idle.emplace(r->key, Pooled{h, slot.bytes});
    else s.allocated -= slot.bytes;
    r->done = true;
    --s.running;
    ++s.completed;
    s.cv_done.notify_all();
    s.cv_work.notify_all();
  }
}

double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

}  // namespace

extern "C" kdmg_status kdmg_server_create(int slots, size_t hbm_budget, kdmg_server** out) {
  KDMG_API_BEGIN
  KDMG_CHECK(out && slots >= 1 && slots <= 64 && hbm_budget > 0, KDMG_EINVAL,
             "kdmg_server_create: slots must be 1..64 and the budget positive");
  *out = nullptr;
  auto s = std::make_unique<kdmg_server>();
  KDMG_HIP(hipGetDevice(&s->device));
  s->budget = hbm_budget;
  for (int w = 0; w < slots; ++w) {
    hipStream_t st = nullptr;
    KDMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    s->streams.push_back(st);
  }
  for (int w = 0; w < slots; ++w) s->workers.emplace_back(worker_main, s.get(), w);
  *out = s.release();
  KDMG_API_END
}

extern "C" kdmg_status kdmg_server_add_config(kdmg_server* s, const kdmg_hierarchy* base, int* config_id) {
  KDMG_API_BEGIN
  KDMG_CHECK(s && base && config_id, KDMG_EINVAL, "kdmg_server_add_config: null argument");
  std::lock_guard<std::mutex> g(s->mu);
  s->cfgs.push_back(base);
  s->tune_mu.push_back(std::make_unique<std::mutex>());
  *config_id = (int)s->cfgs.size() - 1;
  KDMG_API_END
}

extern "C" kdmg_status kdmg_server_request_bytes(kdmg_server* s, int config_id, int nrhs, kdmg_prec prec,
                                                 size_t* bytes) {
  KDMG_API_BEGIN
  KDMG_CHECK(s && bytes && nrhs >= 1, KDMG_EINVAL, "kdmg_server_request_bytes: bad argument");
  std::lock_guard<std::mutex> g(s->mu);
  KDMG_CHECK(config_id >= 0 && config_id < (int)s->cfgs.size(), KDMG_EINVAL, "no such configuration");
  *bytes = derived_footprint(*s->cfgs[config_id], nrhs, prec);
  KDMG_API_END
}

extern "C" kdmg_status kdmg_server_submit(kdmg_server* s, int config_id, double mass, const void* b, void* x,
                                          int nrhs, double tol, kdmg_prec prec, void* stream, long long* ticket) {
  KDMG_API_BEGIN
  KDMG_CHECK(s && b && x && b != x && ticket, KDMG_EINVAL, "kdmg_server_submit: bad pointers");
  KDMG_CHECK(mass > 0.0 && nrhs >= 1 && nrhs <= 1024 && tol > 0.0 && tol < 1.0, KDMG_EINVAL,
             "kdmg_server_submit: bad mass, nrhs or tol");
  KDMG_CHECK(prec == KDMG_FP64 || prec == KDMG_MIXED, KDMG_EINVAL, "kdmg_server_submit: bad precision");
  auto r = std::make_unique<Request>();
  std::lock_guard<std::mutex> g(s->mu);
  KDMG_CHECK(!s->stop, KDMG_EBUSY, "server is shutting down");
  KDMG_CHECK(config_id >= 0 && config_id < (int)s->cfgs.size(), KDMG_EINVAL, "no such configuration");
  const kdmg_hierarchy& base = *s->cfgs[config_id];
  r->id = s->next_id++;
  r->cfg = config_id;
  r->mass = mass;
  r->b = b;
  r->x = x;
  r->nrhs = nrhs;
  r->tol = tol;
  r->prec = prec;
  r->key = shape_of(base, nrhs, prec);
  r->bytes = derived_footprint(base, nrhs, prec);
  KDMG_CHECK(r->bytes <= s->budget, KDMG_ENOMEM, "request needs more device memory than the server budget");
  r->info.resize(nrhs);
  KDMG_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
  if (hipEventRecord(r->ready, (hipStream_t)stream) != hipSuccess) {
    (void)hipEventDestroy(r->ready);
    throw Error(KDMG_EHIP, "kdmg_server_submit: hipEventRecord on the caller's stream failed");
  }
  r->t_sub = Clock::now();
  *ticket = r->id;
  s->queue.push_back(r.get());
  s->reqs.emplace(r->id, std::move(r));
  s->cv_work.notify_one();
  KDMG_API_END
}

extern "C" kdmg_status kdmg_server_poll(kdmg_server* s, long long ticket, int wait, int* done,
                                        kdmg_status* solve_status, kdmg_solve_info* info, double* times) {
  KDMG_API_BEGIN
  KDMG_CHECK(s && done, KDMG_EINVAL, "kdmg_server_poll: null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  KDMG_CHECK(it != s->reqs.end(), KDMG_EINVAL, "kdmg_server_poll: unknown ticket (or already collected)");
  Request* r = it->second.get();
  if (wait) s->cv_done.wait(lk, [&] { return r->done; });
  *done = r->done ? 1 : 0;
  if (!r->done) return KDMG_OK;
  if (solve_status) *solve_status = r->status;
  if (info)
    for (int i = 0; i < r->nrhs; ++i) info[i] = r->info[i];
  if (times) {
    times[0] = secs(r->t_sub, r->t_start);
    times[1] = secs(r->t_start, r->t_end);
    times[2] = secs(r->t_sub, r->t_end);
  }
  if (r->status != KDMG_OK && r->status != KDMG_ENOCONV) set_last_error(r->err);
  s->reqs.erase(it);
  KDMG_API_END
}

extern "C" kdmg_status kdmg_server_stats(kdmg_server* s, long long* completed, int* running, int* peak_running,
                                         size_t* allocated, size_t* peak_allocated) {
  KDMG_API_BEGIN
  KDMG_CHECK(s, KDMG_EINVAL, "kdmg_server_stats: null server");
  std::lock_guard<std::mutex> g(s->mu);
  if (completed) *completed = s->completed;
  if (running) *running = s->running;
  if (peak_running) *peak_running = s->peak_running;
  if (allocated) *allocated = s->allocated;
  if (peak_allocated) *peak_allocated = s->peak_allocated;
  KDMG_API_END
}

extern "C" void kdmg_server_destroy(kdmg_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // finish what was admitted; requests still queued are dropped
    for (Request* q : s->queue) {
      if (q->ready) (void)hipEventDestroy(q->ready);
      q->ready = nullptr;
      q->done = true;
      q->status = KDMG_EBUSY;
      q->err = "server destroyed before the request started";
    }
    s->queue.clear();
    s->stop = true;
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->idle) kdmg_hierarchy_destroy(kv.second.h);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}
