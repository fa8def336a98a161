// serve.hip -- continuous-batching request server (C-ABI in otkm.h).
//
// Requests (n source and n target grid points) queue on the host.  A server
// thread admits them in arrival order while a request slot is free and the
// device bytes of the admitted ones stay within the budget: it reserves the
// request's region in the device arena (its cost matrix and the matrix's
// transpose), copies its points into the slot's pinned, device-mapped host
// buffer, writes the queue entry and raises the queue's tail.  One persistent kernel (serve_kernel.hip) serves
// every size: its workgroups take entries while the host keeps appending,
// build each request's matrix on the device from its points, solve it and
// write plan, duals and cost straight into mapped host memory before
// releasing the request's completion flag, so a request completes as soon as
// its own solve does and joins the running kernel as soon as a workgroup is
// free.  The kernel ends on its own when it stays idle (or when the host,
// with nothing outstanding, raises the quit word); the server thread starts
// it again when entries are waiting and no launch is running.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "launch.hpp"
#include "otkm.h"
#include "runtime.hpp"

using namespace otkm;

namespace {

// Empty-queue polls (about 2 us each) before an idle workgroup leaves: long
// enough that the kernel keeps its width through the gaps of a request
// stream, short enough that a lost host ends it soon.
constexpr int kLinger = 25000;
// The launch holds this many times the workgroups that fit at once: one that
// leaves while others still solve is replaced from the next set, so the
// kernel keeps its width after a quiet spell.
constexpr int kGenerations = 4;
// With nothing outstanding for this long, the host asks the kernel to end.
constexpr double kIdleQuitSeconds = 0.002;

// device bytes of an admitted request: its cost matrix and the matrix's
// transpose (8 n^2), and its share of the per-slot vectors
int64_t request_bytes(int n) { return 8ll * n * n + 64ll * n; }

struct Req {
  uint64_t id = 0;
  int32_t n = 0, slot = -1, status = 0;
  int32_t pos = -1;       // queue position (the completion tag is pos + 1)
  int64_t launch = -1;    // the launch that was running when the request was published, or -1
  int64_t off = -1, abytes = 0, bytes = 0, cost = 0;  // arena offset and size of C; admitted bytes
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool done = false;
  std::vector<int32_t> pts;  // src (2n) then dst (2n)
  std::vector<int32_t> plan;
  std::vector<int64_t> u, v;
};

}  // namespace

struct ot_server {
  ot_serve_cfg cfg{};
  int maxn = OT_MAX_N, slots = 256, cus = 1, dev = 0, qcap = 512, grid = 1;
  char *arena_base = nullptr;
  std::unique_ptr<otkm::Arena> arena;
  hipStream_t ks = nullptr;  // the serving kernel's stream
  hipEvent_t kev = nullptr;  // the running launch's completion
  bool running = false;
  int64_t launches = 0;
  int32_t epoch = 0;         // of the latest launch
  int32_t quit_sent = 0;     // the latest epoch asked to end
  int32_t published = 0;     // queue positions handed out
  // mapped host memory (the kernel reads and writes it over PCIe)
  int32_t *h_tail = nullptr, *h_quit = nullptr;  // [1], [1]
  int32_t *h_desc = nullptr;                     // [qcap][4]
  int32_t *h_pts = nullptr;                      // [slots][4 maxn]
  int32_t *h_plan = nullptr;                     // [slots][maxn]
  int64_t *h_u = nullptr, *h_v = nullptr;        // [slots][maxn]
  int64_t *h_cost = nullptr;                     // [slots]
  int32_t *h_done = nullptr;                     // [slots]
  ot_stats *h_stats = nullptr;                   // [slots]
  // device memory
  int32_t *d_ctl = nullptr;  // head, tail mirror, quit mirror, pad, then the poll time (u64)
  int32_t *d_ws = nullptr;   // grid * ws_ints(maxn)
  std::vector<int> free_slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<Req *> running_reqs;  // published requests not yet complete
  uint64_t next_id = 1;
  int64_t inflight_bytes = 0;
  int inflight = 0;
  double last_busy = 0;
  bool stop = false;
  int fatal = 0;
  ot_serve_counters ctr{};
  std::chrono::steady_clock::time_point t0;
  std::thread worker;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void free_server(ot_server *s) {
  if (s->ks) hipStreamSynchronize(s->ks);
  if (s->kev) hipEventDestroy(s->kev);
  if (s->ks) hipStreamDestroy(s->ks);
  hipFree(s->arena_base);
  hipFree(s->d_ctl);
  hipFree(s->d_ws);
  for (void *p : {(void *)s->h_tail, (void *)s->h_quit, (void *)s->h_desc, (void *)s->h_pts, (void *)s->h_plan,
                  (void *)s->h_u, (void *)s->h_v, (void *)s->h_cost, (void *)s->h_done, (void *)s->h_stats})
    if (p) hipHostFree(p);
  delete s;
}

template <typename T>
T *dptr(T *host) {  // device address of mapped host memory
  void *d = nullptr;
  if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) return nullptr;
  return (T *)d;
}

// A stream on its own hardware queue: a stream created with a CU mask always
// gets one (streams beyond the runtime's queue limit otherwise share queues,
// and work on a shared queue runs in submission order across its streams,
// so a long-running kernel would hold up whatever was queued behind it).
// The mask names every CU.
hipError_t dedicated_stream(hipStream_t *st, int cus) {
  std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0xffffffffu);
  if (cus % 32) mask.back() = (1u << (cus % 32)) - 1;
  return hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data());
}

// Start the kernel.  The device head persists across launches (every entry a
// launch took, it finished), so a launch continues at the first entry not yet
// taken.  Requires s->mu.
int launch(ot_server *s) {
  ServeArgs A;
  A.h_tail = dptr(s->h_tail);
  A.h_quit = dptr(s->h_quit);
  A.desc = dptr(s->h_desc);
  A.pts = dptr(s->h_pts);
  A.head = s->d_ctl;
  A.tail = s->d_ctl + 1;
  A.quit = s->d_ctl + 2;
  A.polled = (uint64_t *)(s->d_ctl + 4);
  A.qcap = s->qcap;
  A.slots = s->slots;
  A.max_n = s->maxn;
  A.epoch = s->epoch + 1;
  A.linger = kLinger;
  A.C = (int32_t *)s->arena_base;
  A.plan = dptr(s->h_plan);
  A.cost = dptr(s->h_cost);
  A.u = dptr(s->h_u);
  A.v = dptr(s->h_v);
  A.stats = dptr(s->h_stats);
  A.done = dptr(s->h_done);
  A.ws = s->d_ws;
  if (!A.h_tail || !A.h_quit || !A.desc || !A.pts || !A.plan || !A.cost || !A.u || !A.v || !A.stats || !A.done)
    return OT_EDEVICE;
  hipError_t e;
  if ((e = launch_serve(A, s->grid, s->ks)) != hipSuccess) return map_hip(e);
  if ((e = hipEventRecord(s->kev, s->ks)) != hipSuccess) return map_hip(e);
  s->epoch = A.epoch;
  s->running = true;
  ++s->launches;
  ++s->ctr.groups;
  return OT_OK;
}

// Retire finished requests and a finished launch.  Returns true when anything
// changed.  Requires s->mu.
bool retire(ot_server *s) {
  bool changed = false;
  const size_t M = (size_t)s->maxn;
  for (size_t i = 0; i < s->running_reqs.size();) {
    Req *r = s->running_reqs[i];
    const int32_t flag = __atomic_load_n(&s->h_done[r->slot], __ATOMIC_ACQUIRE);
    if (flag != r->pos + 1) { ++i; continue; }
    const ot_stats st = s->h_stats[r->slot];
    r->status = (int32_t)st.status;
    r->cost = s->h_cost[r->slot];
    if (r->status == 0) {
      r->plan.assign(s->h_plan + (size_t)r->slot * M, s->h_plan + (size_t)r->slot * M + r->n);
      r->u.assign(s->h_u + (size_t)r->slot * M, s->h_u + (size_t)r->slot * M + r->n);
      r->v.assign(s->h_v + (size_t)r->slot * M, s->h_v + (size_t)r->slot * M + r->n);
    }
    // published while the kernel ran, and completed by that same launch
    if (r->launch >= 0 && r->launch == s->launches && s->running) ++s->ctr.joined;
    r->t_done = s->now();
    r->done = true;
    s->arena->release(r->off, r->abytes);
    s->free_slots.push_back(r->slot);
    s->inflight_bytes -= r->bytes;
    --s->inflight;
    ++s->ctr.completed;
    s->running_reqs[i] = s->running_reqs.back();
    s->running_reqs.pop_back();
    s->last_busy = s->now();
    changed = true;
  }
  if (s->running) {
    const hipError_t q = hipEventQuery(s->kev);
    if (q == hipSuccess) {
      s->running = false;
      changed = true;
    } else if (q != hipErrorNotReady) {
      // the kernel failed: its flags will never arrive, so every waiter is
      // woken with the error instead of waiting forever
      if (s->fatal == 0) s->fatal = map_hip(q);
      changed = true;
    }
  }
  return changed;
}

// Admit queued requests (arrival order, within the budget and the slots) and
// publish them.  Requires s->mu.
bool admit(ot_server *s) {
  bool any = false;
  const size_t M = (size_t)s->maxn;
  int scanned = 0;
  for (auto it = s->pending.begin(); it != s->pending.end() && scanned < 4096; ++scanned) {
    Req *r = *it;
    if (s->free_slots.empty() || s->inflight >= s->cfg.max_inflight) break;
    if (s->inflight_bytes + r->bytes > s->cfg.hbm_budget_bytes) { ++it; continue; }
    const int64_t abytes = 8ll * r->n * r->n;  // C, then its transpose
    const int64_t off = s->arena->alloc(abytes);
    if (off < 0) { ++it; continue; }
    r->off = off;
    r->abytes = abytes;
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    r->t_admit = s->now();
    s->inflight_bytes += r->bytes;
    ++s->inflight;
    s->ctr.peak_inflight_bytes = std::max(s->ctr.peak_inflight_bytes, s->inflight_bytes);
    s->ctr.peak_inflight = std::max<int64_t>(s->ctr.peak_inflight, s->inflight);
    ++s->ctr.admitted;
    std::memcpy(s->h_pts + (size_t)r->slot * 4 * M, r->pts.data(), sizeof(int32_t) * 4 * (size_t)r->n);
    r->pos = s->published++;
    int32_t *e = s->h_desc + 4 * (size_t)(r->pos % s->qcap);
    const uint64_t coff = (uint64_t)(off / 4);
    e[0] = r->slot;
    e[1] = r->n;
    e[2] = (int32_t)(uint32_t)coff;
    e[3] = (int32_t)(uint32_t)(coff >> 32);
    r->launch = s->running ? s->launches : -1;
    s->running_reqs.push_back(r);
    it = s->pending.erase(it);
    any = true;
  }
  if (any) {
    // entries and points are written before the tail that covers them
    __atomic_store_n(s->h_tail, s->published, __ATOMIC_RELEASE);
    s->last_busy = s->now();
  }
  return any;
}

// Start the kernel when entries wait and no launch runs; ask a running launch
// to end when nothing has been outstanding for a while.  Requires s->mu.
bool schedule(ot_server *s) {
  if (!s->running) {
    if (s->running_reqs.empty()) return false;
    // no launch runs, so every flag is final: any entry without its flag waits
    bool waiting = false;
    for (const Req *r : s->running_reqs)
      if (__atomic_load_n(&s->h_done[r->slot], __ATOMIC_ACQUIRE) != r->pos + 1) { waiting = true; break; }
    if (!waiting) return false;
    const int rc = launch(s);
    if (rc != OT_OK) s->fatal = rc;
    return true;
  }
  if (s->quit_sent < s->epoch && s->running_reqs.empty() && s->pending.empty() &&
      s->now() - s->last_busy > kIdleQuitSeconds) {
    __atomic_store_n(s->h_quit, s->epoch, __ATOMIC_RELEASE);
    s->quit_sent = s->epoch;
    return true;
  }
  return false;
}

void worker_main(ot_server *s) {
  hipSetDevice(s->dev);  // the device that was current at ot_serve_open
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->fatal) break;
    bool progressed = retire(s);
    if (progressed) s->cv_done.notify_all();
    progressed = admit(s) || progressed;
    progressed = schedule(s) || progressed;
    if (s->stop && s->pending.empty() && s->running_reqs.empty()) {
      if (!s->running) break;
      if (s->quit_sent < s->epoch) {
        __atomic_store_n(s->h_quit, s->epoch, __ATOMIC_RELEASE);
        s->quit_sent = s->epoch;
      }
    }
    if (!progressed) {
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    } else {
      // let submit, poll and stats in between busy passes: the mutex is not fair
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
  s->cv_done.notify_all();
}

}  // namespace

extern "C" {

int ot_grid_cost_dev(const int32_t *dsrc, const int32_t *ddst, int32_t n, int32_t *dC, void *stream) {
  if (!dsrc || !ddst || !dC || n <= 0) return OT_EINVAL;
  if (n > 65535) return OT_ETOOBIG;
  {
    std::lock_guard<std::mutex> lk(lib_mutex());
    int rc = init_locked();
    if (rc) return rc;
  }
  hipStream_t st = stream ? (hipStream_t)stream : lib_stream();
  return map_hip(launch_grid_cost(dsrc, ddst, n, dC, st));
}

int ot_serve_open(ot_server **out, const ot_serve_cfg *cfg_in) {
  if (!out) return OT_EINVAL;
  ot_serve_cfg cfg{};
  if (cfg_in) cfg = *cfg_in;
  for (int k = 0; k < 5; ++k)
    if (cfg.reserved[k] != 0) return OT_EINVAL;
  if (cfg.hbm_budget_bytes < 0 || cfg.max_inflight < 0 || cfg.max_inflight > 1024 || cfg.streams < 0 ||
      cfg.streams > 8 || cfg.max_n < 0 || cfg.max_n > OT_MAX_N)
    return OT_EINVAL;
  if (cfg.hbm_budget_bytes == 0) cfg.hbm_budget_bytes = 8ll << 30;
  if (cfg.max_inflight == 0) cfg.max_inflight = 256;
  if (cfg.max_n == 0) cfg.max_n = OT_MAX_N;
  if (request_bytes(cfg.max_n) > cfg.hbm_budget_bytes) return OT_ETOOBIG;
  {
    std::lock_guard<std::mutex> lk(lib_mutex());
    int rc = init_locked();
    if (rc) return rc;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return OT_ENODEV;
  auto *s = new ot_server();
  s->dev = dev;
  s->cfg = cfg;
  s->maxn = cfg.max_n;
  s->slots = cfg.max_inflight;
  // more queue entries than slots: entry p's descriptor is rewritten (as
  // entry p + qcap) only after entry p completed
  s->qcap = 2 * s->slots;
  s->cus = device_cus();
  s->t0 = std::chrono::steady_clock::now();
  const size_t M = (size_t)s->maxn, SL = (size_t)s->slots;
  const int occ = serve_occupancy(s->maxn);
  s->grid = std::max(1, std::min(s->slots, occ * s->cus)) * kGenerations;
  hipError_t e = occ > 0 ? hipSuccess : hipErrorInvalidValue;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
  chk(hipMalloc(&s->arena_base, (size_t)cfg.hbm_budget_bytes));
  chk(hipMalloc(&s->d_ctl, 256));
  chk(hipMalloc(&s->d_ws, 4 * ws_ints(s->maxn) * (size_t)s->grid));
  chk(hipHostMalloc(&s->h_tail, 64, mapped));
  chk(hipHostMalloc(&s->h_quit, 64, mapped));
  chk(hipHostMalloc(&s->h_desc, 16 * (size_t)s->qcap, mapped));
  chk(hipHostMalloc(&s->h_pts, 4 * 4 * M * SL, mapped));
  chk(hipHostMalloc(&s->h_plan, 4 * M * SL, mapped));
  chk(hipHostMalloc(&s->h_u, 8 * M * SL, mapped));
  chk(hipHostMalloc(&s->h_v, 8 * M * SL, mapped));
  chk(hipHostMalloc(&s->h_cost, 8 * SL, mapped));
  chk(hipHostMalloc(&s->h_done, 4 * SL, mapped));
  chk(hipHostMalloc(&s->h_stats, sizeof(ot_stats) * SL, mapped));
  chk(dedicated_stream(&s->ks, s->cus));
  chk(hipEventCreateWithFlags(&s->kev, hipEventDisableTiming));
  if (e == hipSuccess) chk(hipMemsetAsync(s->d_ctl, 0, 256, s->ks));
  if (e == hipSuccess) chk(hipStreamSynchronize(s->ks));
  if (e != hipSuccess) {
    const int rc = map_hip(e);
    free_server(s);
    return rc;
  }
  *s->h_tail = 0;
  *s->h_quit = 0;
  std::memset(s->h_done, 0, 4 * SL);
  s->arena.reset(new otkm::Arena(cfg.hbm_budget_bytes));
  for (int k = s->slots - 1; k >= 0; --k) s->free_slots.push_back(k);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return OT_OK;
}

int ot_serve_submit(ot_server *s, const int32_t *src, const int32_t *dst, int32_t n, uint64_t *req_id) {
  if (!s || !src || !dst || !req_id || n <= 0) return OT_EINVAL;
  if (n > s->maxn) return OT_ETOOBIG;
  std::unique_ptr<Req> r(new Req());
  r->n = n;
  r->bytes = request_bytes(n);
  r->pts.resize(4 * (size_t)n);
  std::memcpy(r->pts.data(), src, 8 * (size_t)n);
  std::memcpy(r->pts.data() + 2 * (size_t)n, dst, 8 * (size_t)n);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return OT_EINVAL;
    if (s->fatal) return s->fatal;
    r->id = s->next_id++;
    r->t_submit = s->now();
    *req_id = r->id;
    s->pending.push_back(r.get());
    s->reqs.emplace(r->id, std::move(r));
    ++s->ctr.submitted;
  }
  s->cv_work.notify_one();
  return OT_OK;
}

int ot_serve_poll(ot_server *s, uint64_t req_id, ot_result *out, int32_t timeout_us) {
  if (!s || !out) return OT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return OT_EINVAL;
  Req *r = it->second.get();
  auto ready = [&] { return r->done || s->fatal != 0; };
  if (timeout_us < 0) s->cv_done.wait(lk, ready);
  else s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  if (!r->done) return s->fatal ? s->fatal : 1;
  out->cost = r->cost;
  out->status = r->status;
  out->n = r->n;
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  if (r->status == 0) {
    if (out->plan) std::memcpy(out->plan, r->plan.data(), 4 * (size_t)r->n);
    if (out->u) std::memcpy(out->u, r->u.data(), 8 * (size_t)r->n);
    if (out->v) std::memcpy(out->v, r->v.data(), 8 * (size_t)r->n);
  }
  s->reqs.erase(it);
  return OT_OK;
}

int ot_serve_stats(ot_server *s, ot_serve_counters *out, double *now) {
  if (!s) return OT_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (out) *out = s->ctr;
  if (now) *now = s->now();
  return s->fatal;
}

int ot_serve_close(ot_server *s) {
  if (!s) return OT_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  const int rc = s->fatal;
  free_server(s);
  return rc;
}

}  // extern "C"
