// serve.hip -- continuous-batching request server (C-ABI in otkm.h).
//
// Requests (n source and n target grid points) queue on the host.  A server
// thread admits them as request slots and device bytes free up, builds each
// request's cost matrix on the device from its points, and launches every
// newly admitted group as one persistent batch kernel.  Each size class has
// its own stream, so a group of large requests never holds back small ones,
// and groups launched while others run overlap on the device.  The engine
// writes each request's plan and duals straight into pinned host memory and
// then releases a per-request completion flag, so a request completes as soon
// as its own solve does, not when its whole group does.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
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

constexpr int kClasses = 4;
constexpr int kMaxLanesPerClass = 8;
// One stream per class by default: on the serving workload (Poisson 2000/s,
// n log-uniform in [32, 4096]) four streams per class halved the throughput
// (1493 -> 752 solves/s): concurrent persistent kernels of one class split the
// chip instead of draining one queue longest-first.
constexpr int kDefaultLanesPerClass = 1;
// size classes: (largest n, workgroup width)
constexpr int kClassMaxN[kClasses] = {128, 512, 2048, OT_MAX_N};
constexpr int kClassBlock[kClasses] = {64, 64, 256, 512};

int class_of(int n) {
  for (int c = 0; c < kClasses; ++c)
    if (n <= kClassMaxN[c]) return c;
  return kClasses - 1;
}

int64_t request_bytes(int n) { return 4ll * n * n + 64ll * n; }

struct Req {
  uint64_t id = 0;
  int32_t n = 0, cls = 0, slot = -1, pos = -1, status = 0;
  int64_t off = -1, abytes = 0, bytes = 0, cost = 0;  // arena offset and size of C; admitted bytes
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool done = false;
  int stream = -1;
  uint32_t tag = 0;
  std::vector<int32_t> pts;  // src (2n) then dst (2n)
  std::vector<int32_t> plan;
  std::vector<int64_t> u, v;
};

struct Lane {  // one stream; each size class has cfg.streams of them
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  uint32_t tag = 0;
  std::vector<Req *> group;  // requests admitted for the next launch (cleared once launched)
  int outstanding = 0;       // requests of the launched group not yet retired
  // descriptors of the group in flight (device and pinned staging)
  int64_t *d_coff = nullptr, *d_voff = nullptr, *h_coff = nullptr, *h_voff = nullptr;
  int32_t *d_n = nullptr, *d_order = nullptr, *h_n = nullptr, *h_order = nullptr;
  int32_t *d_head = nullptr, *d_ws = nullptr;
  // per-position results written by the device into pinned memory
  int64_t *h_cost = nullptr;
  ot_stats *h_stats = nullptr;
  int32_t *h_done = nullptr;
};

}  // namespace

struct ot_server {
  ot_serve_cfg cfg{};
  int maxn = OT_MAX_N, slots = 256, cus = 1, dev = 0;
  char *arena_base = nullptr;
  std::unique_ptr<otkm::Arena> arena;
  int32_t *d_pts = nullptr;                   // [slots][4 maxn]
  int32_t *h_pts = nullptr;                   // pinned staging [slots][4 maxn]
  int32_t *h_plan = nullptr;                  // pinned [slots][maxn]
  int64_t *h_u = nullptr, *h_v = nullptr;     // pinned [slots][maxn]
  std::vector<int> free_slots;
  Lane lanes[kClasses * kMaxLanesPerClass];  // lane c * lpc + l: class c, stream l
  int lpc = kDefaultLanesPerClass;
  int nlanes() const { return kClasses * lpc; }
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<Req *> running;
  uint64_t next_id = 1;
  int64_t inflight_bytes = 0;
  int inflight = 0;
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
  for (auto &L : s->lanes) {
    if (L.s) hipStreamSynchronize(L.s);
    if (L.ev) hipEventDestroy(L.ev);
    if (L.s) hipStreamDestroy(L.s);
    hipFree(L.d_coff); hipFree(L.d_voff); hipFree(L.d_n); hipFree(L.d_order); hipFree(L.d_head); hipFree(L.d_ws);
    hipHostFree(L.h_coff); hipHostFree(L.h_voff); hipHostFree(L.h_n); hipHostFree(L.h_order);
    hipHostFree(L.h_cost); hipHostFree(L.h_stats); hipHostFree(L.h_done);
  }
  hipFree(s->arena_base);
  hipFree(s->d_pts);
  hipHostFree(s->h_pts);
  hipHostFree(s->h_plan);
  hipHostFree(s->h_u);
  hipHostFree(s->h_v);
  delete s;
}

template <typename T>
T *dptr(T *host) {  // device address of pinned host memory
  void *d = nullptr;
  if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) return nullptr;
  return (T *)d;
}

// Launch the group collected in lane li.  Requires s->mu.
int launch_group(ot_server *s, int li) {
  Lane &L = s->lanes[li];
  const int c = li / s->lpc;
  const int G = (int)L.group.size();
  const size_t M = (size_t)s->maxn;
  hipError_t e;
  int max_n = 1;
  for (int k = 0; k < G; ++k) {
    Req *r = L.group[k];
    r->pos = k;
    r->stream = li;
    r->tag = L.tag;
    max_n = std::max(max_n, r->n);
    int32_t *hp = s->h_pts + (size_t)r->slot * 4 * M;
    std::memcpy(hp, r->pts.data(), sizeof(int32_t) * 4 * (size_t)r->n);
    int32_t *dp = s->d_pts + (size_t)r->slot * 4 * M;
    if ((e = hipMemcpyAsync(dp, hp, sizeof(int32_t) * 4 * (size_t)r->n, hipMemcpyHostToDevice, L.s)) != hipSuccess)
      return map_hip(e);
    int32_t *Cr = (int32_t *)(s->arena_base + r->off);
    if ((e = launch_grid_cost(dp, dp + 2 * r->n, r->n, Cr, L.s)) != hipSuccess) return map_hip(e);
    L.h_coff[k] = r->off / 4;
    L.h_voff[k] = (int64_t)r->slot * (int64_t)M;
    L.h_n[k] = r->n;
    L.h_order[k] = k;
    L.h_done[k] = 0;
  }
  // longest first inside the group
  std::stable_sort(L.h_order, L.h_order + G, [&](int a, int b) { return L.h_n[a] > L.h_n[b]; });
  if ((e = hipMemcpyAsync(L.d_coff, L.h_coff, 8 * (size_t)G, hipMemcpyHostToDevice, L.s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(L.d_voff, L.h_voff, 8 * (size_t)G, hipMemcpyHostToDevice, L.s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(L.d_n, L.h_n, 4 * (size_t)G, hipMemcpyHostToDevice, L.s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(L.d_order, L.h_order, 4 * (size_t)G, hipMemcpyHostToDevice, L.s)) != hipSuccess) return map_hip(e);
  if ((e = launch_fill_i32(L.d_head, 0, 1, L.s)) != hipSuccess) return map_hip(e);
  const int block = kClassBlock[c];
  const int occ = batch_occupancy(block, max_n);
  if (occ <= 0) return OT_ETOOBIG;
  const int grid = std::max(1, std::min(G, occ * s->cus));
  BatchArgs A;
  A.C = (const int32_t *)s->arena_base;
  A.coff = L.d_coff; A.n = L.d_n; A.voff = L.d_voff; A.order = L.d_order;
  A.count = G; A.nq = G; A.max_n = max_n; A.max_paths = 0;
  A.plan = dptr(s->h_plan); A.cost = dptr(L.h_cost); A.u = dptr(s->h_u); A.v = dptr(s->h_v);
  A.stats = dptr(L.h_stats); A.ws = L.d_ws; A.head = L.d_head; A.done = dptr(L.h_done); A.tag = (int32_t)L.tag;
  if (!A.plan || !A.cost || !A.u || !A.v || !A.stats || !A.done) return OT_EDEVICE;
  if ((e = launch_assign_batch(A, block, grid, L.s)) != hipSuccess) return map_hip(e);
  if ((e = hipEventRecord(L.ev, L.s)) != hipSuccess) return map_hip(e);
  L.busy = true;
  // A retired request may be handed back and freed by ot_serve_poll before this
  // lane's event completes, so the lane keeps a count, never the pointers.
  L.outstanding = G;
  L.group.clear();
  ++s->ctr.groups;
  return OT_OK;
}

// Retire finished requests; returns true when anything changed.  Requires s->mu.
bool retire(ot_server *s) {
  bool changed = false;
  const size_t M = (size_t)s->maxn;
  for (size_t i = 0; i < s->running.size();) {
    Req *r = s->running[i];
    Lane &L = s->lanes[r->stream];
    const int32_t flag = __atomic_load_n(&L.h_done[r->pos], __ATOMIC_ACQUIRE);
    if (flag != (int32_t)r->tag) { ++i; continue; }
    const ot_stats st = L.h_stats[r->pos];
    r->status = (int32_t)st.status;
    r->cost = L.h_cost[r->pos];
    if (r->status == 0) {
      r->plan.assign(s->h_plan + (size_t)r->slot * M, s->h_plan + (size_t)r->slot * M + r->n);
      r->u.assign(s->h_u + (size_t)r->slot * M, s->h_u + (size_t)r->slot * M + r->n);
      r->v.assign(s->h_v + (size_t)r->slot * M, s->h_v + (size_t)r->slot * M + r->n);
    }
    r->t_done = s->now();
    r->done = true;
    --L.outstanding;
    s->arena->release(r->off, r->abytes);
    s->free_slots.push_back(r->slot);
    s->inflight_bytes -= r->bytes;
    --s->inflight;
    ++s->ctr.completed;
    s->running[i] = s->running.back();
    s->running.pop_back();
    changed = true;
  }
  for (int li = 0; li < s->nlanes(); ++li) {
    Lane &L = s->lanes[li];
    if (!L.busy) continue;
    const hipError_t q = hipEventQuery(L.ev);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) {
      // the group's kernel failed: its flags will never arrive, so every waiter
      // is woken with the error instead of waiting forever
      if (s->fatal == 0) s->fatal = map_hip(q);
      changed = true;
      continue;
    }
    if (L.outstanding > 0) continue;  // the flags of a finished kernel are visible on the next pass
    L.busy = false;
    changed = true;
  }
  return changed;
}

// Admit queued requests into free lanes and launch them.  Requires s->mu.
bool admit(ot_server *s) {
  bool any = false;
  // this round's target lane of each class: its first idle stream, if any
  int target[kClasses];
  for (int c = 0; c < kClasses; ++c) {
    target[c] = -1;
    for (int l = 0; l < s->lpc && target[c] < 0; ++l)
      if (!s->lanes[c * s->lpc + l].busy) target[c] = c * s->lpc + l;
  }
  int scanned = 0;
  for (auto it = s->pending.begin(); it != s->pending.end() && scanned < 4096; ++scanned) {
    Req *r = *it;
    if (target[r->cls] < 0) { ++it; continue; }
    if (s->free_slots.empty() || s->inflight >= s->cfg.max_inflight) break;
    if (s->inflight_bytes + r->bytes > s->cfg.hbm_budget_bytes) { ++it; continue; }
    const int64_t abytes = 4ll * r->n * r->n;
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
    s->lanes[target[r->cls]].group.push_back(r);
    s->running.push_back(r);
    it = s->pending.erase(it);
    any = true;
  }
  for (int c = 0; c < kClasses; ++c) {
    if (target[c] < 0) continue;
    Lane &L = s->lanes[target[c]];
    if (L.group.empty()) continue;
    ++L.tag;
    const int rc = launch_group(s, target[c]);
    if (rc != OT_OK) { s->fatal = rc; return any; }
  }
  return any;
}

void worker_main(ot_server *s) {
  hipSetDevice(s->dev);  // the device that was current at ot_serve_open
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    if (s->fatal) break;
    bool progressed = retire(s);
    if (progressed) s->cv_done.notify_all();
    progressed = admit(s) || progressed;
    if (s->stop && s->pending.empty() && s->running.empty()) {
      bool idle = true;
      for (auto &L : s->lanes) idle = idle && !L.busy;
      if (idle) break;
    }
    if (!progressed) s->cv_work.wait_for(lk, std::chrono::microseconds(20));
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
      cfg.streams > kMaxLanesPerClass || cfg.max_n < 0 || cfg.max_n > OT_MAX_N)
    return OT_EINVAL;
  if (cfg.hbm_budget_bytes == 0) cfg.hbm_budget_bytes = 8ll << 30;
  if (cfg.max_inflight == 0) cfg.max_inflight = 256;
  if (cfg.streams == 0) cfg.streams = kDefaultLanesPerClass;
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
  s->cus = device_cus();
  s->t0 = std::chrono::steady_clock::now();
  const size_t M = (size_t)s->maxn, SL = (size_t)s->slots;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chk(hipMalloc(&s->arena_base, (size_t)cfg.hbm_budget_bytes));
  chk(hipMalloc(&s->d_pts, 4 * 4 * M * SL));
  chk(hipHostMalloc(&s->h_pts, 4 * 4 * M * SL, hipHostMallocDefault));
  chk(hipHostMalloc(&s->h_plan, 4 * M * SL, hipHostMallocMapped | hipHostMallocCoherent));
  chk(hipHostMalloc(&s->h_u, 8 * M * SL, hipHostMallocMapped | hipHostMallocCoherent));
  chk(hipHostMalloc(&s->h_v, 8 * M * SL, hipHostMallocMapped | hipHostMallocCoherent));
  const int ws_grid = std::min<int>(s->slots, 8 * s->cus);
  s->lpc = cfg.streams;
  for (int li = 0; li < s->nlanes() && e == hipSuccess; ++li) {
    const int c = li / s->lpc;
    Lane &L = s->lanes[li];
    chk(hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking));
    chk(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
    chk(hipMalloc(&L.d_coff, 8 * SL)); chk(hipMalloc(&L.d_voff, 8 * SL));
    chk(hipMalloc(&L.d_n, 4 * SL)); chk(hipMalloc(&L.d_order, 4 * SL));
    chk(hipMalloc(&L.d_head, 256));
    chk(hipMalloc(&L.d_ws, 4 * ws_ints(std::min(kClassMaxN[c], s->maxn)) * (size_t)std::max(ws_grid, s->slots)));
    chk(hipHostMalloc(&L.h_coff, 8 * SL, hipHostMallocDefault));
    chk(hipHostMalloc(&L.h_voff, 8 * SL, hipHostMallocDefault));
    chk(hipHostMalloc(&L.h_n, 4 * SL, hipHostMallocDefault));
    chk(hipHostMalloc(&L.h_order, 4 * SL, hipHostMallocDefault));
    chk(hipHostMalloc(&L.h_cost, 8 * SL, hipHostMallocMapped | hipHostMallocCoherent));
    chk(hipHostMalloc(&L.h_stats, sizeof(ot_stats) * SL, hipHostMallocMapped | hipHostMallocCoherent));
    chk(hipHostMalloc(&L.h_done, 4 * SL, hipHostMallocMapped | hipHostMallocCoherent));
  }
  if (e != hipSuccess) {
    const int rc = map_hip(e);
    free_server(s);
    return rc;
  }
  for (int li = 0; li < s->nlanes(); ++li) std::memset(s->lanes[li].h_done, 0, 4 * SL);
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
  r->cls = class_of(n);
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
