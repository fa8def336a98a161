// serve.hip -- continuous-batching request server (C-ABI in otkm.h).
//
// Requests (n source and n target grid points) queue on the host.  A server
// thread admits them in arrival order as request slots and device bytes free
// up, builds each admitted request's cost matrix on the device from its
// points and publishes it into its size class's live queue (a ring of request
// slots and a tail counter in device memory, written by a small kernel on the
// same build stream, so an entry becomes visible only after its matrix).  Each class runs one persistent batch kernel at a time; its
// workgroups take entries from the queue while the host keeps appending, so a
// request that arrives while its class's kernel runs joins that kernel as
// soon as a workgroup is free, and workgroups that find the queue empty wait
// a short, bounded while before they leave (the kernel holds several sets of
// workgroups, so one that leaves is replaced while requests keep arriving,
// and the kernel ends soon after they stop).  When the kernel has left with
// entries still unclaimed (they arrived after its last workgroup looked), the
// server launches it again from the first unclaimed entry.  The engine
// writes each request's plan and duals straight into pinned host memory and
// then releases a per-request completion flag, so a request completes as
// soon as its own solve does.
#include <hip/hip_runtime.h>

#include <atomic>
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

constexpr int kClasses = 3;
constexpr int kMaxLanesPerClass = 8;
constexpr int kDefaultLanesPerClass = 1;
// size classes: (largest n, workgroup width).  Each class's kernel runs on a
// stream of its own and the builds on another, each on its own hardware queue
// (dedicated_stream), so no stream waits behind another's long kernel.
constexpr int kClassMaxN[kClasses] = {512, 2048, OT_MAX_N};
constexpr int kClassBlock[kClasses] = {64, 256, 512};
// Empty-queue polls before a workgroup leaves: each is a read of the tail in
// host memory and a short sleep, a few microseconds together.
constexpr int kLinger = 24;
// A class's kernel is launched with this many times the workgroups that fit
// on the device at once.  Workgroups that stay busy keep the first set
// resident; one that finds the queue empty leaves, and a workgroup of the
// next set starts in its place, so the kernel keeps its full width while
// requests arrive and ends soon after they stop.
constexpr int kGenerations = 4;

int class_of(int n) {
  for (int c = 0; c < kClasses; ++c)
    if (n <= kClassMaxN[c]) return c;
  return kClasses - 1;
}

int64_t request_bytes(int n) { return 4ll * n * n + 64ll * n; }

struct Req {
  uint64_t id = 0;
  int32_t n = 0, cls = 0, slot = -1, status = 0;
  int lane = -1;
  int32_t pos = -1;       // position in the lane's queue (the completion tag is pos + 1)
  int64_t launch = -1;    // the lane's launch that was running when the request was published, or -1
  int64_t off = -1, abytes = 0, bytes = 0, cost = 0;  // arena offset and size of C; admitted bytes
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool done = false;
  std::vector<int32_t> pts;  // src (2n) then dst (2n)
  std::vector<int32_t> plan;
  std::vector<int64_t> u, v;
};

struct Build {  // requests of one lane whose matrices and queue entries were queued on the build stream together
  hipEvent_t ev = nullptr;
  std::vector<Req *> reqs;
};

struct Lane {  // one size class's queue and kernel stream
  int cls = 0, max_n = 1, block = 64, grid_max = 1;
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;  // the running kernel's completion
  bool running = false;
  int64_t launches = 0;
  int32_t queued = 0;   // entries handed to the build stream
  int outstanding = 0;  // admitted requests of this lane not yet retired
  std::map<int32_t, int32_t> pend;     // published entries not yet retired: position -> request slot
  int4 *h_stage = nullptr;             // mapped: entry p's {slot, n, coff} at p % qcap, read by the publish kernel
  int32_t *d_ring = nullptr;           // entry p -> request slot, at p % qcap
  int32_t *d_tail = nullptr;           // published entries
  int32_t *d_head = nullptr, *d_ws = nullptr;
  std::deque<Build> building;
};

}  // namespace

struct ot_server {
  ot_serve_cfg cfg{};
  int maxn = OT_MAX_N, slots = 256, cus = 1, dev = 0, qcap = 512;
  char *arena_base = nullptr;
  std::unique_ptr<otkm::Arena> arena;
  hipStream_t sb = nullptr;                   // builds every admitted request's cost matrix
  int32_t *d_pts = nullptr;                   // [slots][4 maxn]
  int32_t *h_pts = nullptr;                   // pinned staging [slots][4 maxn]
  int32_t *h_plan = nullptr;                  // mapped [slots][maxn]
  int64_t *h_u = nullptr, *h_v = nullptr;     // mapped [slots][maxn]
  // per request slot: the descriptor on the device, the results mapped
  int64_t *d_coff = nullptr, *d_voff = nullptr;
  int32_t *d_n = nullptr;
  int64_t *h_cost = nullptr;
  int32_t *h_done = nullptr;
  ot_stats *h_stats = nullptr;
  std::vector<int> free_slots;
  std::vector<hipEvent_t> free_events;
  Lane lanes[kClasses * kMaxLanesPerClass];  // lane c * lpc + l: class c, stream l
  int lpc = kDefaultLanesPerClass;
  int nlanes() const { return kClasses * lpc; }
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req *> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<Req *> running;  // published requests not yet complete
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
    if (s->sb) hipStreamSynchronize(s->sb);
    for (auto &b : L.building) hipEventDestroy(b.ev);
    if (L.ev) hipEventDestroy(L.ev);
    if (L.s) hipStreamDestroy(L.s);
    hipFree(L.d_head); hipFree(L.d_ws); hipFree(L.d_ring); hipFree(L.d_tail);
    hipHostFree(L.h_stage);
  }
  for (hipEvent_t e : s->free_events) hipEventDestroy(e);
  if (s->sb) hipStreamDestroy(s->sb);
  hipFree(s->arena_base);
  hipFree(s->d_pts);
  hipHostFree(s->h_pts);
  hipHostFree(s->h_plan);
  hipHostFree(s->h_u);
  hipHostFree(s->h_v);
  hipFree(s->d_coff); hipFree(s->d_voff); hipFree(s->d_n);
  hipHostFree(s->h_cost); hipHostFree(s->h_done); hipHostFree(s->h_stats);
  delete s;
}

template <typename T>
T *dptr(T *host) {  // device address of mapped host memory
  void *d = nullptr;
  if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) return nullptr;
  return (T *)d;
}

// A stream on its own hardware queue.  Streams beyond the runtime's hardware
// queue limit share queues, and work on a shared queue runs in submission
// order across its streams: a class's long-running kernel would hold up the
// builds and the other classes' kernels queued behind it.  A stream created
// with a CU mask always gets a queue of its own; the mask here names every CU.
hipError_t dedicated_stream(hipStream_t *st, int cus) {
  std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0xffffffffu);
  if (cus % 32) mask.back() = (1u << (cus % 32)) - 1;
  return hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data());
}

// (Re)start lane li's kernel from entry `base`.  Requires s->mu.
int launch_lane(ot_server *s, int li, int32_t base) {
  Lane &L = s->lanes[li];
  hipError_t e;
  if ((e = launch_fill_i32(L.d_head, base, 1, L.s)) != hipSuccess) return map_hip(e);
  const int grid = L.grid_max * kGenerations;
  BatchArgs A;
  A.C = (const int32_t *)s->arena_base;
  A.coff = s->d_coff; A.n = s->d_n; A.voff = s->d_voff; A.order = L.d_ring;
  A.count = s->slots; A.nq = 0; A.max_n = L.max_n; A.max_paths = 0;
  A.plan = dptr(s->h_plan); A.cost = dptr(s->h_cost); A.u = dptr(s->h_u); A.v = dptr(s->h_v);
  A.stats = dptr(s->h_stats); A.ws = L.d_ws; A.head = L.d_head; A.done = dptr(s->h_done); A.tag = 0;
  A.live_tail = L.d_tail; A.qcap = s->qcap; A.linger = kLinger;
  if (!A.plan || !A.cost || !A.u || !A.v || !A.stats || !A.done) return OT_EDEVICE;
  if ((e = launch_assign_batch(A, L.block, grid, L.s)) != hipSuccess) return map_hip(e);
  if ((e = hipEventRecord(L.ev, L.s)) != hipSuccess) return map_hip(e);
  L.running = true;
  ++L.launches;
  ++s->ctr.groups;
  return OT_OK;
}

// Retire finished requests and finished kernels.  Returns true when anything
// changed.  Requires s->mu.
bool retire(ot_server *s) {
  bool changed = false;
  const size_t M = (size_t)s->maxn;
  for (size_t i = 0; i < s->running.size();) {
    Req *r = s->running[i];
    const int32_t flag = __atomic_load_n(&s->h_done[r->slot], __ATOMIC_ACQUIRE);
    if (flag != r->pos + 1) { ++i; continue; }
    Lane &L = s->lanes[r->lane];
    const ot_stats st = s->h_stats[r->slot];
    r->status = (int32_t)st.status;
    r->cost = s->h_cost[r->slot];
    if (r->status == 0) {
      r->plan.assign(s->h_plan + (size_t)r->slot * M, s->h_plan + (size_t)r->slot * M + r->n);
      r->u.assign(s->h_u + (size_t)r->slot * M, s->h_u + (size_t)r->slot * M + r->n);
      r->v.assign(s->h_v + (size_t)r->slot * M, s->h_v + (size_t)r->slot * M + r->n);
    }
    // published while the lane's kernel ran, and completed by that same kernel
    if (r->launch >= 0 && r->launch == L.launches && L.running) ++s->ctr.joined;
    r->t_done = s->now();
    r->done = true;
    --L.outstanding;
    L.pend.erase(r->pos);
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
    if (!L.running) continue;
    const hipError_t q = hipEventQuery(L.ev);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) {
      // the kernel failed: its flags will never arrive, so every waiter is
      // woken with the error instead of waiting forever
      if (s->fatal == 0) s->fatal = map_hip(q);
      changed = true;
      continue;
    }
    L.running = false;
    changed = true;
  }
  return changed;
}

// Admit queued requests (arrival order, within the budget and the slots) and
// queue their cost matrices on the build stream.  Requires s->mu.
bool admit(ot_server *s) {
  bool any = false;
  const size_t M = (size_t)s->maxn;
  std::vector<Req *> batch[kClasses * kMaxLanesPerClass];
  int scanned = 0;
  for (auto it = s->pending.begin(); it != s->pending.end() && scanned < 4096; ++scanned) {
    Req *r = *it;
    if (s->free_slots.empty() || s->inflight >= s->cfg.max_inflight) break;
    if (s->inflight_bytes + r->bytes > s->cfg.hbm_budget_bytes) { ++it; continue; }
    const int64_t abytes = 4ll * r->n * r->n;
    const int64_t off = s->arena->alloc(abytes);
    if (off < 0) { ++it; continue; }
    // the class's lane with the fewest outstanding requests
    int li = r->cls * s->lpc;
    for (int l = 1; l < s->lpc; ++l) {
      const int c = r->cls * s->lpc + l;
      if (s->lanes[c].outstanding < s->lanes[li].outstanding) li = c;
    }
    r->off = off;
    r->abytes = abytes;
    r->slot = s->free_slots.back();
    s->free_slots.pop_back();
    r->lane = li;
    r->t_admit = s->now();
    s->inflight_bytes += r->bytes;
    ++s->inflight;
    ++s->lanes[li].outstanding;
    s->ctr.peak_inflight_bytes = std::max(s->ctr.peak_inflight_bytes, s->inflight_bytes);
    s->ctr.peak_inflight = std::max<int64_t>(s->ctr.peak_inflight, s->inflight);
    ++s->ctr.admitted;
    batch[li].push_back(r);
    it = s->pending.erase(it);
    any = true;
  }
  for (int li = 0; li < s->nlanes(); ++li) {
    if (batch[li].empty()) continue;
    Lane &L = s->lanes[li];
    hipError_t e;
    for (Req *r : batch[li]) {
      int32_t *hp = s->h_pts + (size_t)r->slot * 4 * M;
      std::memcpy(hp, r->pts.data(), sizeof(int32_t) * 4 * (size_t)r->n);
      int32_t *dp = s->d_pts + (size_t)r->slot * 4 * M;
      if ((e = hipMemcpyAsync(dp, hp, sizeof(int32_t) * 4 * (size_t)r->n, hipMemcpyHostToDevice, s->sb)) != hipSuccess ||
          (e = launch_grid_cost(dp, dp + 2 * r->n, r->n, (int32_t *)(s->arena_base + r->off), s->sb)) != hipSuccess) {
        s->fatal = map_hip(e);
        return any;
      }
    }
    // queue entries, published on the device after the matrices above
    const int32_t first = L.queued;
    for (Req *r : batch[li]) {
      r->pos = L.queued++;
      L.h_stage[r->pos % s->qcap] = make_int4(r->slot, r->n, (int)(uint32_t)(r->off / 4),
                                             (int)(uint32_t)((uint64_t)(r->off / 4) >> 32));
    }
    std::atomic_thread_fence(std::memory_order_release);
    if ((e = launch_serve_publish(dptr(L.h_stage), first, L.queued - first, s->qcap, (int64_t)M, L.d_ring, s->d_n,
                                  s->d_coff, s->d_voff, L.d_tail, s->sb)) != hipSuccess) {
      s->fatal = map_hip(e);
      return any;
    }
    Build b;
    if (!s->free_events.empty()) {
      b.ev = s->free_events.back();
      s->free_events.pop_back();
    } else if ((e = hipEventCreateWithFlags(&b.ev, hipEventDisableTiming)) != hipSuccess) {
      s->fatal = map_hip(e);
      return any;
    }
    if ((e = hipEventRecord(b.ev, s->sb)) != hipSuccess) { s->fatal = map_hip(e); return any; }
    b.reqs = std::move(batch[li]);
    L.building.push_back(std::move(b));
  }
  return any;
}

// Take note of the requests whose matrices and queue entries are on the
// device (running from now on), and start the kernel of every lane with
// unclaimed entries and no kernel running.  Requires s->mu.
bool publish(ot_server *s) {
  bool any = false;
  for (int li = 0; li < s->nlanes(); ++li) {
    Lane &L = s->lanes[li];
    while (!L.building.empty()) {
      Build &b = L.building.front();
      const hipError_t q = hipEventQuery(b.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) { s->fatal = map_hip(q); return any; }
      for (Req *r : b.reqs) {
        r->launch = L.running ? L.launches : -1;
        s->running.push_back(r);
        L.pend[r->pos] = r->slot;
      }
      s->free_events.push_back(b.ev);
      L.building.pop_front();
      any = true;
    }
    if (L.running) continue;
    // An ended kernel took a prefix of the entries and completed each one it
    // took, so with no kernel running the flags are final: the next launch
    // starts at the first published entry without its flag (entries not yet
    // retired keep their slots, so their flags are theirs).
    int32_t base = -1;
    for (const auto &pe : L.pend)
      if (__atomic_load_n(&s->h_done[pe.second], __ATOMIC_ACQUIRE) != pe.first + 1) { base = pe.first; break; }
    if (base >= 0) {
      const int rc = launch_lane(s, li, base);
      if (rc != OT_OK) { s->fatal = rc; return any; }
      any = true;
    }
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
    progressed = publish(s) || progressed;
    if (s->stop && s->pending.empty() && s->running.empty()) {
      bool idle = true;
      for (int li = 0; li < s->nlanes(); ++li) idle = idle && !s->lanes[li].running && s->lanes[li].building.empty();
      if (idle) break;
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
  // more ring entries than slots: an entry's ring position is reused only after
  // every earlier entry has been taken (at most `slots` wait at a time)
  s->qcap = 2 * s->slots;
  s->cus = device_cus();
  s->t0 = std::chrono::steady_clock::now();
  const size_t M = (size_t)s->maxn, SL = (size_t)s->slots;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
  chk(hipMalloc(&s->arena_base, (size_t)cfg.hbm_budget_bytes));
  chk(hipMalloc(&s->d_pts, 4 * 4 * M * SL));
  chk(hipHostMalloc(&s->h_pts, 4 * 4 * M * SL, hipHostMallocDefault));
  chk(hipHostMalloc(&s->h_plan, 4 * M * SL, mapped));
  chk(hipHostMalloc(&s->h_u, 8 * M * SL, mapped));
  chk(hipHostMalloc(&s->h_v, 8 * M * SL, mapped));
  chk(hipMalloc(&s->d_coff, 8 * SL));
  chk(hipMalloc(&s->d_voff, 8 * SL));
  chk(hipMalloc(&s->d_n, 4 * SL));
  chk(hipHostMalloc(&s->h_cost, 8 * SL, mapped));
  chk(hipHostMalloc(&s->h_done, 4 * SL, mapped));
  chk(hipHostMalloc(&s->h_stats, sizeof(ot_stats) * SL, mapped));
  s->lpc = cfg.streams;
  chk(dedicated_stream(&s->sb, s->cus));
  for (int li = 0; li < s->nlanes() && e == hipSuccess; ++li) {
    Lane &L = s->lanes[li];
    L.cls = li / s->lpc;
    L.max_n = std::min(kClassMaxN[L.cls], s->maxn);
    L.block = kClassBlock[L.cls];
    const int occ = batch_occupancy(L.block, L.max_n);
    if (occ <= 0) { e = hipErrorInvalidValue; break; }
    L.grid_max = std::max(1, std::min<int>(s->slots, occ * s->cus));
    chk(dedicated_stream(&L.s, s->cus));
    chk(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
    chk(hipMalloc(&L.d_head, 256));
    chk(hipMalloc(&L.d_ws, 4 * ws_ints(L.max_n) * (size_t)L.grid_max * kGenerations));
    chk(hipMalloc(&L.d_ring, 4 * (size_t)s->qcap));
    chk(hipMalloc(&L.d_tail, 256));
    chk(hipHostMalloc(&L.h_stage, sizeof(int4) * (size_t)s->qcap, mapped));
    if (e == hipSuccess) chk(hipMemset(L.d_tail, 0, 256));
  }
  if (e != hipSuccess) {
    const int rc = map_hip(e);
    free_server(s);
    return rc;
  }
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
