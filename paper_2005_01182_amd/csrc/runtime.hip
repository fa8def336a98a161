// runtime.hip -- host runtime and C-ABI of the batched Kuhn-Munkres solver.
//
// Device context (one per process, current device), a library stream for the
// synchronous calls, grow-only device buffers, a per-stream workspace cache for
// the asynchronous calls, host-side validation and error mapping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "launch.hpp"
#include "otkm.h"
#include "runtime.hpp"

namespace otkm {

namespace {

std::mutex g_mu;          // guards the context, the pool and the schedule
bool g_init_done = false;
int g_init_status = OT_ENODEV;
int g_dev = 0;
int g_cus = 0;
hipStream_t g_stream = nullptr;
int g_t64 = 0, g_t256 = 0;  // 0 = defaults
std::atomic<int> g_split_n{0}, g_split_wgs{0};  // 0 = defaults (read without the lock)

// Default size classes of the batch path, as ot_schedule_tune measured them on
// MI355X (instance throughput with every workgroup slot busy): one wavefront
// per instance up to n = 512, 256 lanes up to 1024, 512 lanes above.
constexpr int kDefaultT64 = 512;
constexpr int kDefaultT256 = 1024;

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};
std::map<int, Buf> g_pool;                      // synchronous calls (library stream)
std::map<hipStream_t, std::map<int, Buf>> g_ws; // asynchronous calls, per stream

}  // namespace

int map_hip(hipError_t e) {
  if (e == hipSuccess) return OT_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return OT_ENOMEM;
  if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return OT_ENODEV;
  return OT_EDEVICE;
}

int init_locked() {
  if (g_init_done) return g_init_status;
  g_init_done = true;
  const char *env = std::getenv("OT_DEVICE");
  if (env && std::strcmp(env, "none") == 0) return g_init_status = OT_ENODEV;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return g_init_status = OT_ENODEV;
  if (hipGetDevice(&g_dev) != hipSuccess) return g_init_status = OT_ENODEV;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, g_dev) != hipSuccess) return g_init_status = OT_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return g_init_status = OT_ENODEV;
  g_cus = prop.multiProcessorCount;
  if (hipStreamCreateWithFlags(&g_stream, hipStreamNonBlocking) != hipSuccess) return g_init_status = OT_EDEVICE;
  return g_init_status = OT_OK;
}

hipStream_t lib_stream() { return g_stream; }
int device_cus() { return g_cus; }
std::mutex &lib_mutex() { return g_mu; }

// Grow-only buffer in slot `slot` of the synchronous pool (library stream).
void *pool_get(int slot, size_t bytes, int *err) {
  Buf &b = g_pool[slot];
  if (bytes == 0) bytes = 16;
  if (b.bytes < bytes) {
    if (b.p) {
      // queued work may still use the old buffer; an error it left is reported here
      const hipError_t se = hipStreamSynchronize(g_stream);
      if (se != hipSuccess) { *err = map_hip(se); return nullptr; }
      (void)hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) { *err = map_hip(e); b.p = nullptr; return nullptr; }
    b.bytes = bytes;
  }
  return b.p;
}

// Grow-only workspace tied to a caller stream: work queued on one stream runs
// in order, so reuse across calls on that stream is safe.  Growing
// synchronises the stream first (not allowed during graph capture: the first
// call on a stream, outside capture, should size it).
void *stream_ws(hipStream_t s, int slot, size_t bytes, int *err) {
  Buf &b = g_ws[s][slot];
  if (bytes == 0) bytes = 16;
  if (b.bytes < bytes) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
      *err = OT_EINVAL;
      return nullptr;
    }
    if (b.p) {
      const hipError_t se = hipStreamSynchronize(s);
      if (se != hipSuccess) { *err = map_hip(se); return nullptr; }
      (void)hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) { *err = map_hip(e); b.p = nullptr; return nullptr; }
    b.bytes = bytes;
  }
  return b.p;
}

// Free every workspace cached for stream s (before the caller destroys it).
void stream_ws_free(hipStream_t s) {
  auto it = g_ws.find(s);
  if (it == g_ws.end()) return;
  // the buffers go whatever the stream's last work returned: an error of that
  // work belongs to the call that queued it
  (void)hipStreamSynchronize(s);
  for (auto &kv : it->second)
    if (kv.second.p) (void)hipFree(kv.second.p);
  g_ws.erase(it);
}

void schedule_set_locked(int t64, int t256) {
  g_t64 = t64;
  g_t256 = t256;
}

// Single-instance width (measured on the geometric workload): one wavefront
// needs no workgroup barrier and wins while its 8 columns per lane cover n;
// then 8 wavefronts (at n = 4096, 16 wavefronts have too few registers each).
int default_block(int n) { return n <= 512 ? 64 : 512; }

int schedule_block(int n) {
  const int t64 = g_t64 > 0 ? g_t64 : kDefaultT64;
  const int t256 = g_t256 > 0 ? g_t256 : kDefaultT256;
  if (n <= t64 && n <= 64 * 8) return 64;
  if (n <= t256 && n <= 256 * 8) return 256;
  return 512;
}

static bool block_ok(int block, int n) {
  return (block == 64 || block == 256 || block == 512 || block == 1024) && cpt_for(n, block) != 0;
}

// Host range check: max - min over the given entries must fit 2^31 - 1.
static bool range_ok(const int32_t *C, int64_t count) {
  if (count <= 0) return true;
  int32_t mn = C[0], mx = C[0];
  for (int64_t k = 1; k < count; ++k) {
    mn = std::min(mn, C[k]);
    mx = std::max(mx, C[k]);
  }
  return (int64_t)mx - (int64_t)mn <= 0x7fffffffll;
}

// Workgroups per single instance when neither ot_options.wgs nor .block is
// set.  Exact solves split above the schedule's n_split (ot_split_*); the
// defaults were measured on MI355X (geometric instances): the per-step
// exchange through global memory costs about as much as splitting the sweep
// saves at n = 2048 (128.8 vs 126.2 ms), and wins above (n = 2560: 295 -> 197
// ms, n = 4096: 644 -> 350 ms with 8 workgroups).  Scaled costs make fewer,
// wider steps, where the split pays far below (s = 100: 4 workgroups at
// n = 2048, 76.4 -> 33.3 ms; 2 at n = 1024, 17.7 -> 13.3 ms; 2 at n = 512,
// 10.4 -> 5.0 ms).
constexpr int kDefaultSplitN = 2048, kDefaultSplitWgs = 8;
static int default_wgs(int n, int scale) {
  if (scale > 1) return n > 1024 ? 4 : (n > 256 ? 2 : 1);
  const int sn = g_split_n.load() > 0 ? g_split_n.load() : kDefaultSplitN;
  const int sw = g_split_wgs.load() > 0 ? g_split_wgs.load() : kDefaultSplitWgs;
  return n > sn ? sw : 1;
}

struct Opts {
  int block, max_paths, flags, scale, wgs;
};

static int check_options(const ot_options *opt, int n, Opts *o) {
  o->block = default_block(n);
  o->max_paths = 0;
  o->flags = 0;
  o->scale = 1;
  o->wgs = 1;
  if (opt) {
    for (int k = 0; k < 3; ++k)
      if (opt->reserved[k] != 0) return OT_EINVAL;
    if (opt->max_paths < 0 || (opt->flags & ~(OT_FLAG_PHASE_TIMERS | OT_FLAG_WIDE_KEYS)) != 0 || opt->scale < 0 || opt->wgs < 0 ||
        opt->wgs > kMaxWgs)
      return OT_EINVAL;
    o->max_paths = opt->max_paths;
    o->flags = opt->flags;
    o->scale = opt->scale > 1 ? opt->scale : 1;
    if (opt->wgs > 0) o->wgs = opt->wgs;
    else if (opt->block == 0) o->wgs = default_wgs(n, o->scale);
    if (o->wgs == 1 && opt->block != 0) {
      if (!block_ok(opt->block, n)) return OT_EINVAL;
      o->block = opt->block;
    }
  } else {
    o->wgs = default_wgs(n, 1);
  }
  if (o->wgs > 1) {
    // several workgroups: 256 or 512 threads each, at most 4 columns per lane
    const int b = (opt && opt->block != 0) ? opt->block : 512;
    const int cpt = cpt_for(n, b * o->wgs);
    if ((b != 256 && b != 512) || cpt == 0 || cpt > 4) return OT_EINVAL;
    o->block = b;
  }
  return OT_OK;
}

// Device workspace of the one-instance solve: ints of P.ws, and bytes of the
// grid state (several workgroups only).
static size_t solve_ws_ints(int n, const Opts &o) { return ws_ints(n) * (size_t)o.wgs; }
static size_t solve_grid_bytes(int n, const Opts &o) {
  return o.wgs > 1 ? 8 * grid_ws_u64(o.wgs, o.block * cpt_for(n, o.block * o.wgs)) : 16;
}

// One wavefront holds the whole instance (wave_engine.hpp): it reads C itself,
// so the grid-wide sweeps and the transpose are skipped and a solve is one launch.
static bool wave_solve(int n, const Opts &o) { return o.wgs == 1 && o.block == 64 && n <= 64; }

static hipError_t launch_solve(Problem &P, const Opts &o, uint64_t *gws, hipStream_t s) {
  if (o.wgs > 1) {
    P.grid_ws = gws;
    return launch_assign_grid(P, o.block, o.wgs, s);
  }
  return launch_assign_one(P, o.block, nullptr, s);
}

}  // namespace otkm

using namespace otkm;

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *ot_strerror(int status) {
  switch (status) {
    case OT_OK: return "ok";
    case OT_EINVAL: return "invalid argument";
    case OT_ERANGE: return "cost range exceeds 2^31 - 1";
    case OT_EUNBALANCED: return "supplies and demands do not balance (or are all zero)";
    case OT_ENEGMASS: return "negative supply or demand";
    case OT_ETOOBIG: return "instance too large for the on-chip solver";
    case OT_ENOMEM: return "out of memory";
    case OT_EDEVICE: return "HIP runtime error";
    case OT_ENODEV: return "no usable gfx950 device";
    case OT_EINTERNAL: return "internal solver error (watchdog or invariant)";
    case OT_EINFEASIBLE: return "no matching of the graph covers every row";
    default: return "unknown status";
  }
}

int ot_init(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return init_locked();
}

int ot_assign_ex(const int32_t *C, int32_t n, const ot_options *opt, int32_t *plan, int64_t *cost, int64_t *u,
                 int64_t *v, ot_stats *stats) {
  if (!C || !plan || !cost || n <= 0) return OT_EINVAL;
  if (n > OT_MAX_N) return OT_ETOOBIG;
  Opts o;
  int rc = check_options(opt, n, &o);
  if (rc) return rc;
  const int scale = o.scale;
  if (!range_ok(C, (int64_t)n * n)) return OT_ERANGE;

  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = init_locked())) return rc;
  int err = OT_OK;
  const size_t N = (size_t)n;
  auto *dC = (int32_t *)pool_get(0, 4 * N * N, &err);
  auto *dplan = (int32_t *)pool_get(1, 4 * N, &err);
  auto *du = (int64_t *)pool_get(2, 8 * N, &err);
  auto *dv = (int64_t *)pool_get(3, 8 * N, &err);
  auto *dcost = (int64_t *)pool_get(4, 8, &err);
  auto *dstats = (ot_stats *)pool_get(5, sizeof(ot_stats), &err);
  auto *dws = (int32_t *)pool_get(6, 4 * solve_ws_ints(n, o), &err);
  auto *dgws = (uint64_t *)pool_get(84, solve_grid_bytes(n, o), &err);
  auto *dCT = (int32_t *)pool_get(7, 4 * N * N, &err);
  auto *dCs = scale > 1 ? (int32_t *)pool_get(8, 4 * N * N, &err) : nullptr;
  if (err) return err;
  hipStream_t s = g_stream;
  hipError_t e = hipMemcpyAsync(dC, C, 4 * N * N, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return map_hip(e);
  const int32_t *dsolve = dC;
  if (scale > 1) {
    if ((e = launch_floor_div(dC, n, n, scale, dCs, s)) != hipSuccess) return map_hip(e);
    dsolve = dCs;
  }
  auto *du0 = (int64_t *)pool_get(80, 8 * N, &err);
  auto *drmax = (int32_t *)pool_get(81, 4 * N, &err);
  auto *dpart = (uint64_t *)pool_get(82, init_part_bytes(n, n), &err);
  auto *db = (uint64_t *)pool_get(83, 16 * N, &err);
  if (err) return err;
  Problem P;
  P.C = dsolve; P.n = n; P.ld = n; P.CT = nullptr; P.max_paths = o.max_paths; P.flags = o.flags;
  P.Cout = dC; P.ldo = n; P.dscale = scale;
  P.init_u = nullptr; P.init_b = nullptr; P.init_rmax = nullptr;
  if (!wave_solve(n, o)) {
    // the streaming row sweep reads C first (from HBM when C is cold), the
    // tiled transpose then finds it in the last-level cache
    if ((e = launch_init_sweeps(dsolve, n, n, n, du0, drmax, dpart, db, s)) != hipSuccess) return map_hip(e);
    if ((e = launch_transpose(dsolve, n, n, n, dCT, s)) != hipSuccess) return map_hip(e);
    P.CT = dCT;
    P.init_u = du0; P.init_b = db; P.init_rmax = drmax;
  }
  P.plan = dplan; P.cost = dcost; P.u = du; P.v = dv; P.stats = dstats; P.ws = dws;
  if ((e = launch_solve(P, o, dgws, s)) != hipSuccess) return map_hip(e);
  ot_stats hs;
  std::vector<int32_t> hplan(N);
  std::vector<int64_t> hu(N), hv(N);
  int64_t hcost = 0;
  if ((e = hipMemcpyAsync(&hs, dstats, sizeof hs, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hplan.data(), dplan, 4 * N, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hu.data(), du, 8 * N, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hv.data(), dv, 8 * N, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(&hcost, dcost, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return map_hip(e);
  if (hs.status != 0) return (int)hs.status;
  std::memcpy(plan, hplan.data(), 4 * N);
  *cost = hcost;
  if (u) std::memcpy(u, hu.data(), 8 * N);
  if (v) std::memcpy(v, hv.data(), 8 * N);
  if (stats) *stats = hs;
  return OT_OK;
}

int ot_scale_for(const int32_t *C, int32_t n, double eps, int32_t *scale, int64_t *lower_bound) {
  if (!C || !scale || n <= 0 || !(eps >= 0.0)) return OT_EINVAL;
  if (n > OT_MAX_N) return OT_ETOOBIG;
  if (!range_ok(C, (int64_t)n * n)) return OT_ERANGE;
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = init_locked();
  if (rc) return rc;
  int err = OT_OK;
  const size_t N = (size_t)n;
  auto *dC = (int32_t *)pool_get(0, 4 * N * N, &err);
  auto *du0 = (int64_t *)pool_get(80, 8 * N, &err);
  auto *drmax = (int32_t *)pool_get(81, 4 * N, &err);
  auto *dpart = (uint64_t *)pool_get(82, init_part_bytes(n, n), &err);
  auto *db = (uint64_t *)pool_get(83, 16 * N, &err);
  auto *dlb = (int64_t *)pool_get(85, 8, &err);
  if (err) return err;
  hipStream_t s = g_stream;
  hipError_t e = hipMemcpyAsync(dC, C, 4 * N * N, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return map_hip(e);
  if ((e = launch_init_sweeps(dC, n, n, n, du0, drmax, dpart, db, s)) != hipSuccess) return map_hip(e);
  if ((e = launch_lower_bound(du0, db, n, dlb, s)) != hipSuccess) return map_hip(e);
  int64_t lb = 0;
  if ((e = hipMemcpyAsync(&lb, dlb, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return map_hip(e);
  // n (s - 1) <= eps * lb <= eps * OPT: the scaled solve's cost is within (1 + eps) OPT
  double sf = lb > 0 ? 1.0 + std::floor(eps * (double)lb / (double)n) : 1.0;
  if (sf > 1073741824.0) sf = 1073741824.0;
  *scale = (int32_t)sf;
  if (lower_bound) *lower_bound = lb;
  return OT_OK;
}

int ot_assign(const int32_t *C, int32_t n, int32_t *plan, int64_t *cost, int64_t *u, int64_t *v) {
  return ot_assign_ex(C, n, nullptr, plan, cost, u, v, nullptr);
}

int ot_assign_dev(const int32_t *dC, int32_t n, int32_t ld, const ot_options *opt, int32_t *dplan, int64_t *dcost,
                  int64_t *du, int64_t *dv, ot_stats *dstats, void *stream) {
  if (!dC || !dplan || !dcost || n <= 0 || ld < n) return OT_EINVAL;
  if (n > OT_MAX_N) return OT_ETOOBIG;
  Opts o;
  int rc = check_options(opt, n, &o);
  if (rc) return rc;
  const int scale = o.scale;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = init_locked())) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : g_stream;
  int err = OT_OK;
  auto *dws = (int32_t *)stream_ws(s, 0, 4 * solve_ws_ints(n, o), &err);
  auto *dgws = (uint64_t *)stream_ws(s, 44, solve_grid_bytes(n, o), &err);
  auto *dCT = (int32_t *)stream_ws(s, 3, 4 * (size_t)n * (size_t)n, &err);
  auto *dCs = scale > 1 ? (int32_t *)stream_ws(s, 4, 4 * (size_t)n * (size_t)n, &err) : nullptr;
  if (err) return err;
  hipError_t e;
  const int32_t *dsolve = dC;
  int lds = ld;
  if (scale > 1) {
    if ((e = launch_floor_div(dC, n, ld, scale, dCs, s)) != hipSuccess) return map_hip(e);
    dsolve = dCs;
    lds = n;
  }
  auto *du0 = (int64_t *)stream_ws(s, 40, 8 * (size_t)n, &err);
  auto *drmax = (int32_t *)stream_ws(s, 41, 4 * (size_t)n, &err);
  auto *dpart = (uint64_t *)stream_ws(s, 42, init_part_bytes(n, n), &err);
  auto *db = (uint64_t *)stream_ws(s, 43, 16 * (size_t)n, &err);
  if (err) return err;
  Problem P;
  P.C = dsolve; P.n = n; P.ld = lds; P.CT = nullptr; P.max_paths = o.max_paths; P.flags = o.flags;
  P.Cout = dC; P.ldo = ld; P.dscale = scale;
  P.init_u = nullptr; P.init_b = nullptr; P.init_rmax = nullptr;
  if (!wave_solve(n, o)) {
    // the streaming row sweep reads C first (from HBM when C is cold), the
    // tiled transpose then finds it in the last-level cache
    if ((e = launch_init_sweeps(dsolve, n, n, lds, du0, drmax, dpart, db, s)) != hipSuccess) return map_hip(e);
    if ((e = launch_transpose(dsolve, n, n, lds, dCT, s)) != hipSuccess) return map_hip(e);
    P.CT = dCT;
    P.init_u = du0; P.init_b = db; P.init_rmax = drmax;
  }
  P.plan = dplan; P.cost = dcost; P.u = du; P.v = dv; P.stats = dstats; P.ws = dws;
  return map_hip(launch_solve(P, o, dgws, s));
}

}  // extern "C"

namespace otkm {

// Rectangular solve on device buffers.  The solver's rows are the smaller side:
// C itself when n <= m (its transpose feeds the single-column refreshes), else
// C^T materialised in the workspace (and C serves as that matrix's transpose).
// Then the grid-wide reduction sweeps, the one-instance engine and the
// rectangular outputs.  `get(slot, bytes)` hands out workspace.
template <class Get>
static int rect_pipeline(const int32_t *dC, int n, int m, int ld, const Opts &o, Get get, hipStream_t s,
                         int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats) {
  const bool trans = n > m;
  const int nr = trans ? m : n, nc = trans ? n : m;  // solver rows <= solver columns
  auto *T = (int32_t *)get(0, 4 * (size_t)n * (size_t)m);
  auto *ws = (int32_t *)get(2, 4 * solve_ws_ints(nc, o));
  auto *gws = (uint64_t *)get(12, solve_grid_bytes(nc, o));
  auto *pq = (int32_t *)get(3, 4 * (size_t)nr);
  auto *uq = (int64_t *)get(4, 8 * (size_t)nr);
  auto *vq = (int64_t *)get(5, 8 * (size_t)nc);
  auto *cq = (int64_t *)get(6, 8);
  auto *sq = (ot_stats *)get(7, sizeof(ot_stats));
  auto *u0 = (int64_t *)get(8, 8 * (size_t)nr);
  auto *rmax = (int32_t *)get(9, 4 * (size_t)nr);
  auto *part = (uint64_t *)get(10, init_part_bytes(nr, nc));
  auto *b = (uint64_t *)get(11, 16 * (size_t)nc);
  if (!T || !ws || !gws || !pq || !uq || !vq || !cq || !sq || !u0 || !rmax || !part || !b) return OT_ENOMEM;
  hipError_t e;
  // the transpose of C (m x n, row stride n) is the solver matrix (trans) or its transpose
  if ((e = launch_transpose(dC, n, m, ld, T, s)) != hipSuccess) return map_hip(e);
  const int32_t *A = trans ? T : dC;
  const int lda = trans ? n : ld;
  if ((e = launch_init_sweeps(A, nr, nc, lda, u0, rmax, part, b, s)) != hipSuccess) return map_hip(e);
  Problem P;
  P.C = A; P.n = nc; P.nr = nr; P.ld = lda; P.max_paths = o.max_paths; P.flags = o.flags;
  P.CT = trans ? dC : T; P.ldt = trans ? ld : n;
  P.Cout = nullptr; P.ldo = lda; P.dscale = 1;
  P.init_u = u0; P.init_b = b; P.init_rmax = rmax;
  P.plan = pq; P.cost = cq; P.u = uq; P.v = vq; P.stats = sq; P.ws = ws;
  if ((e = launch_solve(P, o, gws, s)) != hipSuccess) return map_hip(e);
  return map_hip(launch_rect_finish(n, m, trans, pq, uq, vq, cq, sq, dplan, dcost, du, dv, dstats, s));
}

static int rect_check(int32_t n, int32_t m, const ot_options *opt, Opts *o) {
  if (n <= 0 || m <= 0) return OT_EINVAL;
  const int M = std::max(n, m);
  if (M > OT_MAX_N) return OT_ETOOBIG;
  int rc = check_options(opt, M, o);
  if (rc) return rc;
  return o->scale > 1 ? OT_EINVAL : OT_OK;
}

}  // namespace otkm

extern "C" {

int ot_assign_rect(const int32_t *C, int32_t n, int32_t m, const ot_options *opt, int32_t *plan, int64_t *cost,
                   int64_t *u, int64_t *v, ot_stats *stats) {
  if (!C || !plan || !cost) return OT_EINVAL;
  Opts o;
  int rc = rect_check(n, m, opt, &o);
  if (rc) return rc;
  if (!range_ok(C, (int64_t)n * m)) return OT_ERANGE;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = init_locked())) return rc;
  int err = OT_OK;
  const size_t NM = (size_t)n * (size_t)m;
  auto *dC = (int32_t *)pool_get(90, 4 * NM, &err);
  auto *dplan = (int32_t *)pool_get(91, 4 * (size_t)n, &err);
  auto *du = (int64_t *)pool_get(92, 8 * (size_t)n, &err);
  auto *dv = (int64_t *)pool_get(93, 8 * (size_t)m, &err);
  auto *dcost = (int64_t *)pool_get(94, 8, &err);
  auto *dstats = (ot_stats *)pool_get(95, sizeof(ot_stats), &err);
  if (err) return err;
  hipStream_t s = g_stream;
  hipError_t e = hipMemcpyAsync(dC, C, 4 * NM, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return map_hip(e);
  auto get = [&](int slot, size_t bytes) { return pool_get(100 + slot, bytes, &err); };
  rc = rect_pipeline(dC, n, m, m, o, get, s, dplan, dcost, du, dv, dstats);
  if (err) return err;
  if (rc) return rc;
  ot_stats hs;
  std::vector<int32_t> hplan(n);
  std::vector<int64_t> hu(n), hv(m);
  int64_t hcost = 0;
  if ((e = hipMemcpyAsync(&hs, dstats, sizeof hs, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hplan.data(), dplan, 4 * (size_t)n, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return map_hip(e);
  if ((e = hipMemcpyAsync(hu.data(), du, 8 * (size_t)n, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hv.data(), dv, 8 * (size_t)m, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(&hcost, dcost, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return map_hip(e);
  if (hs.status != 0) return (int)hs.status;
  std::memcpy(plan, hplan.data(), 4 * (size_t)n);
  *cost = hcost;
  if (u) std::memcpy(u, hu.data(), 8 * (size_t)n);
  if (v) std::memcpy(v, hv.data(), 8 * (size_t)m);
  if (stats) *stats = hs;
  return OT_OK;
}

int ot_assign_rect_dev(const int32_t *dC, int32_t n, int32_t m, int32_t ld, const ot_options *opt, int32_t *dplan,
                       int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream) {
  if (!dC || !dplan || !dcost || ld < m) return OT_EINVAL;
  Opts o;
  int rc = rect_check(n, m, opt, &o);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = init_locked())) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : g_stream;
  int err = OT_OK;
  auto get = [&](int slot, size_t bytes) { return stream_ws(s, 100 + slot, bytes, &err); };
  rc = rect_pipeline(dC, n, m, ld, o, get, s, dplan, dcost, du, dv, dstats);
  return err ? err : rc;
}

int ot_transpose_batch_dev(int32_t count, int32_t max_n, const int32_t *dC, const int64_t *coff, const int32_t *n,
                           int32_t *dCT, void *stream) {
  if (count < 0 || !dC || !coff || !n || !dCT || max_n <= 0) return OT_EINVAL;
  if (max_n > OT_MAX_N) return OT_ETOOBIG;
  if (count == 0) return OT_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = init_locked();
  if (rc) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : g_stream;
  return map_hip(launch_transpose_batch(dC, coff, n, count, max_n, dCT, s));
}

// ot_assign_batch_dev and ot_assign_batch_ct_dev: ctw, when given, receives
// the transposes (written by the launch's flag pass) and replaces dCT.
static int assign_batch_dev(int32_t count, int32_t max_n, const int32_t *dC, const int32_t *dCT, int32_t *ctw,
                            const int64_t *coff, const int32_t *n, const int64_t *voff, const int32_t *order,
                            int32_t nq, int32_t block, int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv,
                            ot_stats *dstats, void *stream) {
  if (count < 0 || !dC || !coff || !n || !voff || !dplan || !dcost || max_n <= 0) return OT_EINVAL;
  if (!order) nq = count;
  if (nq < 0 || nq > count) return OT_EINVAL;
  if (count == 0 || nq == 0) return OT_OK;
  if (max_n > OT_MAX_N) return OT_ETOOBIG;
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = init_locked();
  if (rc) return rc;
  if (block == 0) block = schedule_block(max_n);
  if (!block_ok(block, max_n)) return OT_EINVAL;
  hipStream_t s = stream ? (hipStream_t)stream : g_stream;
  const int occ = batch_occupancy(block, max_n);
  if (occ <= 0) return OT_ETOOBIG;
  const int grid = std::max(1, std::min<int>(nq, occ * g_cus));
  int err = OT_OK;
  auto *head = (int32_t *)stream_ws(s, 1, 256, &err);
  auto *dws = (int32_t *)stream_ws(s, 2, 4 * ws_ints(max_n) * (size_t)grid, &err);
  auto *kflags = (uint8_t *)stream_ws(s, 5, (size_t)count, &err);
  if (err) return err;
  hipError_t e = launch_fill_i32(head, 0, 1, s);
  if (e != hipSuccess) return map_hip(e);
  BatchArgs A;
  A.C = dC; A.CT = dCT; A.coff = coff; A.n = n; A.voff = voff; A.order = order;
  A.count = count; A.nq = nq; A.max_n = max_n; A.max_paths = 0;
  A.plan = dplan; A.cost = dcost; A.u = du; A.v = dv; A.stats = dstats; A.ws = dws; A.head = head; A.done = nullptr; A.tag = 0;
  A.kflags = kflags; A.head2 = head + 32;  // another 128-byte line of the same buffer
  A.ctw = ctw;
  return map_hip(launch_assign_batch(A, block, grid, s));
}

int ot_assign_batch_dev(int32_t count, int32_t max_n, const int32_t *dC, const int32_t *dCT, const int64_t *coff,
                        const int32_t *n, const int64_t *voff, const int32_t *order, int32_t nq, int32_t block,
                        int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream) {
  return assign_batch_dev(count, max_n, dC, dCT, nullptr, coff, n, voff, order, nq, block, dplan, dcost, du, dv,
                          dstats, stream);
}

int ot_assign_batch_ct_dev(int32_t count, int32_t max_n, const int32_t *dC, int32_t *dCT, const int64_t *coff,
                           const int32_t *n, const int64_t *voff, const int32_t *order, int32_t nq, int32_t block,
                           int32_t *dplan, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats,
                           void *stream) {
  if (!dCT) return OT_EINVAL;
  return assign_batch_dev(count, max_n, dC, nullptr, dCT, coff, n, voff, order, nq, block, dplan, dcost, du, dv,
                          dstats, stream);
}

int ot_assign_batch(int32_t count, const int32_t *const *C, const int32_t *n, int32_t *const *plan, int64_t *cost,
                    int64_t *const *u, int64_t *const *v, int32_t *status) {
  if (count < 0 || (count > 0 && (!C || !n || !plan || !cost || !status))) return OT_EINVAL;
  if (count == 0) return OT_OK;
  std::vector<int64_t> coff(count), voff(count);
  int64_t ctot = 0, vtot = 0;
  for (int k = 0; k < count; ++k) {
    status[k] = OT_OK;
    if (!C[k] || !plan[k] || n[k] <= 0) status[k] = OT_EINVAL;
    else if (n[k] > OT_MAX_N) status[k] = OT_ETOOBIG;
    else if (!range_ok(C[k], (int64_t)n[k] * n[k])) status[k] = OT_ERANGE;
    coff[k] = ctot;
    voff[k] = vtot;
    if (status[k] == OT_OK) { ctot += (int64_t)n[k] * n[k]; vtot += n[k]; }
  }
  // size classes by workgroup width (one wavefront's classes split at n = 64,
  // where the whole instance fits its registers); each class runs longest-first
  std::map<std::pair<int, int>, std::vector<int>> cls;
  for (int k = 0; k < count; ++k)
    if (status[k] == OT_OK) {
      const int b = schedule_block(n[k]);
      cls[{b, b == 64 && n[k] <= 64 ? 0 : 1}].push_back(k);
    }
  if (cls.empty()) return OT_OK;

  std::lock_guard<std::mutex> lk(g_mu);
  int rc = init_locked();
  if (rc) return rc;
  int err = OT_OK;
  hipStream_t s = g_stream;
  auto *dC = (int32_t *)pool_get(10, 4 * (size_t)std::max<int64_t>(ctot, 1), &err);
  auto *dplan = (int32_t *)pool_get(11, 4 * (size_t)std::max<int64_t>(vtot, 1), &err);
  auto *du = (int64_t *)pool_get(12, 8 * (size_t)std::max<int64_t>(vtot, 1), &err);
  auto *dv = (int64_t *)pool_get(13, 8 * (size_t)std::max<int64_t>(vtot, 1), &err);
  auto *dcost = (int64_t *)pool_get(14, 8 * (size_t)count, &err);
  auto *dstats = (ot_stats *)pool_get(15, sizeof(ot_stats) * (size_t)count, &err);
  auto *dcoff = (int64_t *)pool_get(16, 8 * (size_t)count, &err);
  auto *dvoff = (int64_t *)pool_get(17, 8 * (size_t)count, &err);
  auto *dn = (int32_t *)pool_get(18, 4 * (size_t)count, &err);
  auto *dorder = (int32_t *)pool_get(19, 4 * (size_t)count, &err);
  auto *head = (int32_t *)pool_get(20, 4 * 8, &err);
  auto *head2 = (int32_t *)pool_get(21, 4 * 8, &err);
  auto *kflags = (uint8_t *)pool_get(22, (size_t)count, &err);
  if (err) return err;
  hipError_t e;
  for (int k = 0; k < count; ++k)
    if (status[k] == OT_OK &&
        (e = hipMemcpyAsync(dC + coff[k], C[k], 4 * (size_t)n[k] * n[k], hipMemcpyHostToDevice, s)) != hipSuccess)
      return map_hip(e);
  if ((e = hipMemcpyAsync(dcoff, coff.data(), 8 * (size_t)count, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(dvoff, voff.data(), 8 * (size_t)count, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(dn, n, 4 * (size_t)count, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  std::vector<int32_t> order;
  std::vector<std::pair<int, int>> spans;  // (start in order, length) per class
  for (auto &kv : cls) {
    auto &v = kv.second;
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return n[a] > n[b]; });
    spans.push_back({(int)order.size(), (int)v.size()});
    order.insert(order.end(), v.begin(), v.end());
  }
  if ((e = hipMemcpyAsync(dorder, order.data(), 4 * order.size(), hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = launch_fill_i32(head, 0, 8, s)) != hipSuccess) return map_hip(e);
  int ci = 0;
  for (auto &kv : cls) {
    const int block = kv.first.first;
    const auto &v = kv.second;
    int max_n = 0;
    for (int k : v) max_n = std::max(max_n, n[k]);
    const int occ = batch_occupancy(block, max_n);
    if (occ <= 0) return OT_ETOOBIG;
    const int grid = std::max(1, std::min<int>((int)v.size(), occ * g_cus));
    auto *dws = (int32_t *)pool_get(30 + ci, 4 * ws_ints(max_n) * (size_t)grid, &err);
    if (err) return err;
    BatchArgs A;
    A.C = dC; A.coff = dcoff; A.n = dn; A.voff = dvoff; A.order = dorder + spans[ci].first;
    A.count = count; A.nq = spans[ci].second; A.max_n = max_n; A.max_paths = 0;
    A.plan = dplan; A.cost = dcost; A.u = du; A.v = dv; A.stats = dstats; A.ws = dws; A.head = head + ci; A.done = nullptr; A.tag = 0;
    A.kflags = kflags; A.head2 = head2 + ci;
    if ((e = launch_assign_batch(A, block, grid, s)) != hipSuccess) return map_hip(e);
    ++ci;
  }
  std::vector<int32_t> hplan(std::max<int64_t>(vtot, 1));
  std::vector<int64_t> hu(std::max<int64_t>(vtot, 1)), hv(std::max<int64_t>(vtot, 1)), hcost(count);
  std::vector<ot_stats> hs(count);
  if ((e = hipMemcpyAsync(hplan.data(), dplan, 4 * (size_t)vtot, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hu.data(), du, 8 * (size_t)vtot, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hv.data(), dv, 8 * (size_t)vtot, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hcost.data(), dcost, 8 * (size_t)count, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hs.data(), dstats, sizeof(ot_stats) * (size_t)count, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return map_hip(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return map_hip(e);
  for (int k = 0; k < count; ++k) {
    if (status[k] != OT_OK) continue;
    if (hs[k].status != 0) { status[k] = (int32_t)hs[k].status; continue; }
    std::memcpy(plan[k], hplan.data() + voff[k], 4 * (size_t)n[k]);
    cost[k] = hcost[k];
    if (u && u[k]) std::memcpy(u[k], hu.data() + voff[k], 8 * (size_t)n[k]);
    if (v && v[k]) std::memcpy(v[k], hv.data() + voff[k], 8 * (size_t)n[k]);
  }
  return OT_OK;
}

// Host-side mass and range checks shared by the transport entry points.
static int transport_check(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m, int64_t *S) {
  int64_t sr = 0, sc = 0;
  for (int i = 0; i < n; ++i) { if (r[i] < 0) return OT_ENEGMASS; sr += r[i]; }
  for (int j = 0; j < m; ++j) { if (c[j] < 0) return OT_ENEGMASS; sc += c[j]; }
  if (sr != sc || sr < 1) return OT_EUNBALANCED;
  if (sr > OT_MAX_N) return OT_ETOOBIG;
  // range over the entries the unit problem sees (rows and columns with mass)
  bool any = false;
  int32_t mn = 0, mx = 0;
  for (int i = 0; i < n; ++i) {
    if (r[i] == 0) continue;
    for (int j = 0; j < m; ++j) {
      if (c[j] == 0) continue;
      const int32_t x = C[(size_t)i * m + j];
      if (!any) { mn = mx = x; any = true; }
      mn = std::min(mn, x);
      mx = std::max(mx, x);
    }
  }
  if ((int64_t)mx - (int64_t)mn > 0x7fffffffll) return OT_ERANGE;
  *S = sr;
  return OT_OK;
}

static int transport_buffers(TransportArgs &T, int n, int m, int S, bool async, hipStream_t s) {
  int err = OT_OK;
  const size_t SS = (size_t)S;
  auto get = [&](int slot, size_t bytes) -> void * {
    return async ? stream_ws(s, 10 + slot, bytes, &err) : pool_get(40 + slot, bytes, &err);
  };
  T.rowbin = (int32_t *)get(0, 4 * SS);
  T.colbin = (int32_t *)get(1, 4 * SS);
  T.rfirst = (int32_t *)get(2, 4 * (size_t)n);
  T.cfirst = (int32_t *)get(3, 4 * (size_t)m);
  T.gate = (int32_t *)get(4, 16);
  T.Cx = (int32_t *)get(5, 4 * SS * SS);
  T.plan = (int32_t *)get(6, 4 * SS);
  T.U = (int64_t *)get(7, 8 * SS);
  T.V = (int64_t *)get(8, 8 * SS);
  T.ws = (int32_t *)get(9, 4 * ws_ints(S));
  T.CxT = (int32_t *)(async ? stream_ws(s, 25, 4 * SS * SS, &err) : pool_get(70, 4 * SS * SS, &err));
  return err;
}

int ot_transport(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m, int32_t *X,
                 int64_t *cost, int64_t *u, int64_t *v) {
  if (!C || !r || !c || !X || !cost || n <= 0 || m <= 0) return OT_EINVAL;
  int64_t S64 = 0;
  int rc = transport_check(C, r, c, n, m, &S64);
  if (rc) return rc;
  const int S = (int)S64;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = init_locked())) return rc;
  hipStream_t s = g_stream;
  int err = OT_OK;
  const size_t NM = (size_t)n * m;
  TransportArgs T;
  T.n = n; T.m = m; T.S = S; T.max_paths = 0;
  auto *dC = (int32_t *)pool_get(50, 4 * NM, &err);
  auto *dr = (int32_t *)pool_get(51, 4 * (size_t)n, &err);
  auto *dc = (int32_t *)pool_get(52, 4 * (size_t)m, &err);
  T.X = (int32_t *)pool_get(53, 4 * NM, &err);
  T.cost = (int64_t *)pool_get(54, 8, &err);
  T.u = (int64_t *)pool_get(55, 8 * (size_t)n, &err);
  T.v = (int64_t *)pool_get(56, 8 * (size_t)m, &err);
  T.stats = (ot_stats *)pool_get(57, sizeof(ot_stats), &err);
  if (err) return err;
  if ((err = transport_buffers(T, n, m, S, false, s))) return err;
  T.C = dC; T.r = dr; T.c = dc;
  hipError_t e;
  if ((e = hipMemcpyAsync(dC, C, 4 * NM, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(dr, r, 4 * (size_t)n, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(dc, c, 4 * (size_t)m, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = launch_transport(T, default_block(S), s)) != hipSuccess) return map_hip(e);
  ot_stats hs;
  std::vector<int32_t> hX(NM);
  std::vector<int64_t> hu(n), hv(m);
  int64_t hcost = 0;
  if ((e = hipMemcpyAsync(&hs, T.stats, sizeof hs, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hX.data(), T.X, 4 * NM, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hu.data(), T.u, 8 * (size_t)n, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hv.data(), T.v, 8 * (size_t)m, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(&hcost, T.cost, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return map_hip(e);
  if (hs.status != 0) return (int)hs.status;
  std::memcpy(X, hX.data(), 4 * NM);
  *cost = hcost;
  if (u) std::memcpy(u, hu.data(), 8 * (size_t)n);
  if (v) std::memcpy(v, hv.data(), 8 * (size_t)m);
  return OT_OK;
}

int ot_transport_dev(const int32_t *dC, const int32_t *dr, const int32_t *dc, int32_t n, int32_t m, int32_t S,
                     int32_t *dX, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream) {
  if (!dC || !dr || !dc || !dX || !dcost || !du || !dv || n <= 0 || m <= 0 || S <= 0) return OT_EINVAL;
  if (S > OT_MAX_N) return OT_ETOOBIG;
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = init_locked();
  if (rc) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : g_stream;
  TransportArgs T;
  T.C = dC; T.r = dr; T.c = dc; T.n = n; T.m = m; T.S = S; T.max_paths = 0;
  T.X = dX; T.cost = dcost; T.u = du; T.v = dv;
  int err = OT_OK;
  T.stats = dstats ? dstats : (ot_stats *)stream_ws(s, 30, sizeof(ot_stats), &err);
  if (err) return err;
  if ((err = transport_buffers(T, n, m, S, true, s))) return err;
  return map_hip(launch_transport(T, default_block(S), s));
}

int ot_schedule_get(int32_t *t64, int32_t *t256) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (t64) *t64 = g_t64 > 0 ? g_t64 : kDefaultT64;
  if (t256) *t256 = g_t256 > 0 ? g_t256 : kDefaultT256;
  return OT_OK;
}

int ot_split_get(int32_t *n_split, int32_t *wgs) {
  if (n_split) *n_split = g_split_n.load() > 0 ? g_split_n.load() : kDefaultSplitN;
  if (wgs) *wgs = g_split_wgs.load() > 0 ? g_split_wgs.load() : kDefaultSplitWgs;
  return OT_OK;
}

int ot_split_set(int32_t n_split, int32_t wgs) {
  if (n_split < 0 || wgs < 0 || wgs == 1 || wgs > kMaxWgs) return OT_EINVAL;
  g_split_n.store(n_split);
  g_split_wgs.store(wgs);
  return OT_OK;
}

int ot_schedule_set(int32_t t64, int32_t t256) {
  if (t64 < 0 || t256 < 0) return OT_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  g_t64 = t64;
  g_t256 = t256;
  return OT_OK;
}

}  // extern "C"
