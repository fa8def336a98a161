// autotune.hip -- size-class schedule for the batch path, and the split
// schedule of single instances.
//
// For a ladder of instance sizes, time the persistent batch kernel at each
// eligible workgroup width (64, 256, 512 lanes) on synthetic instances and
// keep, per size, the width with the highest instance throughput.  Each probe
// holds enough instances to fill every workgroup slot of the chip several
// times over at the narrowest width, so it measures throughput rather than the
// latency of one wave of instances.  The thresholds are the largest sizes up to
// which the narrower widths win.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "launch.hpp"
#include "otkm.h"
#include "runtime.hpp"

using namespace otkm;

namespace {

// Time one batch of `count` n x n instances at width `block`; returns ms or < 0.
float time_batch(int block, int n, int count, int32_t *dC, int64_t *dcoff, int32_t *dn, int64_t *dvoff,
                 int32_t *dplan, int64_t *dcost, int32_t *head, int32_t *dws, hipStream_t s) {
  const int occ = batch_occupancy(block, n);
  if (occ <= 0) return -1.f;
  const int grid = std::max(1, std::min(count, occ * device_cus()));
  BatchArgs A;
  A.C = dC; A.coff = dcoff; A.n = dn; A.voff = dvoff; A.order = nullptr;
  A.count = count; A.nq = count; A.max_n = n; A.max_paths = 0;
  A.plan = dplan; A.cost = dcost; A.u = nullptr; A.v = nullptr; A.stats = nullptr; A.ws = dws; A.head = head; A.done = nullptr; A.tag = 0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) { hipEventDestroy(e0); return -1.f; }
  float best = -1.f;
  for (int rep = 0; rep < 3; ++rep) {
    launch_fill_i32(head, 0, 1, s);
    hipEventRecord(e0, s);
    if (launch_assign_batch(A, block, grid, s) != hipSuccess) break;
    hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) break;
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best < 0 || ms < best)) best = ms;  // first run warms up
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return best;
}

}  // namespace

extern "C" int ot_schedule_tune(int32_t reps) {
  if (reps < 0) return OT_EINVAL;
  std::lock_guard<std::mutex> lk(lib_mutex());
  int rc = init_locked();
  if (rc) return rc;
  const int sizes[] = {32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  const int widths[] = {64, 256, 512};
  const int64_t budget = 256ll << 20;  // cost entries per probe (1 GiB)
  hipStream_t s = lib_stream();
  int best_w[sizeof(sizes) / sizeof(sizes[0])];
  uint64_t lcg = 0x9e3779b97f4a7c15ull;
  for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]); ++si) {
    const int n = sizes[si];
    int slots = 1;  // workgroup slots of the whole chip at the narrowest eligible width
    for (int w : widths)
      if (cpt_for(n, w) != 0) { slots = std::max(1, batch_occupancy(w, n)) * device_cus(); break; }
    // enough instances to fill every slot reps times over; they cycle through
    // `distinct` matrices (instances only read their matrix), so the probe's
    // memory stays bounded however many instances it holds
    const int count = std::max(4, std::min(65536, std::max(reps, 1) * slots));
    const int distinct = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(count, 64), budget / ((int64_t)n * n)));
    std::vector<int32_t> hC((size_t)distinct * n * n);
    for (auto &x : hC) {
      lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
      x = (int32_t)((lcg >> 33) % 10000);
    }
    std::vector<int64_t> coff(count), voff(count);
    std::vector<int32_t> nn(count, n);
    for (int k = 0; k < count; ++k) { coff[k] = (int64_t)(k % distinct) * n * n; voff[k] = (int64_t)k * n; }
    int err = OT_OK;
    auto *dC = (int32_t *)pool_get(60, 4 * hC.size(), &err);
    auto *dcoff = (int64_t *)pool_get(61, 8 * (size_t)count, &err);
    auto *dvoff = (int64_t *)pool_get(62, 8 * (size_t)count, &err);
    auto *dn = (int32_t *)pool_get(63, 4 * (size_t)count, &err);
    auto *dplan = (int32_t *)pool_get(64, 4 * (size_t)count * n, &err);
    auto *dcost = (int64_t *)pool_get(65, 8 * (size_t)count, &err);
    auto *head = (int32_t *)pool_get(66, 16, &err);
    if (err) return err;
    hipMemcpyAsync(dC, hC.data(), 4 * hC.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dcoff, coff.data(), 8 * (size_t)count, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dvoff, voff.data(), 8 * (size_t)count, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dn, nn.data(), 4 * (size_t)count, hipMemcpyHostToDevice, s);
    float best = -1.f;
    best_w[si] = 1024;
    for (int w : widths) {
      if (cpt_for(n, w) == 0) continue;
      const int occ = batch_occupancy(w, n);
      if (occ <= 0) continue;
      const int grid = std::max(1, std::min(count, occ * device_cus()));
      auto *dws = (int32_t *)pool_get(67, 4 * ws_ints(n) * (size_t)grid, &err);
      if (err) return err;
      const float ms = time_batch(w, n, count, dC, dcoff, dn, dvoff, dplan, dcost, head, dws, s);
      if (ms > 0 && (best < 0 || ms < best)) { best = ms; best_w[si] = w; }
    }
    if (best < 0) return OT_EDEVICE;
  }
  // contiguous prefixes: widths must not narrow as n grows
  int t64 = 0, t256 = 0;
  for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]) && best_w[si] == 64; ++si) t64 = sizes[si];
  t256 = t64;
  for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]) && best_w[si] <= 256; ++si) t256 = std::max(t256, sizes[si]);
  schedule_set_locked(std::max(t64, 1), std::max(t256, std::max(t64, 1)));
  return OT_OK;
}

// ---------------------------------------------------------------------------
// split schedule: from which n one instance runs on several workgroups
// ---------------------------------------------------------------------------
// Times one exact solve per size of a ladder and per workgroup count (1, 4,
// 8) on a synthetic geometric instance (points on a circle against points on
// a square's perimeter, cost = rint(1e4 * distance)), through the public
// device call on a private stream.  n_split = the largest size of the
// contiguous prefix where one workgroup is fastest; the count is the one that
// wins at the largest size.  A split has to win by 2% to count.
namespace {

void geometric_instance(int n, uint64_t seed, std::vector<int32_t> &C) {
  uint64_t x = seed;
  auto uni = [&x]() {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
  };
  std::vector<double> sx(n), sy(n), tx(n), ty(n);
  for (int i = 0; i < n; ++i) {
    const double th = 6.283185307179586 * uni();
    sx[i] = std::cos(th);
    sy[i] = std::sin(th);
  }
  for (int j = 0; j < n; ++j) {
    const double t = 4.0 * uni();
    const int side = std::min(3, (int)t);
    const double f = t - side;
    const double px[4] = {-0.5 + f, 0.5, 0.5 - f, -0.5}, py[4] = {-0.5, -0.5 + f, 0.5, 0.5 - f};
    tx[j] = px[side];
    ty[j] = py[side];
  }
  C.resize((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      C[(size_t)i * n + j] = (int32_t)std::lrint(1e4 * std::hypot(sx[i] - tx[j], sy[i] - ty[j]));
}

}  // namespace

extern "C" int ot_split_tune(void) {
  {
    std::lock_guard<std::mutex> lk(lib_mutex());
    int rc = init_locked();
    if (rc) return rc;
  }
  const int sizes[] = {1536, 2048, 2560, 3072, 4096};
  const int cands[] = {1, 4, 8};
  constexpr int NS = sizeof(sizes) / sizeof(sizes[0]), NC = sizeof(cands) / sizeof(cands[0]);
  const int nmax = sizes[NS - 1];
  hipStream_t s = nullptr;
  int32_t *dC = nullptr, *dplan = nullptr;
  int64_t *dcost = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = OT_OK;
  auto fail = [&rc](int code) { if (rc == OT_OK) rc = code; };
  if (hipStreamCreate(&s) != hipSuccess) return OT_EDEVICE;
  if (hipMalloc(&dC, 4 * (size_t)nmax * nmax) != hipSuccess || hipMalloc(&dplan, 4 * (size_t)nmax) != hipSuccess ||
      hipMalloc(&dcost, 8) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    fail(OT_ENOMEM);
  float ms[NS][NC];
  std::vector<int32_t> hC;
  for (int si = NS - 1; si >= 0 && rc == OT_OK; --si) {  // largest first: the workspaces grow once
    const int n = sizes[si];
    geometric_instance(n, 0x2545f4914f6cdd1dull + (uint64_t)n, hC);
    if (hipMemcpyAsync(dC, hC.data(), 4 * hC.size(), hipMemcpyHostToDevice, s) != hipSuccess) { fail(OT_EDEVICE); break; }
    for (int ci = 0; ci < NC && rc == OT_OK; ++ci) {
      ot_options o = {};
      o.wgs = cands[ci];
      // untimed first solve at the largest size sizes every workspace
      for (int rep = (si == NS - 1) ? 0 : 1; rep < 2 && rc == OT_OK; ++rep) {
        if (hipEventRecord(e0, s) != hipSuccess) { fail(OT_EDEVICE); break; }
        const int r = ot_assign_dev(dC, n, n, &o, dplan, dcost, nullptr, nullptr, nullptr, s);
        if (r != OT_OK) { fail(r); break; }
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { fail(OT_EDEVICE); break; }
        hipEventElapsedTime(&ms[si][ci], e0, e1);
      }
    }
  }
  if (rc == OT_OK) {
    auto best_at = [&](int si) {
      int b = 0;
      for (int ci = 1; ci < NC; ++ci)
        if (ms[si][ci] < 0.98f * ms[si][0] && ms[si][ci] < ms[si][b]) b = ci;
      return b;
    };
    int n_split = 0;
    for (int si = 0; si < NS && best_at(si) == 0; ++si) n_split = sizes[si];
    const int top = best_at(NS - 1);
    if (n_split == 0) n_split = sizes[0] - 1;  // splitting wins from the smallest size tried
    if (top == 0) n_split = OT_MAX_N;           // never split
    ot_split_set(n_split, top == 0 ? 0 : cands[top]);
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(dC);
  hipFree(dplan);
  hipFree(dcost);
  {
    std::lock_guard<std::mutex> lk(lib_mutex());
    stream_ws_free(s);
  }
  hipStreamDestroy(s);
  return rc;
}
