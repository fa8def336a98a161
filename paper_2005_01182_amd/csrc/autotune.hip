// autotune.hip -- size-class schedule for the batch path.
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
