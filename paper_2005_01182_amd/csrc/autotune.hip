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
  const int32_t sizes[] = {32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
  const int32_t widths[] = {64, 256, 512};
  constexpr int NS = sizeof(sizes) / sizeof(sizes[0]), NW = sizeof(widths) / sizeof(widths[0]);
  const int64_t budget = 256ll << 20;  // cost entries per probe (1 GiB)
  hipStream_t s = lib_stream();
  float ms[NS * NW];
  uint64_t lcg = 0x9e3779b97f4a7c15ull;
  for (int si = 0; si < NS; ++si) {
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
    for (int wi = 0; wi < NW; ++wi) {
      const int w = widths[wi];
      ms[si * NW + wi] = -1.f;
      if (cpt_for(n, w) == 0) continue;
      const int occ = batch_occupancy(w, n);
      if (occ <= 0) continue;
      const int grid = std::max(1, std::min(count, occ * device_cus()));
      auto *dws = (int32_t *)pool_get(67, 4 * ws_ints(n) * (size_t)grid, &err);
      if (err) return err;
      ms[si * NW + wi] = time_batch(w, n, count, dC, dcoff, dn, dvoff, dplan, dcost, head, dws, s);
    }
  }
  int32_t t64 = 0, t256 = 0;
  if (ot_schedule_rule(NS, sizes, NW, widths, ms, &t64, &t256) != OT_OK) return OT_EDEVICE;
  schedule_set_locked(t64, t256);
  return OT_OK;
}

// The width per size is the fastest probe (the narrower on a tie); the
// thresholds are the contiguous prefixes of sizes won by one wavefront and by
// at most 256 lanes, so widths never narrow as n grows.
extern "C" int ot_schedule_rule(int32_t nsizes, const int32_t *sizes, int32_t nwidths, const int32_t *widths,
                                const float *ms, int32_t *t64, int32_t *t256) {
  if (nsizes <= 0 || nwidths <= 0 || !sizes || !widths || !ms || !t64 || !t256) return OT_EINVAL;
  for (int si = 1; si < nsizes; ++si)
    if (sizes[si] <= sizes[si - 1]) return OT_EINVAL;
  for (int wi = 0; wi < nwidths; ++wi)
    if (widths[wi] != 64 && widths[wi] != 256 && widths[wi] != 512) return OT_EINVAL;
  std::vector<int> best_w(nsizes);
  for (int si = 0; si < nsizes; ++si) {
    float best = -1.f;
    best_w[si] = 0;
    for (int wi = 0; wi < nwidths; ++wi) {
      const float t = ms[(size_t)si * nwidths + wi];
      if (!(t > 0.f)) continue;  // not run, failed, or NaN
      if (best < 0.f || t < best || (t == best && widths[wi] < best_w[si])) { best = t; best_w[si] = widths[wi]; }
    }
    if (best_w[si] == 0) return OT_EINVAL;  // no probe of this size succeeded
  }
  int a = 0, b = 0;
  for (int si = 0; si < nsizes && best_w[si] == 64; ++si) a = sizes[si];
  b = a;
  for (int si = 0; si < nsizes && best_w[si] <= 256; ++si) b = std::max(b, sizes[si]);
  *t64 = std::max(a, 1);
  *t256 = std::max(b, *t64);
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
  const int32_t sizes[] = {1536, 2048, 2560, 3072, 4096};
  const int32_t cands[] = {1, 4, 8};
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
    int32_t n_split = 0, wgs = 0;
    rc = ot_split_rule(NS, sizes, NC, cands, &ms[0][0], &n_split, &wgs);
    if (rc == OT_OK) ot_split_set(n_split, wgs);
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

// The split rule: a candidate count wins a size when it beats one workgroup by
// more than 2% (and every other candidate); n_split is the largest size of the
// contiguous prefix won by one workgroup (one below the smallest size when a
// split wins from the start, OT_MAX_N when none wins at the largest size), and
// wgs is the count that wins at the largest size (0, the default, when none).
extern "C" int ot_split_rule(int32_t nsizes, const int32_t *sizes, int32_t ncands, const int32_t *cands,
                             const float *ms, int32_t *n_split, int32_t *wgs) {
  if (nsizes <= 0 || ncands <= 0 || !sizes || !cands || !ms || !n_split || !wgs || cands[0] != 1) return OT_EINVAL;
  for (int si = 1; si < nsizes; ++si)
    if (sizes[si] <= sizes[si - 1] || sizes[si] > OT_MAX_N) return OT_EINVAL;
  for (int ci = 1; ci < ncands; ++ci)
    if (cands[ci] < 2 || cands[ci] > kMaxWgs) return OT_EINVAL;
  for (int k = 0; k < nsizes * ncands; ++k)
    if (!(ms[k] > 0.f)) return OT_EINVAL;
  auto best_at = [&](int si) {
    const float *t = ms + (size_t)si * ncands;
    int b = 0;
    for (int ci = 1; ci < ncands; ++ci)
      if (t[ci] < 0.98f * t[0] && t[ci] < t[b]) b = ci;
    return b;
  };
  int ns = 0;
  for (int si = 0; si < nsizes && best_at(si) == 0; ++si) ns = sizes[si];
  const int top = best_at(nsizes - 1);
  if (ns == 0) ns = sizes[0] - 1;  // splitting wins from the smallest size tried
  if (top == 0) ns = OT_MAX_N;     // never split
  *n_split = ns;
  *wgs = top == 0 ? 0 : cands[top];
  return OT_OK;
}
