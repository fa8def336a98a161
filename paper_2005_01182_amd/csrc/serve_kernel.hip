// serve_kernel.hip -- the serving kernel.
//
// One persistent launch serves every request size.  Its workgroups (one per
// CU: the LDS of the largest instance) take requests from a queue that the
// host appends to while the kernel runs; a workgroup builds its request's
// cost matrix from the request's points, solves it with the workgroup engine
// of the request's width, writes the results to host memory and releases the
// request's completion flag, then takes the next request.
//
// Queue protocol (every wait is bounded):
//   * the host writes an entry's descriptor (and the request's points) into
//     mapped host memory, then raises the host tail with a release store;
//   * device memory mirrors the tail; one idle workgroup at a time (at most
//     one per microsecond, device-wide) reads the host tail and the host's
//     quit word and folds them into the mirrors, so PCIe sees about a million
//     small reads a second at most, whatever the grid;
//   * an entry is taken by advancing the device head past it (compare and
//     swap); the head persists across launches, so a new launch continues
//     where the last one stopped, and every entry a workgroup takes it
//     finishes;
//   * a workgroup that finds the queue empty `linger` times in a row (a short
//     sleep each) leaves, and so does one that sees the quit word at or above
//     its launch's epoch (the host raises it once nothing is outstanding).
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "gridcost.hpp"
#include "launch.hpp"

namespace otkm {

constexpr int kServeBlock = 512;
// s_memrealtime ticks (100 MHz) between two reads of the host words
constexpr uint64_t kPollTicks = 100;

// LDS of the serving kernel: the engine's layout for max_n columns, or the
// points of one request (4 max_n words) while its matrix is built.
size_t serve_lds_bytes(int max_n) {
  const size_t e = lds_layout(max_n).total, p = 16 * (size_t)max_n;
  return e > p ? e : p;
}

// Compact keys take the one-instance engine's long-frontier organisation
// (chunks of up to 8 rows, pipelined sweeps and gathers): more registers
// spill, but the large requests that dominate a stream solve faster
// (20-s stream: 1,888 -> 1,942 solves/s, p99 1.01 -> 0.52 s).
template <int CPT>
__device__ __forceinline__ void serve_solve(const Problem &P, char *smem, bool compact) {
  if (compact) {
    Engine<kServeBlock, CPT, true, false, false, true> E;
    E.run(P, smem);
  } else {
    Engine<kServeBlock, CPT> E;
    E.run(P, smem);
  }
}

__global__ __launch_bounds__(kServeBlock) void k_serve(ServeArgs A) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_idx, s_slot, s_n;
  __shared__ int64_t s_coff;
  __shared__ int s_lo[kServeBlock / 64], s_hi[kServeBlock / 64];
  int32_t *ws = A.ws + (size_t)blockIdx.x * ws_ints(A.max_n);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (;;) {
    if (tid == 0) {
      int idx = -1;
      for (int spin = 0;;) {
        const int h = __hip_atomic_load(A.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int t = __hip_atomic_load(A.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (h < t) {
          int hh = h;
          if (__hip_atomic_compare_exchange_strong(A.head, &hh, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)) {
            idx = h;
            break;
          }
          continue;
        }
        if (__hip_atomic_load(A.quit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= A.epoch || spin >= A.linger)
          break;
        ++spin;
        const uint64_t now = wall_clock64();
        uint64_t last = __hip_atomic_load(A.polled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (now - last >= kPollTicks &&
            __hip_atomic_compare_exchange_strong(A.polled, &last, now, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
          const int ht = __hip_atomic_load(A.h_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
          const int hq = __hip_atomic_load(A.h_quit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          __hip_atomic_fetch_max(A.tail, ht, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_max(A.quit, hq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          continue;
        }
        __builtin_amdgcn_s_sleep(32);
      }
      int slot = -1, n = 0;
      int64_t coff = 0;
      if (idx >= 0) {
        // the host wrote the descriptor before the tail that covers it
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const int32_t *e = A.desc + 4 * (size_t)(idx % A.qcap);
        slot = __hip_atomic_load(e + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        n = __hip_atomic_load(e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t lo = (uint32_t)__hip_atomic_load(e + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t hi = (uint32_t)__hip_atomic_load(e + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        coff = (int64_t)(((uint64_t)hi << 32) | lo);
      }
      s_idx = idx;
      s_slot = slot;
      s_n = n;
      s_coff = coff;
    }
    __syncthreads();
    const int idx = s_idx, slot = s_slot, n = s_n;
    const int64_t coff = s_coff;
    __syncthreads();
    if (idx < 0) break;  // every workgroup reaches this exit
    const int32_t tag = idx + 1;
    if ((unsigned)slot >= (unsigned)A.slots) continue;  // no such slot: nothing to report or flag
    const size_t M = (size_t)A.max_n;
    if (n < 1 || n > A.max_n || coff < 0) {
      if (tid == 0) {
        ot_stats s = {};
        s.status = OT_EINVAL;
        A.stats[slot] = s;
        __threadfence_system();
        __hip_atomic_store(&A.done[slot], tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
      continue;
    }
    // ---- the request's points into LDS (host memory, read at system scope)
    int32_t *pts = (int32_t *)smem;  // src x, y (2n) then dst x, y (2n)
    const int32_t *hp = A.pts + (size_t)slot * 4 * M;
    for (int q = tid; q < 4 * n; q += kServeBlock) pts[q] = __hip_atomic_load(hp + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
    // ---- C_ij = round(|src_i - dst_j|), one wavefront per row, lanes along it
    int32_t *C = A.C + coff;
    int lo = 0x7fffffff, hi = 0;
    for (int i = wid; i < n; i += kServeBlock / 64) {
      const int64_t sx = pts[2 * i], sy = pts[2 * i + 1];
      int32_t *row = C + (size_t)i * (size_t)n;
      for (int j = lane; j < n; j += 64) {
        const int64_t dx = sx - pts[2 * n + 2 * j], dy = sy - pts[2 * n + 2 * j + 1];
        const int32_t c = grid_isqrt_round(dx * dx + dy * dy);
        row[j] = c;
        lo = min(lo, c);
        hi = max(hi, c);
      }
    }
    lo = wave_min_i32(lo);
    hi = wave_max_i32(hi);
    if (lane == 0) { s_lo[wid] = lo; s_hi[wid] = hi; }
    // the engine reads C back (and reuses the LDS): every store done and visible
    __threadfence();
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kServeBlock / 64; ++w) { lo = min(lo, s_lo[w]); hi = max(hi, s_hi[w]); }
    // ---- its transpose, CT_ji = C_ij (one wavefront per column of C): a stale
    // column's refresh then reads one contiguous row instead of one memory
    // line per entry, which at full load is most of the HBM traffic
    int32_t *CT = C + (size_t)n * (size_t)n;
    for (int j = wid; j < n; j += kServeBlock / 64) {
      const int64_t tx = pts[2 * n + 2 * j], ty = pts[2 * n + 2 * j + 1];
      int32_t *row = CT + (size_t)j * (size_t)n;
      for (int i = lane; i < n; i += 64) {
        const int64_t dx = pts[2 * i] - tx, dy = pts[2 * i + 1] - ty;
        row[i] = grid_isqrt_round(dx * dx + dy * dy);
      }
    }
    __threadfence();
    __syncthreads();
    // compact keys when the cost range allows them (same results, fewer instructions)
    const bool compact = (int64_t)hi - (int64_t)lo < kCompactRange && n <= kCompactMaxN;
    Problem P;
    P.C = C;
    P.n = n;
    P.ld = n;
    P.CT = CT;
    P.Cout = nullptr;
    P.ldo = n;
    P.dscale = 1;
    P.init_u = nullptr; P.init_b = nullptr; P.init_rmax = nullptr;
    P.max_paths = 0;
    P.flags = 0;
    P.plan = A.plan + slot * M;
    P.cost = A.cost + slot;
    P.u = A.u + slot * M;
    P.v = A.v + slot * M;
    P.stats = A.stats + slot;
    P.ws = ws;
    if (n <= kServeBlock) serve_solve<1>(P, smem, compact);
    else if (n <= 2 * kServeBlock) serve_solve<2>(P, smem, compact);
    else if (n <= 4 * kServeBlock) serve_solve<4>(P, smem, compact);
    else serve_solve<8>(P, smem, compact);
    // outputs live in host memory: every thread's writes visible system-wide
    // before the completion flag is released
    __threadfence_system();
    __syncthreads();
    if (tid == 0) __hip_atomic_store(&A.done[slot], tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    __syncthreads();
  }
}

int serve_occupancy(int max_n) {
  const size_t lds = serve_lds_bytes(max_n);
  if (hipFuncSetAttribute((const void *)k_serve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)k_serve, kServeBlock, lds) != hipSuccess)
    return 0;
  return blocks;
}

hipError_t launch_serve(const ServeArgs &A, int grid, hipStream_t s) {
  const size_t lds = serve_lds_bytes(A.max_n);
  hipLaunchKernelGGL(k_serve, dim3(grid), dim3(kServeBlock), lds, s, A);
  return hipGetLastError();
}

}  // namespace otkm
