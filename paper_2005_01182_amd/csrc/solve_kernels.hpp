// solve_kernels.hpp -- the engine's kernels (one instance per workgroup, one
// instance over several workgroups, persistent batch) and their launch
// helpers.  Each solve_*.hip file instantiates a share of the widths so that
// the library builds in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "engine.hpp"
#include "launch.hpp"
#include "wave_engine.hpp"

namespace otkm {

// ---------------------------------------------------------------------------
// single instance
// ---------------------------------------------------------------------------
// Whether compact (32-bit) keys hold this instance: the cost range from the
// grid-wide initial sweeps is below kCompactRange, n <= kCompactMaxN, and
// every free row is a root.  Uniform over the workgroup; uses the start of
// the LDS before the engine lays it out.
template <int BLOCK>
__device__ __forceinline__ bool compact_keys_fit(const Problem &P, char *smem) {
  constexpr int NW = BLOCK / 64;
  const int nr = (P.nr > 0 && P.nr < P.n) ? P.nr : P.n;
  if (!P.init_u || !P.init_rmax || P.n > kCompactMaxN || (P.max_paths > 0 && P.max_paths < nr) ||
      (P.flags & OT_FLAG_WIDE_KEYS))
    return false;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int64_t mn = INT64_MAX;
  int mx = (int)0x80000000;
  for (int i = tid; i < nr; i += BLOCK) {
    mn = min(mn, P.init_u[i]);
    mx = max(mx, P.init_rmax[i]);
  }
  int lo = wave_min_i32((int)max(mn, (int64_t)INT32_MIN)), hi = wave_max_i32(mx);
  int *red = (int *)smem;
  if (lane == 0) { red[2 * wid] = lo; red[2 * wid + 1] = hi; }
  __syncthreads();
  lo = 0x7fffffff;
  hi = (int)0x80000000;
#pragma unroll
  for (int w = 0; w < NW; ++w) { lo = min(lo, red[2 * w]); hi = max(hi, red[2 * w + 1]); }
  __syncthreads();  // the engine reuses this LDS
  return (int64_t)hi - (int64_t)lo < kCompactRange;
}

template <int BLOCK, int CPT>
__global__ __launch_bounds__(BLOCK) void k_assign_one(Problem P, const int32_t *gate) {
  extern __shared__ __align__(16) char smem[];
  if (gate && *gate != 0) return;  // an earlier stage of this pipeline already failed
  if constexpr (BLOCK == 64 && CPT == 1) {
    if (P.nr == 0 || P.nr == P.n) {  // square, n <= 64: all state in one wavefront's registers
      WaveEngine W;
      W.run(P, smem);
      return;
    }
  }
  constexpr bool kLong = BLOCK <= 512;  // at 1024 threads the registers are too few for LONG
  if (compact_keys_fit<BLOCK>(P, smem)) {
    Engine<BLOCK, CPT, kLong, false, true, true> E;
    E.run(P, smem);
    return;
  }
  Engine<BLOCK, CPT, kLong, false, true> E;
  E.run(P, smem);
}

// ---------------------------------------------------------------------------
// one instance over gridDim.x workgroups (P.grid_ws header zeroed before the
// launch; the grid is at most kMaxWgs workgroups, one per CU, so all of them
// are resident at once)
// ---------------------------------------------------------------------------
template <int BLOCK, int CPT>
__global__ __launch_bounds__(BLOCK) void k_assign_grid(Problem P) {
  extern __shared__ __align__(16) char smem[];
  // every workgroup reads the same sweep results, so all of them pick the same keys
  if (compact_keys_fit<BLOCK>(P, smem)) {
    Engine<BLOCK, CPT, true, true, true, true> E;
    E.run(P, smem);
    return;
  }
  Engine<BLOCK, CPT, true, true, true> E;
  E.run(P, smem);
}

// ---------------------------------------------------------------------------
// persistent batch: each workgroup pops instance indices until the queue is empty
// ---------------------------------------------------------------------------
// Two wavefronts per SIMD: the register budget drops to 256 (a few bytes of
// spill at 8 columns per lane) and twice as many instances share each CU, which
// measured 126k -> 181k solves/s on the embedding batch; three or four per SIMD
// spill heavily and lose.
// COMPACT: the compact-key engine over the instances whose flag is set (the
// 64-bit-key kernel takes the others); without flags the 64-bit-key kernel
// takes every instance.
template <int BLOCK, int CPT, bool COMPACT = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_assign_batch(BatchArgs A) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_idx;
  int32_t *ws = A.ws + (size_t)blockIdx.x * ws_ints(A.max_n);
  constexpr bool kSplit = !(BLOCK == 64 && CPT == 1);  // the one-wavefront class does not split
  const bool split = kSplit && A.kflags && A.head2;
  int32_t *head = (COMPACT || !split) ? A.head : A.head2;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(head, 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= A.nq) break;  // every workgroup reaches this exit once the queue drains
    const int k = A.order ? A.order[idx] : idx;
    if ((unsigned)k >= (unsigned)A.count) continue;  // no such instance: nothing to report or flag
    if (split && (A.kflags[k] != 0) != COMPACT) continue;  // the other kernel's instance
    const int n = A.n[k];
    if (n < 1 || n > A.max_n || n > BLOCK * CPT) {
      if (threadIdx.x == 0) {
        if (A.stats) { ot_stats s = {}; s.status = OT_EINVAL; A.stats[k] = s; }
        if (A.done) {
          __threadfence_system();
          __hip_atomic_store(&A.done[k], A.tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      continue;
    }
    Problem P;
    P.C = A.C + A.coff[k];
    P.n = n;
    P.ld = n;
    P.CT = A.CT ? A.CT + A.coff[k] : nullptr;
    P.Cout = nullptr;
    P.ldo = n;
    P.dscale = 1;
    P.init_u = nullptr; P.init_b = nullptr; P.init_rmax = nullptr;
    P.max_paths = A.max_paths;
    P.flags = 0;
    P.plan = A.plan + A.voff[k];
    P.cost = A.cost + k;
    P.u = A.u ? A.u + A.voff[k] : nullptr;
    P.v = A.v ? A.v + A.voff[k] : nullptr;
    P.stats = A.stats ? A.stats + k : nullptr;
    P.ws = ws;
    if constexpr (BLOCK == 64 && CPT == 1) {  // every instance has n <= 64: one wavefront's registers
      WaveEngine W;
      W.run(P, smem);
    } else {
      Engine<BLOCK, CPT, false, false, false, COMPACT> E;
      E.run(P, smem);
    }
    if (A.done) {
      // outputs may live in host memory: make every thread's writes visible
      // system-wide before the completion flag is released
      __threadfence_system();
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_store(&A.done[k], A.tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
  }
}

__global__ void k_fill_u64(uint64_t *p, uint64_t value, int64_t count);

// Per queue entry (one workgroup each): whether compact keys hold the
// instance (cost range below kCompactRange, n <= kCompactMaxN, every free row
// a root).  One pass over its matrix.
__global__ void k_batch_flags(BatchArgs A);

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
// A kernel's dynamic LDS limit is raised only when a launch needs more than
// it was last raised to, so repeated launches cost no extra runtime call.
template <auto KERNEL>
static hipError_t allow_lds(size_t bytes) {
  static std::atomic<size_t> allowed{0};
  if (bytes <= allowed.load(std::memory_order_acquire)) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute((const void *)KERNEL, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) {
    size_t cur = allowed.load(std::memory_order_relaxed);
    while (cur < bytes && !allowed.compare_exchange_weak(cur, bytes, std::memory_order_release)) {
    }
  }
  return e;
}

// LDS of a kernel of width B for instances of at most n columns: the
// workgroup engine's layout, or the wave engine's copy of C when larger.
template <int B>
static size_t solve_lds(int n) {
  size_t lds = lds_layout(n).total;
  if (B == 64) lds = std::max(lds, wave_lds_bytes(std::min(n, kWaveMaxN)));
  return lds;
}

template <int B, int CPT>
static hipError_t one(const Problem &P, const int32_t *gate, hipStream_t s) {
  const size_t lds = solve_lds<B>(P.n);
  hipError_t e = allow_lds<k_assign_one<B, CPT>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_assign_one<B, CPT>), dim3(1), dim3(B), lds, s, P, gate);
  return hipGetLastError();
}

template <int B, int CPT>
static hipError_t grid(const Problem &P, int wgs, hipStream_t s) {
  const size_t lds = lds_layout(P.n, true).total;
  hipError_t e = allow_lds<k_assign_grid<B, CPT>>(lds);
  if (e != hipSuccess) return e;
  // every tag word must start below the first level
  hipLaunchKernelGGL(k_fill_u64, dim3(16), dim3(256), 0, s, P.grid_ws, (uint64_t)0,
                     (int64_t)grid_ws_u64(wgs, B * CPT));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((k_assign_grid<B, CPT>), dim3(wgs), dim3(B), lds, s, P);
  return hipGetLastError();
}

template <int B, int CPT>
static hipError_t batch(const BatchArgs &A, int grid, hipStream_t s) {
  const size_t lds = solve_lds<B>(A.max_n);
  hipError_t e;
  if constexpr (!(B == 64 && CPT == 1)) {
    if (A.kflags && A.head2) {
      // flags (and the transposes, when asked for), then the compact-key
      // kernel, then the 64-bit-key kernel on the rest
      hipLaunchKernelGGL(k_batch_flags, dim3(A.nq), dim3(256), 0, s, A);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = launch_fill_i32(A.head2, 0, 1, s)) != hipSuccess) return e;
      BatchArgs S = A;
      if (A.ctw) S.CT = A.ctw;
      if ((e = allow_lds<k_assign_batch<B, CPT, true>>(lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_assign_batch<B, CPT, true>), dim3(grid), dim3(B), lds, s, S);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = allow_lds<k_assign_batch<B, CPT>>(lds)) != hipSuccess) return e;
      hipLaunchKernelGGL((k_assign_batch<B, CPT>), dim3(grid), dim3(B), lds, s, S);
      return hipGetLastError();
    }
  }
  if ((e = allow_lds<k_assign_batch<B, CPT>>(lds)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_assign_batch<B, CPT>), dim3(grid), dim3(B), lds, s, A);
  return hipGetLastError();
}

template <int B, int CPT>
static int occ(int max_n) {
  int blocks = 0;
  const size_t lds = solve_lds<B>(max_n);
  if (allow_lds<k_assign_batch<B, CPT>>(lds) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, (const void *)k_assign_batch<B, CPT>, B, lds) != hipSuccess)
    return 0;
  return blocks;
}

}  // namespace otkm
