// bins.hip -- integer transport on the bins (Eq. (1) without unit expansion):
// kernels, launcher and C-ABI (ot_transport_bins, ot_transport_bins_dev).
//
// Pipeline on one stream: k_bins_check (masses: signs, balance, total; sets
// the gate), the KM reduction's grid-wide sweeps over C, a fill of the flow
// matrix, the bin engine on one workgroup (bins_engine.hpp), k_bins_finish
// (flows to the caller's row-major plan and the cost), and the zero-mass
// dual convention of ot_transport.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "bins_engine.hpp"
#include "launch.hpp"
#include "otkm.h"
#include "runtime.hpp"

namespace otkm {

template <int BLOCK, int CPT>
__global__ __launch_bounds__(BLOCK) void k_bins(BinsProblem P, const int32_t *gate) {
  extern __shared__ __align__(16) char smem[];
  if (*gate != 0) return;  // the masses were rejected (status already written)
  BinEngine<BLOCK, CPT> E;
  E.run(P, smem);
}

// Masses: every entry >= 0 and equal totals of at least 1 and at most
// 2^31 - 1, else the status goes to stats and the gate closes.  One workgroup.
__global__ __launch_bounds__(1024) void k_bins_check(const int32_t *r, const int32_t *c, int n, int m, int32_t *gate,
                                                     ot_stats *stats) {
  __shared__ long long s_sum[2];
  __shared__ int s_neg;
  if (threadIdx.x == 0) { s_sum[0] = 0; s_sum[1] = 0; s_neg = 0; }
  __syncthreads();
  long long a = 0, b = 0;
  int neg = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) { neg |= r[i] < 0; a += r[i]; }
  for (int j = threadIdx.x; j < m; j += blockDim.x) { neg |= c[j] < 0; b += c[j]; }
  atomicAdd((unsigned long long *)&s_sum[0], (unsigned long long)a);
  atomicAdd((unsigned long long *)&s_sum[1], (unsigned long long)b);
  if (neg) atomicOr(&s_neg, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int status = 0;
    if (s_neg) status = OT_ENEGMASS;
    else if (s_sum[0] != s_sum[1] || s_sum[0] < 1) status = OT_EUNBALANCED;
    else if (s_sum[0] > 0x7fffffffll) status = OT_ETOOBIG;
    *gate = status;
    if (stats) { ot_stats s = {}; s.status = status; *stats = s; }
  }
}

// X[i][j] = XT[j][i] (64 x 64 tiles through LDS) and cost = sum C_ij X_ij
// (int64, one atomic per tile).  Skipped when the solve failed.
__global__ __launch_bounds__(256) void k_bins_finish(const int32_t *XT, const int32_t *C, int n, int m, int ld,
                                                     int32_t *X, int64_t *cost, const int32_t *gate,
                                                     const ot_stats *stats) {
  if (*gate != 0 || stats->status != 0) return;
  __shared__ int32_t tile[64][65];
  __shared__ long long s_cost;
  const int bi = blockIdx.y * 64, bj = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_cost = 0;
  for (int q = ty; q < 64; q += 4) {
    const int j = bj + q, i = bi + tx;
    if (i < n && j < m) tile[q][tx] = XT[(size_t)j * n + i];
  }
  __syncthreads();
  long long part = 0;
  for (int q = ty; q < 64; q += 4) {
    const int i = bi + q, j = bj + tx;
    if (i < n && j < m) {
      const int32_t x = tile[tx][q];
      X[(size_t)i * m + j] = x;
      part += (long long)x * C[(size_t)i * ld + j];
    }
  }
  part = wave_sum_i64(part);
  if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long *)&s_cost, (unsigned long long)part);
  __syncthreads();
  if (threadIdx.x == 0 && s_cost != 0) atomicAdd((unsigned long long *)cost, (unsigned long long)s_cost);
}

// Zero-mass bins get the tightest feasible duals, as ot_transport's:
// a zero-mass row u_i = min over columns with mass of C_ij - v_j (one
// wavefront per row), then a zero-mass column v_j = min_i C_ij - u_i.
__global__ __launch_bounds__(256) void k_bins_zero_rows(const int32_t *C, int ld, const int32_t *r, const int32_t *c,
                                                        int n, int m, int64_t *u, const int64_t *v,
                                                        const int32_t *gate, const ot_stats *stats) {
  if (*gate != 0 || stats->status != 0) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n || r[i] != 0) return;
  int64_t best = INT64_MAX;
  for (int j = lane; j < m; j += 64)
    if (c[j] > 0) best = min(best, (int64_t)C[(size_t)i * ld + j] - v[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = min(best, (int64_t)__shfl_xor(best, off, 64));
  if (lane == 0) u[i] = best;
}

__global__ void k_bins_zero_cols(const int32_t *C, int ld, const int32_t *c, int n, int m, const int64_t *u,
                                 int64_t *v, const int32_t *gate, const ot_stats *stats) {
  if (*gate != 0 || stats->status != 0) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m || c[j] != 0) return;
  int64_t best = INT64_MAX;
  for (int i = 0; i < n; ++i) best = min(best, (int64_t)C[(size_t)i * ld + j] - u[i]);
  v[j] = best;
}

template <int B, int CPT>
static hipError_t bins_one(const BinsProblem &P, const int32_t *gate, hipStream_t s) {
  const size_t lds = bins_lds(P.n, P.m).total;
  hipError_t e = hipFuncSetAttribute((const void *)k_bins<B, CPT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_bins<B, CPT>), dim3(1), dim3(B), lds, s, P, gate);
  return hipGetLastError();
}

// One workgroup: 64 lanes while 8 columns per lane cover m, else 512.
static hipError_t launch_bins(const BinsProblem &P, const int32_t *gate, hipStream_t s) {
  const int block = P.m <= 512 ? 64 : 512;
  const int cpt = cpt_for(P.m, block);
#define OTKM_BINS(B, K) if (block == B && cpt == K) return bins_one<B, K>(P, gate, s);
  OTKM_BINS(64, 1) OTKM_BINS(64, 2) OTKM_BINS(64, 4) OTKM_BINS(64, 8)
  OTKM_BINS(512, 1) OTKM_BINS(512, 2) OTKM_BINS(512, 4) OTKM_BINS(512, 8)
#undef OTKM_BINS
  return hipErrorInvalidValue;
}

// The whole pipeline on device buffers; `get(slot, bytes)` hands out workspace.
template <class Get>
static int bins_pipeline(const int32_t *dC, const int32_t *dr, const int32_t *dc, int n, int m, int ld, Get get,
                         hipStream_t s, int32_t *dX, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats) {
  const int B = std::max(n, m);
  auto *XT = (int32_t *)get(0, 4 * (size_t)n * (size_t)m);
  auto *ws = (int32_t *)get(1, 4 * ws_ints(B));
  auto *u0 = (int64_t *)get(2, 8 * (size_t)n);
  auto *rmax = (int32_t *)get(3, 4 * (size_t)n);
  auto *part = (uint64_t *)get(4, init_part_bytes(n, m));
  auto *b = (uint64_t *)get(5, 16 * (size_t)m);
  auto *gate = (int32_t *)get(6, 16);
  auto *st = dstats ? dstats : (ot_stats *)get(7, sizeof(ot_stats));
  if (!XT || !ws || !u0 || !rmax || !part || !b || !gate || !st) return OT_ENOMEM;
  hipError_t e;
  hipLaunchKernelGGL(k_bins_check, dim3(1), dim3(1024), 0, s, dr, dc, n, m, gate, st);
  if ((e = hipGetLastError()) != hipSuccess) return map_hip(e);
  if ((e = launch_init_sweeps(dC, n, m, ld, u0, rmax, part, b, s)) != hipSuccess) return map_hip(e);
  if ((e = launch_fill_i32(XT, 0, (int64_t)n * m, s)) != hipSuccess) return map_hip(e);
  if ((e = launch_fill_i32((int32_t *)dcost, 0, 2, s)) != hipSuccess) return map_hip(e);
  BinsProblem P;
  P.C = dC; P.CT = nullptr; P.n = n; P.m = m; P.ld = ld;
  P.init_u = u0; P.init_b = b; P.init_rmax = rmax;
  P.r = dr; P.c = dc; P.XT = XT; P.u = du; P.v = dv; P.stats = st; P.ws = ws;
  if ((e = launch_bins(P, gate, s)) != hipSuccess) return map_hip(e);
  hipLaunchKernelGGL(k_bins_finish, dim3((m + 63) / 64, (n + 63) / 64), dim3(256), 0, s, XT, dC, n, m, ld, dX, dcost,
                     gate, st);
  if ((e = hipGetLastError()) != hipSuccess) return map_hip(e);
  hipLaunchKernelGGL(k_bins_zero_rows, dim3((n + 3) / 4), dim3(256), 0, s, dC, ld, dr, dc, n, m, du, dv, gate, st);
  if ((e = hipGetLastError()) != hipSuccess) return map_hip(e);
  hipLaunchKernelGGL(k_bins_zero_cols, dim3((m + 255) / 256), dim3(256), 0, s, dC, ld, dc, n, m, du, dv, gate, st);
  return map_hip(hipGetLastError());
}

static int bins_shape_ok(int n, int m) {
  if (n <= 0 || m <= 0) return OT_EINVAL;
  if (n > OT_MAX_BINS || m > OT_MAX_BINS) return OT_ETOOBIG;
  return OT_OK;
}

}  // namespace otkm

using namespace otkm;

extern "C" {

int ot_transport_bins(const int32_t *C, const int32_t *r, const int32_t *c, int32_t n, int32_t m, int32_t *X,
                      int64_t *cost, int64_t *u, int64_t *v, ot_stats *stats) {
  if (!C || !r || !c || !X || !cost) return OT_EINVAL;
  int rc = bins_shape_ok(n, m);
  if (rc) return rc;
  int64_t sr = 0, sc = 0;
  for (int i = 0; i < n; ++i) { if (r[i] < 0) return OT_ENEGMASS; sr += r[i]; }
  for (int j = 0; j < m; ++j) { if (c[j] < 0) return OT_ENEGMASS; sc += c[j]; }
  if (sr != sc || sr < 1) return OT_EUNBALANCED;
  if (sr > 0x7fffffffll) return OT_ETOOBIG;
  {
    const size_t NM = (size_t)n * (size_t)m;
    int32_t mn = C[0], mx = C[0];
    for (size_t k = 1; k < NM; ++k) { mn = std::min(mn, C[k]); mx = std::max(mx, C[k]); }
    if ((int64_t)mx - (int64_t)mn > 0x7fffffffll) return OT_ERANGE;
  }
  std::lock_guard<std::mutex> lk(lib_mutex());
  if ((rc = init_locked())) return rc;
  int err = OT_OK;
  const size_t NM = (size_t)n * (size_t)m;
  hipStream_t s = lib_stream();
  auto *dC = (int32_t *)pool_get(120, 4 * NM, &err);
  auto *dr = (int32_t *)pool_get(121, 4 * (size_t)n, &err);
  auto *dc = (int32_t *)pool_get(122, 4 * (size_t)m, &err);
  auto *dX = (int32_t *)pool_get(123, 4 * NM, &err);
  auto *dcost = (int64_t *)pool_get(124, 16, &err);
  auto *du = (int64_t *)pool_get(125, 8 * (size_t)n, &err);
  auto *dv = (int64_t *)pool_get(126, 8 * (size_t)m, &err);
  auto *dst = (ot_stats *)pool_get(127, sizeof(ot_stats), &err);
  if (err) return err;
  hipError_t e;
  if ((e = hipMemcpyAsync(dC, C, 4 * NM, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(dr, r, 4 * (size_t)n, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(dc, c, 4 * (size_t)m, hipMemcpyHostToDevice, s)) != hipSuccess) return map_hip(e);
  auto get = [&](int slot, size_t bytes) { return pool_get(130 + slot, bytes, &err); };
  rc = bins_pipeline(dC, dr, dc, n, m, m, get, s, dX, dcost, du, dv, dst);
  if (err) return err;
  if (rc) return rc;
  ot_stats hs;
  std::vector<int32_t> hX(NM);
  std::vector<int64_t> hu(n), hv(m);
  int64_t hcost = 0;
  if ((e = hipMemcpyAsync(&hs, dst, sizeof hs, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hX.data(), dX, 4 * NM, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hu.data(), du, 8 * (size_t)n, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(hv.data(), dv, 8 * (size_t)m, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipMemcpyAsync(&hcost, dcost, 8, hipMemcpyDeviceToHost, s)) != hipSuccess) return map_hip(e);
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return map_hip(e);
  if (hs.status != 0) return (int)hs.status;
  std::memcpy(X, hX.data(), 4 * NM);
  *cost = hcost;
  if (u) std::memcpy(u, hu.data(), 8 * (size_t)n);
  if (v) std::memcpy(v, hv.data(), 8 * (size_t)m);
  if (stats) *stats = hs;
  return OT_OK;
}

int ot_transport_bins_dev(const int32_t *dC, const int32_t *dr, const int32_t *dc, int32_t n, int32_t m, int32_t ld,
                          int32_t *dX, int64_t *dcost, int64_t *du, int64_t *dv, ot_stats *dstats, void *stream) {
  if (!dC || !dr || !dc || !dX || !dcost || !du || !dv || ld < m) return OT_EINVAL;
  int rc = bins_shape_ok(n, m);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(lib_mutex());
  if ((rc = init_locked())) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : lib_stream();
  int err = OT_OK;
  auto get = [&](int slot, size_t bytes) { return stream_ws(s, 130 + slot, bytes, &err); };
  rc = bins_pipeline(dC, dr, dc, n, m, ld, get, s, dX, dcost, du, dv, dstats);
  return err ? err : rc;
}

}  // extern "C"
