// sparse.hip -- assignment on a sparse cost graph (CSR): kernels and the
// C-ABI calls ot_assign_sparse, ot_assign_sparse_dev and
// ot_assign_sparse_batch_dev.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "launch.hpp"
#include "otkm.h"
#include "runtime.hpp"
#include "sparse_engine.hpp"

namespace otkm {
namespace {

// one instance, one workgroup, the forest kept across augmentations
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_sparse_one(SparseProblem P) {
  extern __shared__ __align__(16) char smem[];
  SparseEngine<BLOCK, true> E;
  E.run(P, smem);
}

// many instances: each workgroup takes one descriptor from the queue and
// solves it (the launch has one workgroup per instance)
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_sparse_batch(const ot_sparse_desc *desc, int count, int max_m,
                                                         int32_t *head) {
  extern __shared__ __align__(16) char smem[];
  __shared__ int s_k;
  if (threadIdx.x == 0) s_k = atomicAdd(head, 1);
  __syncthreads();
  const int k = s_k;
  if (k >= count) return;  // uniform across the workgroup
  const ot_sparse_desc d = desc[k];
  if (d.n < 1 || d.m < d.n || d.m > max_m || !d.ptr || !d.plan || !d.total) {
    if (threadIdx.x == 0 && d.stats) {
      ot_stats s = {};
      s.status = OT_EINVAL;
      *d.stats = s;
    }
    return;
  }
  SparseProblem P;
  P.ptr = d.ptr; P.idx = d.idx; P.cost = d.cost; P.n = d.n; P.m = d.m;
  P.plan = d.plan; P.total = d.total; P.u = d.u; P.v = d.v; P.stats = d.stats;
  SparseEngine<BLOCK> E;
  E.run(P, smem);
}

int block_for(int m) { return m <= 256 ? 64 : 256; }

template <auto KERNEL>
hipError_t set_lds(size_t bytes) {
  return hipFuncSetAttribute((const void *)KERNEL, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_sparse_one(const SparseProblem &P, hipStream_t s) {
  const size_t lds = sparse_lds(P.n, P.m).total;
  hipError_t e;
  if (block_for(P.m) == 64) {
    if ((e = set_lds<k_sparse_one<64>>(lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sparse_one<64>, dim3(1), dim3(64), lds, s, P);
  } else {
    if ((e = set_lds<k_sparse_one<256>>(lds)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sparse_one<256>, dim3(1), dim3(256), lds, s, P);
  }
  return hipGetLastError();
}

// Workgroups of the batch kernel resident at once for instances of at most
// max_m columns (0 on error).
template <int BLOCK>
int sparse_batch_slots(int max_m) {
  const size_t lds = sparse_lds(max_m, max_m).total;
  if (set_lds<k_sparse_batch<BLOCK>>(lds) != hipSuccess) return 0;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_sparse_batch<BLOCK>, BLOCK, lds) != hipSuccess)
    return 0;
  return std::max(1, occ) * device_cus();
}

template <int BLOCK>
hipError_t launch_sparse_batch_t(const ot_sparse_desc *desc, int count, int max_m, int32_t *head, hipStream_t s) {
  const size_t lds = sparse_lds(max_m, max_m).total;
  const int grid = std::max(1, count);  // the caller has checked count against the resident slots
  hipLaunchKernelGGL(k_sparse_batch<BLOCK>, dim3(grid), dim3(BLOCK), lds, s, desc, count, max_m, head);
  return hipGetLastError();
}

// Host-side check of a CSR graph: offsets from 0, non-decreasing, columns in
// range, no column twice in a row.
int validate_csr(const int64_t *ptr, const int32_t *idx, int32_t n, int32_t m) {
  if (ptr[0] != 0) return OT_EINVAL;
  std::vector<int32_t> mark((size_t)m, -1);
  for (int32_t i = 0; i < n; ++i) {
    if (ptr[i + 1] < ptr[i]) return OT_EINVAL;
    for (int64_t q = ptr[i]; q < ptr[i + 1]; ++q) {
      const int32_t j = idx[q];
      if (j < 0 || j >= m || mark[(size_t)j] == i) return OT_EINVAL;
      mark[(size_t)j] = i;
    }
  }
  return OT_OK;
}

}  // namespace
}  // namespace otkm

using namespace otkm;

extern "C" {

int ot_assign_sparse(const int64_t *ptr, const int32_t *idx, const int32_t *cost, int32_t n, int32_t m,
                     int32_t *plan, int64_t *total, int64_t *u, int64_t *v, ot_stats *stats) {
  if (!ptr || !plan || !total || n <= 0 || m < n) return OT_EINVAL;
  if (m > OT_MAX_N) return OT_ETOOBIG;
  const int64_t nnz = ptr[n];
  if (nnz > 0 && (!idx || !cost)) return OT_EINVAL;
  int rc = validate_csr(ptr, idx, n, m);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(lib_mutex());
  if ((rc = init_locked())) return rc;
  hipStream_t s = lib_stream();
  int err = OT_OK;
  const size_t E = (size_t)std::max<int64_t>(nnz, 1);
  auto *dptr = (int64_t *)pool_get(200, 8 * ((size_t)n + 1), &err);
  auto *didx = (int32_t *)pool_get(201, 4 * E, &err);
  auto *dcost = (int32_t *)pool_get(202, 4 * E, &err);
  auto *dplan = (int32_t *)pool_get(203, 4 * (size_t)n, &err);
  auto *du = (int64_t *)pool_get(204, 8 * (size_t)n, &err);
  auto *dv = (int64_t *)pool_get(205, 8 * (size_t)m, &err);
  auto *dtot = (int64_t *)pool_get(206, 8, &err);
  auto *dst = (ot_stats *)pool_get(207, sizeof(ot_stats), &err);
  auto *dcolptr = (int32_t *)pool_get(208, 4 * ((size_t)m + 1), &err);
  auto *dcrow = (int32_t *)pool_get(209, 4 * E, &err);
  auto *dccost = (int32_t *)pool_get(210, 4 * E, &err);
  if (err) return err;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chk(hipMemcpyAsync(dptr, ptr, 8 * ((size_t)n + 1), hipMemcpyHostToDevice, s));
  if (nnz > 0) {
    chk(hipMemcpyAsync(didx, idx, 4 * (size_t)nnz, hipMemcpyHostToDevice, s));
    chk(hipMemcpyAsync(dcost, cost, 4 * (size_t)nnz, hipMemcpyHostToDevice, s));
  }
  SparseProblem P;
  P.ptr = dptr; P.idx = didx; P.cost = dcost; P.n = n; P.m = m;
  P.plan = dplan; P.total = dtot; P.u = du; P.v = dv; P.stats = dst;
  P.colptr = dcolptr; P.crow = dcrow; P.ccost = dccost; P.cap = (int64_t)E;
  if (e == hipSuccess) chk(launch_sparse_one(P, s));
  ot_stats hs{};
  chk(hipMemcpyAsync(&hs, dst, sizeof(ot_stats), hipMemcpyDeviceToHost, s));
  chk(hipStreamSynchronize(s));
  if (e != hipSuccess) return map_hip(e);
  if (stats) *stats = hs;
  if (hs.status != OT_OK) return (int)hs.status;
  chk(hipMemcpyAsync(plan, dplan, 4 * (size_t)n, hipMemcpyDeviceToHost, s));
  chk(hipMemcpyAsync(total, dtot, 8, hipMemcpyDeviceToHost, s));
  if (u) chk(hipMemcpyAsync(u, du, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  if (v) chk(hipMemcpyAsync(v, dv, 8 * (size_t)m, hipMemcpyDeviceToHost, s));
  chk(hipStreamSynchronize(s));
  return map_hip(e);
}

int ot_assign_sparse_dev(const int64_t *dptr, const int32_t *didx, const int32_t *dcost, int32_t n, int32_t m,
                         int64_t nnz, int32_t *dplan, int64_t *dtotal, int64_t *du, int64_t *dv, ot_stats *dstats,
                         void *stream) {
  if (!dptr || !dplan || !dtotal || n <= 0 || m < n || nnz < 0) return OT_EINVAL;
  if (nnz > 0 && (!didx || !dcost)) return OT_EINVAL;
  if (m > OT_MAX_N || nnz > (int64_t)INT32_MAX) return OT_ETOOBIG;  // column offsets are 32-bit
  std::lock_guard<std::mutex> lk(lib_mutex());
  int rc = init_locked();
  if (rc) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : lib_stream();
  int err = OT_OK;
  const size_t E = (size_t)std::max<int64_t>(nnz, 1);
  auto *dcolptr = (int32_t *)stream_ws(s, 200, 4 * ((size_t)m + 1), &err);
  auto *dcrow = (int32_t *)stream_ws(s, 201, 4 * E, &err);
  auto *dccost = (int32_t *)stream_ws(s, 202, 4 * E, &err);
  if (err) return err;
  SparseProblem P;
  P.ptr = dptr; P.idx = didx; P.cost = dcost; P.n = n; P.m = m;
  P.plan = dplan; P.total = dtotal; P.u = du; P.v = dv; P.stats = dstats;
  P.colptr = dcolptr; P.crow = dcrow; P.ccost = dccost; P.cap = nnz;
  return map_hip(launch_sparse_one(P, s));
}

int ot_assign_sparse_batch_dev(int32_t count, const ot_sparse_desc *ddesc, int32_t max_m, void *stream) {
  if (count < 0 || (count > 0 && !ddesc) || max_m < 1) return OT_EINVAL;
  if (max_m > OT_MAX_N) return OT_ETOOBIG;
  if (count == 0) return OT_OK;
  std::lock_guard<std::mutex> lk(lib_mutex());
  int rc = init_locked();
  if (rc) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : lib_stream();
  // at most one instance per resident workgroup: a launch whose workgroups
  // would take further instances from the queue faulted the GPU once on
  // MI355X (4096 k-NN instances, n <= 512) and is refused until its cause is
  // found
  const int slots = block_for(max_m) == 64 ? sparse_batch_slots<64>(max_m) : sparse_batch_slots<256>(max_m);
  if (slots <= 0) return OT_EINTERNAL;
  if (count > slots) return OT_ETOOBIG;
  int err = OT_OK;
  auto *head = (int32_t *)stream_ws(s, 203, 256, &err);
  if (err) return err;
  hipError_t e = launch_fill_i32(head, 0, 1, s);
  if (e != hipSuccess) return map_hip(e);
  e = block_for(max_m) == 64 ? launch_sparse_batch_t<64>(ddesc, count, max_m, head, s)
                             : launch_sparse_batch_t<256>(ddesc, count, max_m, head, s);
  return map_hip(e);
}

}  // extern "C"
