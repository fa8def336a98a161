// solve_grid.hip -- one instance over several workgroups.
#include <hip/hip_runtime.h>

#include "solve_kernels.hpp"

namespace otkm {

__global__ void k_fill_u64(uint64_t *p, uint64_t value, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

hipError_t launch_assign_grid(const Problem &P, int block, int wgs, hipStream_t s) {
  if (wgs < 2 || wgs > kMaxWgs || !P.grid_ws) return hipErrorInvalidValue;
  const int cpt = cpt_for(P.n, block * wgs);
#define OTKM_GRID(B, K) if (block == B && cpt == K) return grid<B, K>(P, wgs, s);
  OTKM_GRID(256, 1) OTKM_GRID(256, 2) OTKM_GRID(256, 4)
  OTKM_GRID(512, 1) OTKM_GRID(512, 2) OTKM_GRID(512, 4)
#undef OTKM_GRID
  return hipErrorInvalidValue;
}

}  // namespace otkm
