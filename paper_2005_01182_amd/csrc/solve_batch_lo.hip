// solve_batch_lo.hip -- persistent batch kernel, widths 64 and 256.
#include <hip/hip_runtime.h>

#include "solve_kernels.hpp"

namespace otkm {

hipError_t launch_assign_batch_lo(const BatchArgs &A, int block, int cpt, int grid, hipStream_t s) {
#define OTKM_BATCH(B, K) if (block == B && cpt == K) return batch<B, K>(A, grid, s);
  OTKM_BATCH(64, 1) OTKM_BATCH(64, 2) OTKM_BATCH(64, 4) OTKM_BATCH(64, 8)
  OTKM_BATCH(256, 1) OTKM_BATCH(256, 2) OTKM_BATCH(256, 4) OTKM_BATCH(256, 8)
#undef OTKM_BATCH
  return hipErrorInvalidValue;
}

int batch_occupancy_lo(int block, int cpt, int max_n) {
#define OTKM_OCC(B, K) if (block == B && cpt == K) return occ<B, K>(max_n);
  OTKM_OCC(64, 1) OTKM_OCC(64, 2) OTKM_OCC(64, 4) OTKM_OCC(64, 8)
  OTKM_OCC(256, 1) OTKM_OCC(256, 2) OTKM_OCC(256, 4) OTKM_OCC(256, 8)
#undef OTKM_OCC
  return -1;
}

}  // namespace otkm
