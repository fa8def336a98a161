// solve_batch_hi.hip -- persistent batch kernel, widths 512 and 1024.
#include <hip/hip_runtime.h>

#include "solve_kernels.hpp"

namespace otkm {

hipError_t launch_assign_batch_hi(const BatchArgs &A, int block, int cpt, int grid, hipStream_t s) {
#define OTKM_BATCH(B, K) if (block == B && cpt == K) return batch<B, K>(A, grid, s);
  OTKM_BATCH(512, 1) OTKM_BATCH(512, 2) OTKM_BATCH(512, 4) OTKM_BATCH(512, 8)
  OTKM_BATCH(1024, 1) OTKM_BATCH(1024, 2) OTKM_BATCH(1024, 4)
#undef OTKM_BATCH
  return hipErrorInvalidValue;
}

int batch_occupancy_hi(int block, int cpt, int max_n) {
#define OTKM_OCC(B, K) if (block == B && cpt == K) return occ<B, K>(max_n);
  OTKM_OCC(512, 1) OTKM_OCC(512, 2) OTKM_OCC(512, 4) OTKM_OCC(512, 8)
  OTKM_OCC(1024, 1) OTKM_OCC(1024, 2) OTKM_OCC(1024, 4)
#undef OTKM_OCC
  return -1;
}

}  // namespace otkm
