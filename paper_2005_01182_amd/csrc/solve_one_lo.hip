// solve_one_lo.hip -- one instance per workgroup, widths 64 and 256.
#include <hip/hip_runtime.h>

#include "solve_kernels.hpp"

namespace otkm {

hipError_t launch_assign_one_lo(const Problem &P, int block, int cpt, const int32_t *gate, hipStream_t s) {
#define OTKM_ONE(B, K) if (block == B && cpt == K) return one<B, K>(P, gate, s);
  OTKM_ONE(64, 1) OTKM_ONE(64, 2) OTKM_ONE(64, 4) OTKM_ONE(64, 8)
  OTKM_ONE(256, 1) OTKM_ONE(256, 2) OTKM_ONE(256, 4) OTKM_ONE(256, 8)
#undef OTKM_ONE
  return hipErrorInvalidValue;
}

}  // namespace otkm
