// solve_one_hi.hip -- one instance per workgroup, widths 512 and 1024.
#include <hip/hip_runtime.h>

#include "solve_kernels.hpp"

namespace otkm {

hipError_t launch_assign_one_hi(const Problem &P, int block, int cpt, const int32_t *gate, hipStream_t s) {
#define OTKM_ONE(B, K) if (block == B && cpt == K) return one<B, K>(P, gate, s);
  OTKM_ONE(512, 1) OTKM_ONE(512, 2) OTKM_ONE(512, 4) OTKM_ONE(512, 8)
  OTKM_ONE(1024, 1) OTKM_ONE(1024, 2) OTKM_ONE(1024, 4)
#undef OTKM_ONE
  return hipErrorInvalidValue;
}

}  // namespace otkm
