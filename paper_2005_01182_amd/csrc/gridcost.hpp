// gridcost.hpp -- exactly rounded Euclidean distance between integer points.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace otkm {

// round(sqrt(d)) for 0 <= d < 2^62: floor(sqrt(d)) from the double estimate,
// corrected to the exact integer, plus one when d - k^2 > k (sqrt(d) is never
// exactly k + 1/2 for integer d, so there are no ties)
__device__ __forceinline__ int32_t grid_isqrt_round(int64_t d) {
  int64_t k = (int64_t)sqrt((double)d);
  while (k * k > d) --k;
  while ((k + 1) * (k + 1) <= d) ++k;
  return (int32_t)(k + ((d - k * k) > k ? 1 : 0));
}

}  // namespace otkm
