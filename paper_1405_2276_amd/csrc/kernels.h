// Device helpers shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

namespace fkf {

typedef double v2d __attribute__((ext_vector_type(2)));

// Sum over the 64 lanes of a wavefront (butterfly; every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

}  // namespace fkf
