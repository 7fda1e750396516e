// bf16.hpp -- binary32 to bfloat16 bit pattern, round to nearest even (NaN
// stays a quiet NaN); shared by the flagger kernels and the stage kernel's
// fused feature pooling.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amrv {

__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

}  // namespace amrv
