// FP64 access to stored deviations for the non-hot kernels (conversions,
// diagnostics, boundary rules): Raw<S>::get widens a stored value exactly,
// Raw<S>::put rounds an FP64 value once to the storage format (S = 0 FP32,
// 1 FP16, 2 BF16; the caller applies the storage scale).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace elbm {

template <int S>
struct Raw;
template <>
struct Raw<0> {
  using T = float;
  __device__ static double get(const T* p) { return double(*p); }
  __device__ static void put(T* p, double v) { *p = float(v); }
};
// FP64 -> FP32 with round-to-odd: a following round-to-nearest-even to a
// format with at least two fewer significand bits then rounds the FP64 value
// correctly (no double rounding).
__device__ __forceinline__ float to_f32_odd(double v) {
  float f = float(v);
  const double back = double(f);
  if (back != v) {
    unsigned int b = __float_as_uint(f);
    if ((b & 1u) == 0u) b += fabs(v) > fabs(back) ? 1u : 0xFFFFFFFFu;
    f = __uint_as_float(b);
  }
  return f;
}

template <>
struct Raw<1> {
  using T = __half;
  __device__ static double get(const T* p) { return double(__half2float(*p)); }
  __device__ static void put(T* p, double v) { *p = __float2half_rn(to_f32_odd(v)); }
};
template <>
struct Raw<2> {
  using T = __hip_bfloat16;
  __device__ static double get(const T* p) { return double(__bfloat162float(*p)); }
  __device__ static void put(T* p, double v) { *p = __float2bfloat16(to_f32_odd(v)); }
};

}  // namespace elbm
