// Vectors stored as complex FP64 (double2) or complex FP32 (float2): loads widen
// to FP64, stores round to the storage type; the arithmetic is FP64 either way.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hps {

// Vectors stored as complex FP64 (double2) or complex FP32 (float2): loads widen
// to FP64, stores round to the storage type; the arithmetic is FP64 either way.
__device__ __forceinline__ double2 ld2(const double2* p, int64_t i) { return p[i]; }
__device__ __forceinline__ double2 ld2(const float2* p, int64_t i) {
  const float2 v = p[i];
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ void st2(double2* p, int64_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void st2(float2* p, int64_t i, double2 v) {
  p[i] = make_float2((float)v.x, (float)v.y);
}

}  // namespace hps
