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

// Loads of a predicated tile (entry i under predicate c): FP64 storage keeps the
// predicated load; FP32 storage loads unconditionally from i, or from the
// in-bounds i_safe when c is false, so that no branch sits between one load
// and the next and the widening conversions wait for all loads at once (a
// conversion inside each predicated branch makes every load wait for itself).
// widen() gives the FP64 value, zero where the predicate was false.
__device__ __forceinline__ double2 ld_tile(const double2* p, int64_t i, int64_t, bool c) {
  return c ? p[i] : make_double2(0.0, 0.0);
}
__device__ __forceinline__ float2 ld_tile(const float2* p, int64_t i, int64_t i_safe, bool c) {
  return p[c ? i : i_safe];
}
__device__ __forceinline__ double2 widen(double2 v, bool) { return v; }
__device__ __forceinline__ double2 widen(float2 v, bool c) {
  return c ? make_double2((double)v.x, (double)v.y) : make_double2(0.0, 0.0);
}

}  // namespace hps
