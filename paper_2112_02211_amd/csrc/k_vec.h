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
// Vectors are stored with the non-temporal hint everywhere: every output of the
// hot path (the sweep's y and face buffer, J^-1's y, the Krylov passes'
// vectors) is a stream of 7 MB to hundreds of MB that the next kernel reads
// from HBM anyway (measured: 16^3 solve 131.6 -> 129.2 ms, 8^3 15.2 -> 14.9 ms;
// FP32 stores: the refinement solve 125.5 -> 124.5 ms).
__device__ __forceinline__ void st2(double2* p, int64_t i, double2 v) {
  typedef double vd2 __attribute__((ext_vector_type(2)));
  vd2 t;
  t.x = v.x;
  t.y = v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<vd2*>(p + i));
}
__device__ __forceinline__ void st2(float2* p, int64_t i, double2 v) {
  typedef float vf2 __attribute__((ext_vector_type(2)));
  vf2 t;
  t.x = (float)v.x;
  t.y = (float)v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<vf2*>(p + i));
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
// Non-temporal loads (streamed data that is not read again soon: the Krylov
// basis of a long vector).
typedef double vnt_d2 __attribute__((ext_vector_type(2)));
typedef float vnt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_nt2(const double2* p) {
  const vnt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const vnt_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_nt2(const float2* p) {
  const vnt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const vnt_f2*>(p));
  return make_float2(v.x, v.y);
}
template <bool NT>
__device__ __forceinline__ double2 ld_tile_h(const double2* p, int64_t i, int64_t i_safe, bool c) {
  if constexpr (NT) return c ? ld_nt2(p + i) : make_double2(0.0, 0.0);
  else return ld_tile(p, i, i_safe, c);
}
template <bool NT>
__device__ __forceinline__ float2 ld_tile_h(const float2* p, int64_t i, int64_t i_safe, bool c) {
  if constexpr (NT) return ld_nt2(p + (c ? i : i_safe));
  else return ld_tile(p, i, i_safe, c);
}
// The value a store of v to storage of the pointer's type keeps, widened again.
__device__ __forceinline__ double2 as_stored(double2 v, const double2*) { return v; }
__device__ __forceinline__ double2 as_stored(double2 v, const float2*) {
  return make_double2((double)(float)v.x, (double)(float)v.y);
}
__device__ __forceinline__ double2 widen(float2 v, bool c) {
  return c ? make_double2((double)v.x, (double)v.y) : make_double2(0.0, 0.0);
}

}  // namespace hps
