// Device-side helpers shared by the kernels: table offsets, complex arithmetic,
// wavefront reductions, local-node index maps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hps {

// Block precisions (storage of the dense preconditioner blocks).
enum BlockPrec { kFP64 = 0, kFP32 = 1, kBF16 = 2 };

// Offsets (in doubles) inside the packed device table  D | D2 | V | W | E | xi | Ed3.
__host__ __device__ constexpr int tab_off_D(int p) { return 0; }
__host__ __device__ constexpr int tab_off_D2(int p) { return p * p; }
__host__ __device__ constexpr int tab_off_V(int p) { return 2 * p * p; }
__host__ __device__ constexpr int tab_off_W(int p) { return 2 * p * p + (p - 2) * (p - 2); }
__host__ __device__ constexpr int tab_off_E(int p) { return 2 * p * p + 2 * (p - 2) * (p - 2); }
__host__ __device__ constexpr int tab_off_xi(int p) { return tab_off_E(p) + (p - 2); }
__host__ __device__ constexpr int tab_off_ed3(int p) { return tab_off_xi(p) + p; }
__host__ __device__ constexpr int tab_size(int p) {
  return tab_off_ed3(p) + (p - 2) * (p - 2) * (p - 2);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// acc += s * a  (real s)
__device__ __forceinline__ void cfma_r(double2& acc, double s, double2 a) {
  acc.x = fma(s, a.x, acc.x);
  acc.y = fma(s, a.y, acc.y);
}

// 16-byte non-temporal loads (streamed data that is not reused soon)
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 ld_nt(const double2* p) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld_nt(const uint4* p) {
  const nt_u4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace hps
