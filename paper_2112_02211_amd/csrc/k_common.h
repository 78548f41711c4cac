// Device-side helpers shared by the kernels: table offsets, complex arithmetic,
// wavefront reductions, local-node index maps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hps {

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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace hps
