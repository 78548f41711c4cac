// Device routines on one leaf shared by the preconditioner kernels: the fast
// diagonalization of the homogenized interior operator (Sec. 4.1, Algorithm 3)
// as line-wise mode products in LDS, and the sparse face couplings F_bi and A_ib.
#pragma once

#include "k_common.h"

namespace hps {

// In-place mode product along axis AX of the n1^3 tensor T by the n1 x n1
// row-major matrix M: T[.., a, ..] <- sum_i M[a][i] T[.., i, ..].
template <int P, int AX, int BD>
__device__ __forceinline__ void mode_product(double2* __restrict__ T, const double* __restrict__ M) {
  constexpr int N1 = P - 2, L = N1 * N1;
  for (int line = threadIdx.x; line < L; line += BD) {
    const int a = line % N1, b = line / N1;
    int base, stride;
    if (AX == 0) { base = N1 * a + L * b; stride = 1; }
    else if (AX == 1) { base = a + L * b; stride = N1; }
    else { base = a + N1 * b; stride = L; }
    double2 v[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) v[i] = T[base + i * stride];
#pragma unroll
    for (int o = 0; o < N1; ++o) {
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < N1; ++i) cfma_r(s, M[o * N1 + i], v[i]);
      T[base + o * stride] = s;
    }
  }
}

// T <- A~_ii^{-1} T = (V x V x V) diag(1 / (-E_Delta - lambda)) (W x W x W) T
template <int P, int BD>
__device__ __forceinline__ void homog_solve(double2* __restrict__ T, const double* __restrict__ tab,
                                            double2 lam) {
  constexpr int NI = (P - 2) * (P - 2) * (P - 2);
  const double* V = tab + tab_off_V(P);
  const double* W = tab + tab_off_W(P);
  const double* Ed3 = tab + tab_off_ed3(P);
  mode_product<P, 0, BD>(T, W);
  __syncthreads();
  mode_product<P, 1, BD>(T, W);
  __syncthreads();
  mode_product<P, 2, BD>(T, W);
  __syncthreads();
  for (int m = threadIdx.x; m < NI; m += BD) {
    // 1 / (a + i b), a = -E - lr, b = -li
    const double a = -Ed3[m] - lam.x, b = -lam.y;
    const double den = 1.0 / (a * a + b * b);
    T[m] = cmul(T[m], make_double2(a * den, -b * den));
  }
  __syncthreads();
  mode_product<P, 0, BD>(T, V);
  __syncthreads();
  mode_product<P, 1, BD>(T, V);
  __syncthreads();
  mode_product<P, 2, BD>(T, V);
  __syncthreads();
}

// Element-parallel form of the same product: one output element per thread,
// out[.., a, ..] = sum_i M[a][i] in[.., i, ..], with M (row major) in LDS.
// Same terms in the same order as mode_product, so the results are identical;
// n1^3 threads work instead of n1^2.
template <int P, int AX, int BD>
__device__ __forceinline__ void mode_product_el(const double2* __restrict__ in,
                                                double2* __restrict__ out,
                                                const double* __restrict__ M) {
  constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L;
  constexpr int stride = AX == 0 ? 1 : (AX == 1 ? N1 : L);
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int o = (m / stride) % N1;
    const int base = m - o * stride;
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < N1; ++i) cfma_r(s, M[o * N1 + i], in[base + i * stride]);
    out[m] = s;
  }
}

// The element-parallel form needs an extra n1^3 LDS tensor; used up to p = 14.
template <int P>
constexpr bool kElementParallel = (P <= 14);

// WV = [W | V] (V^{-1} and V, n1^2 each) from the shared table into LDS
template <int P, int BD>
__device__ __forceinline__ void stage_wv(double* __restrict__ WV, const double* __restrict__ tab) {
  constexpr int Q = (P - 2) * (P - 2);
  for (int k = threadIdx.x; k < 2 * Q; k += BD)
    WV[k] = k < Q ? tab[tab_off_W(P) + k] : tab[tab_off_V(P) + k - Q];
}

// T <- A~_ii^{-1} T as homog_solve, element-parallel: X is an LDS scratch of
// n1^3 entries, WV = [W | V] (n1^2 each) staged in LDS.
template <int P, int BD>
__device__ __forceinline__ void homog_solve_el(double2* __restrict__ T, double2* __restrict__ X,
                                               const double* __restrict__ WV,
                                               const double* __restrict__ tab, double2 lam) {
  constexpr int N1 = P - 2, NI = N1 * N1 * N1;
  const double* W = WV;
  const double* V = WV + N1 * N1;
  const double* Ed3 = tab + tab_off_ed3(P);
  mode_product_el<P, 0, BD>(T, X, W);
  __syncthreads();
  mode_product_el<P, 1, BD>(X, T, W);
  __syncthreads();
  mode_product_el<P, 2, BD>(T, X, W);
  __syncthreads();
  for (int m = threadIdx.x; m < NI; m += BD) {
    const double a = -Ed3[m] - lam.x, b = -lam.y;
    const double den = 1.0 / (a * a + b * b);
    X[m] = cmul(X[m], make_double2(a * den, -b * den));
  }
  __syncthreads();
  mode_product_el<P, 0, BD>(X, T, V);
  __syncthreads();
  mode_product_el<P, 1, BD>(T, X, V);
  __syncthreads();
  mode_product_el<P, 2, BD>(X, T, V);
  __syncthreads();
}

// h_b = x_b - F_bi f_i for face nodes r (strided by BD): the interior part of the
// outward normal derivative along the line through each face node (eq. (flux)).
template <int P, int BD>
__device__ __forceinline__ void face_update(const double2* __restrict__ F, double2* __restrict__ H,
                                            const double* __restrict__ D) {
  constexpr int N1 = P - 2, L = N1 * N1, NB = 6 * L;
  for (int r = threadIdx.x; r < NB; r += BD) {
    const int f = r / L, pos = r - f * L;
    const int ax = f >> 1, hi = f & 1;
    const int a = pos % N1, b = pos / N1;
    int base, stride;
    if (ax == 0) { base = N1 * a + L * b; stride = 1; }
    else if (ax == 1) { base = a + L * b; stride = N1; }
    else { base = a + N1 * b; stride = L; }
    const int e = hi ? P - 1 : 0;
    const double sg = hi ? 1.0 : -1.0;
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < N1; ++t) cfma_r(s, D[e * P + t + 1], F[base + t * stride]);
    const double2 hv = H[r];
    H[r] = make_double2(hv.x - sg * s.x, hv.y - sg * s.y);
  }
}

// T = A_ib u_b: interior rows of -(Dx^2 + Dy^2 + Dz^2) restricted to face columns.
template <int P, int BD>
__device__ __forceinline__ void interior_from_faces(const double2* __restrict__ U,
                                                    double2* __restrict__ T,
                                                    const double* __restrict__ D2) {
  constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L;
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int i = m % N1, j = (m / N1) % N1, k = m / L;
    double2 s = make_double2(0.0, 0.0);
    cfma_r(s, D2[(i + 1) * P + 0], U[0 * L + j + N1 * k]);
    cfma_r(s, D2[(i + 1) * P + P - 1], U[1 * L + j + N1 * k]);
    cfma_r(s, D2[(j + 1) * P + 0], U[2 * L + i + N1 * k]);
    cfma_r(s, D2[(j + 1) * P + P - 1], U[3 * L + i + N1 * k]);
    cfma_r(s, D2[(k + 1) * P + 0], U[4 * L + i + N1 * j]);
    cfma_r(s, D2[(k + 1) * P + P - 1], U[5 * L + i + N1 * j]);
    T[m] = make_double2(-s.x, -s.y);
  }
}

}  // namespace hps
