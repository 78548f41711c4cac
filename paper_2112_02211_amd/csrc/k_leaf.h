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

// The leaf tables in LDS: LT = [W | V | E_Delta | Dlo | Dhi | C0 | C1] (V^{-1}
// and V, n1^2 each; the n1^3 eigenvalue sums; the end rows of D and the end
// columns of D^2 as face_update / interior_from_faces take them, n1 each),
// kLeafTab<P> doubles.  With them in LDS the leaf arithmetic issues no
// vector-memory loads (a load there would wait for every earlier load of the
// wavefront, e.g. the block prefetch).
template <int P>
constexpr int kLeafTab = 2 * (P - 2) * (P - 2) + (P - 2) * (P - 2) * (P - 2) + 4 * (P - 2);
template <int P> constexpr int lt_ed3() { return 2 * (P - 2) * (P - 2); }
template <int P> constexpr int lt_dlo() { return lt_ed3<P>() + (P - 2) * (P - 2) * (P - 2); }
template <int P> constexpr int lt_dhi() { return lt_dlo<P>() + (P - 2); }
template <int P> constexpr int lt_c0() { return lt_dhi<P>() + (P - 2); }
template <int P> constexpr int lt_c1() { return lt_c0<P>() + (P - 2); }

template <int P, int BD>
__device__ __forceinline__ void stage_leaf_tables(double* __restrict__ LT, const double* __restrict__ tab) {
  constexpr int N1 = P - 2, Q = N1 * N1;
  for (int k = threadIdx.x; k < kLeafTab<P>; k += BD) {
    double v;
    if (k < Q) v = tab[tab_off_W(P) + k];
    else if (k < 2 * Q) v = tab[tab_off_V(P) + k - Q];
    else if (k < lt_dlo<P>()) v = tab[tab_off_ed3(P) + k - 2 * Q];
    else if (k < lt_dhi<P>()) v = tab[tab_off_D(P) + 1 + (k - lt_dlo<P>())];
    else if (k < lt_c0<P>()) v = tab[tab_off_D(P) + (P - 1) * P + 1 + (k - lt_dhi<P>())];
    else if (k < lt_c1<P>()) v = tab[tab_off_D2(P) + (k - lt_c0<P>() + 1) * P];
    else v = tab[tab_off_D2(P) + (k - lt_c1<P>() + 1) * P + P - 1];
    LT[k] = v;
  }
}

// T <- A~_ii^{-1} T as homog_solve, element-parallel: X is an LDS scratch of
// n1^3 entries, WVE the tables staged by stage_leaf_tables.
template <int P, int BD>
__device__ __forceinline__ void homog_solve_el(double2* __restrict__ T, double2* __restrict__ X,
                                               const double* __restrict__ WVE, double2 lam) {
  constexpr int N1 = P - 2, NI = N1 * N1 * N1;
  const double* W = WVE;
  const double* V = WVE + N1 * N1;
  const double* Ed3 = WVE + 2 * N1 * N1;
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
// Dlo[t], Dhi[t] (t < n1): entries t + 1 of the first and last rows of D.
template <int P, int BD>
__device__ __forceinline__ void face_update(const double2* __restrict__ F, double2* __restrict__ H,
                                            const double* __restrict__ Dlo,
                                            const double* __restrict__ Dhi) {
  constexpr int N1 = P - 2, L = N1 * N1, NB = 6 * L;
  for (int r = threadIdx.x; r < NB; r += BD) {
    const int f = r / L, pos = r - f * L;
    const int ax = f >> 1, hi = f & 1;
    const int a = pos % N1, b = pos / N1;
    int base, stride;
    if (ax == 0) { base = N1 * a + L * b; stride = 1; }
    else if (ax == 1) { base = a + L * b; stride = N1; }
    else { base = a + N1 * b; stride = L; }
    const double* Dr = hi ? Dhi : Dlo;
    const double sg = hi ? 1.0 : -1.0;
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < N1; ++t) cfma_r(s, Dr[t], F[base + t * stride]);
    const double2 hv = H[r];
    H[r] = make_double2(hv.x - sg * s.x, hv.y - sg * s.y);
  }
}

// T = A_ib u_b: interior rows of -(Dx^2 + Dy^2 + Dz^2) restricted to face columns.
// C0[i cs], C1[i cs] (i < n1): the first and last columns of D^2 in row i + 1.
template <int P, int BD>
__device__ __forceinline__ void interior_from_faces(const double2* __restrict__ U,
                                                    double2* __restrict__ T,
                                                    const double* __restrict__ C0,
                                                    const double* __restrict__ C1, int cs) {
  constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L;
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int i = m % N1, j = (m / N1) % N1, k = m / L;
    double2 s = make_double2(0.0, 0.0);
    cfma_r(s, C0[i * cs], U[0 * L + j + N1 * k]);
    cfma_r(s, C1[i * cs], U[1 * L + j + N1 * k]);
    cfma_r(s, C0[j * cs], U[2 * L + i + N1 * k]);
    cfma_r(s, C1[j * cs], U[3 * L + i + N1 * k]);
    cfma_r(s, C0[k * cs], U[4 * L + i + N1 * j]);
    cfma_r(s, C1[k * cs], U[5 * L + i + N1 * j]);
    T[m] = make_double2(-s.x, -s.y);
  }
}

// The same couplings read straight from the shared table in global memory.
template <int P, int BD>
__device__ __forceinline__ void face_update_g(const double2* __restrict__ F, double2* __restrict__ H,
                                              const double* __restrict__ tab) {
  const double* D = tab + tab_off_D(P);
  face_update<P, BD>(F, H, D + 1, D + (P - 1) * P + 1);
}
template <int P, int BD>
__device__ __forceinline__ void interior_from_faces_g(const double2* __restrict__ U,
                                                      double2* __restrict__ T,
                                                      const double* __restrict__ tab) {
  const double* D2 = tab + tab_off_D2(P);
  interior_from_faces<P, BD>(U, T, D2 + P, D2 + P + P - 1, P);
}

}  // namespace hps
