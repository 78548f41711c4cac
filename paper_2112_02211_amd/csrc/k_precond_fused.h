// The fused preconditioner kernel y = J^{-1} x (Sec. 4, eq. (block_pc),
// Algorithm 4) with its launch geometry and block-stream helpers; the
// launchers live in k_precond.hip.  Kernel code only (a profile of this kernel
// is tied to the hash of this file, k_leaf.h and k_common.h).
#pragma once

#include "k_common.h"
#include "k_leaf.h"

namespace hps {
namespace {

template <int P>
struct PL {
  static constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  static constexpr int KS = 2;                                         // column halves per row
  static constexpr int SLOTS = KS * NB;                                // (row, half) work items
  static constexpr int RPT = (SLOTS + 1023) / 1024;                    // work items per thread
  static constexpr int BD = ((SLOTS + RPT - 1) / RPT + 63) / 64 * 64;  // workgroup size
  static constexpr int NBP = (NB + 3) / 4 * 4;                         // padded column count
  // waves per SIMD for two resident workgroups per CU (one if that needs more
  // than 6, i.e. fewer than 80 VGPRs), given to the compiler as a lower bound
  static constexpr int MINW2 = 2 * BD / 256;
  static constexpr int MINW = MINW2 <= 6 ? (MINW2 > 0 ? MINW2 : 1) : (BD / 256 > 0 ? BD / 256 : 1);
};

// 16-byte column group of the block in each storage precision
template <int PREC> struct BlockIO;
template <> struct BlockIO<kFP64> { static constexpr int CW = 1; };
template <> struct BlockIO<kFP32> { static constexpr int CW = 2; };
template <> struct BlockIO<kBF16> { static constexpr int CW = 4; };

__device__ __forceinline__ float bf_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf_hi(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }

// The first PF column groups of a thread's first (row, half) work item, loaded
// before the leaf arithmetic that precedes the block product (Algorithm 3 and
// the face update), so that HBM is busy during it.  Entries past the item's
// last column group are zero and are not used.
template <int P, int PREC, int PF>
struct BlockPrefetch {
  uint4 v[PF];
  __device__ __forceinline__ void issue(const void* __restrict__ blk, int64_t tau, int ncp) {
    using Q = PL<P>;
    constexpr int NB = Q::NB, KS = Q::KS;
    constexpr int CW = BlockIO<PREC>::CW;
    const int ncg = ncp / CW;
    const int per = (ncg + KS - 1) / KS;
    const int slot = threadIdx.x;
    const bool ok = slot < Q::SLOTS;
    const int sl = ok ? slot : 0;
    const int row = sl % NB, q = sl / NB;
    const int c0 = q * per, c1 = ok ? min(ncg, (q + 1) * per) : c0;
    const uint4* B = static_cast<const uint4*>(blk) + (size_t)tau * ncg * NB + row;
#pragma unroll
    for (int u = 0; u < PF; ++u)
      v[u] = (c0 + u < c1) ? ld_nt(B + (size_t)(c0 + u) * NB) : make_uint4(0, 0, 0, 0);
  }
};

template <int P, int PREC>
struct BlockPrefetch<P, PREC, 0> {
  uint4 v[1];
  __device__ __forceinline__ void issue(const void*, int64_t, int) {}
};

__device__ __forceinline__ double2 as_d2(uint4 a) {
  return make_double2(__hiloint2double(a.y, a.x), __hiloint2double(a.w, a.z));
}

// u_b = S~^{-1} h_b for one leaf.  Work item (row r, half q) accumulates the
// columns of half q of row r; the two halves are combined through LDS.  The
// block is read once, with non-temporal 16-byte loads (it is not reused before
// the next preconditioner call, which reads every other block first).
template <int P, int PREC, int UNR, int PF>
__device__ __forceinline__ void block_gemv(const void* __restrict__ blk, int64_t tau, int ncp,
                                           const double2* __restrict__ H, double2* __restrict__ Up,
                                           double2* __restrict__ U, double2* __restrict__ yb,
                                           const BlockPrefetch<P, PREC, PF>& pf) {
  using Q = PL<P>;
  constexpr int NB = Q::NB, RPT = Q::RPT, BD = Q::BD, KS = Q::KS;
  constexpr int CW = BlockIO<PREC>::CW;
  const int ncg = ncp / CW;
  const int per = (ncg + KS - 1) / KS;
  int rows[RPT], cg0[RPT], cg1[RPT];
  bool ok[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int slot = threadIdx.x + k * BD;
    ok[k] = slot < Q::SLOTS;
    const int sl = ok[k] ? slot : 0;
    rows[k] = sl % NB;
    const int q = sl / NB;
    cg0[k] = q * per;
    cg1[k] = ok[k] ? min(ncg, (q + 1) * per) : cg0[k];
  }
  if (PREC == kFP64) {
    const double2* B = static_cast<const double2*>(blk) + (size_t)tau * ncg * NB;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      double2 acc = make_double2(0.0, 0.0);
      const double2* Br = B + rows[k];
      int cg = cg0[k];
      if (k == 0) {  // the prefetched column groups first
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          if (cg + u < cg1[k]) {
            const double2 sv = as_d2(pf.v[u]), h = H[cg + u];
            acc.x = fma(sv.x, h.x, fma(-sv.y, h.y, acc.x));
            acc.y = fma(sv.x, h.y, fma(sv.y, h.x, acc.y));
          }
        }
        cg = min(cg1[k], cg + PF);
      }
      for (; cg + UNR <= cg1[k]; cg += UNR) {
        double2 sv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u) sv[u] = ld_nt(Br + (size_t)(cg + u) * NB);
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
          const double2 h = H[cg + u];
          acc.x = fma(sv[u].x, h.x, fma(-sv[u].y, h.y, acc.x));
          acc.y = fma(sv[u].x, h.y, fma(sv[u].y, h.x, acc.y));
        }
      }
      for (; cg < cg1[k]; ++cg) {
        const double2 h = H[cg];
        const double2 sv = ld_nt(Br + (size_t)cg * NB);
        acc.x = fma(sv.x, h.x, fma(-sv.y, h.y, acc.x));
        acc.y = fma(sv.x, h.y, fma(sv.y, h.x, acc.y));
      }
      if (ok[k]) Up[threadIdx.x + k * BD] = acc;
    }
  } else {
    // reduced-precision blocks: FP32 arithmetic, h rounded to FP32
    const uint4* B = static_cast<const uint4*>(blk) + (size_t)tau * ncg * NB;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      float2 acc = make_float2(0.f, 0.f);
      const uint4* Br = B + rows[k];
      // one 16-byte column group: CW complex entries
      auto consume = [&](uint4 sv, int cg) {
        const uint32_t wv[4] = {sv.x, sv.y, sv.z, sv.w};
#pragma unroll
        for (int w = 0; w < CW; ++w) {
          const double2 hv = (cg < cg1[k]) ? H[cg * CW + w] : make_double2(0.0, 0.0);
          const float hr = (float)hv.x, hi = (float)hv.y;
          float sr, si;
          if (PREC == kFP32) {
            sr = __uint_as_float(wv[2 * w]);
            si = __uint_as_float(wv[2 * w + 1]);
          } else {
            sr = bf_lo(wv[w]);
            si = bf_hi(wv[w]);
          }
          acc.x = fmaf(sr, hr, fmaf(-si, hi, acc.x));
          acc.y = fmaf(sr, hi, fmaf(si, hr, acc.y));
        }
      };
      int cg0k = cg0[k];
      if (k == 0) {  // the prefetched column groups first
#pragma unroll
        for (int u = 0; u < PF; ++u) consume(pf.v[u], cg0k + u);
        cg0k = min(cg1[k], cg0k + PF);
      }
      for (int cg = cg0k; cg < cg1[k]; cg += UNR) {
        uint4 sv[UNR];
#pragma unroll
        for (int u = 0; u < UNR; ++u)
          sv[u] = (cg + u < cg1[k]) ? ld_nt(Br + (size_t)(cg + u) * NB)
                                    : make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < UNR; ++u) consume(sv[u], cg + u);
      }
      if (ok[k]) Up[threadIdx.x + k * BD] = make_double2((double)acc.x, (double)acc.y);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < NB; r += BD) {
    double2 v = Up[r];
#pragma unroll
    for (int q = 1; q < KS; ++q) v = cadd(v, Up[q * NB + r]);
    U[r] = v;
    yb[r] = v;
  }
}

// g != null: x is A v without the face exchange and the exchange is done here,
// while loading: x_b += the neighbour's outgoing impedance on the partner face
// (the same addition, in the same order, as the exchange kernel of the apply).
// column groups per thread loaded before the leaf arithmetic (fewer for the
// reduced precisions, whose 16-byte groups hold 2 or 4 entries and whose
// products need more registers); none above p = 12, where the LDS allows one
// workgroup per CU and every thread has two work items
template <int P, int PREC>
constexpr int kPrefetch = P > 12 ? 0 : (PREC == kFP64 ? 8 : (PREC == kFP32 ? 4 : 2));

template <int P, int PREC>
__global__ __launch_bounds__(PL<P>::BD, PL<P>::MINW) void k_precond_fused(
    const double2* __restrict__ x, const double2* __restrict__ g, const int* __restrict__ nbr,
    double2* __restrict__ y, const void* __restrict__ blk, int ncp, const double2* __restrict__ lam,
    const double* __restrict__ tab, int64_t nl, int64_t N, int64_t os) {
  using Q = PL<P>;
  constexpr int N1 = Q::N1, L = Q::L, NI = Q::NI, NB = Q::NB, NN = Q::NN, BD = Q::BD;
  __shared__ double2 T[NI];
  __shared__ double2 F[NI];
  __shared__ double2 H[Q::NBP];
  __shared__ double2 U[NB];
  __shared__ double2 Up[Q::SLOTS];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const double2* xv = x + rhs * N + tau * NN;
  double2* yv = y + rhs * N + tau * NN;
  // block and lambda of this leaf (operator groups: of right-hand side rhs's operator)
  const int64_t bk = tau + rhs * os;
  const double2 lm = lam[bk];
  // element-parallel Algorithm 3 while the block product's scratch Up can hold
  // the n1^3 tensor (n1 <= 12); line-wise above that
  constexpr bool EL = Q::SLOTS >= NI;
  __shared__ double LT[EL ? kLeafTab<P> : 1];
  if (EL) stage_leaf_tables<P, BD>(LT, tab);

  for (int m = threadIdx.x; m < NI; m += BD) T[m] = xv[m];
  for (int m = threadIdx.x; m < Q::NBP; m += BD) {
    double2 v = make_double2(0.0, 0.0);
    if (m < NB) {
      v = xv[NI + m];
      if (g) {
        const int f = m / L, pos = m - f * L;
        const int t2 = nbr[tau * 6 + f];
        if (t2 >= 0) {
          const double2 gv = g[(rhs * nl + t2) * NB + (f ^ 1) * L + pos];
          v = make_double2(v.x + gv.x, v.y + gv.y);
        }
      }
    }
    H[m] = v;
  }
  // The first block loads go out now, after every load the leaf arithmetic
  // needs (loads complete in order, so anything issued later would wait for
  // them), and arrive while Algorithm 3 and the face update run.
  BlockPrefetch<P, PREC, kPrefetch<P, PREC>> pf;
  pf.issue(blk, bk, ncp);
  __syncthreads();
  // f_i = A~_ii^{-1} x_i
  if constexpr (EL) homog_solve_el<P, BD>(T, Up, LT, lm);
  else homog_solve<P, BD>(T, tab, lm);
  for (int m = threadIdx.x; m < NI; m += BD) F[m] = T[m];
  // h_b = x_b - F_bi f_i
  if constexpr (EL) face_update<P, BD>(T, H, LT + lt_dlo<P>(), LT + lt_dhi<P>());
  else face_update_g<P, BD>(T, H, tab);
  __syncthreads();
  // u_b = S~^{-1} h_b, written to y_b and kept in LDS
  block_gemv<P, PREC, (PREC == kFP64 ? 8 : 4), kPrefetch<P, PREC>>(blk, bk, ncp, H, Up, U, yv + NI, pf);
  __syncthreads();
  // t = A_ib u_b
  if constexpr (EL) interior_from_faces<P, BD>(U, T, LT + lt_c0<P>(), LT + lt_c1<P>(), 1);
  else interior_from_faces_g<P, BD>(U, T, tab);
  __syncthreads();
  if constexpr (EL) homog_solve_el<P, BD>(T, Up, LT, lm);
  else homog_solve<P, BD>(T, tab, lm);
  for (int m = threadIdx.x; m < NI; m += BD) yv[m] = csub(F[m], T[m]);
}

}  // namespace
}  // namespace hps
