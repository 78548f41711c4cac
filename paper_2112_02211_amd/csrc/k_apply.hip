// y = A x: the matrix-free application of the global HPS operator (Sec. 3.2).
//
// Sweep (Algorithm 1 and the local part of Algorithm 2): one workgroup per leaf
// stages the leaf's n values in LDS on the full p^3 Chebyshev grid (corner and
// edge slots are never touched).  In each of the three axis passes one thread
// computes one output of one grid line: a contraction of the line's p values
// with a row of D^2 (the line's interior outputs; eq. (leafmat), whose
// face-column entries give A_ib v_b) or with an end row of D (the line's two
// face outputs, eq. (flux)).  Interior outputs accumulate through LDS and a
// final coalesced loop subtracts C v (Algorithm 1 with the sign of eq.
// (leafmat)).  Face rows get
// F v = N v + i eta v_b; the outgoing impedance G v = N v - i eta v_b
// (eq. (G)) goes to a face buffer.
//
// Exchange (Algorithm 2, steps 4-6 read with eq. (outgoingimpedance)): every
// face row of leaf tau on an interior face j adds the neighbour's outgoing
// impedance on the partner face j'; shared faces list their nodes in the same
// order on both sides, so no permutation is needed.
#include "hps_internal.h"
#include "k_common.h"

namespace hps {
namespace {

// Axis-pass form per order, from measurement (the apply over about 4 million
// unknowns for every p = 4 ... 16, both forms): line-wise (a thread owns a grid
// line and SR of its outputs, its p inputs in registers, the table rows uniform
// across a wavefront and read through the scalar cache, x-lines padded to p + 1
// in LDS) was 3-19 % faster at p = 8, 9, 12, 13, 14 and 16; element-parallel (a
// thread owns one output, inputs and table entries from LDS) 1-31 % faster at
// the other orders.
template <int P>
constexpr bool kSweepLineWise = (P == 8 || P == 9 || P == 12 || P == 13 || P == 14 || P == 16);

template <int P>
struct Leaf {
  static constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  static constexpr bool LW = kSweepLineWise<P>;
  static constexpr int P1 = LW ? P + 1 : P;          // LDS length of an x-line
  static constexpr int GS = P * P * P1;               // LDS grid size
  static constexpr int SR = 2, SG = (P + SR - 1) / SR, SWPG = (L + 63) / 64, SW = SG * SWPG;
  // LDS grid index of grid point (i, j, k)
  __device__ static __forceinline__ int gidx(int i, int j, int k) { return (k * P + j) * P1 + i; }
  // LDS grid index of local node m
  __device__ static __forceinline__ int grid_of(int m) {
    if (m < NI) {
      const int i = m % N1 + 1, j = (m / N1) % N1 + 1, k = m / L + 1;
      return gidx(i, j, k);
    }
    const int mm = m - NI, f = mm / L, r = mm - f * L;
    const int a = r % N1 + 1, b = r / N1 + 1, e = (f & 1) ? P - 1 : 0;
    const int ax = f >> 1;
    if (ax == 0) return gidx(e, a, b);
    if (ax == 1) return gidx(a, e, b);
    return gidx(a, b, e);
  }
  // first LDS index and stride of the grid line along ax through (a, b) (grid coordinates)
  __device__ static __forceinline__ void line(int ax, int a, int b, int& base, int& stride) {
    if (ax == 0) { base = gidx(0, a, b); stride = 1; }
    else if (ax == 1) { base = gidx(a, 0, b); stride = P1; }
    else { base = gidx(a, b, 0); stride = P * P1; }
  }
};

// Workgroup size: one thread per (line, output) work item of an axis pass,
// L lines of P outputs each, at most 1024 threads.
template <int P>
constexpr int sweep_threads() {
  return (P - 2) * (P - 2) * P >= 1024 ? 1024 : ((P - 2) * (P - 2) * P + 63) / 64 * 64;
}

// One axis pass over the lines of one leaf, AX = 0, 1, 2 (x, y, z).  Work item
// (line, o) contracts the line's p values with row o of R: o = 0 and o = p-1 are
// the line's two face outputs (outward normal derivative, the end rows of D),
// 1 .. p-2 its interior outputs (rows of -D^2, whose end columns are A_ib).
// Interior outputs accumulate in ACC; face outputs go out directly as
// F v = N v + i eta v_b (this leaf's rows) and G v = N v - i eta v_b (the face
// buffer read by the neighbour).
// Output o of the line through (a, b) along AX, s = row o of R times the line:
// a face output goes to y and to the face buffer, an interior one into ACC.
template <int P, int AX>
__device__ __forceinline__ void axis_out(double2 s, double2 ue, int o, int line, int a, int b,
                                         double2* __restrict__ ACC, double eta,
                                         double2* __restrict__ yv, double2* __restrict__ gv) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, NI = Lf::NI;
  if (o == 0 || o == P - 1) {
    const int f = 2 * AX + (o ? 1 : 0);
    yv[NI + f * L + line] = make_double2(s.x - eta * ue.y, s.y + eta * ue.x);
    gv[f * L + line] = make_double2(s.x + eta * ue.y, s.y - eta * ue.x);
  } else {
    int m;
    if (AX == 0) m = (o - 1) + N1 * (a - 1) + L * (b - 1);
    else if (AX == 1) m = (a - 1) + N1 * (o - 1) + L * (b - 1);
    else m = (a - 1) + N1 * (b - 1) + L * (o - 1);
    if (AX == 0) ACC[m] = s;
    else ACC[m] = make_double2(ACC[m].x + s.x, ACC[m].y + s.y);
  }
}

template <int P, int AX>
__device__ __forceinline__ void axis_pass(const double2* __restrict__ U, double2* __restrict__ ACC,
                                          const double* __restrict__ R, const double* __restrict__ tab,
                                          double eta, double2* __restrict__ yv, double2* __restrict__ gv) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, BD = sweep_threads<P>();
  if constexpr (Lf::LW) {
    // line-wise: rows of R (o = 0: -D[0][.], o = p-1: D[p-1][.], else -D2[o][.])
    // straight from the table, at wavefront-uniform addresses
    const double* D = tab + tab_off_D(P);
    const double* D2 = tab + tab_off_D2(P);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int w = wave; w < Lf::SW; w += BD / 64) {
      const int og = w / Lf::SWPG;
      const int line = (w - og * Lf::SWPG) * 64 + lane;
      if (line >= L) continue;
      const int a = line % N1 + 1, b = line / N1 + 1;
      int base, stride;
      Lf::line(AX, a, b, base, stride);
      double2 v[P];
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = U[base + q * stride];
#pragma unroll
      for (int r = 0; r < Lf::SR; ++r) {
        const int o = og * Lf::SR + r;
        if (o >= P) break;
        const double* row = (o == 0) ? D : (o == P - 1 ? D + (P - 1) * P : D2 + o * P);
        const double sg = (o == P - 1) ? 1.0 : -1.0;
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < P; ++q) cfma_r(s, sg * row[q], v[q]);
        axis_out<P, AX>(s, o == 0 ? v[0] : v[P - 1], o, line, a, b, ACC, eta, yv, gv);
      }
    }
  } else {
    for (int w = threadIdx.x; w < L * P; w += BD) {
      const int line = w / P, o = w - line * P;
      const int a = line % N1 + 1, b = line / N1 + 1;  // the two other grid coordinates
      int base, stride;
      Lf::line(AX, a, b, base, stride);
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < P; ++q) cfma_r(s, R[o * P + q], U[base + q * stride]);
      const double2 ue = (o == 0 || o == P - 1) ? U[base + o * stride] : make_double2(0.0, 0.0);
      axis_out<P, AX>(s, ue, o, line, a, b, ACC, eta, yv, gv);
    }
  }
}

template <int P, bool CC>
__global__ __launch_bounds__(sweep_threads<P>()) void k_apply_sweep(
    const double2* __restrict__ x, double2* __restrict__ y, double2* __restrict__ g,
    const void* __restrict__ Cv, const double* __restrict__ tab, double eta, int64_t nl, int64_t N,
    int64_t cs, const double* __restrict__ etas) {
  using Lf = Leaf<P>;
  constexpr int NI = Lf::NI, NN = Lf::NN, NB = Lf::NB;
  constexpr int BD = sweep_threads<P>();
  __shared__ double2 U[Lf::GS];
  __shared__ double2 ACC[NI];
  __shared__ double R[P * P];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const double2* xv = x + rhs * N + tau * NN;
  double2* yv = y + rhs * N + tau * NN;
  double2* gv = g + (rhs * nl + tau) * NB;
  const double* D = tab + tab_off_D(P);
  const double* D2 = tab + tab_off_D2(P);
  // operator groups: right-hand side rhs belongs to operator rhs (its C and eta)
  if (etas) eta = etas[rhs];
  const int64_t cb = rhs * cs + tau * NI;
  // every load of the leaf is issued before the first LDS store (named
  // registers, not an array, so that the staging stays in VGPRs)
  constexpr int NLOAD = (NN + BD - 1) / BD;
  static_assert(NLOAD <= 4, "leaf larger than four loads per thread");
  const int m0 = threadIdx.x, m1 = m0 + BD, m2 = m1 + BD, m3 = m2 + BD;
  double2 t0, t1, t2, t3;
  if (m0 < NN) t0 = xv[m0];
  if (NLOAD > 1 && m1 < NN) t1 = xv[m1];
  if (NLOAD > 2 && m2 < NN) t2 = xv[m2];
  if (NLOAD > 3 && m3 < NN) t3 = xv[m3];
  for (int k = threadIdx.x; k < P * P; k += BD) {
    const int o = k / P, q = k - o * P;
    R[k] = (o == 0) ? -D[q] : (o == P - 1) ? D[(P - 1) * P + q] : -D2[k];
  }
  if (m0 < NN) U[Lf::grid_of(m0)] = t0;
  if (NLOAD > 1 && m1 < NN) U[Lf::grid_of(m1)] = t1;
  if (NLOAD > 2 && m2 < NN) U[Lf::grid_of(m2)] = t2;
  if (NLOAD > 3 && m3 < NN) U[Lf::grid_of(m3)] = t3;
  __syncthreads();
  axis_pass<P, 0>(U, ACC, R, tab, eta, yv, gv);
  __syncthreads();
  axis_pass<P, 1>(U, ACC, R, tab, eta, yv, gv);
  __syncthreads();
  axis_pass<P, 2>(U, ACC, R, tab, eta, yv, gv);
  __syncthreads();
  // interior rows: -(Dx^2 + Dy^2 + Dz^2) v - C v (eq. (leafmat))
  for (int m = threadIdx.x; m < NI; m += BD) {
    const double2 v = U[Lf::grid_of(m)], acc = ACC[m];
    double2 cu;
    if (CC) cu = cmul(static_cast<const double2*>(Cv)[cb + m], v);
    else cu = cscale(v, static_cast<const double*>(Cv)[cb + m]);
    yv[m] = make_double2(acc.x - cu.x, acc.y - cu.y);
  }
}

// Single-pass form: one thread per output computes all three axis sums from the
// LDS grid at once, so there is no accumulator tensor and two workgroups share
// a CU at large p (the other forms keep one there).  Measured 5 % faster than
// element-parallel at p = 15, 5 % slower than line-wise at p = 16.
template <int P> constexpr bool kSweepFused = (P == 15);
constexpr int kFusedThreads = 512;

template <int P, bool CC>
__global__ __launch_bounds__(kFusedThreads, 4) void k_apply_sweep_fe(
    const double2* __restrict__ x, double2* __restrict__ y, double2* __restrict__ g,
    const void* __restrict__ Cv, const double* __restrict__ tab, double eta, int64_t nl, int64_t N,
    int64_t cs, const double* __restrict__ etas) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, NI = Lf::NI, NN = Lf::NN, NB = Lf::NB, BD = kFusedThreads;
  constexpr int RP = P + 1;   // padded rows of the table: lanes reading rows i, i + 1 hit other banks
  __shared__ double2 U[Lf::GS];
  __shared__ double R[P * RP];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const double2* xv = x + rhs * N + tau * NN;
  double2* yv = y + rhs * N + tau * NN;
  double2* gv = g + (rhs * nl + tau) * NB;
  const double* D = tab + tab_off_D(P);
  const double* D2 = tab + tab_off_D2(P);
  if (etas) eta = etas[rhs];
  const int64_t cb = rhs * cs + tau * NI;
  for (int k = threadIdx.x; k < P * P; k += BD) {
    const int o = k / P, q = k - o * P;
    R[o * RP + q] = (o == 0) ? -D[q] : (o == P - 1) ? D[(P - 1) * P + q] : -D2[k];
  }
  for (int m = threadIdx.x; m < NN; m += BD) U[Lf::grid_of(m)] = xv[m];
  __syncthreads();
  // interior rows: -(Dx^2 + Dy^2 + Dz^2) v - C v (eq. (leafmat))
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int i = m % N1 + 1, j = (m / N1) % N1 + 1, k = m / L + 1;
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < P; ++q) cfma_r(s, R[i * RP + q], U[Lf::gidx(q, j, k)]);
#pragma unroll
    for (int q = 0; q < P; ++q) cfma_r(s, R[j * RP + q], U[Lf::gidx(i, q, k)]);
#pragma unroll
    for (int q = 0; q < P; ++q) cfma_r(s, R[k * RP + q], U[Lf::gidx(i, j, q)]);
    const double2 v = U[Lf::gidx(i, j, k)];
    double2 cu;
    if (CC) cu = cmul(static_cast<const double2*>(Cv)[cb + m], v);
    else cu = cscale(v, static_cast<const double*>(Cv)[cb + m]);
    yv[m] = make_double2(s.x - cu.x, s.y - cu.y);
  }
  // face rows: outward normal derivative along the line (the end rows of D),
  // F v = N v + i eta v_b to y, G v = N v - i eta v_b to the face buffer
  for (int r = threadIdx.x; r < NB; r += BD) {
    const int f = r / L, pos = r - f * L;
    const int ax = f >> 1, o = (f & 1) ? P - 1 : 0;
    const int a = pos % N1 + 1, b = pos / N1 + 1;
    int base, stride;
    Lf::line(ax, a, b, base, stride);
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < P; ++q) cfma_r(s, R[o * RP + q], U[base + q * stride]);
    const double2 ue = U[base + o * stride];
    yv[NI + r] = make_double2(s.x - eta * ue.y, s.y + eta * ue.x);
    gv[r] = make_double2(s.x + eta * ue.y, s.y - eta * ue.x);
  }
}

__global__ void k_apply_exchange(double2* __restrict__ y, const double2* __restrict__ g,
                                 const int* __restrict__ nbr, int ni, int nb, int L, int64_t nl,
                                 int64_t N) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nl * nb) return;
  const int rhs = blockIdx.y;
  const int64_t tau = gid / nb;
  const int rr = (int)(gid - tau * nb);
  const int f = rr / L, pos = rr - f * L;
  const int t2 = nbr[tau * 6 + f];
  if (t2 < 0) return;
  const int64_t iy = rhs * N + tau * (ni + nb) + ni + rr;
  const double2 gv = g[(rhs * nl + t2) * nb + (f ^ 1) * L + pos];
  const double2 v = y[iy];
  y[iy] = make_double2(v.x + gv.x, v.y + gv.y);
}

template <int P>
int sweep_launch(hps_ctx* c, const double2* x, double2* y, double2* g, int nrhs, hipEvent_t e0,
                 hipEvent_t e1) {
  dim3 grid((unsigned)c->nl, (unsigned)nrhs);
  const dim3 block(sweep_threads<P>());
  hipError_t e;
  const int64_t cs = c->nop > 1 ? c->nl * c->ni : 0;
  const double* etas = c->nop > 1 ? c->d_eta : nullptr;
  if constexpr (kSweepFused<P>) {
    const dim3 fblock(kFusedThreads);
    if (c->c_complex)
      e = launch_k(c, e0, e1, k_apply_sweep_fe<P, true>, grid, fblock, x, y, g, (const void*)c->d_C,
                   (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
    else
      e = launch_k(c, e0, e1, k_apply_sweep_fe<P, false>, grid, fblock, x, y, g, (const void*)c->d_C,
                   (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
    return check_hip(e, "k_apply_sweep_fe");
  }
  if (c->c_complex)
    e = launch_k(c, e0, e1, k_apply_sweep<P, true>, grid, block, x, y, g, (const void*)c->d_C,
                 (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
  else
    e = launch_k(c, e0, e1, k_apply_sweep<P, false>, grid, block, x, y, g, (const void*)c->d_C,
                 (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
  return check_hip(e, "k_apply_sweep");
}

}  // namespace

int launch_sweep(hps_ctx* c, const double2* x, double2* y, double2* g, int nrhs, hipEvent_t e0,
                 hipEvent_t e1) {
  // an operator group's kernels read operator rhs's C and eta for right-hand side rhs
  if (c->nop > 1 && nrhs != c->nop) return fail(HPS_ERR_ARG, "operator group: one right-hand side per operator");
  switch (c->p) {
    case 4: return sweep_launch<4>(c, x, y, g, nrhs, e0, e1);
    case 5: return sweep_launch<5>(c, x, y, g, nrhs, e0, e1);
    case 6: return sweep_launch<6>(c, x, y, g, nrhs, e0, e1);
    case 7: return sweep_launch<7>(c, x, y, g, nrhs, e0, e1);
    case 8: return sweep_launch<8>(c, x, y, g, nrhs, e0, e1);
    case 9: return sweep_launch<9>(c, x, y, g, nrhs, e0, e1);
    case 10: return sweep_launch<10>(c, x, y, g, nrhs, e0, e1);
    case 11: return sweep_launch<11>(c, x, y, g, nrhs, e0, e1);
    case 12: return sweep_launch<12>(c, x, y, g, nrhs, e0, e1);
    case 13: return sweep_launch<13>(c, x, y, g, nrhs, e0, e1);
    case 14: return sweep_launch<14>(c, x, y, g, nrhs, e0, e1);
    case 15: return sweep_launch<15>(c, x, y, g, nrhs, e0, e1);
    case 16: return sweep_launch<16>(c, x, y, g, nrhs, e0, e1);
    default: return fail(HPS_ERR_UNSUPPORTED, "p out of range");
  }
}

int launch_apply(hps_ctx* c, const double2* x, double2* y, int nrhs) {
  const size_t gbytes = (size_t)nrhs * c->nl * c->nb * sizeof(double2);
  int rc = ws_reserve(c, &c->w_g, gbytes);
  if (rc) return rc;
  double2* g = static_cast<double2*>(c->w_g.ptr);
  TimedPair tp;
  if ((rc = timing_pair(c, 0, &tp))) return rc;
  if ((rc = launch_sweep(c, x, y, g, nrhs, tp.start, nullptr))) {
    timing_drop(c, tp);
    return rc;
  }
  const int64_t total = c->nl * c->nb;
  const int threads = 256;
  const hipError_t e = launch_k(c, nullptr, tp.stop, k_apply_exchange,
                                dim3((unsigned)((total + threads - 1) / threads), nrhs), dim3(threads),
                                y, (const double2*)g, (const int*)c->d_nbr, c->ni, c->nb, c->n1 * c->n1,
                                c->nl, c->N);
  if ((rc = check_hip(e, "k_apply_exchange"))) {
    timing_drop(c, tp);
    return rc;
  }
  return timing_commit(c, 0, tp);
}

}  // namespace hps
