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
#include <mutex>
#include <type_traits>

#include "hps_internal.h"
#include "k_common.h"
#include "k_vec.h"
#include "k_lanes.h"

// Face buffer of the allocation-free apply (hps_apply_noalloc): a file-scope
// device array, one copy per GPU, held until the process ends.  Host code uses
// only the address hipGetSymbolAddress returns for it on each device (the
// array's name on the host is not a device address).
__device__ __align__(256) double2 scratch[HPS_NOALLOC_SCRATCH_BYTES / sizeof(double2)];

namespace hps {
namespace {

// config begin
// Per order: the axis-pass form, the workgroup size and the waves per SIMD the
// register budget must leave room for (so that several leaves share a CU and
// one leaf's loads overlap another's arithmetic).  Forms, from measurement (the
// apply over about 4 million unknowns for every p = 4 ... 16): line-wise (a
// thread owns a grid line and SR of its outputs, its p inputs in registers,
// the table rows uniform across a wavefront and read through the scalar cache,
// x-lines padded to p + 1 in LDS) was 3-19 % faster at p = 8, 9, 12, 13, 14
// and 16; element-parallel (a thread owns one output, inputs and table entries
// from LDS) 1-31 % faster at the other orders; single-pass (one thread per
// output sums all three axes from the LDS grid, no accumulator tensor) 5 %
// faster at p = 15, and at p = 10 once every leaf load was issued before the
// first LDS store: J^-1 A on 16^3 leaves 94-95 -> 83 us, with 64 right-hand
// sides 5.65-5.72 -> 4.42-4.49 ms (8^3 leaves: the solve 14.71 -> 14.66 ms).
enum { kSweepElem = 0, kSweepLine = 1, kSweepSingle = 2 };
template <int P>
constexpr int kSweepForm = (P == 15 || P == 10) ? kSweepSingle
                         : (P == 8 || P == 9 || P == 12 || P == 13 || P == 14 || P == 16) ? kSweepLine
                                                                                          : kSweepElem;
template <int P>
constexpr int kSweepThreads = kSweepForm<P> == kSweepSingle ? 512
                            : (P - 2) * (P - 2) * P >= 1024 ? 1024 : ((P - 2) * (P - 2) * P + 63) / 64 * 64;
template <int P>
constexpr int kSweepMinWaves = kSweepForm<P> == kSweepSingle ? 4 : 1;
template <int P>
constexpr int kSweepOutputs = 2;   // line-wise: outputs of a line per work item
// p = 12 (16^3 leaves): 512 threads, three outputs per work item (one work item
// per wavefront and axis) and registers for six waves per SIMD, so that three
// leaves share a CU; 80 us against 119 us for the apply with 1024 threads (one
// leaf per CU), the best of six shapes measured
template <> constexpr int kSweepThreads<12> = 512;
template <> constexpr int kSweepMinWaves<12> = 6;
template <> constexpr int kSweepOutputs<12> = 3;
// Bank-spread lanes (line-wise form): each axis pass hands its lines to the
// lanes by the residue mod 16 of the line's first LDS index (SweepLanes), so
// that the 16-byte reads of a quarter wavefront fall in different bank groups,
// and the accumulator's strides are congruent mod 16 to the grid's, so that the
// same assignment serves its read-modify-writes.  Grid strides (1, p + 1, SK),
// accumulator strides (1, AJ, AK); at p = 12 (1, 13, 165) and (1, 13, 133) leave
// one residue collision in the three passes (a 10 x 10 block of lines under the
// unpadded k-stride 156 and the packed accumulator had 18), at 52.7 KB of LDS per
// leaf (three leaves per CU as before).  On 16^3 leaves: the solve 100.8 ->
// 99.7 ms, iterative refinement 108.8 -> 107.3 ms (alternating runs).
template <int P>
constexpr bool kSweepBankPerm = P == 12;
template <int P>
constexpr int kSweepGridK = 0;
template <int P>
constexpr int kSweepAccJ = 0;
template <int P>
constexpr int kSweepAccK = 0;
template <> constexpr int kSweepGridK<12> = 165;
template <> constexpr int kSweepAccJ<12> = 13;
template <> constexpr int kSweepAccK<12> = 133;
// config end

template <int P>
struct Leaf {
  static constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  static constexpr bool LW = kSweepForm<P> == kSweepLine;
  static constexpr int P1 = LW ? P + 1 : P;          // LDS length of an x-line
  static constexpr bool BP = LW && kSweepBankPerm<P>;
  // grid strides (1, P1, SK) and accumulator strides (1, AJ, AK)
  static constexpr int SK = BP ? kSweepGridK<P> : P * P1;
  static constexpr int AJ = BP ? kSweepAccJ<P> : N1, AK = BP ? kSweepAccK<P> : L;
  static_assert(SK >= P * P1 && AJ >= N1 && AK >= N1 * AJ, "strides cover the grid");
  static constexpr int GS = BP ? (P - 1) * (1 + P1 + SK) + 1 : P * P * P1;   // LDS grid size
  static constexpr int AS = BP ? (N1 - 1) * (1 + AJ + AK) + 1 : NI;         // accumulator size
  static constexpr int SR = kSweepOutputs<P>, SG = (P + SR - 1) / SR, SWPG = (L + 63) / 64, SW = SG * SWPG;
  // LDS grid index of grid point (i, j, k)
  __device__ static __forceinline__ int gidx(int i, int j, int k) { return i + P1 * j + SK * k; }
  // accumulator index of interior node (i, j, k), 0-based
  __device__ static __forceinline__ int aidx(int i, int j, int k) { return i + AJ * j + AK * k; }
  __device__ static __forceinline__ int acc_of(int m) {
    if constexpr (BP) return aidx(m % N1, (m / N1) % N1, m / L);
    else return m;
  }
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
    else { base = gidx(a, b, 0); stride = SK; }
  }
};

// Lane assignment of the bank-spread form (k_lanes.h): byte AX of word s is
// the line that slot s (= 64 * (wavefront mod lines-per-group) + lane) takes in
// axis pass AX, ordered by the residue mod 16 of the line's first grid index.
template <int P>
constexpr LaneTable make_sweep_lanes() {
  using Lf = Leaf<P>;
  static_assert(Lf::SWPG * 64 <= 128 && Lf::L < 256, "two wavefronts of lines, byte line indices");
  return bank_spread_lanes(Lf::L, [](int ax, int l) {
    const int a = l % Lf::N1 + 1, b = l / Lf::N1 + 1;
    return ax == 0 ? Lf::P1 * a + Lf::SK * b : ax == 1 ? a + Lf::SK * b : a + Lf::P1 * b;
  });
}
__constant__ LaneTable kSweepLanes12 = make_sweep_lanes<12>();

// One axis pass over the lines of one leaf, AX = 0, 1, 2 (x, y, z).  Work item
// (line, o) contracts the line's p values with row o of R: o = 0 and o = p-1 are
// the line's two face outputs (outward normal derivative, the end rows of D),
// 1 .. p-2 its interior outputs (rows of -D^2, whose end columns are A_ib).
// Interior outputs accumulate in ACC; face outputs go out directly as
// F v = N v + i eta v_b (this leaf's rows) and G v = N v - i eta v_b (the face
// buffer read by the neighbour).
// Output o of the line through (a, b) along AX, s = row o of R times the line:
// a face output goes to y and to the face buffer, an interior one into ACC.
template <int P, int AX, typename T>
__device__ __forceinline__ void axis_out(double2 s, double2 ue, int o, int line, int a, int b,
                                         double2* __restrict__ ACC, double eta,
                                         T* __restrict__ yv, T* __restrict__ gv) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, NI = Lf::NI;
  if (o == 0 || o == P - 1) {
    const int f = 2 * AX + (o ? 1 : 0);
    st2(yv, NI + f * L + line, make_double2(s.x - eta * ue.y, s.y + eta * ue.x));
    st2(gv, f * L + line, make_double2(s.x + eta * ue.y, s.y - eta * ue.x));
  } else {
    int m;
    if (AX == 0) m = Lf::aidx(o - 1, a - 1, b - 1);
    else if (AX == 1) m = Lf::aidx(a - 1, o - 1, b - 1);
    else m = Lf::aidx(a - 1, b - 1, o - 1);
    if (AX == 0) ACC[m] = s;
    else ACC[m] = make_double2(ACC[m].x + s.x, ACC[m].y + s.y);
  }
}

template <int P, int AX, typename T>
__device__ __forceinline__ void axis_pass(const double2* __restrict__ U, double2* __restrict__ ACC,
                                          const double* __restrict__ R, const double* __restrict__ tab,
                                          double eta, T* __restrict__ yv, T* __restrict__ gv,
                                          unsigned int lanes) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, BD = kSweepThreads<P>;
  static_assert(!Lf::BP || Lf::SW == BD / 64, "bank-spread lanes: one work item per wavefront and pass");
  if constexpr (Lf::LW) {
    // line-wise: rows of R (o = 0: -D[0][.], o = p-1: D[p-1][.], else -D2[o][.])
    // straight from the table, at wavefront-uniform addresses
    const double* D = tab + tab_off_D(P);
    const double* D2 = tab + tab_off_D2(P);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int w = wave; w < Lf::SW; w += BD / 64) {
      const int og = w / Lf::SWPG;
      const int line = Lf::BP ? (int)((lanes >> (8 * AX)) & 0xffu) : (w - og * Lf::SWPG) * 64 + lane;
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
        axis_out<P, AX, T>(s, o == 0 ? v[0] : v[P - 1], o, line, a, b, ACC, eta, yv, gv);
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
      axis_out<P, AX, T>(s, ue, o, line, a, b, ACC, eta, yv, gv);
    }
  }
}

// Every load of the leaf is issued before the first LDS store, in rounds of up
// to eight loads per thread held in named registers (an indexed array would be
// placed in LDS or scratch by the compiler), then stored to their grid slots.
template <int P, int BD, int R0, typename T>
__device__ __forceinline__ void stage_leaf(const T* __restrict__ xv, double2* __restrict__ U) {
  using Lf = Leaf<P>;
  constexpr int NN = Lf::NN, NLOAD = (NN + BD - 1) / BD;
  const int m0 = threadIdx.x + R0 * BD;
  // storage-type registers (FP32 values are widened only at the LDS store, so
  // that no conversion sits between one load and the next); a lane past the
  // leaf's last value loads that value again and does not store it
  T t0, t1, t2, t3, t4, t5, t6, t7;
#define HPS_LD(k, t) if constexpr (R0 + k < NLOAD) { t = xv[min(m0 + k * BD, NN - 1)]; }
#define HPS_ST(k, t) if constexpr (R0 + k < NLOAD) { if ((R0 + k + 1) * BD <= NN || m0 + k * BD < NN) U[Lf::grid_of(m0 + k * BD)] = widen(t, true); }
  HPS_LD(0, t0) HPS_LD(1, t1) HPS_LD(2, t2) HPS_LD(3, t3)
  HPS_LD(4, t4) HPS_LD(5, t5) HPS_LD(6, t6) HPS_LD(7, t7)
  __builtin_amdgcn_sched_barrier(0);   // every load issued before the first store
  HPS_ST(0, t0) HPS_ST(1, t1) HPS_ST(2, t2) HPS_ST(3, t3)
  HPS_ST(4, t4) HPS_ST(5, t5) HPS_ST(6, t6) HPS_ST(7, t7)
#undef HPS_LD
#undef HPS_ST
  if constexpr (R0 + 8 < NLOAD) stage_leaf<P, BD, R0 + 8, T>(xv, U);
}

template <int P, bool CC, typename T>
__global__ __launch_bounds__(kSweepThreads<P>, kSweepMinWaves<P>) void k_apply_sweep(
    const T* __restrict__ x, T* __restrict__ y, T* __restrict__ g,
    const void* __restrict__ Cv, const double* __restrict__ tab, double eta, int64_t nl, int64_t N,
    int64_t cs, const double* __restrict__ etas) {
  using Lf = Leaf<P>;
  constexpr int NI = Lf::NI, NN = Lf::NN, NB = Lf::NB;
  constexpr int BD = kSweepThreads<P>;
  __shared__ double2 U[Lf::GS];
  __shared__ double2 ACC[Lf::AS];
  __shared__ double R[P * P];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const T* xv = x + rhs * N + tau * NN;
  T* yv = y + rhs * N + tau * NN;
  T* gv = g + (rhs * nl + tau) * NB;
  const double* D = tab + tab_off_D(P);
  const double* D2 = tab + tab_off_D2(P);
  // operator groups: right-hand side rhs belongs to operator rhs (its C and eta)
  if (etas) eta = etas[rhs];
  const int64_t cb = rhs * cs + tau * NI;
  // C at this thread's interior rows, loaded with the leaf (used in the last phase)
  using CT = std::conditional_t<CC, double2, double>;
  constexpr int NLC = (NI + BD - 1) / BD;
  const CT* Cp = static_cast<const CT*>(Cv) + cb;
  CT c0{}, c1{}, c2{}, c3{};
  c0 = Cp[min((int)threadIdx.x, NI - 1)];
  if constexpr (NLC > 1) c1 = Cp[min((int)threadIdx.x + BD, NI - 1)];
  if constexpr (NLC > 2) c2 = Cp[min((int)threadIdx.x + 2 * BD, NI - 1)];
  if constexpr (NLC > 3) c3 = Cp[min((int)threadIdx.x + 3 * BD, NI - 1)];
  for (int k = threadIdx.x; k < P * P; k += BD) {
    const int o = k / P, q = k - o * P;
    R[k] = (o == 0) ? -D[q] : (o == P - 1) ? D[(P - 1) * P + q] : -D2[k];
  }
  // this thread's lines in the three axis passes (bank-spread form)
  unsigned int lanes = 0;
  if constexpr (Lf::BP) {
    static_assert(P == 12, "lane table built for p = 12");
    lanes = kSweepLanes12.w[((int)(threadIdx.x >> 6) % Lf::SWPG) * 64 + (int)(threadIdx.x & 63)];
  }
  stage_leaf<P, BD, 0, T>(xv, U);
  __syncthreads();
  axis_pass<P, 0, T>(U, ACC, R, tab, eta, yv, gv, lanes);
  __syncthreads();
  axis_pass<P, 1, T>(U, ACC, R, tab, eta, yv, gv, lanes);
  __syncthreads();
  axis_pass<P, 2, T>(U, ACC, R, tab, eta, yv, gv, lanes);
  __syncthreads();
  // interior rows: -(Dx^2 + Dy^2 + Dz^2) v - C v (eq. (leafmat)); C was loaded
  // into registers with the leaf, so this phase waits for no memory
#define HPS_CO(k, c)                                                            \
  if constexpr (k < NLC) {                                                      \
    const int m = threadIdx.x + k * BD;                                         \
    if ((k + 1) * BD <= NI || m < NI) {                                         \
      const double2 v = U[Lf::grid_of(m)], acc = ACC[Lf::acc_of(m)];            \
      double2 cu;                                                               \
      if constexpr (CC) cu = cmul(c, v);                                        \
      else cu = cscale(v, c);                                                   \
      st2(yv, m, make_double2(acc.x - cu.x, acc.y - cu.y));                     \
    }                                                                           \
  }
  HPS_CO(0, c0) HPS_CO(1, c1) HPS_CO(2, c2) HPS_CO(3, c3)
#undef HPS_CO
  for (int m = threadIdx.x + 4 * BD; m < NI; m += BD) {   // rows past four per thread
    const double2 v = U[Lf::grid_of(m)], acc = ACC[Lf::acc_of(m)];
    double2 cu;
    if constexpr (CC) cu = cmul(Cp[m], v);
    else cu = cscale(v, Cp[m]);
    st2(yv, m, make_double2(acc.x - cu.x, acc.y - cu.y));
  }
}

// Single-pass form: one thread per output computes all three axis sums from the
// LDS grid at once, so there is no accumulator tensor and more workgroups share
// a CU.
template <int P, bool CC, typename T>
__global__ __launch_bounds__(kSweepThreads<P>, kSweepMinWaves<P>) void k_apply_sweep_fe(
    const T* __restrict__ x, T* __restrict__ y, T* __restrict__ g,
    const void* __restrict__ Cv, const double* __restrict__ tab, double eta, int64_t nl, int64_t N,
    int64_t cs, const double* __restrict__ etas) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, NI = Lf::NI, NN = Lf::NN, NB = Lf::NB, BD = kSweepThreads<P>;
  constexpr int RP = P + 1;   // padded rows of the table: lanes reading rows i, i + 1 hit other banks
  __shared__ double2 U[Lf::GS];
  __shared__ double R[P * RP];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const T* xv = x + rhs * N + tau * NN;
  T* yv = y + rhs * N + tau * NN;
  T* gv = g + (rhs * nl + tau) * NB;
  const double* D = tab + tab_off_D(P);
  const double* D2 = tab + tab_off_D2(P);
  if (etas) eta = etas[rhs];
  const int64_t cb = rhs * cs + tau * NI;
  for (int k = threadIdx.x; k < P * P; k += BD) {
    const int o = k / P, q = k - o * P;
    R[o * RP + q] = (o == 0) ? -D[q] : (o == P - 1) ? D[(P - 1) * P + q] : -D2[k];
  }
  stage_leaf<P, BD, 0, T>(xv, U);
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
    st2(yv, m, make_double2(s.x - cu.x, s.y - cu.y));
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
    st2(yv, NI + r, make_double2(s.x - eta * ue.y, s.y + eta * ue.x));
    st2(gv, r, make_double2(s.x + eta * ue.y, s.y - eta * ue.x));
  }
}

template <typename T>
__global__ void k_apply_exchange(T* __restrict__ y, const T* __restrict__ g,
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
  const double2 gv = ld2(g, (rhs * nl + t2) * nb + (f ^ 1) * L + pos);
  const double2 v = ld2(y, iy);
  st2(y, iy, make_double2(v.x + gv.x, v.y + gv.y));
}

template <int P, typename T>
int sweep_launch(hps_ctx* c, const T* x, T* y, T* g, int nrhs, hipEvent_t e0, hipEvent_t e1) {
  dim3 grid((unsigned)c->nl, (unsigned)nrhs);
  const dim3 block(kSweepThreads<P>);
  hipError_t e;
  const int64_t cs = c->nop > 1 ? c->nl * c->ni : 0;
  const double* etas = c->nop > 1 ? c->d_eta : nullptr;
  if constexpr (kSweepForm<P> == kSweepSingle) {
    if (c->c_complex)
      e = launch_k(c, e0, e1, k_apply_sweep_fe<P, true, T>, grid, block, x, y, g, (const void*)c->d_C,
                   (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
    else
      e = launch_k(c, e0, e1, k_apply_sweep_fe<P, false, T>, grid, block, x, y, g, (const void*)c->d_C,
                   (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
    return check_hip(e, "k_apply_sweep_fe");
  }
  if (c->c_complex)
    e = launch_k(c, e0, e1, k_apply_sweep<P, true, T>, grid, block, x, y, g, (const void*)c->d_C,
                 (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
  else
    e = launch_k(c, e0, e1, k_apply_sweep<P, false, T>, grid, block, x, y, g, (const void*)c->d_C,
                 (const double*)c->d_tab, c->eta, c->nl, c->N, cs, etas);
  return check_hip(e, "k_apply_sweep");
}

}  // namespace

namespace {

template <typename T>
int sweep_dispatch(hps_ctx* c, const T* x, T* y, T* g, int nrhs, hipEvent_t e0, hipEvent_t e1) {
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

}  // namespace

int launch_sweep(hps_ctx* c, const double2* x, double2* y, double2* g, int nrhs, hipEvent_t e0,
                 hipEvent_t e1) {
  return sweep_dispatch(c, x, y, g, nrhs, e0, e1);
}

int launch_sweep(hps_ctx* c, const float2* x, float2* y, float2* g, int nrhs, hipEvent_t e0,
                 hipEvent_t e1) {
  return sweep_dispatch(c, x, y, g, nrhs, e0, e1);
}

namespace {

// sweep, then the exchange, with the face buffer g; timed when tp is given
template <typename T>
int apply_with(hps_ctx* c, const T* x, T* y, T* g, int nrhs, TimedPair* tp) {
  int rc = launch_sweep(c, x, y, g, nrhs, tp ? tp->start : nullptr, nullptr);
  if (rc) return rc;
  const int64_t total = c->nl * c->nb;
  const int threads = 256;
  const hipError_t e = launch_k(c, nullptr, tp ? tp->stop : nullptr, k_apply_exchange<T>,
                                dim3((unsigned)((total + threads - 1) / threads), nrhs), dim3(threads),
                                y, (const T*)g, (const int*)c->d_nbr, c->ni, c->nb, c->n1 * c->n1,
                                c->nl, c->N);
  return check_hip(e, "k_apply_exchange");
}

}  // namespace

int launch_apply(hps_ctx* c, const double2* x, double2* y, int nrhs) {
  const size_t gbytes = (size_t)nrhs * c->nl * c->nb * sizeof(double2);
  int rc = ws_reserve(c, &c->w_g, gbytes);
  if (rc) return rc;
  double2* g = static_cast<double2*>(c->w_g.ptr);
  TimedPair tp;
  if ((rc = timing_pair(c, 0, &tp))) return rc;
  if ((rc = apply_with(c, x, y, g, nrhs, &tp))) {
    timing_drop(c, tp);
    return rc;
  }
  return timing_commit(c, 0, tp);
}

int launch_apply(hps_ctx* c, const float2* x, float2* y, int nrhs) {
  const size_t gbytes = (size_t)nrhs * c->nl * c->nb * sizeof(float2);
  int rc = ws_reserve(c, &c->w_g, gbytes);
  if (rc) return rc;
  return apply_with(c, x, y, static_cast<float2*>(c->w_g.ptr), nrhs, nullptr);
}

int scratch_address(double2** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  if (check_hip(hipGetDevice(&dev), "hipGetDevice")) return HPS_ERR_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return fail(HPS_ERR_DEVICE, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(HPS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    addr[dev] = p;
  }
  *out = static_cast<double2*>(addr[dev]);
  return HPS_OK;
}

int launch_apply_noalloc(hps_ctx* c, const double2* x, double2* y, int nrhs) {
  const size_t gbytes = (size_t)nrhs * c->nl * c->nb * sizeof(double2);
  if (gbytes > (size_t)HPS_NOALLOC_SCRATCH_BYTES)
    return fail(HPS_ERR_ARG, "hps_apply_noalloc: the face buffer needs " + std::to_string(gbytes) +
                                 " bytes, more than the static scratch of " +
                                 std::to_string((size_t)HPS_NOALLOC_SCRATCH_BYTES) + " bytes");
  if (!c->d_scratch) return fail(HPS_ERR_DEVICE, "hps_apply_noalloc: no scratch address for this context");
  return apply_with(c, x, y, c->d_scratch, nrhs, nullptr);
}

}  // namespace hps
