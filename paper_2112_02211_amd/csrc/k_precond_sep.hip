// y = J^{-1} x in the separable form: the same block-diagonal preconditioner
// as the dense-block kernel (Sec. 4, eq. (block_pc): on each leaf the exact
// inverse of the homogenized leaf matrix [[A~_ii, A_ib], [F_bi, F_bb]] with
// C_ii = lambda^tau I), applied without any stored block.
//
// With the face nodes at the interior Chebyshev nodes of each face, every row
// of the homogenized leaf matrix couples nodes of the three grid lines through
// its node only, and a face row (eq. (flux) plus i eta) only nodes of the
// normal line of its face node, which ends at a node of each of the two
// opposite faces.  Per line, the two end values follow from the 2 x 2 face
// system of that line,
//   [u_lo, u_hi] = Fi ([x_lo, x_hi] - Fbi1 u_line),
// and substituting them into the interior rows leaves the Kronecker sum
//   K = -(Lt x I x I + I x Lt x I + I x I x Lt) - lambda I,
//   Lt = D2[1:e, 1:e] - D2[1:e, {0, e}] Fi Fbi1          (complex, n1 x n1),
// which Lt = Vc diag(Ec) Vc^{-1} diagonalizes as Algorithm 3 does the
// Dirichlet interior operator, with complex factors.  So, per leaf:
//
//   g     = Fi [x_lo, x_hi]                       on every grid line
//   r_i   = x_i - A_ib g
//   u_i   = (Vc x Vc x Vc) diag(1 / (-Ec_Delta - lambda)) (Wc x Wc x Wc) r_i
//   u_b   = g - Fi Fbi1 u_line                    on every grid line
//
// One workgroup per (leaf, right-hand side), the leaf in LDS, six complex mode
// products (three forms, chosen per order: kSepForm; at p = 10 and 12 in even /
// odd halves, kSepSplit).  Cost per leaf O(n1^4);
// the kernel reads x and writes y once (32 bytes
// per unknown), where the dense form also streams the n_b x n_b block.  The
// tables (Wc, Vc, Ec, Fi per operator) are built on the host at setup.
#include "hps_internal.h"
#include "k_vec.h"
#include "k_lanes.h"

namespace hps {
namespace {

// config begin
// Per order: the mode-product form, the workgroup size, the waves per SIMD the
// register budget must leave room for, and (line-wise) the outputs of a line
// per work item.  Forms, from measurement (J^-1 over about 4 million unknowns
// for every p = 4 ... 16): line-wise (a thread owns a grid line and R of its
// outputs, the n1 inputs in registers, the matrix rows uniform across a
// wavefront and read through the scalar cache) was 3-32 % faster at p = 8, 10,
// 11 and 13-16, element-parallel (a thread owns one output; inputs and matrix
// entries from LDS) 5-30 % faster at p = 4-7 and 9 and equal at 12; in place
// (a thread owns a whole line and all its outputs, written back over its
// inputs, so no second LDS tensor is needed and two workgroups fit on a CU)
// 28 % faster at p = 16 on 32^3 leaves, 8 % at p = 15, 2-3 % at p = 13, 14.
enum { kSepElem = 0, kSepLine = 1, kSepInPlace = 2 };
template <int P>
constexpr int kSepForm = P >= 13 ? kSepInPlace : (P == 8 || P == 10 || P == 11) ? kSepLine : kSepElem;
template <int P>
constexpr int kSepThreads = kSepForm<P> == kSepInPlace ? 512
                          : ((P - 2) * (P - 2) * (P - 2) + 63) / 64 * 64 < 64 ? 64
                          : ((P - 2) * (P - 2) * (P - 2) + 63) / 64 * 64 > 1024 ? 1024
                          : ((P - 2) * (P - 2) * (P - 2) + 63) / 64 * 64;
template <int P>
constexpr int kSepMinWaves = kSepForm<P> == kSepInPlace ? 4 : 1;
template <int P>
constexpr int kSepOutputs = 2;
// p = 12 (16^3 leaves): line-wise with five outputs per work item on 256
// threads (two items per wavefront and mode product), three leaves per CU;
// 95 us against 118 us element-parallel on 1024 threads, the best of six
// shapes measured
template <> constexpr int kSepForm<12> = kSepLine;
template <> constexpr int kSepThreads<12> = 256;
template <> constexpr int kSepMinWaves<12> = 8;
template <> constexpr int kSepOutputs<12> = 5;
// p = 10: 256 threads (two outputs per work item: one work item per wavefront
// in each product instead of half the wavefronts idle on 512), registers for
// six waves per SIMD, so six leaves share a CU instead of three: J^-1 on 16^3
// leaves 39.1 -> 33.0 us, with 64 right-hand sides 2.37 -> 1.98 ms (on 8^3
// leaves, two per CU, the solve 14.65 -> 14.70 ms).
template <> constexpr int kSepThreads<10> = 256;
template <> constexpr int kSepMinWaves<10> = 6;
// Face values in the second tensor's space (where it holds them): at p = 12 it
// took the leaf from 45.3 to 35.7 KB of LDS, four leaves per CU instead of
// three (before the in-place even / odd products removed that tensor); at
// p = 10 the registers it adds would cost a wavefront per SIMD.
template <int P>
constexpr bool kSepAliasG = P == 12;
// Even / odd mode products (the table's modes split by parity under the flip
// of a line, even n1 only; a work item's output group must hold modes of one
// parity): each product takes half the multiplications.  Measured on 16^3
// leaves: J^-1 at p = 12 80 -> 66 us in the solve (the solve 128.4 -> 124.1
// ms), at p = 10 41.5 -> 39.8 us (64 right-hand sides 2.55 -> 2.40 ms); at
// p = 8 (n1 = 6: one or three outputs per item instead of two) 4-15 % slower.
template <int P>
constexpr bool kSepSplit = P == 12 || P == 10;
// Even / odd products in place: every work item holds its line's inputs in
// registers, so after a barrier it can write its outputs over them and the
// second LDS tensor goes (one work item per wavefront and product).  At
// p = 12: 27.7 KB of LDS per leaf instead of 35.7 (five leaves per CU instead
// of four), J^-1 64.5 -> 62.8 us, the 16^3 solve 124.1 -> 122.9 ms.  At p = 10
// registers, not LDS, set the leaves per CU: in place there was 1-2 % slower on
// 16^3 leaves with 256 threads (and equal with 512).
template <int P>
constexpr bool kSepSplitInPlace = P == 12;
// In-place tensor padded by one entry per xy-plane instead of one per x-line
// (1010 entries instead of 1100 at p = 12: 25.7 KB of LDS per leaf, six
// leaves per CU instead of five); the x-axis products then give neighbouring
// lanes neighbouring planes (stride L + 1) rather than neighbouring rows.
// On 16^3 leaves: J^-1 62.3-63.2 -> 59.0-59.7 us, the solve 101.65 -> 100.8 ms,
// iterative refinement (inner restart 10) 107.35 -> 106.45 ms.
template <int P>
constexpr bool kSepPlanePad = P == 12;
// With plane padding, the in-place products hand each axis pass's lines to the
// lanes by the residue mod 16 of the line's first LDS index (k_lanes.h), so that
// the 16-byte accesses of a quarter wavefront fall in different bank groups
// (at p = 12 one collision left over the three axes, against 12 with x-lines
// in k-major order and the other axes in natural order).  On 16^3 leaves: J^-1
// 62.5 -> 61.7 us in the solve (profiler), the solve 99.7 -> 99.4 ms.
template <int P>
constexpr bool kSepBankPerm = P == 12;
// config end

template <int P>
struct SL {
  static constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  static constexpr bool LW = kSepForm<P> == kSepLine, IP = kSepForm<P> == kSepInPlace;
  static constexpr int BD = kSepThreads<P>;
  static constexpr int MINW = kSepMinWaves<P>;
  static constexpr int ST = sep_table_size(P);
  // line-wise: the LDS tensors pad each x-line to n1 + 1 entries, so the
  // threads of a wavefront that walk neighbouring x-lines read 16-byte words in
  // different banks
  static constexpr bool SIP = kSepSplitInPlace<P>;
  static constexpr int P1 = (LW || IP) ? N1 + 1 : N1;
  // plane padding (in-place line-wise form only): entry (i, j, k) at
  // i + n1 j + (L + 1) k
  static constexpr bool PP = SIP && kSepPlanePad<P>;
  static constexpr int JS = PP ? N1 : P1, KS = PP ? L + 1 : P1 * N1;   // strides of j and k
  static constexpr int SZ = KS * N1, SZX = (IP || SIP) ? 1 : SZ;
  static constexpr bool BPL = PP && kSepBankPerm<P>;   // lanes from a bank-spread table
  // line-wise work items: (output group of R, 64 lines) per wavefront
  static constexpr int R = kSepOutputs<P>, G = (N1 + R - 1) / R, WPG = (L + 63) / 64, W = G * WPG;
  // tables staged in LDS: Ec | Fi, and for the element-parallel form Wc | Vc before them
  static constexpr int CTN = (LW || IP) ? N1 + 4 : ST, CT0 = (LW || IP) ? 0 : 2 * L;
};

template <int P>
__device__ __forceinline__ int lidx(int i, int j, int k) {
  return i + SL<P>::JS * j + SL<P>::KS * k;
}

// 1 / x by the hardware reciprocal estimate refined with two Newton-Raphson
// steps (r <- r + r (1 - x r)); x > 0 and finite here (the squared modulus of
// a diagonal entry of the diagonalized leaf operator).  Against the IEEE
// division: J^-1 at p = 12 on 16^3 leaves 65.2 -> 63.7 us, results within the
// parity bounds of the division (the error of each step squares).
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}

// First entry and stride (padded LDS index) of the grid line along axis ax
// through position (a, b) of the other two axes, lower axis first.
template <int P>
__device__ __forceinline__ void line_of(int ax, int a, int b, int& base, int& stride) {
  using S = SL<P>;
  if (ax == 0) { base = S::JS * a + S::KS * b; stride = 1; }
  else if (ax == 1) { base = a + S::KS * b; stride = S::JS; }
  else { base = a + S::JS * b; stride = S::KS; }
}

// Bank-spread lane table of the in-place products: byte AX of word s is the
// line (a + n1 b) that slot s (= 64 * (wavefront mod lines-per-group) + lane)
// takes in the products along axis AX.
template <int P>
constexpr LaneTable make_sep_lanes() {
  using S = SL<P>;
  static_assert(S::WPG * 64 <= 128 && S::L < 256, "two wavefronts of lines, byte line indices");
  return bank_spread_lanes(S::L, [](int ax, int l) {
    const int a = l % S::N1, b = l / S::N1;
    return ax == 0 ? S::JS * a + S::KS * b : ax == 1 ? a + S::KS * b : a + S::JS * b;
  });
}
__constant__ LaneTable kSepLanes12 = make_sep_lanes<12>();

// out[.., o, ..] = sum_i M[o][i] in[.., i, ..] along axis AX (M complex, row
// major).  SCALE: the output element (i, j, k) is multiplied by
// 1 / (-(Ec_i + Ec_j + Ec_k) - lambda) (the last forward product).
// Line-wise form: M in global memory, read at wavefront-uniform addresses.
template <int P, int AX, bool SCALE, bool INV>
__device__ __forceinline__ void cmode_lw(const double2* __restrict__ in, double2* __restrict__ out,
                                         const double2* __restrict__ M, const double2* __restrict__ Ec,
                                         double2 lm, unsigned int lanes) {
  using S = SL<P>;
  constexpr int N1 = S::N1, L = S::L, R = S::R, WPG = S::WPG, NW = S::BD / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if constexpr (S::SIP) {
    // in place (in == out): every item's inputs to registers, a barrier, then
    // every item's outputs (the barrier is outside any branch)
    static_assert(kSepSplit<P> && S::W <= NW, "one work item per wavefront");
    constexpr int H = N1 / 2;
    const int og = wave / WPG;
    const int line = S::BPL ? (int)((lanes >> (8 * AX)) & 0xffu) : (wave - og * WPG) * 64 + lane;
    const bool act = wave < S::W && line < L;
    // plane padding without the lane table: x-lines in k-major order across the lanes
    constexpr bool KM = S::PP && !S::BPL && AX == 0;
    const int a = act ? (KM ? line / N1 : line % N1) : 0, b = act ? (KM ? line % N1 : line / N1) : 0;
    int base, stride;
    line_of<P>(AX, a, b, base, stride);
    const bool odd = og * R >= H;
    double2 f[H];
    if (act) {
      if constexpr (!INV) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const double2 lo = in[base + i * stride], hi = in[base + (N1 - 1 - i) * stride];
          f[i] = odd ? csub(lo, hi) : cadd(lo, hi);
        }
      } else {
        const int h0 = odd ? H : 0;
#pragma unroll
        for (int q = 0; q < H; ++q) f[q] = in[base + (h0 + q) * stride];
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int o = og * R + r;
        const double2* Mr = INV ? M + (odd ? (o - H) * N1 + H : o * N1) : M + o * N1;
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < H; ++q) cfma(s, Mr[q], f[q]);
        if (SCALE) {
          const double ar = -(Ec[a].x + Ec[b].x + Ec[o].x) - lm.x;
          const double ai = -(Ec[a].y + Ec[b].y + Ec[o].y) - lm.y;
          const double den = recip_nr(ar * ar + ai * ai);
          s = cmul(s, make_double2(ar * den, -ai * den));
        }
        const int pos = (INV && odd) ? N1 - 1 - (o - H) : o;
        out[base + pos * stride] = s;
      }
    }
    return;
  }
  for (int w = wave; w < S::W; w += NW) {
    const int og = w / WPG;
    const int line = (w - og * WPG) * 64 + lane;
    if (line >= L) continue;
    const int a = line % N1, b = line / N1;
    int base, stride;
    line_of<P>(AX, a, b, base, stride);
    if constexpr (kSepSplit<P>) {
      // Modes 0 .. H-1 are even, H .. n1-1 odd (H = n1 / 2): an even row of
      // Wc is symmetric (Wc[o][n1-1-i] = Wc[o][i]), an odd row antisymmetric,
      // and the even / odd columns of Vc likewise.  Forward: fold the line
      // (v_i +/- v_{n1-1-i}, i < H) and take H terms per output.  Inverse:
      // the even group writes A_i = sum_e Vc[i][e] z_e at position i, the odd
      // group B_i = sum_o Vc[i][H + o] z_{H + o} at n1-1-i; the butterflies
      // (A + B, A - B) along all three axes follow the last product.
      static_assert(N1 % 2 == 0 && (N1 / 2) % R == 0, "groups of one parity");
      constexpr int H = N1 / 2;
      const bool odd = og * R >= H;   // uniform across the wavefront
      double2 f[H];
      if constexpr (!INV) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
          const double2 lo = in[base + i * stride], hi = in[base + (N1 - 1 - i) * stride];
          f[i] = odd ? csub(lo, hi) : cadd(lo, hi);
        }
      } else {
        const int h0 = odd ? H : 0;
#pragma unroll
        for (int q = 0; q < H; ++q) f[q] = in[base + (h0 + q) * stride];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int o = og * R + r;
        const double2* Mr = INV ? M + (odd ? (o - H) * N1 + H : o * N1) : M + o * N1;
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < H; ++q) cfma(s, Mr[q], f[q]);
        if (SCALE) {   // AX == 2: output element (a, b, o)
          const double ar = -(Ec[a].x + Ec[b].x + Ec[o].x) - lm.x;
          const double ai = -(Ec[a].y + Ec[b].y + Ec[o].y) - lm.y;
          const double den = recip_nr(ar * ar + ai * ai);
          s = cmul(s, make_double2(ar * den, -ai * den));
        }
        const int pos = (INV && odd) ? N1 - 1 - (o - H) : o;
        out[base + pos * stride] = s;
      }
      continue;
    }
    double2 v[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) v[i] = in[base + i * stride];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int o = og * R + r;
      if (o >= N1) break;
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < N1; ++i) cfma(s, M[o * N1 + i], v[i]);
      if (SCALE) {   // AX == 2: output element (a, b, o)
        const double ar = -(Ec[a].x + Ec[b].x + Ec[o].x) - lm.x;
        const double ai = -(Ec[a].y + Ec[b].y + Ec[o].y) - lm.y;
        const double den = recip_nr(ar * ar + ai * ai);
        s = cmul(s, make_double2(ar * den, -ai * den));
      }
      out[base + o * stride] = s;
    }
  }
}

// Element-parallel form: one output per thread, M staged in LDS (unpadded tensors).
template <int P, int AX, bool SCALE>
__device__ __forceinline__ void cmode_el(const double2* __restrict__ in, double2* __restrict__ out,
                                         const double2* __restrict__ M, const double2* __restrict__ Ec,
                                         double2 lm) {
  using S = SL<P>;
  constexpr int N1 = S::N1, L = S::L, NI = S::NI, BD = S::BD;
  constexpr int stride = AX == 0 ? 1 : (AX == 1 ? N1 : L);
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int o = (m / stride) % N1;
    const int base = m - o * stride;
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < N1; ++i) cfma(s, M[o * N1 + i], in[base + i * stride]);
    if (SCALE) {
      const int i = m % N1, j = (m / N1) % N1, k = m / L;
      const double ar = -(Ec[i].x + Ec[j].x + Ec[k].x) - lm.x;
      const double ai = -(Ec[i].y + Ec[j].y + Ec[k].y) - lm.y;
      const double den = recip_nr(ar * ar + ai * ai);
      s = cmul(s, make_double2(ar * den, -ai * den));
    }
    out[m] = s;
  }
}

// In-place line-wise form: one thread per line computes all n1 outputs of
// its line from the inputs in its registers and writes them over them (lines
// along one axis are disjoint, so no other thread reads them in this product).
template <int P, int AX, bool SCALE>
__device__ __forceinline__ void cmode_ip(double2* __restrict__ T, const double2* __restrict__ M,
                                         const double2* __restrict__ Ec, double2 lm) {
  using S = SL<P>;
  constexpr int N1 = S::N1, L = S::L, BD = S::BD;
  for (int line = threadIdx.x; line < L; line += BD) {
    const int a = line % N1, b = line / N1;
    int base, stride;
    line_of<P>(AX, a, b, base, stride);
    double2 v[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) v[i] = T[base + i * stride];
    // two outputs at a time (four independent accumulation chains); each
    // output's terms are still added in the order i = 0 .. n1-1
#pragma unroll
    for (int o0 = 0; o0 < N1; o0 += 2) {
      double2 s[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        cfma(s[0], M[o0 * N1 + i], v[i]);
        if (o0 + 1 < N1) cfma(s[1], M[(o0 + 1) * N1 + i], v[i]);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int o = o0 + h;
        if (o >= N1) break;
        double2 r = s[h];
        if (SCALE) {
          const double ar = -(Ec[a].x + Ec[b].x + Ec[o].x) - lm.x;
          const double ai = -(Ec[a].y + Ec[b].y + Ec[o].y) - lm.y;
          const double den = recip_nr(ar * ar + ai * ai);
          r = cmul(r, make_double2(ar * den, -ai * den));
        }
        T[base + o * stride] = r;
      }
    }
  }
}

// One mode product in the order's form (INV: a product with Vc); in place, out
// is in (the result is in T).
template <int P, int AX, bool SCALE, bool INV>
__device__ __forceinline__ void cmode(const double2* in, double2* out, const double2* __restrict__ Mg,
                                      const double2* __restrict__ Ml, const double2* __restrict__ Ec,
                                      double2 lm, unsigned int lanes) {
  static_assert(!kSepSplit<P> || SL<P>::LW, "even / odd products in the line-wise form only");
  if constexpr (SL<P>::IP) cmode_ip<P, AX, SCALE>(const_cast<double2*>(in), Mg, Ec, lm);
  else if constexpr (SL<P>::LW) cmode_lw<P, AX, SCALE, INV>(in, out, Mg, Ec, lm, lanes);
  else cmode_el<P, AX, SCALE>(in, out, Ml, Ec, lm);
}

// The butterflies the even / odd inverse products leave: per axis, the pair
// (A at i, B at n1-1-i) of every line becomes (A + B, A - B); one thread per
// group of eight mirror images.
template <int P>
__device__ __forceinline__ void split_butterflies(double2* __restrict__ T) {
  using S = SL<P>;
  constexpr int N1 = S::N1, H = N1 / 2, BD = S::BD;
  for (int g = threadIdx.x; g < H * H * H; g += BD) {
    const int i = g % H, j = (g / H) % H, k = g / (H * H);
    const int ii[2] = {i, N1 - 1 - i}, jj[2] = {j, N1 - 1 - j}, kk[2] = {k, N1 - 1 - k};
    double2 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = T[lidx<P>(ii[q & 1], jj[(q >> 1) & 1], kk[q >> 2])];
#pragma unroll
    for (int bit = 1; bit < 8; bit <<= 1) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q & bit) continue;
        const double2 x = v[q], y = v[q | bit];
        v[q] = cadd(x, y);
        v[q | bit] = csub(x, y);
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) T[lidx<P>(ii[q & 1], jj[(q >> 1) & 1], kk[q >> 2])] = v[q];
  }
}

// The leaf's loads are issued before any of them is used: up to eight interior
// and four face values per thread (plus, with the exchange, the neighbour's
// outgoing impedance on the partner face) in named registers of the storage
// type (an indexed array would go to LDS or scratch), all issued before the
// first LDS store (a scheduling barrier keeps the compiler from interleaving
// them), then widened and stored: interior values to the padded tensor T, face
// values to G.  A lane past the end loads an in-bounds value again and stores
// nothing.  Larger leaves stage the remaining values in plain loops.
template <int P, typename VT, bool HASG>
__device__ __forceinline__ void stage_leaf(const VT* __restrict__ xv, const VT* __restrict__ gb,
                                           const int* nb6, int64_t tau, double2* __restrict__ T,
                                           double2* __restrict__ G) {
  using S = SL<P>;
  constexpr int N1 = S::N1, L = S::L, NI = S::NI, NB = S::NB, BD = S::BD;
  constexpr int NLI = (NI + BD - 1) / BD, NLB = (NB + BD - 1) / BD;
  const int t = threadIdx.x;
  VT a0, a1, a2, a3, a4, a5, a6, a7, x0, x1, x2, x3, g0, g1, g2, g3;
#define HPS_LI(k, r) if constexpr (k < NLI) { r = xv[min(t + k * BD, NI - 1)]; }
#define HPS_LB(k, xr, gr)                                                      \
  if constexpr (k < NLB) {                                                     \
    const int m = min(t + k * BD, NB - 1), f = m / L, pos = m - f * L;         \
    xr = xv[NI + m];                                                            \
    if constexpr (HASG) {                                                       \
      const int t2 = nb6[f];                                                    \
      gr = gb[(t2 >= 0 ? (int64_t)t2 : tau) * NB + (f ^ 1) * L + pos];         \
    }                                                                           \
  }
#define HPS_SI(k, r)                                                                     \
  if constexpr (k < NLI) {                                                               \
    const int m = t + k * BD;                                                            \
    if ((k + 1) * BD <= NI || m < NI) T[lidx<P>(m % N1, (m / N1) % N1, m / L)] = widen(r, true); \
  }
#define HPS_SB(k, xr, gr)                                                      \
  if constexpr (k < NLB) {                                                     \
    const int m = t + k * BD;                                                  \
    if ((k + 1) * BD <= NB || m < NB) {                                        \
      double2 v = widen(xr, true);                                             \
      if (HASG && nb6[m / L] >= 0) v = cadd(v, widen(gr, true));               \
      G[m] = v;                                                                \
    }                                                                          \
  }
  HPS_LI(0, a0) HPS_LI(1, a1) HPS_LI(2, a2) HPS_LI(3, a3)
  HPS_LI(4, a4) HPS_LI(5, a5) HPS_LI(6, a6) HPS_LI(7, a7)
  HPS_LB(0, x0, g0) HPS_LB(1, x1, g1) HPS_LB(2, x2, g2) HPS_LB(3, x3, g3)
  __builtin_amdgcn_sched_barrier(0);
  HPS_SI(0, a0) HPS_SI(1, a1) HPS_SI(2, a2) HPS_SI(3, a3)
  HPS_SI(4, a4) HPS_SI(5, a5) HPS_SI(6, a6) HPS_SI(7, a7)
  HPS_SB(0, x0, g0) HPS_SB(1, x1, g1) HPS_SB(2, x2, g2) HPS_SB(3, x3, g3)
#undef HPS_LI
#undef HPS_LB
#undef HPS_SI
#undef HPS_SB
  for (int m = t + 8 * BD; m < NI; m += BD) T[lidx<P>(m % N1, (m / N1) % N1, m / L)] = widen(xv[m], true);
  for (int m = t + 4 * BD; m < NB; m += BD) {
    double2 v = widen(xv[NI + m], true);
    const int f = m / L;
    if (HASG && nb6[f] >= 0) v = cadd(v, widen(gb[(int64_t)nb6[f] * NB + (f ^ 1) * L + (m - f * L)], true));
    G[m] = v;
  }
}

// g != null: x is A v without the face exchange, added here while loading
// (x_b += the neighbour's outgoing impedance on the partner face), as in the
// dense-block kernel.  Operator groups: right-hand side rhs belongs to
// operator rhs (os = nl: lambda of [rhs][leaf], table of operator rhs).
template <int P, typename VT>
__global__ __launch_bounds__(SL<P>::BD, SL<P>::MINW) void k_precond_sep(
    const VT* __restrict__ x, const VT* __restrict__ g, const int* __restrict__ nbr,
    VT* __restrict__ y, const double2* __restrict__ lam, const double2* __restrict__ sep,
    const double* __restrict__ tab, int64_t nl, int64_t N, int64_t os) {
  using S = SL<P>;
  constexpr int N1 = S::N1, L = S::L, NI = S::NI, NB = S::NB, NN = S::NN, BD = S::BD;
  // The face values G are last read by the interior correction, before the
  // first mode product writes X, so G can live in X's space (kSepAliasG); the
  // face recovery then takes g from registers.
  constexpr bool GX = kSepAliasG<P> && S::SZX >= NB;
  constexpr int NGL = (3 * L + BD - 1) / BD;   // grid lines per thread in the face phases
  __shared__ double2 T[S::SZ];
  __shared__ double2 X[S::SZX];
  __shared__ double2 Gs[GX ? 1 : NB];
  double2* const G = GX ? X : Gs;
  __shared__ double2 CT[S::CTN];    // (Wc | Vc |) Ec | Fi
  __shared__ double RT[4 * N1];     // Dlo | Dhi | C0 | C1
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const VT* xv = x + rhs * N + tau * NN;
  VT* yv = y + rhs * N + tau * NN;
  const double2 lm = lam[tau + rhs * os];
  const double2* st = sep + (os ? (int64_t)rhs * S::ST : 0);
  const double2* Wc = st;          // global: read at wavefront-uniform addresses
  const double2* Vc = st + L;
  // this thread's lines in the three axes' products (bank-spread lanes),
  // loaded with the leaf
  unsigned int lanes = 0;
  if constexpr (S::BPL) {
    static_assert(P == 12, "lane table built for p = 12");
    lanes = kSepLanes12.w[((int)(threadIdx.x >> 6) % S::WPG) * 64 + (int)(threadIdx.x & 63)];
  }
  // table entries: thread k loads entry k of Ec | Fi (| Wc | Vc) and of
  // Dlo | Dhi | C0 | C1 from in-bounds (clamped) addresses without a branch, so
  // that these loads and the leaf's are all in flight together; they are
  // stored to LDS after the leaf's values
  static_assert(4 * N1 <= BD, "table rows per thread");
  const int kr = min((int)threadIdx.x, 4 * N1 - 1), tr = kr % N1, wr = kr / N1;
  const int toff = wr == 0 ? tab_off_D(P) + 1 + tr                  // D[0][1 + t]
                 : wr == 1 ? tab_off_D(P) + (P - 1) * P + 1 + tr    // D[p-1][1 + t]
                 : wr == 2 ? tab_off_D2(P) + (tr + 1) * P           // D2[1 + t][0]
                           : tab_off_D2(P) + (tr + 1) * P + P - 1;  // D2[1 + t][p-1]
  const double rt = tab[toff];
  double2 ct = make_double2(0.0, 0.0);
  if constexpr (S::CTN <= BD) ct = st[2 * L - S::CT0 + min((int)threadIdx.x, S::CTN - 1)];
  int nb6[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) nb6[f] = g ? nbr[tau * 6 + f] : -1;
  if (g) stage_leaf<P, VT, true>(xv, g + (int64_t)rhs * nl * NB, nb6, tau, T, G);
  else stage_leaf<P, VT, false>(xv, nullptr, nb6, tau, T, G);
  if ((int)threadIdx.x < 4 * N1) RT[threadIdx.x] = rt;
  if constexpr (S::CTN <= BD) {
    if ((int)threadIdx.x < S::CTN) CT[threadIdx.x] = ct;
  } else {
    for (int k = threadIdx.x; k < S::CTN; k += BD) CT[k] = st[2 * L - S::CT0 + k];
  }
  __syncthreads();
  const double2* Ec = CT + S::CT0;
  const double2* Wl = CT;           // element-parallel form: Wc, Vc in LDS
  const double2* Vl = CT + L;
  const double2 F0 = Ec[N1], F1 = Ec[N1 + 1], F2 = Ec[N1 + 2], F3 = Ec[N1 + 3];
  const double* Dlo = RT;
  const double* Dhi = RT + N1;
  const double* C0 = RT + 2 * N1;
  const double* C1 = RT + 3 * N1;
  // g = Fi [x_lo, x_hi] on every line, in place (and kept in registers when G
  // shares X's space)
  double2 ga[GX ? NGL : 1], gb[GX ? NGL : 1];
#pragma unroll
  for (int k = 0; k < NGL; ++k) {
    const int ln = threadIdx.x + k * BD;
    if (ln < 3 * L) {
      const int ax = ln / L, pos = ln - ax * L;
      const double2 lo = G[2 * ax * L + pos], hi = G[(2 * ax + 1) * L + pos];
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      cfma(a, F0, lo);
      cfma(a, F1, hi);
      cfma(b, F2, lo);
      cfma(b, F3, hi);
      G[2 * ax * L + pos] = a;
      G[(2 * ax + 1) * L + pos] = b;
      if constexpr (GX) {
        ga[k] = a;
        gb[k] = b;
      }
    }
  }
  __syncthreads();
  // r_i = x_i - A_ib g  (A_ib: -D2[1 + i][{0, p-1}] towards the two ends of each line)
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int i = m % N1, j = (m / N1) % N1, k = m / L;
    const int li = lidx<P>(i, j, k);
    double2 s = T[li];
    cfma_r(s, C0[i], G[0 * L + j + N1 * k]);
    cfma_r(s, C1[i], G[1 * L + j + N1 * k]);
    cfma_r(s, C0[j], G[2 * L + i + N1 * k]);
    cfma_r(s, C1[j], G[3 * L + i + N1 * k]);
    cfma_r(s, C0[k], G[4 * L + i + N1 * j]);
    cfma_r(s, C1[k], G[5 * L + i + N1 * j]);
    T[li] = s;
  }
  __syncthreads();
  // u_i = (Vc x Vc x Vc) diag(1 / (-Ec_Delta - lambda)) (Wc x Wc x Wc) r_i
  // (ping-pong T -> X -> T ..., ending in T; in place: all in T)
  double2* const X1 = (S::IP || S::SIP) ? T : X;
  cmode<P, 0, false, false>(T, X1, Wc, Wl, Ec, lm, lanes);
  __syncthreads();
  cmode<P, 1, false, false>(X1, T, Wc, Wl, Ec, lm, lanes);
  __syncthreads();
  cmode<P, 2, true, false>(T, X1, Wc, Wl, Ec, lm, lanes);
  __syncthreads();
  cmode<P, 0, false, true>(X1, T, Vc, Vl, Ec, lm, lanes);
  __syncthreads();
  cmode<P, 1, false, true>(T, X1, Vc, Vl, Ec, lm, lanes);
  __syncthreads();
  cmode<P, 2, false, true>(X1, T, Vc, Vl, Ec, lm, lanes);
  __syncthreads();
  if constexpr (kSepSplit<P>) {
    split_butterflies<P>(T);
    __syncthreads();
  }
  for (int m = threadIdx.x; m < NI; m += BD) {
    const int i = m % N1, j = (m / N1) % N1, k = m / L;
    st2(yv, m, T[lidx<P>(i, j, k)]);
  }
  // u_b = g - Fi Fbi1 u_line,  Fbi1 u_line = [-sum Dlo u, sum Dhi u]
#pragma unroll
  for (int k = 0; k < NGL; ++k) {
    const int ln = threadIdx.x + k * BD;
    if (ln >= 3 * L) break;
    const int ax = ln / L, pos = ln - ax * L;
    int base, stride;
    line_of<P>(ax, pos % N1, pos / N1, base, stride);
    double2 slo = make_double2(0.0, 0.0), shi = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < N1; ++t) {
      const double2 u = T[base + t * stride];
      cfma_r(slo, -Dlo[t], u);
      cfma_r(shi, Dhi[t], u);
    }
    double2 a, b;
    if constexpr (GX) {
      a = ga[k];
      b = gb[k];
    } else {
      a = G[2 * ax * L + pos];
      b = G[(2 * ax + 1) * L + pos];
    }
    double2 fa = make_double2(0.0, 0.0), fb = make_double2(0.0, 0.0);
    cfma(fa, F0, slo);
    cfma(fa, F1, shi);
    cfma(fb, F2, slo);
    cfma(fb, F3, shi);
    st2(yv, NI + 2 * ax * L + pos, csub(a, fa));
    st2(yv, NI + (2 * ax + 1) * L + pos, csub(b, fb));
  }
}

template <int P, typename VT>
int sep_launch(hps_ctx* c, const VT* x, const VT* g, VT* y, int nrhs, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((unsigned)c->nl, (unsigned)nrhs);
  const dim3 block(SL<P>::BD);
  const int64_t os = c->nop > 1 ? c->nl : 0;
  const hipError_t e = launch_k(c, e0, e1, k_precond_sep<P, VT>, grid, block, x, g, c->d_nbr, y,
                                c->d_lambda, c->d_sep, c->d_tab, c->nl, c->N, os);
  return check_hip(e, "k_precond_sep");
}

}  // namespace

namespace {

template <typename VT>
int sep_dispatch(hps_ctx* c, const VT* x, const VT* g, VT* y, int nrhs, hipEvent_t e0, hipEvent_t e1) {
  if (!c->sep || !c->d_sep) return fail(HPS_ERR_ARG, "the separable J^-1 was not built at setup");
  if (c->nop > 1 && nrhs != c->nop) return fail(HPS_ERR_ARG, "operator group: one right-hand side per operator");
  if (nrhs > 65535) return fail(HPS_ERR_ARG, "at most 65535 right-hand sides per call");
  switch (c->p) {
    case 4: return sep_launch<4>(c, x, g, y, nrhs, e0, e1);
    case 5: return sep_launch<5>(c, x, g, y, nrhs, e0, e1);
    case 6: return sep_launch<6>(c, x, g, y, nrhs, e0, e1);
    case 7: return sep_launch<7>(c, x, g, y, nrhs, e0, e1);
    case 8: return sep_launch<8>(c, x, g, y, nrhs, e0, e1);
    case 9: return sep_launch<9>(c, x, g, y, nrhs, e0, e1);
    case 10: return sep_launch<10>(c, x, g, y, nrhs, e0, e1);
    case 11: return sep_launch<11>(c, x, g, y, nrhs, e0, e1);
    case 12: return sep_launch<12>(c, x, g, y, nrhs, e0, e1);
    case 13: return sep_launch<13>(c, x, g, y, nrhs, e0, e1);
    case 14: return sep_launch<14>(c, x, g, y, nrhs, e0, e1);
    case 15: return sep_launch<15>(c, x, g, y, nrhs, e0, e1);
    case 16: return sep_launch<16>(c, x, g, y, nrhs, e0, e1);
    default: return fail(HPS_ERR_UNSUPPORTED, "p out of range");
  }
}

}  // namespace

int launch_precond_sep(hps_ctx* c, const double2* x, const double2* g, double2* y, int nrhs,
                       hipEvent_t e0, hipEvent_t e1) {
  return sep_dispatch(c, x, g, y, nrhs, e0, e1);
}

int launch_precond_sep(hps_ctx* c, const float2* x, const float2* g, float2* y, int nrhs,
                       hipEvent_t e0, hipEvent_t e1) {
  return sep_dispatch(c, x, g, y, nrhs, e0, e1);
}

}  // namespace hps
