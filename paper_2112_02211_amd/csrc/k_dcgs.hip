// Kernels of the Arnoldi process with delayed reorthogonalization (see
// hps_krylov.h): per step one reduction pass and one update pass over the
// basis.  The small Hessenberg / Givens work of a step runs in workgroup 0 of
// the update pass, off the critical path; a standalone kernel closes the last
// column of a cycle.
// Reductions are deterministic (fixed order), as in k_krylov.hip.
#include "hps_internal.h"
#include "hps_krylov.h"
#include "k_common.h"
#include "k_vec.h"

namespace hps {
namespace {

// Non-temporal basis loads (template flag NT) for long vectors, in the update
// pass and the short-basis reduction: a basis of more than a few hundred MB
// leaves the caches before it is read again (all vector stores carry the hint,
// see st2).  Measured on 6.5M-entry vectors (16^3 leaves, p = 12), together with
// the update pass's stores: update pass 551 -> 483 us, short-basis reduction
// 133 -> 112 us; on 0.46M-entry ones (8^3, p = 10), whose vectors live in the
// last-level cache, the solve was 7 % slower, hence the threshold.  The hint
// slowed the other reductions (2-10 %: there eight wavefronts share u and w
// through the cache) and non-temporal loads of u and w slowed every pass.
constexpr int64_t kNtVector = int64_t(1) << 21;
// Tiles per pass of the split-over-basis reduction (all their loads issued
// before the first use): two for FP32-stored vectors, whose 8-byte loads keep
// half as many bytes in flight (inner solve of iterative refinement on 6.5M
// entries: 236 -> 228 ms), one for FP64 (two: 1.3 % slower).
template <typename VT> constexpr int red_tiles() { return sizeof(VT) == 8 ? 2 : 1; }

constexpr int DW = 8;          // wavefronts of the reduction workgroup (split over k)
constexpr int DT = 64 * DW;    // its threads; one tile = 64 vector entries
constexpr int UT = 256;        // update-pass (and small-step) workgroup
constexpr double kBreakdownTol = 1e-14;  // beta^2 <= tol * ||u||^2: the candidate is in the span
constexpr int64_t kMidVector = 1 << 24;  // reduction grid sizes below / from here
constexpr int kCloseMaxJ = 12;           // last steps whose update pass takes the closing reduction
constexpr int kShortBasis = 12;          // reductions over at most this many basis vectors ...
constexpr int64_t kLongVector = 1 << 21; // ... of at least this many entries split tiles over wavefronts
                                         // (measured: 3 % slower on 0.46M-entry vectors, where u and w
                                         // re-reads hit in cache; faster from 3.67M entries on: the
                                         // 64-vector lock-step solve of those took 9.87 -> 9.46 s).
                                         // Twelve, with one instantiation per basis size, covers every
                                         // reduction of GMRES(10) (the closing one included): on 6.5M
                                         // entries the FP64 solve took 128.6 -> 127.6 ms and iterative
                                         // refinement 124.9 -> 118.2 ms against eight with one
                                         // eight-vector instantiation (sixteen: no further change;
                                         // 1024 workgroups instead of 512: 1 % slower)

// Partials of a_k = sum conj(V_k) u, b_k = sum conj(V_k) w (k < J), c = sum |u|^2,
// d = sum conj(u) w.  Wavefront ky owns basis vectors ky*kc .. ky*kc+kc-1 of the
// tile; wavefront 0 also accumulates c and d.
template <int KC, bool HASW, typename VT>
__global__ __launch_bounds__(DT) void k_dcgs_reduce(const VT* __restrict__ V, int64_t ldv,
                                                    int64_t vbs, int J, const VT* __restrict__ u,
                                                    int64_t ubs, const VT* __restrict__ w,
                                                    int64_t wbs, int64_t n,
                                                    double2* __restrict__ part) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  u += bz * ubs;
  if (HASW) w += bz * wbs;
  const int lane = threadIdx.x & 63, ky = threadIdx.x >> 6;
  const int kc = (J + DW - 1) / DW;
  const int k0 = ky * kc;
  const int kn = max(0, min(kc, J - k0));
  double2 aa[KC], ab[KC];
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) { aa[kk] = make_double2(0.0, 0.0); ab[kk] = make_double2(0.0, 0.0); }
  double cc = 0.0;
  double2 dd = make_double2(0.0, 0.0);
  const unsigned nblk = gridDim.x;
  constexpr int RT = red_tiles<VT>();
  for (int64_t t0 = (int64_t)blockIdx.x * 64 * RT; t0 < n; t0 += (int64_t)nblk * 64 * RT) {
    VT ur[RT], wr[RT], rr[RT][KC];
    bool okt[RT];
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const int64_t i = t0 + s * 64 + lane;
      const bool ok = i < n;
      const int64_t is = ok ? i : n - 1;   // in-bounds entry for unconditional FP32 loads
      okt[s] = ok;
      ur[s] = ld_tile(u, i, is, ok);
      wr[s] = VT{};   // no load at all without w (w is null then)
      if constexpr (HASW) wr[s] = ld_tile(w, i, is, ok);
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const bool c = kk < kn && ok;
        const int ks = k0 + kk < J ? k0 + kk : 0;
        rr[s][kk] = ld_tile(V, (int64_t)(k0 + kk) * ldv + i, (int64_t)ks * ldv + is, c);
      }
    }
#pragma unroll
    for (int s = 0; s < RT; ++s) {
      const bool ok = okt[s];
      const double2 uv = widen(ur[s], ok);
      const double2 wv = widen(wr[s], HASW && ok);
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) {
        const double2 vr = widen(rr[s][kk], kk < kn && ok);
        aa[kk].x = fma(vr.x, uv.x, fma(vr.y, uv.y, aa[kk].x));
        aa[kk].y = fma(vr.x, uv.y, fma(-vr.y, uv.x, aa[kk].y));
        if (HASW) {
          ab[kk].x = fma(vr.x, wv.x, fma(vr.y, wv.y, ab[kk].x));
          ab[kk].y = fma(vr.x, wv.y, fma(-vr.y, wv.x, ab[kk].y));
        }
      }
      if (ky == 0) {
        cc = fma(uv.x, uv.x, fma(uv.y, uv.y, cc));
        if (HASW) {
          dd.x = fma(uv.x, wv.x, fma(uv.y, wv.y, dd.x));
          dd.y = fma(uv.x, wv.y, fma(-uv.y, wv.x, dd.y));
        }
      }
    }
  }
  double2* pz = part + (int64_t)bz * kPartSlots * nblk;
#pragma unroll
  for (int kk = 0; kk < KC; ++kk) {
    if (kk < kn) {
      const double ar = wave_sum(aa[kk].x), ai = wave_sum(aa[kk].y);
      if (lane == 0) pz[(int64_t)(k0 + kk) * nblk + blockIdx.x] = make_double2(ar, ai);
      if (HASW) {
        const double br = wave_sum(ab[kk].x), bi = wave_sum(ab[kk].y);
        if (lane == 0) pz[(int64_t)(kSlotB + k0 + kk) * nblk + blockIdx.x] = make_double2(br, bi);
      }
    }
  }
  if (ky == 0) {
    const double cs = wave_sum(cc);
    const double dr = wave_sum(dd.x), di = wave_sum(dd.y);
    if (lane == 0) {
      pz[(int64_t)kSlotC * nblk + blockIdx.x] = make_double2(cs, 0.0);
      pz[(int64_t)kSlotD * nblk + blockIdx.x] = make_double2(dr, di);
    }
  }
}

// The same partials with the tiles split over the wavefronts instead of the
// basis vectors (for short bases on long vectors): wavefront ky of workgroup g
// takes tiles g * DW + ky, g * DW + ky + DW * nblk, ...; each reads the J <= JM
// basis entries, u and w of its tile once (the split over basis vectors has
// every wavefront read u and w, and leaves wavefronts idle when J < DW).  The
// DW wavefront sums are added in a fixed order through LDS.
template <int JM, bool HASW, typename VT, bool NT>
__global__ __launch_bounds__(DT) void k_dcgs_reduce_es(const VT* __restrict__ V, int64_t ldv,
                                                       int64_t vbs, int J, const VT* __restrict__ u,
                                                       int64_t ubs, const VT* __restrict__ w,
                                                       int64_t wbs, int64_t n,
                                                       double2* __restrict__ part) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  u += bz * ubs;
  if (HASW) w += bz * wbs;
  const int lane = threadIdx.x & 63, ky = threadIdx.x >> 6;
  double2 aa[JM], ab[JM];
#pragma unroll
  for (int k = 0; k < JM; ++k) { aa[k] = make_double2(0.0, 0.0); ab[k] = make_double2(0.0, 0.0); }
  double cc = 0.0;
  double2 dd = make_double2(0.0, 0.0);
  const unsigned nblk = gridDim.x;
  for (int64_t t0 = ((int64_t)blockIdx.x * DW + ky) * 64; t0 < n; t0 += (int64_t)nblk * DW * 64) {
    const int64_t i = t0 + lane;
    const bool ok = i < n;
    const int64_t is = ok ? i : n - 1;
    const VT ur = ld_tile(u, i, is, ok);
    VT wr{};   // no load at all without w (w is null then)
    if constexpr (HASW) wr = ld_tile(w, i, is, ok);
    VT rr[JM];
#pragma unroll
    for (int k = 0; k < JM; ++k)
      rr[k] = ld_tile_h<NT>(V, (int64_t)k * ldv + i, (int64_t)(k < J ? k : 0) * ldv + is, k < J && ok);
    const double2 uv = widen(ur, ok);
    const double2 wv = widen(wr, HASW && ok);
    double2 vr[JM];
#pragma unroll
    for (int k = 0; k < JM; ++k) vr[k] = widen(rr[k], k < J && ok);
#pragma unroll
    for (int k = 0; k < JM; ++k) {
      aa[k].x = fma(vr[k].x, uv.x, fma(vr[k].y, uv.y, aa[k].x));
      aa[k].y = fma(vr[k].x, uv.y, fma(-vr[k].y, uv.x, aa[k].y));
      if (HASW) {
        ab[k].x = fma(vr[k].x, wv.x, fma(vr[k].y, wv.y, ab[k].x));
        ab[k].y = fma(vr[k].x, wv.y, fma(-vr[k].y, wv.x, ab[k].y));
      }
    }
    cc = fma(uv.x, uv.x, fma(uv.y, uv.y, cc));
    if (HASW) {
      dd.x = fma(uv.x, wv.x, fma(uv.y, wv.y, dd.x));
      dd.y = fma(uv.x, wv.y, fma(-uv.y, wv.x, dd.y));
    }
  }
  // wavefront sums: slots 0..J-1 (a), JM..JM+J-1 (b), 2 JM (c), 2 JM + 1 (d)
  constexpr int NS = 2 * JM + 2;
  __shared__ double2 red[DW][NS];
#pragma unroll
  for (int k = 0; k < JM; ++k) {
    if (k < J) {
      const double ar = wave_sum(aa[k].x), ai = wave_sum(aa[k].y);
      if (lane == 0) red[ky][k] = make_double2(ar, ai);
      if (HASW) {
        const double br = wave_sum(ab[k].x), bi = wave_sum(ab[k].y);
        if (lane == 0) red[ky][JM + k] = make_double2(br, bi);
      }
    }
  }
  {
    const double cs = wave_sum(cc);
    const double dr = wave_sum(dd.x), di = wave_sum(dd.y);
    if (lane == 0) {
      red[ky][2 * JM] = make_double2(cs, 0.0);
      red[ky][2 * JM + 1] = make_double2(dr, di);
    }
  }
  __syncthreads();
  double2* pz = part + (int64_t)bz * kPartSlots * nblk;
  const int t = threadIdx.x;
  if (t < NS) {
    const bool isa = t < J, isb = HASW && t >= JM && t < JM + J, isc = t == 2 * JM,
               isd = t == 2 * JM + 1;   // d = 0 without w, as the other form writes it
    if (isa || isb || isc || isd) {
      double2 v = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < DW; ++q) v = cadd(v, red[q][t]);
      const int slot = isa ? t : (isb ? kSlotB + (t - JM) : (isc ? kSlotC : kSlotD));
      pz[(int64_t)slot * nblk + blockIdx.x] = v;
    }
  }
}

// Finish the partials of the slots in use into S[b].red: wavefront q of the grid
// handles slot q (< J), 64 + (q - J) (< 2J, only with w), then c and d.
__global__ __launch_bounds__(256) void k_dcgs_finish(const double2* __restrict__ part, int J,
                                                     int hasw, int nblk, DcgsState* __restrict__ S) {
  const int bz = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nb_slots = hasw ? 2 * J : J;
  int slot;
  if (q < J) slot = q;
  else if (q < nb_slots) slot = kSlotB + (q - J);
  else if (q == nb_slots) slot = kSlotC;
  else if (q == nb_slots + 1 && hasw) slot = kSlotD;
  else return;
  const double2* pp = part + ((int64_t)bz * kPartSlots + slot) * nblk;
  double re = 0.0, im = 0.0;
  for (int b = lane; b < nblk; b += 64) {
    const double2 v = pp[b];
    re += v.x;
    im += v.y;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) S[bz].red[slot] = make_double2(re, im);
}

__global__ void k_dcgs_start(DcgsState* __restrict__ S, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  DcgsState& s = S[b];
  s.flag = 0;
  s.ncols = 0;
  s.res = 0.0;
  s.beta0 = 0.0;   // set by step 0 unless the cycle's first candidate breaks down
  for (int i = 0; i < kDcgsLd; ++i) s.gls[i] = make_double2(0.0, 0.0);
}

// Shared memory of the coefficient and small-step phases of one workgroup.
struct SmallSmem {
  double2 a[kMaxDcgs];      // a = V^H u_j
  double2 b[kDcgsLd];       // b = V^H w
  double2 colh[kDcgsLd];    // Hessenberg column j-1 as built
  double2 colr[kDcgsLd];    // its Givens-rotated copy
  double2 sn[kMaxDcgs];
  double cs[kMaxDcgs];
  double2 ph[UT / 64][kDcgsLd];  // Hbar a over the stored columns, one partial per wavefront
  double2 pt[UT / 64][kMaxDcgs]; // T a, likewise
  double sc[6];                  // beta^2, c, Re/Im a^H b, Re/Im d
};

// Step coefficients from the finished reductions.  Every workgroup that needs
// them computes them with the same operations in the same order, so they all
// take the same breakdown decision.
struct Coef {
  double beta2, c, inv;
  double2 vjw;  // (d - a^H b) / beta
  bool ok;      // false: the candidate lies in the span of the basis (or is not finite)
};

__device__ __forceinline__ Coef dcgs_coeffs(const DcgsState& s, int j, bool hasw, SmallSmem& sm,
                                            double tiny) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const double2 z2 = make_double2(0.0, 0.0);
    const double2 al = lane < j ? s.red[lane] : z2;
    const double2 bl = (hasw && lane < j) ? s.red[kSlotB + lane] : z2;
    sm.a[lane] = al;
    sm.b[lane] = bl;
    const double na2 = wave_sum(al.x * al.x + al.y * al.y);
    const double abr = wave_sum(al.x * bl.x + al.y * bl.y);   // conj(a) b
    const double abi = wave_sum(al.x * bl.y - al.y * bl.x);
    if (lane == 0) {
      const double c = s.red[kSlotC].x;
      const double2 d = hasw ? s.red[kSlotD] : z2;
      sm.sc[0] = c - na2;
      sm.sc[1] = c;
      sm.sc[2] = abr;
      sm.sc[3] = abi;
      sm.sc[4] = d.x;
      sm.sc[5] = d.y;
    }
  }
  __syncthreads();
  Coef cf;
  cf.beta2 = sm.sc[0];
  cf.c = sm.sc[1];
  cf.ok = (cf.beta2 > tiny * cf.c) && isfinite(cf.beta2);
  cf.inv = cf.ok ? 1.0 / sqrt(cf.beta2) : 0.0;
  cf.vjw = make_double2((sm.sc[4] - sm.sc[2]) * cf.inv, (sm.sc[5] - sm.sc[3]) * cf.inv);
  return cf;
}

// Record {estimate, stopped, tag} of a step; the tag is stored last with a
// system-scope release, so a reader that sees the tag sees the rest (ro may
// point into pinned host memory).
__device__ __forceinline__ void publish(double* ro, double res, double stopped,
                                        unsigned long long tag) {
  ro[0] = res;
  ro[1] = stopped;
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(ro + 2), tag, __ATOMIC_RELEASE,
                     __HIP_MEMORY_SCOPE_SYSTEM);
}

// The small work of step j for one right-hand side, by one workgroup of UT
// threads: column j-1 of the Hessenberg matrix is g_{j-1} + a with beta below
// it; it is rotated by the earlier Givens rotations and a new rotation zeroes
// beta (updating the least-squares right-hand side and the residual estimate).
// Unless final_only, g_j = ([b; vjw] - Hbar a) / beta and, flexible, column j
// of T are formed.  flag: an earlier step stopped this cycle.  Publishes the
// record ro = {residual estimate, stopped, tag}.
__device__ void dcgs_small_step(DcgsState& s, int j, int flexible, int final_only, double* ro,
                                unsigned long long tag, SmallSmem& sm, const Coef& cf, int flag) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int ld = kDcgsLd;
  if (flag || !cf.ok) {
    if (tid == 0) {
      if (!flag) s.flag = 1;  // the cycle ends with the columns finished so far
      publish(ro, s.res, 1.0, tag);
    }
    return;
  }
  const double beta = sqrt(cf.beta2), inv = cf.inv;
  const double2 z2 = make_double2(0.0, 0.0);
  // wavefront 0: the state this step reads, loaded before anything waits
  double2 gp = z2, snv = z2, g0 = z2;
  double csv = 0.0;
  if (wv == 0 && j > 0) {
    if (lane < j) gp = s.gprev[lane];
    if (lane < j - 1) {
      csv = s.cs[lane];
      snv = s.sn[lane];
    }
    if (lane == 0) g0 = s.gls[j - 1];
  }
  // partial products over the stored columns 0 .. j-2 of H and 0 .. j-1 of T:
  // thread (wavefront wv, lane i) takes row i and columns 16 wv .. 16 wv + 15.
  // Out-of-range terms read an in-bounds entry and are discarded by a select.
  // (Unrolled by 2 only: this runs inside the update pass, whose occupancy
  // is set by the larger of the two register counts.)
  if (!final_only) {
    const int i = lane;
    double2 ph = z2, pt = z2;
#pragma unroll 2
    for (int k = 0; k < 16; ++k) {
      const int l = 16 * wv + k;
      const bool in = (l <= j - 2) && (l + 1 >= i) && (i <= j);
      const int lc = in ? l : 0;
      const double2 pr = cmul(s.H[i + ld * lc], sm.a[lc]);
      ph.x += in ? pr.x : 0.0;
      ph.y += in ? pr.y : 0.0;
    }
    if (flexible) {
#pragma unroll 2
      for (int k = 0; k < 16; ++k) {
        const int l = 16 * wv + k;
        const bool in = (l < j) && (l >= i);
        const int lc = in ? l : 0;
        const double2 pr = cmul(s.T[i + kMaxDcgs * lc], sm.a[lc]);
        pt.x += in ? pr.x : 0.0;
        pt.y += in ? pr.y : 0.0;
      }
    }
    sm.ph[wv][i] = ph;
    sm.pt[wv][i] = pt;
  }
  if (wv == 0 && j > 0) {
    // column j-1 as built
    if (lane < j) {
      const double2 h = cadd(gp, sm.a[lane]);
      s.H[lane + ld * (j - 1)] = h;
      sm.colh[lane] = h;
    }
    if (lane == 0) {
      s.H[j + ld * (j - 1)] = make_double2(beta, 0.0);
      sm.colh[j] = make_double2(beta, 0.0);
    }
    if (lane < j - 1) {
      sm.cs[lane] = csv;
      sm.sn[lane] = snv;
    }
  }
  __syncthreads();
  if (j == 0) {
    if (tid == 0) {
      s.beta0 = beta;
      s.gls[0] = make_double2(beta, 0.0);
      s.res = beta;
      s.ncols = 0;
    }
  } else if (tid == 0) {
    // earlier rotations, carried in registers; the new rotation zeroes beta
    double2 cur = sm.colh[0];
    for (int i = 0; i < j - 1; ++i) {
      const double cr = sm.cs[i];
      const double2 sn = sm.sn[i], nx = sm.colh[i + 1];
      sm.colr[i] = cadd(cscale(cur, cr), cmul(sn, nx));
      cur = csub(cscale(nx, cr), cmulc(sn, cur));
    }
    const double am = sqrt(cur.x * cur.x + cur.y * cur.y);
    const double r = sqrt(am * am + cf.beta2);
    double cr;
    double2 sn;
    if (am == 0.0) {
      cr = 0.0;
      sn = make_double2(1.0, 0.0);
      sm.colr[j - 1] = make_double2(beta, 0.0);
    } else {
      cr = am / r;
      const double2 ph = make_double2(cur.x / am, cur.y / am);
      sn = make_double2(ph.x * beta / r, ph.y * beta / r);
      sm.colr[j - 1] = make_double2(ph.x * r, ph.y * r);
    }
    sm.colr[j] = z2;
    s.cs[j - 1] = cr;
    s.sn[j - 1] = sn;
    const double2 g1 = make_double2(-(sn.x * g0.x + sn.y * g0.y), -(sn.x * g0.y - sn.y * g0.x));
    s.gls[j] = g1;
    s.gls[j - 1] = cscale(g0, cr);
    s.res = sqrt(g1.x * g1.x + g1.y * g1.y);
    s.ncols = j;
  }
  if (!final_only && wv == 1) {
    // g_j = ([b; vjw] - Hbar a) / beta, with column j-1 of Hbar from colh
    for (int i = lane; i <= j; i += 64) {
      double2 ha = cadd(cadd(sm.ph[0][i], sm.ph[1][i]), cadd(sm.ph[2][i], sm.ph[3][i]));
      if (j > 0) ha = cadd(ha, cmul(sm.colh[i], sm.a[j - 1]));
      const double2 vw = (i < j) ? sm.b[i] : cf.vjw;
      s.gprev[i] = cscale(csub(vw, ha), inv);
    }
    // flexible: z_j = (z'_j - Z_{j-1} a) / beta, i.e. T[:, j] = (e_j - T[:, 0:j] a) / beta
    if (flexible) {
      for (int i = lane; i < j; i += 64) {
        const double2 ta = cadd(cadd(sm.pt[0][i], sm.pt[1][i]), cadd(sm.pt[2][i], sm.pt[3][i]));
        s.T[i + kMaxDcgs * j] = cscale(ta, -inv);
      }
      if (lane == 0) s.T[j + kMaxDcgs * j] = make_double2(inv, 0.0);
    }
  }
  __syncthreads();
  if (wv == 0 && j > 0)
    for (int i = lane; i <= j; i += 64) s.R[i + ld * (j - 1)] = sm.colr[i];
  if (tid == 0) publish(ro, s.res, 0.0, tag);
}

// Standalone small step (closes the last column of a cycle, final_only).
__global__ __launch_bounds__(UT) void k_dcgs_small(DcgsState* __restrict__ S, int j, int flexible,
                                                   int final_only, double* __restrict__ res_out,
                                                   unsigned long long tag, double tiny) {
  DcgsState& s = S[blockIdx.x];
  __shared__ SmallSmem sm;
  const int flag = s.flag;
  const Coef cf = dcgs_coeffs(s, j, !final_only, sm, tiny);
  dcgs_small_step(s, j, flexible, final_only, res_out + 4 * blockIdx.x, tag, sm, cf, flag);
}

// Update pass of step J, with the small step in workgroup 0 of each right-hand side:
// V[J] = (u - V_{0..J-1} a) / beta;  u <- (w - V_{0..J-1} b - V[J] vjw) / beta.
template <typename VT, bool NT>
__global__ __launch_bounds__(UT) void k_dcgs_update(VT* __restrict__ V, int64_t ldv, int64_t vbs,
                                                    int J, VT* __restrict__ u, int64_t ubs,
                                                    const VT* __restrict__ w, int64_t wbs,
                                                    int64_t n, DcgsState* __restrict__ S,
                                                    int flexible, double* __restrict__ res_out,
                                                    unsigned long long tag, double tiny) {
  const int bz = blockIdx.z;
  DcgsState& s = S[bz];
  __shared__ SmallSmem sm;
  const int flag = s.flag;
  const Coef cf = dcgs_coeffs(s, J, true, sm, tiny);
  if (blockIdx.x == 0) dcgs_small_step(s, J, flexible, 0, res_out + 4 * bz, tag, sm, cf, flag);
  if (flag || !cf.ok) return;
  V += bz * vbs;
  u += bz * ubs;
  w += bz * wbs;
  const double inv = cf.inv;
  const double2 cj = cf.vjw;
  const double2* ca = sm.a;
  const double2* cb = sm.b;
  for (int64_t i = (int64_t)blockIdx.x * UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT) {
    double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
    // eight basis vectors per round, the last round predicated (its loads still
    // issue together; coefficients beyond J are zero and so are skipped loads)
    for (int l = 0; l < J; l += 8) {
      VT r[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        r[q] = ld_tile_h<NT>(V, (int64_t)(l + q) * ldv + i, (int64_t)l * ldv + i, l + q < J);
      double2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = widen(r[q], l + q < J);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double2 x = ca[l + q], y = cb[l + q];
        sa.x = fma(v[q].x, x.x, fma(-v[q].y, x.y, sa.x));
        sa.y = fma(v[q].x, x.y, fma(v[q].y, x.x, sa.y));
        sb.x = fma(v[q].x, y.x, fma(-v[q].y, y.y, sb.x));
        sb.y = fma(v[q].x, y.y, fma(v[q].y, y.x, sb.y));
      }
    }
    const double2 uv = widen(ld_tile(u, i, i, true), true);
    const double2 wv = widen(ld_tile(w, i, i, true), true);
    const double2 vj = make_double2((uv.x - sa.x) * inv, (uv.y - sa.y) * inv);
    const double2 t = cmul(vj, cj);
    st2(V, (int64_t)J * ldv + i, vj);
    st2(u, i, make_double2((wv.x - sb.x - t.x) * inv, (wv.y - sb.y - t.y) * inv));
  }
}

// The update pass of the last step J of a cycle with the cycle's closing
// reduction folded in: besides V[J] and the new candidate u it writes, per
// workgroup, the partials of a_k = sum conj(V_k) u (k <= J, V_J included) and
// c = sum |u|^2 of that new candidate (the reduction k_dcgs_reduce would
// otherwise make over the J + 1 basis vectors and u without w).  Every basis
// entry is already in registers, so the reduction costs no HBM traffic.  The
// grid is at most kRedBlocks workgroups, each thread taking entries with a
// grid stride; one instantiation per J (JM = J: the loads carry no predicate).  When the step breaks down
// (or the cycle already stopped) the partials are zero and unused: the
// closing small step then sees the cycle's stop flag.
template <typename VT, bool NT, int JM>
__global__ __launch_bounds__(UT) void k_dcgs_update_close(VT* __restrict__ V, int64_t ldv, int64_t vbs,
                                                          int J, VT* __restrict__ u, int64_t ubs,
                                                          const VT* __restrict__ w, int64_t wbs,
                                                          int64_t n, DcgsState* __restrict__ S,
                                                          int flexible, double* __restrict__ res_out,
                                                          unsigned long long tag, double tiny,
                                                          double2* __restrict__ part) {
  const int bz = blockIdx.z;
  DcgsState& s = S[bz];
  constexpr int JA = JM > 0 ? JM : 1;   // array sizes
  __shared__ SmallSmem sm;
  __shared__ double2 red[UT / 64][JM + 2];
  const int flag = s.flag;
  const Coef cf = dcgs_coeffs(s, JM, true, sm, tiny);
  if (blockIdx.x == 0) dcgs_small_step(s, JM, flexible, 0, res_out + 4 * bz, tag, sm, cf, flag);
  (void)J;
  const unsigned nblk = gridDim.x;
  double2* pz = part + (int64_t)bz * kPartSlots * nblk;
  if (flag || !cf.ok) {
    if ((int)threadIdx.x <= JM) pz[(int64_t)threadIdx.x * nblk + blockIdx.x] = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) pz[(int64_t)kSlotC * nblk + blockIdx.x] = make_double2(0.0, 0.0);
    return;
  }
  V += bz * vbs;
  u += bz * ubs;
  w += bz * wbs;
  const double inv = cf.inv;
  const double2 cj = cf.vjw;
  const double2* ca = sm.a;
  const double2* cb = sm.b;
  double2 acc[JM + 1];
#pragma unroll
  for (int q = 0; q <= JM; ++q) acc[q] = make_double2(0.0, 0.0);
  double cc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * UT + threadIdx.x; i < n; i += (int64_t)nblk * UT) {
    // the step coefficients are read from LDS again on every pass (held in
    // registers they took 8 VGPRs per basis vector: 182 instead of 124 at
    // J = 9, two waves per SIMD instead of four)
    asm volatile("" ::: "memory");
    VT r[JA];
#pragma unroll
    for (int q = 0; q < JM; ++q) r[q] = NT ? ld_nt2(V + (int64_t)q * ldv + i) : V[(int64_t)q * ldv + i];
    const double2 uv = widen(ld_tile(u, i, i, true), true);
    const double2 wv = widen(ld_tile(w, i, i, true), true);
    double2 v[JA];
#pragma unroll
    for (int q = 0; q < JM; ++q) v[q] = widen(r[q], true);
    double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      const double2 x = ca[q], y = cb[q];
      sa.x = fma(v[q].x, x.x, fma(-v[q].y, x.y, sa.x));
      sa.y = fma(v[q].x, x.y, fma(v[q].y, x.x, sa.y));
      sb.x = fma(v[q].x, y.x, fma(-v[q].y, y.y, sb.x));
      sb.y = fma(v[q].x, y.y, fma(v[q].y, y.x, sb.y));
    }
    const double2 vj = make_double2((uv.x - sa.x) * inv, (uv.y - sa.y) * inv);
    const double2 t = cmul(vj, cj);
    const double2 un = make_double2((wv.x - sb.x - t.x) * inv, (wv.y - sb.y - t.y) * inv);
    st2(V, (int64_t)JM * ldv + i, vj);
    st2(u, i, un);
    // the closing sums over the values as stored
    const double2 vs = as_stored(vj, V), us = as_stored(un, u);
#pragma unroll
    for (int q = 0; q < JM; ++q) {
      acc[q].x = fma(v[q].x, us.x, fma(v[q].y, us.y, acc[q].x));
      acc[q].y = fma(v[q].x, us.y, fma(-v[q].y, us.x, acc[q].y));
    }
    acc[JM].x = fma(vs.x, us.x, fma(vs.y, us.y, acc[JM].x));
    acc[JM].y = fma(vs.x, us.y, fma(-vs.y, us.x, acc[JM].y));
    cc = fma(us.x, us.x, fma(us.y, us.y, cc));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q <= JM; ++q) {
    const double ar = wave_sum(acc[q].x), ai = wave_sum(acc[q].y);
    if (lane == 0) red[wv][q] = make_double2(ar, ai);
  }
  {
    const double cs = wave_sum(cc);
    if (lane == 0) red[wv][JM + 1] = make_double2(cs, 0.0);
  }
  __syncthreads();
  // slots 0 .. J: a_k (V_J included); slot C: c
  const int t = threadIdx.x;
  if (t <= JM + 1) {
    double2 v = red[0][t];
#pragma unroll
    for (int q = 1; q < UT / 64; ++q) v = cadd(v, red[q][t]);
    const int slot = t <= JM ? t : kSlotC;
    pz[(int64_t)slot * nblk + blockIdx.x] = v;
  }
}

// y = R^{-1} gls over k = min(kmax, ncols) columns (y zero beyond); flexible: y <- T y.
__global__ __launch_bounds__(64) void k_dcgs_trisolve(DcgsState* __restrict__ S, int kmax,
                                                      int flexible) {
  DcgsState& s = S[blockIdx.x];
  const int lane = threadIdx.x;
  const int k = min(kmax, s.ncols);
  __shared__ double2 g[kDcgsLd], y[kMaxDcgs];
  __shared__ double2 yi;
  for (int i = lane; i < kmax; i += 64) y[i] = make_double2(0.0, 0.0);
  for (int i = lane; i < k; i += 64) g[i] = s.gls[i];
  __syncthreads();
  const int ld = kDcgsLd;
  for (int i = k - 1; i >= 0; --i) {
    if (lane == 0) {
      const double2 dg = s.R[i + ld * i];
      const double dd = dg.x * dg.x + dg.y * dg.y;
      const double2 a = g[i];
      yi = dd > 0.0 ? make_double2((a.x * dg.x + a.y * dg.y) / dd, (a.y * dg.x - a.x * dg.y) / dd)
                    : make_double2(0.0, 0.0);
      y[i] = yi;
    }
    __syncthreads();
    const double2 v = yi;
    for (int l = lane; l < i; l += 64) g[l] = csub(g[l], cmul(s.R[l + ld * i], v));
    __syncthreads();
  }
  for (int i = lane; i < kmax; i += 64) {
    double2 out = y[i];
    if (flexible && i < k) {
      out = make_double2(0.0, 0.0);
      for (int l = i; l < k; ++l) out = cadd(out, cmul(s.T[i + kMaxDcgs * l], y[l]));
    }
    s.y[i] = out;
  }
}

// Restart coefficients (one wavefront per right-hand side), after trisolve:
// t = beta0 e_0 - Hbar_k y over rows 0 .. k (column l of Hbar holds rows
// 0 .. l + 1).  Closed last column (k = K): v_K = (u - V_K a) / beta is not
// stored, so its term t_K v_K = -y_{k-1} (u - V_K a) goes to rsig = -y_{k-1}
// and a y_{k-1} is added to the first K coefficients; otherwise (the cycle
// stopped after k columns) v_k is V[k] and t is the whole combination.  If
// the cycle's first candidate broke down (no V[0] written, beta0 still 0:
// a zero or non-finite residual) the residual stays u.
__global__ __launch_bounds__(64) void k_dcgs_restart_coef(DcgsState* __restrict__ S, int K) {
  DcgsState& s = S[blockIdx.x];
  const int lane = threadIdx.x;
  const int k = min(K, s.ncols);
  const bool closed = k == K;
  const double2 z2 = make_double2(0.0, 0.0);
  const double2 ylast = k > 0 ? s.y[k - 1] : z2;
  constexpr int ld = kDcgsLd;
  for (int i = lane; i < kDcgsLd; i += 64) {
    double2 t = make_double2(i == 0 ? s.beta0 : 0.0, 0.0);
    for (int l = max(0, i - 1); l < k; ++l) t = csub(t, cmul(s.H[i + ld * l], s.y[l]));
    if (closed) t = i < k ? cadd(t, cmul(s.red[i], ylast)) : z2;
    else if (i > k) t = z2;
    s.rc[i] = t;
  }
  const bool none = k == 0 && s.beta0 == 0.0;
  if (none)
    for (int i = lane; i < kDcgsLd; i += 64) s.rc[i] = z2;
  if (lane == 0) {
    s.rsig = closed ? make_double2(-ylast.x, -ylast.y) : (none ? make_double2(1.0, 0.0) : z2);
    s.rk = closed ? k : (none ? 0 : k + 1);
  }
}

// x += V y and u <- V rc + rsig u in one pass over the first rk basis vectors
// of each right-hand side (x's sum in the order of the plain multi-axpy: x
// first, then V[0], V[1], ...).  x may be stored in FP64 over an FP32 basis.
template <typename VT, typename XT, bool NT>
__global__ __launch_bounds__(UT) void k_dcgs_restart(const VT* __restrict__ V, int64_t ldv, int64_t vbs,
                                                     int K, VT* __restrict__ u, int64_t ubs,
                                                     XT* __restrict__ x, int64_t xbs, int64_t n,
                                                     const DcgsState* __restrict__ S) {
  const int bz = blockIdx.z;
  const DcgsState& s = S[bz];
  __shared__ double2 cy[kMaxDcgs + 8], cr[kMaxDcgs + 8];
  const int rk = min(s.rk, K);
  const int k8 = (rk + 7) / 8 * 8;
  for (int l = threadIdx.x; l < k8; l += UT) {
    cy[l] = l < rk ? s.y[l] : make_double2(0.0, 0.0);
    cr[l] = l < rk ? s.rc[l] : make_double2(0.0, 0.0);
  }
  const double2 sg = s.rsig;
  const bool use_u = sg.x != 0.0 || sg.y != 0.0;
  __syncthreads();
  V += bz * vbs;
  u += bz * ubs;
  x += bz * xbs;
  for (int64_t i = (int64_t)blockIdx.x * UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT) {
    double2 sx = widen(ld_tile(x, i, i, true), true);
    double2 su = make_double2(0.0, 0.0);
    for (int l = 0; l < rk; l += 8) {
      VT r[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        r[q] = ld_tile_h<NT>(V, (int64_t)(l + q) * ldv + i, (int64_t)l * ldv + i, l + q < rk);
      double2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = widen(r[q], l + q < rk);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double2 a = cy[l + q], b = cr[l + q];
        sx.x = fma(v[q].x, a.x, fma(-v[q].y, a.y, sx.x));
        sx.y = fma(v[q].x, a.y, fma(v[q].y, a.x, sx.y));
        su.x = fma(v[q].x, b.x, fma(-v[q].y, b.y, su.x));
        su.y = fma(v[q].x, b.y, fma(v[q].y, b.x, su.y));
      }
    }
    if (use_u) {
      const double2 uv = widen(ld_tile(u, i, i, true), true);
      su.x = fma(sg.x, uv.x, fma(-sg.y, uv.y, su.x));
      su.y = fma(sg.x, uv.y, fma(sg.y, uv.x, su.y));
    }
    st2(x, i, sx);
    st2(u, i, su);
  }
}

}  // namespace

namespace {

// The split reduction instantiated for JM = max(J, 1): registers for the basis
// vectors in use only (25-98 VGPRs for one to twelve vectors without w, 36-166
// with w; eight waves per SIMD up to four or five vectors).
template <bool HASW, typename VT, int JM = 1>
void launch_reduce_es(int J, dim3 grid, hipStream_t st, const VT* V, int64_t ldv, int64_t vbs,
                      const VT* u, int64_t ubs, const VT* w, int64_t wbs, int64_t n, double2* part) {
  if constexpr (JM < kShortBasis) {
    if (J > JM) return launch_reduce_es<HASW, VT, JM + 1>(J, grid, st, V, ldv, vbs, u, ubs, w, wbs, n, part);
  }
  hipLaunchKernelGGL((k_dcgs_reduce_es<JM, HASW, VT, true>), grid, dim3(DT), 0, st, V, ldv, vbs, J, u, ubs,
                     w, wbs, n, part);
}

template <typename VT>
int dcgs_reduce(hps_ctx* c, const VT* V, int64_t ldv, int64_t vbs, int J, const VT* u, int64_t ubs,
                const VT* w, int64_t wbs, int64_t n, DcgsState* S, int nbatch, const RedBuf& rb) {
  if (J > kMaxDcgs || nbatch > rb.nbatch) return fail(HPS_ERR_ARG, "reduction too large");
  const int64_t tiles = (n + 63) / 64;
  const int kc = (J + DW - 1) / DW;
  // workgroups: fewer partials to finish on vectors up to 2^24 entries (measured
  // on 0.46M and 6.5M entries: 512 / 256 beat 1024 / 512 by 3.1 % and 1.4 % per
  // solve, 256 / 128 lost 5-12 %); longer vectors keep 1024 / 512
  const bool mid = n < kMidVector;
  const int nblk = (int)std::min<int64_t>(tiles, kc <= 2 ? (mid ? 512 : 1024) : (mid ? 256 : 512));
  dim3 grid(nblk, 1, nbatch);
  const bool hw = w != nullptr;
#define HPS_DR(KC)                                                                            \
  do {                                                                                          \
    if (hw)                                                                                     \
      hipLaunchKernelGGL((k_dcgs_reduce<KC, true, VT>), grid, dim3(DT), 0, c->stream, V, ldv, vbs, J, u, \
                         ubs, w, wbs, n, rb.part);                                              \
    else                                                                                        \
      hipLaunchKernelGGL((k_dcgs_reduce<KC, false, VT>), grid, dim3(DT), 0, c->stream, V, ldv, vbs, J, u, \
                         ubs, w, wbs, n, rb.part);                                              \
  } while (0)
  // short bases on long vectors: tiles split over the wavefronts (measured:
  // the split over basis vectors reached about 2.5 TB/s for J <= 8 on 1e9-entry
  // vectors, where half the wavefronts idle and all re-read u and w)
  if (J <= kShortBasis && n >= kLongVector) {
    static_assert(kLongVector >= kNtVector, "the split reduction takes the non-temporal form");
    if (hw) launch_reduce_es<true, VT>(J, grid, c->stream, V, ldv, vbs, u, ubs, w, wbs, n, rb.part);
    else launch_reduce_es<false, VT>(J, grid, c->stream, V, ldv, vbs, u, ubs, w, wbs, n, rb.part);
  } else if (kc <= 2) HPS_DR(2); else if (kc <= 4) HPS_DR(4); else HPS_DR(8);
#undef HPS_DR
  int rc = check_hip(hipGetLastError(), "k_dcgs_reduce");
  if (rc) return rc;
  const int nslots = (hw ? 2 * J : J) + (hw ? 2 : 1);
  hipLaunchKernelGGL(k_dcgs_finish, dim3((nslots + 3) / 4, nbatch), dim3(256), 0, c->stream, rb.part, J,
                     hw ? 1 : 0, nblk, S);
  return check_hip(hipGetLastError(), "k_dcgs_finish");
}

}  // namespace

int launch_dcgs_reduce(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int J,
                       const double2* u, int64_t ubs, const double2* w, int64_t wbs, int64_t n,
                       DcgsState* S, int nbatch, const RedBuf& rb) {
  return dcgs_reduce(c, V, ldv, vbs, J, u, ubs, w, wbs, n, S, nbatch, rb);
}

int launch_dcgs_reduce(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int J,
                       const float2* u, int64_t ubs, const float2* w, int64_t wbs, int64_t n,
                       DcgsState* S, int nbatch, const RedBuf& rb) {
  return dcgs_reduce(c, V, ldv, vbs, J, u, ubs, w, wbs, n, S, nbatch, rb);
}

int launch_dcgs_small(hps_ctx* c, DcgsState* S, int nbatch, int j, int flexible, int final_only,
                      double* res_out, uint64_t tag) {
  if (j < 0 || j > kMaxDcgs) return fail(HPS_ERR_ARG, "small step beyond the restart limit");
  hipLaunchKernelGGL(k_dcgs_small, dim3(nbatch), dim3(UT), 0, c->stream, S, j, flexible, final_only,
                     res_out, (unsigned long long)tag, kBreakdownTol);
  return check_hip(hipGetLastError(), "k_dcgs_small");
}

namespace {

template <typename VT>
int dcgs_update(hps_ctx* c, VT* V, int64_t ldv, int64_t vbs, int J, VT* u, int64_t ubs, const VT* w,
                int64_t wbs, int64_t n, DcgsState* S, int nbatch, int flexible, double* res_out,
                uint64_t tag) {
  if (J < 0 || J >= kMaxDcgs) return fail(HPS_ERR_ARG, "update beyond the restart limit");
  // enough workgroups that a thread makes few passes (each pass waits for its
  // loads); every workgroup recomputes the step coefficients, a few KB from L2
  // (a cap of 32768 against 8192: 0.6 % faster per solve on 6.5M-entry vectors)
  const int64_t want = (n + UT - 1) / UT;
  const int nblk = (int)std::min<int64_t>(want, 32768);
  TimedPair tp;
  int rc = timing_pair(c, 4, &tp);
  if (rc) return rc;
  rc = check_hip(n >= kNtVector
                     ? launch_k(c, tp.start, tp.stop, k_dcgs_update<VT, true>, dim3(nblk, 1, nbatch),
                                dim3(UT), V, ldv, vbs, J, u, ubs, w, wbs, n, S, flexible, res_out,
                                (unsigned long long)tag, kBreakdownTol)
                     : launch_k(c, tp.start, tp.stop, k_dcgs_update<VT, false>, dim3(nblk, 1, nbatch),
                                dim3(UT), V, ldv, vbs, J, u, ubs, w, wbs, n, S, flexible, res_out,
                                (unsigned long long)tag, kBreakdownTol),
                 "k_dcgs_update");
  if (rc) {
    timing_drop(c, tp);
    return rc;
  }
  // algorithmic bytes: V_0..J-1, u and w read, V_J and u written
  return timing_commit(c, 4, tp, (double)sizeof(VT) * (J + 4) * (double)n * nbatch);
}

// the last update pass of a cycle with its closing reduction (long vectors)
template <typename VT, int JM = 0>
int dcgs_update_close_j(hps_ctx* c, dim3 grid, hipEvent_t e0, hipEvent_t e1, VT* V, int64_t ldv,
                        int64_t vbs, int J, VT* u, int64_t ubs, const VT* w, int64_t wbs, int64_t n,
                        DcgsState* S, int flexible, double* res_out, uint64_t tag, double2* part) {
  if constexpr (JM < kCloseMaxJ) {
    if (J > JM)
      return dcgs_update_close_j<VT, JM + 1>(c, grid, e0, e1, V, ldv, vbs, J, u, ubs, w, wbs, n, S,
                                             flexible, res_out, tag, part);
  }
  return check_hip(launch_k(c, e0, e1, k_dcgs_update_close<VT, true, JM>, grid, dim3(UT), V, ldv, vbs, J,
                            u, ubs, w, wbs, n, S, flexible, res_out, (unsigned long long)tag,
                            kBreakdownTol, part),
                   "k_dcgs_update_close");
}

template <typename VT>
int dcgs_update_close(hps_ctx* c, VT* V, int64_t ldv, int64_t vbs, int J, VT* u, int64_t ubs,
                      const VT* w, int64_t wbs, int64_t n, DcgsState* S, int nbatch, int flexible,
                      double* res_out, uint64_t tag, const RedBuf& rb) {
  if (J < 0 || J > kCloseMaxJ || n < kNtVector || nbatch > rb.nbatch)
    return fail(HPS_ERR_ARG, "closing update: basis too long or vector too short");
  const int64_t tiles = (n + UT - 1) / UT;
  const int nblk = (int)std::min<int64_t>(tiles, kRedBlocks);
  TimedPair tp;
  int rc = timing_pair(c, 4, &tp);
  if (rc) return rc;
  rc = dcgs_update_close_j<VT>(c, dim3(nblk, 1, nbatch), tp.start, tp.stop, V, ldv, vbs, J, u, ubs, w,
                               wbs, n, S, flexible, res_out, tag, rb.part);
  if (rc) {
    timing_drop(c, tp);
    return rc;
  }
  if ((rc = timing_commit(c, 4, tp, (double)sizeof(VT) * (J + 4) * (double)n * nbatch))) return rc;
  // finish a_0 .. a_J and c, as the reduction without w over J + 1 vectors does
  const int nslots = J + 2;
  hipLaunchKernelGGL(k_dcgs_finish, dim3((nslots + 3) / 4, nbatch), dim3(256), 0, c->stream, rb.part, J + 1,
                     0, nblk, S);
  return check_hip(hipGetLastError(), "k_dcgs_finish");
}

}  // namespace

bool dcgs_can_close(int J, int64_t n) { return J >= 0 && J <= kCloseMaxJ && n >= kNtVector; }

int launch_dcgs_update_close(hps_ctx* c, double2* V, int64_t ldv, int64_t vbs, int J, double2* u,
                             int64_t ubs, const double2* w, int64_t wbs, int64_t n, DcgsState* S,
                             int nbatch, int flexible, double* res_out, uint64_t tag, const RedBuf& rb) {
  return dcgs_update_close(c, V, ldv, vbs, J, u, ubs, w, wbs, n, S, nbatch, flexible, res_out, tag, rb);
}
int launch_dcgs_update_close(hps_ctx* c, float2* V, int64_t ldv, int64_t vbs, int J, float2* u,
                             int64_t ubs, const float2* w, int64_t wbs, int64_t n, DcgsState* S,
                             int nbatch, int flexible, double* res_out, uint64_t tag, const RedBuf& rb) {
  return dcgs_update_close(c, V, ldv, vbs, J, u, ubs, w, wbs, n, S, nbatch, flexible, res_out, tag, rb);
}

int launch_dcgs_update(hps_ctx* c, double2* V, int64_t ldv, int64_t vbs, int J, double2* u,
                       int64_t ubs, const double2* w, int64_t wbs, int64_t n, DcgsState* S,
                       int nbatch, int flexible, double* res_out, uint64_t tag) {
  return dcgs_update(c, V, ldv, vbs, J, u, ubs, w, wbs, n, S, nbatch, flexible, res_out, tag);
}

int launch_dcgs_update(hps_ctx* c, float2* V, int64_t ldv, int64_t vbs, int J, float2* u,
                       int64_t ubs, const float2* w, int64_t wbs, int64_t n, DcgsState* S,
                       int nbatch, int flexible, double* res_out, uint64_t tag) {
  return dcgs_update(c, V, ldv, vbs, J, u, ubs, w, wbs, n, S, nbatch, flexible, res_out, tag);
}

int launch_dcgs_start(hps_ctx* c, DcgsState* S, int nbatch) {
  hipLaunchKernelGGL(k_dcgs_start, dim3((nbatch + 63) / 64), dim3(64), 0, c->stream, S, nbatch);
  return check_hip(hipGetLastError(), "k_dcgs_start");
}

int launch_dcgs_trisolve(hps_ctx* c, DcgsState* S, int nbatch, int kmax, int flexible) {
  hipLaunchKernelGGL(k_dcgs_trisolve, dim3(nbatch), dim3(64), 0, c->stream, S, kmax, flexible);
  return check_hip(hipGetLastError(), "k_dcgs_trisolve");
}

int launch_dcgs_restart_coef(hps_ctx* c, DcgsState* S, int nbatch, int K) {
  if (K < 1 || K > kMaxDcgs) return fail(HPS_ERR_ARG, "restart after 1 .. 64 basis vectors");
  hipLaunchKernelGGL(k_dcgs_restart_coef, dim3(nbatch), dim3(64), 0, c->stream, S, K);
  return check_hip(hipGetLastError(), "k_dcgs_restart_coef");
}

namespace {

template <typename VT, typename XT>
int dcgs_restart(hps_ctx* c, const VT* V, int64_t ldv, int64_t vbs, int K, VT* u, int64_t ubs, XT* x,
                 int64_t xbs, int64_t n, DcgsState* S, int nbatch) {
  if (K < 1 || K > kMaxDcgs) return fail(HPS_ERR_ARG, "restart after 1 .. 64 basis vectors");
  const int nblk = (int)std::min<int64_t>((n + UT - 1) / UT, 32768);
  const dim3 grid(nblk, 1, nbatch);
  if (n >= kNtVector)
    hipLaunchKernelGGL((k_dcgs_restart<VT, XT, true>), grid, dim3(UT), 0, c->stream, V, ldv, vbs, K, u,
                       ubs, x, xbs, n, S);
  else
    hipLaunchKernelGGL((k_dcgs_restart<VT, XT, false>), grid, dim3(UT), 0, c->stream, V, ldv, vbs, K, u,
                       ubs, x, xbs, n, S);
  return check_hip(hipGetLastError(), "k_dcgs_restart");
}

}  // namespace

int launch_dcgs_restart(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K, double2* u,
                        int64_t ubs, double2* x, int64_t xbs, int64_t n, DcgsState* S, int nbatch) {
  return dcgs_restart(c, V, ldv, vbs, K, u, ubs, x, xbs, n, S, nbatch);
}

int launch_dcgs_restart(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int K, float2* u,
                        int64_t ubs, float2* x, int64_t xbs, int64_t n, DcgsState* S, int nbatch) {
  return dcgs_restart(c, V, ldv, vbs, K, u, ubs, x, xbs, n, S, nbatch);
}

int launch_dcgs_restart(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int K, float2* u,
                        int64_t ubs, double2* x, int64_t xbs, int64_t n, DcgsState* S, int nbatch) {
  return dcgs_restart(c, V, ldv, vbs, K, u, ubs, x, xbs, n, S, nbatch);
}

}  // namespace hps
