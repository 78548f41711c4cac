// Kernels of the Arnoldi process with delayed reorthogonalization (see
// hps_krylov.h): per step one reduction pass and one update pass over the
// basis, plus a one-wavefront kernel for the small Hessenberg / Givens work.
// Reductions are deterministic (fixed order), as in k_krylov.hip.
#include "hps_internal.h"
#include "hps_krylov.h"
#include "k_common.h"

namespace hps {
namespace {

constexpr int DW = 8;          // wavefronts of the reduction workgroup (split over k)
constexpr int DT = 64 * DW;    // its threads; one tile = 64 vector entries
constexpr int UT = 256;        // update-pass workgroup

// Partials of a_k = sum conj(V_k) u, b_k = sum conj(V_k) w (k < J), c = sum |u|^2,
// d = sum conj(u) w.  Wavefront ky owns basis vectors ky*kc .. ky*kc+kc-1 of the
// tile; wavefront 0 also accumulates c and d.
template <int KC, bool HASW>
__global__ __launch_bounds__(DT) void k_dcgs_reduce(const double2* __restrict__ V, int64_t ldv,
                                                    int64_t vbs, int J, const double2* __restrict__ u,
                                                    int64_t ubs, const double2* __restrict__ w,
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
  for (int64_t t0 = (int64_t)blockIdx.x * 64; t0 < n; t0 += (int64_t)nblk * 64) {
    const int64_t i = t0 + lane;
    const bool ok = i < n;
    const double2 uv = ok ? u[i] : make_double2(0.0, 0.0);
    const double2 wv = (HASW && ok) ? w[i] : make_double2(0.0, 0.0);
    double2 vr[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      vr[kk] = (kk < kn && ok) ? V[(int64_t)(k0 + kk) * ldv + i] : make_double2(0.0, 0.0);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      aa[kk].x = fma(vr[kk].x, uv.x, fma(vr[kk].y, uv.y, aa[kk].x));
      aa[kk].y = fma(vr[kk].x, uv.y, fma(-vr[kk].y, uv.x, aa[kk].y));
      if (HASW) {
        ab[kk].x = fma(vr[kk].x, wv.x, fma(vr[kk].y, wv.y, ab[kk].x));
        ab[kk].y = fma(vr[kk].x, wv.y, fma(-vr[kk].y, wv.x, ab[kk].y));
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
  for (int i = 0; i < kDcgsLd; ++i) s.gls[i] = make_double2(0.0, 0.0);
}

// One step's small work for right-hand side blockIdx.x (see hps_krylov.h).
__global__ __launch_bounds__(64) void k_dcgs_small(DcgsState* __restrict__ S, int j, int flexible,
                                                   int final_only, double* __restrict__ res_out,
                                                   double tiny) {
  DcgsState& s = S[blockIdx.x];
  const int lane = threadIdx.x;
  double* ro = res_out + 2 * blockIdx.x;
  __shared__ double2 a[kMaxDcgs], b[kMaxDcgs];
  __shared__ double2 col[kDcgsLd + 1];
  __shared__ double2 Hs[kDcgsLd * (kMaxDcgs - 1)];   // columns 0 .. j-1 <= 62 of H
  __shared__ double csl[kMaxDcgs];
  __shared__ double2 snl[kMaxDcgs];
  __shared__ double2 Ts[kMaxDcgs * (kMaxDcgs - 1)];  // columns 0 .. j-1 of T
  if (s.flag) {  // an earlier step stopped this cycle: keep the state as it is
    if (lane == 0) { ro[0] = s.res; ro[1] = 1.0; }
    return;
  }
  const double2 z2 = make_double2(0.0, 0.0);
  const double2 al = (lane < j) ? s.red[lane] : z2;
  const double2 bl = (lane < j && !final_only) ? s.red[kSlotB + lane] : z2;
  a[lane] = al;
  b[lane] = bl;
  const double c = s.red[kSlotC].x;
  const double2 d = final_only ? z2 : s.red[kSlotD];
  const double na2 = wave_sum(al.x * al.x + al.y * al.y);
  const double abr = wave_sum(al.x * bl.x + al.y * bl.y);   // conj(a) b
  const double abi = wave_sum(al.x * bl.y - al.y * bl.x);
  const double beta2 = c - na2;
  if (!(beta2 > tiny * c) || !isfinite(beta2)) {
    // the candidate lies in the span of the basis: happy breakdown or lost
    // orthogonality; the cycle ends with the columns finished so far
    if (lane == 0) { s.flag = 1; ro[0] = s.res; ro[1] = 1.0; }
    return;
  }
  const double beta = sqrt(beta2), inv = 1.0 / beta;
  const int ld = kDcgsLd;
  if (j == 0) {
    if (lane == 0) {
      s.beta0 = beta;
      s.gls[0] = make_double2(beta, 0.0);
      s.res = beta;
      s.ncols = 0;
    }
  } else {
    // finish column j-1: H[0:j, j-1] = gprev + a, H[j, j-1] = beta
    for (int i = lane; i < j; i += 64) {
      const double2 h = cadd(s.gprev[i], a[i]);
      s.H[i + ld * (j - 1)] = h;
      col[i] = h;
    }
    if (lane == 0) {
      s.H[j + ld * (j - 1)] = make_double2(beta, 0.0);
      col[j] = make_double2(beta, 0.0);
    }
    for (int i = lane; i < j - 1; i += 64) {
      csl[i] = s.cs[i];
      snl[i] = s.sn[i];
    }
    __syncthreads();
    if (lane == 0) {
      for (int i = 0; i < j - 1; ++i) {
        const double cr = csl[i];
        const double2 sn = snl[i];
        const double2 x0 = col[i], x1 = col[i + 1];
        col[i] = cadd(cscale(x0, cr), cmul(sn, x1));
        col[i + 1] = csub(cscale(x1, cr), cmulc(sn, x0));
      }
      const double2 x0 = col[j - 1];
      const double am = sqrt(x0.x * x0.x + x0.y * x0.y);
      const double r = sqrt(am * am + beta2);
      double cr;
      double2 sn;
      if (am == 0.0) {
        cr = 0.0;
        sn = make_double2(1.0, 0.0);
        col[j - 1] = make_double2(beta, 0.0);
      } else {
        cr = am / r;
        const double2 ph = make_double2(x0.x / am, x0.y / am);
        sn = make_double2(ph.x * beta / r, ph.y * beta / r);
        col[j - 1] = make_double2(ph.x * r, ph.y * r);
      }
      col[j] = make_double2(0.0, 0.0);
      s.cs[j - 1] = cr;
      s.sn[j - 1] = sn;
      const double2 g0 = s.gls[j - 1];
      const double2 g1 = make_double2(-(sn.x * g0.x + sn.y * g0.y), -(sn.x * g0.y - sn.y * g0.x));
      s.gls[j] = g1;
      s.gls[j - 1] = cscale(g0, cr);
      s.res = sqrt(g1.x * g1.x + g1.y * g1.y);
      s.ncols = j;
    }
    __syncthreads();
    for (int i = lane; i <= j; i += 64) s.R[i + ld * (j - 1)] = col[i];
  }
  if (final_only) {
    if (lane == 0) { ro[0] = s.res; ro[1] = 0.0; }
    return;
  }
  // Stage the j finished Hessenberg columns (and T for the flexible variant) in
  // LDS with every load issued up front: the products below then run at LDS
  // latency instead of one dependent global load per term.
  __syncthreads();
  for (int q = lane; q < (j + 1) * j; q += 64) {
    const int l = q / (j + 1), i = q - l * (j + 1);
    Hs[i + ld * l] = s.H[i + ld * l];
  }
  if (flexible)
    for (int q = lane; q < j * j; q += 64) {
      const int l = q / j, i = q - l * j;
      Ts[i + kMaxDcgs * l] = s.T[i + kMaxDcgs * l];
    }
  __syncthreads();
  // flexible: z_j = (z'_j - Z_{j-1} a) / beta, i.e. T[:, j] = (e_j - T[:, 0:j] a) / beta
  if (flexible) {
    for (int i = lane; i < j; i += 64) {
      double2 acc = z2;
      for (int l = i; l < j; ++l) acc = cadd(acc, cmul(Ts[i + kMaxDcgs * l], a[l]));
      s.T[i + kMaxDcgs * j] = cscale(acc, -inv);
    }
    if (lane == 0) s.T[j + kMaxDcgs * j] = make_double2(inv, 0.0);
  }
  // projection of Op v_j on V_j: g_j = ([b; vjw] - Hbar_{j-1} a) / beta
  const double2 vjw = cscale(make_double2(d.x - abr, d.y - abi), inv);
  for (int i = lane; i <= j; i += 64) {
    double2 ha = z2;
    for (int l = (i > 0 ? i - 1 : 0); l < j; ++l) ha = cadd(ha, cmul(Hs[i + ld * l], a[l]));
    const double2 vw = (i < j) ? b[i] : vjw;
    s.gprev[i] = cscale(csub(vw, ha), inv);
  }
  for (int l = lane; l < j; l += 64) {
    s.ca[l] = a[l];
    s.cb[l] = b[l];
  }
  if (lane == 0) {
    s.cb[j] = vjw;
    s.inv_beta = inv;
    ro[0] = s.res;
    ro[1] = 0.0;
  }
}

// V[J] = (u - V_{0..J-1} ca) * inv;  u <- (w - V_{0..J-1} cb - V[J] cb[J]) * inv
__global__ __launch_bounds__(UT) void k_dcgs_update(double2* __restrict__ V, int64_t ldv, int64_t vbs,
                                                    int J, double2* __restrict__ u, int64_t ubs,
                                                    const double2* __restrict__ w, int64_t wbs,
                                                    int64_t n, const DcgsState* __restrict__ S) {
  const int bz = blockIdx.z;
  const DcgsState& s = S[bz];
  if (s.flag) return;
  V += bz * vbs;
  u += bz * ubs;
  w += bz * wbs;
  __shared__ double2 ca[kMaxDcgs], cb[kDcgsLd];
  for (int l = threadIdx.x; l < J; l += UT) ca[l] = s.ca[l];
  for (int l = threadIdx.x; l <= J; l += UT) cb[l] = s.cb[l];
  const double inv = s.inv_beta;
  __syncthreads();
  const double2 cj = cb[J];
  for (int64_t i = (int64_t)blockIdx.x * UT + threadIdx.x; i < n; i += (int64_t)gridDim.x * UT) {
    double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
    int l = 0;
    for (; l + 8 <= J; l += 8) {
      double2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = V[(int64_t)(l + q) * ldv + i];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double2 x = ca[l + q], y = cb[l + q];
        sa.x = fma(v[q].x, x.x, fma(-v[q].y, x.y, sa.x));
        sa.y = fma(v[q].x, x.y, fma(v[q].y, x.x, sa.y));
        sb.x = fma(v[q].x, y.x, fma(-v[q].y, y.y, sb.x));
        sb.y = fma(v[q].x, y.y, fma(v[q].y, y.x, sb.y));
      }
    }
    for (; l < J; ++l) {
      const double2 v = V[(int64_t)l * ldv + i];
      const double2 x = ca[l], y = cb[l];
      sa.x = fma(v.x, x.x, fma(-v.y, x.y, sa.x));
      sa.y = fma(v.x, x.y, fma(v.y, x.x, sa.y));
      sb.x = fma(v.x, y.x, fma(-v.y, y.y, sb.x));
      sb.y = fma(v.x, y.y, fma(v.y, y.x, sb.y));
    }
    const double2 uv = u[i], wv = w[i];
    const double2 vj = make_double2((uv.x - sa.x) * inv, (uv.y - sa.y) * inv);
    const double2 t = cmul(vj, cj);
    V[(int64_t)J * ldv + i] = vj;
    u[i] = make_double2((wv.x - sb.x - t.x) * inv, (wv.y - sb.y - t.y) * inv);
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

}  // namespace

int launch_dcgs_reduce(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int J,
                       const double2* u, int64_t ubs, const double2* w, int64_t wbs, int64_t n,
                       DcgsState* S, int nbatch, const RedBuf& rb) {
  if (J > kMaxDcgs || nbatch > rb.nbatch) return fail(HPS_ERR_ARG, "reduction too large");
  const int64_t tiles = (n + 63) / 64;
  const int kc = (J + DW - 1) / DW;
  const int nblk = (int)std::min<int64_t>(tiles, kc <= 2 ? 1024 : 512);
  dim3 grid(nblk, 1, nbatch);
  const bool hw = w != nullptr;
#define HPS_DR(KC)                                                                              \
  do {                                                                                          \
    if (hw)                                                                                     \
      hipLaunchKernelGGL((k_dcgs_reduce<KC, true>), grid, dim3(DT), 0, c->stream, V, ldv, vbs, J, u, \
                         ubs, w, wbs, n, rb.part);                                              \
    else                                                                                        \
      hipLaunchKernelGGL((k_dcgs_reduce<KC, false>), grid, dim3(DT), 0, c->stream, V, ldv, vbs, J, \
                         u, ubs, w, wbs, n, rb.part);                                           \
  } while (0)
  if (kc <= 2) HPS_DR(2); else if (kc <= 4) HPS_DR(4); else HPS_DR(8);
#undef HPS_DR
  int rc = check_hip(hipGetLastError(), "k_dcgs_reduce");
  if (rc) return rc;
  const int nslots = (hw ? 2 * J : J) + (hw ? 2 : 1);
  hipLaunchKernelGGL(k_dcgs_finish, dim3((nslots + 3) / 4, nbatch), dim3(256), 0, c->stream, rb.part, J,
                     hw ? 1 : 0, nblk, S);
  return check_hip(hipGetLastError(), "k_dcgs_finish");
}

int launch_dcgs_small(hps_ctx* c, DcgsState* S, int nbatch, int j, int flexible, int final_only,
                      double* res_out) {
  hipLaunchKernelGGL(k_dcgs_small, dim3(nbatch), dim3(64), 0, c->stream, S, j, flexible, final_only,
                     res_out, 1e-14);
  return check_hip(hipGetLastError(), "k_dcgs_small");
}

int launch_dcgs_update(hps_ctx* c, double2* V, int64_t ldv, int64_t vbs, int J, double2* u,
                       int64_t ubs, const double2* w, int64_t wbs, int64_t n, const DcgsState* S,
                       int nbatch) {
  const int64_t want = (n + UT - 1) / UT;
  const int nblk = (int)std::min<int64_t>(want, 2048);
  hipLaunchKernelGGL(k_dcgs_update, dim3(nblk, 1, nbatch), dim3(UT), 0, c->stream, V, ldv, vbs, J, u,
                     ubs, w, wbs, n, S);
  return check_hip(hipGetLastError(), "k_dcgs_update");
}

int launch_dcgs_start(hps_ctx* c, DcgsState* S, int nbatch) {
  hipLaunchKernelGGL(k_dcgs_start, dim3((nbatch + 63) / 64), dim3(64), 0, c->stream, S, nbatch);
  return check_hip(hipGetLastError(), "k_dcgs_start");
}

int launch_dcgs_trisolve(hps_ctx* c, DcgsState* S, int nbatch, int kmax, int flexible) {
  hipLaunchKernelGGL(k_dcgs_trisolve, dim3(nbatch), dim3(64), 0, c->stream, S, kmax, flexible);
  return check_hip(hipGetLastError(), "k_dcgs_trisolve");
}

}  // namespace hps
