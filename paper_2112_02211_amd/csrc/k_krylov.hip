// Krylov primitives for the GMRES drivers: multi-dot products (the Arnoldi
// inner products of classical Gram-Schmidt), multi-axpy updates, norms and
// the small Hessenberg / Givens state, all in FP64 on the device.
//
// Reductions are two-level and deterministic: every workgroup reduces its
// slice with wavefront shuffles and LDS and writes one partial per output, and
// a small second kernel sums the partials in a fixed order.  (A last-workgroup
// finish inside the first kernel would need an agent-scope release/acquire in
// every workgroup, i.e. write-back and invalidation of the XCD-local L2
// caches, which costs more than the extra launch.)
#include "hps_internal.h"
#include "hps_krylov.h"
#include "k_common.h"
#include "k_vec.h"

#include <algorithm>

namespace hps {
namespace {

constexpr int RT = 256;         // threads per reduction workgroup
constexpr int RW = RT / 64;     // wavefronts per workgroup
constexpr int KB = 16;          // outputs per workgroup in the multi-dot


// out[k] = sum_n conj(V[k ldv + n]) w[n]; batch b (blockIdx.z) offsets every
// pointer by its batch stride.
__global__ __launch_bounds__(RT) void k_mdot(const double2* __restrict__ V, int64_t ldv,
                                             int64_t vbs, int K, const double2* __restrict__ w,
                                             int64_t wbs, int64_t n, double2* __restrict__ part) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  w += bz * wbs;
  const unsigned nblk = gridDim.x;
  const int k0 = blockIdx.y * KB;
  double2* pz = part + (int64_t)bz * kPartSlots * nblk;
  double2 acc[KB];
#pragma unroll
  for (int kk = 0; kk < KB; ++kk) acc[kk] = make_double2(0.0, 0.0);
  const int kn = min(KB, K - k0);
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)nblk * RT) {
    const double2 wv = w[i];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk)
      if (kk < kn) {
        const double2 v = V[(int64_t)(k0 + kk) * ldv + i];
        acc[kk].x = fma(v.x, wv.x, fma(v.y, wv.y, acc[kk].x));
        acc[kk].y = fma(v.x, wv.y, fma(-v.y, wv.x, acc[kk].y));
      }
  }
  __shared__ double2 red[RW][KB];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int kk = 0; kk < KB; ++kk) {
    if (kk < kn) {
      const double re = wave_sum(acc[kk].x), im = wave_sum(acc[kk].y);
      if (lane == 0) red[wid][kk] = make_double2(re, im);
    }
  }
  __syncthreads();
  if (threadIdx.x < kn) {
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < RW; ++q) s = cadd(s, red[q][threadIdx.x]);
    pz[(int64_t)(blockIdx.y * KB + threadIdx.x) * nblk + blockIdx.x] = s;
  }
}

// w[i] += sign * sum_k V[k ldv + i] coef[k]; optionally nrm2 = ||w||^2 after the update.
// VT: the storage of V and w (complex FP64 or FP32); the sums are FP64.
template <typename VT>
__global__ __launch_bounds__(RT) void k_mupdate(const VT* __restrict__ V, int64_t ldv,
                                                int64_t vbs, int K, const double2* __restrict__ coef,
                                                int64_t cbs, double sign, VT* __restrict__ w,
                                                int64_t wbs, int64_t n, int want_norm,
                                                double2* __restrict__ part) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  w += bz * wbs;
  coef += bz * cbs;
  // coefficients zero-padded to a multiple of 8 (the last round is predicated)
  __shared__ double2 cs[(kMaxRestart + 1 + 7) / 8 * 8];
  const int K8 = (K + 7) / 8 * 8;
  for (int k = threadIdx.x; k < K8; k += RT) {
    const double2 c = k < K ? coef[k] : make_double2(0.0, 0.0);
    cs[k] = make_double2(sign * c.x, sign * c.y);
  }
  __syncthreads();
  const unsigned nblk = gridDim.x;
  double sq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)nblk * RT) {
    double2 a = ld2(w, i);
    for (int k = 0; k < K; k += 8) {
      VT r[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        r[u] = ld_tile(V, (int64_t)(k + u) * ldv + i, (int64_t)k * ldv + i, k + u < K);
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = widen(r[u], k + u < K);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 c = cs[k + u];
        a.x = fma(v[u].x, c.x, fma(-v[u].y, c.y, a.x));
        a.y = fma(v[u].x, c.y, fma(v[u].y, c.x, a.y));
      }
    }
    if (K > 0) st2(w, i, a);
    sq = fma(a.x, a.x, fma(a.y, a.y, sq));
  }
  if (!want_norm) return;
  __shared__ double red[RW];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  sq = wave_sum(sq);
  if (lane == 0) red[wid] = sq;
  __syncthreads();
  double* pz = reinterpret_cast<double*>(part) + (int64_t)bz * nblk;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < RW; ++q) s += red[q];
    pz[blockIdx.x] = s;
  }
}

// y = x * s with s = 1/sqrt(src[b]) (inv_sqrt) or s = src[b]; a zero norm gives 0.
__global__ void k_scale_by(const double2* __restrict__ x, int64_t xbs, double2* __restrict__ y,
                           int64_t ybs, int64_t n, const double* __restrict__ src, int64_t sstride,
                           int inv_sqrt) {
  const int bz = blockIdx.y;
  const double v = src[bz * sstride];
  const double s = inv_sqrt ? (v > 0.0 ? 1.0 / sqrt(v) : 0.0) : v;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 a = x[bz * xbs + i];
  y[bz * ybs + i] = make_double2(a.x * s, a.y * s);
}

__global__ void k_demote_scaled(const double2* __restrict__ x, double s, float2* __restrict__ y,
                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 a = x[i];
  y[i] = make_float2((float)(a.x * s), (float)(a.y * s));
}

template <typename XT>
__global__ void k_axpy_promote(double s, const XT* __restrict__ x, double2* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const XT a = x[i];
  const double2 b = y[i];
  y[i] = make_double2(fma(s, (double)a.x, b.x), fma(s, (double)a.y, b.y));
}

template <typename VT>
__global__ void k_sub_from(const VT* __restrict__ a, VT* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 u = ld2(a, i), v = ld2(y, i);
  st2(y, i, make_double2(u.x - v.x, u.y - v.y));
}


// ------------------------------------------------------------------ CGS2 passes
// Classical Gram-Schmidt passes for up to 64 basis vectors, laid out so that a
// workgroup covers a tile of 128 vector entries with 8 wavefronts: wavefront
// (ky, nx) handles basis vectors k0(ky) .. k0(ky)+kc-1 for the 64 entries of
// sub-tile nx, one entry per lane, and keeps those basis values in registers.
//  * DOT:      out[k] = sum_i conj(V[k][i]) w[i]
//  * UPD_DOT:  w[i] -= sum_k V[k][i] coef[k], then out[k] = sum_i conj(V[k][i]) w_new[i]
//    in the same pass: the per-entry update needs every k, so the wavefronts of
//    a sub-tile combine their partial sums through LDS (double buffered, one
//    barrier per tile) and reuse their register copies of V for the dot.
// Partials per workgroup, finished by the last workgroup as in k_mdot.
constexpr int GK = 4;             // k chunks (wavefront rows)
constexpr int GN = 2;             // entry sub-tiles (wavefront columns)
constexpr int GT = 64 * GK * GN;  // 512 threads

// GKC: largest k chunk per wavefront (K <= 4 GKC); smaller chunks keep fewer
// basis values in registers and so allow more resident wavefronts.
template <bool UPD, int GKC>
__global__ __launch_bounds__(GT) void k_cgs64(const double2* __restrict__ V, int64_t ldv,
                                              int64_t vbs, int K, const double2* __restrict__ coef,
                                              int64_t cbs, double2* __restrict__ w, int64_t wbs,
                                              int64_t n, double2* __restrict__ part) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  w += bz * wbs;
  if (UPD) coef += bz * cbs;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ky = wv % GK, nx = wv / GK;
  const int kc = (K + GK - 1) / GK;
  const int k0 = ky * kc;
  const int kn = max(0, min(kc, K - k0));
  __shared__ double2 sp[2][GK][GN * 64];
  __shared__ double2 red[GN][GK][GKC];
  double2 c[GKC];
#pragma unroll
  for (int kk = 0; kk < GKC; ++kk)
    c[kk] = (UPD && kk < kn) ? coef[k0 + kk] : make_double2(0.0, 0.0);
  double2 acc[GKC];
#pragma unroll
  for (int kk = 0; kk < GKC; ++kk) acc[kk] = make_double2(0.0, 0.0);
  const unsigned nblk = gridDim.x;
  int buf = 0;
  for (int64_t t0 = (int64_t)blockIdx.x * (GN * 64); t0 < n; t0 += (int64_t)nblk * (GN * 64)) {
    const int64_t i = t0 + nx * 64 + lane;
    const bool ok = i < n;
    double2 vr[GKC];
#pragma unroll
    for (int kk = 0; kk < GKC; ++kk)
      vr[kk] = (kk < kn && ok) ? V[(int64_t)(k0 + kk) * ldv + i] : make_double2(0.0, 0.0);
    double2 x = ok ? w[i] : make_double2(0.0, 0.0);
    if (UPD) {
      double2 pacc = make_double2(0.0, 0.0);
#pragma unroll
      for (int kk = 0; kk < GKC; ++kk) {
        pacc.x = fma(vr[kk].x, c[kk].x, fma(-vr[kk].y, c[kk].y, pacc.x));
        pacc.y = fma(vr[kk].x, c[kk].y, fma(vr[kk].y, c[kk].x, pacc.y));
      }
      sp[buf][ky][nx * 64 + lane] = pacc;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < GK; ++q) x = csub(x, sp[buf][q][nx * 64 + lane]);
      if (ky == 0 && ok) w[i] = x;
      buf ^= 1;
    }
#pragma unroll
    for (int kk = 0; kk < GKC; ++kk) {
      acc[kk].x = fma(vr[kk].x, x.x, fma(vr[kk].y, x.y, acc[kk].x));
      acc[kk].y = fma(vr[kk].x, x.y, fma(-vr[kk].y, x.x, acc[kk].y));
    }
  }
#pragma unroll
  for (int kk = 0; kk < GKC; ++kk) {
    if (kk < kn) {
      const double re = wave_sum(acc[kk].x), im = wave_sum(acc[kk].y);
      if (lane == 0) red[nx][ky][kk] = make_double2(re, im);
    }
  }
  __syncthreads();
  double2* pz = part + (int64_t)bz * kPartSlots * nblk;
  if ((int)threadIdx.x < K) {
    const int k = threadIdx.x, qy = k / kc, kk = k - qy * kc;
    double2 sacc = make_double2(0.0, 0.0);
    for (int q = 0; q < GN; ++q) sacc = cadd(sacc, red[q][qy][kk]);
    pz[(int64_t)k * nblk + blockIdx.x] = sacc;
  }
}

// out[b * obs + k] = sum over workgroups of the complex partials of output k;
// one wavefront per output (grid.x covers the outputs four at a time).
__global__ __launch_bounds__(256) void k_finish_c(const double2* __restrict__ part, int K, int nblk,
                                                  double2* __restrict__ out, int64_t obs) {
  const int bz = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double2* pz = part + (int64_t)bz * kPartSlots * nblk;
  const int k = blockIdx.x * 4 + wv;
  if (k < K) {
    double re = 0.0, im = 0.0;
    const double2* pp = pz + (int64_t)k * nblk;
    for (int b = lane; b < nblk; b += 64) {
      const double2 v = pp[b];
      re += v.x;
      im += v.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) out[bz * obs + k] = make_double2(re, im);
  }
}

// out[b * ostride] = sum over workgroups of the real partials
__global__ __launch_bounds__(256) void k_finish_r(const double2* __restrict__ part, int nblk,
                                                  double* __restrict__ out, int64_t ostride) {
  const int bz = blockIdx.x;
  const double* pz = reinterpret_cast<const double*>(part) + (int64_t)bz * nblk;
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += pz[b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[bz * ostride] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ----------------------------------------------------------- Hessenberg state
// Start a cycle: g = (beta, 0, ...), beta = sqrt(nrm2).
__global__ void k_gm_start(GmresState* __restrict__ S, int nb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  GmresState& s = S[b];
  const double beta = sqrt(s.nrm2);
  s.beta = beta;
  for (int i = 0; i <= kMaxRestart; ++i) s.g[i] = make_double2(0.0, 0.0);
  s.g[0] = make_double2(beta, 0.0);
  s.res = beta;
}

// Column j of the Hessenberg matrix from the two Gram-Schmidt passes, the
// previous rotations applied, a new complex Givens rotation zeroing the
// subdiagonal, and the updated residual estimate |g_{j+1}|.  One wavefront per
// right-hand side: the column is staged in LDS in parallel, the (inherently
// sequential) rotations run on LDS values, and the column is written back in
// parallel.
__global__ __launch_bounds__(64) void k_gm_givens(GmresState* __restrict__ S, int j, double tiny) {
  GmresState& s = S[blockIdx.x];
  __shared__ double2 h[kMaxRestart + 2];
  __shared__ double csl[kMaxRestart];
  __shared__ double2 snl[kMaxRestart];
  const int lane = threadIdx.x;
  for (int i = lane; i <= j; i += 64) h[i] = cadd(s.h1[i], s.h2[i]);
  for (int i = lane; i < j; i += 64) { csl[i] = s.cs[i]; snl[i] = s.sn[i]; }
  const double hn = sqrt(s.nrm2);
  __syncthreads();
  if (lane == 0) {
    h[j + 1] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
      const double c = csl[i];
      const double2 sn = snl[i];
      const double2 a = h[i], bb = h[i + 1];
      // [c, sn; -conj(sn), c] [a; b]
      h[i] = cadd(cscale(a, c), cmul(sn, bb));
      h[i + 1] = csub(cscale(bb, c), cmulc(sn, a));
    }
    const double2 a = h[j];
    const double bm = hn;
    const double am = sqrt(a.x * a.x + a.y * a.y);
    const double r = sqrt(am * am + bm * bm);
    double c;
    double2 sn;
    if (r == 0.0) {
      c = 1.0;
      sn = make_double2(0.0, 0.0);
    } else if (am == 0.0) {
      c = 0.0;
      sn = make_double2(1.0, 0.0);
      h[j] = make_double2(bm, 0.0);
    } else {
      c = am / r;
      const double2 ph = make_double2(a.x / am, a.y / am);
      sn = make_double2(ph.x * bm / r, ph.y * bm / r);  // phase(a) conj(b) / r with b real
      h[j] = make_double2(ph.x * r, ph.y * r);
    }
    h[j + 1] = make_double2(0.0, 0.0);
    s.cs[j] = c;
    s.sn[j] = sn;
    const double2 gj = s.g[j];
    const double2 g1 = make_double2(-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x));
    s.g[j + 1] = g1;  // -conj(sn) g_j
    s.g[j] = cscale(gj, c);
    s.res = sqrt(g1.x * g1.x + g1.y * g1.y);
    s.breakdown = (hn <= tiny * (r > 0 ? r : 1.0)) ? 1 : 0;
  }
  __syncthreads();
  double2* col = &s.H[(int64_t)j * (kMaxRestart + 1)];
  for (int i = lane; i <= j + 1; i += 64) col[i] = h[i];
}

// out[2 b] = residual estimate, out[2 b + 1] = breakdown flag of right-hand side b
__global__ void k_gm_collect(const GmresState* __restrict__ S, int nb, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  out[2 * b] = S[b].res;
  out[2 * b + 1] = (double)S[b].breakdown;
}

// y = R^{-1} g for the leading k x k triangle of the rotated Hessenberg matrix
// (column-oriented back substitution: after y_i is known every row above it
// is updated in parallel).  R is staged in LDS when it fits.
constexpr int TRI_LDS = 56;
__global__ __launch_bounds__(256) void k_gm_trisolve(GmresState* __restrict__ S, int k) {
  GmresState& s = S[blockIdx.x];
  __shared__ double2 R[TRI_LDS * TRI_LDS];
  __shared__ double2 g[kMaxRestart + 1];
  __shared__ double2 yi;
  const int ld = kMaxRestart + 1;
  const bool lds = k <= TRI_LDS;
  for (int i = threadIdx.x; i < k; i += blockDim.x) g[i] = s.g[i];
  if (lds)
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
      const int col = t / k, row = t - col * k;
      R[col * TRI_LDS + row] = s.H[(int64_t)col * ld + row];
    }
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    if (threadIdx.x == 0) {
      const double2 d = lds ? R[i * TRI_LDS + i] : s.H[(int64_t)i * ld + i];
      const double dd = d.x * d.x + d.y * d.y;
      const double2 a = g[i];
      const double2 v = dd > 0.0 ? make_double2((a.x * d.x + a.y * d.y) / dd, (a.y * d.x - a.x * d.y) / dd)
                                 : make_double2(0.0, 0.0);
      yi = v;
      s.y[i] = v;
    }
    __syncthreads();
    const double2 v = yi;
    for (int l = threadIdx.x; l < i; l += blockDim.x) {
      const double2 rl = lds ? R[i * TRI_LDS + l] : s.H[(int64_t)i * ld + l];
      g[l] = csub(g[l], cmul(rl, v));
    }
    __syncthreads();
  }
}

}  // namespace

int red_buf(hps_ctx* c, int kmax, int nbatch, RedBuf* rb) {
  (void)kmax;
  const int nblk = kRedBlocks;
  const size_t need = (size_t)kPartSlots * nblk * sizeof(double2) * nbatch;
  int rc = ws_reserve(c, &c->w_red, need);
  if (rc) return rc;
  rb->part = static_cast<double2*>(c->w_red.ptr);
  rb->counter = nullptr;
  rb->nblk = nblk;
  rb->nbatch = nbatch;
  return HPS_OK;
}

static int nblocks_for(int64_t n, int nblk) {
  const int64_t want = (n + RT - 1) / RT;
  return (int)(want < nblk ? (want > 0 ? want : 1) : nblk);
}

static int finish_c(hps_ctx* c, const RedBuf& rb, int K, int nblk, double2* out, int64_t obs,
                    int nbatch) {
  hipLaunchKernelGGL(k_finish_c, dim3((K + 3) / 4, nbatch), dim3(256), 0, c->stream, rb.part, K, nblk,
                     out, obs);
  return check_hip(hipGetLastError(), "k_finish_c");
}

int launch_mdot_b(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K, const double2* w,
                  int64_t wbs, int64_t n, double2* out, int64_t obs, int nbatch, const RedBuf& rb) {
  if (K <= 0) return HPS_OK;
  const int gy = (K + KB - 1) / KB;
  if (gy * KB > kPartSlots || nbatch > rb.nbatch) return fail(HPS_ERR_ARG, "multi-dot too large");
  const int nblk = nblocks_for(n, rb.nblk);
  dim3 grid(nblk, gy, nbatch);
  hipLaunchKernelGGL(k_mdot, grid, dim3(RT), 0, c->stream, V, ldv, vbs, K, w, wbs, n, rb.part);
  int rc = check_hip(hipGetLastError(), "k_mdot");
  if (rc) return rc;
  return finish_c(c, rb, K, nblk, out, obs, nbatch);
}

template <typename VT>
static int mupdate_b(hps_ctx* c, const VT* V, int64_t ldv, int64_t vbs, int K, const double2* coef,
                     int64_t cbs, double sign, VT* w, int64_t wbs, int64_t n, double* nrm2,
                     int64_t nstride, int nbatch, const RedBuf& rb) {
  if (K > kMaxRestart + 1 || nbatch > rb.nbatch) return fail(HPS_ERR_ARG, "update too large");
  const int nblk = nblocks_for(n, rb.nblk);
  dim3 grid(nblk, 1, nbatch);
  hipLaunchKernelGGL(k_mupdate<VT>, grid, dim3(RT), 0, c->stream, V, ldv, vbs, K, coef, cbs, sign, w,
                     wbs, n, nrm2 ? 1 : 0, rb.part);
  int rc = check_hip(hipGetLastError(), "k_mupdate");
  if (rc || !nrm2) return rc;
  hipLaunchKernelGGL(k_finish_r, dim3(nbatch), dim3(256), 0, c->stream, rb.part, nblk, nrm2, nstride);
  return check_hip(hipGetLastError(), "k_finish_r");
}

int launch_mupdate_b(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K,
                     const double2* coef, int64_t cbs, double sign, double2* w, int64_t wbs,
                     int64_t n, double* nrm2, int64_t nstride, int nbatch, const RedBuf& rb) {
  return mupdate_b(c, V, ldv, vbs, K, coef, cbs, sign, w, wbs, n, nrm2, nstride, nbatch, rb);
}

int launch_mupdate_b(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int K,
                     const double2* coef, int64_t cbs, double sign, float2* w, int64_t wbs,
                     int64_t n, double* nrm2, int64_t nstride, int nbatch, const RedBuf& rb) {
  return mupdate_b(c, V, ldv, vbs, K, coef, cbs, sign, w, wbs, n, nrm2, nstride, nbatch, rb);
}

int launch_norm2_b(hps_ctx* c, const float2* w, int64_t wbs, int64_t n, double* nrm2, int64_t nbs,
                   int nbatch, const RedBuf& rb) {
  return launch_mupdate_b(c, (const float2*)nullptr, 0, 0, 0, nullptr, 0, 0.0, const_cast<float2*>(w),
                          wbs, n, nrm2, nbs, nbatch, rb);
}

int launch_demote_scaled(hps_ctx* c, const double2* x, double s, float2* y, int64_t n) {
  const int threads = 256;
  hipLaunchKernelGGL(k_demote_scaled, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                     c->stream, x, s, y, n);
  return check_hip(hipGetLastError(), "k_demote_scaled");
}

int launch_axpy_promote(hps_ctx* c, double s, const float2* x, double2* y, int64_t n) {
  const int threads = 256;
  hipLaunchKernelGGL(k_axpy_promote<float2>, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                     c->stream, s, x, y, n);
  return check_hip(hipGetLastError(), "k_axpy_promote");
}

int launch_axpy_promote(hps_ctx* c, double s, const double2* x, double2* y, int64_t n) {
  const int threads = 256;
  hipLaunchKernelGGL(k_axpy_promote<double2>, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads),
                     0, c->stream, s, x, y, n);
  return check_hip(hipGetLastError(), "k_axpy_promote");
}

int launch_mdot(hps_ctx* c, const double2* V, int64_t ldv, int K, const double2* w, int64_t n,
                double2* out, const RedBuf& rb) {
  return launch_mdot_b(c, V, ldv, 0, K, w, 0, n, out, 0, 1, rb);
}

int launch_mupdate(hps_ctx* c, const double2* V, int64_t ldv, int K, const double2* coef,
                   double sign, double2* w, int64_t n, double* nrm2, const RedBuf& rb) {
  return launch_mupdate_b(c, V, ldv, 0, K, coef, 0, sign, w, 0, n, nrm2, 0, 1, rb);
}

int launch_norm2(hps_ctx* c, const double2* w, int64_t n, double* nrm2, const RedBuf& rb) {
  return launch_mupdate_b(c, (const double2*)nullptr, 0, 0, 0, nullptr, 0, 0.0, const_cast<double2*>(w),
                          0, n, nrm2, 0, 1, rb);
}

int launch_norm2_b(hps_ctx* c, const double2* w, int64_t wbs, int64_t n, double* nrm2, int64_t nbs,
                   int nbatch, const RedBuf& rb) {
  return launch_mupdate_b(c, (const double2*)nullptr, 0, 0, 0, nullptr, 0, 0.0, const_cast<double2*>(w),
                          wbs, n, nrm2, nbs, nbatch, rb);
}

int launch_scale_by(hps_ctx* c, const double2* x, double2* y, int64_t n, const double* s,
                    int inv_sqrt) {
  return launch_scale_by_b(c, x, 0, y, 0, n, s, 0, inv_sqrt, 1);
}

int launch_scale_by_b(hps_ctx* c, const double2* x, int64_t xbs, double2* y, int64_t ybs, int64_t n,
                      const double* s, int64_t sstride, int inv_sqrt, int nbatch) {
  const int threads = 256;
  hipLaunchKernelGGL(k_scale_by, dim3((unsigned)((n + threads - 1) / threads), nbatch),
                     dim3(threads), 0, c->stream, x, xbs, y, ybs, n, s, sstride, inv_sqrt);
  return check_hip(hipGetLastError(), "k_scale_by");
}

int launch_sub_from(hps_ctx* c, const double2* a, double2* y, int64_t n) {
  const int threads = 256;
  hipLaunchKernelGGL(k_sub_from<double2>, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads),
                     0, c->stream, a, y, n);
  return check_hip(hipGetLastError(), "k_sub_from");
}

int launch_sub_from(hps_ctx* c, const float2* a, float2* y, int64_t n) {
  const int threads = 256;
  hipLaunchKernelGGL(k_sub_from<float2>, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads),
                     0, c->stream, a, y, n);
  return check_hip(hipGetLastError(), "k_sub_from");
}

int launch_gm_start(hps_ctx* c, GmresState* S, int nb) {
  hipLaunchKernelGGL(k_gm_start, dim3((nb + 63) / 64), dim3(64), 0, c->stream, S, nb);
  return check_hip(hipGetLastError(), "k_gm_start");
}

int launch_gm_givens(hps_ctx* c, GmresState* S, int nb, int j) {
  hipLaunchKernelGGL(k_gm_givens, dim3(nb), dim3(64), 0, c->stream, S, j, 1e-14);
  return check_hip(hipGetLastError(), "k_gm_givens");
}

int launch_gm_collect(hps_ctx* c, const GmresState* S, int nb, double* out) {
  hipLaunchKernelGGL(k_gm_collect, dim3((nb + 63) / 64), dim3(64), 0, c->stream, S, nb, out);
  return check_hip(hipGetLastError(), "k_gm_collect");
}

int launch_gm_trisolve(hps_ctx* c, GmresState* S, int nb, int k) {
  hipLaunchKernelGGL(k_gm_trisolve, dim3(nb), dim3(256), 0, c->stream, S, k);
  return check_hip(hipGetLastError(), "k_gm_trisolve");
}

int launch_cgs_pass(hps_ctx* c, bool update, const double2* V, int64_t ldv, int64_t vbs, int K,
                    const double2* coef, int64_t cbs, double2* w, int64_t wbs, int64_t n,
                    double2* out, int64_t obs, int nbatch, const RedBuf& rb) {
  if (K <= 0) return HPS_OK;
  if (K > 64) {
    // long cycles: separate update and dot kernels
    if (update) {
      int rc = launch_mupdate_b(c, V, ldv, vbs, K, coef, cbs, -1.0, w, wbs, n, nullptr, 0, nbatch, rb);
      if (rc) return rc;
    }
    return launch_mdot_b(c, V, ldv, vbs, K, w, wbs, n, out, obs, nbatch, rb);
  }
  if (nbatch > rb.nbatch) return fail(HPS_ERR_ARG, "batch too large");
  const int64_t tiles = (n + GN * 64 - 1) / (GN * 64);
  const int kc = (K + GK - 1) / GK;
  // more workgroups when fewer registers are live (see GKC)
  const int want = kc <= 4 ? 1024 : (kc <= 8 ? 768 : 512);
  const int nblk = (int)std::min<int64_t>(tiles, std::min(want, rb.nblk));
  dim3 grid(nblk, 1, nbatch);
#define HPS_CGS(U, KC)                                                                      \
  hipLaunchKernelGGL((k_cgs64<U, KC>), grid, dim3(GT), 0, c->stream, V, ldv, vbs, K, coef, cbs, w, \
                     wbs, n, rb.part)
  if (update) {
    if (kc <= 4) HPS_CGS(true, 4); else if (kc <= 8) HPS_CGS(true, 8); else HPS_CGS(true, 16);
  } else {
    if (kc <= 4) HPS_CGS(false, 4); else if (kc <= 8) HPS_CGS(false, 8); else HPS_CGS(false, 16);
  }
#undef HPS_CGS
  int rc = check_hip(hipGetLastError(), "k_cgs64");
  if (rc) return rc;
  return finish_c(c, rb, K, nblk, out, obs, nbatch);
}

}  // namespace hps
