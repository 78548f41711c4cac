// Krylov primitives for the GMRES drivers: multi-dot products (the Arnoldi
// inner products of classical Gram-Schmidt), multi-axpy updates, norms and
// the small Hessenberg / Givens state, all in FP64 on the device.
//
// Reductions are two-level and deterministic: every workgroup reduces its
// slice with wavefront shuffles and LDS and writes one partial per output;
// the workgroup that finishes last (an agent-scope counter) sums the partials
// in a fixed order and resets the counter, so no second launch is needed.
#include "hps_internal.h"
#include "hps_krylov.h"
#include "k_common.h"

namespace hps {
namespace {

constexpr int RT = 256;         // threads per reduction workgroup
constexpr int RW = RT / 64;     // wavefronts per workgroup
constexpr int KB = 16;          // outputs per workgroup in the multi-dot

__device__ __forceinline__ bool arrive_last(unsigned* counter, unsigned nblk) {
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (prev == nblk - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// out[k] = sum_n conj(V[k ldv + n]) w[n]; batch b (blockIdx.z) offsets every
// pointer by its batch stride.
__global__ __launch_bounds__(RT) void k_mdot(const double2* __restrict__ V, int64_t ldv,
                                             int64_t vbs, int K, const double2* __restrict__ w,
                                             int64_t wbs, int64_t n, double2* __restrict__ part,
                                             double2* __restrict__ out, int64_t obs,
                                             unsigned* __restrict__ counter) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  w += bz * wbs;
  out += bz * obs;
  const unsigned nblk = gridDim.x;
  const int k0 = blockIdx.y * KB;
  double2* pz = part + ((int64_t)bz * gridDim.y * KB) * nblk;
  unsigned* cz = counter + bz * gridDim.y + blockIdx.y;
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
  if (!arrive_last(cz, nblk)) return;
  for (int kk = wid; kk < kn; kk += RW) {
    double re = 0.0, im = 0.0;
    const double2* pp = pz + (int64_t)(blockIdx.y * KB + kk) * nblk;
    for (unsigned b = lane; b < nblk; b += 64) {
      const double2 v = pp[b];
      re += v.x;
      im += v.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) out[k0 + kk] = make_double2(re, im);
  }
  if (threadIdx.x == 0) *cz = 0u;
}

// w[i] += sign * sum_k V[k ldv + i] coef[k]; optionally nrm2 = ||w||^2 after the update.
__global__ __launch_bounds__(RT) void k_mupdate(const double2* __restrict__ V, int64_t ldv,
                                                int64_t vbs, int K, const double2* __restrict__ coef,
                                                int64_t cbs, double sign, double2* __restrict__ w,
                                                int64_t wbs, int64_t n, double* __restrict__ nrm2,
                                                int64_t nstride, double2* __restrict__ part,
                                                unsigned* __restrict__ counter) {
  const int bz = blockIdx.z;
  V += bz * vbs;
  w += bz * wbs;
  coef += bz * cbs;
  __shared__ double2 cs[kMaxRestart + 1];
  for (int k = threadIdx.x; k < K; k += RT) {
    const double2 c = coef[k];
    cs[k] = make_double2(sign * c.x, sign * c.y);
  }
  __syncthreads();
  const unsigned nblk = gridDim.x;
  double sq = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)nblk * RT) {
    double2 a = w[i];
    int k = 0;
    for (; k + 4 <= K; k += 4) {
      double2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = V[(int64_t)(k + u) * ldv + i];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 c = cs[k + u];
        a.x = fma(v[u].x, c.x, fma(-v[u].y, c.y, a.x));
        a.y = fma(v[u].x, c.y, fma(v[u].y, c.x, a.y));
      }
    }
    for (; k < K; ++k) {
      const double2 v = V[(int64_t)k * ldv + i];
      const double2 c = cs[k];
      a.x = fma(v.x, c.x, fma(-v.y, c.y, a.x));
      a.y = fma(v.x, c.y, fma(v.y, c.x, a.y));
    }
    w[i] = a;
    sq = fma(a.x, a.x, fma(a.y, a.y, sq));
  }
  if (!nrm2) return;
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
  unsigned* cz = counter + bz;
  if (!arrive_last(cz, nblk)) return;
  if (wid == 0) {
    double s = 0.0;
    for (unsigned b = lane; b < nblk; b += 64) s += pz[b];
    s = wave_sum(s);
    if (lane == 0) nrm2[bz * nstride] = s;
  }
  if (threadIdx.x == 0) *cz = 0u;
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

__global__ void k_sub_from(const double2* __restrict__ a, double2* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 u = a[i], v = y[i];
  y[i] = make_double2(u.x - v.x, u.y - v.y);
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
// subdiagonal, and the updated residual estimate |g_{j+1}|.
__global__ void k_gm_givens(GmresState* __restrict__ S, int nb, int j, double tiny) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  GmresState& s = S[b];
  double2* h = &s.H[(int64_t)j * (kMaxRestart + 1)];
  for (int i = 0; i <= j; ++i) h[i] = cadd(s.h1[i], s.h2[i]);
  const double hn = sqrt(s.nrm2);
  h[j + 1] = make_double2(hn, 0.0);
  for (int i = 0; i < j; ++i) {
    const double c = s.cs[i];
    const double2 sn = s.sn[i];
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
    sn = make_double2(ph.x * bm / r, ph.y * bm / r);   // phase(a) * conj(b) / r, b real
    h[j] = make_double2(ph.x * r, ph.y * r);
  }
  h[j + 1] = make_double2(0.0, 0.0);
  s.cs[j] = c;
  s.sn[j] = sn;
  const double2 gj = s.g[j];
  s.g[j + 1] = make_double2(-(sn.x * gj.x + sn.y * gj.y), -(sn.x * gj.y - sn.y * gj.x));  // -conj(sn) g_j
  s.g[j] = cscale(gj, c);
  s.res = sqrt(s.g[j + 1].x * s.g[j + 1].x + s.g[j + 1].y * s.g[j + 1].y);
  s.breakdown = (hn <= tiny * (r > 0 ? r : 1.0)) ? 1 : 0;
}

// y = R^{-1} g for the leading k x k triangle of the rotated Hessenberg matrix.
__global__ void k_gm_trisolve(GmresState* __restrict__ S, int nb, int k) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  GmresState& s = S[b];
  for (int i = k - 1; i >= 0; --i) {
    double2 acc = s.g[i];
    for (int jj = i + 1; jj < k; ++jj)
      acc = csub(acc, cmul(s.H[(int64_t)jj * (kMaxRestart + 1) + i], s.y[jj]));
    const double2 d = s.H[(int64_t)i * (kMaxRestart + 1) + i];
    const double dd = d.x * d.x + d.y * d.y;
    s.y[i] = dd > 0.0 ? make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                      : make_double2(0.0, 0.0);
  }
}

}  // namespace

int red_buf(hps_ctx* c, int kmax, RedBuf* rb) {
  const int nblk = kRedBlocks;
  const size_t part_bytes = (size_t)(kmax + KB) * nblk * sizeof(double2) * kMaxBatch;
  const size_t cnt_bytes = sizeof(unsigned) * 4096;
  const size_t need = part_bytes + cnt_bytes;
  const bool fresh = c->w_red.bytes < need;
  int rc = ws_reserve(c, &c->w_red, need);
  if (rc) return rc;
  rb->part = static_cast<double2*>(c->w_red.ptr);
  rb->counter = reinterpret_cast<unsigned*>(static_cast<char*>(c->w_red.ptr) + part_bytes);
  rb->nblk = nblk;
  if (fresh) HPS_TRY_HIP(hipMemsetAsync(rb->counter, 0, cnt_bytes, c->stream));
  return HPS_OK;
}

static int nblocks_for(int64_t n, int nblk) {
  const int64_t want = (n + RT - 1) / RT;
  return (int)(want < nblk ? (want > 0 ? want : 1) : nblk);
}

int launch_mdot_b(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K, const double2* w,
                  int64_t wbs, int64_t n, double2* out, int64_t obs, int nbatch, const RedBuf& rb) {
  if (K <= 0) return HPS_OK;
  const int gy = (K + KB - 1) / KB;
  if ((int64_t)gy * nbatch > 4096 - kMaxBatch || K > kMaxRestart + 1 || nbatch > kMaxBatch)
    return fail(HPS_ERR_ARG, "multi-dot too large");
  dim3 grid(nblocks_for(n, rb.nblk), gy, nbatch);
  hipLaunchKernelGGL(k_mdot, grid, dim3(RT), 0, c->stream, V, ldv, vbs, K, w, wbs, n, rb.part, out,
                     obs, rb.counter);
  return check_hip(hipGetLastError(), "k_mdot");
}

int launch_mupdate_b(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K,
                     const double2* coef, int64_t cbs, double sign, double2* w, int64_t wbs,
                     int64_t n, double* nrm2, int64_t nstride, int nbatch, const RedBuf& rb) {
  if (K > kMaxRestart + 1 || nbatch > kMaxBatch) return fail(HPS_ERR_ARG, "update too large");
  dim3 grid(nblocks_for(n, rb.nblk), 1, nbatch);
  hipLaunchKernelGGL(k_mupdate, grid, dim3(RT), 0, c->stream, V, ldv, vbs, K, coef, cbs, sign, w,
                     wbs, n, nrm2, nstride, rb.part, rb.counter + 4096 - kMaxBatch);
  return check_hip(hipGetLastError(), "k_mupdate");
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
  return launch_mupdate_b(c, nullptr, 0, 0, 0, nullptr, 0, 0.0, const_cast<double2*>(w), 0, n,
                          nrm2, 0, 1, rb);
}

int launch_norm2_b(hps_ctx* c, const double2* w, int64_t wbs, int64_t n, double* nrm2, int64_t nbs,
                   int nbatch, const RedBuf& rb) {
  return launch_mupdate_b(c, nullptr, 0, 0, 0, nullptr, 0, 0.0, const_cast<double2*>(w), wbs, n,
                          nrm2, nbs, nbatch, rb);
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
  hipLaunchKernelGGL(k_sub_from, dim3((unsigned)((n + threads - 1) / threads)), dim3(threads), 0,
                     c->stream, a, y, n);
  return check_hip(hipGetLastError(), "k_sub_from");
}

int launch_gm_start(hps_ctx* c, GmresState* S, int nb) {
  hipLaunchKernelGGL(k_gm_start, dim3((nb + 63) / 64), dim3(64), 0, c->stream, S, nb);
  return check_hip(hipGetLastError(), "k_gm_start");
}

int launch_gm_givens(hps_ctx* c, GmresState* S, int nb, int j) {
  hipLaunchKernelGGL(k_gm_givens, dim3((nb + 63) / 64), dim3(64), 0, c->stream, S, nb, j, 1e-14);
  return check_hip(hipGetLastError(), "k_gm_givens");
}

int launch_gm_trisolve(hps_ctx* c, GmresState* S, int nb, int k) {
  hipLaunchKernelGGL(k_gm_trisolve, dim3((nb + 63) / 64), dim3(64), 0, c->stream, S, nb, k);
  return check_hip(hipGetLastError(), "k_gm_trisolve");
}

}  // namespace hps
