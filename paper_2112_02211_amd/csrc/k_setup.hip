// Setup kernels: medium at the nodes, the homogenization constant lambda^tau,
// the homogenized Schur complements S~^tau and the packing of their inverses
// into the block layout streamed by the preconditioner (Sec. 4.1, Sec. 5.1).
#include "hps_internal.h"
#include "k_common.h"

namespace hps {
namespace {

// Physical coordinate of grid node g (0..p-1) along one axis of leaf e.
__device__ __forceinline__ double grid_x(const double* xi, double lo, double h, int e, int g) {
  return lo + h * ((double)e + 0.5 * (xi[g] + 1.0));
}

// C = kappa^2 (1 - b) at the interior nodes of every leaf (Sec. 2.1: the diagonal
// of C^tau; only its interior part enters the operator).
__global__ void k_eval_medium(int kind, const double* __restrict__ xi, int p, int E0, int E1,
                              double lo0, double lo1, double lo2, double h, double kappa2,
                              const double* __restrict__ bc, const double2* __restrict__ ba,
                              int nbump, double width, const double2* __restrict__ nodal,
                              int64_t nl, int c_complex, void* __restrict__ Cout) {
  const int n1 = p - 2, ni = n1 * n1 * n1, nb = 6 * n1 * n1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nl * ni) return;
  const int64_t tau = gid / ni;
  const int m = (int)(gid - tau * ni);
  double2 b = make_double2(0.0, 0.0);
  if (kind == HPS_MEDIUM_NODAL) {
    b = nodal[tau * (ni + nb) + m];
  } else if (kind == HPS_MEDIUM_BUMPS) {
    const int ex = (int)(tau % E0), ey = (int)((tau / E0) % E1), ez = (int)(tau / ((int64_t)E0 * E1));
    const int i = m % n1, j = (m / n1) % n1, k = m / (n1 * n1);
    const double x = grid_x(xi, lo0, h, ex, i + 1);
    const double y = grid_x(xi, lo1, h, ey, j + 1);
    const double z = grid_x(xi, lo2, h, ez, k + 1);
    const double iw2 = 1.0 / (width * width);
    for (int q = 0; q < nbump; ++q) {
      const double dx = x - bc[3 * q], dy = y - bc[3 * q + 1], dz = z - bc[3 * q + 2];
      const double g = exp(-(dx * dx + dy * dy + dz * dz) * iw2);
      b.x += ba[q].x * g;
      b.y += ba[q].y * g;
    }
  }
  if (c_complex) {
    static_cast<double2*>(Cout)[gid] = make_double2(kappa2 * (1.0 - b.x), -kappa2 * b.y);
  } else {
    static_cast<double*>(Cout)[gid] = kappa2 * (1.0 - b.x);
  }
}

// lambda^tau = (max + min)/2 of diag(C_ii) per leaf (Sec. 4.1), taken on the
// real and imaginary parts separately.  If -E_Delta - lambda comes within
// 1e-3 |lambda| of zero (a Dirichlet resonance of the homogenized interior
// operator, on which the paper is silent) lambda is moved to lambda (1 + 0.01 i).
// delta > 0: lambda rounded to the grid of spacing delta kappa^2 (real and
// imaginary parts, floor(x / h + 1/2) h) before the resonance guard.
__global__ __launch_bounds__(256) void k_lambda(const void* __restrict__ Cv, int c_complex,
                                                int ni, const double* __restrict__ Ed3,
                                                double delta, double kappa,
                                                double2* __restrict__ lam, int* __restrict__ shifted) {
  const int64_t tau = blockIdx.x;
  __shared__ double red[4][256];
  double mnr = 1e300, mxr = -1e300, mni = 1e300, mxi = -1e300;
  for (int m = threadIdx.x; m < ni; m += blockDim.x) {
    double re, im = 0.0;
    if (c_complex) {
      const double2 v = static_cast<const double2*>(Cv)[tau * ni + m];
      re = v.x;
      im = v.y;
    } else {
      re = static_cast<const double*>(Cv)[tau * ni + m];
    }
    mnr = fmin(mnr, re); mxr = fmax(mxr, re);
    mni = fmin(mni, im); mxi = fmax(mxi, im);
  }
  red[0][threadIdx.x] = mnr; red[1][threadIdx.x] = mxr;
  red[2][threadIdx.x] = mni; red[3][threadIdx.x] = mxi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
      red[2][threadIdx.x] = fmin(red[2][threadIdx.x], red[2][threadIdx.x + s]);
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
    }
    __syncthreads();
  }
  double lr = 0.5 * (red[0][0] + red[1][0]);
  double li = 0.5 * (red[2][0] + red[3][0]);
  if (delta > 0.0) {
    const double h = delta * kappa * kappa;
    lr = floor(lr / h + 0.5) * h;
    li = floor(li / h + 0.5) * h;
  }
  __syncthreads();
  // distance of lambda to the spectrum of -L3
  double dmin = 1e300;
  for (int m = threadIdx.x; m < ni; m += blockDim.x) {
    const double dr = -Ed3[m] - lr;
    dmin = fmin(dmin, sqrt(dr * dr + li * li));
  }
  red[0][threadIdx.x] = dmin;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[0][threadIdx.x] = fmin(red[0][threadIdx.x], red[0][threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mag = sqrt(lr * lr + li * li);
    const int sh = red[0][0] < 1e-3 * mag;
    // lambda (1 + 0.01 i) = (lr - 0.01 li) + i (li + 0.01 lr)
    lam[tau] = sh ? make_double2(lr - 0.01 * li, li + 0.01 * lr) : make_double2(lr, li);
    shifted[tau] = sh;
  }
}

// S~^tau = F_bb - P diag(d_tau) Q with d_tau[m] = 1 / (-E_Delta[m] - lambda^tau),
// for the leaves e0 .. e0+ne-1, written column major ([leaf][col][row]).
// F_bb: on face f (axis ax, endpoint e, sign s) row r holds s D[e][e] + i eta on
// the diagonal and s D[e][e'] at the node of the opposite face on the same
// normal line (eq. (flux) restricted to face columns, plus i eta I).
constexpr int SB = 64;   // output tile
constexpr int SK = 16;   // inner tile
__global__ __launch_bounds__(256) void k_build_schur(const double* __restrict__ P,
                                                     const double* __restrict__ Q,
                                                     const double* __restrict__ Ed3,
                                                     const double2* __restrict__ lam,
                                                     const double* __restrict__ D, int p, int nb,
                                                     int ni, double eta, int e0,
                                                     double2* __restrict__ S) {
  __shared__ double Ps[SB][SK + 1];
  __shared__ double Qr[SK][SB + 1];
  __shared__ double Qi[SK][SB + 1];
  const int r0 = blockIdx.x * SB, c0 = blockIdx.y * SB;
  const int e = blockIdx.z;
  const double2 lm = lam[e0 + e];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double ar[4][4], ai[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) { ar[a][b] = 0.0; ai[a][b] = 0.0; }
  for (int k0 = 0; k0 < ni; k0 += SK) {
    for (int t = threadIdx.x; t < SB * SK; t += 256) {
      const int rr = t / SK, kk = t % SK;
      const int r = r0 + rr, k = k0 + kk;
      Ps[rr][kk] = (r < nb && k < ni) ? P[(size_t)r * ni + k] : 0.0;
    }
    for (int t = threadIdx.x; t < SB * SK; t += 256) {
      const int kk = t / SB, cc = t % SB;
      const int k = k0 + kk, cix = c0 + cc;
      double qr = 0.0, qi = 0.0;
      if (k < ni && cix < nb) {
        // d = 1 / (a + i b) with a = -E - lr, b = -li
        const double a = -Ed3[k] - lm.x, b = -lm.y;
        const double den = 1.0 / (a * a + b * b);
        const double q = Q[(size_t)k * nb + cix];
        qr = q * a * den;
        qi = -q * b * den;
      }
      Qr[kk][cc] = qr;
      Qi[kk][cc] = qi;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SK; ++kk) {
      double pa[4], qb[4], qc[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) pa[a] = Ps[ty * 4 + a][kk];
#pragma unroll
      for (int b = 0; b < 4; ++b) { qb[b] = Qr[kk][tx * 4 + b]; qc[b] = Qi[kk][tx * 4 + b]; }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          ar[a][b] = fma(pa[a], qb[b], ar[a][b]);
          ai[a][b] = fma(pa[a], qc[b], ai[a][b]);
        }
    }
    __syncthreads();
  }
  const int n1 = p - 2, L = n1 * n1;
  double2* Se = S + (size_t)e * nb * nb;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = r0 + ty * 4 + a, cix = c0 + tx * 4 + b;
      if (r >= nb || cix >= nb) continue;
      double fr = 0.0, fi = 0.0;
      const int f = r / L;
      const int ax_hi = f & 1;
      const int ep = ax_hi ? p - 1 : 0, eo = ax_hi ? 0 : p - 1;
      const double sg = ax_hi ? 1.0 : -1.0;
      if (cix == r) {
        fr = sg * D[ep * p + ep];
        fi = eta;
      } else if (cix == r + (ax_hi ? -L : L)) {
        fr = sg * D[ep * p + eo];
      }
      Se[(size_t)cix * nb + r] = make_double2(fr - ar[a][b], fi - ai[a][b]);
    }
}

__device__ __forceinline__ uint32_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// Column-major inverse blocks [leaf][col][row] (complex double) into the
// streamed layout [leaf][col group][row][cw] in the requested precision; the
// padded columns are zero.
__global__ void k_pack_blocks(const double2* __restrict__ Sinv, int nb, int ncp, int prec,
                              int64_t e0, int ne, void* __restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)ne * ncp * nb;
  if (gid >= total) return;
  const int64_t e = gid / ((int64_t)ncp * nb);
  const int rem = (int)(gid - e * (int64_t)ncp * nb);
  const int c = rem / nb, r = rem % nb;
  const double2 v = (c < nb) ? Sinv[((size_t)e * nb + c) * nb + r] : make_double2(0.0, 0.0);
  const int cw = prec == kFP64 ? 1 : (prec == kFP32 ? 2 : 4);
  const int64_t eo = e0 + e;
  const int64_t idx = ((eo * (ncp / cw) + c / cw) * nb + r) * cw + (c % cw);
  if (prec == kFP64) {
    static_cast<double2*>(out)[idx] = v;
  } else if (prec == kFP32) {
    static_cast<float2*>(out)[idx] = make_float2((float)v.x, (float)v.y);
  } else {
    static_cast<uint32_t*>(out)[idx] = f2bf((float)v.x) | (f2bf((float)v.y) << 16);
  }
}

}  // namespace

int launch_eval_medium(hps_ctx* c, const hps_medium* b, const double* d_bump_c,
                       const double2* d_bump_a, int nbump) {
  const int64_t total = c->nl * c->ni;
  const int kind = b ? b->kind : HPS_MEDIUM_ZERO;
  const int threads = 256;
  const int64_t blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(k_eval_medium, dim3((unsigned)blocks), dim3(threads), 0, c->stream, kind,
                     c->d_tab + tab_off_xi(c->p), c->p, c->E[0], c->E[1], c->lo[0], c->lo[1],
                     c->lo[2], c->h, c->kappa * c->kappa, d_bump_c, d_bump_a, nbump,
                     b ? b->width : 1.0,
                     (kind == HPS_MEDIUM_NODAL) ? reinterpret_cast<const double2*>(b->nodal) : nullptr,
                     c->nl, c->c_complex, c->d_C);
  return check_hip(hipGetLastError(), "k_eval_medium");
}

int launch_lambda(hps_ctx* c) {
  int* d_sh = nullptr;
  int rc = dev_alloc(c, (void**)&d_sh, sizeof(int) * c->nl);
  if (rc) return rc;
  hipLaunchKernelGGL(k_lambda, dim3((unsigned)c->nl), dim3(256), 0, c->stream, c->d_C,
                     c->c_complex, c->ni, c->d_tab + tab_off_ed3(c->p), c->lambda_bucket, c->kappa,
                     c->d_lambda, d_sh);
  rc = check_hip(hipGetLastError(), "k_lambda");
  if (rc) return rc;
  std::vector<int> sh(c->nl);
  HPS_TRY_HIP(hipMemcpyAsync(sh.data(), d_sh, sizeof(int) * c->nl, hipMemcpyDeviceToHost, c->stream));
  HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  HPS_TRY_HIP(hipFree(d_sh));
  c->dev_bytes -= sizeof(int) * c->nl;
  c->n_shifted = 0;
  for (int v : sh) c->n_shifted += v;
  return HPS_OK;
}

int launch_build_schur(hps_ctx* c, const double* dP, const double* dQ, const double2* lam, int e0,
                       int ne, double2* S) {
  dim3 grid((c->nb + SB - 1) / SB, (c->nb + SB - 1) / SB, ne);
  hipLaunchKernelGGL(k_build_schur, grid, dim3(256), 0, c->stream, dP, dQ,
                     c->d_tab + tab_off_ed3(c->p), lam, c->d_tab + tab_off_D(c->p), c->p,
                     c->nb, c->ni, c->eta, e0, S);
  return check_hip(hipGetLastError(), "k_build_schur");
}

int launch_pack_blocks(hps_ctx* c, const double2* Sinv, int e0, int ne, int prec) {
  const Blocks& B = c->blk[prec];
  const int64_t total = (int64_t)ne * B.ncp * c->nb;
  const int threads = 256;
  hipLaunchKernelGGL(k_pack_blocks, dim3((unsigned)((total + threads - 1) / threads)),
                     dim3(threads), 0, c->stream, Sinv, c->nb, B.ncp, prec, (int64_t)e0, ne,
                     B.data);
  return check_hip(hipGetLastError(), "k_pack_blocks");
}

}  // namespace hps
