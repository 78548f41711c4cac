// y = A x: the matrix-free application of the global HPS operator (Sec. 3.2).
//
// Sweep (Algorithm 1 and the local part of Algorithm 2): one workgroup per leaf
// stages the leaf's n values in LDS on the full p^3 Chebyshev grid (corner and
// edge slots are never touched).  Each thread owns one grid line per axis,
// keeps its p values in registers and contracts them with the rows of D^2 (the
// line's interior outputs; eq. (leafmat), whose face-column entries give
// A_ib v_b) and with the end rows of D (the line's two face outputs, eq.
// (flux)).  The three axis passes accumulate through LDS; the last one
// subtracts C v (Algorithm 1 with the sign of eq. (leafmat)).  Face rows get
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

template <int P>
struct Leaf {
  static constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  // grid index ((k P + j) P + i) of local node m
  __device__ static __forceinline__ int grid_of(int m) {
    if (m < NI) {
      const int i = m % N1 + 1, j = (m / N1) % N1 + 1, k = m / L + 1;
      return (k * P + j) * P + i;
    }
    const int mm = m - NI, f = mm / L, r = mm - f * L;
    const int a = r % N1 + 1, b = r / N1 + 1, e = (f & 1) ? P - 1 : 0;
    const int ax = f >> 1;
    if (ax == 0) return (b * P + a) * P + e;
    if (ax == 1) return (b * P + e) * P + a;
    return (e * P + b) * P + a;
  }
};

template <int P>
constexpr int sweep_threads() {
  return ((P - 2) * (P - 2) + 63) / 64 * 64;
}

// One axis pass over the lines of one leaf.  AX = 0, 1, 2 (x, y, z).
template <int P, int AX, bool CC>
__device__ __forceinline__ void axis_pass(const double2* __restrict__ U, double2* __restrict__ ACC,
                                          const double* __restrict__ D, const double* __restrict__ D2,
                                          double eta, double2* __restrict__ yv, double2* __restrict__ gv,
                                          const void* __restrict__ Cv, int64_t tau, int line) {
  using Lf = Leaf<P>;
  constexpr int N1 = Lf::N1, L = Lf::L, NI = Lf::NI;
  const int a = line % N1 + 1, b = line / N1 + 1;  // the two other grid coordinates
  int base, stride;
  if (AX == 0) { base = (b * P + a) * P; stride = 1; }
  else if (AX == 1) { base = b * P * P + a; stride = P; }
  else { base = b * P + a; stride = P * P; }
  double2 u[P];
#pragma unroll
  for (int q = 0; q < P; ++q) u[q] = U[base + q * stride];
  // interior outputs along the line
#pragma unroll
  for (int t = 1; t < P - 1; ++t) {
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < P; ++q) cfma_r(s, D2[t * P + q], u[q]);
    int m;
    if (AX == 0) m = (t - 1) + N1 * (a - 1) + L * (b - 1);
    else if (AX == 1) m = (a - 1) + N1 * (t - 1) + L * (b - 1);
    else m = (a - 1) + N1 * (b - 1) + L * (t - 1);
    if (AX == 0) {
      ACC[m] = make_double2(-s.x, -s.y);
    } else if (AX == 1) {
      const double2 c = ACC[m];
      ACC[m] = make_double2(c.x - s.x, c.y - s.y);
    } else {
      const double2 c = ACC[m];
      double2 cu;
      if (CC) {
        const double2 cc = static_cast<const double2*>(Cv)[tau * NI + m];
        cu = cmul(cc, u[t]);
      } else {
        const double cr = static_cast<const double*>(Cv)[tau * NI + m];
        cu = cscale(u[t], cr);
      }
      yv[m] = make_double2(c.x - s.x - cu.x, c.y - s.y - cu.y);
    }
  }
  // the two face outputs of the line: outward normal derivative +/- i eta u
  double2 lo = make_double2(0.0, 0.0), hi = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < P; ++q) {
    cfma_r(lo, -D[q], u[q]);
    cfma_r(hi, D[(P - 1) * P + q], u[q]);
  }
  const int flo = 2 * AX, fhi = 2 * AX + 1;
  const double2 ul = u[0], uh = u[P - 1];
  yv[NI + flo * L + line] = make_double2(lo.x - eta * ul.y, lo.y + eta * ul.x);
  yv[NI + fhi * L + line] = make_double2(hi.x - eta * uh.y, hi.y + eta * uh.x);
  gv[flo * L + line] = make_double2(lo.x + eta * ul.y, lo.y - eta * ul.x);
  gv[fhi * L + line] = make_double2(hi.x + eta * uh.y, hi.y - eta * uh.x);
}

template <int P, bool CC>
__global__ __launch_bounds__(sweep_threads<P>()) void k_apply_sweep(
    const double2* __restrict__ x, double2* __restrict__ y, double2* __restrict__ g,
    const void* __restrict__ Cv, const double* __restrict__ tab, double eta, int64_t nl, int64_t N) {
  using Lf = Leaf<P>;
  constexpr int L = Lf::L, NN = Lf::NN, NB = Lf::NB;
  constexpr int BD = sweep_threads<P>();
  __shared__ double2 U[P * P * P];
  __shared__ double2 ACC[Lf::NI];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const double2* xv = x + rhs * N + tau * NN;
  double2* yv = y + rhs * N + tau * NN;
  double2* gv = g + (rhs * nl + tau) * NB;
  const double* D = tab + tab_off_D(P);
  const double* D2 = tab + tab_off_D2(P);
  constexpr int NLOAD = (NN + BD - 1) / BD;
  double2 tmp[NLOAD];
#pragma unroll
  for (int s = 0; s < NLOAD; ++s) {
    const int m = threadIdx.x + s * BD;
    if (m < NN) tmp[s] = xv[m];
  }
#pragma unroll
  for (int s = 0; s < NLOAD; ++s) {
    const int m = threadIdx.x + s * BD;
    if (m < NN) U[Lf::grid_of(m)] = tmp[s];
  }
  __syncthreads();
  const int line = threadIdx.x;
  if (line < L) axis_pass<P, 0, CC>(U, ACC, D, D2, eta, yv, gv, Cv, tau, line);
  __syncthreads();
  if (line < L) axis_pass<P, 1, CC>(U, ACC, D, D2, eta, yv, gv, Cv, tau, line);
  __syncthreads();
  if (line < L) axis_pass<P, 2, CC>(U, ACC, D, D2, eta, yv, gv, Cv, tau, line);
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
int sweep_launch(hps_ctx* c, const double2* x, double2* y, double2* g, int nrhs) {
  dim3 grid((unsigned)c->nl, (unsigned)nrhs);
  if (c->c_complex)
    hipLaunchKernelGGL((k_apply_sweep<P, true>), grid, dim3(sweep_threads<P>()), 0, c->stream, x, y,
                       g, c->d_C, c->d_tab, c->eta, c->nl, c->N);
  else
    hipLaunchKernelGGL((k_apply_sweep<P, false>), grid, dim3(sweep_threads<P>()), 0, c->stream, x,
                       y, g, c->d_C, c->d_tab, c->eta, c->nl, c->N);
  return check_hip(hipGetLastError(), "k_apply_sweep");
}

}  // namespace

int launch_apply(hps_ctx* c, const double2* x, double2* y, int nrhs) {
  const size_t gbytes = (size_t)nrhs * c->nl * c->nb * sizeof(double2);
  int rc = ws_reserve(c, &c->w_g, gbytes);
  if (rc) return rc;
  double2* g = static_cast<double2*>(c->w_g.ptr);
  hipEvent_t ev0;
  if ((rc = timing_begin(c, &ev0))) return rc;
  switch (c->p) {
    case 4: rc = sweep_launch<4>(c, x, y, g, nrhs); break;
    case 5: rc = sweep_launch<5>(c, x, y, g, nrhs); break;
    case 6: rc = sweep_launch<6>(c, x, y, g, nrhs); break;
    case 7: rc = sweep_launch<7>(c, x, y, g, nrhs); break;
    case 8: rc = sweep_launch<8>(c, x, y, g, nrhs); break;
    case 9: rc = sweep_launch<9>(c, x, y, g, nrhs); break;
    case 10: rc = sweep_launch<10>(c, x, y, g, nrhs); break;
    case 11: rc = sweep_launch<11>(c, x, y, g, nrhs); break;
    case 12: rc = sweep_launch<12>(c, x, y, g, nrhs); break;
    case 13: rc = sweep_launch<13>(c, x, y, g, nrhs); break;
    case 14: rc = sweep_launch<14>(c, x, y, g, nrhs); break;
    case 15: rc = sweep_launch<15>(c, x, y, g, nrhs); break;
    case 16: rc = sweep_launch<16>(c, x, y, g, nrhs); break;
    default: return fail(HPS_ERR_UNSUPPORTED, "p out of range");
  }
  if (rc) return rc;
  const int64_t total = c->nl * c->nb;
  const int threads = 256;
  hipLaunchKernelGGL(k_apply_exchange, dim3((unsigned)((total + threads - 1) / threads), nrhs),
                     dim3(threads), 0, c->stream, y, g, c->d_nbr, c->ni, c->nb, c->n1 * c->n1, c->nl,
                     c->N);
  if ((rc = check_hip(hipGetLastError(), "k_apply_exchange"))) return rc;
  return timing_end(c, 0, ev0);
}

}  // namespace hps
