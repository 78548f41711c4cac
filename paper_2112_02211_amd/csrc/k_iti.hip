// The face-reduced form of the HPS system with the exact impedance-to-impedance
// (ItI) maps of the leaves (Sec. 2.2), and the interface rule that a leaf's
// incoming impedance on a shared face is minus the neighbour's outgoing
// impedance there (eq. (2x2)).
//
// Unknowns: the incoming impedance f on every leaf face, [rhs][leaf][n_b] in
// the leaf's face order.  On each leaf the outgoing impedance is g = R f + h,
// with the exact ItI map
//     R = I - 2 i eta S^{-1},   S = F_bb - F_bi A_ii^{-1} A_ib
// (the exact Schur complement: A_ii carries the variable C = kappa^2 (1 - b)),
// and the source term h = 2 i eta S^{-1} F_bi A_ii^{-1} s_i = (I - R) F_bi v
// with v = A_ii^{-1} s_i.  With Pi the exchange (the neighbour's values on
// each shared face, 0 on the domain boundary) the system is
//     (I + Pi R) f = t - Pi h,
// and the leaf solution is recovered from f as
//     u_b = S^{-1} (f - F_bi v) = (I - R)(f - F_bi v) / (2 i eta),
//     u_i = v - A_ii^{-1} A_ib u_b.
// Its solution is the same discrete u as that of A u = b.
//
// Stored per leaf: R (n_b x n_b, FP64 complex) and A_ii^{-1} (n_i x n_i).  The
// hot operator is one streaming pass over all R (a dense block-diagonal
// product, HBM-bound like the preconditioner's block stream) and the face
// exchange.  The setup factors A_ii and S with rocSOLVER and forms X =
// A_ii^{-1} A_ib and F_bi X with rocBLAS batched GEMMs.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <string>
#include <vector>

#include "hps_internal.h"

namespace hps {
namespace {

// A_ii of leaves e0 .. e0+ne-1, column-major (element (r, c) at c * ni + r):
// the interior rows of -(D2 x I x I + I x D2 x I + I x I x D2) at interior
// columns, minus diag(C).
__global__ void k_build_aii(const double* __restrict__ D2, int p, int n1, int ni,
                            const void* __restrict__ Cv, int cplx, int64_t e0, int ne,
                            double2* __restrict__ A) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)ni * ni;
  if (gid >= per * ne) return;
  const int e = (int)(gid / per);
  const int64_t rc = gid - (int64_t)e * per;
  const int col = (int)(rc / ni), row = (int)(rc - (int64_t)col * ni);
  const int ri = row % n1, rj = (row / n1) % n1, rk = row / (n1 * n1);
  const int ci = col % n1, cj = (col / n1) % n1, ck = col / (n1 * n1);
  double v = 0.0;
  if (rj == cj && rk == ck) v -= D2[(1 + ri) * p + 1 + ci];
  if (ri == ci && rk == ck) v -= D2[(1 + rj) * p + 1 + cj];
  if (ri == ci && rj == cj) v -= D2[(1 + rk) * p + 1 + ck];
  double2 out = make_double2(v, 0.0);
  if (row == col) {
    const int64_t ci64 = (e0 + e) * (int64_t)ni + row;
    if (cplx) {
      const double2 cc = static_cast<const double2*>(Cv)[ci64];
      out.x -= cc.x;
      out.y -= cc.y;
    } else {
      out.x -= static_cast<const double*>(Cv)[ci64];
    }
  }
  A[gid] = out;
}

// dst[e] = src for e < ne (complex, len entries each)
__global__ void k_bcast(const double2* __restrict__ src, int64_t len, int ne, double2* __restrict__ dst) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= len * ne) return;
  dst[gid] = src[gid % len];
}

// R = I - 2 i eta S^{-1} of leaves e0 .., column-major n_b x n_b
__global__ void k_iti_pack(const double2* __restrict__ Sinv, int nb, double eta, int64_t e0, int ne,
                           double2* __restrict__ R) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nb * nb;
  if (gid >= per * ne) return;
  const int64_t rc = gid % per;
  const int col = (int)(rc / nb), row = (int)(rc - (int64_t)col * nb);
  const double2 s = Sinv[gid];
  // -2 i eta (x + i y) = 2 eta y - 2 i eta x
  R[e0 * per + gid] = make_double2((row == col ? 1.0 : 0.0) + 2.0 * eta * s.y, -2.0 * eta * s.x);
}

// Placement of one leaf's part of a vector: base + rhs * r + tau * l + o.
struct VecAt {
  int64_t r, l;
  int o;
};

// y_tau = a0 z_tau + a1 M_tau x_tau for every leaf tau (grid x) and
// right-hand side (grid y).  M_tau: rows x cols, column-major; complex and one
// per leaf (REAL false), or one real matrix shared by all leaves (REAL true).
// Vectors: x (cols entries), y and z (rows entries) each with its own
// placement; z may be null.  x is staged in
// LDS; a thread owns rows r, r + BD, ... and streams its row of M column by
// column (consecutive threads read consecutive addresses), eight columns of
// loads in flight.
template <bool REAL, int BD>
__global__ __launch_bounds__(BD) void k_bgemv(const void* __restrict__ M, int rows, int cols,
                                              const double2* __restrict__ x, VecAt xa, const double2* z,
                                              VecAt za, double2* y, VecAt ya, double2 a0, double2 a1) {
  extern __shared__ double2 xs[];
  const int64_t tau = blockIdx.x, rhs = blockIdx.y;
  const double2* xv = x + rhs * xa.r + tau * xa.l + xa.o;
  for (int k = threadIdx.x; k < cols; k += BD) xs[k] = xv[k];
  __syncthreads();
  const int64_t yb = rhs * ya.r + tau * ya.l + ya.o;
  const int64_t zb = rhs * za.r + tau * za.l + za.o;
  constexpr int U = 8;
  for (int r = threadIdx.x; r < rows; r += BD) {
    double ar = 0.0, ai = 0.0;
    if constexpr (REAL) {
      const double* Mr = static_cast<const double*>(M) + r;
      int c = 0;
      for (; c + U <= cols; c += U) {
        double m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = Mr[(int64_t)(c + u) * rows];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double2 xv2 = xs[c + u];
          ar = fma(m[u], xv2.x, ar);
          ai = fma(m[u], xv2.y, ai);
        }
      }
      for (; c < cols; ++c) {
        const double mv = Mr[(int64_t)c * rows];
        ar = fma(mv, xs[c].x, ar);
        ai = fma(mv, xs[c].y, ai);
      }
    } else {
      const double2* Mc = static_cast<const double2*>(M) + tau * (int64_t)rows * cols + r;
      int c = 0;
      for (; c + U <= cols; c += U) {
        double2 m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) m[u] = ld_nt(Mc + (int64_t)(c + u) * rows);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double2 xv2 = xs[c + u];
          ar = fma(m[u].x, xv2.x, ar);
          ar = fma(-m[u].y, xv2.y, ar);
          ai = fma(m[u].x, xv2.y, ai);
          ai = fma(m[u].y, xv2.x, ai);
        }
      }
      for (; c < cols; ++c) {
        const double2 mv = ld_nt(Mc + (int64_t)c * rows);
        ar = fma(mv.x, xs[c].x, ar);
        ar = fma(-mv.y, xs[c].y, ar);
        ai = fma(mv.x, xs[c].y, ai);
        ai = fma(mv.y, xs[c].x, ai);
      }
    }
    double2 out = cmul(a1, make_double2(ar, ai));
    if (z) out = cadd(out, cmul(a0, z[zb + r]));
    y[yb + r] = out;
  }
}

// y = f + sgn * Pi g over face vectors; f is read at f + rhs * fr + tau * fl +
// fo (a face vector: fl = n_b, fo = 0; or the face rows of a volume vector:
// fl = n, fo = n_i) and may be null; g and y are face vectors [rhs][leaf][n_b].
__global__ void k_iti_exchange(const double2* __restrict__ f, int64_t fr, int64_t fl, int fo,
                               const double2* __restrict__ g, const int* __restrict__ nbr,
                               double2* __restrict__ y, int64_t nl, int nb, int L, double sgn,
                               int nrhs) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = nl * nb;
  if (gid >= per * nrhs) return;
  const int64_t rhs = gid / per;
  const int64_t k = gid - rhs * per;
  const int64_t tau = k / nb;
  const int rr = (int)(k - tau * nb);
  const int face = rr / L, pos = rr - face * L;
  double2 v = f ? f[rhs * fr + tau * fl + fo + rr] : make_double2(0.0, 0.0);
  const int t2 = nbr[tau * 6 + face];
  if (t2 >= 0) {
    const double2 gv = g[(rhs * nl + t2) * nb + (face ^ 1) * L + pos];
    v.x += sgn * gv.x;
    v.y += sgn * gv.y;
  }
  y[gid] = v;
}

// c = a - b elementwise
__global__ void k_sub(const double2* __restrict__ a, const double2* __restrict__ b,
                      double2* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = csub(a[i], b[i]);
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int bgemv_threads(int rows) { return std::min(1024, (rows + 63) / 64 * 64); }

template <bool REAL, int BD>
hipError_t bgemv_bd(hps_ctx* c, hipEvent_t e0, hipEvent_t e1, dim3 g, size_t lds, const void* M, int rows,
                    int cols, const double2* x, VecAt xa, const double2* z, VecAt za, double2* y, VecAt ya,
                    double2 a0, double2 a1) {
  return launch_k_lds(c, e0, e1, k_bgemv<REAL, BD>, g, dim3(BD), lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
}

template <bool REAL>
hipError_t bgemv_t(hps_ctx* c, hipEvent_t e0, hipEvent_t e1, const void* M, int rows, int cols,
                   const double2* x, VecAt xa, const double2* z, VecAt za, double2* y, VecAt ya, double2 a0,
                   double2 a1, int nrhs) {
  const dim3 g((unsigned)c->nl, (unsigned)nrhs);
  const size_t lds = sizeof(double2) * cols;
  switch (bgemv_threads(rows)) {
    case 64:  return bgemv_bd<REAL, 64>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 128: return bgemv_bd<REAL, 128>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 192: return bgemv_bd<REAL, 192>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 256: return bgemv_bd<REAL, 256>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 320: return bgemv_bd<REAL, 320>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 384: return bgemv_bd<REAL, 384>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 512: return bgemv_bd<REAL, 512>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 640: return bgemv_bd<REAL, 640>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    case 768: return bgemv_bd<REAL, 768>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
    default:  return bgemv_bd<REAL, 1024>(c, e0, e1, g, lds, M, rows, cols, x, xa, z, za, y, ya, a0, a1);
  }
}

// Workspace of the face-system solve, per right-hand side:
//   V [nl][ni]  A_ii^{-1} s_i        W [nl][nb]  F_bi V
//   H [nl][nb]  right-hand side of the face system, later f - W
//   Q [nl][ni]  A_ib u_b
struct ItiWs {
  double2 *V, *W, *H, *Q;
};

int iti_ws(hps_ctx* c, int nrhs, ItiWs* w) {
  const int64_t nv = c->nl * (int64_t)c->ni * nrhs, nf = c->nl * (int64_t)c->nb * nrhs;
  int rc = ws_reserve(c, &c->w_iti, sizeof(double2) * (2 * nv + 2 * nf));
  if (rc) return rc;
  double2* p = static_cast<double2*>(c->w_iti.ptr);
  w->V = p;
  w->W = p + nv;
  w->H = w->W + nf;
  w->Q = w->H + nf;
  return HPS_OK;
}

const double2 kOne = make_double2(1.0, 0.0), kZero = make_double2(0.0, 0.0);

}  // namespace

int64_t iti_ws_bytes(const hps_ctx* c, int nrhs) {
  return (int64_t)sizeof(double2) * (2 * c->nl * (int64_t)c->ni + 2 * c->nl * (int64_t)c->nb) * nrhs;
}

int iti_build(hps_ctx* c) {
  if (c->d_itiR) return HPS_OK;
  if (c->nop > 1) return fail(HPS_ERR_UNSUPPORTED, "the face-reduced system is not available for operator groups");
  const int ni = c->ni, nb = c->nb;
  const int64_t nl = c->nl;
  std::vector<double> Fbi, Nbb, Aib;
  build_face_operators(c->tab, &Fbi, &Nbb, &Aib);
  // complex copies for the setup GEMMs; F_bb = N_bb + i eta I
  std::vector<double2> Fbi_c(Fbi.size()), Aib_c(Aib.size()), Fbb_c(Nbb.size());
  for (size_t i = 0; i < Fbi.size(); ++i) Fbi_c[i] = make_double2(Fbi[i], 0.0);
  for (size_t i = 0; i < Aib.size(); ++i) Aib_c[i] = make_double2(Aib[i], 0.0);
  for (size_t i = 0; i < Nbb.size(); ++i) Fbb_c[i] = make_double2(Nbb[i], 0.0);
  for (int r = 0; r < nb; ++r) Fbb_c[(size_t)r * nb + r].y += c->eta;

  int rc;
  double2 *R = nullptr, *Ainv = nullptr;
  double *dFbi = nullptr, *dAib = nullptr;
  if ((rc = dev_alloc(c, (void**)&R, sizeof(double2) * nl * nb * nb))) return rc;
  if ((rc = dev_alloc(c, (void**)&Ainv, sizeof(double2) * nl * ni * ni))) {
    hipFree(R);
    c->dev_bytes -= sizeof(double2) * nl * nb * nb;
    return rc;
  }
  c->d_itiR = R;       // owned by the context from here (freed on error below or by hps_free)
  c->d_Ainv = Ainv;
  if ((rc = dev_alloc(c, (void**)&dFbi, sizeof(double) * Fbi.size()))) return rc;
  c->d_Fbi = dFbi;
  if ((rc = dev_alloc(c, (void**)&dAib, sizeof(double) * Aib.size()))) return rc;
  c->d_Aib = dAib;
  HPS_TRY_HIP(hipMemcpyAsync(dFbi, Fbi.data(), sizeof(double) * Fbi.size(), hipMemcpyHostToDevice, c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(dAib, Aib.data(), sizeof(double) * Aib.size(), hipMemcpyHostToDevice, c->stream));

  // temporaries: shared complex operands, and per chunk X = A_ii^{-1} A_ib and S
  const size_t per_leaf = sizeof(double2) * ((size_t)ni * nb + (size_t)nb * nb);
  int64_t chunk = std::max<int64_t>(1, (int64_t)((1ull << 30) / per_leaf));
  chunk = std::min(chunk, nl);
  double2 *dFbi_c = nullptr, *dAib_c = nullptr, *dFbb_c = nullptr, *X = nullptr, *S = nullptr;
  rocblas_int *ipiv = nullptr, *info = nullptr;
  auto cleanup = [&]() {
    hipFree(dFbi_c);
    hipFree(dAib_c);
    hipFree(dFbb_c);
    hipFree(X);
    hipFree(S);
    hipFree(ipiv);
    hipFree(info);
  };
  auto tmp = [&](void** p, size_t bytes) -> int {
    const hipError_t e = hipMalloc(p, bytes);
    return e == hipSuccess ? HPS_OK
                           : fail(e == hipErrorOutOfMemory ? HPS_ERR_OOM : HPS_ERR_DEVICE,
                                  "ItI setup: device allocation failed");
  };
  if ((rc = tmp((void**)&dFbi_c, sizeof(double2) * Fbi_c.size())) ||
      (rc = tmp((void**)&dAib_c, sizeof(double2) * Aib_c.size())) ||
      (rc = tmp((void**)&dFbb_c, sizeof(double2) * Fbb_c.size())) ||
      (rc = tmp((void**)&X, sizeof(double2) * (size_t)ni * nb * chunk)) ||
      (rc = tmp((void**)&S, sizeof(double2) * (size_t)nb * nb * chunk)) ||
      (rc = tmp((void**)&ipiv, sizeof(rocblas_int) * (size_t)std::max(ni, nb) * chunk)) ||
      (rc = tmp((void**)&info, sizeof(rocblas_int) * chunk))) {
    cleanup();
    return rc;
  }
  HPS_TRY_HIP(hipMemcpyAsync(dFbi_c, Fbi_c.data(), sizeof(double2) * Fbi_c.size(), hipMemcpyHostToDevice, c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(dAib_c, Aib_c.data(), sizeof(double2) * Aib_c.size(), hipMemcpyHostToDevice, c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(dFbb_c, Fbb_c.data(), sizeof(double2) * Fbb_c.size(), hipMemcpyHostToDevice, c->stream));
  rocblas_handle handle;
  if (rocblas_create_handle(&handle) != rocblas_status_success) {
    cleanup();
    return fail(HPS_ERR_DEVICE, "rocblas_create_handle failed");
  }
  rocblas_set_stream(handle, c->stream);
  std::vector<rocblas_int> hinfo(chunk);
  auto check_info = [&](int ne, int64_t e0, const char* what) -> int {
    HPS_TRY_HIP(hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * ne, hipMemcpyDeviceToHost, c->stream));
    HPS_TRY_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i < ne; ++i)
      if (hinfo[i] != 0)
        return fail(HPS_ERR_NUMERIC, std::string(what) + " of leaf " + std::to_string(e0 + i) + " is singular");
    return HPS_OK;
  };
  const rocblas_double_complex one{1.0, 0.0}, zero{0.0, 0.0}, mone{-1.0, 0.0};
  int status = HPS_OK;
  for (int64_t e0 = 0; e0 < nl && status == HPS_OK; e0 += chunk) {
    const int ne = (int)std::min<int64_t>(chunk, nl - e0);
    auto* A = reinterpret_cast<rocblas_double_complex*>(Ainv + e0 * (int64_t)ni * ni);
    const int64_t na = (int64_t)ni * ni * ne;
    hipLaunchKernelGGL(k_build_aii, dim3(blocks_for(na, 256)), dim3(256), 0, c->stream, c->d_tab + tab_off_D2(c->p),
                       c->p, c->n1, ni, c->d_C, c->c_complex, e0, ne, reinterpret_cast<double2*>(A));
    if ((status = check_hip(hipGetLastError(), "k_build_aii"))) break;
    if (rocsolver_zgetrf_strided_batched(handle, ni, ni, A, ni, (rocblas_stride)ni * ni, ipiv, ni, info, ne) !=
        rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocsolver getrf (A_ii) failed");
      break;
    }
    if ((status = check_info(ne, e0, "interior block A_ii"))) break;
    if (rocsolver_zgetri_strided_batched(handle, ni, A, ni, (rocblas_stride)ni * ni, ipiv, ni, info, ne) !=
        rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocsolver getri (A_ii) failed");
      break;
    }
    auto* Xc = reinterpret_cast<rocblas_double_complex*>(X);
    auto* Sc = reinterpret_cast<rocblas_double_complex*>(S);
    // X = A_ii^{-1} A_ib
    if (rocblas_zgemm_strided_batched(handle, rocblas_operation_none, rocblas_operation_none, ni, nb, ni, &one, A,
                                      ni, (rocblas_stride)ni * ni,
                                      reinterpret_cast<const rocblas_double_complex*>(dAib_c), ni, 0, &zero, Xc,
                                      ni, (rocblas_stride)ni * nb, ne) != rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocblas gemm (A_ii^-1 A_ib) failed");
      break;
    }
    // S = F_bb - F_bi X
    const int64_t ns = (int64_t)nb * nb * ne;
    hipLaunchKernelGGL(k_bcast, dim3(blocks_for(ns, 256)), dim3(256), 0, c->stream, dFbb_c, (int64_t)nb * nb, ne, S);
    if ((status = check_hip(hipGetLastError(), "k_bcast"))) break;
    if (rocblas_zgemm_strided_batched(handle, rocblas_operation_none, rocblas_operation_none, nb, nb, ni, &mone,
                                      reinterpret_cast<const rocblas_double_complex*>(dFbi_c), nb, 0, Xc, ni,
                                      (rocblas_stride)ni * nb, &one, Sc, nb, (rocblas_stride)nb * nb, ne) !=
        rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocblas gemm (F_bi X) failed");
      break;
    }
    if (rocsolver_zgetrf_strided_batched(handle, nb, nb, Sc, nb, (rocblas_stride)nb * nb, ipiv, nb, info, ne) !=
        rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocsolver getrf (S) failed");
      break;
    }
    if ((status = check_info(ne, e0, "Schur complement S"))) break;
    if (rocsolver_zgetri_strided_batched(handle, nb, Sc, nb, (rocblas_stride)nb * nb, ipiv, nb, info, ne) !=
        rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocsolver getri (S) failed");
      break;
    }
    hipLaunchKernelGGL(k_iti_pack, dim3(blocks_for(ns, 256)), dim3(256), 0, c->stream, S, nb, c->eta, e0, ne, R);
    if ((status = check_hip(hipGetLastError(), "k_iti_pack"))) break;
  }
  hipStreamSynchronize(c->stream);
  rocblas_destroy_handle(handle);
  cleanup();
  if (status) {
    hipFree(c->d_itiR);
    hipFree(c->d_Ainv);
    c->d_itiR = c->d_Ainv = nullptr;
    c->dev_bytes -= sizeof(double2) * nl * ((size_t)nb * nb + (size_t)ni * ni);
  }
  return status;
}

// y = f + Pi (R f)   (face vectors, nrhs of them)
int launch_iti_apply(hps_ctx* c, const double2* f, double2* y, int nrhs) {
  const int64_t nf = c->nl * (int64_t)c->nb;
  int rc = ws_reserve(c, &c->w_g, sizeof(double2) * nf * nrhs);
  if (rc) return rc;
  double2* g = static_cast<double2*>(c->w_g.ptr);
  TimedPair tp;
  if ((rc = timing_pair(c, 3, &tp))) return rc;
  const VecAt face{nf, c->nb, 0};
  hipError_t e = bgemv_t<false>(c, tp.start, tp.stop, c->d_itiR, c->nb, c->nb, f, face, nullptr, face, g, face,
                                kZero, kOne, nrhs);
  if ((rc = check_hip(e, "k_bgemv (R f)"))) {
    timing_drop(c, tp);
    return rc;
  }
  if ((rc = timing_commit(c, 3, tp))) return rc;
  const int64_t tot = nf * nrhs;
  hipLaunchKernelGGL(k_iti_exchange, dim3(blocks_for(tot, 256)), dim3(256), 0, c->stream, f, nf, (int64_t)c->nb, 0, g,
                     c->d_nbr, y, c->nl, c->nb, c->n1 * c->n1, 1.0, nrhs);
  return check_hip(hipGetLastError(), "k_iti_exchange");
}

// From the assembled volume right-hand side b (s_i at interior rows, t on the
// boundary faces): V = A_ii^{-1} s_i, W = F_bi V and, if rhs_f is given, the
// right-hand side t - Pi (W - R W) of the face system.
int iti_prepare(hps_ctx* c, const double2* b, int nrhs, double2* rhs_f) {
  ItiWs w;
  int rc = iti_ws(c, nrhs, &w);
  if (rc) return rc;
  const int ni = c->ni, nb = c->nb, n = c->n;
  const int64_t N = c->N, nf = c->nl * (int64_t)nb, nv = c->nl * (int64_t)ni;
  const VecAt vol_i{N, n, 0}, leaf_i{nv, ni, 0}, face{nf, nb, 0};
  HPS_TRY_HIP(bgemv_t<false>(c, nullptr, nullptr, c->d_Ainv, ni, ni, b, vol_i, nullptr, leaf_i, w.V, leaf_i,
                             kZero, kOne, nrhs));
  HPS_TRY_HIP(bgemv_t<true>(c, nullptr, nullptr, c->d_Fbi, nb, ni, w.V, leaf_i, nullptr, face, w.W, face, kZero,
                            kOne, nrhs));
  if (!rhs_f) return HPS_OK;
  // H = W - R W, then rhs_f = t - Pi H (b's face rows hold t on the boundary, 0 elsewhere)
  HPS_TRY_HIP(bgemv_t<false>(c, nullptr, nullptr, c->d_itiR, nb, nb, w.W, face, w.W, face, w.H, face, kOne,
                             make_double2(-1.0, 0.0), nrhs));
  const int64_t tot = nf * nrhs;
  hipLaunchKernelGGL(k_iti_exchange, dim3(blocks_for(tot, 256)), dim3(256), 0, c->stream, b, N, (int64_t)n, ni, w.H,
                     c->d_nbr, rhs_f, c->nl, nb, c->n1 * c->n1, -1.0, nrhs);
  return check_hip(hipGetLastError(), "k_iti_exchange (rhs)");
}

// u from the face solution f (V and W of iti_prepare in the workspace):
// u_b = (D - R D) / (2 i eta) with D = f - W, u_i = V - A_ii^{-1} (A_ib u_b).
int iti_finish(hps_ctx* c, const double2* f, double2* u, int nrhs) {
  ItiWs w;
  int rc = iti_ws(c, nrhs, &w);
  if (rc) return rc;
  const int ni = c->ni, nb = c->nb, n = c->n;
  const int64_t N = c->N, nf = c->nl * (int64_t)nb, nv = c->nl * (int64_t)ni;
  hipLaunchKernelGGL(k_sub, dim3(blocks_for(nf * nrhs, 256)), dim3(256), 0, c->stream, f, w.W, w.H, nf * nrhs);
  HPS_TRY_HIP(hipGetLastError());
  const double s = 1.0 / (2.0 * c->eta);   // 1 / (2 i eta) = -i s
  const VecAt vol_i{N, n, 0}, vol_b{N, n, ni}, leaf_i{nv, ni, 0}, face{nf, nb, 0};
  HPS_TRY_HIP(bgemv_t<false>(c, nullptr, nullptr, c->d_itiR, nb, nb, w.H, face, w.H, face, u, vol_b,
                             make_double2(0.0, -s), make_double2(0.0, s), nrhs));
  HPS_TRY_HIP(bgemv_t<true>(c, nullptr, nullptr, c->d_Aib, ni, nb, u, vol_b, nullptr, leaf_i, w.Q, leaf_i, kZero,
                            kOne, nrhs));
  HPS_TRY_HIP(bgemv_t<false>(c, nullptr, nullptr, c->d_Ainv, ni, ni, w.Q, leaf_i, w.V, leaf_i, u, vol_i, kOne,
                             make_double2(-1.0, 0.0), nrhs));
  return HPS_OK;
}

}  // namespace hps

using namespace hps;

extern "C" int hps_iti_build(hps_ctx* c) {
  if (!c) return fail(HPS_ERR_ARG, "hps_iti_build: ctx is NULL");
  return iti_build(c);
}

extern "C" int hps_iti_apply(hps_ctx* c, const hps_z* f, hps_z* y, int nrhs) {
  if (!c || !f || !y || nrhs < 1) return fail(HPS_ERR_ARG, "hps_iti_apply: bad arguments");
  if (!c->d_itiR) return fail(HPS_ERR_ARG, "hps_iti_apply: call hps_iti_build first");
  return launch_iti_apply(c, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(y), nrhs);
}

extern "C" int hps_iti_rhs(hps_ctx* c, const hps_z* s, const hps_z* t, hps_z* rhs_f, int nrhs) {
  if (!c || !s || !rhs_f || nrhs < 1) return fail(HPS_ERR_ARG, "hps_iti_rhs: bad arguments");
  if (!c->d_itiR) return fail(HPS_ERR_ARG, "hps_iti_rhs: call hps_iti_build first");
  int rc = ws_reserve(c, &c->w_b, sizeof(double2) * c->N * nrhs);
  if (rc) return rc;
  double2* b = static_cast<double2*>(c->w_b.ptr);
  if ((rc = launch_assemble_rhs(c, reinterpret_cast<const double2*>(s), reinterpret_cast<const double2*>(t), b,
                                nrhs)))
    return rc;
  return iti_prepare(c, b, nrhs, reinterpret_cast<double2*>(rhs_f));
}

extern "C" int hps_iti_recover(hps_ctx* c, const hps_z* s, const hps_z* t, const hps_z* f, hps_z* u, int nrhs) {
  if (!c || !s || !f || !u || nrhs < 1) return fail(HPS_ERR_ARG, "hps_iti_recover: bad arguments");
  if (!c->d_itiR) return fail(HPS_ERR_ARG, "hps_iti_recover: call hps_iti_build first");
  int rc = ws_reserve(c, &c->w_b, sizeof(double2) * c->N * nrhs);
  if (rc) return rc;
  double2* b = static_cast<double2*>(c->w_b.ptr);
  if ((rc = launch_assemble_rhs(c, reinterpret_cast<const double2*>(s), reinterpret_cast<const double2*>(t), b,
                                nrhs)))
    return rc;
  if ((rc = iti_prepare(c, b, nrhs, nullptr))) return rc;
  return iti_finish(c, reinterpret_cast<const double2*>(f), reinterpret_cast<double2*>(u), nrhs);
}

extern "C" int64_t hps_iti_bytes(int p, const int n_elem[3]) {
  if (p < kMinP || p > kMaxP || !n_elem || n_elem[0] < 1 || n_elem[1] < 1 || n_elem[2] < 1)
    return fail(HPS_ERR_ARG, "hps_iti_bytes: bad arguments");
  const int64_t n1 = p - 2, ni = n1 * n1 * n1, nb = 6 * n1 * n1;
  const int64_t nl = (int64_t)n_elem[0] * n_elem[1] * n_elem[2];
  return 16 * nl * (nb * nb + ni * ni) + 8 * 2 * ni * nb;
}
