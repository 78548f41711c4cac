// Block GMRES(m) for k right-hand sides at once (many right-hand sides in one
// Krylov space): left preconditioned with the FP64 J^{-1} (stored blocks or the
// separable form), on J^{-1} A X = J^{-1} B.  Block Arnoldi with classical
// Gram-Schmidt twice against all previous blocks and CholQR2 for the new
// block; the block least-squares problem is kept triangular by Householder
// reflections on the host.  Each right-hand side stops on its own PCRR
// ||J^{-1}(b - A x)|| <= tol ||J^{-1} b|| (the block iterates until all have).
//
// Device work is the operator on k columns (hps_op_left's kernels) and
// rocBLAS GEMMs on the tall-skinny blocks: H = V^H W, W -= V H, the k x k Gram
// matrix W^H W, W R^{-1}, X += V Y.  Host work is O(m k^3) per step.
#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "hps_internal.h"

namespace hps {
namespace {

using cd = std::complex<double>;

struct Blas {
  rocblas_handle h = nullptr;
  ~Blas() {
    if (h) rocblas_destroy_handle(h);
  }
};

int blas_ok(rocblas_status s, const char* what) {
  return s == rocblas_status_success ? HPS_OK : fail(HPS_ERR_DEVICE, std::string(what) + " failed");
}

// C (m x n, ldc) = alpha op(A) op(B) + beta C, column major, complex.
int zgemm(rocblas_handle h, bool ca, int m, int n, int64_t kk, cd alpha, const double2* A, int64_t lda,
          const double2* B, int64_t ldb, cd beta, double2* C, int64_t ldc) {
  const rocblas_double_complex al(alpha.real(), alpha.imag()), be(beta.real(), beta.imag());
  return blas_ok(rocblas_zgemm(h, ca ? rocblas_operation_conjugate_transpose : rocblas_operation_none,
                               rocblas_operation_none, m, n, (rocblas_int)kk, &al,
                               reinterpret_cast<const rocblas_double_complex*>(A), (rocblas_int)lda,
                               reinterpret_cast<const rocblas_double_complex*>(B), (rocblas_int)ldb, &be,
                               reinterpret_cast<rocblas_double_complex*>(C), (rocblas_int)ldc),
                 "rocblas_zgemm");
}

// Split-K scratch: partial products of C = A^H B over chunks of the long
// dimension (the product's m x n tiles are too few to fill the GPU), summed by
// a matrix-vector product with a vector of ones.
struct SplitK {
  static constexpr int kChunks = 256;
  double2* part = nullptr;   // kChunks + 1 partial m x n products
  double2* ones = nullptr;   // kChunks + 1 ones
  int64_t cap = 0;           // entries of one partial
};

// C (m x n) = A^H B with A (K x m, lda), B (K x n, ldb), K long.
int zgemm_ct(rocblas_handle h, int m, int n, int64_t K, const double2* A, int64_t lda, const double2* B,
             int64_t ldb, double2* C, const SplitK& sk) {
  const int64_t L = (K + SplitK::kChunks - 1) / SplitK::kChunks;
  const int full = (int)(K / L);
  const int64_t rest = K - (int64_t)full * L;
  if ((int64_t)m * n > sk.cap || L < 4096) return zgemm(h, true, m, n, K, 1.0, A, lda, B, ldb, 0.0, C, m);
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  if (rocblas_zgemm_strided_batched(
          h, rocblas_operation_conjugate_transpose, rocblas_operation_none, m, n, (rocblas_int)L, &one,
          reinterpret_cast<const rocblas_double_complex*>(A), (rocblas_int)lda, L,
          reinterpret_cast<const rocblas_double_complex*>(B), (rocblas_int)ldb, L, &zero,
          reinterpret_cast<rocblas_double_complex*>(sk.part), m, (rocblas_stride)m * n, full) !=
      rocblas_status_success)
    return fail(HPS_ERR_DEVICE, "rocblas_zgemm_strided_batched failed");
  int nparts = full;
  if (rest > 0) {
    int rc = zgemm(h, true, m, n, rest, 1.0, A + (int64_t)full * L, lda, B + (int64_t)full * L, ldb, 0.0,
                   sk.part + (int64_t)full * m * n, m);
    if (rc) return rc;
    ++nparts;
  }
  return blas_ok(rocblas_zgemv(h, rocblas_operation_none, m * n, nparts, &one,
                               reinterpret_cast<const rocblas_double_complex*>(sk.part), m * n,
                               reinterpret_cast<const rocblas_double_complex*>(sk.ones), 1, &zero,
                               reinterpret_cast<rocblas_double_complex*>(C), 1),
                 "rocblas_zgemv");
}

// Gram matrix G = X^H X (k x k) of the k columns of X (N x k), on the host.
int gram(hps_ctx* c, rocblas_handle h, const double2* X, int64_t N, int k, double2* dG,
         std::vector<cd>& G, const SplitK& sk) {
  int rc = zgemm_ct(h, k, k, N, X, N, X, N, dG, sk);
  if (rc) return rc;
  G.resize((size_t)k * k);
  HPS_TRY_HIP(hipMemcpyAsync(G.data(), dG, sizeof(double2) * k * k, hipMemcpyDeviceToHost, c->stream));
  HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  return HPS_OK;
}

// Cholesky G = R^H R (R upper, column major k x k); false if not positive definite.
bool cholesky(const std::vector<cd>& G, int k, std::vector<cd>& R) {
  R.assign((size_t)k * k, 0.0);
  double gmax = 0.0;
  for (int i = 0; i < k; ++i) gmax = std::max(gmax, G[i + (size_t)k * i].real());
  for (int j = 0; j < k; ++j) {
    cd s = G[j + (size_t)k * j];
    for (int l = 0; l < j; ++l) s -= std::conj(R[l + (size_t)k * j]) * R[l + (size_t)k * j];
    if (!(s.real() > 1e-28 * gmax)) return false;
    const double d = std::sqrt(s.real());
    R[j + (size_t)k * j] = d;
    for (int i = j + 1; i < k; ++i) {
      cd t = G[j + (size_t)k * i];
      for (int l = 0; l < j; ++l) t -= std::conj(R[l + (size_t)k * j]) * R[l + (size_t)k * i];
      R[j + (size_t)k * i] = t / d;
    }
  }
  return true;
}

// Inverse of an upper triangular k x k matrix (column major).
std::vector<cd> tri_inverse(const std::vector<cd>& R, int k) {
  std::vector<cd> X((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    X[j + (size_t)k * j] = 1.0 / R[j + (size_t)k * j];
    for (int i = j - 1; i >= 0; --i) {
      cd s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += R[i + (size_t)k * l] * X[l + (size_t)k * j];
      X[i + (size_t)k * j] = -s / R[i + (size_t)k * i];
    }
  }
  return X;
}

// R2 R1 for upper triangular k x k factors.
std::vector<cd> tri_mul(const std::vector<cd>& A, const std::vector<cd>& B, int k) {
  std::vector<cd> C((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j; ++i) {
      cd s = 0.0;
      for (int l = i; l <= j; ++l) s += A[i + (size_t)k * l] * B[l + (size_t)k * j];
      C[i + (size_t)k * j] = s;
    }
  return C;
}

// CholQR2: Q R = X (N x k) with Q written to dst, R (upper) returned; tmp is a
// second N x k buffer.  HPS_ERR_BREAKDOWN when the columns are (numerically)
// dependent.
int cholqr2(hps_ctx* c, rocblas_handle h, const double2* X, double2* tmp, double2* dst, int64_t N,
            int k, double2* dG, std::vector<cd>& R, const SplitK& sk) {
  std::vector<cd> G, R1, R2;
  const double2* src = X;
  double2* outs[2] = {tmp, dst};
  for (int pass = 0; pass < 2; ++pass) {
    int rc = gram(c, h, src, N, k, dG, G, sk);
    if (rc) return rc;
    std::vector<cd>& Rp = pass ? R2 : R1;
    // Cholesky of the column-equilibrated Gram matrix D^-1 G D^-1 (D = its
    // column norms), R = Rs D: columns of very different length (converged and
    // unconverged right-hand sides in a restart residual) stay well conditioned
    std::vector<double> dn(k);
    for (int i = 0; i < k; ++i) dn[i] = std::sqrt(std::max(G[i + (size_t)k * i].real(), 0.0));
    bool ok = true;
    for (int i = 0; i < k; ++i) ok = ok && dn[i] > 0.0;
    if (ok) {
      for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) G[i + (size_t)k * j] /= dn[i] * dn[j];
      ok = cholesky(G, k, Rp);
    }
    if (!ok)
      return fail(HPS_ERR_BREAKDOWN,
                  "block GMRES: the block's columns are linearly dependent (use the lock-step solver)");
    for (int j = 0; j < k; ++j)
      for (int i = 0; i <= j; ++i) Rp[i + (size_t)k * j] *= dn[j];
    const std::vector<cd> Ri = tri_inverse(Rp, k);
    HPS_TRY_HIP(hipMemcpyAsync(dG, Ri.data(), sizeof(double2) * k * k, hipMemcpyHostToDevice, c->stream));
    if ((rc = zgemm(h, false, (int)N, k, k, 1.0, src, N, dG, k, 0.0, outs[pass], N))) return rc;
    src = outs[pass];
  }
  R = tri_mul(R2, R1, k);
  return HPS_OK;
}

// Householder reflector of x (length n) so that (I - tau v v^H) x = alpha e_1.
void householder(std::vector<cd>& x, cd& tau, cd& alpha) {
  double nrm = 0.0;
  for (const cd& v : x) nrm += std::norm(v);
  nrm = std::sqrt(nrm);
  if (nrm == 0.0) {
    tau = 0.0;
    alpha = 0.0;
    return;
  }
  const cd x0 = x[0];
  const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0);
  alpha = -ph * nrm;
  x[0] = x0 - alpha;
  double vv = 0.0;
  for (const cd& v : x) vv += std::norm(v);
  tau = 2.0 / vv;
}

}  // namespace

int run_block_gmres(hps_ctx* c, int prec, const double2* b, double2* x, int k, double tol, int m,
                    int maxit, bool use_x0, double* rhs_res, hps_stats* st) {
  const double t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  const int64_t N = c->N;
  const int64_t nk = N * k;
  const int K = (m + 1) * k;   // rows of the block Hessenberg matrix
  // workspace: basis V ((m+1) k columns), W, TMP, PB = J^-1 B, small matrices
  const int64_t pcap = (int64_t)m * k * k;   // largest partial: (m k) x k
  const size_t bytes = sizeof(double2) * ((size_t)nk * (m + 1) + 3 * (size_t)nk) +
                       sizeof(double2) * ((size_t)K * k + 64) +
                       sizeof(double2) * ((size_t)(SplitK::kChunks + 1) * (pcap + 1));
  int rc = ws_reserve(c, &c->w_krylov, bytes);
  if (rc) return rc;
  double2* V = static_cast<double2*>(c->w_krylov.ptr);
  double2* W = V + (size_t)nk * (m + 1);
  double2* TMP = W + nk;
  double2* PB = TMP + nk;
  double2* dS = PB + nk;   // K x k small matrices (H column blocks, Y, R^-1)
  SplitK sk;
  sk.part = dS + (size_t)K * k + 64;
  sk.ones = sk.part + (size_t)(SplitK::kChunks + 1) * pcap;
  sk.cap = pcap;
  {
    std::vector<double2> ones(SplitK::kChunks + 1, make_double2(1.0, 0.0));
    HPS_TRY_HIP(hipMemcpyAsync(sk.ones, ones.data(), sizeof(double2) * ones.size(), hipMemcpyHostToDevice,
                               c->stream));
    HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  }
  Blas bl;
  if (rocblas_create_handle(&bl.h) != rocblas_status_success)
    return fail(HPS_ERR_DEVICE, "rocblas_create_handle failed");
  rocblas_set_stream(bl.h, c->stream);

  // J^-1 B and its column norms
  if ((rc = launch_precond(c, b, PB, k, prec))) return rc;
  std::vector<cd> G;
  if ((rc = gram(c, bl.h, PB, N, k, dS, G, sk))) return rc;
  std::vector<double> bnorm(k), res(k, 0.0), est(k, 0.0);
  for (int r = 0; r < k; ++r) bnorm[r] = std::sqrt(std::max(0.0, G[r + (size_t)k * r].real()));
  int its = 0, restarts = 0;
  bool all_done = false;
  // residual R = J^-1 (B - A X) into W and its column norms
  auto residual = [&](bool zero_x) -> int {
    int e;
    if (zero_x) {
      HPS_TRY_HIP(hipMemcpyAsync(W, PB, sizeof(double2) * nk, hipMemcpyDeviceToDevice, c->stream));
    } else {
      if ((e = launch_op_left(c, x, TMP, W, k, prec))) return e;
      if ((e = launch_sub_from(c, PB, W, nk))) return e;   // W = PB - W
    }
    if ((e = gram(c, bl.h, W, N, k, dS, G, sk))) return e;
    all_done = true;
    for (int r = 0; r < k; ++r) {
      res[r] = bnorm[r] > 0 ? std::sqrt(std::max(0.0, G[r + (size_t)k * r].real())) / bnorm[r] : 0.0;
      if (res[r] > tol) all_done = false;
    }
    return HPS_OK;
  };
  if (!use_x0) HPS_TRY_HIP(hipMemsetAsync(x, 0, sizeof(double2) * nk, c->stream));
  if ((rc = residual(!use_x0))) return rc;
  while (!all_done && its < maxit) {
    // V_0 R_0 = R
    std::vector<cd> R0;
    if ((rc = cholqr2(c, bl.h, W, TMP, V, N, k, dS, R0, sk))) return rc;
    // host: block Hessenberg H (K x m k, column major), right-hand side S (K x k)
    std::vector<cd> H((size_t)K * m * k, 0.0), S((size_t)K * k, 0.0);
    for (int j = 0; j < k; ++j)
      for (int i = 0; i <= j; ++i) S[i + (size_t)K * j] = R0[i + (size_t)k * j];
    std::vector<std::vector<cd>> hv;    // Householder vectors (length 2k) per column
    std::vector<cd> htau;
    int steps = 0;
    for (int j = 0; j < m && its < maxit; ++j) {
      double2* Vj = V + (size_t)nk * j;
      // W = J^-1 A V_j
      if ((rc = launch_op_left(c, Vj, TMP, W, k, prec))) return rc;
      // classical Gram-Schmidt twice against V_0 .. V_j (all (j+1) k columns)
      const int cols = (j + 1) * k;
      std::vector<cd> hc((size_t)cols * k, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        if ((rc = zgemm_ct(bl.h, cols, k, N, V, N, W, N, dS, sk))) return rc;
        std::vector<cd> part((size_t)cols * k);
        HPS_TRY_HIP(hipMemcpyAsync(part.data(), dS, sizeof(double2) * cols * k, hipMemcpyDeviceToHost,
                                   c->stream));
        if ((rc = zgemm(bl.h, false, (int)N, k, cols, -1.0, V, N, dS, cols, 1.0, W, N))) return rc;
        HPS_TRY_HIP(hipStreamSynchronize(c->stream));
        for (size_t q = 0; q < part.size(); ++q) hc[q] += part[q];
      }
      // V_{j+1} R_{j+1} = W
      std::vector<cd> Rn;
      if ((rc = cholqr2(c, bl.h, W, TMP, V + (size_t)nk * (j + 1), N, k, dS, Rn, sk))) return rc;
      // block column j of H: rows 0 .. (j+1)k from hc, rows (j+1)k .. (j+2)k from Rn
      for (int cc = 0; cc < k; ++cc) {
        cd* col = &H[(size_t)K * (j * k + cc)];
        for (int i = 0; i < cols; ++i) col[i] = hc[i + (size_t)cols * cc];
        for (int i = 0; i <= cc; ++i) col[cols + i] = Rn[i + (size_t)k * cc];
      }
      // the reflectors of earlier block columns (reflector q acts on rows
      // q .. q + len_q - 1, len_q = its vector's length), then k new ones on
      // rows j k .. (j+2) k - 1, each applied to the rest of this block column
      // and to the right-hand side block S
      const size_t nprev = hv.size();   // = j k
      for (int cc = 0; cc < k; ++cc) {
        cd* col = &H[(size_t)K * (j * k + cc)];
        for (size_t q = 0; q < nprev; ++q) {
          const std::vector<cd>& v = hv[q];
          cd s = 0.0;
          for (size_t t = 0; t < v.size(); ++t) s += std::conj(v[t]) * col[q + t];
          s *= htau[q];
          for (size_t t = 0; t < v.size(); ++t) col[q + t] -= s * v[t];
        }
      }
      for (int cc = 0; cc < k; ++cc) {
        cd* col = &H[(size_t)K * (j * k + cc)];
        const int r0 = j * k + cc, len = (j + 2) * k - r0;
        std::vector<cd> v(col + r0, col + r0 + len);
        cd tau, alpha;
        householder(v, tau, alpha);
        col[r0] = alpha;
        for (int t = 1; t < len; ++t) col[r0 + t] = 0.0;
        for (int c2 = cc + 1; c2 < k; ++c2) {
          cd* col2 = &H[(size_t)K * (j * k + c2)];
          cd s = 0.0;
          for (int t = 0; t < len; ++t) s += std::conj(v[t]) * col2[r0 + t];
          s *= tau;
          for (int t = 0; t < len; ++t) col2[r0 + t] -= s * v[t];
        }
        for (int c2 = 0; c2 < k; ++c2) {
          cd* sc = &S[(size_t)K * c2];
          cd s = 0.0;
          for (int t = 0; t < len; ++t) s += std::conj(v[t]) * sc[r0 + t];
          s *= tau;
          for (int t = 0; t < len; ++t) sc[r0 + t] -= s * v[t];
        }
        hv.push_back(std::move(v));
        htau.push_back(tau);
      }
      ++its;
      steps = j + 1;
      // residual estimate per right-hand side: rows (j+1) k .. (j+2) k of S
      bool done = true;
      for (int r = 0; r < k; ++r) {
        double s2 = 0.0;
        for (int i = cols; i < cols + k; ++i) s2 += std::norm(S[i + (size_t)K * r]);
        est[r] = bnorm[r] > 0 ? std::sqrt(s2) / bnorm[r] : 0.0;
        if (est[r] > tol) done = false;
      }
      if (done) break;
    }
    // Y = T^{-1} S (T the (steps k) upper triangle of the rotated H), X += V Y
    const int n = steps * k;
    std::vector<cd> Y((size_t)n * k, 0.0);
    for (int r = 0; r < k; ++r)
      for (int i = n - 1; i >= 0; --i) {
        cd s = S[i + (size_t)K * r];
        for (int l = i + 1; l < n; ++l) s -= H[i + (size_t)K * l] * Y[l + (size_t)n * r];
        Y[i + (size_t)n * r] = s / H[i + (size_t)K * i];
      }
    HPS_TRY_HIP(hipMemcpyAsync(dS, Y.data(), sizeof(double2) * n * k, hipMemcpyHostToDevice, c->stream));
    if ((rc = zgemm(bl.h, false, (int)N, k, n, 1.0, V, N, dS, n, 1.0, x, N))) return rc;
    ++restarts;
    if ((rc = residual(false))) return rc;
  }
  HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  if (rhs_res)
    for (int r = 0; r < k; ++r) rhs_res[r] = res[r];
  if (st) {
    double we = 0.0, wt = 0.0;
    for (int r = 0; r < k; ++r) {
      we = std::max(we, est[r]);
      wt = std::max(wt, res[r]);
    }
    st->iters = its;
    st->restarts = restarts;
    st->converged = all_done ? 1 : 0;
    st->lambda_shifted = c->n_shifted;
    st->t_setup = c->t_setup;
    st->rel_res = we;
    st->true_rel_res = wt;
    st->t_solve = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
  }
  return all_done ? HPS_OK : HPS_NOT_CONVERGED;
}

}  // namespace hps
