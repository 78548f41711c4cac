// Host construction of the one-leaf tables (Sec. 2.1 and Sec. 4.1):
//   Chebyshev-Lobatto nodes and differentiation matrices on a leaf of side h,
//   the eigendecomposition L1 = V E V^{-1} of the interior second-derivative
//   block used by the fast diagonalization of the homogenized interior
//   operator, and the two real matrices P = F_bi (V x V x V) and
//   Q = (V x V x V)^{-1} A_ib that turn the homogenized Schur complement
//   S~ = F_bb - F_bi A~_ii^{-1} A_ib (eq. (schur_pc)) into
//   S~ = F_bb - P diag(1 / (-E_Delta - lambda)) Q for every leaf.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <numeric>

#include "hps_internal.h"

namespace hps {
namespace {

// Row-major dense helpers for tiny matrices.
using Mat = std::vector<double>;

// Differentiation matrix of the degree p-1 interpolant at the nodes x, from the
// barycentric form of the Lagrange basis: D_ij = (w_j / w_i) / (x_i - x_j) for
// i != j, with the diagonal set so that every row sums to zero (exact for
// constants).  Chebyshev-Lobatto weights: w_j = (-1)^j, halved at the ends.
Mat cheb_diff(const std::vector<double>& x) {
  const int p = (int)x.size();
  std::vector<double> w(p);
  for (int j = 0; j < p; ++j) w[j] = ((j & 1) ? -1.0 : 1.0) * ((j == 0 || j == p - 1) ? 0.5 : 1.0);
  Mat D(p * p, 0.0);
  for (int i = 0; i < p; ++i) {
    double s = 0.0;
    for (int j = 0; j < p; ++j) {
      if (j == i) continue;
      D[i * p + j] = (w[j] / w[i]) / (x[i] - x[j]);
      s += D[i * p + j];
    }
    D[i * p + i] = -s;
  }
  return D;
}

// LU with partial pivoting of an n x n row-major matrix, in place.
bool lu_factor(Mat& A, std::vector<int>& piv, int n) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int m = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[m * n + k])) m = i;
    piv[k] = m;
    if (A[m * n + k] == 0.0) return false;
    if (m != k)
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[m * n + j]);
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] /= A[k * n + k];
      const double f = A[i * n + k];
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
    }
  }
  return true;
}

void lu_solve(const Mat& LU, const std::vector<int>& piv, int n, std::vector<double>& b) {
  for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
    b[i] /= LU[i * n + i];
  }
}

// Eigenvalues of a real matrix whose spectrum is real: shifted QR iteration
// (Francis' basic algorithm with a Wilkinson shift taken from the trailing
// 2 x 2 block), deflating the last row of the active block once it vanishes.
// The QR factorization of each step is by Householder reflections.
bool real_eigenvalues(Mat A, int n, std::vector<double>& ev) {
  ev.clear();
  double anorm = 0.0;
  for (double v : A) anorm = std::max(anorm, std::fabs(v));
  int m = n;
  int iter = 0;
  while (m > 0) {
    if (m == 1) {
      ev.push_back(A[0]);
      break;
    }
    // deflation test on the last row of the active m x m block
    double off = 0.0;
    for (int j = 0; j < m - 1; ++j) off = std::max(off, std::fabs(A[(m - 1) * n + j]));
    if (off <= 1e-15 * anorm) {
      ev.push_back(A[(m - 1) * n + (m - 1)]);
      --m;
      iter = 0;
      continue;
    }
    if (++iter > 500) return false;
    // Wilkinson shift
    const double a = A[(m - 2) * n + (m - 2)], b = A[(m - 2) * n + (m - 1)];
    const double c = A[(m - 1) * n + (m - 2)], d = A[(m - 1) * n + (m - 1)];
    const double tr = 0.5 * (a - d);
    const double disc = tr * tr + b * c;
    double mu = d;
    if (disc >= 0.0) {
      const double r = std::sqrt(disc);
      const double l1 = d + tr + r, l2 = d + tr - r;  // eigenvalues of the 2x2 block
      mu = (std::fabs(l1 - d) < std::fabs(l2 - d)) ? l1 : l2;
    }
    if (iter % 11 == 10) mu += 0.5 * off;  // exceptional shift
    // B = A_m - mu I = Q R (Householder), A_m <- R Q + mu I
    Mat B(m * m), Qm(m * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) B[i * m + j] = A[i * n + j] - (i == j ? mu : 0.0);
    for (int i = 0; i < m; ++i) Qm[i * m + i] = 1.0;
    for (int k = 0; k < m - 1; ++k) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += B[i * m + k] * B[i * m + k];
      s = std::sqrt(s);
      if (s == 0.0) continue;
      std::vector<double> v(m, 0.0);
      const double alpha = B[k * m + k] > 0 ? -s : s;
      v[k] = B[k * m + k] - alpha;
      for (int i = k + 1; i < m; ++i) v[i] = B[i * m + k];
      double vv = 0.0;
      for (int i = k; i < m; ++i) vv += v[i] * v[i];
      if (vv == 0.0) continue;
      // B <- (I - 2 v v^T / vv) B ; Qm <- Qm (I - 2 v v^T / vv)
      for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int i = k; i < m; ++i) t += v[i] * B[i * m + j];
        t *= 2.0 / vv;
        for (int i = k; i < m; ++i) B[i * m + j] -= t * v[i];
      }
      for (int i = 0; i < m; ++i) {
        double t = 0.0;
        for (int j = k; j < m; ++j) t += Qm[i * m + j] * v[j];
        t *= 2.0 / vv;
        for (int j = k; j < m; ++j) Qm[i * m + j] -= t * v[j];
      }
    }
    // A_m = R Qm + mu I  (B now holds R)
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int k = i; k < m; ++k) t += B[i * m + k] * Qm[k * m + j];
        A[i * n + j] = t + (i == j ? mu : 0.0);
      }
  }
  return (int)ev.size() == n;
}

// Complex dense helpers (row major) for the separable form of the homogenized
// leaf solve.
using cd = std::complex<double>;
using CMat = std::vector<cd>;

bool clu_factor(CMat& A, std::vector<int>& piv, int n) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int m = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A[i * n + k]) > std::abs(A[m * n + k])) m = i;
    piv[k] = m;
    if (A[m * n + k] == 0.0) return false;
    if (m != k)
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[m * n + j]);
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] /= A[k * n + k];
      const cd f = A[i * n + k];
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
    }
  }
  return true;
}

void clu_solve(const CMat& LU, const std::vector<int>& piv, int n, std::vector<cd>& b) {
  for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
  for (int i = n - 1; i >= 0; --i) {
    for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
    b[i] /= LU[i * n + i];
  }
}

// Eigenvalues of a complex matrix: shifted QR iteration on the full matrix
// (complex Householder QR per step, Wilkinson shift from the trailing 2 x 2
// block, an exceptional shift every 11 steps without deflation), deflating the
// last row of the active block once it vanishes.
bool complex_eigenvalues(CMat A, int n, std::vector<cd>& ev) {
  ev.clear();
  double anorm = 0.0;
  for (const cd& v : A) anorm = std::max(anorm, std::abs(v));
  int m = n, iter = 0;
  while (m > 0) {
    if (m == 1) {
      ev.push_back(A[0]);
      break;
    }
    double off = 0.0;
    for (int j = 0; j < m - 1; ++j) off = std::max(off, std::abs(A[(m - 1) * n + j]));
    if (off <= 1e-15 * anorm) {
      ev.push_back(A[(m - 1) * n + (m - 1)]);
      --m;
      iter = 0;
      continue;
    }
    if (++iter > 500) return false;
    const cd a = A[(m - 2) * n + (m - 2)], b = A[(m - 2) * n + (m - 1)];
    const cd c = A[(m - 1) * n + (m - 2)], d = A[(m - 1) * n + (m - 1)];
    const cd tr = 0.5 * (a - d);
    const cd r = std::sqrt(tr * tr + b * c);
    const cd l1 = d + tr + r, l2 = d + tr - r;
    cd mu = (std::abs(l1 - d) < std::abs(l2 - d)) ? l1 : l2;
    if (iter % 11 == 10) mu += 0.5 * off;
    CMat B(m * m), Qm(m * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) B[i * m + j] = A[i * n + j] - (i == j ? mu : cd(0.0));
    for (int i = 0; i < m; ++i) Qm[i * m + i] = 1.0;
    for (int k = 0; k < m - 1; ++k) {
      double s = 0.0;
      for (int i = k; i < m; ++i) s += std::norm(B[i * m + k]);
      s = std::sqrt(s);
      if (s == 0.0) continue;
      const cd bkk = B[k * m + k];
      const cd ph = std::abs(bkk) > 0.0 ? bkk / std::abs(bkk) : cd(1.0);
      const cd alpha = -ph * s;
      std::vector<cd> v(m, 0.0);
      v[k] = bkk - alpha;
      for (int i = k + 1; i < m; ++i) v[i] = B[i * m + k];
      double vv = 0.0;
      for (int i = k; i < m; ++i) vv += std::norm(v[i]);
      if (vv == 0.0) continue;
      // B <- (I - 2 v v^H / vv) B ; Qm <- Qm (I - 2 v v^H / vv)
      for (int j = 0; j < m; ++j) {
        cd t = 0.0;
        for (int i = k; i < m; ++i) t += std::conj(v[i]) * B[i * m + j];
        t *= 2.0 / vv;
        for (int i = k; i < m; ++i) B[i * m + j] -= t * v[i];
      }
      for (int i = 0; i < m; ++i) {
        cd t = 0.0;
        for (int j = k; j < m; ++j) t += Qm[i * m + j] * v[j];
        t *= 2.0 / vv;
        for (int j = k; j < m; ++j) Qm[i * m + j] -= t * std::conj(v[j]);
      }
    }
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        cd t = 0.0;
        for (int k = i; k < m; ++k) t += B[i * m + k] * Qm[k * m + j];
        A[i * n + j] = t + (i == j ? mu : cd(0.0));
      }
  }
  return (int)ev.size() == n;
}

}  // namespace

std::string build_tables(int p, double h, HostTables* t) {
  if (p < kMinP || p > kMaxP) return "p out of range";
  const int n1 = p - 2;
  t->p = p;
  t->n1 = n1;
  t->ni = n1 * n1 * n1;
  t->nb = 6 * n1 * n1;
  t->n = t->ni + t->nb;
  t->h = h;
  t->xi.resize(p);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < p; ++j) t->xi[j] = -std::cos(pi * j / (p - 1));
  // exact symmetric values: the node set is symmetric about 0
  for (int j = 0; j < p / 2; ++j) t->xi[p - 1 - j] = -t->xi[j];
  if (p % 2) t->xi[p / 2] = 0.0;
  Mat D = cheb_diff(t->xi);
  const double sc = 2.0 / h;
  for (double& v : D) v *= sc;
  Mat D2(p * p, 0.0);
  for (int i = 0; i < p; ++i)
    for (int k = 0; k < p; ++k)
      for (int j = 0; j < p; ++j) D2[i * p + j] += D[i * p + k] * D[k * p + j];
  t->D = D;
  t->D2 = D2;

  // L1 = D2[1:p-1, 1:p-1] and its eigendecomposition
  Mat L1(n1 * n1);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) L1[i * n1 + j] = D2[(i + 1) * p + (j + 1)];
  std::vector<double> ev;
  if (!real_eigenvalues(L1, n1, ev)) return "eigenvalues of L1 did not converge";
  std::sort(ev.begin(), ev.end());
  double l1norm = 0.0;
  for (double v : L1) l1norm = std::max(l1norm, std::fabs(v));
  // eigenvectors by inverse iteration with a slightly perturbed shift
  Mat V(n1 * n1, 0.0);
  for (int k = 0; k < n1; ++k) {
    const double lam = ev[k];
    double gap = 1e300;
    for (int j = 0; j < n1; ++j)
      if (j != k) gap = std::min(gap, std::fabs(ev[j] - lam));
    const double shift = lam + 1e-10 * std::max(std::fabs(lam), 1.0);
    Mat M = L1;
    for (int i = 0; i < n1; ++i) M[i * n1 + i] -= shift;
    std::vector<int> piv;
    if (!lu_factor(M, piv, n1)) return "inverse iteration: singular shift";
    std::vector<double> x(n1);
    for (int i = 0; i < n1; ++i) x[i] = 1.0 + 0.1 * std::sin(1.7 * i + 0.3 * k);
    for (int it = 0; it < 4; ++it) {
      lu_solve(M, piv, n1, x);
      double nrm = 0.0;
      for (double v : x) nrm += v * v;
      nrm = std::sqrt(nrm);
      for (double& v : x) v /= nrm;
    }
    // sign convention: largest component positive
    int im = 0;
    for (int i = 1; i < n1; ++i)
      if (std::fabs(x[i]) > std::fabs(x[im])) im = i;
    if (x[im] < 0)
      for (double& v : x) v = -v;
    for (int i = 0; i < n1; ++i) V[i * n1 + k] = x[i];
    // residual check ||L1 v - lam v|| / ||L1||
    double r = 0.0;
    for (int i = 0; i < n1; ++i) {
      double s = -lam * x[i];
      for (int j = 0; j < n1; ++j) s += L1[i * n1 + j] * x[j];
      r = std::max(r, std::fabs(s));
    }
    if (r > 1e-9 * l1norm) return "eigenvector residual too large";
    (void)gap;
  }
  // W = V^{-1}
  Mat LU = V;
  std::vector<int> piv;
  if (!lu_factor(LU, piv, n1)) return "eigenvector matrix singular";
  Mat W(n1 * n1);
  for (int j = 0; j < n1; ++j) {
    std::vector<double> e(n1, 0.0);
    e[j] = 1.0;
    lu_solve(LU, piv, n1, e);
    for (int i = 0; i < n1; ++i) W[i * n1 + j] = e[i];
  }
  // reconstruction check ||V E W - L1||
  double rec = 0.0;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      double s = 0.0;
      for (int k = 0; k < n1; ++k) s += V[i * n1 + k] * ev[k] * W[k * n1 + j];
      rec = std::max(rec, std::fabs(s - L1[i * n1 + j]));
    }
  if (rec > 1e-9 * l1norm) return "eigendecomposition reconstruction error too large";
  t->V = V;
  t->W = W;
  t->E = ev;

  // P = F_bi (V x V x V): for a face node r on face f (axis ax, endpoint e,
  // sign sg, tangential coordinates (a, b)), F_bi[r, :] has sg * D[e][1 + i] at
  // the interior nodes of the normal line, so
  //   P[r, (al0, al1, al2)] = sg * dv_e[al_ax] * V[a][al_t1] * V[b][al_t2]
  // with dv_e[al] = sum_i D[e][1 + i] V[i][al].
  // Q = (W x W x W) A_ib: A_ib[m, r] = -D2[1 + i_ax(m)][e] on the same line, so
  //   Q[(al0, al1, al2), r] = -qv_e[al_ax] * W[al_t1][a] * W[al_t2][b]
  // with qv_e[al] = sum_i W[al][i] D2[1 + i][e].
  const int nb = t->nb, ni = t->ni, L = n1 * n1;
  t->P.assign((size_t)nb * ni, 0.0);
  t->Q.assign((size_t)ni * nb, 0.0);
  for (int f = 0; f < 6; ++f) {
    const int ax = face_axis(f);
    const int e = face_high(f) ? p - 1 : 0;
    const double sg = face_high(f) ? 1.0 : -1.0;
    int t1 = -1, t2 = -1;
    for (int a = 0; a < 3; ++a)
      if (a != ax) {
        if (t1 < 0) t1 = a; else t2 = a;
      }
    std::vector<double> dv(n1, 0.0), qv(n1, 0.0);
    for (int al = 0; al < n1; ++al)
      for (int i = 0; i < n1; ++i) {
        dv[al] += D[e * p + 1 + i] * V[i * n1 + al];
        qv[al] += W[al * n1 + i] * D2[(1 + i) * p + e];
      }
    for (int b = 0; b < n1; ++b)
      for (int a = 0; a < n1; ++a) {
        const int r = f * L + a + n1 * b;
        for (int g2 = 0; g2 < n1; ++g2)
          for (int g1 = 0; g1 < n1; ++g1)
            for (int g0 = 0; g0 < n1; ++g0) {
              const int al[3] = {g0, g1, g2};
              const int m = g0 + n1 * (g1 + n1 * g2);
              t->P[(size_t)r * ni + m] =
                  sg * dv[al[ax]] * V[a * n1 + al[t1]] * V[b * n1 + al[t2]];
              t->Q[(size_t)m * nb + r] =
                  -qv[al[ax]] * W[al[t1] * n1 + a] * W[al[t2] * n1 + b];
            }
      }
  }
  return std::string();
}

// The face rows and the interior-to-face coupling of the (exact) leaf matrix,
// which do not depend on the medium (C sits on the interior diagonal only):
//   F_bi (nb x ni): on face f (axis ax, endpoint e, outward sign sg) at
//     tangential position (a, b), sg * D[e][1 + i] at the interior node i of
//     the normal line through (a, b);
//   N_bb (nb x nb): the same derivative row at the two face nodes of that
//     line, sg * D[e][e] on the diagonal and sg * D[e][p-1-e] at the node of
//     the opposite face (F_bb = N_bb + i eta I);
//   A_ib (ni x nb): the interior row of node (i0, i1, i2) has -D2[1 + i_ax][e]
//     at the face node where its line along axis ax ends (endpoint e).
// All column-major (element (r, c) at c * rows + r).
void build_face_operators(const HostTables& t, std::vector<double>* Fbi, std::vector<double>* Nbb,
                          std::vector<double>* Aib) {
  const int p = t.p, n1 = t.n1, ni = t.ni, nb = t.nb, L = n1 * n1;
  Fbi->assign((size_t)nb * ni, 0.0);
  Nbb->assign((size_t)nb * nb, 0.0);
  Aib->assign((size_t)ni * nb, 0.0);
  for (int f = 0; f < 6; ++f) {
    const int ax = face_axis(f);
    const int e = face_high(f) ? p - 1 : 0;
    const double sg = face_high(f) ? 1.0 : -1.0;
    int t1 = -1, t2 = -1;
    for (int a = 0; a < 3; ++a)
      if (a != ax) {
        if (t1 < 0) t1 = a; else t2 = a;
      }
    for (int b = 0; b < n1; ++b)
      for (int a = 0; a < n1; ++a) {
        const int r = f * L + a + n1 * b;          // face node
        const int ro = (f ^ 1) * L + a + n1 * b;   // the other end of its normal line
        for (int i = 0; i < n1; ++i) {
          int g[3];
          g[ax] = i;
          g[t1] = a;
          g[t2] = b;
          const int m = g[0] + n1 * (g[1] + n1 * g[2]);
          (*Fbi)[(size_t)m * nb + r] = sg * t.D[e * p + 1 + i];
          (*Aib)[(size_t)r * ni + m] = -t.D2[(1 + i) * p + e];
        }
        (*Nbb)[(size_t)r * nb + r] += sg * t.D[e * p + e];
        (*Nbb)[(size_t)ro * nb + r] += sg * t.D[e * p + (p - 1 - e)];
      }
  }
}

// The separable form of the homogenized leaf solve.  The leaf matrix with
// C_ii = lambda I couples each node only along the three grid lines through
// it, and every face row (eq. (flux) plus i eta) lies on the normal line of its
// face node, whose two ends are face nodes of opposite faces.  Eliminating the
// two end values of every line with the 2 x 2 face system of that line,
//   [u_lo, u_hi] = Fi ([x_lo, x_hi] - Fbi1 u_line),
//   Fbb1 = [[-D00 + i eta, -D0e], [De0, Dee + i eta]] (e = p - 1), Fi = Fbb1^{-1},
//   Fbi1 = [-D[0][1:e]; D[e][1:e]],
// leaves on the interior the operator -(Lt x I x I + I x Lt x I + I x I x Lt) - lambda
// with Lt = D2[1:e, 1:e] - D2[1:e, {0, e}] Fi Fbi1, a complex n1 x n1 matrix.
// With Lt = Vc diag(Ec) Vc^{-1} the interior solve is a fast diagonalization
// as in Algorithm 3, now with complex factors.  Packed table (complex, row
// major): [Wc = Vc^{-1} | Vc | Ec | Fi]; for even n1 the modes are split into
// even and odd ones under the flip of a line (below).
std::string build_sep_table(const HostTables& t, double eta, std::vector<double>* out) {
  const int p = t.p, n1 = t.n1, e = p - 1;
  const std::vector<double>& D = t.D;
  const std::vector<double>& D2 = t.D2;
  const cd ie(0.0, eta);
  const cd f00 = -D[0] + ie, f01 = -D[e], f10 = D[e * p], f11 = D[e * p + e] + ie;
  const cd det = f00 * f11 - f01 * f10;
  if (std::abs(det) == 0.0) return "face system of a grid line is singular";
  const cd Fi[4] = {f11 / det, -f01 / det, -f10 / det, f00 / det};
  CMat Lt(n1 * n1);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      // D2[1 + i][{0, e}] Fi [-D[0][1 + j]; D[e][1 + j]]
      const cd g0 = Fi[0] * (-D[1 + j]) + Fi[1] * D[e * p + 1 + j];
      const cd g1 = Fi[2] * (-D[1 + j]) + Fi[3] * D[e * p + 1 + j];
      Lt[i * n1 + j] = D2[(1 + i) * p + 1 + j] - (D2[(1 + i) * p] * g0 + D2[(1 + i) * p + e] * g1);
    }
  double lnorm = 0.0;
  for (const cd& v : Lt) lnorm = std::max(lnorm, std::abs(v));
  // eigenpairs of an n x n complex matrix: eigenvalues sorted by real, then
  // imaginary part; eigenvectors (columns of X, row major) by inverse
  // iteration with a slightly perturbed shift, unit norm, largest component
  // real and positive
  auto eig = [&](const CMat& A, int n, std::vector<cd>& ev, CMat& X) -> std::string {
    if (!complex_eigenvalues(A, n, ev)) return "eigenvalues of the line operator did not converge";
    std::sort(ev.begin(), ev.end(), [](const cd& a, const cd& b) {
      return a.real() != b.real() ? a.real() < b.real() : a.imag() < b.imag();
    });
    X.assign((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
      const cd lam = ev[k];
      const cd shift = lam + 1e-10 * std::max(std::abs(lam), 1.0);
      CMat M = A;
      for (int i = 0; i < n; ++i) M[i * n + i] -= shift;
      std::vector<int> piv;
      if (!clu_factor(M, piv, n)) return "inverse iteration: singular shift";
      std::vector<cd> x(n);
      for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.1 * std::sin(1.7 * i + 0.3 * k);
      for (int it = 0; it < 4; ++it) {
        clu_solve(M, piv, n, x);
        double nrm = 0.0;
        for (const cd& v : x) nrm += std::norm(v);
        nrm = std::sqrt(nrm);
        for (cd& v : x) v /= nrm;
      }
      int im = 0;
      for (int i = 1; i < n; ++i)
        if (std::abs(x[i]) > std::abs(x[im])) im = i;
      const cd ph = std::abs(x[im]) / x[im];
      for (cd& v : x) v *= ph;
      double r = 0.0;
      for (int i = 0; i < n; ++i) {
        cd s = -lam * x[i];
        for (int j = 0; j < n; ++j) s += A[i * n + j] * x[j];
        r = std::max(r, std::abs(s));
      }
      if (r > 1e-9 * lnorm) return "line operator: eigenvector residual too large";
      for (int i = 0; i < n; ++i) X[i * n + k] = x[i];
    }
    return std::string();
  };
  auto inverse = [&](const CMat& A, int n, CMat& Ai) -> bool {
    CMat LU = A;
    std::vector<int> piv;
    if (!clu_factor(LU, piv, n)) return false;
    Ai.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
      std::vector<cd> col(n, 0.0);
      col[j] = 1.0;
      clu_solve(LU, piv, n, col);
      for (int i = 0; i < n; ++i) Ai[i * n + j] = col[i];
    }
    return true;
  };
  std::vector<cd> ev(n1);
  CMat V(n1 * n1, 0.0), W(n1 * n1, 0.0);
  if (n1 % 2 == 0) {
    // Lt commutes with the flip J (i <-> n1-1-i: the two faces of a line mirror
    // each other), so its eigenvectors are even ([y; J y]) or odd ([y; -J y]),
    // with y an eigenvector of Le = L11 + L12 J or Lo = L11 - L12 J (h x h,
    // h = n1 / 2).  Even modes come first, then odd ones; with
    // Ye = [y_e / sqrt 2], Yo likewise, Vc = [[Ye, Yo], [J Ye, -J Yo]] and
    // Wc = Vc^{-1} = [[Ye^{-1}, Ye^{-1} J], [Yo^{-1}, -Yo^{-1} J]] / 2 hold
    // the structure exactly, which the p = 12 kernel uses (each mode product
    // then takes half the multiplications).
    const int h = n1 / 2;
    double asym = 0.0;
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j)
        asym = std::max(asym, std::abs(Lt[i * n1 + j] - Lt[(n1 - 1 - i) * n1 + (n1 - 1 - j)]));
    if (asym > 1e-12 * lnorm) return "line operator: not symmetric under the flip of a line";
    for (int sgn = 0; sgn < 2; ++sgn) {
      const double s = sgn == 0 ? 1.0 : -1.0;
      CMat Lh((size_t)h * h);
      for (int i = 0; i < h; ++i)
        for (int j = 0; j < h; ++j) Lh[i * h + j] = Lt[i * n1 + j] + s * Lt[i * n1 + (n1 - 1 - j)];
      std::vector<cd> eh;
      CMat Y, Yi;
      std::string err = eig(Lh, h, eh, Y);
      if (!err.empty()) return err;
      for (cd& v : Y) v *= std::sqrt(0.5);
      if (!inverse(Y, h, Yi)) return "line operator: eigenvector matrix singular";
      for (int k = 0; k < h; ++k) {
        const int col = sgn * h + k;
        ev[col] = eh[k];
        for (int i = 0; i < h; ++i) {
          V[i * n1 + col] = Y[i * h + k];
          V[(n1 - 1 - i) * n1 + col] = s * Y[i * h + k];
          W[col * n1 + i] = 0.5 * Yi[k * h + i];
          W[col * n1 + (n1 - 1 - i)] = 0.5 * s * Yi[k * h + i];
        }
      }
    }
  } else {
    std::string err = eig(Lt, n1, ev, V);
    if (!err.empty()) return err;
    if (!inverse(V, n1, W)) return "line operator: eigenvector matrix singular";
  }
  double rec = 0.0;
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      cd s = 0.0;
      for (int k = 0; k < n1; ++k) s += V[i * n1 + k] * ev[k] * W[k * n1 + j];
      rec = std::max(rec, std::abs(s - Lt[i * n1 + j]));
    }
  if (rec > 1e-9 * lnorm) return "line operator: eigendecomposition reconstruction error too large";
  out->assign(2 * (size_t)sep_table_size(p), 0.0);
  auto put = [&](int k, cd v) {
    (*out)[2 * k] = v.real();
    (*out)[2 * k + 1] = v.imag();
  };
  const int Q = n1 * n1;
  for (int k = 0; k < Q; ++k) {
    put(k, W[k]);
    put(Q + k, V[k]);
  }
  for (int k = 0; k < n1; ++k) put(2 * Q + k, ev[k]);
  for (int k = 0; k < 4; ++k) put(2 * Q + n1 + k, Fi[k]);
  return std::string();
}

}  // namespace hps
