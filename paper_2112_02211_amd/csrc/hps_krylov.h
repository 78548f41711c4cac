// Device-resident state of the GMRES drivers and the batched Krylov launchers.
#pragma once

#include "hps_internal.h"

namespace hps {

constexpr int kMaxRestart = 200;  // largest Krylov dimension per cycle
constexpr int kMaxBatch = 64;     // right-hand sides iterated in lock step
constexpr int kRedBlocks = 1024;  // most workgroups of a reduction (one partial each)
constexpr int kPartSlots = 224;   // partial outputs per right-hand side (>= kMaxRestart + 1, KB-rounded)

// Hessenberg matrix (column major, leading dimension kMaxRestart + 1), Givens
// rotations, right-hand side g of the small least-squares problem, and the
// scalars one Arnoldi step exchanges between kernels.  One per right-hand side.
struct GmresState {
  double2 H[(kMaxRestart + 1) * kMaxRestart];
  double cs[kMaxRestart];
  double2 sn[kMaxRestart];
  double2 g[kMaxRestart + 1];
  double2 y[kMaxRestart];
  double2 h1[kMaxRestart + 1];
  double2 h2[kMaxRestart + 1];
  double nrm2;
  double beta;
  double res;
  int breakdown;
  int pad;
};

int launch_mdot_b(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K, const double2* w,
                  int64_t wbs, int64_t n, double2* out, int64_t obs, int nbatch, const RedBuf& rb);
int launch_mupdate_b(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K,
                     const double2* coef, int64_t cbs, double sign, double2* w, int64_t wbs,
                     int64_t n, double* nrm2, int64_t nstride, int nbatch, const RedBuf& rb);
// vectors stored in complex FP32: x += sign V coef, and squared norms (FP64 sums)
int launch_mupdate_b(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int K,
                     const double2* coef, int64_t cbs, double sign, float2* w, int64_t wbs,
                     int64_t n, double* nrm2, int64_t nstride, int nbatch, const RedBuf& rb);
int launch_norm2_b(hps_ctx* c, const float2* w, int64_t wbs, int64_t n, double* nrm2, int64_t nbs,
                   int nbatch, const RedBuf& rb);
// y = demote(s * x) (complex FP64 to FP32) and y += s * promote(x) (FP32 into FP64)
int launch_demote_scaled(hps_ctx* c, const double2* x, double s, float2* y, int64_t n);
int launch_axpy_promote(hps_ctx* c, double s, const float2* x, double2* y, int64_t n);
int launch_axpy_promote(hps_ctx* c, double s, const double2* x, double2* y, int64_t n);
int launch_norm2_b(hps_ctx* c, const double2* w, int64_t wbs, int64_t n, double* nrm2, int64_t nbs,
                   int nbatch, const RedBuf& rb);
int launch_scale_by_b(hps_ctx* c, const double2* x, int64_t xbs, double2* y, int64_t ybs, int64_t n,
                      const double* s, int64_t sstride, int inv_sqrt, int nbatch);
// One classical Gram-Schmidt pass against the K leading basis vectors:
// update == false: out = V^H w;  update == true: w -= V coef, then out = V^H w.
int launch_cgs_pass(hps_ctx* c, bool update, const double2* V, int64_t ldv, int64_t vbs, int K,
                    const double2* coef, int64_t cbs, double2* w, int64_t wbs, int64_t n,
                    double2* out, int64_t obs, int nbatch, const RedBuf& rb);
int launch_gm_start(hps_ctx* c, GmresState* S, int nb);
int launch_gm_givens(hps_ctx* c, GmresState* S, int nb, int j);
int launch_gm_collect(hps_ctx* c, const GmresState* S, int nb, double* out);
int launch_gm_trisolve(hps_ctx* c, GmresState* S, int nb, int k);

}  // namespace hps

namespace hps {

// ----------------------------------------------------------------------------
// Arnoldi with delayed reorthogonalization (two passes over the basis per step).
// At step j the basis V_0..V_{j-1} is orthonormal and u_j is the candidate for
// v_j after one projection.  The operator is applied to u_j itself (w = Op u_j);
// one reduction pass gives a = V^H u_j, b = V^H w, c = ||u_j||^2, d = u_j^H w;
// then beta = sqrt(c - ||a||^2), column j-1 of the Hessenberg matrix is
// (g_{j-1} + a, beta), v_j = (u_j - V a) / beta, and one update pass writes v_j
// and the next candidate u_{j+1} = (w - V b - v_j (d - a^H b) / beta) / beta.
// The projection of Op v_j on V_j, needed for column j, is
// g_j = ([b; (d - a^H b) / beta] - Hbar a) / beta.  With a flexible
// preconditioner the raw preconditioned candidates Z' are kept and the
// corrections accumulate in an upper triangular T with Z = Z' T.
constexpr int kMaxDcgs = 64;
constexpr int kDcgsLd = kMaxDcgs + 1;
constexpr int kSlotB = 64, kSlotC = 128, kSlotD = 129, kDcgsSlots = 130;

struct DcgsState {
  double2 H[kDcgsLd * kMaxDcgs];    // Hessenberg matrix as built (column major)
  double2 R[kDcgsLd * kMaxDcgs];    // its Givens-rotated copy
  double2 T[kMaxDcgs * kMaxDcgs];   // flexible: Z = Z' T (column major, upper triangular)
  double2 red[kDcgsSlots];          // finished reductions: a | b | c | d
  double cs[kMaxDcgs];
  double2 sn[kMaxDcgs];
  double2 gls[kDcgsLd];             // right-hand side of the small least-squares problem
  double2 gprev[kDcgsLd];           // projection of the last operator image (next column)
  double2 y[kMaxDcgs];
  double2 rc[kDcgsLd];              // restart: the new residual's coefficients over V
  double2 rsig;                     // ... and over the last candidate u
  double beta0;
  double res;
  int flag;                         // nonzero: the candidate fell into the basis (stop the cycle)
  int ncols;                        // finished Hessenberg columns
  int rk;                           // restart: basis vectors the new residual combines
};

// The update pass of the last step J of a cycle (long vectors, J <= 12: see
// dcgs_can_close) with the cycle's closing reduction folded in: S[b].red gets
// a_k (k <= J) and c of the new candidate, as launch_dcgs_reduce over the
// J + 1 basis vectors and u without w would give them.
bool dcgs_can_close(int J, int64_t n);
int launch_dcgs_update_close(hps_ctx* c, double2* V, int64_t ldv, int64_t vbs, int J, double2* u,
                             int64_t ubs, const double2* w, int64_t wbs, int64_t n, DcgsState* S,
                             int nbatch, int flexible, double* res_out, uint64_t tag, const RedBuf& rb);
int launch_dcgs_update_close(hps_ctx* c, float2* V, int64_t ldv, int64_t vbs, int J, float2* u,
                             int64_t ubs, const float2* w, int64_t wbs, int64_t n, DcgsState* S,
                             int nbatch, int flexible, double* res_out, uint64_t tag, const RedBuf& rb);
// reduction pass: partials of a, b (j basis vectors), c, d, finished into S[b].red
int launch_dcgs_reduce(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int J,
                       const double2* u, int64_t ubs, const double2* w, int64_t wbs, int64_t n,
                       DcgsState* S, int nbatch, const RedBuf& rb);
// the same over vectors stored in complex FP32 (sums in FP64)
int launch_dcgs_reduce(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int J,
                       const float2* u, int64_t ubs, const float2* w, int64_t wbs, int64_t n,
                       DcgsState* S, int nbatch, const RedBuf& rb);
// standalone small step (one workgroup per right-hand side); final_only: only close column j-1
int launch_dcgs_small(hps_ctx* c, DcgsState* S, int nbatch, int j, int flexible, int final_only,
                      double* res_out, uint64_t tag);
// update pass: V[J] = v_j, u <- u_{j+1}
// update pass of step J (writes V[J] and the next candidate); its workgroup 0 per
// right-hand side also runs the small step of J and writes the record
// res_out[4 r .. 4 r + 2] = {estimate, stopped, tag} (tag last, system-scope
// release; res_out may be pinned host memory)
int launch_dcgs_update(hps_ctx* c, double2* V, int64_t ldv, int64_t vbs, int J, double2* u,
                       int64_t ubs, const double2* w, int64_t wbs, int64_t n, DcgsState* S,
                       int nbatch, int flexible, double* res_out, uint64_t tag);
int launch_dcgs_update(hps_ctx* c, float2* V, int64_t ldv, int64_t vbs, int J, float2* u,
                       int64_t ubs, const float2* w, int64_t wbs, int64_t n, DcgsState* S,
                       int nbatch, int flexible, double* res_out, uint64_t tag);
int launch_dcgs_start(hps_ctx* c, DcgsState* S, int nbatch);
// y = R^{-1} gls over the finished columns (at most kmax); flexible: y <- T y
int launch_dcgs_trisolve(hps_ctx* c, DcgsState* S, int nbatch, int kmax, int flexible);
// Restart of left GMRES without applying the operator: after trisolve, with k
// finished columns and K written basis vectors, the residual of the updated
// iterate is r' = r - Op V_k y = V_{k+1} (beta0 e_0 - Hbar_k y) (Arnoldi
// relation).  When the last column was closed (k = K), v_K = (u - V_K a)/beta
// is not stored and r' = V_K (beta0 e_0 - H_K y + a y_{k-1}) - y_{k-1} u; after
// an early stop (k < K) v_k is V[k].  The coefficients go to S.rc / S.rsig.
int launch_dcgs_restart_coef(hps_ctx* c, DcgsState* S, int nbatch, int K);
// One pass over V[0..K-1]: x += V y and u <- V rc + rsig u (the next cycle's
// first candidate), per right-hand side.
int launch_dcgs_restart(hps_ctx* c, const double2* V, int64_t ldv, int64_t vbs, int K, double2* u,
                        int64_t ubs, double2* x, int64_t xbs, int64_t n, DcgsState* S, int nbatch);
int launch_dcgs_restart(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int K, float2* u,
                        int64_t ubs, float2* x, int64_t xbs, int64_t n, DcgsState* S, int nbatch);
// the same with the iterate x in FP64 over an FP32 basis
int launch_dcgs_restart(hps_ctx* c, const float2* V, int64_t ldv, int64_t vbs, int K, float2* u,
                        int64_t ubs, double2* x, int64_t xbs, int64_t n, DcgsState* S, int nbatch);

}  // namespace hps
