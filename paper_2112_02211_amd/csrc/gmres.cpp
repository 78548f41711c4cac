// GMRES drivers for A u = b (Sec. 4, eq. (globalsystem); Sec. 5.2 uses a
// restarted GMRES with matrix-free operator and preconditioner shells).
//
//  * left preconditioned GMRES(m) on J^{-1} A x = J^{-1} b in FP64, stopping on
//    the preconditioned residual reduction ||J^{-1}(b - A x)|| <= tol ||J^{-1} b||
//    (the PCRR of Sec. 6), x0 = 0 unless an initial guess is given;
//  * right preconditioned flexible GMRES(m) in FP64 whose preconditioner may
//    use reduced-precision blocks (the preconditioner then changes from step
//    to step by rounding, which the flexible variant tolerates), stopping on
//    the true residual ||b - A x|| <= tol ||b||;
//  * the same two methods in lock step over many right-hand sides: one
//    batched operator and one batched preconditioner application per step,
//    inner products and rotations per right-hand side.
//
// Arnoldi orthogonalization: by default the delayed-reorthogonalization
// process of hps_krylov.h (one reduction pass and one update pass over the
// basis per step, restart <= 64); otherwise classical Gram-Schmidt applied
// twice (CGS2) in three passes (h1 = V^H w; w -= V h1 fused with h2 = V^H w;
// w -= V h2 with the norm).
// Everything except the loop control lives on the device; the host reads the
// residual estimates back every check_every steps.
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <type_traits>
#include <vector>

#include "hps_internal.h"
#include "hps_krylov.h"

namespace hps {
namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int pinned(hps_ctx* c, void** out) {
  if (!c->h_pinned) HPS_TRY_HIP(hipHostMalloc(&c->h_pinned, 1 << 16, hipHostMallocDefault));
  *out = c->h_pinned;
  return HPS_OK;
}

double bytes_apply(const hps_ctx* c) {
  return 32.0 * c->N + (c->c_complex ? 16.0 : 8.0) * c->nl * c->ni + 32.0 * c->nl * c->nb;
}

double bytes_precond(const hps_ctx* c, int q) {
  if (q == kFP64 && c->sep) return 32.0 * c->N;   // separable form: x in, y out
  const double beta = q == kFP64 ? 16.0 : (q == kFP32 ? 8.0 : 4.0);
  double b = beta * c->nblocks * (double)c->nb * c->blk[q].ncp + 32.0 * c->N;
  // lambda buckets: the H and U panels go through HBM (written, then read)
  if (c->lambda_bucket > 0.0) b += 2.0 * c->nl * (double)c->nb * (beta + (q == kFP64 ? 16.0 : 8.0));
  return b;
}

struct Job {
  int nrhs;          // right-hand sides iterated in lock step
  bool flexible;     // right preconditioning with stored Z
  int prec;          // block precision index inside J^{-1}
  double* rhs_res = nullptr;  // host, nrhs: final relative residual of each right-hand side
  bool face = false; // the face-reduced system (I + Pi R) f (no preconditioner) instead of A
  int64_t n = 0;     // vector length per right-hand side
};

// The operator of a job: A and J^{-1}, or the face-reduced operator with the
// identity in place of the preconditioner.
int job_apply(hps_ctx* c, const Job& job, const double2* x, double2* y, int nb) {
  return job.face ? launch_iti_apply(c, x, y, nb) : launch_apply(c, x, y, nb);
}
int job_precond(hps_ctx* c, const Job& job, const double2* x, double2* y, int nb) {
  if (job.face) {
    HPS_TRY_HIP(hipMemcpyAsync(y, x, sizeof(double2) * job.n * nb, hipMemcpyDeviceToDevice, c->stream));
    return HPS_OK;
  }
  return launch_precond(c, x, y, nb, job.prec);
}
int job_op_left(hps_ctx* c, const Job& job, const double2* x, double2* tmp, double2* y, int nb) {
  return job.face ? launch_iti_apply(c, x, y, nb) : launch_op_left(c, x, tmp, y, nb, job.prec);
}
// vectors in FP32 (the inner solve of iterative refinement): A and the separable J^{-1}
int job_apply(hps_ctx* c, const Job&, const float2* x, float2* y, int nb) {
  return launch_apply(c, x, y, nb);
}
int job_precond(hps_ctx* c, const Job&, const float2* x, float2* y, int nb) {
  return launch_precond(c, x, y, nb);
}
int job_op_left(hps_ctx* c, const Job&, const float2* x, float2* tmp, float2* y, int nb) {
  return launch_op_left(c, x, tmp, y, nb);
}

// Algorithmic bytes of the timed apply and preconditioner launches of a solve.
// Left preconditioning with fewer than kBatchedMinRhs right-hand sides fuses
// the face exchange into J^{-1}: the apply is the sweep alone (x, y, C and the
// face buffer written) and J^{-1} also reads the face buffer.
void solve_bytes_stats(const hps_ctx* c, const Job& job, int nb, hps_stats* st) {
  const double face = 16.0 * c->nl * (double)c->nb;
  if (job.face) {
    // the ItI block stream (R, f in, g out) and the exchange (f, g in, y out)
    st->bytes_apply = face * c->nb + 2.0 * face + 3.0 * face;
    st->bytes_precond = 0.0;
    return;
  }
  const bool fused = !job.flexible && (nb < kBatchedMinRhs || c->nop > 1) && !(c->lambda_bucket > 0.0);
  st->bytes_apply = bytes_apply(c) - (fused ? face : 0.0);
  st->bytes_precond = bytes_precond(c, job.prec) + (fused ? face : 0.0);
}

int solver_events(hps_ctx* c, hipEvent_t* evs) {
  for (int i = 0; i < 2; ++i) {
    if (!c->ev_solver[i]) HPS_TRY_HIP(hipEventCreateWithFlags(&c->ev_solver[i], hipEventDisableTiming));
    evs[i] = c->ev_solver[i];
  }
  return HPS_OK;
}


// Lock-step (F)GMRES over nb right-hand sides stored one after the other.
// b: nb*N device, x: nb*N device (initial guess if use_x0).
int run_gmres(hps_ctx* c, const Job& job, const double2* b, double2* x, double tol, int m,
              int maxit, int use_x0, int check_every, hps_stats* st) {
  const int64_t N = job.n;
  const int nb = job.nrhs;
  const int64_t NB = N * nb;  // one batched vector
  // workspace: V (m+1 batched vectors), Z (m, flexible only), tmp
  const size_t vec_bytes = sizeof(double2) * NB;
  const size_t need = vec_bytes * ((size_t)(m + 1) + (job.flexible ? m : 0) + 1);
  int rc = ws_reserve(c, &c->w_krylov, need);
  if (rc) return rc;
  rc = ws_reserve(c, &c->w_small, sizeof(GmresState) * nb + 4 * sizeof(double) * nb);
  if (rc) return rc;
  RedBuf rb;
  if ((rc = red_buf(c, m + 1, nb, &rb))) return rc;
  double2* V = static_cast<double2*>(c->w_krylov.ptr);
  double2* Z = job.flexible ? V + (size_t)(m + 1) * NB : nullptr;
  double2* tmp = V + (size_t)((m + 1) + (job.flexible ? m : 0)) * NB;
  GmresState* S = static_cast<GmresState*>(c->w_small.ptr);
  // two slots of (residual estimate, breakdown) per right-hand side
  double* d_res = reinterpret_cast<double*>(S + nb);
  const int64_t sst = sizeof(GmresState) / sizeof(double2);  // state stride in double2 units
  static_assert(sizeof(GmresState) % sizeof(double2) == 0, "state stride");
  double* nrm2 = &S[0].nrm2;
  const int64_t nrm_stride = sizeof(GmresState) / sizeof(double);
  void* hp = nullptr;
  if ((rc = pinned(c, &hp))) return rc;
  double* hbuf = static_cast<double*>(hp);
  hipEvent_t evs[2];
  if ((rc = solver_events(c, evs))) return rc;

  auto Vj = [&](int j) { return V + (size_t)j * NB; };
  auto Zj = [&](int j) { return Z + (size_t)j * NB; };
  // norm^2 of every right-hand side's part of a batched vector into S[r].nrm2
  auto norms = [&](const double2* v) -> int {
    return launch_norm2_b(c, v, N, N, nrm2, nrm_stride, nb, rb);
  };
  auto read_nrm2 = [&](std::vector<double>& out) -> int {
    HPS_TRY_HIP(hipMemcpy2DAsync(hbuf, sizeof(double), nrm2, sizeof(GmresState), sizeof(double), nb,
                                 hipMemcpyDeviceToHost, c->stream));
    HPS_TRY_HIP(hipStreamSynchronize(c->stream));
    out.assign(hbuf, hbuf + nb);
    return HPS_OK;
  };
  // residual source r = b - A x (or b when x = 0) into tmp, then the cycle's
  // first vector: left: J^{-1} r; flexible: r
  auto residual = [&](bool x_zero) -> int {
    int e;
    if (x_zero) {
      HPS_TRY_HIP(hipMemcpyAsync(tmp, b, vec_bytes, hipMemcpyDeviceToDevice, c->stream));
    } else {
      if ((e = job_apply(c, job, x, tmp, nb))) return e;
      if ((e = launch_sub_from(c, b, tmp, NB))) return e;
    }
    if (!job.flexible) {
      if ((e = job_precond(c, job, tmp, Vj(0), nb))) return e;
    } else {
      HPS_TRY_HIP(hipMemcpyAsync(Vj(0), tmp, vec_bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    return norms(Vj(0));
  };

  const double t0 = now();
  // normalizer: ||J^{-1} b|| (left) or ||b|| (flexible), per right-hand side
  std::vector<double> bn2, beta2;
  if ((rc = residual(true))) return rc;
  if ((rc = read_nrm2(bn2))) return rc;
  std::vector<double> bnorm(nb);
  for (int r = 0; r < nb; ++r) bnorm[r] = std::sqrt(bn2[r]);
  if (use_x0) {
    if ((rc = residual(false))) return rc;
    if ((rc = read_nrm2(beta2))) return rc;
  } else {
    HPS_TRY_HIP(hipMemsetAsync(x, 0, vec_bytes, c->stream));
    beta2 = bn2;
  }
  for (int r = 0; r < nb; ++r)
    if (!std::isfinite(beta2[r]) || !std::isfinite(bn2[r]))
      return fail(HPS_ERR_NUMERIC, "non-finite residual norm (NaN or Inf in the data)");

  int its = 0, restarts = 0;
  std::vector<int> done(nb, 0);
  std::vector<double> est(nb, 0.0);
  auto all_done = [&]() {
    for (int r = 0; r < nb; ++r)
      if (!done[r]) return false;
    return true;
  };
  for (int r = 0; r < nb; ++r) {
    done[r] = (bnorm[r] == 0.0) || (std::sqrt(beta2[r]) <= tol * bnorm[r]);
    est[r] = bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0;
  }
  bool breakdown = false;
  while (!all_done() && its < maxit) {
    // V0 = r / beta; g = (beta, 0, ...)
    if ((rc = launch_scale_by_b(c, Vj(0), N, Vj(0), N, N, nrm2, nrm_stride, 1, nb))) return rc;
    if ((rc = launch_gm_start(c, S, nb))) return rc;
    int k = 0;
    int pending = -1;
    for (int j = 0; j < m && its < maxit; ++j) {
      // w_j = J^{-1} A v_j (left) or A M^{-1} v_j (flexible), into V[j+1]
      if (!job.flexible) {
        if ((rc = job_op_left(c, job, Vj(j), tmp, Vj(j + 1), nb))) return rc;
      } else {
        if ((rc = launch_precond(c, Vj(j), Zj(j), nb, job.prec))) return rc;
        if ((rc = launch_apply(c, Zj(j), Vj(j + 1), nb))) return rc;
      }
      // CGS2 against V[0..j], per right-hand side, in three passes over the
      // basis: h1 = V^H w;  w -= V h1 and h2 = V^H w (fused);  w -= V h2 with
      // ||w||^2.  The Hessenberg column is h1 + h2.
      if ((rc = launch_cgs_pass(c, false, V, NB, N, j + 1, nullptr, 0, Vj(j + 1), N, N, S[0].h1,
                                sst, nb, rb)))
        return rc;
      if ((rc = launch_cgs_pass(c, true, V, NB, N, j + 1, S[0].h1, sst, Vj(j + 1), N, N, S[0].h2,
                                sst, nb, rb)))
        return rc;
      if ((rc = launch_mupdate_b(c, V, NB, N, j + 1, S[0].h2, sst, -1.0, Vj(j + 1), N, N, nrm2,
                                 nrm_stride, nb, rb)))
        return rc;
      if ((rc = launch_gm_givens(c, S, nb, j))) return rc;
      if ((rc = launch_scale_by_b(c, Vj(j + 1), N, Vj(j + 1), N, N, nrm2, nrm_stride, 1, nb)))
        return rc;
      ++its;
      k = j + 1;
      // The residual estimate of step j is copied to pinned memory behind an
      // event; the host looks at it only after step j+1 has been queued, so the
      // device never waits for the host.
      const bool last = (j == m - 1) || its >= maxit;
      const bool want = (its % check_every == 0) || last;
      if (want) {
        const int slot = j & 1;
        if ((rc = launch_gm_collect(c, S, nb, d_res + 2 * slot * nb))) return rc;
        HPS_TRY_HIP(hipMemcpyAsync(hbuf + 2 * slot * nb, d_res + 2 * slot * nb,
                                   2 * sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
        HPS_TRY_HIP(hipEventRecord(evs[slot], c->stream));
      }
      auto converged_at = [&](int step) -> int {
        const int slot = step & 1;
        HPS_TRY_HIP(hipEventSynchronize(evs[slot]));
        bool all = true;
        for (int r = 0; r < nb; ++r) {
          const double res = hbuf[2 * (slot * nb + r)];
          const int bd = hbuf[2 * (slot * nb + r) + 1] != 0.0;
          if (!std::isfinite(res)) return fail(HPS_ERR_NUMERIC, "non-finite residual estimate");
          est[r] = bnorm[r] > 0 ? res / bnorm[r] : 0.0;
          if (bd) breakdown = true;
          if (!(done[r] || res <= tol * bnorm[r] || bd)) all = false;
        }
        return all ? 1 : 0;
      };
      if (pending >= 0) {
        const int cv = converged_at(pending);
        pending = -1;
        if (cv < 0) return cv;
        if (cv) break;  // step j is already queued; its column is used as well
      }
      if (last) {
        const int cv = converged_at(j);
        if (cv < 0) return cv;
        break;
      }
      if (want) pending = j;
    }
    // x += V y (left) or Z y (flexible), per right-hand side
    if ((rc = launch_gm_trisolve(c, S, nb, k))) return rc;
    if ((rc = launch_mupdate_b(c, job.flexible ? Z : V, NB, N, k, S[0].y, sst, 1.0, x, N, N,
                               nullptr, 0, nb, rb)))
      return rc;
    ++restarts;
    // true residual of the new iterate (preconditioned for the left variant)
    if ((rc = residual(false))) return rc;
    if ((rc = read_nrm2(beta2))) return rc;
    for (int r = 0; r < nb; ++r) {
      if (!std::isfinite(beta2[r])) return fail(HPS_ERR_NUMERIC, "non-finite residual");
      const double rr = bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0;
      if (rr <= tol) done[r] = 1;
    }
    if (breakdown && !all_done()) {
      // an exact invariant subspace without convergence can only come from
      // rounding; one more cycle from the current iterate decides
      breakdown = false;
    }
  }
  if (job.rhs_res)
    for (int r = 0; r < nb; ++r) job.rhs_res[r] = bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0;
  if (st) {
    double worst_est = 0.0, worst_true = 0.0;
    for (int r = 0; r < nb; ++r) {
      worst_est = std::max(worst_est, est[r]);
      worst_true = std::max(worst_true, bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0);
    }
    st->iters = its;
    st->restarts = restarts;
    st->converged = all_done() ? 1 : 0;
    st->lambda_shifted = c->n_shifted;
    st->t_setup = c->t_setup;
    st->rel_res = worst_est;
    st->true_rel_res = worst_true;
    st->t_solve = now() - t0;
    solve_bytes_stats(c, job, nb, st);
  }
  return all_done() ? HPS_OK : HPS_NOT_CONVERGED;
}


// (F)GMRES(m) with the delayed-reorthogonalization Arnoldi process (two passes
// over the basis per step, see hps_krylov.h); m <= kMaxDcgs.  Same stopping
// rules, restart policy and pipelined residual checks as run_gmres.
// VT: storage of the vectors (complex FP64, or complex FP32 for the inner solve
// of iterative refinement, whose basis lives in its own workspace); XT: storage
// of the iterate x (FP64 over an FP32 basis for that inner solve, one
// right-hand side).
template <typename VT, typename XT = VT>
int run_dcgs(hps_ctx* c, const Job& job, const VT* b, XT* x, double tol, int m, int maxit,
             int use_x0, int check_every, hps_stats* st) {
  constexpr bool kMixed = !std::is_same<VT, XT>::value;
  static_assert(!kMixed || (std::is_same<VT, float2>::value && std::is_same<XT, double2>::value),
                "the only mixed storage is an FP64 iterate over an FP32 basis");
  const int64_t N = job.n;
  const int nb = job.nrhs;
  const int64_t NB = N * nb;
  const size_t vec_bytes = sizeof(VT) * NB;
  if (kMixed && (nb != 1 || job.flexible)) return fail(HPS_ERR_ARG, "FP64 iterate: one right-hand side, left GMRES");
  // V (m), candidate U, operator image W, TMP, Z' (m, flexible)
  const size_t need = vec_bytes * ((size_t)m + 3 + (job.flexible ? m : 0));
  Workspace* wk = sizeof(VT) == sizeof(double2) ? &c->w_krylov : &c->w_krylov32;
  int rc = ws_reserve(c, wk, need);
  if (rc) return rc;
  rc = ws_reserve(c, &c->w_small, sizeof(DcgsState) * nb + 6 * sizeof(double) * nb);
  if (rc) return rc;
  RedBuf rb;
  if ((rc = red_buf(c, kMaxDcgs + 1, nb, &rb))) return rc;
  VT* V = static_cast<VT*>(wk->ptr);
  VT* U = V + (size_t)m * NB;
  VT* W = U + NB;
  VT* TMP = W + NB;
  VT* Z = job.flexible ? TMP + NB : nullptr;
  DcgsState* S = static_cast<DcgsState*>(c->w_small.ptr);
  double* d_res = reinterpret_cast<double*>(S + nb);   // 4 doubles per rhs (last column)
  double* d_nrm = d_res + 4 * nb;                        // norms^2 per rhs
  static_assert(sizeof(DcgsState) % sizeof(double2) == 0, "state stride");
  const int64_t sst = sizeof(DcgsState) / sizeof(double2);
  void* hp = nullptr;
  if ((rc = pinned(c, &hp))) return rc;
  double* hbuf = static_cast<double*>(hp);
  // Residual records: the update pass of step j writes {estimate, stopped, tag}
  // for every right-hand side straight into pinned host memory (slot j & 1),
  // the tag last with a system-scope release; the host waits for the tag of
  // the step it reads.  No copy and no event is queued per step.
  double* hrec = hbuf;                 // 2 slots x nb x 4 doubles
  double* hnrm = hbuf + 8 * nb;        // norms^2 read back at restarts
  void* drec_v = nullptr;
  HPS_TRY_HIP(hipHostGetDevicePointer(&drec_v, hrec, 0));
  double* drec = static_cast<double*>(drec_v);
  const uint64_t epoch = (uint64_t)(++c->solve_epoch) << 32;
  auto Vj = [&](int j) { return V + (size_t)j * NB; };
  auto Zj = [&](int j) { return Z + (size_t)j * NB; };

  auto read_norms = [&](std::vector<double>& out) -> int {
    HPS_TRY_HIP(hipMemcpyAsync(hnrm, d_nrm, sizeof(double) * nb, hipMemcpyDeviceToHost, c->stream));
    HPS_TRY_HIP(hipStreamSynchronize(c->stream));
    out.assign(hnrm, hnrm + nb);
    return HPS_OK;
  };
  // wait until every right-hand side's record in `slot` carries `tag`
  auto wait_records = [&](int slot, uint64_t tag) -> int {
    for (int r = 0; r < nb; ++r) {
      const uint64_t* tp = reinterpret_cast<const uint64_t*>(hrec + 4 * (slot * nb + r) + 2);
      for (long spins = 1; __atomic_load_n(tp, __ATOMIC_ACQUIRE) != tag; ++spins) {
        if ((spins & 255) == 0) {
          const hipError_t e = hipStreamQuery(c->stream);
          if (e == hipSuccess) {  // all queued work is done: the record must be there
            if (__atomic_load_n(tp, __ATOMIC_ACQUIRE) == tag) break;
            return fail(HPS_ERR_DEVICE, "residual record of a finished step is missing");
          }
          if (e != hipErrorNotReady) return check_hip(e, "hipStreamQuery");
        }
        std::this_thread::yield();
      }
    }
    return HPS_OK;
  };
  // first candidate of a cycle: left J^-1 (b - A x), flexible b - A x (unnormalized), and its norm
  auto residual = [&](bool x_zero) -> int {
    int e;
    if (x_zero) {
      HPS_TRY_HIP(hipMemcpyAsync(TMP, b, vec_bytes, hipMemcpyDeviceToDevice, c->stream));
    } else {
      if constexpr (kMixed) {   // the FP32 operator on x rounded to FP32 (W is free here)
        if ((e = launch_demote_scaled(c, x, 1.0, W, N))) return e;
        if ((e = job_apply(c, job, W, TMP, nb))) return e;
      } else {
        if ((e = job_apply(c, job, x, TMP, nb))) return e;
      }
      if ((e = launch_sub_from(c, b, TMP, NB))) return e;
    }
    if (!job.flexible) {
      if ((e = job_precond(c, job, TMP, U, nb))) return e;
    } else {
      HPS_TRY_HIP(hipMemcpyAsync(U, TMP, vec_bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    return launch_norm2_b(c, U, N, N, d_nrm, 1, nb, rb);
  };

  const double t0 = now();
  std::vector<double> bn2, beta2;
  if ((rc = residual(true))) return rc;
  if ((rc = read_norms(bn2))) return rc;
  std::vector<double> bnorm(nb);
  for (int r = 0; r < nb; ++r) bnorm[r] = std::sqrt(bn2[r]);
  if (use_x0) {
    if ((rc = residual(false))) return rc;
    if ((rc = read_norms(beta2))) return rc;
  } else {
    HPS_TRY_HIP(hipMemsetAsync(x, 0, sizeof(XT) * NB, c->stream));
    beta2 = bn2;
  }
  for (int r = 0; r < nb; ++r)
    if (!std::isfinite(beta2[r]) || !std::isfinite(bn2[r]))
      return fail(HPS_ERR_NUMERIC, "non-finite residual norm (NaN or Inf in the data)");
  int its = 0, restarts = 0;
  std::vector<int> done(nb, 0);
  std::vector<double> est(nb, 0.0);
  auto all_done = [&]() {
    for (int r = 0; r < nb; ++r)
      if (!done[r]) return false;
    return true;
  };
  for (int r = 0; r < nb; ++r) {
    done[r] = (bnorm[r] == 0.0) || (std::sqrt(beta2[r]) <= tol * bnorm[r]);
    est[r] = bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0;
  }
  while (!all_done() && its < maxit) {
    if ((rc = launch_dcgs_start(c, S, nb))) return rc;
    int pending = -1;
    uint64_t pending_tag = 0;
    int written = 0;      // basis vectors V[0..written-1] written by update passes
    auto converged_at = [&](int step, uint64_t tag) -> int {
      const int slot = step & 1;
      int e = wait_records(slot, tag);
      if (e) return e;
      bool all = true;
      for (int r = 0; r < nb; ++r) {
        const double res = hrec[4 * (slot * nb + r)];
        const bool flag = hrec[4 * (slot * nb + r) + 1] != 0.0;
        if (!std::isfinite(res)) return fail(HPS_ERR_NUMERIC, "non-finite residual estimate");
        est[r] = bnorm[r] > 0 ? res / bnorm[r] : 0.0;
        if (!(done[r] || res <= tol * bnorm[r] || flag)) all = false;
      }
      return all ? 1 : 0;
    };
    bool stopped = false;   // the step records said every right-hand side is done or stuck
    bool closed = false;    // the last update pass made the closing reduction
    int last_step = -1;     // the last step's record, read after the closing work is queued
    uint64_t last_tag = 0;
    for (int j = 0; j < m && its < maxit; ++j) {
      // operator image of the candidate: left J^-1 A u, flexible A M^-1 u (z'_j kept)
      if (!job.flexible) {
        if ((rc = job_op_left(c, job, U, TMP, W, nb))) return rc;
      } else {
        if ((rc = job_precond(c, job, U, Zj(j), nb))) return rc;
        if ((rc = job_apply(c, job, Zj(j), W, nb))) return rc;
      }
      if ((rc = launch_dcgs_reduce(c, V, NB, N, j, U, N, W, N, N, S, nb, rb))) return rc;
      const int slot = j & 1;
      ++its;
      const uint64_t tag = epoch | (uint64_t)its;
      const bool last = (j == m - 1) || its >= maxit;
      // the last update pass of a cycle also makes the closing reduction
      closed = last && dcgs_can_close(j, N);
      if ((rc = closed ? launch_dcgs_update_close(c, V, NB, N, j, U, N, W, N, N, S, nb,
                                                  job.flexible ? 1 : 0, drec + 4 * slot * nb, tag, rb)
                       : launch_dcgs_update(c, V, NB, N, j, U, N, W, N, N, S, nb, job.flexible ? 1 : 0,
                                            drec + 4 * slot * nb, tag)))
        return rc;
      written = j + 1;
      const bool want = (its % check_every == 0) || last;
      if (pending >= 0) {
        const int cv = converged_at(pending, pending_tag);
        pending = -1;
        if (cv < 0) return cv;
        if (cv) {
          stopped = true;
          break;
        }
      }
      if (last) {
        last_step = j;
        last_tag = tag;
        break;
      }
      if (want) {
        pending = j;
        pending_tag = tag;
      }
    }
    // close the last column: reduction of the current candidate against the
    // basis (a no-op for right-hand sides whose cycle already stopped), unless
    // the last update pass made it
    if (!closed && (rc = launch_dcgs_reduce(c, V, NB, N, written, U, N, nullptr, 0, N, S, nb, rb)))
      return rc;
    if ((rc = launch_dcgs_small(c, S, nb, written, job.flexible ? 1 : 0, 1, d_res, 0))) return rc;
    if ((rc = launch_dcgs_trisolve(c, S, nb, written, job.flexible ? 1 : 0))) return rc;
    // left GMRES on FP64 vectors: x += V y and the next residual from the
    // Arnoldi relation in one pass (no operator application, no host round
    // trip).  Flexible GMRES takes the iterate from Z; an FP32-stored iterate
    // keeps the recomputed residual below, because the recursion does not see
    // x's rounding to FP32 (with it inner solves took 20 % more steps), so the
    // inner solves of iterative refinement keep x in FP64.
    const bool implicit = !job.flexible && sizeof(XT) == sizeof(double2);
    if (implicit) {
      if ((rc = launch_dcgs_restart_coef(c, S, nb, written))) return rc;
      if ((rc = launch_dcgs_restart(c, (const VT*)V, NB, N, written, U, N, x, N, N, S, nb))) return rc;
    } else if constexpr (!kMixed) {
      if ((rc = launch_mupdate_b(c, (const VT*)(job.flexible ? Z : V), NB, N, written, S[0].y, sst, 1.0,
                                 x, N, N, nullptr, 0, nb, rb)))
        return rc;
    }
    ++restarts;
    if (last_step >= 0) {   // read while the closing work runs
      const int cv = converged_at(last_step, last_tag);
      if (cv < 0) return cv;
      stopped = cv != 0;
    }
    // the next cycle starts from the implicit residual unless the records say
    // the solve may be over (then the true residual decides) or the step
    // budget is spent
    if (implicit && !stopped && its < maxit) continue;
    if ((rc = residual(false))) return rc;
    if ((rc = read_norms(beta2))) return rc;
    for (int r = 0; r < nb; ++r) {
      if (!std::isfinite(beta2[r])) return fail(HPS_ERR_NUMERIC, "non-finite residual");
      const double rr = bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0;
      if (rr <= tol) done[r] = 1;
    }
  }
  if (job.rhs_res)
    for (int r = 0; r < nb; ++r) job.rhs_res[r] = bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0;
  if (st) {
    double worst_est = 0.0, worst_true = 0.0;
    for (int r = 0; r < nb; ++r) {
      worst_est = std::max(worst_est, est[r]);
      worst_true = std::max(worst_true, bnorm[r] > 0 ? std::sqrt(beta2[r]) / bnorm[r] : 0.0);
    }
    st->iters = its;
    st->restarts = restarts;
    st->converged = all_done() ? 1 : 0;
    st->lambda_shifted = c->n_shifted;
    st->t_setup = c->t_setup;
    st->rel_res = worst_est;
    st->true_rel_res = worst_true;
    st->t_solve = now() - t0;
    solve_bytes_stats(c, job, nb, st);
  }
  return all_done() ? HPS_OK : HPS_NOT_CONVERGED;
}

// Iterative refinement (one right-hand side): an FP64 outer loop on the true
// residual r = b - A x (FP64 apply), each correction from an inner left-
// preconditioned GMRES(m) with the delayed-reorthogonalization Arnoldi whose
// vectors (basis, candidate, operator image) are stored in complex FP32, with
// the FP32-storage A and the separable J^{-1}, started from 0 on r / ||r||
// and stopped at the preconditioned residual reduction inner_tol (or at a
// tenth of the reduction the outer tolerance still needs, if that is larger);
// then x += ||r|| d in FP64.  The inner iterate d is kept in FP64, so the inner
// restarts take the residual from the Arnoldi relation.  Stops when ||b - A x|| <= tol ||b||, when the
// residual stops decreasing, or after maxit inner steps.
int run_ir(hps_ctx* c, const double2* b, double2* x, double tol, int m, int maxit, int use_x0,
           int check_every, double inner_tol, double* rhs_res, hps_stats* st) {
  const int64_t N = c->N;
  int rc = ws_reserve(c, &c->w_ir, 2 * sizeof(double2) * N + sizeof(float2) * N + 64);
  if (rc) return rc;
  double2* r = static_cast<double2*>(c->w_ir.ptr);
  double2* d64 = r + N;   // the inner correction, kept in FP64 (see run_dcgs)
  float2* r32 = reinterpret_cast<float2*>(d64 + N);
  double* d_nrm = reinterpret_cast<double*>(r32 + N);
  RedBuf rb;
  if ((rc = red_buf(c, kMaxDcgs + 1, 1, &rb))) return rc;
  void* hp = nullptr;
  if ((rc = pinned(c, &hp))) return rc;
  double* hn = static_cast<double*>(hp) + 4096;   // past the inner solve's records
  auto norm = [&](const double2* v, double* out) -> int {
    int e = launch_norm2_b(c, v, N, N, d_nrm, 1, 1, rb);
    if (e) return e;
    HPS_TRY_HIP(hipMemcpyAsync(hn, d_nrm, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HPS_TRY_HIP(hipStreamSynchronize(c->stream));
    *out = std::sqrt(*hn);
    if (!std::isfinite(*out)) return fail(HPS_ERR_NUMERIC, "non-finite residual norm (NaN or Inf in the data)");
    return HPS_OK;
  };
  auto residual = [&]() -> int {   // r = b - A x
    int e = launch_apply(c, x, r, 1);
    if (e) return e;
    return launch_sub_from(c, b, r, N);
  };
  const double t0 = now();
  double bn = 0.0, rn = 0.0;
  if ((rc = norm(b, &bn))) return rc;
  if (use_x0) {
    if ((rc = residual())) return rc;
  } else {
    HPS_TRY_HIP(hipMemsetAsync(x, 0, sizeof(double2) * N, c->stream));
    HPS_TRY_HIP(hipMemcpyAsync(r, b, sizeof(double2) * N, hipMemcpyDeviceToDevice, c->stream));
  }
  if ((rc = norm(r, &rn))) return rc;
  Job job;
  job.flexible = false;
  job.prec = kFP64;
  job.n = N;
  job.nrhs = 1;
  int its = 0, outer = 0;
  double prev = HUGE_VAL;
  bool done = bn == 0.0 || rn <= tol * bn;
  while (!done && its < maxit && rn < prev) {
    if ((rc = launch_demote_scaled(c, r, 1.0 / rn, r32, N))) return rc;
    hps_stats one{};
    const int inner_max = std::max(m, std::min(maxit - its, 40 * m));
    // an inner solve need not reduce its residual much below what the outer
    // tolerance still asks for (with a margin of 10 for the gap between the
    // inner preconditioned residual and the outer true one): the last
    // refinement of a solve is then short instead of a full inner_tol
    const double itol = std::max(inner_tol, std::min(0.5, 0.1 * tol * bn / rn));
    const int r1 = run_dcgs<float2, double2>(c, job, r32, d64, itol, m, inner_max, 0, check_every, &one);
    if (r1 < 0) return r1;
    its += one.iters;
    ++outer;
    if ((rc = launch_axpy_promote(c, rn, d64, x, N))) return rc;
    if ((rc = residual())) return rc;
    prev = rn;
    if ((rc = norm(r, &rn))) return rc;
    done = rn <= tol * bn;
  }
  const double rel = bn > 0.0 ? rn / bn : 0.0;
  if (rhs_res) *rhs_res = rel;
  if (st) {
    st->iters = its;
    st->restarts = outer;
    st->converged = done ? 1 : 0;
    st->lambda_shifted = c->n_shifted;
    st->t_setup = c->t_setup;
    st->rel_res = rel;
    st->true_rel_res = rel;
    st->t_solve = now() - t0;
    // the inner step's launches: the sweep (x in and y out in FP32, C, the FP32
    // face buffer written) and J^{-1} (y in and out in FP32, the face buffer read)
    const double face = 8.0 * c->nl * (double)c->nb;
    st->bytes_apply = 16.0 * N + (c->c_complex ? 16.0 : 8.0) * c->nl * c->ni + face;
    st->bytes_precond = 16.0 * N + face;
  }
  return done ? HPS_OK : HPS_NOT_CONVERGED;
}

int run_solver(hps_ctx* c, const Job& job, const double2* b, double2* x, double tol, int m,
               int maxit, int use_x0, int check_every, int orth, hps_stats* st) {
  if (orth == 0 && m <= kMaxDcgs)
    return run_dcgs(c, job, b, x, tol, m, maxit, use_x0, check_every, st);
  return run_gmres(c, job, b, x, tol, m, maxit, use_x0, check_every, st);
}
}  // namespace
}  // namespace hps

using namespace hps;

extern "C" int64_t hps_solve_bytes(const hps_ctx* c, int restart, int nrhs, const hps_solve_opts* so) {
  if (!c || restart < 1 || restart > kMaxRestart || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments");
  hps_solve_opts o{};
  if (so) o = *so;
  if (o.solver == HPS_SOLVER_ITI) {
    // face vectors: basis + U, W, TMP (DCGS) or basis + tmp (CGS2), the face
    // right-hand side and solution, the leaf workspace, b, the g buffer
    const int64_t vf = 16 * c->nl * (int64_t)c->nb;
    int64_t bytes = vf * (restart + 3) + 2 * vf + iti_ws_bytes(c, 1) + vf;
    bytes += (int64_t)sizeof(GmresState) + 32 + (int64_t)kPartSlots * kRedBlocks * 16;
    bytes += 16 * c->N * nrhs;
    return bytes;
  }
  if (o.solver == HPS_SOLVER_IR) {
    // FP64 residual and correction, FP32 residual; the inner FP32 basis, U, W
    // and TMP; the FP64 face buffer; the small state, the reduction partials, b
    int64_t bytes = 2 * 16 * c->N + 8 * c->N + 64 + 8 * c->N * (int64_t)(restart + 3);
    bytes += 16 * c->nl * (int64_t)c->nb + (int64_t)sizeof(DcgsState) + 6 * 8 + 8;
    bytes += (int64_t)kPartSlots * kRedBlocks * 16 + 16 * c->N * nrhs;
    return bytes;
  }
  const bool fp64_pc = o.precond_prec == 0 || o.precond_prec == HPS_PREC_FP64 ||
                       o.precond_prec == HPS_PREC_SEPARABLE;
  if (o.solver == HPS_SOLVER_BGMRES) {
    // basis ((m+1) k vectors), W, TMP, J^-1 B, small matrices, the face buffer
    // and (dense blocks, k >= 4) the GEMM panels of J^-1, the assembled b
    const int64_t k = std::min(nrhs, kMaxBatch);
    int64_t bytes = 16 * c->N * k * (restart + 4) + 16 * (int64_t)(restart + 1) * k * k + 1024;
    bytes += 16 * k * c->nl * c->nb;
    if (!c->sep && k >= kBatchedMinRhs) bytes += k * c->nl * c->nb * 32 + 256;
    bytes += 16 * c->N * nrhs;
    return bytes;
  }
  const bool flexible = o.solver == HPS_SOLVER_FGMRES || !fp64_pc;
  const bool lock = o.solver == HPS_SOLVER_BLOCK || c->nop > 1 || (o.solver == HPS_SOLVER_FGMRES && nrhs > 1);
  const int64_t nbat = lock ? std::min(nrhs, kMaxBatch) : 1;
  const int64_t vec = 16 * c->N * nbat;
  int64_t bytes = vec * ((restart + 1) + (flexible ? restart : 0) + 1);  // basis (+Z) + tmp
  bytes += (int64_t)sizeof(GmresState) * nbat + 32 * nbat;               // Hessenberg state
  bytes += (int64_t)kPartSlots * kRedBlocks * 16 * nbat;                  // reduction partials
  bytes += 16 * nbat * c->nl * c->nb;                                     // face buffer
  if (((nbat >= kBatchedMinRhs && c->nop == 1) || c->lambda_bucket > 0.0) && !(fp64_pc && c->sep))
    bytes += nbat * c->nl * c->nb * (16 + 16) + 256;                      // H, U panels
  bytes += 16 * c->N * nrhs;                                              // assembled b
  return bytes;
}

extern "C" int hps_gmres(hps_ctx* c, const hps_z* s, const hps_z* t, double tol, int restart,
                         hps_z* u, int nrhs, const hps_solve_opts* so, hps_stats* st) {
  if (!c || !s || !u || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_gmres");
  if (!(tol > 0.0) || !(tol < 1.0)) return fail(HPS_ERR_ARG, "tol must lie in (0, 1)");
  if (restart < 1 || restart > kMaxRestart) return fail(HPS_ERR_ARG, "restart must lie in [1, 200]");
  hps_solve_opts o{};
  if (so) o = *so;
  const int maxit = o.max_iters > 0 ? o.max_iters : 20000;
  const int check_every = o.check_every > 0 ? o.check_every : 1;
  int prec = kFP64;
  if (o.precond_prec == HPS_PREC_FP32) prec = kFP32;
  else if (o.precond_prec == HPS_PREC_BF16) prec = kBF16;
  else if (o.precond_prec == HPS_PREC_SEPARABLE) {
    if (!c->sep) return fail(HPS_ERR_ARG, "the separable J^-1 was not built at setup");
  } else if (o.precond_prec != 0 && o.precond_prec != HPS_PREC_FP64)
    return fail(HPS_ERR_ARG, "unknown precond_prec");
  if (!c->blk[prec].data && !(prec == kFP64 && c->sep))
    return fail(HPS_ERR_ARG, "precond_prec blocks were not built at setup");
  if (o.solver < 0 || o.solver > 5) return fail(HPS_ERR_ARG, "unknown solver");
  if (o.solver == HPS_SOLVER_IR) {
    if (!c->sep) return fail(HPS_ERR_ARG, "iterative refinement needs the separable J^-1 (HPS_PREC_SEPARABLE)");
    if (c->nop > 1) return fail(HPS_ERR_UNSUPPORTED, "iterative refinement: operator groups are not supported");
    if (o.precond_prec != 0 && o.precond_prec != HPS_PREC_FP64 && o.precond_prec != HPS_PREC_SEPARABLE)
      return fail(HPS_ERR_ARG, "iterative refinement runs the separable J^-1 (precond_prec must be 0)");
    if (o.inner_tol < 0.0 || !(o.inner_tol < 1.0))
      return fail(HPS_ERR_ARG, "inner_tol must lie in [0, 1)");
    if (restart > kMaxDcgs) return fail(HPS_ERR_ARG, "iterative refinement: restart must be at most 64");
  }
  if (o.solver == HPS_SOLVER_BGMRES) {
    if (prec != kFP64) return fail(HPS_ERR_ARG, "block GMRES runs the FP64 preconditioner");
    if (c->nop > 1) return fail(HPS_ERR_UNSUPPORTED, "block GMRES: operator groups run lock-step");
    if (nrhs > kMaxBatch) return fail(HPS_ERR_ARG, "block GMRES: at most 64 right-hand sides");
  }
  if (c->nop > 1 && nrhs != c->nop)
    return fail(HPS_ERR_ARG, "operator group: one right-hand side per operator (nrhs = number of operators)");
  if (o.solver == HPS_SOLVER_ITI) {
    if (!c->d_itiR) return fail(HPS_ERR_ARG, "the face-reduced solver needs hps_iti_build first");
    if (o.use_x0) return fail(HPS_ERR_ARG, "the face-reduced solver starts from f = 0 (use_x0 unsupported)");
    if (o.precond_prec != 0 && o.precond_prec != HPS_PREC_FP64)
      return fail(HPS_ERR_ARG, "the face-reduced solver has no preconditioner (precond_prec must be 0)");
  }
  if (o.solver == HPS_SOLVER_GMRES && prec != kFP64)
    return fail(HPS_ERR_ARG, "left GMRES runs the FP64 preconditioner; use FGMRES for reduced precision");
  // b for every right-hand side, in a workspace kept between calls
  int rc = ws_reserve(c, &c->w_b, sizeof(double2) * c->N * nrhs);
  if (rc) return rc;
  double2* bvec = static_cast<double2*>(c->w_b.ptr);
  rc = launch_assemble_rhs(c, reinterpret_cast<const double2*>(s), reinterpret_cast<const double2*>(t),
                           bvec, nrhs);
  double2* x = reinterpret_cast<double2*>(u);
  if (rc == HPS_OK && o.solver == HPS_SOLVER_ITI) {
    // face-reduced system: right-hand side t - Pi h, GMRES on (I + Pi R) f,
    // then the leaf solves; one right-hand side at a time
    const int64_t nf = c->nl * (int64_t)c->nb;
    Job job;
    job.flexible = false;
    job.prec = kFP64;
    job.face = true;
    job.n = nf;
    job.nrhs = 1;
    hps_stats acc{};
    // face right-hand side and solution after the basis in the Krylov workspace
    for (int r = 0; r < nrhs && (rc == HPS_OK || rc == HPS_NOT_CONVERGED); ++r) {
      int r1 = ws_reserve(c, &c->w_op, sizeof(double2) * 2 * nf);
      if (r1) { rc = r1; break; }
      double2* rf = static_cast<double2*>(c->w_op.ptr);
      double2* ff = rf + nf;
      if ((r1 = iti_prepare(c, bvec + (size_t)r * c->N, 1, rf))) { rc = r1; break; }
      job.rhs_res = o.rhs_rel_res ? o.rhs_rel_res + r : nullptr;
      hps_stats one{};
      r1 = run_solver(c, job, rf, ff, tol, restart, maxit, 0, check_every, o.orth, &one);
      if (r1 < 0) { rc = r1; break; }
      if (r1 == HPS_NOT_CONVERGED) rc = r1;
      // the workspace of iti_prepare (v, F_bi v) is untouched by the solve
      if ((r1 = iti_finish(c, ff, x + (size_t)r * c->N, 1))) { rc = r1; break; }
      acc.iters += one.iters;
      acc.restarts += one.restarts;
      acc.rel_res = std::max(acc.rel_res, one.rel_res);
      acc.true_rel_res = std::max(acc.true_rel_res, one.true_rel_res);
      acc.t_solve += one.t_solve;
      acc.bytes_apply = one.bytes_apply;
      acc.bytes_precond = one.bytes_precond;
    }
    acc.converged = rc == HPS_OK;
    acc.lambda_shifted = c->n_shifted;
      acc.t_setup = c->t_setup;
    if (st) *st = acc;
  } else if (rc == HPS_OK && o.solver == HPS_SOLVER_IR) {
    const double itol = o.inner_tol > 0.0 ? o.inner_tol : 1e-3;
    hps_stats acc{};
    for (int r = 0; r < nrhs; ++r) {
      hps_stats one{};
      const int r1 = run_ir(c, bvec + (size_t)r * c->N, x + (size_t)r * c->N, tol, restart, maxit,
                            o.use_x0, check_every, itol, o.rhs_rel_res ? o.rhs_rel_res + r : nullptr,
                            &one);
      if (r1 < 0) { rc = r1; break; }
      if (r1 == HPS_NOT_CONVERGED) rc = r1;
      acc.iters += one.iters;
      acc.restarts += one.restarts;
      acc.rel_res = std::max(acc.rel_res, one.rel_res);
      acc.true_rel_res = std::max(acc.true_rel_res, one.true_rel_res);
      acc.t_solve += one.t_solve;
      acc.bytes_apply = one.bytes_apply;
      acc.bytes_precond = one.bytes_precond;
    }
    acc.converged = rc == HPS_OK;
    acc.lambda_shifted = c->n_shifted;
    acc.t_setup = c->t_setup;
    if (st) *st = acc;
  } else if (rc == HPS_OK && o.solver == HPS_SOLVER_BGMRES) {
    rc = run_block_gmres(c, prec, bvec, x, nrhs, tol, restart, maxit, o.use_x0 != 0, o.rhs_rel_res, st);
    if (st) {
      Job job;
      job.flexible = false;
      job.prec = prec;
      job.n = c->N;
      job.nrhs = nrhs;
      solve_bytes_stats(c, job, nrhs, st);
    }
  } else if (rc == HPS_OK) {
    Job job;
    job.flexible = (o.solver == HPS_SOLVER_FGMRES) || prec != kFP64;
    job.prec = prec;
    job.n = c->N;
    // operator groups always run their right-hand sides in lock step (one per
    // operator), and so does flexible GMRES on several right-hand sides (the
    // same iterations as one at a time)
    if (o.solver == HPS_SOLVER_BLOCK || c->nop > 1 || (o.solver == HPS_SOLVER_FGMRES && nrhs > 1)) {
      hps_stats acc{};
      for (int r0 = 0; r0 < nrhs && (rc == HPS_OK || rc == HPS_NOT_CONVERGED); r0 += kMaxBatch) {
        job.nrhs = std::min(kMaxBatch, nrhs - r0);
        job.rhs_res = o.rhs_rel_res ? o.rhs_rel_res + r0 : nullptr;
        hps_stats one{};
        const int r1 = run_solver(c, job, bvec + (size_t)r0 * c->N, x + (size_t)r0 * c->N, tol,
                                  restart, maxit, o.use_x0, check_every, o.orth, &one);
        if (r1 < 0) { rc = r1; break; }
        if (r1 == HPS_NOT_CONVERGED) rc = r1;
        acc.iters = std::max(acc.iters, one.iters);
        acc.restarts = std::max(acc.restarts, one.restarts);
        acc.rel_res = std::max(acc.rel_res, one.rel_res);
        acc.true_rel_res = std::max(acc.true_rel_res, one.true_rel_res);
        acc.t_solve += one.t_solve;
        acc.bytes_apply = one.bytes_apply;
        acc.bytes_precond = one.bytes_precond;
      }
      acc.converged = rc == HPS_OK;
      acc.lambda_shifted = c->n_shifted;
      acc.t_setup = c->t_setup;
      if (st) *st = acc;
    } else {
      job.nrhs = 1;
      hps_stats acc{};
      for (int r = 0; r < nrhs; ++r) {
        job.rhs_res = o.rhs_rel_res ? o.rhs_rel_res + r : nullptr;
        hps_stats one{};
        const int r1 = run_solver(c, job, bvec + (size_t)r * c->N, x + (size_t)r * c->N, tol,
                                  restart, maxit, o.use_x0, check_every, o.orth, &one);
        if (r1 < 0) { rc = r1; break; }
        if (r1 == HPS_NOT_CONVERGED) rc = r1;
        acc.iters += one.iters;
        acc.restarts += one.restarts;
        acc.rel_res = std::max(acc.rel_res, one.rel_res);
        acc.true_rel_res = std::max(acc.true_rel_res, one.true_rel_res);
        acc.t_solve += one.t_solve;
        acc.bytes_apply = one.bytes_apply;
        acc.bytes_precond = one.bytes_precond;
      }
      acc.converged = rc == HPS_OK;
      acc.lambda_shifted = c->n_shifted;
      acc.t_setup = c->t_setup;
      if (st) *st = acc;
    }
  }
  const int rs = check_hip(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return rc != HPS_OK && rc != HPS_NOT_CONVERGED ? rc : (rs ? rs : rc);
}
