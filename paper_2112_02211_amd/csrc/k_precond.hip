// y = J^{-1} x: the homogenized block-Jacobi preconditioner (Sec. 4, eq.
// (block_pc), Algorithm 4).  J^{-1} is block diagonal; on each leaf it is the
// exact inverse of the homogenized leaf matrix [[A~_ii, A_ib], [F_bi, F_bb]]:
//
//   f_i = A~_ii^{-1} x_i                  (Algorithm 3: fast diagonalization)
//   h_b = x_b - F_bi f_i
//   u_b = S~^{-1} h_b                     (dense n_b x n_b block, streamed)
//   y_i = f_i - A~_ii^{-1} (A_ib u_b),    y_b = u_b
//
// (Algorithm 4 as printed returns -u_b on the faces; the signs above are the
// ones of eq. (block_pc), i.e. the exact block solve.)
//
// One workgroup per leaf.  Algorithm 3 runs in LDS as line-wise mode products:
// a thread owns one grid line per axis, keeps its n1 values in registers and
// multiplies them by V^{-1} (or V), so each mode product reads and writes the
// tensor once.  The block product streams S~^{-1} from HBM with one row per
// thread: the block is stored column-group major ([col group][row][cw]), so a
// wavefront's 16-byte loads for one column group are contiguous, and h_b is
// broadcast from LDS.  No cross-lane reduction is needed.
#include "hps_internal.h"
#include "k_precond_fused.h"

namespace hps {
namespace {

template <int P>
int precond_launch(hps_ctx* c, const double2* x, const double2* g, double2* y, int nrhs, int prec,
                   hipEvent_t e0, hipEvent_t e1) {
  const Blocks& B = c->blk[prec];
  const dim3 grid((unsigned)c->nl, (unsigned)nrhs);
  const dim3 block(PL<P>::BD);
  const void* blk = B.data;
  const int* nbr = c->d_nbr;
  const int64_t os = c->nop > 1 ? c->nl : 0;   // operator groups: blocks and lambda per operator
  hipError_t e;
  switch (prec) {
    case kFP64:
      e = launch_k(c, e0, e1, k_precond_fused<P, kFP64>, grid, block, x, g, nbr, y, blk, B.ncp,
                   c->d_lambda, c->d_tab, c->nl, c->N, os);
      break;
    case kFP32:
      e = launch_k(c, e0, e1, k_precond_fused<P, kFP32>, grid, block, x, g, nbr, y, blk, B.ncp,
                   c->d_lambda, c->d_tab, c->nl, c->N, os);
      break;
    default:
      e = launch_k(c, e0, e1, k_precond_fused<P, kBF16>, grid, block, x, g, nbr, y, blk, B.ncp,
                   c->d_lambda, c->d_tab, c->nl, c->N, os);
      break;
  }
  return check_hip(e, "k_precond_fused");
}

}  // namespace

int launch_precond_fused(hps_ctx* c, const double2* x, const double2* g, double2* y, int nrhs,
                         int prec, hipEvent_t e0, hipEvent_t e1) {
  if (prec < 0 || prec > 2 || !c->blk[prec].data)
    return fail(HPS_ERR_ARG, "requested block precision was not built at setup");
  // the fused kernel reads block tau (+ nl * operator) for leaf tau: one block per leaf only
  if (c->nblocks != c->nl) return fail(HPS_ERR_ARG, "fused J^-1 needs one block per leaf");
  if (c->nop > 1 && nrhs != c->nop) return fail(HPS_ERR_ARG, "operator group: one right-hand side per operator");
  switch (c->p) {
    case 4: return precond_launch<4>(c, x, g, y, nrhs, prec, e0, e1);
    case 5: return precond_launch<5>(c, x, g, y, nrhs, prec, e0, e1);
    case 6: return precond_launch<6>(c, x, g, y, nrhs, prec, e0, e1);
    case 7: return precond_launch<7>(c, x, g, y, nrhs, prec, e0, e1);
    case 8: return precond_launch<8>(c, x, g, y, nrhs, prec, e0, e1);
    case 9: return precond_launch<9>(c, x, g, y, nrhs, prec, e0, e1);
    case 10: return precond_launch<10>(c, x, g, y, nrhs, prec, e0, e1);
    case 11: return precond_launch<11>(c, x, g, y, nrhs, prec, e0, e1);
    case 12: return precond_launch<12>(c, x, g, y, nrhs, prec, e0, e1);
    case 13: return precond_launch<13>(c, x, g, y, nrhs, prec, e0, e1);
    case 14: return precond_launch<14>(c, x, g, y, nrhs, prec, e0, e1);
    case 15: return precond_launch<15>(c, x, g, y, nrhs, prec, e0, e1);
    case 16: return precond_launch<16>(c, x, g, y, nrhs, prec, e0, e1);
    default: return fail(HPS_ERR_UNSUPPORTED, "p out of range");
  }
}

int launch_precond(hps_ctx* c, const double2* x, double2* y, int nrhs, int prec) {
  if (prec == kFP64 && c->sep) {
    TimedPair tp;
    int rc = timing_pair(c, 1, &tp);
    if (rc) return rc;
    if ((rc = launch_precond_sep(c, x, nullptr, y, nrhs, tp.start, tp.stop))) {
      timing_drop(c, tp);
      return rc;
    }
    return timing_commit(c, 1, tp);
  }
  if (prec < 0 || prec > 2 || !c->blk[prec].data)
    return fail(HPS_ERR_ARG, "requested block precision was not built at setup");
  TimedPair tp;
  int rc = timing_pair(c, 1, &tp);
  if (rc) return rc;
  // the GEMM path shares one block across right-hand sides: not for operator groups
  if ((nrhs >= kBatchedMinRhs || c->lambda_bucket > 0.0) && c->nop == 1)
    rc = launch_precond_batched(c, x, y, nrhs, prec, tp.start, tp.stop);
  else rc = launch_precond_fused(c, x, nullptr, y, nrhs, prec, tp.start, tp.stop);
  if (rc) {
    timing_drop(c, tp);
    return rc;
  }
  return timing_commit(c, 1, tp);
}

int launch_op_left(hps_ctx* c, const double2* x, double2* tmp, double2* y, int nrhs, int prec) {
  int rc;
  const bool sep = prec == kFP64 && c->sep;
  if (!sep && (nrhs >= kBatchedMinRhs || c->lambda_bucket > 0.0) && c->nop == 1) {
    if ((rc = launch_apply(c, x, tmp, nrhs))) return rc;
    return launch_precond(c, tmp, y, nrhs, prec);
  }
  if (!sep && (prec < 0 || prec > 2 || !c->blk[prec].data))
    return fail(HPS_ERR_ARG, "requested block precision was not built at setup");
  if ((rc = ws_reserve(c, &c->w_g, (size_t)nrhs * c->nl * c->nb * sizeof(double2)))) return rc;
  double2* g = static_cast<double2*>(c->w_g.ptr);
  TimedPair ta, tp;
  if ((rc = timing_pair(c, 0, &ta))) return rc;
  if ((rc = launch_sweep(c, x, tmp, g, nrhs, ta.start, ta.stop))) {
    timing_drop(c, ta);
    return rc;
  }
  if ((rc = timing_commit(c, 0, ta))) return rc;
  if ((rc = timing_pair(c, 1, &tp))) return rc;
  if ((rc = sep ? launch_precond_sep(c, tmp, g, y, nrhs, tp.start, tp.stop)
                : launch_precond_fused(c, tmp, g, y, nrhs, prec, tp.start, tp.stop))) {
    timing_drop(c, tp);
    return rc;
  }
  return timing_commit(c, 1, tp);
}

int launch_op_left(hps_ctx* c, const float2* x, float2* tmp, float2* y, int nrhs) {
  if (!c->sep) return fail(HPS_ERR_ARG, "vectors in FP32 need the separable J^-1");
  int rc = ws_reserve(c, &c->w_g, (size_t)nrhs * c->nl * c->nb * sizeof(float2));
  if (rc) return rc;
  float2* g = static_cast<float2*>(c->w_g.ptr);
  TimedPair ta, tp;
  if ((rc = timing_pair(c, 0, &ta))) return rc;
  if ((rc = launch_sweep(c, x, tmp, g, nrhs, ta.start, ta.stop))) {
    timing_drop(c, ta);
    return rc;
  }
  if ((rc = timing_commit(c, 0, ta))) return rc;
  if ((rc = timing_pair(c, 1, &tp))) return rc;
  if ((rc = launch_precond_sep(c, tmp, g, y, nrhs, tp.start, tp.stop))) {
    timing_drop(c, tp);
    return rc;
  }
  return timing_commit(c, 1, tp);
}

int launch_precond(hps_ctx* c, const float2* x, float2* y, int nrhs) {
  if (!c->sep) return fail(HPS_ERR_ARG, "vectors in FP32 need the separable J^-1");
  return launch_precond_sep(c, x, static_cast<const float2*>(nullptr), y, nrhs, nullptr, nullptr);
}

}  // namespace hps
