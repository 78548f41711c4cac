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
