// Right-hand side assembly (Sec. 3.1): the global vector b carries s at the
// interior nodes of every leaf, t at face nodes on the boundary of the domain,
// and zero at interface face nodes (the rows that enforce f^alpha = -g^beta).
#include "hps_internal.h"
#include "k_common.h"

namespace hps {
namespace {

__global__ void k_assemble_rhs(const double2* __restrict__ s, const double2* __restrict__ t,
                               double2* __restrict__ b, const int* __restrict__ nbr, int ni, int n,
                               int L, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t off = (int64_t)blockIdx.y * N + i;
  const int64_t tau = i / n;
  const int m = (int)(i - tau * n);
  double2 v;
  if (m < ni) {
    v = s[off];
  } else {
    const int f = (m - ni) / L;
    v = (t && nbr[tau * 6 + f] < 0) ? t[off] : make_double2(0.0, 0.0);   // t null: no boundary data
  }
  b[off] = v;
}

}  // namespace

int launch_assemble_rhs(hps_ctx* c, const double2* s, const double2* t, double2* b, int nrhs) {
  const int threads = 256;
  hipLaunchKernelGGL(k_assemble_rhs, dim3((unsigned)((c->N + threads - 1) / threads), nrhs),
                     dim3(threads), 0, c->stream, s, t, b, c->d_nbr, c->ni, c->n, c->n1 * c->n1,
                     c->N);
  return check_hip(hipGetLastError(), "k_assemble_rhs");
}

}  // namespace hps
