// C-ABI entry points: context setup and teardown, node table, and the
// stream-ordered wrappers of the hot-path operators.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <vector>

#include "hps_internal.h"
#include "hps_krylov.h"
#include "k_common.h"

namespace hps {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return HPS_OK;
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return (e == hipErrorOutOfMemory) ? HPS_ERR_OOM : HPS_ERR_DEVICE;
}

int dev_alloc(hps_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return HPS_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? HPS_ERR_OOM : HPS_ERR_DEVICE,
                "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  c->dev_bytes += bytes;
  return HPS_OK;
}

int ws_reserve(hps_ctx* c, Workspace* w, size_t bytes) {
  if (w->bytes >= bytes) return HPS_OK;
  if (w->ptr) {
    HPS_TRY_HIP(hipStreamSynchronize(c->stream));
    HPS_TRY_HIP(hipFree(w->ptr));
    c->dev_bytes -= w->bytes;
    w->ptr = nullptr;
    w->bytes = 0;
  }
  int rc = dev_alloc(c, &w->ptr, bytes);
  if (rc) return rc;
  w->bytes = bytes;
  return HPS_OK;
}

int timing_pair(hps_ctx* c, int kind, TimedPair* tp) {
  tp->start = tp->stop = nullptr;
  if (!c->timing) return HPS_OK;
  if (kind < 0 || kind >= kTimingKinds) return fail(HPS_ERR_ARG, "timing kind out of range");
  if (c->t_seq[kind]++ % c->timing != 0) return HPS_OK;  // not sampled
  while (c->ev_free.size() < 2) {
    hipEvent_t e;
    HPS_TRY_HIP(hipEventCreate(&e));
    c->ev_free.push_back(e);
  }
  tp->start = c->ev_free.back();
  c->ev_free.pop_back();
  tp->stop = c->ev_free.back();
  c->ev_free.pop_back();
  return HPS_OK;
}

void timing_drop(hps_ctx* c, const TimedPair& tp) {
  if (tp.start) c->ev_free.push_back(tp.start);
  if (tp.stop) c->ev_free.push_back(tp.stop);
}

int timing_commit(hps_ctx* c, int kind, const TimedPair& tp, double bytes) {
  if (!tp.start) return HPS_OK;
  if (kind < 0 || kind >= kTimingKinds) {
    c->ev_free.push_back(tp.start);
    c->ev_free.push_back(tp.stop);
    return fail(HPS_ERR_ARG, "timing kind out of range");
  }
  c->ev_pending[kind].emplace_back(tp.start, tp.stop);
  c->ev_bytes[kind].push_back(bytes);
  if (c->ev_pending[kind].size() >= 4096) return timing_collect(c);
  return HPS_OK;
}

int timing_collect(hps_ctx* c) {
  static_assert(sizeof(c->ev_pending) / sizeof(c->ev_pending[0]) == kTimingKinds, "timing kinds");
  int rc = HPS_OK;
  for (int k = 0; k < kTimingKinds; ++k) {
    for (size_t i = 0; i < c->ev_pending[k].size(); ++i) {
      auto& pr = c->ev_pending[k][i];
      if (rc == HPS_OK) {
        float ms = 0.f;
        rc = check_hip(hipEventSynchronize(pr.second), "hipEventSynchronize");
        if (rc == HPS_OK) rc = check_hip(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
        if (rc == HPS_OK) {
          c->t_ms[k] += ms;
          c->t_cnt[k] += 1.0;
          c->t_bytes[k] += c->ev_bytes[k][i];
        }
      }
      // every event goes back to the pool exactly once, also after an error
      c->ev_free.push_back(pr.first);
      c->ev_free.push_back(pr.second);
    }
    c->ev_pending[k].clear();
    c->ev_bytes[k].clear();
  }
  return rc;
}

namespace {

int prec_index(int prec_flag) {
  switch (prec_flag) {
    case HPS_PREC_FP64: return kFP64;
    case HPS_PREC_FP32: return kFP32;
    case HPS_PREC_BF16: return kBF16;
    case HPS_PREC_SEPARABLE: return kFP64;
    default: return -1;
  }
}

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Lambda buckets: leaves whose (rounded, guarded) lambda are equal share one
// block.  Buckets are numbered in order of their first leaf; d_bpos gives each
// leaf's position when the leaves are sorted by bucket (stable in leaf order).
int make_buckets(hps_ctx* c) {
  const int64_t nl = c->nl;
  std::vector<double2> lam(nl);
  HPS_TRY_HIP(hipMemcpyAsync(lam.data(), c->d_lambda, sizeof(double2) * nl, hipMemcpyDeviceToHost,
                             c->stream));
  HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  auto less = [](const std::pair<double, double>& a, const std::pair<double, double>& b) {
    return a.first < b.first || (a.first == b.first && a.second < b.second);
  };
  std::map<std::pair<double, double>, int, decltype(less)> id(less);
  std::vector<int> bkt(nl), count;
  std::vector<double2> blam;
  for (int64_t t = 0; t < nl; ++t) {
    const auto key = std::make_pair(lam[t].x, lam[t].y);
    auto it = id.find(key);
    if (it == id.end()) {
      it = id.emplace(key, (int)blam.size()).first;
      blam.push_back(lam[t]);
      count.push_back(0);
    }
    bkt[t] = it->second;
    ++count[it->second];
  }
  const int nbk = (int)blam.size();
  std::vector<int> bofs(nbk + 1, 0), fill(nbk, 0), pos(nl);
  for (int b = 0; b < nbk; ++b) bofs[b + 1] = bofs[b] + count[b];
  for (int64_t t = 0; t < nl; ++t) pos[t] = bofs[bkt[t]] + fill[bkt[t]]++;
  // GEMM groups: each bucket's positions in runs of at most kGroupLeaves
  std::vector<int> gofs(1, 0), gblk;
  int group_leaves = 1;
  for (int b = 0; b < nbk; ++b)
    for (int s = bofs[b]; s < bofs[b + 1]; s += kGroupLeaves) {
      const int e = std::min(bofs[b + 1], s + kGroupLeaves);
      gofs.push_back(e);
      gblk.push_back(b);
      group_leaves = std::max(group_leaves, e - s);
    }
  const int ng = (int)gblk.size();
  int rc;
  if ((rc = dev_alloc(c, (void**)&c->d_bpos, sizeof(int) * nl))) return rc;
  if ((rc = dev_alloc(c, (void**)&c->d_blam, sizeof(double2) * nbk))) return rc;
  if ((rc = dev_alloc(c, (void**)&c->d_gofs, sizeof(int) * (ng + 1)))) return rc;
  if ((rc = dev_alloc(c, (void**)&c->d_gblk, sizeof(int) * ng))) return rc;
  HPS_TRY_HIP(hipMemcpyAsync(c->d_bpos, pos.data(), sizeof(int) * nl, hipMemcpyHostToDevice, c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(c->d_blam, blam.data(), sizeof(double2) * nbk, hipMemcpyHostToDevice,
                             c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(c->d_gofs, gofs.data(), sizeof(int) * (ng + 1), hipMemcpyHostToDevice,
                             c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(c->d_gblk, gblk.data(), sizeof(int) * ng, hipMemcpyHostToDevice, c->stream));
  HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  c->nblocks = nbk;
  c->ngroups = ng;
  c->group_leaves = group_leaves;
  return HPS_OK;
}

// Inverse of every homogenized Schur complement S~^tau, packed per precision.
int build_blocks(hps_ctx* c, int precs) {
  const int nb = c->nb;
  for (int q = 0; q < 3; ++q) {
    if (!(precs & (1 << q))) continue;
    const int cw = block_cw(q);
    Blocks& B = c->blk[q];
    B.ncp = (nb + cw - 1) / cw * cw;
    B.bytes = (size_t)c->nblocks * c->nop * B.ncp * nb * (q == kFP64 ? 16 : (q == kFP32 ? 8 : 4));
    int rc = dev_alloc(c, &B.data, B.bytes);
    if (rc) return rc;
  }
  // shared real factors P, Q on the device
  double *dP = nullptr, *dQ = nullptr;
  int rc = dev_alloc(c, (void**)&dP, sizeof(double) * c->tab.P.size());
  if (rc) return rc;
  rc = dev_alloc(c, (void**)&dQ, sizeof(double) * c->tab.Q.size());
  if (rc) return rc;
  HPS_TRY_HIP(hipMemcpyAsync(dP, c->tab.P.data(), sizeof(double) * c->tab.P.size(),
                             hipMemcpyHostToDevice, c->stream));
  HPS_TRY_HIP(hipMemcpyAsync(dQ, c->tab.Q.data(), sizeof(double) * c->tab.Q.size(),
                             hipMemcpyHostToDevice, c->stream));
  const size_t blk_bytes = (size_t)nb * nb * sizeof(double2);
  int64_t chunk = (int64_t)((1ull << 30) / blk_bytes);
  if (chunk < 1) chunk = 1;
  if (chunk > c->nblocks) chunk = c->nblocks;
  // one block per leaf, or per lambda bucket
  const double2* lam = c->lambda_bucket > 0.0 ? c->d_blam : c->d_lambda;
  double2* S = nullptr;
  rocblas_int *ipiv = nullptr, *info = nullptr;
  rc = dev_alloc(c, (void**)&S, blk_bytes * chunk);
  if (rc) return rc;
  rc = dev_alloc(c, (void**)&ipiv, sizeof(rocblas_int) * nb * chunk);
  if (rc) return rc;
  rc = dev_alloc(c, (void**)&info, sizeof(rocblas_int) * chunk);
  if (rc) return rc;
  rocblas_handle handle;
  if (rocblas_create_handle(&handle) != rocblas_status_success)
    return fail(HPS_ERR_DEVICE, "rocblas_create_handle failed");
  rocblas_set_stream(handle, c->stream);
  std::vector<rocblas_int> hinfo(chunk);
  int status = HPS_OK;
  // operator by operator (each with its own eta); blocks of operator op start at op * nblocks
  const double eta0 = c->eta;
  for (int op = 0; op < c->nop && status == HPS_OK; ++op) {
  c->eta = c->etas.empty() ? eta0 : c->etas[op];
  const double2* lam_op = lam + (int64_t)op * c->nblocks;
  for (int64_t e0 = 0; e0 < c->nblocks && status == HPS_OK; e0 += chunk) {
    const int ne = (int)std::min<int64_t>(chunk, c->nblocks - e0);
    status = launch_build_schur(c, dP, dQ, lam_op, (int)e0, ne, S);
    if (status) break;
    auto* A = reinterpret_cast<rocblas_double_complex*>(S);
    if (rocsolver_zgetrf_strided_batched(handle, nb, nb, A, nb, (rocblas_stride)nb * nb, ipiv, nb,
                                         info, ne) != rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocsolver getrf failed");
      break;
    }
    hipMemcpyAsync(hinfo.data(), info, sizeof(rocblas_int) * ne, hipMemcpyDeviceToHost, c->stream);
    hipStreamSynchronize(c->stream);
    for (int i = 0; i < ne; ++i)
      if (hinfo[i] != 0) {
        status = fail(HPS_ERR_NUMERIC, std::string("homogenized Schur complement of ") +
                                           (c->lambda_bucket > 0.0 ? "bucket " : "leaf ") +
                                           std::to_string(e0 + i) +
                                           (c->nop > 1 ? " of operator " + std::to_string(op) : "") +
                                           " is singular");
        break;
      }
    if (status) break;
    if (rocsolver_zgetri_strided_batched(handle, nb, A, nb, (rocblas_stride)nb * nb, ipiv, nb, info,
                                         ne) != rocblas_status_success) {
      status = fail(HPS_ERR_DEVICE, "rocsolver getri failed");
      break;
    }
    for (int q = 0; q < 3 && status == HPS_OK; ++q)
      if (c->blk[q].data) status = launch_pack_blocks(c, S, (int)(op * c->nblocks + e0), ne, q);
  }
  }
  c->eta = eta0;
  hipStreamSynchronize(c->stream);
  rocblas_destroy_handle(handle);
  hipFree(S);
  hipFree(ipiv);
  hipFree(info);
  hipFree(dP);
  hipFree(dQ);
  c->dev_bytes -= blk_bytes * chunk + sizeof(rocblas_int) * (nb + 1) * chunk +
                  sizeof(double) * (c->tab.P.size() + c->tab.Q.size());
  if (status == HPS_OK) status = check_hip(hipGetLastError(), "block build");
  return status;
}

}  // namespace
}  // namespace hps

using namespace hps;

extern "C" {

const char* hps_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// Setup of nop operators on one mesh (nop = 1: hps_setup).  media: nop entries or NULL.
int setup_impl(const hps_domain* d, int nop, const double* kappas, const double* etas,
               const hps_medium* media, int p, int q, const int n_elem[3], const hps_opts* o,
               hps_ctx** out) {
  g_err.clear();
  if (!out) return fail(HPS_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!d || !n_elem) return fail(HPS_ERR_ARG, "domain or n_elem is NULL");
  if (p < kMinP || p > kMaxP) return fail(HPS_ERR_UNSUPPORTED, "p must lie in [4, 16]");
  if (q != p - 2) return fail(HPS_ERR_UNSUPPORTED, "q must equal p - 2 (face nodes are the interior Chebyshev nodes of each face)");
  for (int op = 0; op < nop; ++op) {
    const double kappa = kappas[op], eta = etas[op];
    if (!(kappa > 0.0) || !std::isfinite(kappa) || !std::isfinite(eta) || eta == 0.0)
      return fail(HPS_ERR_ARG, "kappa must be positive and eta nonzero");
  }
  if (o && (!(o->lambda_bucket >= 0.0) || !std::isfinite(o->lambda_bucket)))
    return fail(HPS_ERR_ARG, "lambda_bucket must be a finite number >= 0");
  if (nop > 1 && o && o->lambda_bucket > 0.0)
    return fail(HPS_ERR_UNSUPPORTED, "lambda buckets are not available for operator groups");
  double hs[3];
  for (int a = 0; a < 3; ++a) {
    if (n_elem[a] < 1) return fail(HPS_ERR_ARG, "n_elem must be >= 1");
    hs[a] = (d->hi[a] - d->lo[a]) / n_elem[a];
    if (!(hs[a] > 0.0)) return fail(HPS_ERR_ARG, "empty domain");
  }
  if (std::fabs(hs[1] - hs[0]) > 1e-12 * hs[0] || std::fabs(hs[2] - hs[0]) > 1e-12 * hs[0])
    return fail(HPS_ERR_ARG, "leaves must be cubes");
  for (int op = 0; op < nop; ++op) {
    const hps_medium* b = media ? &media[op] : nullptr;
    if (b && b->kind == HPS_MEDIUM_BUMPS && b->n_bumps > 0 &&
        (!b->centres || !b->amps || !(b->width > 0.0)))
      return fail(HPS_ERR_ARG, "bump medium needs centres, amplitudes and a positive width");
    if (b && b->kind == HPS_MEDIUM_NODAL && !b->nodal) return fail(HPS_ERR_ARG, "nodal medium is NULL");
    if (b && (b->kind < 0 || b->kind > 2)) return fail(HPS_ERR_ARG, "unknown medium kind");
  }
  const int precs = (o && o->block_precs) ? o->block_precs : HPS_PREC_FP64;
  if (precs & ~15) return fail(HPS_ERR_ARG, "unknown block precision bits");
  if ((precs & HPS_PREC_SEPARABLE) && (precs & HPS_PREC_FP64))
    return fail(HPS_ERR_ARG, "HPS_PREC_SEPARABLE replaces the FP64 blocks (do not set both)");
  if ((precs & HPS_PREC_SEPARABLE) && o && o->lambda_bucket > 0.0)
    return fail(HPS_ERR_ARG, "lambda buckets share dense blocks; the separable J^-1 has none");

  const double t0 = now();
  hps_ctx* c = new hps_ctx();
  c->p = p;
  c->n1 = p - 2;
  c->ni = c->n1 * c->n1 * c->n1;
  c->nb = 6 * c->n1 * c->n1;
  c->n = c->ni + c->nb;
  for (int a = 0; a < 3; ++a) { c->E[a] = n_elem[a]; c->lo[a] = d->lo[a]; }
  c->nl = (int64_t)n_elem[0] * n_elem[1] * n_elem[2];
  c->N = c->nl * c->n;
  c->nop = nop;
  c->kappas.assign(kappas, kappas + nop);
  c->etas.assign(etas, etas + nop);
  c->kappa = kappas[0];
  c->eta = etas[0];
  c->h = hs[0];
  c->stream = o ? static_cast<hipStream_t>(o->stream) : nullptr;
  c->verbose = o ? o->verbose : 0;
  c->lambda_bucket = o ? o->lambda_bucket : 0.0;
  c->nblocks = c->nl;
  hipGetDevice(&c->device);

  auto bail = [&](int rc) {
    hps_free(c);
    return rc;
  };
  std::string err = build_tables(p, c->h, &c->tab);
  if (!err.empty()) return bail(fail(HPS_ERR_NUMERIC, err));

  // packed table D | D2 | V | W | E | xi | Ed3
  std::vector<double> tab(tab_size(p), 0.0);
  std::copy(c->tab.D.begin(), c->tab.D.end(), tab.begin() + tab_off_D(p));
  std::copy(c->tab.D2.begin(), c->tab.D2.end(), tab.begin() + tab_off_D2(p));
  std::copy(c->tab.V.begin(), c->tab.V.end(), tab.begin() + tab_off_V(p));
  std::copy(c->tab.W.begin(), c->tab.W.end(), tab.begin() + tab_off_W(p));
  std::copy(c->tab.E.begin(), c->tab.E.end(), tab.begin() + tab_off_E(p));
  std::copy(c->tab.xi.begin(), c->tab.xi.end(), tab.begin() + tab_off_xi(p));
  const int n1 = c->n1;
  for (int k = 0; k < n1; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i)
        tab[tab_off_ed3(p) + i + n1 * (j + n1 * k)] = c->tab.E[i] + c->tab.E[j] + c->tab.E[k];
  // the static face buffer of hps_apply_noalloc on this device
  int rc = scratch_address(&c->d_scratch);
  if (rc) return bail(rc);
  if ((rc = dev_alloc(c, (void**)&c->d_tab, sizeof(double) * tab.size()))) return bail(rc);
  if ((rc = check_hip(hipMemcpyAsync(c->d_tab, tab.data(), sizeof(double) * tab.size(),
                                     hipMemcpyHostToDevice, c->stream), "upload tables")))
    return bail(rc);
  c->dt = DevTables{c->d_tab + tab_off_D(p), c->d_tab + tab_off_D2(p), c->d_tab + tab_off_V(p),
                    c->d_tab + tab_off_W(p), c->d_tab + tab_off_E(p)};

  // neighbour table, leaves numbered x fastest
  std::vector<int> nbr(c->nl * 6);
  for (int64_t t = 0; t < c->nl; ++t) {
    const int e[3] = {(int)(t % c->E[0]), (int)((t / c->E[0]) % c->E[1]),
                      (int)(t / ((int64_t)c->E[0] * c->E[1]))};
    for (int f = 0; f < 6; ++f) {
      int g[3] = {e[0], e[1], e[2]};
      const int ax = face_axis(f);
      g[ax] += face_high(f) ? 1 : -1;
      nbr[t * 6 + f] = (g[ax] < 0 || g[ax] >= c->E[ax])
                           ? -1
                           : (int)(g[0] + (int64_t)c->E[0] * (g[1] + (int64_t)c->E[1] * g[2]));
    }
  }
  if ((rc = dev_alloc(c, (void**)&c->d_nbr, sizeof(int) * nbr.size()))) return bail(rc);
  if ((rc = check_hip(hipMemcpyAsync(c->d_nbr, nbr.data(), sizeof(int) * nbr.size(),
                                     hipMemcpyHostToDevice, c->stream), "upload neighbours")))
    return bail(rc);

  // medium: C = kappa^2 (1 - b) at interior nodes, and lambda^tau, operator by
  // operator into slices of C and lambda (C is complex for all if any needs it)
  c->c_complex = 0;
  for (int op = 0; op < nop; ++op) {
    const hps_medium* b = media ? &media[op] : nullptr;
    if (b && b->kind == HPS_MEDIUM_NODAL) c->c_complex = 1;
    if (b && b->kind == HPS_MEDIUM_BUMPS)
      for (int i = 0; i < b->n_bumps; ++i)
        if (b->amps[i].im != 0.0) c->c_complex = 1;
  }
  const size_t cslice = (size_t)c->nl * c->ni * (c->c_complex ? 16 : 8);
  if ((rc = dev_alloc(c, &c->d_C, cslice * nop))) return bail(rc);
  if ((rc = dev_alloc(c, (void**)&c->d_lambda, sizeof(double2) * c->nl * nop))) return bail(rc);
  void* const C0 = c->d_C;
  double2* const lam0 = c->d_lambda;
  int shifted = 0;
  for (int op = 0; op < nop && rc == HPS_OK; ++op) {
    const hps_medium* b = media ? &media[op] : nullptr;
    int nbump = 0;
    double* d_bc = nullptr;
    double2* d_ba = nullptr;
    if (b && b->kind == HPS_MEDIUM_BUMPS && b->n_bumps > 0) {
      nbump = b->n_bumps;
      if ((rc = dev_alloc(c, (void**)&d_bc, sizeof(double) * 3 * nbump))) break;
      if ((rc = dev_alloc(c, (void**)&d_ba, sizeof(double2) * nbump))) break;
      hipMemcpyAsync(d_bc, b->centres, sizeof(double) * 3 * nbump, hipMemcpyHostToDevice, c->stream);
      hipMemcpyAsync(d_ba, b->amps, sizeof(double2) * nbump, hipMemcpyHostToDevice, c->stream);
    }
    c->kappa = kappas[op];
    c->d_C = static_cast<char*>(C0) + cslice * op;
    c->d_lambda = lam0 + c->nl * op;
    rc = launch_eval_medium(c, b, d_bc, d_ba, nbump);
    if (!rc) rc = launch_lambda(c);
    shifted += c->n_shifted;
    hipStreamSynchronize(c->stream);
    if (d_bc) { hipFree(d_bc); c->dev_bytes -= sizeof(double) * 3 * nbump; }
    if (d_ba) { hipFree(d_ba); c->dev_bytes -= sizeof(double2) * nbump; }
  }
  c->d_C = C0;
  c->d_lambda = lam0;
  c->kappa = kappas[0];
  c->n_shifted = shifted;
  if (rc) return bail(rc);
  if (nop > 1) {
    if ((rc = dev_alloc(c, (void**)&c->d_eta, sizeof(double) * nop))) return bail(rc);
    if ((rc = check_hip(hipMemcpyAsync(c->d_eta, etas, sizeof(double) * nop, hipMemcpyHostToDevice,
                                       c->stream), "upload eta")))
      return bail(rc);
  }
  if (c->lambda_bucket > 0.0 && (rc = make_buckets(c))) return bail(rc);
  const double t1 = now();
  // separable form of the FP64 J^-1: one table per operator (its eta)
  if (precs & HPS_PREC_SEPARABLE) {
    const int ts = sep_table_size(p);
    std::vector<double> all((size_t)2 * ts * nop), one;
    for (int op = 0; op < nop; ++op) {
      err = build_sep_table(c->tab, etas[op], &one);
      if (!err.empty()) return bail(fail(HPS_ERR_NUMERIC, err));
      std::copy(one.begin(), one.end(), all.begin() + (size_t)2 * ts * op);
    }
    if ((rc = dev_alloc(c, (void**)&c->d_sep, sizeof(double) * all.size()))) return bail(rc);
    if ((rc = check_hip(hipMemcpyAsync(c->d_sep, all.data(), sizeof(double) * all.size(),
                                       hipMemcpyHostToDevice, c->stream), "upload separable tables")))
      return bail(rc);
    c->sep = 1;
  }
  // dense homogenized blocks
  int pb = 0;
  if (precs & HPS_PREC_FP64) pb |= 1 << kFP64;
  if (precs & HPS_PREC_FP32) pb |= 1 << kFP32;
  if (precs & HPS_PREC_BF16) pb |= 1 << kBF16;
  if (pb && (rc = build_blocks(c, pb))) return bail(rc);
  if ((rc = check_hip(hipStreamSynchronize(c->stream), "setup"))) return bail(rc);
  c->t_setup = now() - t0;
  if (c->verbose)
    std::fprintf(stderr, "[hps] setup: tables+medium %.3f s, blocks %.3f s, %.2f GB on device\n",
                 t1 - t0, now() - t1, c->dev_bytes / 1e9);
  *out = c;
  return HPS_OK;
}

}  // namespace

extern "C" {

int hps_setup(const hps_domain* d, double kappa, double eta, const hps_medium* b, int p, int q,
              const int n_elem[3], const hps_opts* o, hps_ctx** out) {
  return setup_impl(d, 1, &kappa, &eta, b, p, q, n_elem, o, out);
}

int hps_setup_group(const hps_domain* d, int nop, const double* kappa, const double* eta,
                    const hps_medium* media, int p, int q, const int n_elem[3], const hps_opts* o,
                    hps_ctx** out) {
  g_err.clear();
  if (out) *out = nullptr;
  if (nop < 1 || nop > kMaxBatch || !kappa || !eta)
    return fail(HPS_ERR_ARG, "hps_setup_group: needs 1 <= nop <= 64 and kappa, eta arrays");
  return setup_impl(d, nop, kappa, eta, media, p, q, n_elem, o, out);
}

int hps_num_operators(const hps_ctx* c) { return c ? c->nop : -1; }

int hps_set_timing(hps_ctx* c, int enable) {
  if (!c) return fail(HPS_ERR_ARG, "ctx is NULL");
  if (enable < 0) return fail(HPS_ERR_ARG, "timing period must be >= 0");
  c->timing = enable;
  for (int k = 0; k < kTimingKinds; ++k) c->t_seq[k] = 0;
  return HPS_OK;
}

int hps_kernel_times(hps_ctx* c, double out[8], int reset) {
  if (!c || !out) return fail(HPS_ERR_ARG, "NULL argument");
  int rc = timing_collect(c);
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) {
    out[2 * k] = c->t_ms[k];
    out[2 * k + 1] = c->t_cnt[k];
    if (reset) c->t_ms[k] = c->t_cnt[k] = c->t_bytes[k] = 0.0;
  }
  return HPS_OK;
}

int hps_arnoldi_times(hps_ctx* c, double out[3], int reset) {
  if (!c || !out) return fail(HPS_ERR_ARG, "NULL argument");
  int rc = timing_collect(c);
  if (rc) return rc;
  out[0] = c->t_ms[4];
  out[1] = c->t_cnt[4];
  out[2] = c->t_bytes[4];
  if (reset) c->t_ms[4] = c->t_cnt[4] = c->t_bytes[4] = 0.0;
  return HPS_OK;
}

void hps_free(hps_ctx* c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  for (auto& v : c->ev_pending)
    for (auto& pr : v) { hipEventDestroy(pr.first); hipEventDestroy(pr.second); }
  for (auto e : c->ev_free) hipEventDestroy(e);
  for (auto e : c->ev_solver)
    if (e) hipEventDestroy(e);
  hipFree(c->d_tab);
  hipFree(c->d_nbr);
  hipFree(c->d_C);
  hipFree(c->d_lambda);
  hipFree(c->d_eta);
  hipFree(c->d_bpos);
  hipFree(c->d_gofs);
  hipFree(c->d_gblk);
  hipFree(c->d_blam);
  for (auto& B : c->blk) hipFree(B.data);
  hipFree(c->d_sep);
  hipFree(c->d_itiR);
  hipFree(c->d_Ainv);
  hipFree(c->d_Fbi);
  hipFree(c->d_Aib);
  hipFree(c->w_iti.ptr);
  hipFree(c->w_g.ptr);
  hipFree(c->w_red.ptr);
  hipFree(c->w_krylov.ptr);
  hipFree(c->w_krylov32.ptr);
  hipFree(c->w_ir.ptr);
  hipFree(c->w_small.ptr);
  hipFree(c->w_batch.ptr);
  hipFree(c->w_op.ptr);
  hipFree(c->w_b.ptr);
  if (c->h_pinned) hipHostFree(c->h_pinned);
  delete c;
}

int64_t hps_num_unknowns(const hps_ctx* c) { return c ? c->N : -1; }

int64_t hps_num_blocks(const hps_ctx* c) { return c ? c->nblocks : -1; }

int hps_separable_table(int p, double h, double eta, double* out) {
  g_err.clear();
  if (!out) return fail(HPS_ERR_ARG, "out is NULL");
  if (p < kMinP || p > kMaxP) return fail(HPS_ERR_UNSUPPORTED, "p must lie in [4, 16]");
  if (!(h > 0.0) || !std::isfinite(h) || !std::isfinite(eta) || eta == 0.0)
    return fail(HPS_ERR_ARG, "h must be positive and eta finite and nonzero");
  HostTables t;
  std::string err = build_tables(p, h, &t);
  if (err.empty()) {
    std::vector<double> tab;
    err = build_sep_table(t, eta, &tab);
    if (err.empty()) std::copy(tab.begin(), tab.end(), out);
  }
  return err.empty() ? HPS_OK : fail(HPS_ERR_NUMERIC, err);
}

int64_t hps_setup_bytes(int p, const int n_elem[3], int block_precs, int complex_medium,
                        int64_t* transient) {
  if (p < kMinP || p > kMaxP || !n_elem) return fail(HPS_ERR_ARG, "bad sizes");
  for (int a = 0; a < 3; ++a)
    if (n_elem[a] < 1) return fail(HPS_ERR_ARG, "bad sizes");
  const int64_t n1 = p - 2, ni = n1 * n1 * n1, nb = 6 * n1 * n1;
  const int64_t nl = (int64_t)n_elem[0] * n_elem[1] * n_elem[2];
  const int precs = block_precs ? block_precs : HPS_PREC_FP64;
  int64_t bytes = (int64_t)sizeof(double) * tab_size(p) + (int64_t)sizeof(int) * 6 * nl +
                  nl * ni * (complex_medium ? 16 : 8) + 16 * nl;
  if (precs & HPS_PREC_SEPARABLE) bytes += 16 * (int64_t)sep_table_size(p);
  const int bits[3] = {HPS_PREC_FP64, HPS_PREC_FP32, HPS_PREC_BF16};
  for (int q = 0; q < 3; ++q) {
    if (!(precs & bits[q])) continue;
    const int64_t cw = block_cw(q);
    const int64_t ncp = (nb + cw - 1) / cw * cw;
    bytes += nl * ncp * nb * (q == kFP64 ? 16 : (q == kFP32 ? 8 : 4));
  }
  if (transient && !(precs & (HPS_PREC_FP64 | HPS_PREC_FP32 | HPS_PREC_BF16))) {
    *transient = 0;   // separable form only: no block build
  } else if (transient) {
    const int64_t blk = nb * nb * 16;
    int64_t chunk = (int64_t)((1ull << 30) / blk);
    if (chunk < 1) chunk = 1;
    if (chunk > nl) chunk = nl;
    // Schur chunk, pivots, P and Q, and room for the solver library's workspace
    *transient = chunk * (blk + 4 * (nb + 1)) + 16 * ni * nb + (int64_t)(256ll << 20);
  }
  return bytes;
}

int hps_trim(hps_ctx* c) {
  if (!c) return fail(HPS_ERR_ARG, "ctx is NULL");
  HPS_TRY_HIP(hipStreamSynchronize(c->stream));
  Workspace* ws[] = {&c->w_g, &c->w_red, &c->w_krylov, &c->w_krylov32, &c->w_ir, &c->w_small,
                     &c->w_batch, &c->w_op, &c->w_b, &c->w_iti};
  for (Workspace* w : ws) {
    if (w->ptr) {
      HPS_TRY_HIP(hipFree(w->ptr));
      c->dev_bytes -= w->bytes;
    }
    w->ptr = nullptr;
    w->bytes = 0;
  }
  return HPS_OK;
}

int64_t hps_device_bytes(const hps_ctx* c) { return c ? (int64_t)c->dev_bytes : -1; }

int hps_set_stream(hps_ctx* c, void* stream) {
  if (!c) return fail(HPS_ERR_ARG, "ctx is NULL");
  c->stream = static_cast<hipStream_t>(stream);
  return HPS_OK;
}

int hps_nodes(const hps_ctx* c, double* xyz) {
  if (!c || !xyz) return fail(HPS_ERR_ARG, "NULL argument");
  const int p = c->p, n1 = c->n1, L = n1 * n1;
  std::vector<int> gi(c->n * 3);
  for (int m = 0; m < c->n; ++m) {
    int g[3];
    if (m < c->ni) {
      g[0] = m % n1 + 1; g[1] = (m / n1) % n1 + 1; g[2] = m / L + 1;
    } else {
      const int mm = m - c->ni, f = mm / L, r = mm % L;
      const int ax = face_axis(f);
      int t1 = -1, t2 = -1;
      for (int a = 0; a < 3; ++a)
        if (a != ax) { if (t1 < 0) t1 = a; else t2 = a; }
      g[ax] = face_high(f) ? p - 1 : 0;
      g[t1] = r % n1 + 1;
      g[t2] = r / n1 + 1;
    }
    for (int a = 0; a < 3; ++a) gi[m * 3 + a] = g[a];
  }
  for (int64_t t = 0; t < c->nl; ++t) {
    const int64_t e[3] = {t % c->E[0], (t / c->E[0]) % c->E[1], t / ((int64_t)c->E[0] * c->E[1])};
    for (int m = 0; m < c->n; ++m)
      for (int a = 0; a < 3; ++a)
        xyz[(t * c->n + m) * 3 + a] =
            c->lo[a] + c->h * ((double)e[a] + 0.5 * (c->tab.xi[gi[m * 3 + a]] + 1.0));
  }
  return HPS_OK;
}

int hps_lambdas(const hps_ctx* c, hps_z* lam) {
  if (!c || !lam) return fail(HPS_ERR_ARG, "NULL argument");
  int rc = check_hip(hipMemcpyAsync(lam, c->d_lambda, sizeof(double2) * c->nl * c->nop,
                                    hipMemcpyDeviceToHost, c->stream), "lambda copy");
  if (rc) return rc;
  return check_hip(hipStreamSynchronize(c->stream), "lambda copy");
}

int hps_apply(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs) {
  if (!c || !x || !y || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_apply");
  return launch_apply(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), nrhs);
}

int hps_apply_noalloc(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs) {
  if (!c || !x || !y || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_apply_noalloc");
  return launch_apply_noalloc(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), nrhs);
}

int hps_precond_prec(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs, int prec) {
  if (!c || !x || !y || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_precond");
  const int q = prec_index(prec);
  if (q < 0) return fail(HPS_ERR_ARG, "unknown precision");
  return launch_precond(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), nrhs, q);
}

int hps_precond(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs) {
  return hps_precond_prec(c, x, y, nrhs, HPS_PREC_FP64);
}

int hps_op_left_f32(hps_ctx* c, const void* x, void* y, int nrhs) {
  if (!c || !x || !y || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_op_left_f32");
  if (c->nop > 1) return fail(HPS_ERR_ARG, "hps_op_left_f32: operator groups are not supported");
  int rc = ws_reserve(c, &c->w_op, sizeof(float2) * (size_t)c->N * nrhs);
  if (rc) return rc;
  return launch_op_left(c, static_cast<const float2*>(x), static_cast<float2*>(c->w_op.ptr),
                        static_cast<float2*>(y), nrhs);
}

int hps_precond_f32(hps_ctx* c, const void* x, void* y, int nrhs) {
  if (!c || !x || !y || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_precond_f32");
  if (c->nop > 1) return fail(HPS_ERR_ARG, "hps_precond_f32: operator groups are not supported");
  return launch_precond(c, static_cast<const float2*>(x), static_cast<float2*>(y), nrhs);
}

int hps_op_left(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs) {
  if (!c || !x || !y || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_op_left");
  int rc = ws_reserve(c, &c->w_op, sizeof(double2) * (size_t)c->N * nrhs);
  if (rc) return rc;
  return launch_op_left(c, reinterpret_cast<const double2*>(x), static_cast<double2*>(c->w_op.ptr),
                        reinterpret_cast<double2*>(y), nrhs, kFP64);
}

int hps_assemble_rhs(hps_ctx* c, const hps_z* s, const hps_z* t, hps_z* b, int nrhs) {
  if (!c || !s || !b || nrhs < 1) return fail(HPS_ERR_ARG, "bad arguments to hps_assemble_rhs");
  return launch_assemble_rhs(c, reinterpret_cast<const double2*>(s),
                             reinterpret_cast<const double2*>(t), reinterpret_cast<double2*>(b), nrhs);
}

}  // extern "C"
