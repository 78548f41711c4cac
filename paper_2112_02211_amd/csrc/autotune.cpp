// Tile-shape autotuner of the many-right-hand-side block GEMM (U = S~^{-1} H on
// the matrix cores, one GEMM per leaf).  The shape (wavefronts per workgroup,
// column panel) that runs fastest depends on the order p, the block precision
// and the number of right-hand sides: a 64-column panel wastes three quarters
// of the matrix-core work on 16 right-hand sides, while narrow panels re-read
// the block for every panel.  The autotuner times every shape on a context's
// own blocks and records the fastest in a process-wide table keyed by
// (p, precision, right-hand sides); the table can be saved to and loaded from a
// text file.  Every shape accumulates in the same order, so the choice never
// changes results.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include "hps_internal.h"

namespace hps {
namespace {

struct Entry {
  int shape;
  double ms;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int>, Entry>& table() {
  static std::map<std::tuple<int, int, int>, Entry> t;
  return t;
}

int prec_index_of(int flag) {
  switch (flag) {
    case HPS_PREC_FP64: return kFP64;
    case HPS_PREC_FP32: return kFP32;
    case HPS_PREC_BF16: return kBF16;
    default: return -1;
  }
}

int prec_flag_of(int q) { return q == kFP64 ? HPS_PREC_FP64 : (q == kFP32 ? HPS_PREC_FP32 : HPS_PREC_BF16); }

// built-in rule: the narrowest column panel that holds every column (8
// wavefronts per workgroup: measured no slower than 4 on small launches)
int rule_shape(int ncols) { return ncols <= 16 ? 2 : (ncols <= 32 ? 1 : 0); }

}  // namespace

int gemm_shape(int p, int prec, int ncols) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = table().find(std::make_tuple(p, prec, ncols));
  return it != table().end() ? it->second.shape : rule_shape(ncols);
}

}  // namespace hps

using namespace hps;

extern "C" int hps_autotune(hps_ctx* c, int nrhs, int prec_flag, int reps, int* shape_out) {
  if (!c) return fail(HPS_ERR_ARG, "hps_autotune: context is NULL");
  // lambda buckets: one GEMM per bucket, for any number of right-hand sides,
  // keyed by the columns of the largest bucket (at most one 64-column panel)
  const bool bk = c->lambda_bucket > 0.0;
  if (nrhs < (bk ? 1 : kBatchedMinRhs) || nrhs > 64 || reps < 1)
    return fail(HPS_ERR_ARG, "hps_autotune: needs nrhs <= 64 (and >= 4 with one block per leaf), reps >= 1");
  const int q = prec_index_of(prec_flag);
  if (q < 0 || !c->blk[q].data) return fail(HPS_ERR_ARG, "hps_autotune: block precision not built");
  const int key = bk ? std::min<int64_t>(64, (int64_t)c->group_leaves * nrhs) : nrhs;
  const GemmGroups gg{c->d_gofs, c->d_gblk, c->ngroups, c->group_leaves};
  size_t hpad = 0;
  int rc = ws_reserve(c, &c->w_batch, batch_panel_bytes(c, nrhs, q, &hpad));
  if (rc) return rc;
  void* Hb = c->w_batch.ptr;
  void* Ub = static_cast<char*>(c->w_batch.ptr) + hpad;
  HPS_TRY_HIP(hipMemsetAsync(Hb, 0, hpad, c->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HPS_TRY_HIP(hipEventCreate(&e0));
  if ((rc = check_hip(hipEventCreate(&e1), "hipEventCreate"))) {
    hipEventDestroy(e0);
    return rc;
  }
  int best = -1;
  double best_ms = 0.0;
  const Blocks& B = c->blk[q];
  for (int sh = 0; sh < kGemmShapes && rc == HPS_OK; ++sh) {
    rc = check_hip(gemm_launch(c, q, sh, B.data, B.ncp, Hb, Ub, nrhs, nullptr, nullptr,
                                 bk ? &gg : nullptr), "gemm");
    if (rc) break;
    rc = check_hip(hipEventRecord(e0, c->stream), "hipEventRecord");
    for (int r = 0; r < reps && rc == HPS_OK; ++r)
      rc = check_hip(gemm_launch(c, q, sh, B.data, B.ncp, Hb, Ub, nrhs, nullptr, nullptr,
                                 bk ? &gg : nullptr), "gemm");
    if (rc) break;
    rc = check_hip(hipEventRecord(e1, c->stream), "hipEventRecord");
    if (!rc) rc = check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    const double per = ms / reps;
    if (!rc && (best < 0 || per < best_ms)) {
      best = sh;
      best_ms = per;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    table()[std::make_tuple(c->p, q, key)] = Entry{best, best_ms};
  }
  if (shape_out) *shape_out = best;
  return HPS_OK;
}

extern "C" int hps_autotune_set(int p, int prec_flag, int nrhs, int shape) {
  const int q = prec_index_of(prec_flag);
  if (p < 4 || p > 16 || q < 0 || nrhs < 1 || shape < -1 || shape >= kGemmShapes)
    return fail(HPS_ERR_ARG, "hps_autotune_set: bad arguments");
  std::lock_guard<std::mutex> lk(g_mu);
  if (shape < 0) table().erase(std::make_tuple(p, q, nrhs));
  else table()[std::make_tuple(p, q, nrhs)] = Entry{shape, 0.0};
  return HPS_OK;
}

extern "C" int hps_autotune_get(int p, int prec_flag, int nrhs, int* shape) {
  const int q = prec_index_of(prec_flag);
  if (p < 4 || p > 16 || q < 0 || nrhs < 1 || !shape) return fail(HPS_ERR_ARG, "hps_autotune_get: bad arguments");
  *shape = gemm_shape(p, q, nrhs);
  return HPS_OK;
}

extern "C" int hps_autotune_save(const char* path) {
  if (!path) return fail(HPS_ERR_ARG, "hps_autotune_save: path is NULL");
  std::ofstream f(path);
  if (!f) return fail(HPS_ERR_ARG, std::string("hps_autotune_save: cannot write ") + path);
  f << "# block GEMM tile shapes: gemm p precision_flag nrhs shape ms_per_launch\n";
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : table()) {
    int p, q, n;
    std::tie(p, q, n) = kv.first;
    char line[128];
    std::snprintf(line, sizeof(line), "gemm %d %d %d %d %.6f\n", p, prec_flag_of(q), n, kv.second.shape,
                  kv.second.ms);
    f << line;
  }
  return f ? HPS_OK : fail(HPS_ERR_ARG, "hps_autotune_save: write failed");
}

extern "C" int hps_autotune_load(const char* path) {
  if (!path) return fail(HPS_ERR_ARG, "hps_autotune_load: path is NULL");
  std::ifstream f(path);
  if (!f) return fail(HPS_ERR_ARG, std::string("hps_autotune_load: cannot read ") + path);
  std::map<std::tuple<int, int, int>, Entry> got;
  std::string line;
  int lineno = 0;
  while (std::getline(f, line)) {
    ++lineno;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream in(line);
    std::string tag;
    int p = 0, flag = 0, n = 0, sh = -1;
    double ms = 0.0;
    if (!(in >> tag >> p >> flag >> n >> sh >> ms) || tag != "gemm" || p < 4 || p > 16 ||
        prec_index_of(flag) < 0 || n < 1 || sh < 0 || sh >= kGemmShapes)
      return fail(HPS_ERR_ARG, "hps_autotune_load: bad line " + std::to_string(lineno) + " in " + path);
    got[std::make_tuple(p, prec_index_of(flag), n)] = Entry{sh, ms};
  }
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : got) table()[kv.first] = kv.second;
  return HPS_OK;
}
