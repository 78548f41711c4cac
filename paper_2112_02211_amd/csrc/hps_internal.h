// Internal declarations of the HPS library: the context, the host tables and
// the launchers of the device kernels.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hps.h"
#include "k_common.h"

namespace hps {

constexpr int kMinP = 4;
constexpr int kMaxP = 16;

// ---------------------------------------------------------------- host tables
// One-leaf tables shared by every leaf (they do not depend on the medium).
struct HostTables {
  int p = 0, n1 = 0, ni = 0, nb = 0, n = 0;
  double h = 0.0;
  std::vector<double> xi;   // p reference Chebyshev-Lobatto nodes, ascending
  std::vector<double> D;    // p x p first derivative on a leaf of side h, row major
  std::vector<double> D2;   // p x p, D * D
  std::vector<double> V;    // n1 x n1 eigenvectors of L1 = D2[1:p-1, 1:p-1] (columns)
  std::vector<double> W;    // n1 x n1, V^{-1}
  std::vector<double> E;    // n1 eigenvalues of L1 (real, negative)
  std::vector<double> P;    // nb x ni, F_bi (V x V x V)            (setup only)
  std::vector<double> Q;    // ni x nb, (V x V x V)^{-1} A_ib       (setup only)
};

// Builds every table; returns an empty string or an error message.
std::string build_tables(int p, double h, HostTables* t);
// F_bi, N_bb (F_bb without the i eta I) and A_ib of the leaf matrix, column-major.
void build_face_operators(const HostTables& t, std::vector<double>* Fbi, std::vector<double>* Nbb,
                          std::vector<double>* Aib);
// Complex entries of the separable table of one operator: [Wc | Vc | Ec | Fi],
// n1^2 + n1^2 + n1 + 4 (layout in build_sep_table).
__host__ __device__ constexpr int sep_table_size(int p) { return 2 * (p - 2) * (p - 2) + (p - 2) + 4; }
// The separable form of the homogenized leaf solve for impedance parameter eta
// (2 * sep_table_size(p) doubles, real and imaginary parts interleaved).
std::string build_sep_table(const HostTables& t, double eta, std::vector<double>* out);

// Face f (0..5): axis = f/2, high side = f%2, outward sign -1 / +1.
inline int face_axis(int f) { return f >> 1; }
inline int face_high(int f) { return f & 1; }

// --------------------------------------------------------------- device views
struct DevTables {
  const double* D;    // p x p
  const double* D2;   // p x p
  const double* V;    // n1 x n1
  const double* W;    // n1 x n1
  const double* E;    // n1
};

// Column-group width (complex numbers per 16-byte group) of the block layout.
inline int block_cw(int prec) { return prec == kFP64 ? 1 : (prec == kFP32 ? 2 : 4); }

struct Blocks {
  void* data = nullptr;   // [leaf][col group][row][cw complex]
  int ncp = 0;            // padded column count (multiple of cw)
  size_t bytes = 0;
};

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

}  // namespace hps

constexpr int kTimingKinds = 5;

struct hps_ctx {
  int p = 0, n1 = 0, ni = 0, nb = 0, n = 0;
  int E[3] = {0, 0, 0};
  int64_t nl = 0, N = 0;
  double kappa = 0, eta = 0, h = 0, lo[3] = {0, 0, 0};
  hipStream_t stream = nullptr;
  int device = 0;
  int verbose = 0;

  hps::HostTables tab;
  double* d_tab = nullptr;          // D | D2 | V | W | E
  hps::DevTables dt{};
  int* d_nbr = nullptr;             // [nl][6], -1 on the boundary
  int c_complex = 0;                // C stored as complex (else real)
  void* d_C = nullptr;              // [nop][nl][ni] kappa^2 (1 - b) at interior nodes
  double2* d_lambda = nullptr;      // [nop][nl] lambda^tau (rounded when lambda_bucket > 0)
  // operator groups (hps_setup_group): nop operators on the same mesh (same
  // leaves, tables and neighbours) with their own kappa, eta and medium; C,
  // lambda and the blocks are stored per operator ([op][...]) and a vector of
  // the group holds one right-hand side per operator ([op][N])
  int nop = 1;
  std::vector<double> kappas, etas;  // per operator
  double* d_eta = nullptr;           // [nop] (groups only)
  // lambda buckets (lambda_bucket > 0): leaves with equal rounded lambda share
  // one block; buckets are numbered in order of their first leaf
  double lambda_bucket = 0.0;
  int64_t nblocks = 0;              // stored blocks: nl, or the number of buckets
  int* d_bpos = nullptr;            // [nl] position of the leaf in bucket order
  double2* d_blam = nullptr;        // [nblocks] the bucket's lambda
  // J^-1 GEMM groups: each bucket split into runs of at most kGroupLeaves
  // consecutive positions, so that one large bucket (the background medium)
  // spreads over many workgroups
  int64_t ngroups = 0;
  int* d_gofs = nullptr;            // [ngroups + 1] first position of each group
  int* d_gblk = nullptr;            // [ngroups] block (bucket) of each group
  int group_leaves = 1;             // leaves in the largest group
  int n_shifted = 0;
  double t_setup = 0.0;  // seconds of hps_setup (host wall clock, device synchronized)
  // device address of the static face buffer of hps_apply_noalloc on the
  // context's device (from hipGetSymbolAddress at setup)
  double2* d_scratch = nullptr;
  hps::Blocks blk[3];
  // separable form of the FP64 J^-1 (block_precs has HPS_PREC_SEPARABLE): no
  // FP64 blocks; one complex table per operator
  int sep = 0;
  double2* d_sep = nullptr;         // [nop][sep_table_size(p)]
  // face-reduced system with the exact ItI maps (built by hps_iti_build)
  double2* d_itiR = nullptr;        // [nl][nb cols][nb rows]  R^tau = I - 2 i eta S^{tau,-1}
  double2* d_Ainv = nullptr;        // [nl][ni cols][ni rows]  (A_ii^tau)^{-1}
  double* d_Fbi = nullptr;          // nb x ni, column-major (shared by all leaves)
  double* d_Aib = nullptr;          // ni x nb, column-major (shared by all leaves)

  // reusable workspaces (grown on demand)
  hps::Workspace w_g;               // outgoing impedance buffer
  hps::Workspace w_red;             // reduction partials + counters
  hps::Workspace w_krylov;          // Krylov bases etc.
  hps::Workspace w_krylov32;        // FP32 Krylov basis of the inner solve of iterative refinement
  hps::Workspace w_ir;              // iterative refinement: FP64 residual, FP32 residual and correction
  hps::Workspace w_small;           // Hessenberg / Givens state
  hps::Workspace w_batch;           // many-rhs preconditioner: H and U panels
  hps::Workspace w_op;              // A x inside hps_op_left
  hps::Workspace w_b;               // assembled right-hand sides inside hps_gmres
  hps::Workspace w_iti;             // face-system solve: v, w, h and q of every leaf
  void* h_pinned = nullptr;         // small pinned host buffer for scalars
  uint32_t solve_epoch = 0;         // tags the residual records of each solve
  size_t dev_bytes = 0;

  hipEvent_t ev_solver[2] = {nullptr, nullptr};  // residual-check events of the solvers

  // optional kernel timing: event pairs per launch kind (kTimingKinds: 0 operator,
  // 1 preconditioner, 2 many-rhs block GEMM, 3 ItI block product of the face system,
  // 4 Arnoldi update pass), with the algorithmic HBM bytes of each timed launch
  int timing = 0;                   // 0 off, k > 0: time every k-th launch of each kind
  std::vector<hipEvent_t> ev_free;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[kTimingKinds];
  std::vector<double> ev_bytes[kTimingKinds];
  double t_ms[kTimingKinds] = {};
  double t_cnt[kTimingKinds] = {};
  double t_bytes[kTimingKinds] = {};
  uint64_t t_seq[kTimingKinds] = {};    // launches seen per kind (sampling)
};

namespace hps {

// error reporting ----------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);
#define HPS_TRY_HIP(expr)                                       \
  do {                                                          \
    int _rc = ::hps::check_hip((expr), #expr);                  \
    if (_rc != HPS_OK) return _rc;                              \
  } while (0)

int ws_reserve(hps_ctx* c, Workspace* w, size_t bytes);
int dev_alloc(hps_ctx* c, void** p, size_t bytes);

// launchers (all stream ordered on c->stream) ------------------------------
// setup
int launch_eval_medium(hps_ctx* c, const hps_medium* b, const double* d_bump_c,
                       const double2* d_bump_a, int nbump);
int launch_lambda(hps_ctx* c);
int launch_build_schur(hps_ctx* c, const double* dP, const double* dQ, const double2* lam, int e0,
                       int ne, double2* S /* [ne][nb][nb] column major */);
int launch_pack_blocks(hps_ctx* c, const double2* Sinv, int e0, int ne, int prec);
int launch_node_coords(hps_ctx* c, double* d_xyz);

// Kernel timing (no-op unless c->timing): a pair of events that the launches
// attach to their own dispatches (hipExtLaunchKernelGGL takes the kernels'
// start and end timestamps), so timing puts no extra packets on the stream.
struct TimedPair {
  hipEvent_t start = nullptr, stop = nullptr;
};
int timing_pair(hps_ctx* c, int kind, TimedPair* tp);  // kind: 0 apply, 1 J^-1, 2 GEMM, 3 ItI, 4 update
int timing_commit(hps_ctx* c, int kind, const TimedPair& tp, double bytes = 0.0);
void timing_drop(hps_ctx* c, const TimedPair& tp);  // return unused events to the pool
int timing_collect(hps_ctx* c);

// Launch on the context's stream; e0 / e1 (either may be null) take the
// kernel's start / end timestamps.
template <typename... KArgs, typename... Args>
inline hipError_t launch_k(hps_ctx* c, hipEvent_t e0, hipEvent_t e1, void (*kern)(KArgs...), dim3 g,
                           dim3 b, Args... args) {
  hipExtLaunchKernelGGL(kern, g, b, 0, c->stream, e0, e1, 0, args...);
  return hipGetLastError();
}
// launch_k with dynamic LDS
template <typename... KArgs, typename... Args>
inline hipError_t launch_k_lds(hps_ctx* c, hipEvent_t e0, hipEvent_t e1, void (*kern)(KArgs...), dim3 g,
                               dim3 b, size_t lds, Args... args) {
  hipExtLaunchKernelGGL(kern, g, b, lds, c->stream, e0, e1, 0, args...);
  return hipGetLastError();
}

// hot path
int launch_apply(hps_ctx* c, const double2* x, double2* y, int nrhs);
// launch_apply with the face buffer in the library's static device array
// (no allocation); scratch_address looks up that array's address on the
// current device (once per device, cached)
int launch_apply_noalloc(hps_ctx* c, const double2* x, double2* y, int nrhs);
int scratch_address(double2** out);
int launch_precond(hps_ctx* c, const double2* x, double2* y, int nrhs, int prec);
// y = J^{-1} A x with the face exchange of A fused into the preconditioner's
// load (one leaf per workgroup); tmp receives A x without the exchange.  With
// kBatchedMinRhs or more right-hand sides and dense blocks: launch_apply, then
// launch_precond (the separable form is fused for any nrhs).
int launch_op_left(hps_ctx* c, const double2* x, double2* tmp, double2* y, int nrhs, int prec);
// vectors stored in complex FP32 (the inner solve of iterative refinement):
// A x (sweep and exchange), J^{-1} A x and J^{-1} x with the separable J^{-1};
// FP64 arithmetic inside the kernels
int launch_apply(hps_ctx* c, const float2* x, float2* y, int nrhs);
int launch_op_left(hps_ctx* c, const float2* x, float2* tmp, float2* y, int nrhs);
int launch_precond(hps_ctx* c, const float2* x, float2* y, int nrhs);
// the sweep alone: y = A x without the neighbours' outgoing impedance, which
// goes to g ([rhs][leaf][6][q^2]); e0 / e1 as in launch_k
int launch_sweep(hps_ctx* c, const double2* x, double2* y, double2* g, int nrhs, hipEvent_t e0,
                 hipEvent_t e1);
// the same with vectors stored in complex FP32 (FP64 arithmetic inside)
int launch_sweep(hps_ctx* c, const float2* x, float2* y, float2* g, int nrhs, hipEvent_t e0,
                 hipEvent_t e1);
// J^{-1} (y + exchange(g)) for nrhs < kBatchedMinRhs; g == null: J^{-1} y
int launch_precond_fused(hps_ctx* c, const double2* y, const double2* g, double2* z, int nrhs,
                         int prec, hipEvent_t e0, hipEvent_t e1);
// block GMRES(m) on k right-hand sides, left preconditioned with the FP64 J^-1 (block_gmres.cpp)
int run_block_gmres(hps_ctx* c, int prec, const double2* b, double2* x, int k, double tol, int m,
                    int maxit, bool use_x0, double* rhs_res, hps_stats* st);
// J^{-1} (y + exchange(g)) in the separable form (no blocks; any nrhs); g == null: J^{-1} y
int launch_precond_sep(hps_ctx* c, const double2* y, const double2* g, double2* z, int nrhs,
                       hipEvent_t e0, hipEvent_t e1);
int launch_precond_sep(hps_ctx* c, const float2* y, const float2* g, float2* z, int nrhs,
                       hipEvent_t e0, hipEvent_t e1);
// many right-hand sides: block product as a GEMM on the matrix cores; with lambda
// buckets (any nrhs) one GEMM per bucket over all its leaves' columns
int launch_precond_batched(hps_ctx* c, const double2* x, double2* y, int nrhs, int prec,
                           hipEvent_t e0, hipEvent_t e1);
// Tile shapes of the block GEMM: index -> (wavefronts per workgroup, column
// panel): 0 (8, 64), 1 (8, 32), 2 (8, 16), 3 (4, 64), 4 (4, 32), 5 (4, 16).
constexpr int kGemmShapes = 6;
// the shape used for (p, block precision index, columns of the widest GEMM
// group): the tuned one if the autotuner has recorded it, else the built-in
// rule (the narrowest column panel that holds the columns)
int gemm_shape(int p, int prec, int ncols);
// leaves per GEMM group with lambda buckets
constexpr int kGroupLeaves = 16;
// GEMM groups: group g multiplies block gblk[g] (g if null) with the columns of
// positions gofs[g] .. gofs[g+1]-1 (nrhs columns each) of the H panel
struct GemmGroups {
  const int* gofs;
  const int* gblk;
  int64_t ngroups;
  int max_leaves;   // positions in the largest group
};
// the GEMM U = S~^{-1} H of one batched J^-1 (H, U panels as launch_precond_batched
// lays them out)
hipError_t gemm_launch(hps_ctx* c, int prec, int shape, const void* blk, int ncp, const void* Hb,
                       void* Ub, int nrhs, hipEvent_t e0, hipEvent_t e1,
                       const GemmGroups* gg = nullptr);
// face-reduced system with the exact ItI maps (k_iti.hip)
int iti_build(hps_ctx* c);
int launch_iti_apply(hps_ctx* c, const double2* f, double2* y, int nrhs);   // y = f + Pi R f
int iti_prepare(hps_ctx* c, const double2* b, int nrhs, double2* rhs_f);    // face right-hand side
int iti_finish(hps_ctx* c, const double2* f, double2* u, int nrhs);         // leaf recovery
int64_t iti_ws_bytes(const hps_ctx* c, int nrhs);
// bytes of the H and U panels of a batched J^-1 (the w_batch workspace)
size_t batch_panel_bytes(const hps_ctx* c, int nrhs, int prec, size_t* hpad);
constexpr int kBatchedMinRhs = 4;   // from this many right-hand sides on, J^-1 uses the GEMM path
int launch_assemble_rhs(hps_ctx* c, const double2* s, const double2* t, double2* b, int nrhs);

// Krylov primitives over vectors of length n (complex)
struct RedBuf {
  double2* part;      // partial sums
  unsigned* counter;  // one counter per concurrent reduction slot
  int nblk;
  int nbatch;         // batches the partial buffer holds
};
int red_buf(hps_ctx* c, int kmax, int nbatch, RedBuf* rb);
// out[k] = sum_n conj(V[k*ldv + n]) w[n], k < K.
int launch_mdot(hps_ctx* c, const double2* V, int64_t ldv, int K, const double2* w, int64_t n,
                double2* out, const RedBuf& rb);
// w[n] += sign * sum_k V[k*ldv + n] coef[k]; if nrm2 != null: *nrm2 = ||w_new||^2.
int launch_mupdate(hps_ctx* c, const double2* V, int64_t ldv, int K, const double2* coef,
                   double sign, double2* w, int64_t n, double* nrm2, const RedBuf& rb);
// *nrm2 = ||w||^2
int launch_norm2(hps_ctx* c, const double2* w, int64_t n, double* nrm2, const RedBuf& rb);
// y = x * (1/sqrt(*nrm2)) (or by *scale if inv_sqrt == 0)
int launch_scale_by(hps_ctx* c, const double2* x, double2* y, int64_t n, const double* s,
                    int inv_sqrt);
// y = a - y
int launch_sub_from(hps_ctx* c, const double2* a, double2* y, int64_t n);
int launch_sub_from(hps_ctx* c, const float2* a, float2* y, int64_t n);

}  // namespace hps
