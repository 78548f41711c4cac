/*
 * hps.h - C-ABI of the MI355X (gfx950) hot path of the iterative HPS solver for
 * the variable-coefficient Helmholtz impedance problem
 *
 *     -Lap u - kappa^2 (1 - b(x)) u = s   in a box Omega,
 *      du/dn + i eta u              = t   on its boundary        (Sec. 1, eq. (diffhelm))
 *
 * discretized by the Hierarchical Poincare-Steklov method on a uniform mesh of
 * cubic leaves (Sec. 2) and solved by GMRES with the locally homogenized
 * block-Jacobi preconditioner (Sec. 4).  Paper: Lucero Lorca, Beams, Beecroft,
 * Gillman, arXiv 2112.02211.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * Unknowns.  p Chebyshev-Lobatto nodes per leaf direction (the paper's n_c),
 *   n1 = q = p - 2, n_i = n1^3 interior and n_b = 6 n1^2 face nodes per leaf,
 *   n = n_i + n_b per leaf, N = n * (number of leaves).  Leaves own their face
 *   nodes, so interior interfaces carry two copies (Sec. 3.1, remark).
 * Layout.  Leaves are numbered x fastest: tau = ex + E1 (ey + E2 ez).  A vector
 *   is leaf-major: [leaf][local node].  Inside a leaf: the n_i interior nodes
 *   (x fastest, then y, then z), then faces 1..6 = -x,+x,-y,+y,-z,+z (eq.
 *   (flux)), each face's n1^2 nodes ordered in its two tangential axes, the
 *   lower axis fastest.  Several right-hand sides are stored one after the
 *   other: vector r occupies elements [r*N, (r+1)*N).
 * Complex numbers are interleaved (re, im) doubles (hps_z).
 * Memory.  Pointers named "device" are HIP device memory owned by the caller;
 *   the library reads or writes them during the call (stream ordered) and never
 *   keeps them.  The context owns everything else it allocates and releases it
 *   in hps_free.
 * Streams.  Every call is ordered on the stream set in hps_opts (or
 *   hps_set_stream); 0 means the default stream.  A context is not thread
 *   safe; calls on different contexts may run concurrently.
 * Errors.  0 = HPS_OK.  HPS_NOT_CONVERGED (1): the solver stopped at its
 *   iteration limit; outputs hold the last iterate and the stats are filled.
 *   Negative values are errors; the message is in hps_last_error() (thread
 *   local) and outputs are unspecified.
 */
#ifndef HPS_H
#define HPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPS_OK 0
#define HPS_NOT_CONVERGED 1
#define HPS_ERR_ARG (-1)
#define HPS_ERR_UNSUPPORTED (-2)
#define HPS_ERR_OOM (-3)
#define HPS_ERR_DEVICE (-4)
#define HPS_ERR_BREAKDOWN (-5)
#define HPS_ERR_NUMERIC (-6)

typedef struct hps_ctx hps_ctx;
typedef struct { double re, im; } hps_z;

/* Axis-aligned box Omega = [lo, hi]; hi - lo must be the same multiple of
 * the leaf side on every axis (cubic leaves, Sec. 2 remark on uniform meshes). */
typedef struct { double lo[3], hi[3]; } hps_domain;

/* Medium b(x) of eq. (diffhelm). */
#define HPS_MEDIUM_ZERO 0   /* b = 0 */
#define HPS_MEDIUM_NODAL 1  /* nodal: device array of N complex values in library node order */
#define HPS_MEDIUM_BUMPS 2  /* b(x) = sum_k amp_k exp(-|x - c_k|^2 / width^2) */
typedef struct {
  int kind;
  int n_bumps;
  const double* centres; /* host, n_bumps x 3 */
  const hps_z* amps;     /* host, n_bumps */
  double width;
  const hps_z* nodal;    /* device, N values (HPS_MEDIUM_NODAL) */
} hps_medium;

/* Storage precisions of the dense per-leaf blocks S~^{tau,-1} (Sec. 4, eq.
 * (schur_pc)); a bit mask in hps_opts.block_precs selects which are built. */
#define HPS_PREC_FP64 1
#define HPS_PREC_FP32 2
#define HPS_PREC_BF16 4
/* The FP64 J^-1 in separable form: the same preconditioner (on each leaf the
 * exact inverse of the homogenized leaf matrix of eq. (block_pc) at lambda^tau)
 * applied with no stored block.  With the face nodes at the interior Chebyshev
 * nodes of each face, that matrix couples nodes along grid lines only, and each
 * face row (eq. (flux) plus i eta) stays on the normal line of its node;
 * eliminating the two end values of every line (a 2 x 2 system per line)
 * leaves a Kronecker sum of one complex n1 x n1 line operator on the interior,
 * which a complex fast diagonalization inverts as Algorithm 3 does the
 * Dirichlet one.  Setup builds one small table per operator (no dense
 * inverses, no solver library); J^-1 reads x and writes y once.  In
 * block_precs: exclusive of HPS_PREC_FP64 (it replaces the FP64 blocks), may be
 * combined with HPS_PREC_FP32 / HPS_PREC_BF16, and requires lambda_bucket = 0.
 * Every call that takes an FP64 J^-1 (hps_precond, hps_op_left, hps_gmres with
 * precond_prec 0 or HPS_PREC_FP64) then uses it; as a prec argument
 * HPS_PREC_SEPARABLE names it explicitly.  hps_autotune does not apply.  One
 * launch covers up to 65535 right-hand sides (more: HPS_ERR_ARG); the result
 * equals the dense-block J^-1 up to rounding (both are exact inverses of the
 * same leaf matrix). */
#define HPS_PREC_SEPARABLE 8

/* The table the separable form is applied with, for a leaf of side h at order
 * p and impedance parameter eta (host only: no device call; for inspection
 * and tests).  out: host, 2 (2 n1^2 + n1 + 4) doubles, n1 = p - 2, complex
 * entries with real and imaginary parts interleaved: Wc = Vc^{-1} (n1 x n1,
 * row major), Vc (the eigenvectors of the line operator Lt as columns, row
 * major), Ec (its n1 eigenvalues), Fi (the inverse 2 x 2 face system of a line,
 * row major: rows lo, hi).  For even n1 the modes come in two halves: first
 * those whose eigenvectors are even under the flip i <-> n1-1-i of a line
 * (Lt commutes with it: the two faces of a line mirror each other), then the
 * odd ones, each half sorted by real, then imaginary part, and the parity of
 * the columns of Vc and the rows of Wc is exact; for odd n1 all n1 are sorted
 * that way.  HPS_ERR_NUMERIC if the eigendecomposition fails its
 * reconstruction check (or, for even n1, Lt is not symmetric under the flip). */
int hps_separable_table(int p, double h, double eta, double* out);

typedef struct {
  int block_precs;     /* OR of HPS_PREC_* (see HPS_PREC_SEPARABLE); 0 means HPS_PREC_FP64 */
  void* stream;        /* hipStream_t; 0 = default stream */
  int verbose;         /* nonzero: setup timings on stderr */
  double lambda_bucket;/* 0: one homogenized block per leaf (the paper's method, Sec. 4.1).
                          delta > 0: each leaf's lambda is rounded to the grid of spacing
                          delta * kappa^2 in its real and imaginary parts (floor(x / h + 1/2) h)
                          before the resonance guard, and leaves with equal rounded lambda share
                          one block (the reuse suggested in the remark of Sec. 4.1); J^-1 is then
                          the exact inverse of the homogenized leaf matrix at the rounded lambda,
                          applied by GEMMs over runs of up to 16 leaves sharing a block, for
                          any number of right-hand sides up to 65535 (more: the J^-1 calls
                          return HPS_ERR_DEVICE).  See hps_num_blocks. */
} hps_opts;

/* Solvers for hps_gmres. */
#define HPS_SOLVER_GMRES 0   /* left preconditioned GMRES(m) on J^-1 A x = J^-1 b (eq. (globalsystem)), FP64 */
#define HPS_SOLVER_FGMRES 1  /* right preconditioned flexible GMRES(m), FP64 outer; J^-1 in precond_prec;
                                several right-hand sides advance in lock step as with
                                HPS_SOLVER_BLOCK (one Krylov space each, stopped on its own true
                                residual; "iters" is then the largest count) */
#define HPS_SOLVER_BLOCK 2   /* lock-step GMRES(m): one Krylov space per right-hand side, up to 64
                                advanced together (J^-1 of 4 or more as a GEMM on the matrix
                                cores); left preconditioned with FP64 blocks, flexible otherwise */
#define HPS_SOLVER_ITI 3     /* GMRES(m) on the face-reduced system (I + Pi R) f = t - Pi h with the
                                exact ItI maps R of the leaves (Sec. 2.2, interface rule of eq.
                                (2x2)), no preconditioner, then the leaf solves for u: the same
                                discrete u.  Needs hps_iti_build; use_x0 and reduced precision are
                                rejected.  Stopping test on ||t - Pi h - (I + Pi R) f|| relative to
                                ||t - Pi h||; iterations and residuals refer to the face system. */

#define HPS_SOLVER_BGMRES 4  /* block GMRES(m): all right-hand sides (up to 64) in one block Krylov
                                space, left preconditioned with the FP64 J^-1 (blocks or separable);
                                block Arnoldi by classical Gram-Schmidt twice, CholQR2 (on column-
                                equilibrated Gram matrices) for each new block, the block least-
                                squares problem by Householder reflections on the host.  Each
                                right-hand side is checked on its own PCRR; the block iterates
                                until all pass; "iters" counts block steps.  HPS_ERR_BREAKDOWN if a
                                block's columns become linearly dependent (identical right-hand
                                sides, say): the lock-step solver has no such limit. */
#define HPS_SOLVER_IR 5      /* iterative refinement: an FP64 outer loop on the true residual
                                r = b - A x (FP64 operator), each correction d from an inner left-
                                preconditioned GMRES(m) whose vectors are stored in complex FP32
                                (basis, operator and J^-1 kernels read and write FP32, arithmetic
                                FP64 inside), started from 0 on r / ||r|| and stopped at the
                                preconditioned residual reduction inner_tol, or at a tenth of the
                                reduction the outer tolerance still needs when that is larger (the
                                last refinement is short); x += ||r|| d in FP64.
                                Stops when ||r|| <= tol ||b||.  Needs the separable J^-1
                                (HPS_PREC_SEPARABLE; no operator groups); "iters" counts inner
                                steps, "restarts" refinement steps; bytes_apply / bytes_precond
                                are those of the inner FP32 launches. */

typedef struct {
  int solver;          /* HPS_SOLVER_* (default GMRES) */
  int max_iters;       /* total Arnoldi steps; 0 = 20000 */
  int use_x0;          /* nonzero: u holds the initial guess on entry */
  int precond_prec;    /* HPS_PREC_* used inside J^-1 (must have been built); 0 = FP64 */
  int check_every;     /* host convergence poll interval in iterations; 0 = 1 */
  int orth;            /* 0: delayed-reorthogonalization Gram-Schmidt (restart <= 64, else CGS2);
                          1: classical Gram-Schmidt twice (CGS2) */
  double* rhs_rel_res; /* NULL, or host array of nrhs: on return the final relative residual of
                          each right-hand side, in the norm its stopping test uses */
  double inner_tol;    /* HPS_SOLVER_IR: relative tolerance of each inner FP32 solve (its
                          preconditioned residual reduction); 0 = 1e-3 */
} hps_solve_opts;

typedef struct {
  int iters;            /* Arnoldi steps taken (per right-hand side for lock-step solves) */
  int restarts;
  int converged;
  int lambda_shifted;   /* number of leaves whose lambda was moved off a resonance */
  double rel_res;       /* final residual estimate, relative (preconditioned for GMRES) */
  double true_rel_res;  /* recomputed at the end from x: same norm as rel_res */
  double t_setup;       /* seconds hps_setup took for this context (host wall clock) */
  double t_solve;       /* seconds, host wall clock around the solve */
  double bytes_apply;   /* algorithmic HBM bytes of one hps_apply */
  double bytes_precond; /* algorithmic HBM bytes of one hps_precond */
} hps_stats;

/* Build a context: node tables, medium at the nodes, C = kappa^2 (1 - b),
 * lambda^tau (Sec. 4.1), and every block S~^{tau,-1} (Sec. 5.1: precomputed
 * before the iteration), in the precisions asked for.
 *   d        box; n_elem[3] leaves per axis (each >= 1)
 *   kappa    wave number (> 0); eta impedance parameter (the paper sets eta = kappa)
 *   b        medium (NULL = zero)
 *   p, q     Chebyshev nodes per leaf direction (3 <= p <= 16) and face nodes per
 *            face edge; q must equal p - 2 (HPS_ERR_UNSUPPORTED otherwise)
 *   o        options (NULL = defaults)
 *   out      receives the context.
 * Errors: HPS_ERR_ARG (bad sizes, non-cubic leaves), HPS_ERR_UNSUPPORTED,
 * HPS_ERR_OOM, HPS_ERR_DEVICE, HPS_ERR_NUMERIC (a singular leaf block). */
int hps_setup(const hps_domain* d, double kappa, double eta, const hps_medium* b,
              int p, int q, const int n_elem[3], const hps_opts* o, hps_ctx** out);

/* Operator group: nop operators (1 <= nop <= 64) on the same mesh (d, n_elem,
 * p, q) with their own wave number kappa[op], impedance parameter eta[op] and
 * medium media[op] (media NULL: all zero), built into one context so that
 * every launch of the solve covers all of them (the batching of many small
 * meshes in one launch; the leaves, tables and neighbours are shared, C,
 * lambda and the blocks are stored per operator).  A vector of a group holds
 * one right-hand side per operator, [op][N]: hps_apply, hps_precond,
 * hps_op_left and hps_gmres take nrhs = nop (HPS_ERR_ARG otherwise), and
 * hps_gmres iterates the nop systems in lock step, each with its own Krylov
 * space, whatever solver is asked for (GMRES: left FP64; FGMRES or reduced
 * precision: flexible).  hps_lambdas returns nop * N_l values.  Not combined
 * with lambda buckets or the face-reduced system (HPS_ERR_UNSUPPORTED).
 * Errors as hps_setup. */
int hps_setup_group(const hps_domain* d, int nop, const double* kappa, const double* eta,
                    const hps_medium* media, int p, int q, const int n_elem[3], const hps_opts* o,
                    hps_ctx** out);
/* Operators of a context: 1, or nop of hps_setup_group; -1 for NULL. */
int hps_num_operators(const hps_ctx* c);

/* N = (#leaves) * (p-2)^2 (p+4). */
int64_t hps_num_unknowns(const hps_ctx* c);

/* Physical coordinates of the N unknowns, library order; xyz_host is N x 3 host doubles. */
int hps_nodes(const hps_ctx* c, double* xyz_host);

/* Per-leaf homogenization constant lambda^tau (after the resonance guard);
 * lam_host receives (#leaves) complex values (#operators * #leaves for a group). */
int hps_lambdas(const hps_ctx* c, hps_z* lam_host);

/* Number of stored homogenized blocks: the number of leaves, or of distinct
 * rounded lambdas with opts.lambda_bucket > 0; -1 for a NULL context. */
int64_t hps_num_blocks(const hps_ctx* c);

/* Set the stream used by subsequent calls (hipStream_t; 0 = default). */
int hps_set_stream(hps_ctx* c, void* stream);

/* y = A x (Sec. 3.2, Algorithm 2): leaf rows by tensor-product contractions
 * (Algorithm 1, eq. (leafmat)) plus the outgoing impedance of each neighbour
 * on shared faces (eq. (outgoingimpedance)).  x, y: device, nrhs * N complex;
 * must not overlap. */
int hps_apply(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs);

/* hps_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bit for bit, but the face buffer between
 * the sweep and the exchange (nrhs * #leaves * 6 (p-2)^2 complex values) lives
 * in a static device array of HPS_NOALLOC_SCRATCH_BYTES that the library holds
 * on each GPU until the process ends, instead of a context workspace.  The call
 * allocates nothing, records no timing events, and needs no clearing of the
 * array (the sweep writes every entry the exchange reads).  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads, other contexts) race and must be ordered by the caller.
 * x, y: device, nrhs * N complex; must not overlap.
 * Errors: HPS_ERR_ARG (bad arguments, or a face buffer larger than
 * HPS_NOALLOC_SCRATCH_BYTES: at most 65536 face nodes' worth of leaves times
 * right-hand sides per MiB), HPS_ERR_DEVICE. */
#define HPS_NOALLOC_SCRATCH_BYTES (64u << 20)
int hps_apply_noalloc(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs);

/* y = J^{-1} x (Sec. 4, Algorithm 4, eq. (block_pc)) with the FP64 blocks.
 * x, y: device, nrhs * N complex; must not overlap. */
int hps_precond(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs);

/* y = J^{-1} A x with the FP64 blocks: the left-preconditioned operator the
 * GMRES of Sec. 5.2 iterates on (eq. (block_pc) applied after Algorithm 2; its
 * spectrum is the one Sec. 4.2 studies).  Same result as hps_apply followed by
 * hps_precond, bit for bit; with fewer than 4 right-hand sides the face
 * exchange of A runs inside the preconditioner's load (one kernel fewer).
 * x, y: device, nrhs * N complex; must not overlap.  Uses a context-owned
 * workspace of nrhs * N complex (released by hps_trim). */
int hps_op_left(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs);

/* Face-reduced system with the exact impedance-to-impedance maps (Sec. 2.2):
 * the unknowns are the incoming impedance f on every leaf face, stored
 * [rhs][leaf][n_b] in the leaf's face order; a leaf's outgoing impedance is
 * g = R f + h with R = I - 2 i eta S^-1 (S = F_bb - F_bi A_ii^-1 A_ib, the exact
 * Schur complement with the variable medium) and h caused by the interior
 * source; on a shared face the incoming impedance is minus the neighbour's
 * outgoing one (eq. (2x2)), on the boundary it is t.
 *
 * hps_iti_build: forms R and A_ii^-1 of every leaf (rocSOLVER LU and inverse,
 * rocBLAS batched GEMMs); device memory 16 N_l (n_b^2 + n_i^2) bytes
 * (hps_iti_bytes), kept until hps_free.  Idempotent.  HPS_ERR_NUMERIC if a
 * leaf's A_ii or S is singular, HPS_ERR_OOM if the memory is not there. */
int hps_iti_build(hps_ctx* c);
/* y = f + Pi (R f): the face-reduced operator (one streaming pass over every
 * R, then the face exchange).  f, y: device, nrhs * N_l * n_b complex, must
 * not overlap. */
int hps_iti_apply(hps_ctx* c, const hps_z* f, hps_z* y, int nrhs);
/* rhs_f = t - Pi h for the data (s, t) of hps_assemble_rhs (device, nrhs * N
 * complex); rhs_f: device, nrhs * N_l * n_b. */
int hps_iti_rhs(hps_ctx* c, const hps_z* s, const hps_z* t, hps_z* rhs_f, int nrhs);
/* u from the incoming impedance f: on each leaf the solve with source s at the
 * interior rows and f at the face rows.  u: device, nrhs * N complex. */
int hps_iti_recover(hps_ctx* c, const hps_z* s, const hps_z* t, const hps_z* f, hps_z* u, int nrhs);
/* Device bytes hps_iti_build allocates for this mesh (persistent part). */
int64_t hps_iti_bytes(int p, const int n_elem[3]);

/* As hps_precond with the blocks stored in precision prec (HPS_PREC_*; must
 * have been built).  Reduced-precision blocks are applied with FP32 arithmetic. */
int hps_precond_prec(hps_ctx* c, const hps_z* x, hps_z* y, int nrhs, int prec);

/* Right-hand side b of Sec. 3.1: s at interior nodes, t at face nodes on the
 * boundary of Omega, 0 at interface nodes.  s, t, b: device, nrhs * N complex
 * in library node order (entries of s and t at other nodes are ignored); t may
 * be NULL for zero boundary data (no N-vector of zeros needs to exist).  The
 * same holds for t in hps_gmres, hps_iti_rhs and hps_iti_recover. */
int hps_assemble_rhs(hps_ctx* c, const hps_z* s, const hps_z* t, hps_z* b, int nrhs);

/* Solve A u = b(s, t) (Sec. 4, eq. (globalsystem)) by the solver in so.
 *   s, t     device, nrhs * N complex (see hps_assemble_rhs; t may be NULL)
 *   tol      relative residual target, each right-hand side: ||J^-1 r|| <=
 *            tol ||J^-1 b|| with left preconditioning (HPS_SOLVER_GMRES, and
 *            BLOCK with FP64 blocks: the paper's PCRR, Sec. 6), ||r|| <= tol ||b||
 *            for the flexible solvers
 *   restart  Krylov dimension m per cycle (1..200)
 *   u        device, nrhs * N complex: the solution (initial guess if use_x0)
 *   so       NULL = defaults; st may be NULL.
 * Uses context-owned workspaces (basis, nrhs * N complex for b; released by
 * hps_trim).  With use_x0 a call continues from u: one call per restart cycle
 * (max_iters = restart) is the same iteration as one long call.
 * Returns HPS_OK, HPS_NOT_CONVERGED, or an error. */
int hps_gmres(hps_ctx* c, const hps_z* s, const hps_z* t, double tol, int restart,
              hps_z* u, int nrhs, const hps_solve_opts* so, hps_stats* st);

/* The inner operators of HPS_SOLVER_IR on vectors stored in complex FP32
 * (interleaved re, im floats): y = J^{-1} A x (eq. (block_pc) after Algorithm 2,
 * face exchange fused into J^{-1}) and y = J^{-1} x, with the separable J^{-1};
 * every kernel widens its loads to FP64, computes in FP64 and rounds its
 * stores to FP32.  x, y: device, nrhs * N complex64; must not overlap.
 * Errors: HPS_ERR_ARG (bad arguments, separable J^-1 not built, operator
 * group), HPS_ERR_OOM, HPS_ERR_DEVICE. */
int hps_op_left_f32(hps_ctx* c, const void* x, void* y, int nrhs);
int hps_precond_f32(hps_ctx* c, const void* x, void* y, int nrhs);

/* Kernel timing with HIP events attached to the kernel dispatches themselves
 * (start and end timestamps of the launch) for operator launches (sweep, plus
 * the exchange when it is a separate kernel), preconditioner launches and the
 * many-right-hand-side block GEMM, by the solvers and by hps_apply /
 * hps_precond.  enable = 0 switches it off; enable = k > 0 times every k-th
 * launch of each kind (each timed launch costs a few microseconds of stream
 * time, so a period of 8 to 16 keeps a timed solve close to an untimed one).
 * Negative values: HPS_ERR_ARG. */
int hps_set_timing(hps_ctx* c, int enable);

/* Totals since the last reset: out[0] = operator milliseconds, out[1] =
 * operator launches, out[2] = preconditioner milliseconds, out[3] =
 * preconditioner launches, out[4] = milliseconds of the many-right-hand-side
 * block GEMM kernel alone, out[5] = its launches, out[6] = milliseconds of the
 * ItI block product of the face-reduced system (hps_iti_apply), out[7] = its
 * launches.  Synchronizes the stream.  reset != 0 clears them. */
int hps_kernel_times(hps_ctx* c, double out[8], int reset);

/* The Arnoldi update pass (one launch per Arnoldi step, the basis read once;
 * with the dense blocks replaced by the separable J^-1 it is the largest
 * kernel of a solve; on long vectors the last one of a restart cycle also makes
 * the cycle's closing reduction from the values it holds), timed like the
 * kinds above: out[0] = milliseconds of the
 * timed launches, out[1] = their number, out[2] = their algorithmic HBM bytes
 * (per right-hand side and step j: basis vectors 0..j-1 and two vectors read,
 * two written, 16 N (j + 4) bytes).  Synchronizes the stream; reset != 0
 * clears them (independently of hps_kernel_times). */
int hps_arnoldi_times(hps_ctx* c, double out[3], int reset);

/* Tile shapes of the many-right-hand-side block GEMM inside J^-1 (4 to 64
 * right-hand sides; the batching pattern on top of Sec. 4): shape index ->
 * (wavefronts per workgroup, right-hand sides per column panel): 0 (8, 64),
 * 1 (8, 32), 2 (8, 16), 3 (4, 64), 4 (4, 32), 5 (4, 16).  All shapes give
 * identical results.  The library uses the shape recorded for (p, precision,
 * nrhs) in a process-wide table (thread-safe), else the narrowest column panel
 * that holds all right-hand sides.  With lambda buckets the GEMM runs over
 * runs of up to 16 leaves of one bucket, and the key's nrhs is the column
 * count of the widest run, min(64, its leaves * nrhs). */
#define HPS_GEMM_SHAPES 6
/* Time every shape on c's blocks of precision prec (HPS_PREC_*, built at setup)
 * for nrhs right-hand sides (4..64; 1..64 with lambda buckets), reps launches
 * each, and record the fastest under the key above; *shape_out (may be NULL)
 * receives it.  Uses the context's panel workspace and synchronizes its
 * stream. */
int hps_autotune(hps_ctx* c, int nrhs, int prec, int reps, int* shape_out);
/* Record shape for (p, prec, nrhs); shape = -1 removes the entry. */
int hps_autotune_set(int p, int prec, int nrhs, int shape);
/* *shape = the shape the library uses for (p, prec, nrhs). */
int hps_autotune_get(int p, int prec, int nrhs, int* shape);
/* Write the table as text, one "gemm p prec nrhs shape ms_per_launch" line per
 * entry; merge such a file into the table (HPS_ERR_ARG on a malformed line,
 * the table unchanged). */
int hps_autotune_save(const char* path);
int hps_autotune_load(const char* path);

/* Device bytes hps_setup keeps for a mesh of n_elem leaves at order p with the
 * block precisions block_precs (tables, medium, blocks); *transient receives
 * the extra bytes setup needs while it builds the blocks (NULL allowed).
 * Returns a negative error code for invalid sizes. */
/* (With lambda buckets the blocks take at most this much: the plan counts one
 * block per leaf.) */
int64_t hps_setup_bytes(int p, const int n_elem[3], int block_precs, int complex_medium,
                        int64_t* transient);

/* Device bytes hps_gmres needs for a solve with this context (solver
 * workspaces, which the context keeps for reuse, plus the right-hand side it
 * assembles for the call).  so as for hps_gmres (NULL = defaults). */
int64_t hps_solve_bytes(const hps_ctx* c, int restart, int nrhs, const hps_solve_opts* so);

/* Release the solver and operator workspaces of an idle context (the blocks,
 * tables and medium stay).  They are allocated again by the next call. */
int hps_trim(hps_ctx* c);

/* Device bytes held by the context (blocks, tables, workspaces). */
int64_t hps_device_bytes(const hps_ctx* c);

/* Message of the last error on this thread ("" if none). */
const char* hps_last_error(void);

/* Release a context (NULL is ignored). */
void hps_free(hps_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* HPS_H */
