// J^{-1} applied to many right-hand sides at once (the batching pattern on top
// of Sec. 4, eq. (block_pc) and Algorithm 4).  With k right-hand sides the
// dense block product of every leaf, u_b = S~^{-1} h_b, becomes a complex GEMM
// (n_b x n_b) * (n_b x k): the block is streamed from HBM once for all k
// columns and the product runs on the matrix cores.  Three kernels:
//
//   pre   per (leaf, rhs): f_i = A~_ii^{-1} x_i (Algorithm 3), y_i = f_i,
//         h_b = x_b - F_bi f_i written to H[leaf][rhs][n_b] in the GEMM precision
//   gemm  per (leaf, 128-row panel, 64-column panel): U = S~^{-1} H on MFMA
//   post  per (leaf, rhs): y_b = u_b, y_i = f_i - A~_ii^{-1} (A_ib u_b)
//
// U is kept in FP32 for FP32 / BF16 blocks (their products accumulate in FP32).
//
// With lambda buckets (leaves sharing one block) the H and U panels are laid
// out in bucket order and the GEMM runs once per bucket over the columns of
// all its leaves: the block is read once for the whole bucket.
//
// The complex product is split into real matrix-core products:
//   Re U = Re S Re H - Im S Im H,   Im U = Re S Im H + Im S Re H.
// Precisions: FP64 blocks on v_mfma_f64_16x16x4 (FP64 accumulate), FP32 blocks
// on v_mfma_f32_16x16x4 and BF16 blocks on v_mfma_f32_16x16x16_bf16 (FP32
// accumulate); H is rounded to the block precision.
#include "hps_internal.h"
#include "k_common.h"
#include "k_leaf.h"

#include <type_traits>

namespace hps {
namespace {

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
typedef short ms4 __attribute__((ext_vector_type(4)));

constexpr int PB = 256;  // threads of the pre / post kernels

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// ------------------------------------------------------------------ pre / post
// (Algorithm 3 line-wise here: these kernels run many small workgroups per CU,
// where LDS bandwidth, not idle threads, bounds the mode products.)
template <int P, int PREC>
// pos != null (lambda buckets): the leaf's panel is at its position in bucket
// order, so that each bucket's columns are contiguous.
__global__ __launch_bounds__(PB) void k_precond_pre(const double2* __restrict__ x,
                                                    double2* __restrict__ y, void* __restrict__ Hb,
                                                    const double2* __restrict__ lam,
                                                    const double* __restrict__ tab, int64_t N,
                                                    int nrhs, const int* __restrict__ pos) {
  constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  __shared__ double2 T[NI];
  __shared__ double2 H[NB];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  const double2* xv = x + rhs * N + tau * NN;
  double2* yv = y + rhs * N + tau * NN;
  for (int m = threadIdx.x; m < NI; m += PB) T[m] = xv[m];
  for (int m = threadIdx.x; m < NB; m += PB) H[m] = xv[NI + m];
  __syncthreads();
  homog_solve<P, PB>(T, tab, lam[tau]);
  for (int m = threadIdx.x; m < NI; m += PB) yv[m] = T[m];
  face_update_g<P, PB>(T, H, tab);
  __syncthreads();
  const int64_t hoff = ((pos ? (int64_t)pos[tau] : tau) * nrhs + rhs) * NB;
  for (int r = threadIdx.x; r < NB; r += PB) {
    const double2 h = H[r];
    if (PREC == kFP64) {
      static_cast<double2*>(Hb)[hoff + r] = h;
    } else if (PREC == kFP32) {
      static_cast<float2*>(Hb)[hoff + r] = make_float2((float)h.x, (float)h.y);
    } else {
      static_cast<uint32_t*>(Hb)[hoff + r] = bf16_rne((float)h.x) | (bf16_rne((float)h.y) << 16);
    }
  }
}

// UF: U is stored as float2 (FP32 / BF16 blocks, whose products accumulate in
// FP32 anyway) instead of double2 (FP64 blocks).
template <int P, bool UF>
__global__ __launch_bounds__(PB) void k_precond_post(double2* __restrict__ y,
                                                     const void* __restrict__ Ub,
                                                     const double2* __restrict__ lam,
                                                     const double* __restrict__ tab, int64_t N,
                                                     int nrhs, const int* __restrict__ pos) {
  constexpr int N1 = P - 2, L = N1 * N1, NI = N1 * L, NB = 6 * L, NN = NI + NB;
  __shared__ double2 T[NI];
  __shared__ double2 U[NB];
  const int64_t tau = blockIdx.x;
  const int rhs = blockIdx.y;
  double2* yv = y + rhs * N + tau * NN;
  const int64_t uoff = ((pos ? (int64_t)pos[tau] : tau) * nrhs + rhs) * NB;
  for (int r = threadIdx.x; r < NB; r += PB) {
    double2 u;
    if (UF) {
      const float2 f = static_cast<const float2*>(Ub)[uoff + r];
      u = make_double2((double)f.x, (double)f.y);
    } else {
      u = static_cast<const double2*>(Ub)[uoff + r];
    }
    U[r] = u;
    yv[NI + r] = u;
  }
  __syncthreads();
  interior_from_faces_g<P, PB>(U, T, tab);
  __syncthreads();
  homog_solve<P, PB>(T, tab, lam[tau]);
  for (int m = threadIdx.x; m < NI; m += PB) yv[m] = csub(yv[m], T[m]);
}

// ------------------------------------------------------------------------ GEMM
// Workgroup: 8 wavefronts; wavefront w owns rows r0 + 16 w .. +16 of a 128-row
// panel and all 64 columns of a column panel (4 tiles of 16).  MFMA operand
// lanes: row (or column) = lane % 16, k-slot group g = lane / 16.  Accumulator
// register r of a lane holds column lane % 16 and row 4 g + r for the FP32 and
// BF16 instructions but row g + 4 r for v_mfma_f64_16x16x4 (layouts checked
// on the device with an in-bounds probe of the builtins).  One 16-byte load of the
// block per lane supplies CW consecutive inner indices of its row; the k-slots
// of each MFMA are mapped to inner indices so that A and B agree:
//   FP64 (CW = 1): slot g      <-> inner kb + g
//   FP32 (CW = 2): slot g, s   <-> inner kb + 2 g + s  (two MFMA steps)
//   BF16 (CW = 4): slot (g, e) <-> inner kb + 4 g + e  (one step, 4 values per lane)
// H for the column panel is staged in LDS, KT inner indices at a time.
// Tile shape (template): GW wavefronts per workgroup, each owning 16 rows, and a
// column panel of GCOLS right-hand sides (GCOLS / 16 column tiles per
// wavefront).  Every shape accumulates the inner index in the same order, so
// the shapes give identical results; the autotuner picks among them.

template <int PREC> struct GemmTraits;
// PAD: extra columns per LDS row of the staged H.  The four k-slot groups of a
// wavefront read rows CW apart; with 16-, 32- or 64-entry rows those rows start
// on the same LDS bank, so the padding shifts them onto disjoint banks (BF16:
// 16 words apart, conflict-free; FP32: 32 words, the two passes an 8-byte read
// needs).
template <> struct GemmTraits<kFP64> { using H = double2; static constexpr int CW = 1, KT = 32, PAD = 0; };
template <> struct GemmTraits<kFP32> { using H = float2; static constexpr int CW = 2, KT = 64, PAD = 8; };
template <> struct GemmTraits<kBF16> { using H = uint32_t; static constexpr int CW = 4, KT = 64, PAD = 4; };

template <int PREC, int GW, int GCOLS>
__global__ __launch_bounds__(64 * GW) void k_block_gemm(const void* __restrict__ blk, int ncp,
                                                        const void* __restrict__ Hb,
                                                        void* __restrict__ Ub, int NB,
                                                        int nrhs, const int* __restrict__ gofs,
                                                        const int* __restrict__ gblk) {
  constexpr int GROWS = 16 * GW;    // rows per workgroup
  constexpr int GCT = GCOLS / 16;   // column tiles per wavefront
  using TR = GemmTraits<PREC>;
  using HT = typename TR::H;
  // inner indices per stage (FP64 with 64-column panels: 16, for the registers)
  constexpr int KT = (PREC == kFP64 && GCOLS == 64) ? 16 : TR::KT;
  constexpr int CW = TR::CW, CH = 4 * CW;  // inner indices per MFMA chunk
  // narrow panels load H one stage ahead (latency-bound small groups); 64-column
  // panels load it in the stage (registers for occupancy)
  constexpr bool HPF = GCOLS <= 32;
  __shared__ HT Bs[KT][GCOLS + TR::PAD];
  // group: a leaf (nrhs columns), or with gofs a run of leaves of one lambda
  // bucket, whose columns are the nrhs columns of each leaf, stored
  // contiguously, and whose block is gblk[group]
  const int64_t grp = blockIdx.x;
  int64_t cb = grp * nrhs;
  int ncols = nrhs;
  int64_t tau = grp;   // block index
  if (gofs) {
    cb = (int64_t)gofs[grp] * nrhs;
    ncols = (gofs[grp + 1] - gofs[grp]) * nrhs;
    tau = gblk[grp];
  }
  const int r0 = blockIdx.y * GROWS;
  const int c0 = blockIdx.z * GCOLS;
  if (c0 >= ncols) return;  // a column panel past this group's columns (whole workgroup)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int row = r0 + wv * 16 + li;
  const int rowc = row < NB ? row : NB - 1;  // clamp: loads in bounds, results discarded
  const int ncg = ncp / CW;
  const uint4* B = static_cast<const uint4*>(blk) + (size_t)tau * ncg * NB;
  const HT* Hl = static_cast<const HT*>(Hb) + (size_t)cb * NB;

  using Acc = typename std::conditional<PREC == kFP64, md4, mf4>::type;
  Acc are[GCT], aim[GCT];
#pragma unroll
  for (int t = 0; t < GCT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) { are[t][r] = 0; aim[t][r] = 0; }
  }

  // Block fragments of one stage (KT inner indices), software pipelined: the
  // loads of stage kt + KT (block and H) are issued before the products of
  // stage kt, so one stage of memory latency is hidden behind the matrix-core
  // work.
  constexpr int NCH = KT / CH;
  auto load_stage = [&](int kt, uint4* dst) {
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int cg = (kt + c * CH) / CW + g;
      dst[c] = (kt < NB && cg < ncg) ? ld_nt(B + (size_t)cg * NB + rowc) : make_uint4(0, 0, 0, 0);
    }
  };
  // H[c0 .. c0+GCOLS-1][kt .. kt+KT-1] of one stage, HR entries per thread,
  // loaded into registers (one stage ahead when HPF), then stored as Bs[inner][col]
  constexpr int HN = KT * GCOLS, HR = (HN + 64 * GW - 1) / (64 * GW);
  auto load_h = [&](int kt, HT* dst) {
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int idx = threadIdx.x + i * 64 * GW;
      const int col = idx / KT, kin = idx - col * KT;
      const int cc = c0 + col, kk = kt + kin;
      dst[i] = (idx < HN && cc < ncols && kk < NB) ? Hl[(size_t)cc * NB + kk] : HT{};
    }
  };
  uint4 a16[NCH], nx16[NCH];
  HT hr[HR];
  load_stage(0, a16);
  if constexpr (HPF) load_h(0, hr);
  for (int kt = 0; kt < NB; kt += KT) {
    __syncthreads();
    if constexpr (!HPF) load_h(kt, hr);
#pragma unroll
    for (int i = 0; i < HR; ++i) {
      const int idx = threadIdx.x + i * 64 * GW;
      const int col = idx / KT, kin = idx - col * KT;
      if (idx < HN) Bs[kin][col] = hr[i];
    }
    __syncthreads();
    load_stage(kt + KT, nx16);
    if constexpr (HPF) load_h(kt + KT, hr);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int kin0 = c * CH + CW * g;  // first inner index (within the stage) of this lane
      if constexpr (PREC == kFP64) {
        const double ar = __hiloint2double(a16[c].y, a16[c].x);
        const double ai = __hiloint2double(a16[c].w, a16[c].z);
        // each accumulator takes its two products of a chunk in the same order as
        // always (re: ar br, then -ai bi; im: ar bi, then ai br); the products of
        // different accumulators are interleaved so that no matrix-core
        // instruction waits on the one just issued
        double2 bv[GCT];
#pragma unroll
        for (int t = 0; t < GCT; ++t) bv[t] = reinterpret_cast<const double2&>(Bs[kin0][t * 16 + li]);
#pragma unroll
        for (int t = 0; t < GCT; ++t) {
          are[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bv[t].x, are[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bv[t].y, aim[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < GCT; ++t) {
          are[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, -bv[t].y, are[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bv[t].x, aim[t], 0, 0, 0);
        }
      } else if constexpr (PREC == kFP32) {
        const float a_r[2] = {__uint_as_float(a16[c].x), __uint_as_float(a16[c].z)};
        const float a_i[2] = {__uint_as_float(a16[c].y), __uint_as_float(a16[c].w)};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          float2 bv[GCT];
#pragma unroll
          for (int t = 0; t < GCT; ++t) bv[t] = reinterpret_cast<const float2&>(Bs[kin0 + s][t * 16 + li]);
#pragma unroll
          for (int t = 0; t < GCT; ++t) {
            are[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_r[s], bv[t].x, are[t], 0, 0, 0);
            aim[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_r[s], bv[t].y, aim[t], 0, 0, 0);
          }
#pragma unroll
          for (int t = 0; t < GCT; ++t) {
            are[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_i[s], -bv[t].y, are[t], 0, 0, 0);
            aim[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_i[s], bv[t].x, aim[t], 0, 0, 0);
          }
        }
      } else {
        // four (re, im) bf16 pairs -> four re and four im values per lane
        const uint32_t w4[4] = {a16[c].x, a16[c].y, a16[c].z, a16[c].w};
        ms4 a_r, a_i;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          a_r[e] = (short)(w4[e] & 0xFFFFu);
          a_i[e] = (short)(w4[e] >> 16);
        }
#pragma unroll
        for (int t = 0; t < GCT; ++t) {
          ms4 b_r, b_i, b_ni;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t hv = reinterpret_cast<const uint32_t&>(Bs[kin0 + e][t * 16 + li]);
            b_r[e] = (short)(hv & 0xFFFFu);
            b_i[e] = (short)(hv >> 16);
            b_ni[e] = (short)((hv >> 16) ^ 0x8000u);
          }
          are[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_r, b_r, are[t], 0, 0, 0);
          are[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_i, b_ni, are[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_r, b_i, aim[t], 0, 0, 0);
          aim[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_i, b_r, aim[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) a16[c] = nx16[c];
  }
  // accumulator lane layout: column c0 + 16 t + li; row r0 + 16 wv + (4 g + r)
  // (FP32, BF16) or r0 + 16 wv + (g + 4 r) (FP64)
#pragma unroll
  for (int t = 0; t < GCT; ++t) {
    const int col = c0 + t * 16 + li;
    if (col >= ncols) continue;
    const size_t uo = ((size_t)cb + col) * NB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = r0 + wv * 16 + (PREC == kFP64 ? g + 4 * r : 4 * g + r);
      if (rr >= NB) continue;
      if constexpr (PREC == kFP64)
        static_cast<double2*>(Ub)[uo + rr] = make_double2((double)are[t][r], (double)aim[t][r]);
      else
        static_cast<float2*>(Ub)[uo + rr] = make_float2((float)are[t][r], (float)aim[t][r]);
    }
  }
}

struct GemmGrid {
  const int* gofs;   // null: one group per leaf
  const int* gblk;
  int64_t ngroups;
  int maxcols;       // columns of the widest group
};

template <int PREC, int GW, int GCOLS>
hipError_t gemm_launch_t(hps_ctx* c, const void* blk, int ncp, const void* Hb, void* Ub, int nrhs,
                         hipEvent_t e0, hipEvent_t e1, const GemmGrid& gg) {
  const int64_t panels = ((int64_t)gg.maxcols + GCOLS - 1) / GCOLS;
  if (panels > 65535) return hipErrorInvalidConfiguration;  // grid z limit: too many columns per block
  const dim3 g3((unsigned)gg.ngroups, (unsigned)((c->nb + 16 * GW - 1) / (16 * GW)), (unsigned)panels);
  return launch_k(c, e0, e1, k_block_gemm<PREC, GW, GCOLS>, g3, dim3(64 * GW), blk, ncp, Hb, Ub, c->nb,
                  nrhs, gg.gofs, gg.gblk);
}

template <int PREC>
hipError_t gemm_launch_p(hps_ctx* c, int shape, const void* blk, int ncp, const void* Hb, void* Ub,
                         int nrhs, hipEvent_t e0, hipEvent_t e1, const GemmGrid& gg) {
  switch (shape) {
    case 0: return gemm_launch_t<PREC, 8, 64>(c, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
    case 1: return gemm_launch_t<PREC, 8, 32>(c, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
    case 2: return gemm_launch_t<PREC, 8, 16>(c, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
    case 3: return gemm_launch_t<PREC, 4, 64>(c, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
    case 4: return gemm_launch_t<PREC, 4, 32>(c, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
    default: return gemm_launch_t<PREC, 4, 16>(c, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
  }
}

}  // namespace

hipError_t gemm_launch(hps_ctx* c, int prec, int shape, const void* blk, int ncp, const void* Hb,
                       void* Ub, int nrhs, hipEvent_t e0, hipEvent_t e1, const GemmGroups* grp) {
  const GemmGrid gg = grp ? GemmGrid{grp->gofs, grp->gblk, grp->ngroups, grp->max_leaves * nrhs}
                          : GemmGrid{nullptr, nullptr, c->nl, nrhs};
  if (prec == kFP64) return gemm_launch_p<kFP64>(c, shape, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
  if (prec == kFP32) return gemm_launch_p<kFP32>(c, shape, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
  return gemm_launch_p<kBF16>(c, shape, blk, ncp, Hb, Ub, nrhs, e0, e1, gg);
}

namespace {

template <int P>
int batched_launch(hps_ctx* c, const double2* x, double2* y, int nrhs, int prec, void* Hb,
                   void* Ub, hipEvent_t e0, hipEvent_t e1) {
  const dim3 g2((unsigned)c->nl, (unsigned)nrhs);
  // with lambda buckets: panels in bucket order, one GEMM group per bucket
  const bool bk = c->lambda_bucket > 0.0;
  const int* pos = bk ? c->d_bpos : nullptr;
  hipError_t e;
  switch (prec) {
    case kFP64:
      e = launch_k(c, e0, nullptr, k_precond_pre<P, kFP64>, g2, dim3(PB), x, y, Hb, c->d_lambda,
                   c->d_tab, c->N, nrhs, pos);
      break;
    case kFP32:
      e = launch_k(c, e0, nullptr, k_precond_pre<P, kFP32>, g2, dim3(PB), x, y, Hb, c->d_lambda,
                   c->d_tab, c->N, nrhs, pos);
      break;
    default:
      e = launch_k(c, e0, nullptr, k_precond_pre<P, kBF16>, g2, dim3(PB), x, y, Hb, c->d_lambda,
                   c->d_tab, c->N, nrhs, pos);
      break;
  }
  int rc = check_hip(e, "k_precond_pre");
  if (rc) return rc;
  const Blocks& Bk = c->blk[prec];
  TimedPair tg;
  if ((rc = timing_pair(c, 2, &tg))) return rc;
  const GemmGroups gg{c->d_gofs, c->d_gblk, c->ngroups, c->group_leaves};
  const int cols = bk ? c->group_leaves * nrhs : nrhs;         // widest group
  e = gemm_launch(c, prec, gemm_shape(c->p, prec, std::min(64, cols)), Bk.data, Bk.ncp, Hb, Ub, nrhs,
                  tg.start, tg.stop, bk ? &gg : nullptr);
  if ((rc = check_hip(e, "k_block_gemm"))) {
    timing_drop(c, tg);
    return rc;
  }
  if ((rc = timing_commit(c, 2, tg))) return rc;
  if (prec == kFP64)
    e = launch_k(c, nullptr, e1, k_precond_post<P, false>, g2, dim3(PB), y, (const void*)Ub,
                 c->d_lambda, c->d_tab, c->N, nrhs, pos);
  else
    e = launch_k(c, nullptr, e1, k_precond_post<P, true>, g2, dim3(PB), y, (const void*)Ub,
                 c->d_lambda, c->d_tab, c->N, nrhs, pos);
  return check_hip(e, "k_precond_post");
}

}  // namespace

size_t batch_panel_bytes(const hps_ctx* c, int nrhs, int prec, size_t* hpad) {
  const size_t hel = prec == kFP64 ? 16 : (prec == kFP32 ? 8 : 4);
  const size_t hbytes = (size_t)c->nl * nrhs * c->nb * hel;
  const size_t ubytes = (size_t)c->nl * nrhs * c->nb * (prec == kFP64 ? 16 : 8);
  *hpad = (hbytes + 255) / 256 * 256;
  return *hpad + ubytes;
}

int launch_precond_batched(hps_ctx* c, const double2* x, double2* y, int nrhs, int prec,
                           hipEvent_t e0, hipEvent_t e1) {
  size_t hpad = 0;
  int rc = ws_reserve(c, &c->w_batch, batch_panel_bytes(c, nrhs, prec, &hpad));
  if (rc) return rc;
  void* Hb = c->w_batch.ptr;
  void* Ub = static_cast<char*>(c->w_batch.ptr) + hpad;
  switch (c->p) {
    case 4: return batched_launch<4>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 5: return batched_launch<5>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 6: return batched_launch<6>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 7: return batched_launch<7>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 8: return batched_launch<8>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 9: return batched_launch<9>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 10: return batched_launch<10>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 11: return batched_launch<11>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 12: return batched_launch<12>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 13: return batched_launch<13>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 14: return batched_launch<14>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 15: return batched_launch<15>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    case 16: return batched_launch<16>(c, x, y, nrhs, prec, Hb, Ub, e0, e1);
    default: return fail(HPS_ERR_UNSUPPORTED, "p out of range");
  }
}

}  // namespace hps
