// Internal declarations shared by the host orchestration (npga_api.cpp) and
// the HIP kernels (*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "npga.h"

namespace npga {

constexpr int kThreads = 256;               // workgroup size of the solver kernels
constexpr int kMaxSlots = NPGA_MAX_N / 256; // per-thread entries of an n-vector

// Termination codes kept in DevState::done.
enum DoneCode : int32_t {
  kRunning = 0,
  kConverged = 1,
  kMaxIter = 2,
  kNumeric = 3,
  kBracket = 4,
};

// Tail modes of the reduce-and-update kernel.
enum TailMode : int32_t {
  kTailNpga = 0,   // NPGA step (Algorithm 1) with the periodic stopping test
  kTailPower = 1,  // power-method step
  kTailGrad = 2,   // gradient and objective only (no update)
  kTailCG = 3,     // refinement: conjugate gradient on the identified face
  kTailAdj = 4,    // adjoint: projected conjugate gradient on the face's KKT system
  kTailLanczos = 5,  // Lanczos step for ||L_eff||_2^2 (step-size estimate)
  kTailPdas = 6,   // refinement: inexact primal-dual active-set method (CG on the face)
};

constexpr int kPdasMaxOuter = 40;  // face updates of one refinement round before the fallback

constexpr int kLanczosMax = 64;  // Lanczos steps kept in DevState

// Solver state resident in the workspace.  Written only by the single
// "tail" workgroup of a launch and read by every workgroup of later
// launches, so kernel boundaries order all accesses.
struct alignas(256) DevState {
  int32_t done;         // DoneCode
  int32_t iter;         // k: index of the current iterate x^k
  int32_t stop_iter;    // k at which the stopping test passed in the main phase
  int32_t max_iter;     // last iteration index allowed in the current phase
  uint32_t ticket;      // unused (kept for layout)
  int32_t check_every;
  int32_t restart;      // adaptive restart on/off in the current phase
  int32_t proj_flags;   // bit 0: a projection hit its pass cap; bit 1: bracket failure
  double t;             // FISTA t_k
  double beta;          // beta_{k-1} (0 at k = 0)
  double alpha;         // fixed step
  double gamma;         // ridge
  double r;             // target return
  double tol;           // stopping tolerance of the current phase
  double tolphi;        // absolute tolerance of |mu^T x - r| in the dual search
  double nu, tau;       // warm start of the step projection
  double nu_c, tau_c;   // warm start of the stopping-test projection
  double residual;      // last stopping residual
  double stop_residual; // residual when the main test passed
  double usq;           // ||L_eff^T x^k||^2 from the last sweep (float64 sum)
  double usq_sweep;     // the sweep's per-workgroup ||L^T x||^2 partials summed in a fixed order
  double objective;     // f(x^k) at the last test
  double rho2;          // power method: ||L_eff^T u||^2 (Rayleigh value)
  double mu_max, mu_absmax;
  double n_nonfinite;   // count of non-finite inputs seen by the prepare kernel
  int32_t n_restarts;
  int32_t support;
  double lambda_kkt, nu_kkt; // multipliers recovered from the stopping-test projection
  double lipschitz;     // estimated L_f
  // face conjugate-gradient refinement
  double cg_rr;         // ||r_k||^2 of the projected gradient on the face
  double cg_rr0;        // ||r||^2 at the start of the current CG cycle
  int32_t cg_active;    // return constraint held as an equality on the face
  int32_t cg_restart;   // next direction is the projected gradient
  int32_t cg_iter;      // refinement iterations so far
  int32_t cg_cycles;    // CG restarts (active-set changes)
  int32_t cg_released;  // indices released from the zero set
  int32_t cg_blocked;   // indices fixed at zero by a blocking step
  double cg_best_rr;    // smallest ||r||^2 seen in the current CG round
  int32_t cg_best_it;   // iteration at which it was seen
  int32_t cg_kkt;       // 1 if the round ended on the KKT test
  int32_t cg_window;         // iterations without halving ||r||^2 that end a refinement round
  int32_t cg_pg;             // 1: a projected-gradient step w is pending (its H (w - x) is being swept)
  double cg_pg_nu;           // return multiplier of that step's projection
  int32_t const_momentum;    // 1: beta_k = beta_const instead of the t_k sequence
  double beta_const;
  // Lanczos tridiagonal T_m of L_eff L_eff^T (step-size estimate)
  int32_t lz_m;
  double lz_theta;                 // largest Ritz value of T_m
  double lz_tol;                   // stop when the Ritz residual is below lz_tol theta
  int32_t dykstra_iters;           // sweep budget of Dykstra's projections (when the tails run them)
  // adaptive backtracking (Sec. 3.1)
  double bt_rho;                   // step shrink factor
  int32_t bt_pending;              // 1: x^k is a trial point of the step from y^{k-1}
  int32_t bt_rejections;           // trial steps refused so far
  int32_t bt_consec;               // refusals of the current trial
  double lz_alpha[kLanczosMax];
  double lz_beta[kLanczosMax];
  // inexact primal-dual active-set refinement
  int32_t pdas_outer;              // face updates in the current round
  int32_t pdas_final;              // 1: the face is settled, CG runs to the KKT tolerance
  int32_t pdas_failed;             // 1: the round hit kPdasMaxOuter (x was projected onto F)
  int32_t pdas_moved;              // indices moved by face updates in the current round
  double pdas_eta2;                // inner CG tolerance ||r||^2 <= eta2 ||r_0||^2
  double pcg_rz;                   // preconditioned face CG: g^T z of the current direction
  int32_t pcg_todo;                // after the tail: 0 nothing, 1 next direction, 2 new face
  int32_t pcg_arrive;              // workgroups of the direction's last launch that have finished
  double pcg_lam0, pcg_nu0;        // the tail's least-squares multipliers of the current g
  // adjoint results
  double adj_alam, adj_anu;  // multipliers of the adjoint system (a_lam, a_nu)
  double adj_dgamma;         // dl/dgamma
  double adj_res;            // relative projected residual of the adjoint solve
};

// Host-visible status block copied back once per chunk of iterations.
struct alignas(64) HostStatus {
  int32_t done;
  int32_t iter;
  int32_t stop_iter;
  int32_t proj_flags;
  double residual;
  double mu_max;
  double n_nonfinite;
  double rho2;
};

// Everything a solver kernel needs, passed by value.
struct SolveArgs {
  const void *L;       // n x cols, leading dim ld (float32 or bfloat16 bits)
  int32_t dtype;       // NPGA_F32 or NPGA_BF16
  int64_t ld;
  int64_t n;
  int64_t cols;
  const double *mu;    // n
  float *xs;           // sweep input, float32, padded to 256 * slots with zeros
  double *xbuf0;       // iterate ping-pong buffers (float64, n)
  double *xbuf1;
  double *gbuf0;       // gradient ping-pong buffers (float64, n)
  double *gbuf1;
  float *partials;     // sweep partial sums, [grid][ldp]
  double *usq_part;    // per-workgroup partial ||L^T x||^2, [grid]
  int64_t ldp;         // leading dimension of partials (>= 256 * slots)
  int32_t sweep_grid;  // number of workgroups of the sweep launch
  int32_t mode;        // TailMode
  int32_t dykstra;     // 1: the tails project by Dykstra's method (their DYK instantiation)
  int32_t backtrack;   // 1: adaptive backtracking (the tails' BT instantiation)
  double *ybt;         // backtracking: y^k of the pending trial (n)
  double *gybt;        // backtracking: grad f(y^k) (n)
  DevState *st;
  // refinement anchor (all null outside the refinement phase): the sweep
  // runs on d = x - xa and adds the float64 anchor terms
  const double *xa;    // anchor x_a (n)
  const double *ga;    // 2 L (L^T x_a), float64 products (n)
  const double *ua;    // L^T x_a, float64 products (cols; factor path only)
  // face conjugate-gradient refinement vectors (float64, n)
  double *pvec;        // search direction p
  double *fvec;        // 1 where x_i is free on the face, 0 where x_i is fixed at 0
  double *gvec;        // gradient maintained by linearity
  // when set (the last iteration of a chunk), the one-workgroup tail stores
  // st->done here at its end: a word of pinned host memory the host reads
  // once the chunk's event has passed
  int32_t *host_done;
  // preconditioned face solves of the active-set refinement (null: plain CG):
  // Y = H Omega row-major (n x kPreK float32) and column-major (column c at
  // pre_yt + c ldp), pre_mat = S, the Cholesky factor of K and scalars,
  // a1 / a2 = M_F^{-1} 1_F / M_F^{-1} mu_F (n)
  const float *pre_y;
  const float *pre_yt;
  double *pre_mat;
  double *pre_a1;
  double *pre_a2;
  // a direction on an unchanged face spread over one workgroup per 256
  // rows: z = M_F^{-1} r before its projection (n) and the workgroups'
  // partial sums (kPreMaxRowBlocks x (kPreK + 5))
  double *pre_z;
  double *pre_part;
  // the row blocks' partial products of a face change, per block of 512
  // rows: Y_F^T Y_F, then Omega^T Y (kPreMaxRowBlocks / 2 x 2 x kPreK^2);
  // from kPreGpartT, Y_F^T 1_F and Y_F^T mu_F (2 x kPreK per block)
  double *pre_gpart;
};

// Rank of the Nystrom sketch of the refinement's preconditioner, the
// per-thread rows of its 512-thread kernel, and the doubles of pre_mat.
constexpr int kPreK = 32;
constexpr int kPcgMaxE = 16;
constexpr int kPreMatDoubles = 2 * kPreK * kPreK + 8;
constexpr int kPreMaxSplits = 64;  // period ranges of the multi-vector product's G GEMM
constexpr int kPreMaxRowBlocks = 32;  // 256-row blocks of the spread direction (n <= 8192)
constexpr int kPreGpartT = kPreMaxRowBlocks * kPreK * kPreK;
constexpr int kPreGpartDoubles = kPreGpartT + kPreMaxRowBlocks * kPreK;

// m independent solves sharing L (one target return per solve).  Target j
// uses the SolveArgs of target 0 with every per-target pointer advanced by
// j strides; the gradient of all targets comes from two skinny GEMMs,
//     U^T = X^T L   (Ut[j + t ldut] = sum_i X[i, j] L[i, t])
//     G   = L U     (split over t: P[s][i][j] partial sums)
// followed by a reduce that applies each target's epilogue.
struct BatchArgs {
  SolveArgs base;      // target 0; base.xs is X (n x m float32, column stride ldx)
  int32_t m;
  int64_t vstride;     // doubles between consecutive targets' n-vectors
  int64_t gstride;     // doubles between targets' gradient buffers (gbuf0/gbuf1)
  int64_t ldx;         // floats between consecutive columns of X
  float *Ut;           // U^T, m x cols, leading dim ldut
  int64_t ldut;
  float *P;            // G partials: P[(s * n + i) * ldpm + j]
  int64_t ldpm;
  int32_t splits;      // number of t-ranges of the G GEMM
  int64_t kchunk;      // t-range length of one split (multiple of 32)
  double *usq_part;    // per-tile ||U_{:,j}||^2 partials: [tile * ldq + j]
  int64_t ldq;
  int32_t utiles;      // number of row tiles of the U GEMM
  // GEMM columns are the running targets only: column c < *mact is target
  // act[c] (ascending); U^T and P are indexed by c, everything else by j
  const int32_t *act;
  const int32_t *mact;
  // bfloat16 factors on the bfloat16 matrix cores (null otherwise): a
  // row-major copy Lt[i * ldlt + t] of L and U as three bfloat16 planes
  // U16[pl * u16plane + c * ldu16 + t]
  const uint16_t *Lt;
  int64_t ldlt;
  uint16_t *U16;
  int64_t ldu16;
  int64_t u16plane;
  // covariance form (base.L = Sigma, n x n float32, base.cols = n): the
  // gradient is 2 Sigma X by one GEMM split over the contraction into
  // `splits` ranges of `kchunk` rows; the tails take f = x^T g / 2
  int32_t covariance;
  // when set, Sigma as three bfloat16 planes (row i of plane p at
  // Sp + p spplane + i ldsp, zeros past n): the GEMM runs on the bfloat16
  // matrix cores with X split into planes as it is staged
  const uint16_t *Sp;
  int64_t ldsp;
  int64_t spplane;
};

// Tile configuration of the two batched GEMMs.
struct BatchConfig {
  int32_t u_bm, u_bn;  // U GEMM tile (rows of U = periods t, columns = targets)
  int32_t g_bm, g_bn;  // G GEMM tile (rows of G = assets i, columns = targets)
  int32_t splits;      // t-splits of the G GEMM
};

constexpr int kBatchConfigs = 12;
extern const BatchConfig kBatchConfigTable[kBatchConfigs];
int batch_default_config(int64_t n, int64_t cols, int32_t m);

// Workspace carving for a solve.
struct SolveLayout {
  size_t off_state, off_status_dev, off_xs, off_x0, off_x1, off_g0, off_g1, off_part, off_usq,
      off_sigma, off_planes, off_vecs, off_bt, off_xa, off_ga, off_ua, total;
  // the refinement's preconditioner (pcg): Y, pre_mat, a1, a2, and the
  // multi-vector product's GEMM buffers (Omega, U^T, split partials, column
  // sums, active list)
  size_t off_pre_y, off_pre_yt, off_pre_mat, off_pre_a1, off_pre_a2, off_pre_x, off_pre_ut, off_pre_p, off_pre_usq,
      off_pre_act, off_pre_z, off_pre_part, off_pre_gpart;
  bool pcg;
  int32_t slots;
  int32_t sweep_grid;
  int64_t ldp;
};

int slots_for(int64_t n);
SolveLayout solve_layout(int64_t n, int64_t cols, int path, bool pcg = false);
int sweep_grid_for(int64_t cols);

// ---- launchers (defined in the .hip files; return hipError_t as int) ----
int launch_prepare(const SolveArgs &a, hipStream_t s);
int launch_set_vector(double *dst, const float *src32, const double *src64, int64_t n, double fill,
                      float *xs, hipStream_t s);
int launch_random_unit(double *u, float *xs, int64_t n, uint64_t seed, hipStream_t s);
int launch_sweep(const SolveArgs &a, int slots, hipStream_t s);
int launch_reduce_tail(const SolveArgs &a, int slots, hipStream_t s);
int launch_tail(const SolveArgs &a, int slots, int covariance, hipStream_t s);
int launch_project_init(const SolveArgs &a, int slots, int use_x0, hipStream_t s);
int launch_project_only(const double *v, const double *mu, int64_t n, double *x, DevState *st,
                        int slots, hipStream_t s);
int launch_project_dykstra(const double *v, const double *mu, int64_t n, double *x, DevState *st, int max_iter,
                           double tol, int slots, hipStream_t s);
int launch_finalize(const SolveArgs &a, float *x_out, int slots, hipStream_t s);
int launch_phase(DevState *st, int32_t phase_kind, double tol, int32_t max_iter, int32_t restart,
                 hipStream_t s);
int launch_set_tolphi(DevState *st, double proj_tol, hipStream_t s);
int launch_set_alpha(DevState *st, double step_safety, hipStream_t s, double alpha_fixed = 0.0);  // also beta_const

int launch_lanczos_init(const SolveArgs &a, double tol, hipStream_t s);

// Symmetric rank-T update Sigma = L L^T (MFMA) and the covariance-path kernels.
int launch_syrk(const float *L, int64_t n, int64_t T, int64_t ld, float *Sigma, int64_t lds,
                hipStream_t s);
int launch_symv_tail(const SolveArgs &a, const float *Sigma, int64_t lds, int slots,
                     hipStream_t s);
int launch_symv(const SolveArgs &a, const float *Sigma, int64_t lds, int slots, hipStream_t s);
// Sigma = L L^T by bfloat16 matrix cores on three-plane operands; planes:
// syrk_split_bytes(n, T) bytes of scratch (16-byte aligned)
size_t syrk_split_bytes(int64_t n, int64_t T);
int launch_syrk_split(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *planes, float *Sigma,
                      int64_t lds, hipStream_t s);
// C (M x N) = A B, A[m + k lda] (rows contiguous), B[k + n ldb] (contraction
// contiguous), on the same three-plane bfloat16 matrix cores; planes:
// gemm_split_bytes(M, N, K) bytes of scratch (16-byte aligned)
size_t gemm_split_bytes(int64_t m, int64_t ncols, int64_t K);
int launch_gemm_split(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc, int64_t M,
                      int64_t N, int64_t K, uint16_t *planes, hipStream_t s);
// Three bfloat16 planes of `rows` float32 rows contiguous along T (row j at
// X + j ldx): P[p plane + j ldt + t], zeros for t in [T, ldt), ldt % 8 == 0.
int launch_split_rows(const float *X, int64_t rows, int64_t T, int64_t ldx, uint16_t *P, int64_t ldt,
                      int64_t plane, hipStream_t s);

// Preconditioner set-up of the refinement: Omega (signs) into the batched
// GEMM input X (column c at X + c ldx), and Y[i][c] = 2 sum_s P[s][i][c]
// (the split partials of the GEMM pair, fixed order) in float32, row-major
// into Y and column-major (column c at Yt + c ldyt) into Yt.
int launch_pre_omega(float *X, int64_t ldx, int64_t n, hipStream_t s);
int launch_pre_reduce(const float *P, int64_t ldpm, int32_t splits, int64_t n, float *Y, float *Yt, int64_t ldyt,
                      hipStream_t s);
// Preconditioned start of a refinement round (after launch_cg_init): the
// first round forms S and estimates sigma, later rounds reuse them.
int launch_pcg_init(const SolveArgs &a, int slots, bool first, hipStream_t s);

// Float64 anchor gradient for the refinement phase.
int launch_precise_gradient(const SolveArgs &a, const double *x, double *u_out, double *g_out,
                            double *part, int slots, hipStream_t s);
// The same for a batch: G[j ldg + i] = 2 (L L^T x_j)_i for every target j
// with st[j].done == kConverged (X[j ldxv + i]), 0 for the others; scratch:
// precise_batch_bytes(n, T, m, npad) bytes (256-byte aligned), npad >= n.
struct PreciseBatchPlan {
  int64_t kc;       // periods per range of the split G GEMM (a multiple of 16)
  int32_t splits;   // number of ranges
  int64_t ldu;      // leading dimension of U^T (float64, m x T)
  size_t u_bytes;
};
PreciseBatchPlan precise_batch_plan(int64_t n, int64_t T, int32_t m);
size_t precise_batch_bytes(int64_t n, int64_t T, int32_t m, int64_t npad);
int launch_precise_gradient_batched(const void *L, int32_t dtype, int64_t ld, int64_t n, int64_t T,
                                    const double *X, int64_t ldxv, int32_t m, const DevState *st, double *scratch,
                                    int64_t npad, double *G, int64_t ldg, hipStream_t s);
int launch_phase_reset(DevState *st, double tol, int32_t max_iter, int32_t window, hipStream_t s);
int launch_cg_init(const SolveArgs &a, int slots, hipStream_t s);
int launch_add_ridge(const SolveArgs &a, hipStream_t s);  // gbuf0 += 2 gamma pvec

// Batched solves (npga_batched.hip).
int launch_bgemm(const BatchArgs &b, const BatchConfig &c, hipStream_t s);
int launch_breduce_tail(const BatchArgs &b, int slots, hipStream_t s);
int launch_bproject_init(const BatchArgs &b, int slots, hipStream_t s);
int launch_bcg_init(const BatchArgs &b, int slots, hipStream_t s);
int launch_bfinalize(const BatchArgs &b, float *X, int64_t ldx_out, hipStream_t s);
int launch_bset_x0(const BatchArgs &b, const float *X0, int64_t ldx0, hipStream_t s);
int launch_bcopy_step(const BatchArgs &b, const DevState *src, hipStream_t s);
int launch_bload_x(const BatchArgs &b, const float *X, int64_t ldx_in, hipStream_t s);
int launch_bphase_reset(const BatchArgs &b, double tol, int32_t max_iter, hipStream_t s);
int launch_bcopy_anchor(const BatchArgs &b, hipStream_t s);
int launch_bstatus(const BatchArgs &b, int32_t *out, int32_t *act, int32_t *mact, hipStream_t s);
int launch_bact_all(const BatchArgs &b, int32_t *act, int32_t *mact, hipStream_t s);
int launch_zero_f32(float *p, int64_t count, hipStream_t s);
int launch_b16_gemm(const BatchArgs &b, const BatchConfig &c, hipStream_t s);
int launch_transpose16(const uint16_t *L, int64_t ld, int64_t n, int64_t T, uint16_t *Lt, int64_t ldlt,
                       hipStream_t s);
int launch_widen_bf16(const uint16_t *L, int64_t ld, int64_t n, int64_t T, float *L32, int64_t ld32, hipStream_t s);

// Adjoint (npga_adjoint.hip).  Vectors: x* in xbuf1, the face gradient
// 2 L L^T x* in ga, the loss gradient rhs in xa, the CG iterate in xbuf0.
int launch_adj_face(const SolveArgs &a, int slots, double act_tol, hipStream_t s);
int launch_adj_init(const SolveArgs &a, const double *rhs, int slots, hipStream_t s);
int launch_adj_rhs(int64_t n, double gamma, const double *gl, const double *abase, const double *hab, double *rhs,
                   hipStream_t s);
int launch_adj_accum(const SolveArgs &a, double *abase, hipStream_t s);
int launch_adj_finish(const SolveArgs &a, const double *gl, const double *abase, const double *hab,
                      double *dl_dmu, int slots, hipStream_t s);
int launch_adj_dL(const double *ahat, const double *x, const double *u, const double *v, int64_t n, int64_t cols,
                  float *dL, int64_t ldg, hipStream_t s);

// Factor build.
int launch_to_bf16(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *Lb, int64_t ldb,
                   hipStream_t s);
int launch_build_factor(const float *R, int64_t n, int64_t T, int64_t ldr, float *L, int64_t ldl,
                        double *mu_out, double *part, int grid, double *nonfinite,
                        hipStream_t s);

}  // namespace npga
