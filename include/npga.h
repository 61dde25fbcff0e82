/*
 * npga.h - C ABI of libnpga, a gfx950 (MI355X) implementation of the NPGA
 * mean-variance solver and the Sketch-Truncate-Ridge (STR) factor builder of
 * Niu and Wang, "Scalable Mean-Variance Portfolio Optimization via Subspace
 * Embeddings and GPU-Friendly Nesterov-Accelerated Projected Gradient"
 * (arXiv 2604.02917).
 *
 * Problem (eq. mv, Sec. 1; unified model eq. npga-unified-grad, Sec. 3.1):
 *     minimise   f(x) = ||L_eff^T x||_2^2 + gamma ||x||_2^2
 *     over       F = { x in R^n : 1^T x = 1, mu^T x >= r, x >= 0 }.
 * The feasible set has no other bounds (Sec. 1 and Sec. 3.1).
 *
 * Conventions shared by every entry point
 *   - Pointers are DEVICE pointers unless the argument is marked (host).
 *   - Matrices are column-major: element (i, j) of an m x c matrix with
 *     leading dimension ld is at p[i + j * ld].  For the factor L (n x T)
 *     period t's n-vector is contiguous.
 *   - Float32 matrices must be 16-byte aligned and ld must be a multiple of
 *     4 (the kernels load float4).  Bfloat16 factors must be 8-byte aligned
 *     with ld a multiple of 4; with 16-byte alignment and ld a multiple of 8
 *     the gradient sweep loads 8 entries per lane (the fast layout).  The
 *     caller's buffer must hold ld * cols elements; rows n..ld-1 may be read
 *     but are masked and never used as data.
 *   - All work is enqueued on `stream`.  Entry points that fill a host
 *     result struct synchronise `stream` before returning.
 *   - The library never allocates device memory.  Scratch space is the
 *     caller's workspace `ws` (256-byte aligned) of at least the size the
 *     matching *_workspace_size function returns.  The library keeps no
 *     state between calls except a small pinned host status buffer per
 *     host thread (allocated on first use, kept until the process ends);
 *     every entry point that uses it synchronises `stream` before
 *     returning.  Calls from different host threads, on different streams
 *     with distinct workspaces, may run concurrently; calls sharing a
 *     workspace must not.
 *   - Return value: an npga_status code.  No C++ exception crosses the ABI.
 *     Arguments are validated before anything is enqueued; on
 *     NPGA_ERR_INVALID nothing has been launched.
 */
#ifndef NPGA_H
#define NPGA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest n supported by the register-resident projection and the fused
 * gradient sweep: one 256-thread workgroup holds 32 entries per thread. */
#define NPGA_MAX_N 8192

typedef enum npga_status {
  NPGA_OK = 0,
  NPGA_ERR_INVALID = 1,       /* bad argument; nothing was launched          */
  NPGA_ERR_INFEASIBLE = 2,    /* r > max_i mu_i, so F is empty (Sec. 3.1)    */
  NPGA_ERR_NOT_CONVERGED = 3, /* max_iter reached; x is the last iterate (in F) */
  NPGA_ERR_BRACKET = 4,       /* the dual search of Pi_F failed to bracket   */
  NPGA_ERR_NUMERIC = 5,       /* NaN or Inf met in the data or the iteration */
  NPGA_ERR_WORKSPACE = 6,     /* workspace missing, misaligned or too small  */
  NPGA_ERR_HIP = 7,           /* a HIP runtime call failed                   */
  NPGA_ERR_UNSUPPORTED = 8    /* valid request the library does not implement */
} npga_status;

typedef enum npga_path {
  NPGA_PATH_AUTO = 0, /* SYRK for a float32 factor with cols >= n whose SYRK
                         workspace (Sigma + the split planes of L, about 1.5 L)
                         is at most 4 GiB; GEMV otherwise (npga_auto_path)      */
  NPGA_PATH_GEMV = 1, /* grad = 2 L (L^T x): one fused sweep over L per step */
  NPGA_PATH_SYRK = 2  /* Sigma = L L^T once (MFMA), then grad = 2 Sigma x     */
} npga_path;

/* Effective factor L_eff and ridge gamma of the unified model
 * (Sec. 3.1, Tab. model-mapping): L (full), L Phi (sketch) or U_ell S_ell (STR). */
typedef enum npga_dtype {
  NPGA_F32 = 0,   /* float32 factor                                            */
  NPGA_BF16 = 1   /* bfloat16 factor (16-bit storage, float32 accumulation)    */
} npga_dtype;

typedef struct npga_factor {
  int64_t n;         /* assets: 1 <= n <= NPGA_MAX_N                              */
  int64_t cols;      /* columns of L_eff (T, s or ell), >= 1                      */
  int64_t ld;        /* leading dimension in elements, >= n, multiple of 4       */
  const void *L;     /* device, column-major n x cols: float32, or bfloat16 bits
                        (16-byte aligned for float32, 8-byte for bfloat16)        */
  const double *mu;  /* device, n expected returns (float64)                      */
  double gamma;      /* ridge >= 0                                                */
  int32_t dtype;     /* npga_dtype of L; the covariance (SYRK) path needs F32     */
  int32_t reserved;
} npga_factor;

/* Solver options (host).  npga_default_options fills the defaults shown. */
typedef struct npga_options {
  double tol;            /* eps of the stopping rule ||Pi_F(x - a grad f(x)) - x||_2 <= eps
                            (Sec. 3.1 "Stopping condition"); default 1e-6           */
  int32_t check_every;   /* residual cadence in iterations (Sec. 5.1); default 5     */
  int32_t max_iter;      /* default 200000                                            */
  double proj_tol;       /* dual search stops at |mu^T x - r| <= proj_tol * max(|r|, max|mu|);
                            default 1e-12 (the search normally finishes exactly)      */
  int32_t power_iters;   /* sweeps for ||L_eff||_2 (Sec. 3.1 Remark): the cap of the
                            Lanczos estimate (at most 64), or the power-method count;
                            default 20                                                 */
  double step_safety;    /* alpha = 1 / (step_safety * L_f_estimate), >= 1; default 1.05 */
  int32_t refine;        /* 1 = FP64 KKT refinement after the stop; default 1         */
  int32_t path;          /* npga_path; default NPGA_PATH_AUTO                          */
  uint64_t seed;         /* seed of the power-method start vector; default 1          */
  int32_t warm_start;    /* 1 = x holds x^0 on entry (projected onto F first)          */
  int32_t restart;       /* 1 = adaptive gradient restart of the momentum; default 0  */
  double refine_tol;     /* unused by the face-CG refinement, which stops on its own
                            KKT test (projected gradient <= 1e-10 of the gradient on
                            the support, no negative reduced cost); kept for ABI
                            stability; default 1e-9                                   */
  int32_t refine_max_iter; /* iteration cap of the refinement phase; default 20000    */
  int32_t momentum;      /* 0: the t_k sequence of Algorithm 1 (default); 1: the constant
                            beta = (1 - sqrt(alpha m_f))/(1 + sqrt(alpha m_f)) with
                            m_f = 2 gamma (Sec. 3.1 "Strongly convex specialization");
                            needs gamma > 0, else NPGA_ERR_INVALID                     */
  int32_t step_estimator; /* 0: Lanczos on L_eff L_eff^T (default), stopped when the
                            Ritz residual beta_m |s_m| is below tol theta, tol =
                            min(1e-2, max((step_safety - 1)/4, 1e-4)) for a single
                            solve and 1e-4 for a batched one; 1: the power
                            method of the paper's Remark.  Both approach ||L_eff||^2
                            from below; step_safety covers the remainder              */
  int32_t batch_config;  /* batched solves: tile configuration 0..NPGA_BATCH_CONFIGS-1
                            (see npga_batched_tune), or -1 for the built-in choice
                            from the shape; default -1                               */
  double alpha;          /* > 0: the fixed step of Algorithm 1, given by the caller
                            (Algorithm 1 takes alpha as an input; convergence needs
                            alpha <= 1/L_f); no step estimate is made.  0 (default):
                            alpha = 1/(step_safety L_f_hat) from the estimate.  Any
                            other value: NPGA_ERR_INVALID                            */
  int32_t projection;    /* step projections Pi_F: 0 = the exact scalar dual search,
                            falling back to Dykstra's alternating projections onto
                            Delta and H (Sec. 3.1) if it cannot bracket nu (default);
                            1 = Dykstra only (to 1e-14 or dykstra_iters sweeps; the
                            result lies on the simplex, mu^T x >= r to that accuracy) */
  int32_t dykstra_iters; /* sweep budget of Dykstra's method; default 5000            */
  double backtrack_rho;  /* 0 (default): fixed step.  In (0, 1): the adaptive
                            backtracking of Sec. 3.1 from the trial step alpha
                            (estimated, or the caller's): a new iterate x^{k+1} is
                            kept if f(x^{k+1}) <= f(y^k) + <grad f(y^k), d> +
                            ||d||^2/(2 alpha), d = x^{k+1} - y^k (tested as d^T Q d <=
                            ||d||^2/(2 alpha), exact for this quadratic f, with 1e-6
                            of sum |d|(|grad f(x)| + |grad f(y)|) allowed for the
                            float32 products), else alpha <- rho alpha and the step
                            is redone.  Single solves only (batched: INVALID)      */
  int32_t refine_method; /* refinement of a single solve: 0 (default) = choose from the
                            shape (below); 1 = inexact primal-dual active-set method:
                            CG on a face without step limits, the face then moved by
                            the KKT sign rules, several indices at once (falls back to 2
                            when the face does not settle); 2 = face CG with blocking
                            steps (one index fixed per block)                        */
  int32_t refine_plain_cg; /* 0 (default): the active-set refinement's face CG is
                            preconditioned on the factor path for n >= 2048 by a
                            rank-32 randomized Nystrom approximation of H (one
                            multi-vector product per refinement; the path of the
                            face solves changes, not the KKT test that ends them);
                            1: plain face CG                                      */
} npga_options;

/* Result of a solve (host). */
typedef struct npga_result {
  int32_t status;         /* npga_status of the solve                                */
  int32_t iters;          /* NPGA iterations until the stopping test first passed   */
  int32_t refine_iters;   /* iterations spent in the refinement phase               */
  int32_t support;        /* number of x_i > 0                                       */
  int32_t return_active;  /* 1 if the return constraint binds (nu > 0)              */
  int32_t refined;        /* 1 if the refinement ended on its KKT test               */
  int32_t path_used;      /* npga_path actually run                                  */
  int32_t step_sweeps;    /* gradient sweeps spent on the step-size estimate        */
  double residual;        /* stopping residual when the test first passed           */
  double final_residual;  /* residual of the returned x                             */
  double objective;       /* f(x) of the returned x, accumulated in float64         */
  double nu;              /* multiplier of mu^T x >= r (from the projection)        */
  double lambda;          /* multiplier of 1^T x = 1                                 */
  double alpha;           /* step size used                                          */
  double lipschitz;       /* estimated L_f = 2 ||L_eff||_2^2 + 2 gamma              */
  double time_ms;         /* host wall time of the whole call                       */
  double time_to_tol_ms;  /* GPU time from entry until the stopping test first passed */
  double setup_ms;        /* GPU time of checks, SYRK and step-size estimate          */
  double sweep_ms;        /* mean duration of the gradient launch (fused sweep, or the
                             covariance-path SYMV+tail), timed with HIP events on
                             `stream` around one launch per chunk of the main phase   */
  int32_t sweep_samples;  /* number of launches averaged into sweep_ms               */
  int32_t dykstra_used;   /* 1 if the step projections ran by Dykstra's method: asked
                             for (projection = 1), or the dual search could not
                             bracket nu and the solve was repeated with it          */
  int32_t backtracks;     /* trial steps refused by backtracking (main phase)       */
  int32_t refine_fallback; /* 1 if the refinement's face updates did not settle and it
                             finished with blocking face CG steps                   */
} npga_result;

/* Fill `opt` (host) with the defaults documented above. */
void npga_default_options(npga_options *opt);

/* Text for a status code (static storage). */
const char *npga_status_string(int status);

/* sizeof of this header's structures, for bindings that lay them out themselves:
 * which = 0 npga_options, 1 npga_result, 2 npga_factor, 3 npga_str_options,
 * 4 npga_backward_result; 0 for any other value.  Host only.               */
size_t npga_struct_size(int32_t which);

/* ---------------------------------------------------------------------------
 * npga_build_factor - sample mean and centred covariance factor (Sec. 2.1):
 *     mu = (1/T) R 1_T,     L = (R - mu 1_T^T) / sqrt(T - 1),
 * so that Sigma = L L^T is the unbiased sample covariance.
 *   R      device, n x T float32 returns, column-major, leading dim ldr
 *   L      device, n x T float32 output, leading dim ldl; may equal R when
 *          ldl == ldr (in place)
 *   mu_out device, n float64 output (sums accumulated in float64)
 *   ws     device workspace of npga_build_factor_workspace_size(n, T) bytes
 *          (per-workgroup partial row sums)
 * Requires 1 <= n <= NPGA_MAX_N, T >= 2, ldr, ldl >= n and multiples of 4.
 * Returns NPGA_ERR_NUMERIC (after the kernels ran) if R holds NaN or Inf.
 * Synchronises `stream`.
 * ------------------------------------------------------------------------- */
size_t npga_build_factor_workspace_size(int64_t n, int64_t T);
int npga_build_factor(const float *R, int64_t n, int64_t T, int64_t ldr,
                      float *L, int64_t ldl, double *mu_out, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* ---------------------------------------------------------------------------
 * npga_to_bf16 - Lb = bfloat16(L) by round-to-nearest-even, the storage of
 * a reduced-precision factor (sweeps then read half the bytes and
 * accumulate in float32).  L device float32 n x T (ld, multiple of 4), Lb
 * device 16-bit n x T (ldb >= n, multiple of 4, 8-byte aligned).
 * ------------------------------------------------------------------------- */
int npga_to_bf16(const float *L, int64_t n, int64_t T, int64_t ld, uint16_t *Lb, int64_t ldb,
                 hipStream_t stream);

/* ---------------------------------------------------------------------------
 * npga_solve - Algorithm 1 (NPGA, Sec. 3.1) with the fixed step
 * alpha = 1 / (step_safety * L_f_hat), L_f_hat from Lanczos (or the power
 * method) on L_eff (Sec. 3.1 Remark), FISTA momentum t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2,
 * beta_k = (t_k - 1)/t_{k+1}, and x^{k+1} = Pi_F(y^k - alpha grad f(y^k)).
 * Pi_F is computed exactly by the scalar dual search of eq. projF-dualpath
 * (Sec. 3.1).  The stopping rule is checked every check_every iterations.
 * With refine = 1 a float64 KKT refinement follows (mixed-precision
 * iterative refinement): the gradient at the stopping point x_a is
 * recomputed with float64 products, later gradients are
 * g_a + 2 L L^T (x - x_a) + 2 gamma x with the float32 sweep applied to the
 * small correction x - x_a, and the face of the active set is solved by an
 * inexact primal-dual active-set method (CG on the face, the KKT sign rules
 * move the face; on the factor path from n = 2048 the face CG is
 * preconditioned by a rank-32 Nystrom approximation of H built from one
 * multi-vector product, unless opt->refine_plain_cg) or, per refine_method,
 * by face CG with blocking steps; the result is re-anchored in float64 once
 * and the refinement ends on the KKT test (res->refined = 1).
 *   f      (host) effective factor and ridge; n <= NPGA_MAX_N
 *   r      target return R_target; r > max mu gives NPGA_ERR_INFEASIBLE
 *   opt    (host) options, or NULL for the defaults
 *   x      device, n float32: x^0 on entry if opt->warm_start, the solution
 *          on exit.  On NOT_CONVERGED it holds the last iterate, which lies
 *          in F.
 *   res    (host) result, may be NULL
 *   ws     device workspace of npga_solve_workspace_size(n, cols, opt) bytes
 * Synchronises `stream`.
 * ------------------------------------------------------------------------- */
size_t npga_solve_workspace_size(int64_t n, int64_t cols, const npga_options *opt);

/* The path NPGA_PATH_AUTO runs for a factor of this shape and npga_dtype
 * (Sec. 3.1: the factor form costs O(n cols) per iteration, the explicit
 * covariance O(n^2) after an O(n^2 cols) product): NPGA_PATH_SYRK when dtype
 * is NPGA_F32, cols >= n and the covariance path's workspace is at most
 * 4 GiB, else NPGA_PATH_GEMV; -1 for an invalid shape or dtype.  Host only.
 * npga_solve_workspace_size with opt->path = AUTO (or opt NULL) sizes for
 * the float32 choice, which also covers a bfloat16 factor (GEMV).           */
int npga_auto_path(int64_t n, int64_t cols, int32_t dtype);
int npga_solve(const npga_factor *f, double r, const npga_options *opt, float *x,
               npga_result *res, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Step-level entry points (each is one step of the solve, exposed so that
 * it can be checked on its own).
 *
 * npga_project_dykstra - x = Pi_F(v) by Dykstra's alternating projections
 *   onto Delta and H = {mu^T x >= r} (Sec. 3.1 fallback; Bauschke and
 *   Borwein 1996): y = Pi_Delta(x + p), p += x - y, x = Pi_H(y + q), q += y - x
 *   from x = v, until ||x - y||_2 and the change of y are <= tol, or max_iter
 *   sweeps (then NPGA_ERR_NOT_CONVERGED, x still returned).  x receives y (on
 *   the simplex exactly); nu_tau (host, may be NULL) the multipliers fitted on
 *   its support; iters (host, may be NULL) the sweeps.  Arguments as for
 *   npga_project.
 *
 * npga_project - x = Pi_F(v) for F above (Sec. 3.1: simplex threshold of
 *   eq. simplex-tau / simplex-proj, return face by eq. projF-dualpath).
 *   v, mu device float64 (n); x device float64 (n) output; nu_tau (host,
 *   may be NULL) receives {nu, tau}.  Returns NPGA_ERR_INFEASIBLE if
 *   r > max mu.  Uses ws of npga_solve_workspace_size(n, 1, NULL) bytes.
 *
 * npga_gradient - g = 2 L_eff (L_eff^T x) + 2 gamma x and
 *   f = ||L_eff^T x||^2 + gamma ||x||^2 (eq. npga-unified-grad) by the
 *   fused single-pass sweep.  x device float32 (n), g device float64 (n),
 *   f_out (host, may be NULL).  ws as for npga_solve.  Synchronises
 *   `stream` before returning.
 *
 * npga_spectral_norm_sq - ||L_eff||_2^2 estimated from a seeded Gaussian
 *   start (Sec. 3.1 Remark): method 1 = `iters` power-method steps (the last
 *   Rayleigh value ||L_eff^T u||^2); method 0 = Lanczos on L_eff L_eff^T, at
 *   most min(iters, 64) steps, stopped when the residual of the largest Ritz
 *   pair is below 1e-4 of the Ritz value (an eigenvalue of L_eff L_eff^T
 *   lies that close).  Both are lower bounds.  steps_out (host,
 *   may be NULL) receives the sweeps used.
 *
 * npga_syrk - Sigma = L L^T (n x n float32, column-major, leading dim lds,
 *   both triangles written) by float32 MFMA with float64 accumulation
 *   across k-chunks.  Explicit-covariance form of Sec. 3.1 (gradient 2 Sigma x).
 *
 * npga_syrk_split - the same Sigma on the bfloat16 matrix cores: every entry
 *   of L is split exactly into three bfloat16 planes (24 significant bits)
 *   and the six plane products of weight >= 2^-24 are accumulated in float32
 *   (float64 every 256 periods), which matches the float32 product to its
 *   rounding.  ws (device, 256-byte aligned) holds the planes:
 *   npga_syrk_split_workspace_size(n, T) bytes (3 n ceil64(T) bfloat16).
 *   L 16-byte aligned, ld % 4 == 0.  The solve's covariance path uses it.
 *   NPGA_ERR_WORKSPACE if ws is missing or small.
 * ------------------------------------------------------------------------- */
int npga_project(const double *v, const double *mu, int64_t n, double r, double *x,
                 double *nu_tau, void *ws, size_t ws_bytes, hipStream_t stream);
int npga_project_dykstra(const double *v, const double *mu, int64_t n, double r, int32_t max_iter,
                         double tol, double *x, double *nu_tau, int32_t *iters, void *ws,
                         size_t ws_bytes, hipStream_t stream);
int npga_gradient(const npga_factor *f, const float *x, double *g, double *f_out,
                  void *ws, size_t ws_bytes, hipStream_t stream);
int npga_spectral_norm_sq(const npga_factor *f, int32_t iters, uint64_t seed, int32_t method,
                          double *out, int32_t *steps_out, void *ws, size_t ws_bytes,
                          hipStream_t stream);
int npga_syrk(const float *L, int64_t n, int64_t T, int64_t ld, float *Sigma, int64_t lds,
              hipStream_t stream);
size_t npga_syrk_split_workspace_size(int64_t n, int64_t T);
int npga_syrk_split(const float *L, int64_t n, int64_t T, int64_t ld, float *Sigma, int64_t lds, void *ws,
                    size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * npga_sketch_str - Sketch-Truncate-Ridge (Sec. 2.5; App. D):
 *     Y = L S                       (sketch stage, S T x k, entries N(0, 1/k)),
 *     Y = U Sig V^T, keep ell       (truncation stage),
 *     L_eff = Y V_ell = U_ell Sig_ell  (n x ell; App. D "STR as one sketch"),
 *     gamma = ridge_coef * trace(Y Y^T) / n   (ridge stage; untruncated Y).
 *   L       device n x T float32 (ldl)
 *   S_opt   device T x k float32 column-major with leading dim lds >= T, or
 *           NULL to draw S on the device from `seed` (npga_sketch_str_ex)
 *   Leff    device n x ell float32 output (ldle >= n, multiple of 4)
 *   sigma   device ell float32 output: leading singular values of Y
 *   gamma_out (host) receives gamma
 *   ws      npga_sketch_workspace_size(n, T, k, ell) bytes (it includes the
 *           three bfloat16 planes of L and S, 6 (n + k) ceil64(T) bytes)
 * Requires 1 <= ell <= k <= 8192.  Y = L S runs on the bfloat16 matrix
 * cores with three-plane operands (the six plane products of weight
 * >= 2^-24 per entry product; float32 accumulation, float64 every 256
 * periods), as accurate as a float32 product.  The truncation computes the
 * top-ell eigenpairs of G = Y^T Y with a float64 Householder
 * tridiagonalisation, Sturm-count multisection and inverse iteration;
 * L_eff = Y V_ell is then the same Sigma_hat as U_ell S_ell^2 U_ell^T for
 * any orthonormal basis V_ell of that eigenspace.  Synchronises `stream`.
 * ------------------------------------------------------------------------- */
size_t npga_sketch_workspace_size(int64_t n, int64_t T, int64_t k, int64_t ell);

/* ---------------------------------------------------------------------------
 * npga_sketch_str_ex - the STR build with the options of Sec. 2.3, 2.5 and
 * App. D (npga_sketch_str is this call with a fixed ell, the trace ridge and
 * a Gaussian S, drawn on the device when S_opt is NULL):
 *   sketch    NPGA_SKETCH_GAUSSIAN: Phi = S given (so->S, leading dim lds)
 *             or drawn on the device from Philox4x32-10 (Salmon et al., SC
 *             2011; counter (t, j, 0, 0), key so->seed; Box-Muller on the
 *             first two output words: S[t, j] = sqrt(-2 ln u1) cos(2 pi u2)
 *             / sqrt(k), u1 = (w0 + 1/2) 2^-32, u2 = w1 2^-32);
 *             NPGA_SKETCH_COUNT: CountSketch Phi(t, h(t)) = s(t) with the
 *             caller's so->cs_bucket (device T int32 in [0, k), else
 *             NPGA_ERR_INVALID) and so->cs_sign (device T float32, +-1);
 *   ell_rule  NPGA_ELL_FIXED: ell = so->ell; NPGA_ELL_KNEE: App. D knee rule
 *             ell = max{i : lam_i/lam_1 >= tau, lam_{i+1}/lam_i <= rho} over
 *             the so->ell + 1 leading eigenvalues lam_i = sigma_i^2 of G
 *             (so the cap so->ell < k); NPGA_ERR_INVALID if no i qualifies;
 *   ridge     kappa_tar > 1: gamma = sigma_1^2/(kappa_tar - 1) (App. D, gives
 *             kappa(Sigma_hat) <= kappa_tar); else ridge_coef tr(Y Y^T)/n.
 * Leff (n x ell_out, ldle) and sigma (ell_out values) as npga_sketch_str;
 * *ell_out (host, may be NULL) receives the ell used.  ws:
 * npga_sketch_ex_workspace_size(n, T, so).  Synchronises `stream`.
 *
 * npga_philox_sketch - the on-device Gaussian sketch alone: S (T x k,
 * leading dim lds >= T) as above; raw (device 2 T k uint32, or NULL)
 * receives the two output words of entry (t, j) at 2 (t + j T).
 * ------------------------------------------------------------------------- */
typedef enum npga_sketch_kind { NPGA_SKETCH_GAUSSIAN = 0, NPGA_SKETCH_COUNT = 1 } npga_sketch_kind;
typedef enum npga_ell_rule { NPGA_ELL_FIXED = 0, NPGA_ELL_KNEE = 1 } npga_ell_rule;
typedef struct npga_str_options {
  int32_t sketch;            /* npga_sketch_kind                               */
  int32_t ell_rule;          /* npga_ell_rule                                  */
  int64_t k;                 /* sketch width s; default 4096                   */
  int64_t ell;               /* kept rank, or the knee rule's cap; default 512 */
  double ridge_coef;         /* default 1e-4                                   */
  double kappa_tar;          /* > 1 selects the kappa_tar ridge; default 0     */
  double knee_tau, knee_rho; /* defaults 1e-3, 0.9                             */
  uint64_t seed;             /* Philox key; default 3                          */
  const float *S;            /* device Gaussian sketch or NULL                 */
  int64_t lds;
  const int32_t *cs_bucket;  /* device, CountSketch                            */
  const float *cs_sign;      /* device, CountSketch                            */
} npga_str_options;
void npga_default_str_options(npga_str_options *so);
size_t npga_sketch_ex_workspace_size(int64_t n, int64_t T, const npga_str_options *so);
int npga_sketch_str_ex(const float *L, int64_t n, int64_t T, int64_t ldl, const npga_str_options *so,
                       float *Leff, int64_t ldle, float *sigma, int64_t *ell_out, double *gamma_out,
                       void *ws, size_t ws_bytes, hipStream_t stream);
int npga_philox_sketch(uint64_t seed, int64_t T, int64_t k, float *S, int64_t lds, uint32_t *raw,
                       hipStream_t stream);
int npga_sketch_str(const float *L, int64_t n, int64_t T, int64_t ldl, int64_t k,
                    int64_t ell, double ridge_coef, uint64_t seed, const float *S_opt,
                    int64_t lds, float *Leff, int64_t ldle, float *sigma, double *gamma_out,
                    void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * npga_solve_batched - m independent solves of eq. mv on one factor, one
 * target return r_j per solve (points of the efficient frontier, Sec. 5).
 * Every target runs Algorithm 1 with its own iterate, momentum, projection
 * and stopping test (Sec. 3.1), the shared step alpha = 1/(safety L_f_hat)
 * of one step estimate, and a float64 face refinement (face CG with
 * blocking steps; the float64 anchor gradients of all targets come from
 * two float64 matrix-core GEMMs with L).  The gradients of all targets
 * come from matrix-core GEMMs on the targets still running: in the factor form (opt->path GEMV)
 * two per iteration, U^T = X^T L and G = 2 L U, so L is read twice per
 * iteration for all m targets; in the covariance form (opt->path SYRK, or
 * AUTO with the single solve's rule: cols >= n and Sigma plus the SYRK
 * planes within 4 GiB) Sigma = L L^T is formed once (split-plane SYRK on
 * the float32 values of L, also for a bfloat16 factor) and each iteration
 * takes G = 2 Sigma X from one GEMM split over the contraction (Sec. 3.1,
 * explicit covariance).  A target that has stopped keeps its x and is
 * skipped by the tails.
 *   f          factor (float32 or bfloat16), gamma >= 0
 *   r_targets  host, m target returns, each <= max(mu) (else
 *              NPGA_ERR_INFEASIBLE before any iteration)
 *   m          1 <= m <= NPGA_MAX_BATCH
 *   X          device n x m float32, column j = x_j, leading dim ldx >= n;
 *              read as x^0 when opt->warm_start, always written
 *   res        host, m results (may be NULL); time_to_tol_ms of target j is
 *              the GPU time from entry to the end of the chunk of
 *              check_every iterations in which its stopping test passed;
 *              sweep_ms is the mean time of one iteration's gradient GEMMs
 *              over the full batch (the U+G pair, or the Sigma X GEMM)
 *   ws         npga_batched_workspace_size(n, cols, m, opt) bytes (with the
 *              covariance form: Sigma, the SYRK's bfloat16 planes of L and a
 *              float32 copy of a bfloat16 factor; never less than the factor
 *              form needs)
 * Returns NPGA_OK when every target returned NPGA_OK, else the status of the
 * first target that did not; res[j].path_used reports the form (GEMV or
 * SYRK).  Synchronises `stream`.
 *
 * npga_gradient_batched - G[:, j] = 2 L (L^T X[:, j]) + 2 gamma X[:, j] and
 * f_out[j] = ||L^T X[:, j]||^2 + gamma ||X[:, j]||^2 (float64 sums) for
 * m columns, by the batched GEMMs.  G device n x m float64 (ldg >= n);
 * f_out host m or NULL (then the call does not synchronise).  config as in
 * npga_options.batch_config.  ws: npga_batched_workspace_size(n, cols, m, NULL).
 *
 * npga_batched_tune - times each tile configuration on this factor and m
 * (reps U+G GEMM pairs each, HIP events on `stream`) and returns the fastest
 * in *best; ms_out (host, NPGA_BATCH_CONFIGS entries, may be NULL) receives
 * the mean time per pair.  Uses the workspace of npga_solve_batched.
 * ------------------------------------------------------------------------- */
#define NPGA_MAX_BATCH 1024
#define NPGA_BATCH_CONFIGS 12
size_t npga_batched_workspace_size(int64_t n, int64_t cols, int32_t m, const npga_options *opt);
int npga_solve_batched(const npga_factor *f, const double *r_targets, int32_t m,
                       const npga_options *opt, float *X, int64_t ldx, npga_result *res,
                       void *ws, size_t ws_bytes, hipStream_t stream);
int npga_gradient_batched(const npga_factor *f, const float *X, int64_t ldx, int32_t m,
                          double *G, int64_t ldg, double *f_out, int32_t config, void *ws,
                          size_t ws_bytes, hipStream_t stream);
int npga_batched_tune(const npga_factor *f, int32_t m, int32_t reps, int32_t *best,
                      float *ms_out, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * npga_backward - gradients of a loss l(x*) through the solution map
 * x*(mu, L, r, gamma) of eq. mv, by implicit differentiation of the KKT
 * conditions (Sec. 3.1 "Stopping condition") on the face of x*: the
 * support S = {x*_i > 0} and the return row when mu^T x* - r <= 1e-6
 * max(|r|, max|mu|) with a nonnegative multiplier.  With a the solution of
 *     H_SS a + a_lam 1 + a_nu mu_S = dl/dx_S,  1^T a = 0,  mu_S^T a = 0
 * (H = 2 (L L^T + gamma I); the mu row dropped when the return constraint
 * is not in the face), the gradients are
 *     dl/dmu_S = nu a - a_nu x*_S,  dl/dmu_{S^c} = 0,  dl/dr = a_nu,
 *     dl/dgamma = -2 a^T x*,        dl/dL = -2 (a u^T + x* v^T),
 * u = L^T x*, v = L^T a.  a is found by projected conjugate gradients with
 * the fused sweep for H p (float32 products) and one float64-anchored
 * correction round; for n >= 2048 with cols >= n the CG is preconditioned
 * by the same rank-32 Nystrom sketch of H as npga_solve's refinement (its
 * buffers are part of npga_backward_workspace_size).  The formula assumes the face does not change under a
 * small perturbation; res->degenerate = 1 flags a zero x_i with near-zero
 * reduced cost, |S| = 1, or mu constant on S.
 *   x_star   device n float32: a solution (e.g. from npga_solve)
 *   dl_dx    device n float32: gradient of the loss at x_star
 *   dl_dmu   device n float64 output
 *   dl_dL    device n x cols float32 output (column-major, leading dim
 *            ldg >= n), or NULL to skip it
 *   res      host, may be NULL
 *   ws       npga_backward_workspace_size(n, cols) bytes
 * Synchronises `stream`.  Returns NPGA_ERR_NOT_CONVERGED if the adjoint
 * iteration hit its cap (outputs still written).
 * ------------------------------------------------------------------------- */
typedef struct npga_backward_result {
  int32_t status;
  int32_t cg_iters;       /* projected-CG iterations, both rounds            */
  int32_t support;        /* |S|                                              */
  int32_t return_active;  /* 1 if the return row is in the face             */
  int32_t degenerate;     /* 1 if the face may change under perturbation     */
  int32_t reserved;
  double nu, lambda;      /* multipliers of f at x* (least squares on S)     */
  double dl_dr;           /* a_nu                                             */
  double dl_dgamma;       /* -2 a^T x*                                        */
  double residual;        /* ||projected residual|| / ||dl/dx_S||, float64   */
  double time_ms;         /* host wall time                                   */
} npga_backward_result;
size_t npga_backward_workspace_size(int64_t n, int64_t cols);
int npga_backward(const npga_factor *f, double r, const float *x_star, const float *dl_dx,
                  double *dl_dmu, float *dl_dL, int64_t ldg, npga_backward_result *res,
                  void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * npga_gradient_noalloc - npga_gradient without a workspace argument, for
 * callers that cannot allocate device memory (code being captured into a
 * HIP graph, serving loops that must not call the allocator).  Same result
 * as npga_gradient on the same stream, bit for bit (same kernels, same
 * launch shapes): g = 2 L_eff (L_eff^T x) + 2 gamma x, f = ||L_eff^T x||^2 +
 * gamma ||x||^2.
 *   f      (host) factor; any n <= NPGA_MAX_N and any cols fit
 *   x      device n float32;  g  device n float64 (8-byte aligned) output
 *   f_out  (host) objective, or NULL: then the call does not synchronise
 *          `stream` and enqueues kernels only (capturable)
 * Scratch: a file-scope device array of npga_gradient_noalloc_max_bytes()
 * bytes (8.25 MiB), one per device, held until the process ends; the first
 * call on a device looks up its address (make that call outside a graph
 * capture).  Every call on a device uses the same array and overwrites the
 * previous call's contents: calls that overlap on one device (two streams or
 * two host threads) race and must be serialised by the caller.  Allocates
 * nothing: no device, host or pinned allocation on any call.
 * Errors: NPGA_ERR_INVALID (bad factor or pointers, nothing launched),
 * NPGA_ERR_WORKSPACE (the request would not fit the array; cannot happen
 * for a valid factor), NPGA_ERR_HIP.
 * ------------------------------------------------------------------------- */
size_t npga_gradient_noalloc_max_bytes(void);
int npga_gradient_noalloc(const npga_factor *f, const float *x, double *g, double *f_out, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* NPGA_H */
