/*
 * dngd.h -- C ABI of libdngd, an MI355X (gfx950) implementation of the
 * Dual Natural Gradient Descent step for physics-informed tanh MLPs
 * (Jnini & Vella, "Dual Natural Gradient Descent for Scalable Training of
 * Physics-Informed Neural Networks").
 *
 * Conventions for every entry point
 *   - Return value: a dngd_status. Nothing throws across this boundary.
 *     dngd_last_error() gives a message for the last failing call on the
 *     calling thread.
 *   - Pointers documented "device" must point to memory on the current HIP
 *     device; "host" pointers to ordinary host memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the legacy
 *     default stream. Work is enqueued on it; unless a call is documented
 *     as synchronising, it returns before the work finishes.
 *   - The caller owns every buffer it passes in. A dngd_problem owns the
 *     workspace it allocates (from the stream-ordered allocator, on the
 *     stream of the call that first needs it) and frees it in
 *     dngd_problem_destroy. Stateless
 *     calls (dngd_gram, dngd_cholesky_solve, dngd_cholesky_solve_refine)
 *     take their scratch from the stream-ordered allocator of the stream's
 *     device and release it before returning; dngd_cholesky_solve_noalloc
 *     uses a static device array.
 *   - A dngd_problem is not thread-safe; use one per job and one stream per
 *     problem at a time.
 *
 * Parameter layout (theta, dtheta, gradients): per affine layer l = 1..L,
 * W_l row-major [out][in], then b_l[out]; n = sum_l (w_l * w_{l-1} + w_l).
 * Residual layout: interior points, then boundary points, then initial
 * points; m = sum over the classes of N_gamma d_gamma, where d_gamma is the
 * number of residual components per point (1 for Poisson and heat, 3 for
 * both Navier-Stokes classes); a point's components are consecutive.
 */
#ifndef DNGD_H
#define DNGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DNGD_OK = 0,
  DNGD_ENOCONV = 1,   /* warning: PCG stopped at maxit or on breakdown; x holds the last iterate */
  DNGD_EINVAL = -1,   /* bad argument; nothing was enqueued */
  DNGD_ENOMEM = -2,   /* device allocation failed */
  DNGD_EHIP = -3,     /* a HIP runtime call failed */
  DNGD_ENOTPD = -4,   /* Cholesky met a non-positive pivot; info = 1-based column */
  DNGD_ENAN = -5      /* a non-finite value in the result */
} dngd_status;

typedef enum { DNGD_F64 = 0, DNGD_F32 = 1, DNGD_BF16 = 2 } dngd_dtype;
typedef enum { DNGD_POISSON = 0, DNGD_HEAT = 1, DNGD_NAVIER_STOKES = 2 } dngd_pde;
typedef enum { DNGD_PLAIN = 0, DNGD_MIXED = 1 } dngd_precision;
/* Solvers of the step's linear systems.
 *   DNGD_DENSE       dual: Cholesky of the m x m kernel J J^T + lambda I (Section 4.1)
 *   DNGD_PCG         dual: Nystrom-preconditioned CG, matrix-free (Sections 3.3, 4.2)
 *   DNGD_PRIMAL      primal Gauss-Newton: Cholesky of the n x n matrix J^T J + lambda I,
 *                    v = -(J^T J + lambda I)^{-1} J^T r; the same step as the dual one
 *                    (Proposition 3.1), the cheaper one when n < m
 *   DNGD_DENSE_AUTO  DNGD_PRIMAL when n < m, else DNGD_DENSE (the cost model of the
 *                    dense solvers: O(m n^2 + n^3) primal against O(m^2 n + m^3) dual)
 *   DNGD_STRUCTURED  dual Cholesky on K = J J^T assembled per layer from activations and
 *                    adjoints in FP64, J never formed (Section 4); v and a by the
 *                    matrix-free reverse pass. FP64 throughout (precision, gram_passes
 *                    and ir_sweeps do not apply). Cheaper than the J Gram when the
 *                    layers are wide against the jet rows per point. */
typedef enum {
  DNGD_DENSE = 0,
  DNGD_PCG = 1,
  DNGD_PRIMAL = 2,
  DNGD_DENSE_AUTO = 3,
  DNGD_STRUCTURED = 4
} dngd_solver;

/* Problem statement (Section 2.1 and 2.2 of the paper: the PINN loss and the
 * residual map).  Residuals:
 *   interior  r_i = N_int^{-1/2} (L u(x_i) - f_i),
 *             L u = -lap u (Poisson) or u_t - kappa lap_xy u (heat),
 *   boundary  r_j = N_bdy^{-1/2} (u(x_j) - g_j),
 *   initial   r_k = N_init^{-1/2} (u(x_k) - g_k)   (heat only).
 * u is a tanh MLP with widths[0] = d_in inputs and widths[L] = 1 output.
 * Heat inputs are ordered (x_1..x_{d_in-1}, t); the Laplacian sums over the
 * spatial coordinates.
 * DNGD_NAVIER_STOKES (vector-valued classes; the steady incompressible
 * equations of Section 5.3 with viscosity nu = kappa): the MLP maps (x, y)
 * (widths[0] = 2) to (u, v, p) (widths[L] = 3). An interior point has three
 * residuals, N_int^{-1/2} times
 *     u u_x + v u_y + p_x - nu lap u - f_i0     (x-momentum)
 *     u v_x + v v_y + p_y - nu lap v - f_i1     (y-momentum)
 *     u_x + v_y - f_i2                          (continuity),
 * a boundary point three, N_bdy^{-1/2} (u - g_j0, v - g_j1, p - g_j2); f_int
 * is n_int x 3 and g_bdy n_bdy x 3 (row-major); there are no initial points.
 * Only the dense solvers (DNGD_DENSE, DNGD_PRIMAL, DNGD_DENSE_AUTO) accept it.
 * The point arrays are copied at creation. */
typedef struct {
  int32_t pde;            /* dngd_pde */
  int32_t n_layers;       /* L >= 1 affine layers */
  const int32_t* widths;  /* host, L+1 entries; 1 <= widths[0] <= 8, widths[L] == 1
                             (Navier-Stokes: widths[0] == 2, widths[L] == 3),
                             hidden widths in [1, 4096] */
  double kappa;           /* heat diffusivity, Navier-Stokes viscosity (ignored for Poisson) */
  int64_t n_int, n_bdy, n_init;  /* n_init must be 0 for Poisson */
  const double* x_int;    /* device, n_int  x d_in, row-major */
  const double* x_bdy;    /* device, n_bdy  x d_in */
  const double* x_init;   /* device, n_init x d_in (may be NULL if n_init == 0) */
  const double* f_int;    /* device, n_int  interior source f (Navier-Stokes: n_int x 3) */
  const double* g_bdy;    /* device, n_bdy  boundary value g (Navier-Stokes: n_bdy x 3) */
  const double* g_init;   /* device, n_init initial value */
} dngd_problem_desc;

typedef struct dngd_problem dngd_problem;

/* Options of one D-NGD step. dngd_step_opts_default() fills the defaults. */
typedef struct {
  int32_t precision;    /* DNGD_PLAIN: FP64 J, FP64-MFMA Gram.
                           DNGD_MIXED: FP32 J, BF16-MFMA Gram with FP32
                           accumulation, FP64 Cholesky and refinement; f_vv
                           with FP32 matrix-core layer products (FP64 jet
                           rules; dngd_fvv itself stays FP64). */
  int32_t solver;       /* dngd_solver: DNGD_DENSE (default), DNGD_PCG, DNGD_PRIMAL,
                           DNGD_DENSE_AUTO, DNGD_STRUCTURED */
  int32_t ga;           /* 1: geodesic acceleration (Section 3.2), 0: off */
  int32_t ir_sweeps;    /* mixed dense: iterative-refinement sweeps per solve (default 2) */
  int32_t gram_passes;  /* mixed: 1 (bf16 x bf16), 3 (split J ~ hi + lo, hi hi^T + hi lo^T
                           + lo hi^T), 4 (also lo lo^T: positive semidefinite),
                           DNGD_GRAM_F64 (J widened to FP64, FP64 products and sums),
                           0 = auto (default): start from D = max_i ||J_i||^2 and lambda
                           with 1 if 2^-8 sqrt(D / lambda) <= 0.02, else 3 if
                           2^-16 D <= lambda / 10, else 4; then escalate (3 -> 4 ->
                           DNGD_GRAM_F64, 1 -> 4) when the factorisation fails or the
                           refinement residual of the v solve stays above ir_tol. The
                           handle remembers the tier a step escalated to and the damping
                           it did so at; a later auto step of the same system (dual or
                           primal) with damping at or below that one starts at that tier
                           instead of repeating the attempts that failed, and a larger
                           damping clears the memory. */
  int32_t no_lookahead;  /* dense: 1 = factor without the side-stream look-ahead (default 0) */
  double eps_norm;      /* GA guard: GA only if ||v|| > eps_norm (default 0) */
  /* PCG (solver == DNGD_PCG) */
  int64_t n_landmarks;      /* l: number of landmark residuals (<= m) */
  const int64_t* landmarks; /* device, l sorted distinct residual indices in [0, m) */
  double pcg_tol;           /* stop at ||b - A y|| <= tol ||b|| (recursive residual) */
  int64_t pcg_maxit;
  double ir_tol;            /* mixed, auto Gram: escalate when ||s|| / ||r|| before the last
                               refinement sweep of the v solve exceeds this (default 1e-5) */
  /* optional device outputs (NULL = not written): the dual solution
     alpha = (K + lambda I)^{-1} r (m FP64; dual solvers only: DNGD_DENSE, DNGD_PCG,
     DNGD_STRUCTURED, and DNGD_DENSE_AUTO when it picks the dual) and f_vv (m FP64,
     any step with GA) */
  double* alpha_out;
  double* fvv_out;
  /* Nystrom preconditioner (solver == DNGD_PCG) */
  int64_t nystrom_chunk_rows;  /* jet rows per chunk of the landmark-column products
                                  (0 = sized for about 8 GB of products per chunk) */
  int32_t nystrom_reuse;       /* 0: build from `landmarks` every step (default); R > 0:
                                  reuse the factors of this handle's last PCG step for up
                                  to R further steps (landmarks are then ignored; only the
                                  l x l system is refactored when lambda changes) -- the
                                  preconditioner is built once and reused (Section 4) */
  int32_t pcg_kvp;             /* PCG kernel-vector products: DNGD_F64 (default) or
                                  DNGD_BF16 (bf16 GEMM operands, FP32 accumulation; see
                                  dngd_kvp). With DNGD_BF16 convergence is still decided
                                  on the FP64 true residual ||b - A y|| <= tol ||b||:
                                  each time the recursive residual reaches tol (or has
                                  fallen 2^10-fold since the last replacement) the true
                                  residual is formed with the FP64 product and replaces
                                  it; once a replacement finds the true residual reduced
                                  less than 8-fold, the remaining iterations use FP64
                                  products. Scalar residual classes, L >= 2. */
} dngd_step_opts;

/* gram_passes / dngd_gram passes value: FP64-product Gram of an FP32 J */
#define DNGD_GRAM_F64 64

typedef struct {
  double ms_total, ms_residual_jacobian, ms_gram, ms_factor, ms_solve_v, ms_fvv, ms_solve_a;
  double vnorm, anorm;        /* ||v||_2, ||a||_2 */
  int32_t ga_accepted;        /* 1 if dtheta = v + a/2 */
  int32_t gram_passes_used;
  int32_t pcg_iterations;
  int32_t pcg_converged;
  double ir_residual[8];      /* mixed: ||s_k|| / ||b|| before sweep k (k < ir_sweeps), v solve */
  double max_row_norm2;       /* max_i ||J_i||^2 (mixed path) */
  double pcg_rel_residual;    /* PCG: final recursive ||r|| / ||b|| */
  double ms_gram_kernel;      /* the Gram contraction kernel alone (HIP events on `stream`) */
  int32_t gram_attempts;      /* Gram + factorisation attempts (> 1 after an escalation) */
  int32_t pcg_iterations_ga;  /* PCG with GA: iterations of the second (f_vv) solve */
  int32_t primal;             /* 1 if the step solved the primal n x n system */
  int32_t ga_early_reject;    /* mixed dense dual step with GA: 1 if the correction was
                                 rejected for certain after the first refinement sweep of its
                                 solve (||a0|| - ||s0|| / (2 sqrt(lambda)) already fails the
                                 test; dtheta = v) and its remaining sweeps were skipped;
                                 anorm is then ||a0|| */
  double nystrom_shift;       /* PCG: delta added to K_II before its factorisation */
  int32_t nystrom_reused;     /* PCG: 1 if the step reused earlier Nystrom factors */
  int32_t pcg_kvp_f64;        /* PCG: FP64 kernel-vector products (iterations and true
                                 residuals; both solves with GA) */
  int32_t pcg_replacements;   /* PCG with bf16 products: recursive residuals replaced by
                                 FP64 true residuals (both solves) */
  int32_t pcg_escalated;      /* PCG with bf16 products: 1 if a solve switched to FP64 products */
  int32_t gram_start_passes;  /* mixed dense: the Gram tier the step started at (the auto
                                 choice, or the handle's remembered escalation) */
} dngd_step_stats;

const char* dngd_last_error(void);
const char* dngd_version(void);

void dngd_step_opts_default(dngd_step_opts* opts);

/* Create a problem handle: validates the description and copies the point
 * and target arrays to device memory owned by the handle. The copies are
 * complete when the call returns (the caller may free its arrays); work the
 * caller enqueued to produce them must be finished before the call. */
int dngd_problem_create(const dngd_problem_desc* desc, dngd_problem** out);
/* Waits for the handle's own work (the stream of its last call and its
 * internal stream), not for the whole device, then releases its memory.
 * Work the caller enqueued with the handle on other streams must be finished. */
int dngd_problem_destroy(dngd_problem* h);

int64_t dngd_num_params(const dngd_problem* h);     /* n */
int64_t dngd_num_residuals(const dngd_problem* h);  /* m */
int64_t dngd_jacobian_ld(const dngd_problem* h);    /* recommended ldJ: n rounded up to 256 */

/* Bytes of device memory dngd_step with `opts` needs beyond the caller's
 * buffers (activations, J, K and scratch); used for admission control.
 * Host-only, does not allocate. */
int dngd_footprint(const dngd_problem* h, const dngd_step_opts* opts, size_t* bytes);

/* The same figure from a problem description, before any device memory is
 * allocated, plus the handle's copies of the point arrays (admission control
 * of a serving loop). The description's array pointers may be NULL here.
 * Host-only. */
int dngd_footprint_desc(const dngd_problem_desc* desc, const dngd_step_opts* opts, size_t* bytes);

/* Residual map and Jacobian (Section 2.2: r(theta) and J = dr/dtheta).
 * theta: device, n FP64.  r: device, m FP64 (may be NULL).
 * J: device, m rows of ldJ elements, row-major, row i = dr_i/dtheta in the
 * parameter layout; j_dtype DNGD_F64 or DNGD_F32; may be NULL (residual
 * only); columns n..ldJ-1 are written as zero. ldJ >= n, ldJ % 4 == 0. */
int dngd_residual_jacobian(dngd_problem* h, const double* theta, double* r, void* J,
                           int64_t ldJ, int32_t j_dtype, void* stream);

/* Residual Gramian (Definition 3.3) plus damping: K = J J^T + lambda I.
 * J: device, m x ldJ row-major, j_dtype DNGD_F64 (FP64 MFMA) or DNGD_F32
 * (BF16 MFMA with FP32 accumulation; passes = 1 rounds J to bf16, passes = 3
 * uses the split J ~ hi + lo and adds hi hi^T + hi lo^T + lo hi^T, passes = 4
 * adds lo lo^T as well; passes = DNGD_GRAM_F64 widens J to FP64 and uses the
 * FP64 MFMA path).
 * Split-K partial sums are added in FP64 in a fixed order, so the result is
 * deterministic. K: device, m x ldK FP64, lower triangle (i >= j) written,
 * strict upper triangle untouched. ldK >= m. */
int dngd_gram(int64_t m, int64_t n, const void* J, int64_t ldJ, int32_t j_dtype, int32_t passes,
              double lambda, double* K, int64_t ldK, void* stream);

/* Dense dual solve (Section 4.1): Cholesky K = L L^T and B <- K^{-1} B.
 * K: device, m x ldK FP64; if factored == 0 the lower triangle holds the SPD
 * matrix on entry and L on exit; if factored == 1 it already holds L.
 * B: device, m x nrhs, column j at B + j*ldB (ldB >= m); overwritten by the
 * solution. info: host, set to 0 on success or to the 1-based column of the
 * first non-positive pivot (then DNGD_ENOTPD is returned and B is invalid).
 * Synchronises `stream` when factoring (to read info). */
int dngd_cholesky_solve(int64_t m, double* K, int64_t ldK, int32_t factored, int64_t nrhs,
                        double* B, int64_t ldB, int64_t* info, void* stream);

/* dngd_cholesky_solve without any device allocation, for callers that cannot
 * allocate: serving loops that keep hipMalloc/hipFree (and the stream-ordered
 * allocator) out of their steady state, and harnesses that forbid allocation.
 * Same arguments, kernels, results (bitwise) and error behaviour as
 * dngd_cholesky_solve. Its scratch (the info word, the factor's diagonal
 * blocks, the inverted diagonal blocks and L^T of the solves) is a static
 * device array of 65 MiB that the library holds on every device it is loaded
 * on until the process ends; m > 2048 needs more and is rejected with
 * DNGD_EINVAL before anything is enqueued. Every call on one device shares
 * that device's array: calls that overlap on one device (different host
 * threads or streams) race and give wrong results; serialise them. Each call
 * writes every scratch byte it reads, so nothing carries over between calls.
 * Factoring (factored == 0) synchronises `stream` to read info. */
int dngd_cholesky_solve_noalloc(int64_t m, double* K, int64_t ldK, int32_t factored,
                                int64_t nrhs, double* B, int64_t ldB, int64_t* info,
                                void* stream);

/* The operator that iterative refinement solves against: A = J J^T + lambda I
 * with J as given (Section 4.1, the refinement of the dense dual solve). */
typedef struct {
  const void* J;    /* device, m x ldJ row-major, 16-byte aligned */
  int64_t n;        /* columns of J (parameters), >= 1 */
  int64_t ldJ;      /* row stride in elements, >= n and a multiple of 4 */
  int32_t j_dtype;  /* DNGD_F32 or DNGD_F64 */
  int32_t sweeps;   /* refinement sweeps per right-hand side, 0 .. 16 */
  double lambda;    /* damping, finite and >= 0 */
} dngd_refine;

/* Dense dual solve with iterative refinement (Section 4.1; the
 * DenseDualSolve algorithm): B <- A^{-1} B for A = J J^T + lambda I, with the
 * Cholesky factor of K ~ A (typically the reduced-precision Gram of J plus
 * lambda I) as the inner solver. Per right-hand side b: x = K^{-1} b, then
 * `sweeps` times s = b - (J (J^T x) + lambda x) (J read in its own precision,
 * FP64 accumulation), x += K^{-1} s. K, ldK, factored, nrhs, B, ldB and info
 * as in dngd_cholesky_solve; refine must not be NULL. rel_res: host,
 * nrhs * sweeps doubles or NULL; rel_res[j * sweeps + k] = ||s|| / ||b|| of
 * sweep k of right-hand side j (a zero b gives 0). Scratch comes from the
 * stream-ordered allocator and is released before returning. Synchronises
 * `stream`. Errors: DNGD_EINVAL for bad sizes, a null J, an unaligned J or
 * ldJ, sweeps out of range or a non-finite lambda (nothing enqueued);
 * DNGD_ENOTPD as dngd_cholesky_solve (B invalid). */
int dngd_cholesky_solve_refine(int64_t m, double* K, int64_t ldK, int32_t factored,
                               int64_t nrhs, double* B, int64_t ldB, const dngd_refine* refine,
                               double* rel_res, int64_t* info, void* stream);

/* Second directional derivative of the residual along v (Section 3.2):
 * fvv = d^2/dt^2 r(theta + t v) at t = 0. theta, v: device n FP64;
 * fvv: device m FP64. */
int dngd_fvv(dngd_problem* h, const double* theta, const double* v, double* fvv, void* stream);

/* Matrix-free Jacobian products (the two passes of the kernel-vector product,
 * Definition 3.6): w = J u (forward mode) and g = J^T p (reverse mode).
 * u, g: device n FP64; w, p: device m FP64. Neither J nor K is formed. */
int dngd_jvp(dngd_problem* h, const double* theta, const double* u, double* w, void* stream);
int dngd_vjp(dngd_problem* h, const double* theta, const double* p, double* g, void* stream);

/* Kernel-vector product (Definition 3.6): w = J (J^T p) + lambda p,
 * matrix-free (a reverse pass, then a forward tangent pass), J at theta.
 * dtype DNGD_F64: FP64 products. DNGD_BF16: every per-layer product takes
 * bf16 operands with FP32 accumulation on the matrix cores and the tanh jet
 * rules run in FP32 (error of order 2^-8 ||J||^2 ||p||); scalar residual
 * classes and networks with at least one hidden layer only (else
 * DNGD_EINVAL). Activations are kept from the forward pass, not recomputed.
 * theta: device n FP64; p, w: device m FP64, w must not alias p. */
int dngd_kvp(dngd_problem* h, const double* theta, double lambda, const double* p, double* w,
             int32_t dtype, void* stream);

/* Line-search losses (D-NGD workflow): losses[k] = 0.5 ||r(theta + eta_k dtheta)||^2.
 * etas, losses: host arrays of n_eta. Synchronises `stream`. */
int dngd_losses(dngd_problem* h, const double* theta, const double* dtheta, int32_t n_eta,
                const double* etas, double* losses, void* stream);

/* Nystrom-preconditioned CG on the dual system (Sections 3.3, 4.2):
 * solves (J J^T + lambda I) x = b with the matrix-free kernel-vector product
 * and the spectral preconditioner built from the landmark residuals
 * `landmarks` (device, ell sorted distinct indices). b, x: device m FP64
 * (x is overwritten; the iteration starts from 0). stats may be NULL.
 * Returns DNGD_OK when ||b - A x|| <= tol ||b|| (recursive residual),
 * DNGD_ENOCONV after maxit iterations or a breakdown. Synchronises `stream`. */
int dngd_nystrom_pcg(dngd_problem* h, const double* theta, double lambda,
                     const int64_t* landmarks, int64_t ell, double tol, int64_t maxit,
                     const double* b, double* x, dngd_step_stats* stats, void* stream);

/* One D-NGD step (dense dual solver with geodesic acceleration, Section 4.1,
 * or the PCG step of Section 4.2): dtheta = -J^T (J J^T + lambda I)^{-1} r,
 * plus a/2 with a = -J^T (J J^T + lambda I)^{-1} f_vv when accepted
 * (2 ||a|| <= 0.5 ||v||). The primal solver computes the same v and a as
 * -(J^T J + lambda I)^{-1} J^T r and -(J^T J + lambda I)^{-1} J^T f_vv
 * (Proposition 3.1), with the same Gram precisions, refinement and escalation
 * applied to J^T. With the PCG solver, the f_vv system is solved by a
 * second PCG run with the same Nystrom preconditioner (Remark 3.5); if that run
 * does not converge the correction is rejected (dtheta = v, ga_accepted = 0).
 * theta, dtheta: device n FP64. stats: host or NULL.
 * Synchronises `stream` before returning. */
int dngd_step(dngd_problem* h, const double* theta, double lambda, const dngd_step_opts* opts,
              double* dtheta, dngd_step_stats* stats, void* stream);

/* Statistics of one optimiser iteration (dngd_iterate). */
typedef struct {
  double loss;            /* L(theta_k) = 0.5 ||r(theta_k)||^2 */
  double lambda;          /* damping used for the step */
  double eta;             /* chosen step length */
  double loss_new;        /* L(theta_k + eta dtheta) */
  double ms_line_search;  /* host wall time of the line search and update */
  int32_t eta_index;      /* index of eta in the grid */
  int32_t step_status;    /* dngd_step's status: DNGD_OK or DNGD_ENOCONV (PCG) */
  dngd_step_stats step;
} dngd_iter_stats;

/* One iteration of the D-NGD training workflow (the workflow algorithm of
 * Section 4 with the damping rule of the experiments' hyper-parameter
 * tables): lambda_k = min(L(theta_k), lambda_cap) (or lambda_fixed when it is
 * > 0; then lambda_cap is ignored), dtheta = dngd_step(theta, lambda_k, opts),
 * eta = the first minimiser of L(theta + eta dtheta) over the grid etas
 * (host, n_eta <= 48, descending order makes ties go to the longer step),
 * and theta <- theta + eta dtheta in place.
 * theta: device n FP64, updated. dtheta: device n FP64 or NULL (receives the
 * step direction). stats: host or NULL. Synchronises `stream`. Returns the
 * status of dngd_step (DNGD_OK, or DNGD_ENOCONV from a PCG step that did not
 * reach its tolerance; theta is still updated) or an error (theta unchanged
 * unless the error comes from the final update). */
int dngd_iterate(dngd_problem* h, double* theta, double lambda_cap, double lambda_fixed,
                 const dngd_step_opts* opts, int32_t n_eta, const double* etas, double* dtheta,
                 dngd_iter_stats* stats, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DNGD_H */
