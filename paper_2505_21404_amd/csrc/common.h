// Internal declarations shared by the libdngd sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

namespace dngd {

// ---------------------------------------------------------------------------
// error reporting (thread-local message, status codes of dngd.h)

void set_error(const char* fmt, ...);
int hip_fail(hipError_t e, const char* what, const char* file, int line);

#define DNGD_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) return ::dngd::hip_fail(e_, #call, __FILE__, __LINE__); \
  } while (0)

#define DNGD_LAUNCH_CHECK()                                                   \
  do {                                                                        \
    hipError_t e_ = hipGetLastError();                                        \
    if (e_ != hipSuccess) return ::dngd::hip_fail(e_, "kernel launch", __FILE__, __LINE__); \
  } while (0)

#define DNGD_REQUIRE(cond, ...)                                               \
  do {                                                                        \
    if (!(cond)) { ::dngd::set_error(__VA_ARGS__); return -1; }               \
  } while (0)

constexpr int kMaxDin = 8;        // input dimension limit (channels = d_in + 2)
constexpr int kMaxChannels = kMaxDin + 2;
constexpr int kMaxLayers = 16;
constexpr int kMaxWidth = 4096;

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// ---------------------------------------------------------------------------
// network geometry on the "jet row" layout.
//
// Every collocation point contributes C rows to the activation matrices: an
// interior point carries value, d_in input-gradient and one Laplacian channel
// (C_int = d_in + 2); a boundary or initial point carries its value only.
// Rows: interior point i, channel c -> i*C_int + c; then boundary points;
// then initial points. Activations of layer l are R x w_l FP64 row-major.

struct Geometry {
  int pde = 0;
  int L = 0;                 // affine layers
  int widths[kMaxLayers + 1] = {0};
  int64_t w_off[kMaxLayers] = {0};  // offset of W_l in theta
  int64_t b_off[kMaxLayers] = {0};  // offset of b_l in theta
  int64_t n = 0;             // parameters
  int64_t m = 0;             // residuals
  int64_t n_int = 0, n_bdy = 0, n_init = 0;
  int d_in = 0;
  int nlap = 0;              // Laplacian coordinates (d_in, or d_in - 1 for heat)
  int C_int = 0;             // channels per interior point
  int64_t R_int = 0;         // n_int * C_int
  int64_t R = 0;             // total jet rows
  double kappa = 0.0;
  double c_int = 0.0, c_bdy = 0.0, c_init = 0.0;  // N^{-1/2} class scales
  int max_width = 0;
  int d_out = 1;             // network outputs (widths[L])
  int r_int = 1, r_bdy = 1;  // residual components per interior / boundary point
};

// pde value of the steady incompressible Navier-Stokes family (dngd.h)
constexpr int kNavierStokes = 2;

// Device-side description of where a point's rows are and how its residual
// is formed from the output jet. Passed by value to kernels.
struct RowMap {
  int64_t n_int, n_bdy, n_init;
  int64_t R_int;
  int C_int;
  int d_in;
  int nlap;
  int pde;
  double kappa, c_int, c_bdy, c_init;  // kappa: heat diffusivity or Navier-Stokes viscosity
  int d_out;                  // network outputs
  int r_int, r_bdy;           // residual components per interior / boundary point
  int64_t res_bdy0, res_init0;  // first residual index of the boundary / initial class
};

RowMap row_map(const Geometry& g);

// ---------------------------------------------------------------------------
// FP64 MFMA GEMM: C = alpha * op(A) * op(B)^T-ish + beta * C (see gemm_f64.hip)

enum GemmMode {
  GEMM_FULL = 0,
  GEMM_SYRK_LOWER = 1,     // square, lower tiles only, writes row >= col
  GEMM_PARTIAL_LOWER = 2,  // lower tiles, split-K partials to work
  GEMM_FULL_LOWER = 4      // all tiles, writes only elements with row >= col
};

// op(A) is M x K: a_kcontig -> A[m*lda + k], else A[k*lda + m].
// op(B) is N x K: b_kcontig -> B[n*ldb + k], else B[k*ldb + n].
// C[m*ldc + n] = alpha * sum_k opA[m][k] opB[n][k] + beta * C  (GEMM_FULL)
// GEMM_SYRK_LOWER: only tiles/elements with m >= n (square M == N).
// GEMM_PARTIAL_LOWER: lower tiles, split-K; tile partials to `work`.
// own_cus > 0 (K-contiguous SYRK): a persistent launch of at most own_cus
// workgroups, each reserving a whole CU's LDS, so no other workgroup shares
// their CUs; the remaining CUs stay free for latency-bound kernels running
// beside it on another stream.
int gemm_f64(hipStream_t s, GemmMode mode, bool a_kcontig, bool b_kcontig, int64_t M, int64_t N,
             int64_t K, double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
             double beta, double* C, int64_t ldc, double* work = nullptr, int splits = 1,
             int own_cus = 0);

// Batched GEMM_FULL: matrix z = (z / n_inner, z % n_inner) starts at
// A + zo * a_out + zi * a_in (likewise B, C); n_outer * n_inner matrices.
// Lower-tile split-K partials of A A^T for FP32 A (M x K, K-contiguous),
// widened to FP64 on load: 128 x 128 tiles, work as in GEMM_PARTIAL_LOWER.
int gemm_f64_syrk_partial_f32(hipStream_t s, int64_t M, int64_t K, const float* A, int64_t lda,
                              double* work, int splits);
int gemm_f64_batched(hipStream_t s, bool a_kcontig, bool b_kcontig, int64_t M, int64_t N,
                     int64_t K, double alpha, const double* A, int64_t lda, int64_t a_out,
                     int64_t a_in, const double* B, int64_t ldb, int64_t b_out, int64_t b_in,
                     double beta, double* C, int64_t ldc, int64_t c_out, int64_t c_in,
                     int64_t n_outer, int64_t n_inner);

// Lower-triangular tile count for an M x M matrix with tile edge T.
int64_t lower_tiles(int64_t M, int tile);

// ---------------------------------------------------------------------------
// Gram (gram.hip)

// passes value of the FP64-product Gram of an FP32 J (dngd.h: DNGD_GRAM_F64)
constexpr int kGramF64 = 64;

size_t gram_workspace_bytes(int64_t m, int64_t n, int j_dtype, int passes, int* splits_out);
// ev_begin/ev_end (optional) are recorded on `s` around the contraction kernel alone
int gram_launch(hipStream_t s, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
                int passes, double lambda, double* K, int64_t ldK, void* work, size_t work_bytes,
                hipEvent_t ev_begin = nullptr, hipEvent_t ev_end = nullptr);

// ---------------------------------------------------------------------------
// Cholesky and triangular solves (chol.hip)

size_t chol_workspace_bytes(int64_t m);
// Factor the lower triangle in place; *dinfo (device int64) = 0 or first bad
// column (1-based); work: chol_workspace_bytes(m) of device scratch (the
// factored diagonal blocks until the final write-back); dinv (device, m
// doubles, may be null) receives 1 / L_ii.
// With `side` and two events the trailing update runs one block ahead on the
// side stream; `s` has joined it when the call's work on `s` completes.
int chol_factor(hipStream_t s, int64_t m, double* K, int64_t ldK, int64_t* dinfo, double* work,
                double* dinv, hipStream_t side = nullptr, hipEvent_t ev_panel = nullptr,
                hipEvent_t ev_trail = nullptr);
// Solves with a stored factor L: chol_prepare_solve builds the inverted
// diagonal blocks, their transposes and U = L^T into `aux`
// (chol_solve_aux_bytes(m) bytes, device); then chol_solve overwrites b with
// (L L^T)^{-1} b. aux also holds the solve's temporary vector, so one aux
// serves one solve at a time. chol_solve_aux_bytes(m) >=
// chol_workspace_bytes(m), so the same buffer can serve as chol_factor's work
// before chol_prepare_solve overwrites it.
int64_t chol_solve_block(int64_t m);
size_t chol_solve_aux_bytes(int64_t m);
int chol_prepare_solve(hipStream_t s, int64_t m, const double* L, int64_t ldL, double* aux);
int chol_solve(hipStream_t s, int64_t m, const double* L, int64_t ldL, const double* aux,
               double* b);
// y = alpha A x + beta y (A: M x K row-major)
int gemv_rows(hipStream_t s, int64_t M, int64_t K, const double* A, int64_t lda, const double* x,
              double alpha, double beta, double* y);
// B <- L^{-1} B for lower-triangular L (ell x ell) and B (ell x N row-major, ldB)
int trsm_lower_left(hipStream_t s, int64_t ell, const double* L, int64_t ldL, int64_t N, double* B,
                    int64_t ldB);

// ---------------------------------------------------------------------------
// vector kernels (blas1.hip)

// y = alpha * J^T x  (J m x ldJ, FP32 or FP64), deterministic split-M
size_t gemv_t_workspace_bytes(int64_t m, int64_t n);
int gemv_t(hipStream_t s, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
           const double* x, double alpha, double* y, double* work);
// out = r - J t - lam * x   (any of r, x may be null -> treated as 0); out has m entries
int gemv_n_residual(hipStream_t s, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
                    const double* t, const double* r, const double* x, double lam, double* out);
// deterministic sum of squares of n values -> *out (device double)
int sumsq(hipStream_t s, int64_t n, const double* x, double* out, double* work);
// max of n values -> *out (device double); NaN if any value is NaN, -inf if n == 0
int vmax(hipStream_t s, int64_t n, const double* x, double* out, double* work);
int axpy(hipStream_t s, int64_t n, double a, const double* x, double* y);  // y += a x
int xpby(hipStream_t s, int64_t n, const double* x, double beta, double* y);  // y = x + beta y
// deterministic dot product -> *out (device); work holds 256 doubles
int dot(hipStream_t s, int64_t n, const double* x, const double* y, double* out, double* work);
// z = (x - z) / lam  (last step of the Woodbury form of the preconditioner)
int woodbury_finish(hipStream_t s, int64_t n, const double* x, double inv_lam, double* z);
// out[i*ell + j] = A[i*lda + idx[j]] for i, j < ell (idx values < lda)
int gather_cols(hipStream_t s, int64_t ell, const double* A, int64_t lda, const int64_t* idx,
                double* out);
constexpr size_t kReduceWorkBytes = 256 * sizeof(double);
int copy(hipStream_t s, int64_t n, const double* x, double* y);
int fill(hipStream_t s, int64_t n, double v, double* y);
// dst (cols x rows, row-major ldd) = src^T for src (rows x cols, row-major lds), FP32 or FP64
int transpose_rm(hipStream_t s, int64_t rows, int64_t cols, const void* src, int64_t lds,
                 int j_dtype, void* dst, int64_t ldd);
// K[i][i] += v for i < n
int add_diag(hipStream_t s, int64_t n, double* K, int64_t ldK, double v);
// out[i] = ||A_i||^2 for the rows of A (rows x cols, row-major, FP32 or FP64)
int rownorm2(hipStream_t s, int64_t rows, int64_t cols, const void* A, int64_t lda, int j_dtype,
             double* out);
// dtheta = v + coef * a with coef = 0.5 if ||v|| > eps and 2||a|| <= 0.5 ||v|| else 0;
// norms2 = {||v||^2, ||a||^2} on device; flag_out (device int) = accepted.
int ga_combine(hipStream_t s, int64_t n, const double* v, const double* a, const double* norms2,
               double eps, double* dtheta, int* flag_out);

// ---------------------------------------------------------------------------
// network kernels (net.hip)

int net_input_layer(hipStream_t s, const RowMap& rm, const double* x_int, const double* x_bdy,
                    const double* x_init, double* A0, int d_in);
int net_bias_act(hipStream_t s, const RowMap& rm, int w, const double* b, double* Z, double* A);
int net_act_adjoint(hipStream_t s, const RowMap& rm, int w, const double* Z, const double* Abar,
                    double* Zbar);
// out[row * nout + o] = X[row] . wv[o*w..] + beta * Y[row] . wv2[o*w..]
int net_rowdot(hipStream_t s, int64_t R, int w, int nout, const double* X, const double* wv,
               double beta, const double* Y, const double* wv2, double* out);
int net_residual(hipStream_t s, const RowMap& rm, const double* U, const double* bias,
                 const double* f_int, const double* g_bdy, const double* g_init, double* r);
int net_linear_residual(hipStream_t s, const RowMap& rm, const double* U, const double* bias,
                        double* out);
// reverse-pass seeds (R x d_out): d/dU of sum_k w_k r_k with w = p (null: the
// Jacobian's, component comp of every point); U, bias: the forward's output jets
int net_seeds(hipStream_t s, const RowMap& rm, const double* U, const double* bias,
              const double* p, int comp, double* seed);
int net_outer_seed(hipStream_t s, int64_t R, int w, int nout, const double* seed,
                   const double* wL, double* Abar);
// Navier-Stokes residual t-derivatives (order 1: J dir, order 2: f_vv)
int net_ns_tangent(hipStream_t s, const RowMap& rm, const double* U0, const double* b0,
                   const double* U1, const double* c1, const double* U2, int order, double* out);
// pidx == null: the rows of residual component comp of every point (every row
// for one-component classes); else row q of J is point pidx[q] (q < nrows)
int net_jacobian_rows(hipStream_t s, const Geometry& g, const RowMap& rm, const double* const* A,
                      const double* const* Zbar, const double* seed, void* J, int64_t ldJ,
                      int j_dtype, double* rownorm2, const int64_t* pidx = nullptr,
                      int64_t nrows = 0, int comp = 0);
int net_tangent_act(hipStream_t s, const RowMap& rm, int w, const double* b1, const double* Z0,
                    double* Z1, double* Z2, double* A1, double* A2, int order);
// Nystrom landmark columns without J (net.hip)
int net_gather_rows(hipStream_t s, int64_t nrows, int w, const int64_t* rows, const double* src,
                    double* dst);
int net_nystrom_combine(hipStream_t s, const RowMap& rm, int64_t p0, int64_t np, int64_t row0,
                        const double* Gp, const double* Hp, int64_t ld, int64_t ell,
                        const int64_t* qoff, double* Mt, int64_t ldM, int accumulate,
                        int lower = 0);
int net_colsum_value_rows(hipStream_t s, const RowMap& rm, int w, const double* Zbar, double* out,
                          double* work);


// ---------------------------------------------------------------------------
// bf16 GEMMs with FP32 accumulation (gemm_bf16.hip). Operands bf16 (raw
// uint16 storage), row-major, K-contiguous: C = A0 B0^T + A1 B1^T (segment 1
// optional, K1 = 0), K0, K1 multiples of 32, leading dimensions multiples of
// 8, 16-byte aligned bases.
// C (M x N, FP64) = sum_s alpha_s A_s (M x K_s) B_s (N x K_s)^T + beta C for
// nseg = 1 or 2 segments of FP64 operands, row-major along K; operands are
// rounded to FP32 and multiplied on the FP32 matrix cores (gemm_f32.hip)
int gemm_f32_nt(hipStream_t s, int64_t M, int64_t N, int nseg, const double* const* A,
                const int64_t* lda, const double* const* B, const int64_t* ldb, const int64_t* K,
                const double* alpha, double beta, double* C, int64_t ldc);
int gemm_bf16_nt(hipStream_t s, int64_t M, int64_t N, const uint16_t* A0, int64_t lda0,
                 const uint16_t* B0, int64_t ldb0, int64_t K0, const uint16_t* A1, int64_t lda1,
                 const uint16_t* B1, int64_t ldb1, int64_t K1, float* C, int64_t ldc);
// Split-K variant (long K): FP64 sums of the split partials into C (ldc);
// column bias_col (if >= 0) goes to bias[row] instead.
int gemm_bf16_nt_split(hipStream_t s, int64_t M, int64_t N, const uint16_t* A, int64_t lda,
                       const uint16_t* B, int64_t ldb, int64_t K, double* C, int64_t ldc,
                       int64_t bias_col, double* bias, float* work, size_t work_bytes);
size_t gemm_bf16_split_work_bytes(int64_t M, int64_t N, int64_t K);

// low-precision product helpers (lowp.hip)
int lp_to_f32(hipStream_t s, int64_t n, const double* x, float* y);
int lp_to_bf16_pad(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                   uint16_t* dst, int64_t ldd);
int lp_transpose(hipStream_t s, const RowMap& rm, int64_t rows, int64_t cols, const void* src,
                 int src_bf16, int64_t lds, uint16_t* dst, int64_t ldd, int64_t rpad,
                 int indicator);
int lp_seed_row(hipStream_t s, int64_t R, int64_t rpad, const double* seed, uint16_t* out);
int lp_act_adjoint(hipStream_t s, const RowMap& rm, int w, int64_t ldz, const float* Zf,
                   const float* Ab, const double* seed, const double* wL, uint16_t* Zb);
int lp_tangent_act(hipStream_t s, const RowMap& rm, int w, int64_t lda, const double* b1,
                   const float* Zf, const float* Z1, uint16_t* A1);
int lp_rowdot(hipStream_t s, int64_t R, int w, int64_t ld, const uint16_t* X, const double* wx,
              const uint16_t* Y, const double* wy, double* out);

}  // namespace dngd
