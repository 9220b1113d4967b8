// HBM-bound vector kernels of the dense dual step (Section 4.1): the
// recovery product J^T y (velocity and acceleration, alpha form of the dual
// recovery formula), the refinement residual s = r - J (J^T x) - lambda x,
// deterministic norms and the geodesic-acceleration acceptance rule.
//
// J^T y: J is m x ldJ row-major, so a column sum is a strided reduction.
// Each thread owns 4 adjacent columns (one 16-byte FP32 / 32-byte FP64 load
// per row, coalesced across the wave) and a contiguous band of rows; the
// per-band partial sums are added in FP64 in band order by a second kernel.
// J t: 4 rows per workgroup so each slab of t (FP64, 2x the bytes of an FP32
// row slab) is loaded once for 4 rows, with enough workgroups to fill the chip.
// Both read J once per call, through nontemporal (streaming) loads.
#include "common.h"

namespace dngd {

namespace {

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  __device__ static inline void load(const float* p, double (&v)[4]) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
  }
  // J read once per call: a streaming (nontemporal) load
  __device__ static inline void stream(const float* p, double (&v)[4]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 x = __builtin_nontemporal_load(reinterpret_cast<const f4*>(p));
    v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
  }
};
template <>
struct Vec4<double> {
  __device__ static inline void load(const double* p, double (&v)[4]) {
    const double2 x = *reinterpret_cast<const double2*>(p);
    const double2 y = *reinterpret_cast<const double2*>(p + 2);
    v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
  }
  __device__ static inline void stream(const double* p, double (&v)[4]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 x = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    const d2 y = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p + 2));
    v[0] = x[0]; v[1] = x[1]; v[2] = y[0]; v[3] = y[1];
  }
};

template <typename T>
__global__ __launch_bounds__(256) void gemv_t_partial_kernel(int64_t m, int64_t n,
                                                             const T* __restrict__ J, int64_t ldJ,
                                                             const double* __restrict__ x,
                                                             int64_t rows_per, double* __restrict__ part) {
  const int64_t c = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per;
  const int64_t r1 = min(m, r0 + rows_per);
  double acc[4] = {0, 0, 0, 0};
  if (c < n) {
    for (int64_t r = r0; r < r1; ++r) {
      double v[4];
      Vec4<T>::stream(J + r * ldJ + c, v);
      const double xr = x[r];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += v[e] * xr;
    }
    double* out = part + (int64_t)blockIdx.y * n;
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (c + e < n) out[c + e] = acc[e];
  }
}

__global__ __launch_bounds__(256) void gemv_t_reduce_kernel(int64_t n, int splits,
                                                            const double* __restrict__ part,
                                                            double alpha, double* __restrict__ y) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int k = 0; k < splits; ++k) s += part[(int64_t)k * n + c];
  y[c] = alpha * s;
}

constexpr int GN_ROWS = 4;

template <typename T>
__global__ __launch_bounds__(256) void gemv_n_kernel(int64_t m, int64_t n, const T* __restrict__ J,
                                                     int64_t ldJ, const double* __restrict__ t,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ x, double lam,
                                                     double* __restrict__ out) {
  __shared__ double red[4][GN_ROWS];
  const int64_t row0 = (int64_t)blockIdx.x * GN_ROWS;
  double acc[GN_ROWS];
#pragma unroll
  for (int q = 0; q < GN_ROWS; ++q) acc[q] = 0.0;
  // all loads of an iteration unconditional (rows beyond m read row m - 1 and
  // are dropped at the end): a conditional load is waited for before the
  // next one is issued
  for (int64_t k = (int64_t)threadIdx.x * 4; k < n; k += 1024) {
    double tv[4], v[GN_ROWS][4];
    if (k + 3 < n) {
      Vec4<double>::load(t + k, tv);
#pragma unroll
      for (int q = 0; q < GN_ROWS; ++q) Vec4<T>::stream(J + min(row0 + q, m - 1) * ldJ + k, v[q]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t kc = min(k + e, n - 1);
        tv[e] = t[kc];
#pragma unroll
        for (int q = 0; q < GN_ROWS; ++q) v[q][e] = (double)J[min(row0 + q, m - 1) * ldJ + kc];
        if (k + e >= n) {
          tv[e] = 0.0;
#pragma unroll
          for (int q = 0; q < GN_ROWS; ++q) v[q][e] = 0.0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < GN_ROWS; ++q)
      acc[q] += v[q][0] * tv[0] + v[q][1] * tv[1] + v[q][2] * tv[2] + v[q][3] * tv[3];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < GN_ROWS; ++q) {
    double s = acc[q];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) red[wave][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < GN_ROWS) {
    const int q = threadIdx.x;
    const int64_t row = row0 + q;
    if (row < m) {
      const double jt = red[0][q] + red[1][q] + red[2][q] + red[3][q];
      double o = -jt;
      if (r) o += r[row];
      if (x) o -= lam * x[row];
      out[row] = o;
    }
  }
}

constexpr int SS_BLOCKS = 256;

__global__ __launch_bounds__(256) void sumsq_partial_kernel(int64_t n, const double* __restrict__ x,
                                                            double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)SS_BLOCKS * 256)
    s += x[i] * x[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void sumsq_final_kernel(const double* __restrict__ part,
                                                          double* __restrict__ out) {
  __shared__ double red[4];
  double s = part[threadIdx.x];  // SS_BLOCKS == 256
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// max with NaN propagation: a NaN anywhere makes the result NaN
__device__ inline double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return b > a ? b : a;
}

__global__ __launch_bounds__(256) void vmax_partial_kernel(int64_t n, const double* __restrict__ x,
                                                           double* __restrict__ part) {
  __shared__ double red[4];
  double s = -HUGE_VAL;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)SS_BLOCKS * 256)
    s = nanmax(s, x[i]);
  for (int off = 32; off > 0; off >>= 1) s = nanmax(s, __shfl_xor(s, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void vmax_final_kernel(const double* __restrict__ part,
                                                         double* __restrict__ out) {
  __shared__ double red[4];
  double s = part[threadIdx.x];  // SS_BLOCKS == 256
  for (int off = 32; off > 0; off >>= 1) s = nanmax(s, __shfl_xor(s, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = nanmax(nanmax(red[0], red[1]), nanmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void dot_partial_kernel(int64_t n, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          double* __restrict__ part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)SS_BLOCKS * 256)
    s += x[i] * y[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// z = (x - z) * inv_lam
__global__ void woodbury_finish_kernel(int64_t n, const double* __restrict__ x, double inv_lam,
                                       double* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) z[i] = (x[i] - z[i]) * inv_lam;
}

// out[i*ell + j] = A[i*lda + idx[j]]  (i, j < ell)
__global__ void gather_cols_kernel(int64_t ell, const double* __restrict__ A, int64_t lda,
                                   const int64_t* __restrict__ idx, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= ell * ell) return;
  const int64_t i = e / ell, j = e % ell;
  out[e] = A[i * lda + idx[j]];
}

// y = x + beta * y
__global__ void xpby_kernel(int64_t n, const double* __restrict__ x, double beta,
                            double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[i] + beta * y[i];
}

__global__ void axpy_kernel(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}
__global__ void copy_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = x[i];
}
__global__ void fill_kernel(int64_t n, double v, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = v;
}

// dst[j][i] = src[i][j] for src rows x cols (row-major, lds), dst cols x rows
// (row-major, ldd): 64 x 64 tiles through LDS, both sides coalesced.
template <typename T>
__global__ __launch_bounds__(256) void transpose_rm_kernel(int64_t rows, int64_t cols,
                                                           const T* __restrict__ src, int64_t lds,
                                                           T* __restrict__ dst, int64_t ldd) {
  __shared__ T tile[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    tile[i][tx] = (r < rows && c < cols) ? src[r * lds + c] : T(0);
  }
  __syncthreads();
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < cols && r < rows) dst[c * ldd + r] = tile[tx][i];
  }
}

// out[i] = sum_k A[i][k]^2 (one workgroup per row, fixed reduction order)
template <typename T>
__global__ __launch_bounds__(256) void rownorm2_kernel(int64_t cols, const T* __restrict__ A,
                                                       int64_t lda, double* __restrict__ out) {
  __shared__ double red[4];
  const T* a = A + (int64_t)blockIdx.x * lda;
  double ss = 0.0;
  for (int64_t k = threadIdx.x; k < cols; k += 256) {
    const double x = (double)a[k];
    ss += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void add_diag_kernel(int64_t n, double* __restrict__ K, int64_t ldK, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) K[i * ldK + i] += v;
}

__global__ void ga_combine_kernel(int64_t n, const double* __restrict__ v, const double* __restrict__ a,
                                  const double* __restrict__ norms2, double eps,
                                  double* __restrict__ dtheta, int* flag_out) {
  const double vn = sqrt(norms2[0]);
  const double an = sqrt(norms2[1]);
  const bool acc = (vn > eps) && (2.0 * an <= 0.5 * vn);
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  // a rejected correction leaves v exactly and never reads a (which the
  // early rejection does not compute: 0 * a would turn stale non-finite
  // values into NaN)
  if (i < n) dtheta[i] = acc ? v[i] + 0.5 * a[i] : v[i];
  if (i == 0 && flag_out) *flag_out = acc ? 1 : 0;
}

int gemv_t_splits(int64_t m, int64_t n) {
  const int64_t cb = cdiv(n, 1024);
  int64_t s = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, cb));
  s = std::min<int64_t>(s, cdiv(m, 32));
  s = std::min<int64_t>(s, 64);
  return (int)std::max<int64_t>(1, s);
}

}  // namespace

size_t gemv_t_workspace_bytes(int64_t m, int64_t n) {
  return (size_t)gemv_t_splits(m, n) * (size_t)n * sizeof(double);
}

int gemv_t(hipStream_t s, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
           const double* x, double alpha, double* y, double* work) {
  DNGD_REQUIRE(ldJ % 4 == 0, "gemv_t: ldJ %% 4 != 0");
  const int S = gemv_t_splits(m, n);
  const int64_t rows_per = cdiv(m, S);
  dim3 grid((unsigned)cdiv(n, 1024), (unsigned)S);
  if (j_dtype == 0)
    hipLaunchKernelGGL(gemv_t_partial_kernel<double>, grid, dim3(256), 0, s, m, n,
                       static_cast<const double*>(J), ldJ, x, rows_per, work);
  else
    hipLaunchKernelGGL(gemv_t_partial_kernel<float>, grid, dim3(256), 0, s, m, n,
                       static_cast<const float*>(J), ldJ, x, rows_per, work);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(gemv_t_reduce_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, S,
                     work, alpha, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int gemv_n_residual(hipStream_t s, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
                    const double* t, const double* r, const double* x, double lam, double* out) {
  DNGD_REQUIRE(ldJ % 4 == 0, "gemv_n: ldJ %% 4 != 0");
  dim3 grid((unsigned)cdiv(m, GN_ROWS));
  if (j_dtype == 0)
    hipLaunchKernelGGL(gemv_n_kernel<double>, grid, dim3(256), 0, s, m, n,
                       static_cast<const double*>(J), ldJ, t, r, x, lam, out);
  else
    hipLaunchKernelGGL(gemv_n_kernel<float>, grid, dim3(256), 0, s, m, n,
                       static_cast<const float*>(J), ldJ, t, r, x, lam, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int sumsq(hipStream_t s, int64_t n, const double* x, double* out, double* work) {
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(SS_BLOCKS), dim3(256), 0, s, n, x, work);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(sumsq_final_kernel, dim3(1), dim3(256), 0, s, work, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int vmax(hipStream_t s, int64_t n, const double* x, double* out, double* work) {
  hipLaunchKernelGGL(vmax_partial_kernel, dim3(SS_BLOCKS), dim3(256), 0, s, n, x, work);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(vmax_final_kernel, dim3(1), dim3(256), 0, s, work, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int dot(hipStream_t s, int64_t n, const double* x, const double* y, double* out, double* work) {
  hipLaunchKernelGGL(dot_partial_kernel, dim3(SS_BLOCKS), dim3(256), 0, s, n, x, y, work);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(sumsq_final_kernel, dim3(1), dim3(256), 0, s, work, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int gather_cols(hipStream_t s, int64_t ell, const double* A, int64_t lda, const int64_t* idx,
                double* out) {
  hipLaunchKernelGGL(gather_cols_kernel, dim3((unsigned)cdiv(ell * ell, 256)), dim3(256), 0, s, ell,
                     A, lda, idx, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int woodbury_finish(hipStream_t s, int64_t n, const double* x, double inv_lam, double* z) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(woodbury_finish_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, x,
                     inv_lam, z);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int xpby(hipStream_t s, int64_t n, const double* x, double beta, double* y) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(xpby_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, x, beta, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int axpy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, a, x, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}
int copy(hipStream_t s, int64_t n, const double* x, double* y) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, x, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}
int fill(hipStream_t s, int64_t n, double v, double* y) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, v, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}
int ga_combine(hipStream_t s, int64_t n, const double* v, const double* a, const double* norms2,
               double eps, double* dtheta, int* flag_out) {
  hipLaunchKernelGGL(ga_combine_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, v, a,
                     norms2, eps, dtheta, flag_out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int transpose_rm(hipStream_t s, int64_t rows, int64_t cols, const void* src, int64_t lds,
                 int j_dtype, void* dst, int64_t ldd) {
  if (rows <= 0 || cols <= 0) return 0;
  DNGD_REQUIRE(lds >= cols && ldd >= rows, "transpose_rm: leading dimension too small");
  const dim3 grid((unsigned)cdiv(cols, 64), (unsigned)cdiv(rows, 64));
  if (j_dtype == 0)
    hipLaunchKernelGGL(transpose_rm_kernel<double>, grid, dim3(256), 0, s, rows, cols,
                       static_cast<const double*>(src), lds, static_cast<double*>(dst), ldd);
  else
    hipLaunchKernelGGL(transpose_rm_kernel<float>, grid, dim3(256), 0, s, rows, cols,
                       static_cast<const float*>(src), lds, static_cast<float*>(dst), ldd);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int rownorm2(hipStream_t s, int64_t rows, int64_t cols, const void* A, int64_t lda, int j_dtype,
             double* out) {
  if (rows <= 0) return 0;
  if (j_dtype == 0)
    hipLaunchKernelGGL(rownorm2_kernel<double>, dim3((unsigned)rows), dim3(256), 0, s, cols,
                       static_cast<const double*>(A), lda, out);
  else
    hipLaunchKernelGGL(rownorm2_kernel<float>, dim3((unsigned)rows), dim3(256), 0, s, cols,
                       static_cast<const float*>(A), lda, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int add_diag(hipStream_t s, int64_t n, double* K, int64_t ldK, double v) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, n, K, ldK, v);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
