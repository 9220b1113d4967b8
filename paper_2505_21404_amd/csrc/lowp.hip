// Element-wise and layout kernels of the low-precision kernel-vector product
// (Definition 3.6 with bf16 GEMM operands and FP32 accumulation): bf16 and
// FP32 copies of the step's activations, transposes for the products that
// contract over jet rows, and the jet rules of the tanh layer (adjoint and
// first-order tangent) evaluated in FP32 with bf16 outputs.
//
// Every bf16 matrix is row-major with its row length rounded up to a
// multiple of 32 (the GEMM's K step) and the padding columns written as zero,
// so that padded contractions add nothing. Matrices transposed for the
// weight gradients have one column per jet row, rounded up the same way, and
// may carry one extra row marking the value rows (1 on a point's value row,
// 0 elsewhere): the bias gradient then comes out of the same product.
#include "common.h"

namespace dngd {

namespace {

__device__ inline uint16_t to_bf16(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
}
__device__ inline float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline bool value_row(const RowMap& rm, int64_t r) {
  return r >= rm.R_int || (r % rm.C_int) == 0;
}

__device__ inline void point_rows_lp(const RowMap& rm, int64_t p, int64_t& base, int& C) {
  if (p < rm.n_int) {
    base = p * rm.C_int;
    C = rm.C_int;
  } else {
    base = rm.R_int + (p - rm.n_int);
    C = 1;
  }
}

__global__ void to_f32_kernel(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// dst[r][c] = bf16(src[r][c]) for c < cols, 0 for cols <= c < ldd
__global__ void to_bf16_pad_kernel(int64_t rows, int64_t cols, const double* __restrict__ src,
                                   int64_t lds, uint16_t* __restrict__ dst, int64_t ldd) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * ldd) return;
  const int64_t r = i / ldd, c = i % ldd;
  dst[i] = c < cols ? to_bf16((float)src[r * lds + c]) : (uint16_t)0;
}

template <typename T>
__device__ inline uint16_t as_bf16(T x);
template <>
__device__ inline uint16_t as_bf16<double>(double x) {
  return to_bf16((float)x);
}
template <>
__device__ inline uint16_t as_bf16<uint16_t>(uint16_t x) {
  return x;
}

// dst[c][r] = bf16(src[r][c]) for c < cols, r < rows; 0 for rows <= r < rpad;
// with `indicator`, row `cols` of dst marks the value rows. 64 x 64 tiles
// through LDS; grid (cdiv(rpad, 64), cdiv(cols + indicator, 64)).
template <typename T>
__global__ __launch_bounds__(256) void transpose_bf16_kernel(RowMap rm, int64_t rows, int64_t cols,
                                                             const T* __restrict__ src,
                                                             int64_t lds, uint16_t* __restrict__ dst,
                                                             int64_t ldd, int64_t rpad,
                                                             int indicator) {
  __shared__ uint16_t tile[64][66];
  const int64_t r0 = (int64_t)blockIdx.x * 64, c0 = (int64_t)blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int i = ty; i < 64; i += 4) {
    const int64_t r = r0 + i, c = c0 + tx;
    uint16_t v = 0;
    if (r < rows) {
      if (c < cols) v = as_bf16<T>(src[r * lds + c]);
      else if (indicator && c == cols) v = value_row(rm, r) ? (uint16_t)0x3f80 : (uint16_t)0;
    }
    tile[i][tx] = v;
  }
  __syncthreads();
  const int64_t ncols = cols + (indicator ? 1 : 0);
  for (int i = ty; i < 64; i += 4) {
    const int64_t c = c0 + i, r = r0 + tx;
    if (c < ncols && r < rpad) dst[c * ldd + r] = tile[tx][i];
  }
}

// seedT[r] = bf16(seed[r]) (r < R), 0 up to rpad
__global__ void seed_row_kernel(int64_t R, int64_t rpad, const double* __restrict__ seed,
                                uint16_t* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r < rpad) out[r] = r < R ? to_bf16((float)seed[r]) : (uint16_t)0;
}

struct TanhF {
  float s1, s2, s3;
  __device__ inline explicit TanhF(float z) {
    const float s0 = tanhf(z);
    s1 = 1.0f - s0 * s0;
    s2 = -2.0f * s0 * s1;
    s3 = s1 * (6.0f * s0 * s0 - 2.0f);
  }
};

// Adjoint of the jet activation (FP32): Zb from Ab and the pre-activation
// jets Zf; Ab is either an FP32 matrix (ld w) or, for the last hidden layer,
// seed[row] * wL[o] (the output layer's weights). Threads cover ldz columns:
// columns w .. ldz-1 are written as zero.
__global__ __launch_bounds__(256) void act_adjoint_lp_kernel(RowMap rm, int w, int64_t ldz,
                                                             const float* __restrict__ Zf,
                                                             const float* __restrict__ Ab,
                                                             const double* __restrict__ seed,
                                                             const double* __restrict__ wL,
                                                             uint16_t* __restrict__ Zb) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= npts * ldz) return;
  const int64_t p = idx / ldz;
  const int o = (int)(idx % ldz);
  int64_t base;
  int C;
  point_rows_lp(rm, p, base, C);
  uint16_t* zb = Zb + base * ldz + o;
  if (o >= w) {
    for (int c = 0; c < C; ++c) zb[(int64_t)c * ldz] = 0;
    return;
  }
  const float* z = Zf + base * w + o;
  auto ab = [&](int c) -> float {
    return Ab ? Ab[(base + c) * w + o] : (float)(seed[base + c] * wL[o]);
  };
  const TanhF s(z[0]);
  if (C == 1) {
    zb[0] = to_bf16(ab(0) * s.s1);
    return;
  }
  const int d = rm.d_in;
  const float abl = ab(1 + d);
  const float zl = z[(int64_t)(1 + d) * w];
  float gg = 0.0f, ag = 0.0f;
  for (int k = 0; k < d; ++k) {
    const float g = z[(int64_t)(1 + k) * w];
    const float agk = ab(1 + k);
    if (k < rm.nlap) gg += g * g;
    ag += agk * g;
    zb[(int64_t)(1 + k) * ldz] = to_bf16(s.s1 * agk + ((k < rm.nlap) ? 2.0f * s.s2 * abl * g : 0.0f));
  }
  zb[0] = to_bf16(ab(0) * s.s1 + s.s2 * ag + abl * (s.s2 * zl + s.s3 * gg));
  zb[(int64_t)(1 + d) * ldz] = to_bf16(s.s1 * abl);
}

// First-order tangent of the jet activation (FP32): A1 = jet(tanh'(z0)) *
// (z1 + b1 on the value channel), written as bf16 with ld lda (columns w ..
// lda-1 zero). For a boundary or initial row only the value channel exists.
__global__ __launch_bounds__(256) void tangent_act_lp_kernel(RowMap rm, int w, int64_t lda,
                                                             const double* __restrict__ b1,
                                                             const float* __restrict__ Zf,
                                                             const float* __restrict__ Z1,
                                                             uint16_t* __restrict__ A1) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= npts * lda) return;
  const int64_t p = idx / lda;
  const int o = (int)(idx % lda);
  int64_t base;
  int C;
  point_rows_lp(rm, p, base, C);
  uint16_t* a = A1 + base * lda + o;
  if (o >= w) {
    for (int c = 0; c < C; ++c) a[(int64_t)c * lda] = 0;
    return;
  }
  const float* z0 = Zf + base * w + o;
  const float* z1 = Z1 + base * w + o;
  const TanhF s(z0[0]);
  const float z1v = z1[0] + (b1 ? (float)b1[o] : 0.0f);
  if (C == 1) {
    a[0] = to_bf16(s.s1 * z1v);
    return;
  }
  // P = jet of tanh'(z0): value s1, gradient s2 g0, Laplacian s2 l0 + s3 |g0|^2
  const int d = rm.d_in;
  float gg = 0.0f, cross = 0.0f;
  for (int k = 0; k < d; ++k) {
    const float g0 = z0[(int64_t)(1 + k) * w];
    const float g1 = z1[(int64_t)(1 + k) * w];
    if (k < rm.nlap) {
      gg += g0 * g0;
      cross += (s.s2 * g0) * g1;
    }
    // (P z1) gradient: P.v z1.g + z1.v P.g
    a[(int64_t)(1 + k) * lda] = to_bf16(s.s1 * g1 + z1v * s.s2 * g0);
  }
  const float l0 = z0[(int64_t)(1 + d) * w];
  const float l1 = z1[(int64_t)(1 + d) * w];
  const float Pl = s.s2 * l0 + s.s3 * gg;
  a[0] = to_bf16(s.s1 * z1v);
  a[(int64_t)(1 + d) * lda] = to_bf16(s.s1 * l1 + z1v * Pl + 2.0f * cross);
}

// out[r] = X[r] . wx + Y[r] . wy over the first w columns (X, Y bf16 with
// row stride ld, a multiple of 8; Y may be null), FP64 sums. One wave per row.
__global__ __launch_bounds__(256) void rowdot_lp_kernel(int64_t R, int w, int64_t ld,
                                                        const uint16_t* __restrict__ X,
                                                        const double* __restrict__ wx,
                                                        const uint16_t* __restrict__ Y,
                                                        const double* __restrict__ wy,
                                                        double* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= R) return;
  double s = 0.0;
  for (int k0 = 8 * lane; k0 < w; k0 += 512) {
    const uint4 xv = *reinterpret_cast<const uint4*>(X + row * ld + k0);
    const uint32_t xs[4] = {xv.x, xv.y, xv.z, xv.w};
    uint32_t ys[4] = {0, 0, 0, 0};
    if (Y) {
      const uint4 yv = *reinterpret_cast<const uint4*>(Y + row * ld + k0);
      ys[0] = yv.x;
      ys[1] = yv.y;
      ys[2] = yv.z;
      ys[3] = yv.w;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + e;
      if (k < w) {
        const uint16_t xh = (uint16_t)(xs[e >> 1] >> (16 * (e & 1)));
        s += (double)from_bf16(xh) * wx[k];
        if (Y) {
          const uint16_t yh = (uint16_t)(ys[e >> 1] >> (16 * (e & 1)));
          s += (double)from_bf16(yh) * wy[k];
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) out[row] = s;
}

inline unsigned blocks_of(int64_t n, int bs = 256) { return (unsigned)cdiv(n, bs); }

}  // namespace

int lp_to_f32(hipStream_t s, int64_t n, const double* x, float* y) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(to_f32_kernel, dim3(blocks_of(n)), dim3(256), 0, s, n, x, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int lp_to_bf16_pad(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                   uint16_t* dst, int64_t ldd) {
  if (rows * ldd <= 0) return 0;
  hipLaunchKernelGGL(to_bf16_pad_kernel, dim3(blocks_of(rows * ldd)), dim3(256), 0, s, rows, cols,
                     src, lds, dst, ldd);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int lp_transpose(hipStream_t s, const RowMap& rm, int64_t rows, int64_t cols, const void* src,
                 int src_bf16, int64_t lds, uint16_t* dst, int64_t ldd, int64_t rpad,
                 int indicator) {
  DNGD_REQUIRE(rpad >= rows && ldd >= rpad, "lp_transpose: bad padding");
  const dim3 grid((unsigned)cdiv(rpad, 64), (unsigned)cdiv(cols + (indicator ? 1 : 0), 64));
  if (src_bf16)
    hipLaunchKernelGGL(transpose_bf16_kernel<uint16_t>, grid, dim3(256), 0, s, rm, rows, cols,
                       static_cast<const uint16_t*>(src), lds, dst, ldd, rpad, indicator);
  else
    hipLaunchKernelGGL(transpose_bf16_kernel<double>, grid, dim3(256), 0, s, rm, rows, cols,
                       static_cast<const double*>(src), lds, dst, ldd, rpad, indicator);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int lp_seed_row(hipStream_t s, int64_t R, int64_t rpad, const double* seed, uint16_t* out) {
  hipLaunchKernelGGL(seed_row_kernel, dim3(blocks_of(rpad)), dim3(256), 0, s, R, rpad, seed, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int lp_act_adjoint(hipStream_t s, const RowMap& rm, int w, int64_t ldz, const float* Zf,
                   const float* Ab, const double* seed, const double* wL, uint16_t* Zb) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  DNGD_REQUIRE(Ab || (seed && wL), "lp_act_adjoint: no adjoint source");
  hipLaunchKernelGGL(act_adjoint_lp_kernel, dim3(blocks_of(npts * ldz)), dim3(256), 0, s, rm, w,
                     ldz, Zf, Ab, seed, wL, Zb);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int lp_tangent_act(hipStream_t s, const RowMap& rm, int w, int64_t lda, const double* b1,
                   const float* Zf, const float* Z1, uint16_t* A1) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  hipLaunchKernelGGL(tangent_act_lp_kernel, dim3(blocks_of(npts * lda)), dim3(256), 0, s, rm, w,
                     lda, b1, Zf, Z1, A1);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int lp_rowdot(hipStream_t s, int64_t R, int w, int64_t ld, const uint16_t* X, const double* wx,
              const uint16_t* Y, const double* wy, double* out) {
  DNGD_REQUIRE(ld % 8 == 0 && ld >= w, "lp_rowdot: ld must be a multiple of 8 and >= w");
  hipLaunchKernelGGL(rowdot_lp_kernel, dim3(blocks_of(R, 4)), dim3(256), 0, s, R, w, ld, X, wx, Y,
                     wy, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
