// FP32 GEMMs on the matrix cores for FP64 data: the per-layer products of the
// second-order tangent pass (f_vv, Section 3.2) inside the mixed step, where
// FP32 products are accurate enough for the geodesic correction.
//
//   C (M x N, FP64) = sum over segments s of alpha_s A_s (M x K_s) . B_s (N x K_s)^T
//                     + beta C
//
// Every operand is FP64, row-major with the contraction along a row; it is
// rounded to FP32 (B_s after scaling by alpha_s) as it is staged into LDS, and
// the products accumulate in FP32 (v_mfma_f32_32x32x2_f32). Two segments let
// Z = a0 V^T + a1 W^T run as one product with one store.
//
// Tile: 128 x 128 per workgroup of 4 waves (2 x 2), each wave 64 x 64 = 2 x 2
// accumulators. K advances 32 per step: each thread fetches 16 elements of
// each operand a step ahead into registers (as FP64, so the current step's
// products run while they are in flight) and stores them, converted, into a
// double-buffered LDS stage whose rows are padded to 33 floats (the 32 rows a
// fragment read touches fall in distinct banks). Rows beyond M or N read the
// last row and are not stored; K beyond K_s reads zeros. (16-element steps, or
// converting as the loads return, were 1-5% slower; 128 x 64 tiles, twice the
// workgroups, 15% slower.)
#include "common.h"

namespace dngd {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 128;          // tile edge
constexpr int KS = 32;           // K per step
constexpr int RS = KS + 1;       // LDS row stride in floats
constexpr int NTH = 256;
constexpr int PER = TM * KS / NTH;  // elements of one operand per thread and step

struct Segs32 {
  const double* A[2];
  const double* B[2];
  int64_t lda[2], ldb[2], K[2];
  double alpha[2];
  int64_t steps0;  // K steps of segment 0
  int64_t steps;   // K steps in total
};

__global__ __launch_bounds__(256) void gemm_f32_nt_kernel(int64_t M, int64_t N, Segs32 sg,
                                                          double beta, double* __restrict__ C,
                                                          int64_t ldc, int64_t tiles_n) {
  __shared__ float la[2][TM * RS];
  __shared__ float lb[2][TM * RS];
  const int64_t ti = blockIdx.x / tiles_n, tj = blockIdx.x % tiles_n;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // element q of a step: row (q NTH + t) / KS, column (q NTH + t) % KS. The
  // loads land in registers as FP64 and are converted only when stored, so
  // the products of the current step run while they are in flight.
  double ra[PER], rb[PER];
  int64_t kend = 0;   // elements of the loaded step's K range in its segment
  double al = 1.0;    // its segment's alpha
  auto gload = [&](int64_t step) {
    const int s = step < sg.steps0 ? 0 : 1;
    const int64_t k0 = (step - (s ? sg.steps0 : 0)) * KS;
    const double* A = sg.A[s];
    const double* B = sg.B[s];
    const int64_t lda = sg.lda[s], ldb = sg.ldb[s], K = sg.K[s];
    kend = K - k0;
    al = sg.alpha[s];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = q * NTH + t, r = e / KS, c = e % KS;
      const int64_t kc = min(k0 + c, K - 1);
      ra[q] = A[min(ti * TM + r, M - 1) * lda + kc];
      rb[q] = B[min(tj * TM + r, N - 1) * ldb + kc];
    }
  };
  auto lstore = [&](int st) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = q * NTH + t, r = e / KS, c = e % KS;
      const bool in = c < kend;
      la[st][r * RS + c] = in ? (float)ra[q] : 0.0f;
      lb[st][r * RS + c] = in ? (float)(al * rb[q]) : 0.0f;
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  // v_mfma_f32_32x32x2_f32: lane l gives A[row l % 32][k l / 32] and
  // B[col l % 32][k l / 32]
  auto compute = [&](int st) {
#pragma unroll
    for (int kk = 0; kk < KS; kk += 2) {
      const int kl = kk + (lane >> 5);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = la[st][(wm * 64 + i * 32 + (lane & 31)) * RS + kl];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = lb[st][(wn * 64 + j * 32 + (lane & 31)) * RS + kl];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  const int64_t ns = sg.steps;
  if (ns > 0) {
    gload(0);
    lstore(0);
    __syncthreads();
    for (int64_t it = 0; it < ns; ++it) {
      const int st = (int)(it & 1);
      if (it + 1 < ns) gload(it + 1);
      compute(st);
      if (it + 1 < ns) lstore(st ^ 1);
      __syncthreads();
    }
  }
  // accumulator v of block (i, j): row 8 (v / 4) + 4 (lane / 32) + v % 4, col lane % 32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = ti * TM + wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int64_t col = tj * TM + wn * 64 + j * 32 + (lane & 31);
        if (row < M && col < N) {
          double* c = C + row * ldc + col;
          const double x = (double)acc[i][j][v];
          *c = (beta == 0.0) ? x : x + beta * *c;
        }
      }
}

}  // namespace

int gemm_f32_nt(hipStream_t s, int64_t M, int64_t N, int nseg, const double* const* A,
                const int64_t* lda, const double* const* B, const int64_t* ldb, const int64_t* K,
                const double* alpha, double beta, double* C, int64_t ldc) {
  DNGD_REQUIRE(nseg == 1 || nseg == 2, "gemm_f32_nt: one or two segments");
  if (M <= 0 || N <= 0) return 0;
  Segs32 sg{};
  for (int q = 0; q < nseg; ++q) {
    DNGD_REQUIRE(A[q] && B[q] && K[q] >= 1 && lda[q] >= K[q] && ldb[q] >= K[q],
                 "gemm_f32_nt: bad segment %d", q);
    sg.A[q] = A[q];
    sg.B[q] = B[q];
    sg.lda[q] = lda[q];
    sg.ldb[q] = ldb[q];
    sg.K[q] = K[q];
    sg.alpha[q] = alpha[q];
  }
  sg.steps0 = cdiv(K[0], KS);
  sg.steps = sg.steps0 + (nseg == 2 ? cdiv(K[1], KS) : 0);
  const int64_t tiles_n = cdiv(N, TM);
  hipLaunchKernelGGL(gemm_f32_nt_kernel, dim3((unsigned)(cdiv(M, TM) * tiles_n)), dim3(NTH), 0, s,
                     M, N, sg, beta, C, ldc, tiles_n);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
