// bf16 GEMMs on the matrix cores with FP32 accumulation: the per-layer
// products of the low-precision kernel-vector product (Definition 3.6 with
// bf16 operands) and of the landmark columns of the Nystrom construction
// (Section 3.3).
//
//   C (M x N) = sum over segments s of A_s (M x K_s) . B_s (N x K_s)^T
//
// Every operand is bf16, row-major with the contraction along a row
// ("K-contiguous"): the products that contract over jet rows (the weight
// gradients) take operands transposed once when they are produced, so a
// single tile loader serves every product. K_s % 32 == 0, leading dimensions
// % 8 == 0 and 16-byte aligned bases (callers zero-pad their bf16 copies).
// Two segments let Z1 = H V^T + A1 W^T run as one product with one store.
//
// Output: FP32 C (row-major, ldc), or split-K partial tiles that
// gemm_bf16_reduce sums in FP64 in split order (deterministic) into an FP64
// matrix, with one column optionally routed to a separate vector (the bias
// gradient rides along as the last column of a weight gradient).
//
// Tile: 256 x 256 per workgroup of 8 waves (2 x 4), each wave 128 x 64 =
// 4 x 2 accumulators of v_mfma_f32_32x32x16_bf16. K advances 32 per step;
// each lane moves two 16-byte chunks of each operand per step, prefetched two
// steps ahead in registers and stored into a double-buffered LDS stage
// (chunk c of row r at c ^ ((r >> 2) & 3): the 16 rows a fragment read
// touches per cycle fall in distinct bank groups). Rows beyond M or N read
// the last row (their results are not stored). Launch index -> tile is
// remapped so that each XCD receives a contiguous run of tiles (tiles of one
// A row panel side by side share it in that XCD's L2).
#include "common.h"

namespace dngd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte chunk

constexpr int BT = 256;    // tile edge
constexpr int NTH = 512;   // threads per workgroup
constexpr int SK = 32;     // K per step (bf16 elements)
constexpr int ROWB = SK * 2;  // bytes per plane row
constexpr int NXCD = 8;


__device__ inline int poff(int r, int c) { return r * ROWB + ((c ^ ((r >> 2) & 3)) << 4); }

struct Segs {
  const uint16_t* A[2];
  const uint16_t* B[2];
  int64_t lda[2], ldb[2];
  int64_t steps0;  // K steps of segment 0
  int64_t steps;   // K steps in total
};

template <bool PARTIAL>
__global__ __launch_bounds__(512) void gemm_bf16_nt_kernel(int64_t M, int64_t N, Segs sg,
                                                           float* __restrict__ out, int64_t ldc,
                                                           int64_t tiles_n, int64_t ntiles,
                                                           int64_t per_xcd, int splits,
                                                           int64_t steps_per_split) {
  __shared__ __attribute__((aligned(16))) char lds[2][2][BT * ROWB];  // [stage][A, B]

  const int64_t lin = blockIdx.x;
  const int64_t slot = (lin % NXCD) * per_xcd + lin / NXCD;
  if (slot >= ntiles * (int64_t)splits) return;  // padding slots
  const int64_t split = slot / ntiles;
  const int64_t tile = slot % ntiles;
  const int64_t ti = tile / tiles_n, tj = tile % tiles_n;
  const int64_t s_beg = split * steps_per_split;
  const int64_t s_end = min(sg.steps, s_beg + steps_per_split);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;

  // load geometry: chunk lch (8 bf16) of rows lrow[0], lrow[1] of each panel
  const int lch = t & 3;
  int lrow[2];
  int64_t ra[2], rb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    lrow[q] = (t >> 2) + 128 * q;
    ra[q] = min(ti * BT + lrow[q], M - 1);
    rb[q] = min(tj * BT + lrow[q], N - 1);
  }
  // two register sets (distinct arrays: an array indexed by the set would be
  // kept in scratch memory)
  u32x4 ga0[2], gb0[2], ga1[2], gb1[2];
  auto gload = [&](u32x4 (&ga)[2], u32x4 (&gb)[2], int64_t k) __attribute__((always_inline)) {
    // segment by selects, not by indexing (an indexed kernel argument would
    // be copied to scratch memory)
    const bool s1 = k >= sg.steps0;
    const uint16_t* A = s1 ? sg.A[1] : sg.A[0];
    const uint16_t* B = s1 ? sg.B[1] : sg.B[0];
    const int64_t lda = s1 ? sg.lda[1] : sg.lda[0];
    const int64_t ldb = s1 ? sg.ldb[1] : sg.ldb[0];
    const int64_t kk = (k - (s1 ? sg.steps0 : 0)) * SK + 8 * lch;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ga[q] = *reinterpret_cast<const u32x4*>(A + ra[q] * lda + kk);
      gb[q] = *reinterpret_cast<const u32x4*>(B + rb[q] * ldb + kk);
    }
  };
  auto stage_store = [&](const u32x4 (&ga)[2], const u32x4 (&gb)[2], int st)
                         __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<u32x4*>(lds[st][0] + poff(lrow[q], lch)) = ga[q];
      *reinterpret_cast<u32x4*>(lds[st][1] + poff(lrow[q], lch)) = gb[q];
    }
  };

  f32x16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  auto frag = [&](const char* plane, int r, int sl) __attribute__((always_inline)) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(plane + poff(r, 2 * sl + (lane >> 5)));
  };
  auto compute = [&](int st) __attribute__((always_inline)) {
    const char* Ap = lds[st][0];
    const char* Bp = lds[st][1];
#pragma unroll
    for (int sl = 0; sl < SK / 16; ++sl) {
      bf16x8 a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = frag(Ap, wm * 128 + i * 32 + (lane & 31), sl);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = frag(Bp, wn * 64 + j * 32 + (lane & 31), sl);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };

  const int64_t nk = s_end > s_beg ? s_end - s_beg : 0;
  if (nk > 0) {
    // invariant at the top of each half-iteration: stage st holds step it,
    // register set st ^ 1 holds (or is loading) step it + 1
    gload(ga0, gb0, s_beg);
    if (nk > 1) gload(ga1, gb1, s_beg + 1);
    stage_store(ga0, gb0, 0);
    __syncthreads();
    int64_t it = 0;
    for (; it + 3 < nk; it += 2) {
      gload(ga0, gb0, s_beg + it + 2);
      __builtin_amdgcn_sched_barrier(0);
      compute(0);
      stage_store(ga1, gb1, 1);
      __syncthreads();
      gload(ga1, gb1, s_beg + it + 3);
      __builtin_amdgcn_sched_barrier(0);
      compute(1);
      stage_store(ga0, gb0, 0);
      __syncthreads();
    }
    // the last one to three steps: stage st holds step it, register set 1
    // holds step it + 1
    int st = 0;
    for (; it < nk; ++it) {
      compute(st);
      if (it + 1 < nk) stage_store(ga1, gb1, st ^ 1);
      __syncthreads();
      if (it + 2 < nk) gload(ga1, gb1, s_beg + it + 2);
      st ^= 1;
    }
  }

  // accumulator v of block (i, j): row 8 (v/4) + 4 (lane/32) + v%4, col lane%32
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wm * 128 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int cl = wn * 64 + j * 32 + (lane & 31);
        if (PARTIAL) {
          out[(split * ntiles + tile) * (int64_t)(BT * BT) + rl * BT + cl] = acc[i][j][v];
        } else {
          const int64_t row = ti * BT + rl, col = tj * BT + cl;
          if (row < M && col < N) out[row * ldc + col] = acc[i][j][v];
        }
      }
}

// C[row][col] (col != bias_col) or bias[row] (col == bias_col) = the FP64 sum
// of the split partials in split order. One thread per 4 consecutive columns.
__global__ __launch_bounds__(256) void gemm_bf16_reduce_kernel(int64_t M, int64_t N,
                                                               const float* __restrict__ work,
                                                               int splits, int64_t tiles_n,
                                                               int64_t ntiles,
                                                               double* __restrict__ C,
                                                               int64_t ldc, int64_t bias_col,
                                                               double* __restrict__ bias) {
  const int64_t tile = blockIdx.x;
  const int64_t ti = tile / tiles_n, tj = tile % tiles_n;
  const int base = (blockIdx.y * 256 + threadIdx.x) * 4;
  const int rl = base / BT, cl0 = base % BT;
  const int64_t row = ti * BT + rl;
  if (row >= M) return;
  double s[4] = {0, 0, 0, 0};
  for (int sp = 0; sp < splits; ++sp) {
    const float4 p = *reinterpret_cast<const float4*>(
        work + ((int64_t)sp * ntiles + tile) * (BT * BT) + rl * BT + cl0);
    s[0] += (double)p.x;
    s[1] += (double)p.y;
    s[2] += (double)p.z;
    s[3] += (double)p.w;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t col = tj * BT + cl0 + e;
    if (col >= N) continue;
    if (col == bias_col) bias[row] = s[e];
    else C[row * ldc + col] = s[e];
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int check_segs(int64_t M, int64_t N, const uint16_t* A0, int64_t lda0, const uint16_t* B0,
               int64_t ldb0, int64_t K0, const uint16_t* A1, int64_t lda1, const uint16_t* B1,
               int64_t ldb1, int64_t K1, Segs& sg) {
  DNGD_REQUIRE(M >= 1 && N >= 1 && K0 >= 0 && K1 >= 0, "gemm_bf16: bad sizes");
  DNGD_REQUIRE(K0 % SK == 0 && K1 % SK == 0, "gemm_bf16: K must be a multiple of %d", SK);
  DNGD_REQUIRE(lda0 % 8 == 0 && ldb0 % 8 == 0 && lda0 >= K0 && ldb0 >= K0 && aligned16(A0) &&
                   aligned16(B0),
               "gemm_bf16: segment 0 needs ld %% 8 == 0, ld >= K and 16-byte aligned bases");
  if (K1 > 0)
    DNGD_REQUIRE(A1 && B1 && lda1 % 8 == 0 && ldb1 % 8 == 0 && lda1 >= K1 && ldb1 >= K1 &&
                     aligned16(A1) && aligned16(B1),
                 "gemm_bf16: segment 1 needs ld %% 8 == 0, ld >= K and 16-byte aligned bases");
  sg.A[0] = A0;
  sg.B[0] = B0;
  sg.lda[0] = lda0;
  sg.ldb[0] = ldb0;
  sg.A[1] = K1 > 0 ? A1 : A0;
  sg.B[1] = K1 > 0 ? B1 : B0;
  sg.lda[1] = K1 > 0 ? lda1 : lda0;
  sg.ldb[1] = K1 > 0 ? ldb1 : ldb0;
  sg.steps0 = K0 / SK;
  sg.steps = (K0 + K1) / SK;
  return 0;
}

}  // namespace

int gemm_bf16_nt(hipStream_t s, int64_t M, int64_t N, const uint16_t* A0, int64_t lda0,
                 const uint16_t* B0, int64_t ldb0, int64_t K0, const uint16_t* A1, int64_t lda1,
                 const uint16_t* B1, int64_t ldb1, int64_t K1, float* C, int64_t ldc) {
  Segs sg;
  int rc = check_segs(M, N, A0, lda0, B0, ldb0, K0, A1, lda1, B1, ldb1, K1, sg);
  if (rc) return rc;
  DNGD_REQUIRE(ldc >= N, "gemm_bf16: ldc < N");
  const int64_t tiles_n = cdiv(N, BT), ntiles = cdiv(M, BT) * tiles_n;
  const int64_t per_xcd = cdiv(ntiles, NXCD);
  hipLaunchKernelGGL(gemm_bf16_nt_kernel<false>, dim3((unsigned)(per_xcd * NXCD)), dim3(NTH), 0,
                     s, M, N, sg, C, ldc, tiles_n, ntiles, per_xcd, 1, sg.steps);
  DNGD_LAUNCH_CHECK();
  return 0;
}

size_t gemm_bf16_split_work_bytes(int64_t M, int64_t N, int64_t K) {
  const int64_t ntiles = cdiv(M, BT) * cdiv(N, BT);
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>(cdiv(1024, ntiles), K / (SK * 64)));
  return (size_t)splits * ntiles * BT * BT * sizeof(float);
}

int gemm_bf16_nt_split(hipStream_t s, int64_t M, int64_t N, const uint16_t* A, int64_t lda,
                       const uint16_t* B, int64_t ldb, int64_t K, double* C, int64_t ldc,
                       int64_t bias_col, double* bias, float* work, size_t work_bytes) {
  Segs sg;
  int rc = check_segs(M, N, A, lda, B, ldb, K, nullptr, 0, nullptr, 0, 0, sg);
  if (rc) return rc;
  DNGD_REQUIRE(bias_col < 0 || bias, "gemm_bf16: bias column without a bias vector");
  const int64_t tiles_n = cdiv(N, BT), ntiles = cdiv(M, BT) * tiles_n;
  // enough (split, tile) workgroups to fill the chip, each at least 64 steps
  const int64_t splits =
      std::max<int64_t>(1, std::min<int64_t>(cdiv(1024, ntiles), K / (SK * 64)));
  DNGD_REQUIRE(work_bytes >= (size_t)splits * ntiles * BT * BT * sizeof(float),
               "gemm_bf16: split workspace too small");
  const int64_t sps = cdiv(sg.steps, splits);
  const int64_t per_xcd = cdiv(ntiles * splits, NXCD);
  hipLaunchKernelGGL(gemm_bf16_nt_kernel<true>, dim3((unsigned)(per_xcd * NXCD)), dim3(NTH), 0, s,
                     M, N, sg, work, (int64_t)0, tiles_n, ntiles, per_xcd, (int)splits, sps);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(gemm_bf16_reduce_kernel, dim3((unsigned)ntiles, BT * BT / 1024), dim3(256), 0,
                     s, M, N, work, (int)splits, tiles_n, ntiles, C, ldc, bias_col, bias);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
