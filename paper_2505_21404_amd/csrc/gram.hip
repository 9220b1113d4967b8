// Residual Gramian K = J J^T + lambda I (Definition 3.3; assembled in the dense
// dual solver of Section 4.1), as a lower-triangle SYRK over row-major J.
//
// J is m x ldJ row-major: both operands of K = J J^T are "K-contiguous"
// (the contraction runs along a row of J), so every lane loads contiguous
// 16-byte chunks and no transpose is needed anywhere.
//
// Mixed path (FP32 J): v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
// J is rounded to bf16 while it is staged into LDS (no bf16 copy of J in
// HBM). PASSES == 3 keeps the rounding residual as a second bf16 term,
// J = hi + lo, and accumulates hi hi^T + hi lo^T + lo hi^T (the lo lo^T term
// is below FP32 resolution), so K carries ~16 bits of J instead of 8.
// Plain path (FP64 J): the FP64 MFMA GEMM in split-K partial mode.
//
// Workgroup tile 128 x 128 of K (4 waves, 64 x 64 each = 2 x 2 MFMA 32x32),
// K-step 64 elements. LDS rows are 64 bf16 = 8 chunks of 16 B; chunk c of row
// r is stored at c ^ (r & 7) so the 32 lanes reading 32 rows of one chunk hit
// distinct banks.
//
// Only lower-triangle tiles are launched. Tiles are numbered row-major over
// the lower triangle and the launch index is remapped so that each XCD
// (workgroups go round-robin over the 8 XCDs) receives a contiguous run of
// tiles, which share row panels of J in that XCD's L2.
//
// Split-K partial tiles (FP32 or FP64) are summed in FP64 in split order by
// gram_reduce, which also adds lambda on the diagonal: deterministic.
#include "common.h"

namespace dngd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int GT = 128;   // tile edge
constexpr int GK = 64;    // K step (elements)
constexpr int NXCD = 8;

__device__ inline void tri_decode_g(int64_t t, int64_t& i, int64_t& j) {
  int64_t ii = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}

union Chunk {
  uint4 u;
  bf16x8 h;
};

// Round 8 floats to bf16 (RNE); optionally produce the bf16 residual.
__device__ inline void split8(const float4& a, const float4& b, Chunk& hi, Chunk& lo, bool want_lo) {
  float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)f[e];
    hi.h[e] = h;
    if (want_lo) lo.h[e] = (__bf16)(f[e] - (float)h);
  }
}

template <int PASSES>
__global__ __launch_bounds__(256) void gram_bf16_kernel(int64_t m, int64_t n,
                                                        const float* __restrict__ J, int64_t ldJ,
                                                        float* __restrict__ work,
                                                        int64_t k_per_split, int64_t ntiles,
                                                        int64_t per_xcd) {
  constexpr bool LO = (PASSES == 3);
  __shared__ uint4 Ahi[GT * 8];
  __shared__ uint4 Bhi[GT * 8];
  __shared__ uint4 Alo[LO ? GT * 8 : 1];
  __shared__ uint4 Blo[LO ? GT * 8 : 1];

  const int64_t logical = (int64_t)(blockIdx.x % NXCD) * per_xcd + blockIdx.x / NXCD;
  if (logical >= ntiles) return;
  int64_t ti, tj;
  tri_decode_g(logical, ti, tj);
  const bool diag = (ti == tj);
  const int split = blockIdx.y;
  const int64_t kbeg = (int64_t)split * k_per_split;
  const int64_t kend = min(n, kbeg + k_per_split);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // loader geometry: thread -> row (t >> 1), 32 consecutive k (t & 1)
  const int lrow = t >> 1;
  const int lhalf = t & 1;
  const int64_t arow = ti * GT + lrow, brow = tj * GT + lrow;
  const bool aok = arow < m, bok = brow < m;
  const float* pa = J + (aok ? arow : 0) * ldJ;
  const float* pb = J + (bok ? brow : 0) * ldJ;

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  float4 ra[8], rb[8];
  auto gload = [&](int64_t k0) {
    const int64_t kb = k0 + lhalf * 32;
    const bool full = (kb + 32 <= kend);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t k = kb + 4 * q;
      if (full) {
        ra[q] = aok ? *reinterpret_cast<const float4*>(pa + k) : float4{0, 0, 0, 0};
        if (!diag) rb[q] = bok ? *reinterpret_cast<const float4*>(pb + k) : float4{0, 0, 0, 0};
      } else {
        float xa[4], xb[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool kin = (k + e) < kend;
          xa[e] = (aok && kin) ? pa[k + e] : 0.0f;
          xb[e] = (!diag && bok && kin) ? pb[k + e] : 0.0f;
        }
        ra[q] = float4{xa[0], xa[1], xa[2], xa[3]};
        if (!diag) rb[q] = float4{xb[0], xb[1], xb[2], xb[3]};
      }
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int chunk = lhalf * 4 + c;
      const int slot = lrow * 8 + (chunk ^ (lrow & 7));
      Chunk h, l;
      split8(ra[2 * c], ra[2 * c + 1], h, l, LO);
      Ahi[slot] = h.u;
      if (LO) Alo[slot] = l.u;
      if (!diag) {
        split8(rb[2 * c], rb[2 * c + 1], h, l, LO);
        Bhi[slot] = h.u;
        if (LO) Blo[slot] = l.u;
      }
    }
  };

  const uint4* BH = diag ? Ahi : Bhi;
  const uint4* BL = diag ? Alo : Blo;

  const int64_t nk = (kend > kbeg) ? (kend - kbeg + GK - 1) / GK : 0;
  if (nk > 0) gload(kbeg);
  for (int64_t it = 0; it < nk; ++it) {
    sstore();
    __syncthreads();
    if (it + 1 < nk) gload(kbeg + (it + 1) * GK);
#pragma unroll
    for (int s = 0; s < GK / 16; ++s) {
      const int chunk = s * 2 + (lane >> 5);
      Chunk ah[2], bh[2], al[2], bl[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wm * 64 + i * 32 + (lane & 31);
        ah[i].u = Ahi[r * 8 + (chunk ^ (r & 7))];
        if (LO) al[i].u = Alo[r * 8 + (chunk ^ (r & 7))];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = wn * 64 + j * 32 + (lane & 31);
        bh[j].u = BH[r * 8 + (chunk ^ (r & 7))];
        if (LO) bl[j].u = BL[r * 8 + (chunk ^ (r & 7))];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i].h, bh[j].h, acc[i][j], 0, 0, 0);
          if (LO) {
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i].h, bl[j].h, acc[i][j], 0, 0, 0);
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i].h, bh[j].h, acc[i][j], 0, 0, 0);
          }
        }
    }
    __syncthreads();
  }

  // accumulator v of tile (i, j): row 8 (v/4) + 4 (lane/32) + v%4, col lane%32
  float* out = work + ((int64_t)split * ntiles + logical) * (GT * GT);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wm * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int cl = wn * 64 + j * 32 + (lane & 31);
        out[rl * GT + cl] = acc[i][j][v];
      }
}

template <typename P>
__global__ __launch_bounds__(256) void gram_reduce_kernel(int64_t m, const P* __restrict__ work,
                                                          int splits, int64_t ntiles,
                                                          double lambda, double* __restrict__ K,
                                                          int64_t ldK) {
  int64_t ti, tj;
  tri_decode_g(blockIdx.x, ti, tj);
  const int base = (blockIdx.y * 256 + threadIdx.x) * 4;  // 4 consecutive elements
  const int rl = base / GT, cl0 = base % GT;
  const int64_t row = ti * GT + rl;
  if (row >= m) return;
  double s[4] = {0, 0, 0, 0};
  for (int sp = 0; sp < splits; ++sp) {
    const P* p = work + ((int64_t)sp * ntiles + blockIdx.x) * (GT * GT) + rl * GT + cl0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] += (double)p[e];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t col = tj * GT + cl0 + e;
    if (col < m && col <= row) K[row * ldK + col] = s[e] + (row == col ? lambda : 0.0);
  }
}

int choose_splits(int64_t ntiles, int64_t n) {
  int64_t s = cdiv(1536, ntiles);
  const int64_t smax = std::max<int64_t>(1, n / 2048);
  if (s > smax) s = smax;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  return (int)s;
}

}  // namespace

size_t gram_workspace_bytes(int64_t m, int64_t n, int j_dtype, int passes, int* splits_out) {
  (void)passes;
  const int64_t nt = lower_tiles(m, GT);
  const int s = choose_splits(nt, n);
  if (splits_out) *splits_out = s;
  const size_t esz = (j_dtype == 0) ? sizeof(double) : sizeof(float);
  return (size_t)s * (size_t)nt * GT * GT * esz;
}

int gram_launch(hipStream_t st, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
                int passes, double lambda, double* K, int64_t ldK, void* work,
                size_t work_bytes) {
  int splits = 1;
  const size_t need = gram_workspace_bytes(m, n, j_dtype, passes, &splits);
  DNGD_REQUIRE(work_bytes >= need, "gram: workspace too small (%zu < %zu)", work_bytes, need);
  const int64_t nt = lower_tiles(m, GT);
  const int64_t kps = round_up(cdiv(n, splits), GK);
  if (j_dtype == 0) {
    int rc = gemm_f64(st, GEMM_PARTIAL_LOWER, true, true, m, m, n, 1.0,
                      static_cast<const double*>(J), ldJ, static_cast<const double*>(J), ldJ, 0.0,
                      nullptr, 0, static_cast<double*>(work), splits);
    if (rc) return rc;
    hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3((unsigned)nt, GT * GT / 1024), dim3(256),
                       0, st, m, static_cast<const double*>(work), splits, nt, lambda, K, ldK);
    DNGD_LAUNCH_CHECK();
    return 0;
  }
  DNGD_REQUIRE(ldJ % 4 == 0, "gram: FP32 J needs ldJ %% 4 == 0");
  DNGD_REQUIRE(passes == 1 || passes == 3, "gram: passes must be 1 or 3");
  const int64_t per_xcd = cdiv(nt, NXCD);
  dim3 grid((unsigned)(per_xcd * NXCD), (unsigned)splits);
  if (passes == 3)
    hipLaunchKernelGGL(gram_bf16_kernel<3>, grid, dim3(256), 0, st, m, n,
                       static_cast<const float*>(J), ldJ, static_cast<float*>(work), kps, nt,
                       per_xcd);
  else
    hipLaunchKernelGGL(gram_bf16_kernel<1>, grid, dim3(256), 0, st, m, n,
                       static_cast<const float*>(J), ldJ, static_cast<float*>(work), kps, nt,
                       per_xcd);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(gram_reduce_kernel<float>, dim3((unsigned)nt, GT * GT / 1024), dim3(256), 0,
                     st, m, static_cast<const float*>(work), splits, nt, lambda, K, ldK);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
