// Residual Gramian K = J J^T + lambda I (Definition 3.3; assembled in the dense
// dual solver of Section 4.1), as a lower-triangle SYRK over row-major J.
//
// J is m x ldJ row-major: both operands of K = J J^T are "K-contiguous"
// (the contraction runs along a row of J), so every lane loads contiguous
// 16-byte chunks and no transpose is needed anywhere.
//
// Mixed path (FP32 J): v_mfma_f32_32x32x16_bf16 with FP32 accumulation. J is
// rounded to bf16 (RNE) as it is staged into LDS (no bf16 copy of J in HBM). PASSES == 3 keeps the rounding residual as a second bf16 term,
// J ~ hi + lo, and accumulates hi hi^T + hi lo^T + lo hi^T, so K carries ~16
// bits of J instead of 8. Dropping lo lo^T makes that K indefinite by up to
// ||lo lo^T|| (~2^-16 max_i ||J_i||^2), which matters only when the damping is
// that small; PASSES == 4 adds lo lo^T, so K = (hi + lo)(hi + lo)^T is
// positive semidefinite up to the FP32 accumulation error.
// Plain path (FP64 J): the FP64 MFMA GEMM in split-K partial mode. FP32 J
// with passes == kGramF64 takes the same FP64 path, widening J on load (the
// products of FP32 values are exact in FP64): the accurate fallback of the
// mixed path when bf16 products or FP32 accumulation are too coarse for the
// damping.
//
// Only lower-triangle tiles are launched. Tiles are numbered row-major over
// the lower triangle and the launch index is remapped so that each XCD
// (workgroups go round-robin over the 8 XCDs) receives a contiguous run of
// tiles of one split, which share row panels of J in that XCD's L2.
//
// Split-K partial tiles (FP32 or FP64) are summed in FP64 in split order by
// gram_reduce, which also adds lambda on the diagonal: deterministic. The
// FP32 accumulation error of a partial grows with the number of terms it
// holds while the FP64 sum of S partials does not, so the bf16 path uses
// many short splits (~4096 terms each), run in batches of at most 64 splits
// whose sums are added into K in order.
#include "common.h"

namespace dngd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int GT = 128;   // tile edge of the FP64 path
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

// 256 x 256 tile of K per workgroup: 8 waves in a 2 x 4 grid (two per SIMD,
// so one wave's conversion work runs under the other's MFMAs), each a
// 128 x 64 block = 4 x 2 MFMA 32x32 accumulators. K advances SK elements per
// step (SK = 16: one MFMA K-slice; SK = 32: two). The FP32 slabs of both row
// panels are loaded into registers ahead of use (each lane 32 B = 8 floats of
// a row), split once into bf16 hi (and lo) planes and stored in LDS (one
// 16-byte store per plane), double-buffered, so every element is converted
// once per workgroup and the MFMA fragments are read as ready bf16 (one
// ds_read_b128 per operand). The main loop has no branches: B is loaded even
// on diagonal tiles, and the last, partial step of the K range reads a
// zero-padded copy of the last columns.
//   SK = 16 prefetches two steps ahead (two register sets): each step converts
//           data that arrived a step earlier;
//   SK = 32 prefetches one step ahead (the registers of a second set would
//           not fit) but touches each row of J half as often per byte, which
//           wins when rows are far apart (a row per 2 MB page or more: the
//           address translations, not the bytes, then bound the loads).
// Scheduling hints interleave the conversion and its LDS stores with the
// MFMAs. LDS plane rows are SK bf16 = SK/8 chunks of 16 B; chunk c of row r
// sits at c ^ swizzle(r), which makes the 16 rows a fragment read touches per
// cycle land in 16 distinct 16-byte bank groups (64 banks).
constexpr int BT = 256;   // tile edge
constexpr int NTH = 512;  // threads per workgroup
constexpr int SKMAX = 32;  // widest step; K-split lengths are multiples of it
constexpr int JTS = SKMAX;  // row stride of the zero-padded copy of J's last columns

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

__device__ inline unsigned int pk_bf16(float a, float b) {
  return __builtin_bit_cast(unsigned int, __builtin_convertvector((f32x2){a, b}, bf16x2));
}
// byte offset of (row r, chunk c) in a plane of SK-element rows
template <int SK>
__device__ inline int poff(int r, int c) {
  constexpr int PCH = SK / 8;
  const int sw = (SK == 32) ? ((r >> 2) & 3) : ((r >> 3) & 1);
  return r * (PCH * 16) + ((c ^ sw) << 4);
}

// rounding residual of the pair packed in h: (x - hi(x), y - hi(y))
__device__ inline unsigned int pk_lo(float x, float y, unsigned int h) {
  return pk_bf16(x - __uint_as_float(h << 16), y - __uint_as_float(h & 0xffff0000u));
}

template <int PASSES, int SK>
__global__ __launch_bounds__(512) void gram_bf16_kernel(int64_t m, int64_t n,
                                                        const float* __restrict__ J, int64_t ldJ,
                                                        float* __restrict__ work,
                                                        int64_t k_per_split, int64_t ntiles,
                                                        int splits,
                                                        int64_t split0,
                                                        const float* __restrict__ Jt) {
  constexpr bool LO = (PASSES >= 3);
  constexpr bool LOLO = (PASSES == 4);
  constexpr int PCH = SK / 8;              // 16-byte bf16 chunks per plane row
  constexpr int LPR = SK / 8;              // loading lanes per row (8 floats each)
  constexpr int NQ = BT * LPR / NTH;       // rows per thread per panel and step
  constexpr int DEEP = (SK == 16) ? 2 : 1;  // register sets of prefetched steps
  constexpr int PLANE = BT * PCH * 16;     // bytes per plane per stage
  // stage s: A hi, B hi, A lo, B lo
  __shared__ __attribute__((aligned(16))) char lds[2][LO ? 4 : 2][PLANE];

  // launch index -> (split, tile): workgroups go round-robin over the XCDs;
  // each XCD owns a band of consecutive tiles and walks it split after split,
  // so all XCDs work on the same split at a time (its slab of J stays in the
  // memory-side cache) and tiles of one band share row panels in the XCD's L2
  const int64_t lin = blockIdx.x;
  const int64_t xcd = lin % NXCD, kx = lin / NXCD;
  const int64_t q = ntiles / NXCD, rr = ntiles % NXCD;
  const int64_t tb = q + (xcd < rr ? 1 : 0);            // tiles in this XCD's band
  const int64_t t0 = xcd * q + min(xcd, rr);
  if (tb == 0 || kx >= tb * (int64_t)splits) return;   // padding slots
  const int64_t lsplit = kx / tb;                       // split within this launch
  const int64_t split = split0 + lsplit;                // split of the whole K range
  const int64_t logical = t0 + kx % tb;
  int64_t ti, tj;
  tri_decode_g(logical, ti, tj);
  const int64_t kbeg = split * k_per_split;
  const int64_t kend = min(n, kbeg + k_per_split);

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 2, wn = wave & 3;   // 2 x 4 waves

  // load geometry: load q of a panel covers row (NTH / LPR) q + t / LPR,
  // floats 8 (t % LPR) .. +7 of the step. Rows beyond m read row m - 1
  // (their K entries are discarded). The last, partial step of the K range
  // (n % SK columns) is read from Jt, those columns copied zero-padded (row
  // stride JTS), so that every step is the same vector load.
  const int lch = t % LPR;                  // 8-float chunk within the step
  int lrow[NQ];
  const float* pa[NQ];
  const float* pb[NQ];
  const float* qa[NQ];
  const float* qb[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    lrow[q] = (NTH / LPR) * q + t / LPR;
    const int64_t ra_ = min(ti * BT + lrow[q], m - 1), rb_ = min(tj * BT + lrow[q], m - 1);
    pa[q] = J + ra_ * ldJ + kbeg + 8 * lch;
    pb[q] = J + rb_ * ldJ + kbeg + 8 * lch;
    qa[q] = Jt + ra_ * JTS + 8 * lch;
    qb[q] = Jt + rb_ * JTS + 8 * lch;
  }
  // prefetched FP32 slabs: [register set][q][half]
  float4 ra[DEEP][NQ][2], rb[DEEP][NQ][2];
  // step sidx of this split; B is loaded even on diagonal tiles (same rows,
  // L2 hits), which keeps the main loop free of branches
  const int64_t len = kend > kbeg ? kend - kbeg : 0;
  const int64_t nfull = len / SK;
  const int64_t nk = nfull + ((len % SK) != 0 ? 1 : 0);
  auto gload = [&](int rs, int64_t sidx) {
    const bool inJ = sidx < nfull;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const float* a = inJ ? pa[q] + sidx * SK : qa[q];
      const float* b = inJ ? pb[q] + sidx * SK : qb[q];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        ra[rs][q][h] = *reinterpret_cast<const float4*>(a + 4 * h);
        rb[rs][q][h] = *reinterpret_cast<const float4*>(b + 4 * h);
      }
    }
  };
  // split 8 floats into bf16 hi (and lo) and store one 16-byte chunk per plane
  auto put = [&](char* hp, char* lp, int r, const float4& x, const float4& y) {
    const uint4 h{pk_bf16(x.x, x.y), pk_bf16(x.z, x.w), pk_bf16(y.x, y.y), pk_bf16(y.z, y.w)};
    const int off = poff<SK>(r, lch);
    *reinterpret_cast<uint4*>(hp + off) = h;
    if (LO)
      *reinterpret_cast<uint4*>(lp + off) = uint4{pk_lo(x.x, x.y, h.x), pk_lo(x.z, x.w, h.y),
                                                  pk_lo(y.x, y.y, h.z), pk_lo(y.z, y.w, h.w)};
  };
  auto stage_store = [&](int rs, int st) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      put(lds[st][0], LO ? lds[st][2] : nullptr, lrow[q], ra[rs][q][0], ra[rs][q][1]);
      put(lds[st][1], LO ? lds[st][3] : nullptr, lrow[q], rb[rs][q][0], rb[rs][q][1]);
    }
  };

  f32x16 acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  auto frag = [&](const char* plane, int r, int sl) -> bf16x8 {
    Chunk c;
    c.u = *reinterpret_cast<const uint4*>(plane + poff<SK>(r, 2 * sl + (lane >> 5)));
    return c.h;
  };
  // products of one stage; each accumulator is revisited only after the 7
  // others, so back-to-back MFMAs never wait on each other
  auto compute = [&](int st) {
    const char* Ah = lds[st][0];
    const char* Bh = lds[st][1];
    const char* Al = LO ? lds[st][2] : nullptr;
    const char* Bl = LO ? lds[st][3] : nullptr;
#pragma unroll
    for (int sl = 0; sl < SK / 16; ++sl) {
      bf16x8 ah[4], al[4], bh[2], bl[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ra_ = wm * 128 + i * 32 + (lane & 31);
        ah[i] = frag(Ah, ra_, sl);
        if (LO) al[i] = frag(Al, ra_, sl);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int rb_ = wn * 64 + j * 32 + (lane & 31);
        bh[j] = frag(Bh, rb_, sl);
        if (LO) bl[j] = frag(Bl, rb_, sl);
      }
      // all fragment reads of the slice issue before its products
      __builtin_amdgcn_sched_group_barrier(0x100, LO ? 12 : 6, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      if (LO) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
      if (LOLO) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bl[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  constexpr int NMF = (SK / 16) * 8 * (1 + (LO ? 2 : 0) + (LOLO ? 1 : 0));  // MFMAs per step
  constexpr int NDW = 2 * NQ * (LO ? 2 : 1);                              // LDS stores per step
  // SK = 16: the conversion spreads over the whole step (its data arrived a
  // step ago); SK = 32: over the second half (its loads were issued at the
  // start of this step)
  auto hints = [&]() {
    constexpr int FREE = (DEEP == 2) ? 0 : NMF / 2;  // leading MFMAs without conversion work
    constexpr int PER = (NMF - FREE) / NDW;
#pragma unroll
    for (int i = 0; i < FREE; ++i) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
#pragma unroll
    for (int i = 0; i < NMF - FREE; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);               // one MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, DEEP == 2 ? 2 : 4, 0);  // VALU
      if (i % PER == PER - 1) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS store
    }
  };
  if (nk > 0) {
    int64_t it = 0;
    if constexpr (DEEP == 2) {
      gload(0, 0);
      if (nk > 1) gload(1, 1);
      stage_store(0, 0);
      __syncthreads();
      // invariant: stage 0 holds step it, register set 1 holds step it+1
      for (; it + 3 < nk; it += 2) {
        gload(0, it + 2);
        __builtin_amdgcn_sched_barrier(0);
        compute(0);
        stage_store(1, 1);
        hints();
        __syncthreads();
        gload(1, it + 3);
        __builtin_amdgcn_sched_barrier(0);
        compute(1);
        stage_store(0, 0);
        hints();
        __syncthreads();
      }
      // drain the last one to three steps (stage st holds step it, register
      // set 1 holds step it+1)
      int st = 0;
      for (; it < nk; ++it) {
        compute(st);
        if (it + 1 < nk) stage_store(1, st ^ 1);
        __syncthreads();
        if (it + 2 < nk) gload(1, it + 2);
        st ^= 1;
      }
    } else {
      gload(0, 0);
      stage_store(0, 0);
      __syncthreads();
      for (; it + 1 < nk; ++it) {
        gload(0, it + 1);
        __builtin_amdgcn_sched_barrier(0);
        compute((int)(it & 1));
        stage_store(0, (int)(it & 1) ^ 1);
        hints();
        __syncthreads();
      }
      compute((int)(it & 1));
    }
  }

  // accumulator v of block (i, j): row 8 (v/4) + 4 (lane/32) + v%4, col lane%32
  float* out = work + (lsplit * ntiles + logical) * (BT * BT);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = wm * 128 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int cl = wn * 64 + j * 32 + (lane & 31);
        out[rl * BT + cl] = acc[i][j][v];
      }
}

// Jt (m x JTS, row-major) = columns n0 .. n-1 of J, zero-padded to JTS columns.
__global__ void gram_tail_kernel(int64_t m, int64_t n, int64_t n0, const float* __restrict__ J,
                                 int64_t ldJ, float* __restrict__ Jt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m * JTS) return;
  const int64_t r = i / JTS, c = n0 + i % JTS;
  Jt[i] = c < n ? J[r * ldJ + c] : 0.0f;
}

// K (lower triangle) = [K +] sum of the partial tiles in split order [+ lambda I]:
// the first batch of splits writes K and adds lambda, later batches accumulate.
template <typename P, int T>
__global__ __launch_bounds__(256) void gram_reduce_kernel(int64_t m, const P* __restrict__ work,
                                                          int splits, int64_t ntiles,
                                                          double lambda, double* __restrict__ K,
                                                          int64_t ldK, int accumulate) {
  int64_t ti, tj;
  tri_decode_g(blockIdx.x, ti, tj);
  const int base = (blockIdx.y * 256 + threadIdx.x) * 4;  // 4 consecutive elements
  const int rl = base / T, cl0 = base % T;
  const int64_t row = ti * T + rl;
  if (row >= m) return;
  double s[4] = {0, 0, 0, 0};
  for (int sp = 0; sp < splits; ++sp) {
    const P* p = work + ((int64_t)sp * ntiles + blockIdx.x) * (T * T) + rl * T + cl0;
    // each partial is read once: streaming (nontemporal) loads
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] += (double)__builtin_nontemporal_load(p + e);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t col = tj * T + cl0 + e;
    if (col < m && col <= row) {
      double* k = K + row * ldK + col;
      *k = accumulate ? *k + s[e] : s[e] + (row == col ? lambda : 0.0);
    }
  }
}

// FP64 path: enough splits to fill the chip.
int choose_splits_f64(int64_t ntiles, int64_t n) {
  int64_t s = cdiv(1536, ntiles);
  s = std::min<int64_t>(s, std::max<int64_t>(1, n / 2048));
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

// bf16 path: <= ~4096 terms per split (accuracy) and enough workgroups to
// fill the chip. At most kSplitBatch splits are in flight (the workspace);
// more are run in batches whose partials are added into K in order.
constexpr int kSplitBatch = 64;
int64_t choose_splits_bf16(int64_t ntiles, int64_t n) {
  int64_t s = std::max<int64_t>(cdiv(n, 4096), std::min<int64_t>(cdiv(3072, ntiles), kSplitBatch));
  s = std::min<int64_t>(s, std::max<int64_t>(1, cdiv(n, SKMAX)));
  return std::max<int64_t>(1, s);
}

// Step length of the bf16 kernel: 32 once a row of J spans a 2 MB page or
// more (then each row touched costs an address translation, so fewer touches
// per byte win), else 16 (two steps in flight).
int gram_step_len(int64_t ldJ) { return ldJ * (int64_t)sizeof(float) >= (2 << 20) ? 32 : 16; }

}  // namespace

size_t gram_workspace_bytes(int64_t m, int64_t n, int j_dtype, int passes, int* splits_out) {
  if (j_dtype == 0 || passes == kGramF64) {
    const int64_t nt = lower_tiles(m, GT);
    const int s = choose_splits_f64(nt, n);
    if (splits_out) *splits_out = s;
    return (size_t)s * (size_t)nt * GT * GT * sizeof(double);
  }
  const int64_t nt = lower_tiles(m, BT);
  const int64_t s = choose_splits_bf16(nt, n);
  if (splits_out) *splits_out = (int)s;
  // partial tiles, then the zero-padded last columns (m x JTS)
  return (size_t)std::min<int64_t>(s, kSplitBatch) * (size_t)nt * BT * BT * sizeof(float) +
         (size_t)round_up(m * JTS * (int64_t)sizeof(float), 256);
}

int gram_launch(hipStream_t st, int64_t m, int64_t n, const void* J, int64_t ldJ, int j_dtype,
                int passes, double lambda, double* K, int64_t ldK, void* work, size_t work_bytes,
                hipEvent_t ev_begin, hipEvent_t ev_end) {
  int splits = 1;
  const size_t need = gram_workspace_bytes(m, n, j_dtype, passes, &splits);
  DNGD_REQUIRE(work_bytes >= need, "gram: workspace too small (%zu < %zu)", work_bytes, need);
  const bool bf16_path = !(j_dtype == 0 || passes == kGramF64);
  float* Jt = nullptr;
  if (bf16_path) {
    DNGD_REQUIRE(ldJ % 4 == 0 && reinterpret_cast<uintptr_t>(J) % 16 == 0,
                 "gram: FP32 J needs ldJ %% 4 == 0 and a 16-byte aligned base");
    const int64_t nt = lower_tiles(m, BT);
    Jt = reinterpret_cast<float*>(static_cast<char*>(work) +
                                  (size_t)std::min<int64_t>(splits, kSplitBatch) * nt * BT * BT *
                                      sizeof(float));
    const int sk = gram_step_len(ldJ);
    if (n % sk != 0) {
      hipLaunchKernelGGL(gram_tail_kernel, dim3((unsigned)cdiv(m * JTS, 256)), dim3(256), 0, st,
                         m, n, n - n % sk, static_cast<const float*>(J), ldJ, Jt);
      DNGD_LAUNCH_CHECK();
    }
  }
  if (ev_begin) DNGD_HIP(hipEventRecord(ev_begin, st));
  if (!bf16_path) {
    const int64_t nt = lower_tiles(m, GT);
    int rc = (j_dtype == 0)
                 ? gemm_f64(st, GEMM_PARTIAL_LOWER, true, true, m, m, n, 1.0,
                            static_cast<const double*>(J), ldJ, static_cast<const double*>(J),
                            ldJ, 0.0, nullptr, 0, static_cast<double*>(work), splits)
                 : gemm_f64_syrk_partial_f32(st, m, n, static_cast<const float*>(J), ldJ,
                                             static_cast<double*>(work), splits);
    if (rc) return rc;
    if (ev_end) DNGD_HIP(hipEventRecord(ev_end, st));
    hipLaunchKernelGGL((gram_reduce_kernel<double, GT>), dim3((unsigned)nt, GT * GT / 1024),
                       dim3(256), 0, st, m, static_cast<const double*>(work), splits, nt, lambda,
                       K, ldK, 0);
    DNGD_LAUNCH_CHECK();
    return 0;
  }
  DNGD_REQUIRE(passes == 1 || passes == 3 || passes == 4, "gram: passes must be 1, 3, 4 or %d",
               kGramF64);
  const int64_t nt = lower_tiles(m, BT);
  const int64_t kps = round_up(cdiv(n, splits), SKMAX);
  const int sk = gram_step_len(ldJ);
  for (int64_t s0 = 0; s0 < splits; s0 += kSplitBatch) {
    const int sb = (int)std::min<int64_t>(kSplitBatch, splits - s0);
    const int64_t per_xcd = (int64_t)sb * cdiv(nt, NXCD);  // slots of the largest band
    // one workgroup per (split, tile); the kernel derives both from blockIdx.x
    const dim3 grid((unsigned)(per_xcd * NXCD));
    float* w = static_cast<float*>(work);
    const float* Jf = static_cast<const float*>(J);
    if (passes == 4)
      hipLaunchKernelGGL((sk == 16 ? gram_bf16_kernel<4, 16> : gram_bf16_kernel<4, 32>), grid,
                         dim3(512), 0, st, m, n, Jf, ldJ, w, kps, nt, sb, s0, Jt);
    else if (passes == 3)
      hipLaunchKernelGGL((sk == 16 ? gram_bf16_kernel<3, 16> : gram_bf16_kernel<3, 32>), grid,
                         dim3(512), 0, st, m, n, Jf, ldJ, w, kps, nt, sb, s0, Jt);
    else
      hipLaunchKernelGGL((sk == 16 ? gram_bf16_kernel<1, 16> : gram_bf16_kernel<1, 32>), grid,
                         dim3(512), 0, st, m, n, Jf, ldJ, w, kps, nt, sb, s0, Jt);
    DNGD_LAUNCH_CHECK();
    if (ev_end && s0 + sb >= splits) DNGD_HIP(hipEventRecord(ev_end, st));
    hipLaunchKernelGGL((gram_reduce_kernel<float, BT>), dim3((unsigned)nt, BT * BT / 1024),
                       dim3(256), 0, st, m, static_cast<const float*>(work), sb, nt, lambda, K,
                       ldK, s0 > 0 ? 1 : 0);
    DNGD_LAUNCH_CHECK();
  }
  return 0;
}

}  // namespace dngd
