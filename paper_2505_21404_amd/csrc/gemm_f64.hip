// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4f64).
//
// Used for the tanh-MLP layer products on the jet-row activations (forward,
// adjoint and t-tangent streams), the plain FP64 residual Gramian
// K = J J^T (Definition 3.3) and the trailing update of the blocked Cholesky
// factorisation (dense dual solver, Section 4.1).
//
// Tiling: 256 threads = 4 waves in a 2 x 2 grid; a workgroup owns a BM x BN
// tile of C, a wave (BM/2) x (BN/2), i.e. (BM/32) x (BN/32) MFMA 16x16
// accumulators. K advances 16 at a time through LDS stored k-major
// (As[k][m]), so each group of 16 lanes reads 128 contiguous bytes per
// fragment load (conflict-free). The next K slab is prefetched into
// registers while the current one feeds the MFMAs.
#include "common.h"

namespace dngd {

typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int KS = 16;  // K step
constexpr int kPartialFull = 3;  // split-K full GEMM: tile partials, then gemm_reduce_full
constexpr int kBatched = 5;      // full GEMM over a batch of matrices (blockIdx.z)

// C[row][col] = alpha x + beta C[row][col] for one wave's TM x TN accumulator
// tiles: element v of tile (i, j) sits at row = r0 + 16 i + 4 v, col = c0 + 16 j
// (r0, c0 carry the wave's and the lane's offsets). Elements outside M x N,
// or above the diagonal when `lower`, are left alone. With beta != 0 the C
// values of one tile row are read together, unconditionally from clamped
// in-bounds addresses (a conditional load is waited for before the next one
// is issued); beta == 0 reads nothing.
template <int TM, int TN>
__device__ inline void store_c(const f64x4 (&acc)[TM][TN], int64_t M, int64_t N, double alpha,
                               double beta, double* __restrict__ C, int64_t ldc, int64_t r0,
                               int64_t c0, bool lower) {
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    double old[TN][4];
    if (beta != 0.0) {
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          old[j][v] = C[min(r0 + 16 * i + 4 * v, M - 1) * ldc + min(c0 + 16 * j, N - 1)];
    }
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * i + 4 * v, col = c0 + 16 * j;
        if (row < M && col < N && (!lower || row >= col))
          C[row * ldc + col] =
              (beta == 0.0) ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * old[j][v];
      }
  }
}

// The same update with all of a small tile's C values read up front
// (load_c, unconditional from clamped addresses): issued before the first
// operand stage, the loads travel with it instead of costing the epilogue a
// round trip of its own.
template <int TM, int TN>
__device__ inline void load_c(double (&old)[TM][TN][4], int64_t M, int64_t N,
                              const double* __restrict__ C, int64_t ldc, int64_t r0, int64_t c0) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        old[i][j][v] = C[min(r0 + 16 * i + 4 * v, M - 1) * ldc + min(c0 + 16 * j, N - 1)];
}
template <int TM, int TN>
__device__ inline void store_c_pre(const f64x4 (&acc)[TM][TN], const double (&old)[TM][TN][4],
                                   int64_t M, int64_t N, double alpha, double beta,
                                   double* __restrict__ C, int64_t ldc, int64_t r0, int64_t c0,
                                   bool lower) {
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + 16 * i + 4 * v, col = c0 + 16 * j;
        if (row < M && col < N && (!lower || row >= col))
          C[row * ldc + col] =
              (beta == 0.0) ? alpha * acc[i][j][v] : alpha * acc[i][j][v] + beta * old[i][j][v];
      }
}

__device__ inline void tri_decode(int64_t t, int64_t& i, int64_t& j) {
  int64_t ii = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}

// Load a (rows x KS) slab of op(X) (rows along M or N) into registers,
// widened to FP64 (TI = float: FP32 inputs, exact products in FP64).
// kcontig: X[row*ld + k]; else X[k*ld + row].
template <int ROWS, bool KCONTIG, typename TI = double>
struct SlabLoader {
  static constexpr int PER = ROWS * KS / 256;  // doubles per thread
  __device__ static inline void load(double (&r)[PER], const TI* __restrict__ X, int64_t ld,
                                     int64_t row0, int64_t nrows, int64_t k0, int64_t kend) {
    const int t = threadIdx.x;
    if (KCONTIG) {
      // thread -> one row, PER consecutive k
      constexpr int PARTS = 256 / ROWS;
      const int row = t % ROWS;
      const int part = t / ROWS;
      const int64_t gr = row0 + row;
      const int64_t kb = k0 + part * PER;
      const bool rok = gr < nrows;
      const TI* p = X + (rok ? gr : 0) * ld;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int64_t k = kb + e;
        r[e] = (rok && k < kend) ? (double)p[k] : 0.0;
      }
      (void)PARTS;
    } else {
      // thread -> one k, PER consecutive rows
      constexpr int TPK = ROWS / PER;  // threads per k row
      const int k = t / TPK;
      const int rb = (t % TPK) * PER;
      const int64_t gk = k0 + k;
      const bool kok = gk < kend;
      const TI* p = X + (kok ? gk : 0) * ld;
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int64_t gr = row0 + rb + e;
        r[e] = (kok && gr < nrows) ? (double)p[gr] : 0.0;
      }
    }
  }
  __device__ static inline void store(const double (&r)[PER], double (*S)[ROWS]) {
    const int t = threadIdx.x;
    if (KCONTIG) {
      const int row = t % ROWS;
      const int part = t / ROWS;
#pragma unroll
      for (int e = 0; e < PER; ++e) S[part * PER + e][row] = r[e];
    } else {
      constexpr int TPK = ROWS / PER;
      const int k = t / TPK;
      const int rb = (t % TPK) * PER;
#pragma unroll
      for (int e = 0; e < PER; ++e) S[k][rb + e] = r[e];
    }
  }
};

struct Batch {
  int64_t inner = 1;                 // batch index z -> (z / inner, z % inner)
  int64_t a_out = 0, a_in = 0, b_out = 0, b_in = 0, c_out = 0, c_in = 0;  // element strides
};

template <int BM, int BN, bool AK, bool BKC, int MODE, typename TI = double>
__global__ __launch_bounds__(256) void gemm_f64_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const TI* __restrict__ A, int64_t lda,
    const TI* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    double* __restrict__ work, int64_t k_per_split, int64_t ntiles, Batch bt) {
  if (MODE == kBatched) {
    const int64_t zo = blockIdx.z / bt.inner, zi = blockIdx.z % bt.inner;
    A += zo * bt.a_out + zi * bt.a_in;
    B += zo * bt.b_out + zi * bt.b_in;
    C += zo * bt.c_out + zi * bt.c_in;
  }
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ double As[KS][BM];
  __shared__ double Bs[KS][BN];

  constexpr bool PARTIAL = (MODE == GEMM_PARTIAL_LOWER || MODE == kPartialFull);
  int64_t tm, tn;
  if (MODE == GEMM_FULL || MODE == kPartialFull || MODE == GEMM_FULL_LOWER || MODE == kBatched) {
    tm = blockIdx.x;
    tn = blockIdx.y;
  } else {
    tri_decode(blockIdx.x, tm, tn);
  }
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int split = (MODE == GEMM_PARTIAL_LOWER) ? blockIdx.y : ((MODE == kPartialFull) ? blockIdx.z : 0);
  const int64_t kbeg = PARTIAL ? (int64_t)split * k_per_split : 0;
  const int64_t kend = PARTIAL ? min(K, kbeg + k_per_split) : K;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  f64x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  using LA = SlabLoader<BM, AK, TI>;
  using LB = SlabLoader<BN, BKC, TI>;
  double ra[LA::PER], rb[LB::PER];
  const int64_t nk = (kend > kbeg) ? (kend - kbeg + KS - 1) / KS : 0;
  if (nk > 0) {
    LA::load(ra, A, lda, m0, M, kbeg, kend);
    LB::load(rb, B, ldb, n0, N, kbeg, kend);
  }
  for (int64_t it = 0; it < nk; ++it) {
    LA::store(ra, As);
    LB::store(rb, Bs);
    __syncthreads();
    if (it + 1 < nk) {
      const int64_t k0 = kbeg + (it + 1) * KS;
      LA::load(ra, A, lda, m0, M, k0, kend);
      LB::load(rb, B, ldb, n0, N, k0, kend);
    }
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      double a[TM], b[TN];
      const int kr = kk + (lane >> 4);
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  // epilogue: accumulator element v of tile (i, j) is C[row][col] with
  // row = 16 i + lane / 16 + 4 v, col = 16 j + lane % 16 (wave-relative;
  // lane layout of v_mfma_f64_16x16x4f64 checked on the device)
  if (MODE == GEMM_PARTIAL_LOWER || MODE == kPartialFull) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rl = wm * WM + i * 16 + (lane >> 4) + 4 * v;
          const int cl = wn * WN + j * 16 + (lane & 15);
          const double x = acc[i][j][v];
          if (MODE == GEMM_PARTIAL_LOWER) {
            work[(((int64_t)split * ntiles + blockIdx.x) * BM + rl) * BN + cl] = x;
          } else {
            const int64_t tile = ((int64_t)split * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            work[(tile * BM + rl) * BN + cl] = x;
          }
        }
  } else {  // C itself (the *_LOWER modes: elements with row >= col only)
    store_c(acc, M, N, alpha, beta, C, ldc, m0 + wm * WM + (lane >> 4),
            n0 + wn * WN + (lane & 15), !(MODE == GEMM_FULL || MODE == kBatched));
  }
}

// ---------------------------------------------------------------------------
// K-contiguous operands (C = alpha A B^T + beta C, A: M x K and B: N x K both
// row-major), the common case of every product on this path: BM x BM tiles,
// 4 waves in a 2 x 2 grid, K advancing NTK doubles per stage (16, or 32 for
// the factorisation's short-K updates, whose time is one DMA round trip per
// stage, and for its CU-owning trailing update, which has the LDS). Both row
// panels go from HBM straight into LDS (global_load_lds, 16 B per lane),
// double buffered; a plane row holds NTK/2 chunks of 16 B,
// chunk c of row r stored at c ^ sw(r) with sw(r) = (r >> 1) & 7 for 8 chunks
// (two 128-byte rows share a 256-byte bank window) and r & 15 for 16 chunks,
// so the 16 rows of a fragment read hit 16 distinct bank groups. Each MFMA
// pair takes both values of one 16-byte read: lane group g = lane / 16 feeds
// k = k0 + 2 g to the first v_mfma_f64_16x16x4f64 and k0 + 2 g + 1 to the
// second (the order of the k terms is a permutation).
// Needs lda, ldb even and 16-byte aligned A, B (the host checks).
typedef __attribute__((address_space(3))) void lds_void_t;
constexpr int NTK = 16;  // default doubles of K per stage

template <int KS>
__device__ inline int ntsw(int r) { return KS == 16 ? ((r >> 1) & 7) : (r & 15); }
template <int KS>
__device__ inline int ntoff(int r, int c) { return r * (KS * 8) + ((c ^ ntsw<KS>(r)) << 4); }

// (waves_per_eu caps the VGPRs at 256 so that two workgroups fit a CU; the
// CU-owning SYRK instance cannot have two for its LDS, and says so)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
// TI = float: FP32 operands (the FP64-product Gram of an FP32 Jacobian). A
// stage of KS = 32 floats has the byte layout of 16 doubles; each lane reads
// the FP32 pair of its k pair (8 bytes) and widens it before the FP64 MFMAs.
// Needs lda, ldb multiples of 4 and 16-byte aligned A, B.
template <int BM, int MODE, int KS = NTK, typename TI = double>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void gemm_f64_nt_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const TI* __restrict__ A, int64_t lda,
    const TI* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    double* __restrict__ work, int64_t k_per_split, int64_t ntiles) {
  constexpr bool F32 = sizeof(TI) == 4;
  static_assert(!F32 || KS == 32, "FP32 operands take 32-element stages");
  constexpr int SWK = F32 ? KS / 2 : KS;  // the swizzle of a 128- or 256-byte plane row
  constexpr int BN = BM;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int EPC = 16 / (int)sizeof(TI);  // elements per 16-byte chunk
  constexpr int CH = KS / EPC;        // 16-byte chunks per plane row
  constexpr int RPI = 64 / CH;        // plane rows per DMA instruction (1 KB)
  constexpr int JPT = BM / RPI / 4;   // DMA instructions per wave per operand per stage
  constexpr int PLANE = BM * KS * (int)sizeof(TI);
  __shared__ __attribute__((aligned(16))) char sA0[PLANE];
  __shared__ __attribute__((aligned(16))) char sB0[PLANE];
  __shared__ __attribute__((aligned(16))) char sA1[PLANE];
  __shared__ __attribute__((aligned(16))) char sB1[PLANE];

  constexpr bool PARTIAL = (MODE == GEMM_PARTIAL_LOWER || MODE == kPartialFull);
  // A SYRK launch with fewer workgroups than tiles is persistent: workgroup b
  // takes tiles b, b + gridDim.x, ... (the main loop ends on a barrier, so the
  // LDS planes are free for the next tile). Every other launch: one tile.
  for (int64_t bx = blockIdx.x;; bx += gridDim.x) {
    if (MODE == GEMM_SYRK_LOWER && bx >= ntiles) break;
    int64_t tm, tn;
    if (MODE == GEMM_FULL || MODE == kPartialFull || MODE == GEMM_FULL_LOWER) {
      tm = bx;
      tn = blockIdx.y;
    } else {
      tri_decode(bx, tm, tn);
    }
    const int64_t m0 = tm * BM, n0 = tn * BN;
    const int split = (MODE == GEMM_PARTIAL_LOWER) ? blockIdx.y : ((MODE == kPartialFull) ? blockIdx.z : 0);
    const int64_t kbeg = PARTIAL ? (int64_t)split * k_per_split : 0;
    const int64_t kend = PARTIAL ? min(K, kbeg + k_per_split) : K;
    // the B panel is the A panel (a diagonal tile of a symmetric product)
    const bool same = (A == B) && (lda == ldb) && (m0 == n0);

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;

    // DMA geometry: wave w, instruction j fills slots ((w JPT + j) * 64 + lane):
    // row (w JPT + j) * RPI + lane / CH, physical chunk lane % CH <- logical chunk
    // (lane % CH) ^ sw(row). Rows beyond M (N) read the last row.
    auto dma = [&](int64_t k0, char* dA, char* dB) {
#pragma unroll
      for (int j = 0; j < JPT; ++j) {
        const int r = (wave * JPT + j) * RPI + lane / CH;
        const int64_t k = k0 + EPC * ((lane % CH) ^ ntsw<SWK>(r));
        const int64_t kk = (k < K) ? k : 0;  // in bounds; k >= kend is masked at the read
        // the source pointer is cast to its concrete type: an argument whose
        // type depends on TI would leave the device builtin to template
        // instantiation, which the host pass does not complete (the kernel's
        // host stub is then never emitted)
        const int64_t ia = min(m0 + r, M - 1) * lda + kk, ib = min(n0 + r, N - 1) * ldb + kk;
        char* la = dA + (wave * JPT + j) * 1024;
        char* lb = dB + (wave * JPT + j) * 1024;
        if constexpr (F32) {
          __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(A) + ia,
                                           (lds_void_t*)la, 16, 0, 0);
          if (!same)
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const float*>(B) + ib,
                                             (lds_void_t*)lb, 16, 0, 0);
        } else {
          __builtin_amdgcn_global_load_lds(reinterpret_cast<const double*>(A) + ia,
                                           (lds_void_t*)la, 16, 0, 0);
          if (!same)
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const double*>(B) + ib,
                                             (lds_void_t*)lb, 16, 0, 0);
        }
      }
    };

    f64x4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

    const int g = lane >> 4;
    auto compute = [&](const char* SA, const char* SB, int64_t k0) {
      const bool tail = (k0 + KS > kend);
#pragma unroll
      for (int kp = 0; kp < KS / 8; ++kp) {
        const int c = kp * 4 + g;  // logical chunk: k = k0 + 2 c, 2 c + 1
        bool ok0 = true, ok1 = true;
        if (tail) {
          ok0 = k0 + 2 * c < kend;
          ok1 = k0 + 2 * c + 1 < kend;
        }
        // the k pair (2 c, 2 c + 1) of a plane row: a 16-byte chunk of
        // doubles, or half of one (chunk c / 2, 8-byte half c % 2) of floats
        auto frag = [&](const char* S, int row) -> double2 {
          if constexpr (F32) {
            const float2 f = *reinterpret_cast<const float2*>(
                S + ntoff<SWK>(row, c >> 1) + ((c & 1) << 3));
            return double2{(double)f.x, (double)f.y};
          } else {
            return *reinterpret_cast<const double2*>(S + ntoff<SWK>(row, c));
          }
        };
        double2 a[TM], b[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          a[i] = frag(SA, wm * WM + i * 16 + (lane & 15));
          if (!ok0) a[i].x = 0.0;
          if (!ok1) a[i].y = 0.0;
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          b[j] = frag(SB, wn * WN + j * 16 + (lane & 15));
          if (!ok0) b[j].x = 0.0;
          if (!ok1) b[j].y = 0.0;
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].x, b[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i].y, b[j].y, acc[i][j], 0, 0, 0);
      }
    };

    const int64_t nk = (kend > kbeg) ? (kend - kbeg + KS - 1) / KS : 0;
    // 64-wide tiles (the factorisation's latency-bound updates) read C up front
    constexpr bool PRE = (BM == 64) && !PARTIAL;
    const int64_t cr0 = m0 + wm * WM + (lane >> 4), cc0 = n0 + wn * WN + (lane & 15);
    double cold[PRE ? TM : 1][PRE ? TN : 1][4];
    if (PRE && beta != 0.0) load_c(cold, M, N, C, ldc, cr0, cc0);
    if (nk > 0) dma(kbeg, sA0, sB0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int64_t it = 0; it < nk; it += 2) {
      if (it + 1 < nk) dma(kbeg + (it + 1) * KS, sA1, sB1);
      compute(sA0, same ? sA0 : sB0, kbeg + it * KS);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (it + 1 < nk) {
        if (it + 2 < nk) dma(kbeg + (it + 2) * KS, sA0, sB0);
        compute(sA1, same ? sA1 : sB1, kbeg + (it + 1) * KS);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
      }
    }

    // epilogue as in gemm_f64_kernel: element v of tile (i, j) is C[row][col]
    // with row = 16 i + lane / 16 + 4 v, col = 16 j + lane % 16 (wave-relative)
    if (MODE == GEMM_PARTIAL_LOWER || MODE == kPartialFull) {
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rl = wm * WM + i * 16 + (lane >> 4) + 4 * v;
            const int cl = wn * WN + j * 16 + (lane & 15);
            const double x = acc[i][j][v];
            if (MODE == GEMM_PARTIAL_LOWER) {
              work[(((int64_t)split * ntiles + bx) * BM + rl) * BN + cl] = x;
            } else {
              const int64_t tile =
                  ((int64_t)split * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
              work[(tile * BM + rl) * BN + cl] = x;
            }
          }
    } else if constexpr (PRE) {
      store_c_pre(acc, cold, M, N, alpha, beta, C, ldc, cr0, cc0, MODE != GEMM_FULL);
    } else {
      store_c(acc, M, N, alpha, beta, C, ldc, cr0, cc0, MODE != GEMM_FULL);
    }
    if (MODE != GEMM_SYRK_LOWER) break;
  }
}
#pragma clang diagnostic pop

template <int BM, int BN>
__global__ __launch_bounds__(256) void gemm_reduce_full_kernel(int64_t M, int64_t N, int splits,
                                                               const double* __restrict__ work,
                                                               double alpha, double beta,
                                                               double* __restrict__ C, int64_t ldc) {
  const int e = (blockIdx.z * 256 + threadIdx.x);
  const int rl = e / BN, cl = e % BN;
  const int64_t row = (int64_t)blockIdx.x * BM + rl, col = (int64_t)blockIdx.y * BN + cl;
  if (row >= M || col >= N) return;
  double s = 0.0;
  for (int sp = 0; sp < splits; ++sp) {
    const int64_t tile = ((int64_t)sp * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    s += work[(tile * BM + rl) * BN + cl];
  }
  double* p = C + row * ldc + col;
  *p = (beta == 0.0) ? alpha * s : alpha * s + beta * *p;
}

template <int BM, int BN, bool AK, bool BKC>
int launch_split_full(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                      double* C, int64_t ldc, double* work, int splits) {
  const int64_t kps = round_up(cdiv(K, splits), KS);
  dim3 grid((unsigned)cdiv(M, BM), (unsigned)cdiv(N, BN), (unsigned)splits);
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, AK, BKC, kPartialFull>), grid, dim3(256), 0, s, M, N,
                     K, alpha, A, lda, B, ldb, beta, C, ldc, work, kps, (int64_t)0, Batch{});
  DNGD_LAUNCH_CHECK();
  dim3 g2(grid.x, grid.y, BM * BN / 256);
  hipLaunchKernelGGL((gemm_reduce_full_kernel<BM, BN>), g2, dim3(256), 0, s, M, N, splits, work,
                     alpha, beta, C, ldc);
  DNGD_LAUNCH_CHECK();
  return 0;
}

template <int BM, int BN, bool AK, bool BKC, int MODE>
int launch(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
           int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
           double* work, int splits) {
  dim3 grid;
  int64_t ntiles = 0, kps = K;
  if (MODE == GEMM_FULL || MODE == GEMM_FULL_LOWER) {
    grid = dim3((unsigned)cdiv(M, BM), (unsigned)cdiv(N, BN), 1);
  } else {
    ntiles = lower_tiles(M, BM);
    kps = (MODE == GEMM_PARTIAL_LOWER) ? round_up(cdiv(K, splits), KS) : K;
    grid = dim3((unsigned)ntiles, (MODE == GEMM_PARTIAL_LOWER) ? (unsigned)splits : 1u, 1);
  }
  if (grid.x == 0 || grid.y == 0) return 0;
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, AK, BKC, MODE>), grid, dim3(256), 0, s, M, N, K,
                     alpha, A, lda, B, ldb, beta, C, ldc, work, kps, ntiles, Batch{});
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace

int gemm_f64_batched(hipStream_t s, bool a_kcontig, bool b_kcontig, int64_t M, int64_t N,
                     int64_t K, double alpha, const double* A, int64_t lda, int64_t a_out,
                     int64_t a_in, const double* B, int64_t ldb, int64_t b_out, int64_t b_in,
                     double beta, double* C, int64_t ldc, int64_t c_out, int64_t c_in,
                     int64_t n_outer, int64_t n_inner) {
  if (M <= 0 || N <= 0 || n_outer * n_inner <= 0) return 0;
  Batch bt;
  bt.inner = n_inner;
  bt.a_out = a_out, bt.a_in = a_in, bt.b_out = b_out, bt.b_in = b_in, bt.c_out = c_out,
  bt.c_in = c_in;
  const dim3 grid((unsigned)cdiv(M, 64), (unsigned)cdiv(N, 64), (unsigned)(n_outer * n_inner));
#define DNGD_BATCH_CASE(AKV, BKV)                                                              \
  if (a_kcontig == AKV && b_kcontig == BKV) {                                                 \
    hipLaunchKernelGGL((gemm_f64_kernel<64, 64, AKV, BKV, kBatched>), grid, dim3(256), 0, s, M, \
                       N, K, alpha, A, lda, B, ldb, beta, C, ldc, nullptr, K, (int64_t)0, bt);  \
    DNGD_LAUNCH_CHECK();                                                                      \
    return 0;                                                                                 \
  }
  DNGD_BATCH_CASE(true, true)
  DNGD_BATCH_CASE(true, false)
  DNGD_BATCH_CASE(false, true)
  DNGD_BATCH_CASE(false, false)
#undef DNGD_BATCH_CASE
  return -1;
}

static int gemm_f64_syrk_partial_f32_generic(hipStream_t s, int64_t M, int64_t K, const float* A,
                                             int64_t lda, double* work, int splits) {
  if (M <= 0) return 0;
  const int64_t ntiles = lower_tiles(M, 128);
  const int64_t kps = round_up(cdiv(K, splits), KS);
  hipLaunchKernelGGL((gemm_f64_kernel<128, 128, true, true, GEMM_PARTIAL_LOWER, float>),
                     dim3((unsigned)ntiles, (unsigned)splits), dim3(256), 0, s, M, M, K, 1.0, A,
                     lda, A, lda, 0.0, nullptr, 0, work, kps, ntiles, Batch{});
  DNGD_LAUNCH_CHECK();
  return 0;
}

int64_t lower_tiles(int64_t M, int tile) {
  const int64_t t = cdiv(M, tile);
  return t * (t + 1) / 2;
}

namespace {

// LDS of one CU: a workgroup that reserves all of it (static arrays plus
// dynamic LDS) has its CU to itself
constexpr size_t kLdsPerCu = 160 * 1024;

template <int BM, int MODE, int KS = NTK, typename TI = double>
int launch_nt(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const TI* A,
              int64_t lda, const TI* B, int64_t ldb, double beta, double* C, int64_t ldc,
              double* work, int splits, int own_cus = 0) {
  const size_t static_lds = 4 * (size_t)BM * KS * sizeof(TI);
  static_assert(4 * (size_t)BM * KS * sizeof(TI) <= kLdsPerCu, "LDS planes exceed a CU");
  const size_t dyn = own_cus > 0 ? kLdsPerCu - static_lds : 0;
  dim3 grid;
  int64_t ntiles = 0, kps = K;
  if (MODE == GEMM_FULL || MODE == GEMM_FULL_LOWER) {
    grid = dim3((unsigned)cdiv(M, BM), (unsigned)cdiv(N, BM), 1);
  } else if (MODE == kPartialFull) {
    kps = round_up(cdiv(K, splits), KS);
    grid = dim3((unsigned)cdiv(M, BM), (unsigned)cdiv(N, BM), (unsigned)splits);
  } else {
    ntiles = lower_tiles(M, BM);
    kps = (MODE == GEMM_PARTIAL_LOWER) ? round_up(cdiv(K, splits), KS) : K;
    grid = dim3((unsigned)ntiles, (MODE == GEMM_PARTIAL_LOWER) ? (unsigned)splits : 1u, 1);
  }
  if (grid.x == 0 || grid.y == 0) return 0;
  if (own_cus > 0) {  // persistent: as few workgroups as the same number of rounds needs
    const int64_t rounds = cdiv(grid.x, own_cus);
    grid.x = (unsigned)cdiv(grid.x, rounds);
  }
  hipLaunchKernelGGL((gemm_f64_nt_kernel<BM, MODE, KS, TI>), grid, dim3(256), (unsigned)dyn, s, M, N, K,
                     alpha, A, lda, B, ldb, beta, C, ldc, work, kps, ntiles);
  DNGD_LAUNCH_CHECK();
  if (MODE == kPartialFull) {
    dim3 g2(grid.x, grid.y, BM * BM / 256);
    hipLaunchKernelGGL((gemm_reduce_full_kernel<BM, BM>), g2, dim3(256), 0, s, M, N, splits, work,
                       alpha, beta, C, ldc);
    DNGD_LAUNCH_CHECK();
  }
  return 0;
}

bool nt_ok(const double* A, int64_t lda, const double* B, int64_t ldb) {
  return ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0 &&
         lda % 2 == 0 && ldb % 2 == 0;
}

}  // namespace

int gemm_f64(hipStream_t s, GemmMode mode, bool a_kcontig, bool b_kcontig, int64_t M, int64_t N,
             int64_t K, double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
             double beta, double* C, int64_t ldc, double* work, int splits, int own_cus) {
  if (M <= 0 || N <= 0) return 0;
  if (a_kcontig && b_kcontig && nt_ok(A, lda, B, ldb)) {
    if (mode == GEMM_PARTIAL_LOWER)
      return launch_nt<128, GEMM_PARTIAL_LOWER>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                work, splits);
    if (mode == GEMM_FULL_LOWER)  // short-K factorisation updates: 32 per stage
      return launch_nt<64, GEMM_FULL_LOWER, 32>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                                work, 1);
    if (mode == GEMM_SYRK_LOWER) {
      // a workgroup that owns its CU has the LDS for 32 doubles of K per stage
      if (M >= 1024 && own_cus > 0)
        return launch_nt<128, GEMM_SYRK_LOWER, 32>(s, M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                   ldc, work, 1, own_cus);
      if (M >= 1024)
        return launch_nt<128, GEMM_SYRK_LOWER>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                                               work, 1);
      return launch_nt<64, GEMM_SYRK_LOWER>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work,
                                            1, own_cus);
    }
    if (splits > 1) {
      DNGD_REQUIRE(work != nullptr, "gemm_f64: split-K needs a workspace");
      return launch_nt<64, kPartialFull>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work,
                                         splits);
    }
    if ((cdiv(M, 128) * cdiv(N, 128)) >= 256)
      return launch_nt<128, GEMM_FULL>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, 1);
    return launch_nt<64, GEMM_FULL>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, 1);
  }
  if (mode == GEMM_PARTIAL_LOWER) {
    return launch<128, 128, true, true, GEMM_PARTIAL_LOWER>(s, M, N, K, alpha, A, lda, B, ldb,
                                                             beta, C, ldc, work, splits);
  }
  if (mode == GEMM_FULL_LOWER) {
    DNGD_REQUIRE(a_kcontig && b_kcontig, "gemm_f64: FULL_LOWER needs K-contiguous operands");
    return launch<64, 64, true, true, GEMM_FULL_LOWER>(s, M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                        ldc, work, 1);
  }
  if (mode == GEMM_SYRK_LOWER) {
    if (M >= 1024)
      return launch<128, 128, true, true, GEMM_SYRK_LOWER>(s, M, N, K, alpha, A, lda, B, ldb,
                                                            beta, C, ldc, work, 1);
    return launch<64, 64, true, true, GEMM_SYRK_LOWER>(s, M, N, K, alpha, A, lda, B, ldb, beta,
                                                        C, ldc, work, 1);
  }
  if (splits > 1) {
    DNGD_REQUIRE(work != nullptr, "gemm_f64: split-K needs a workspace");
#define DNGD_SPLIT_CASE(AKV, BKV)                                                            \
    if (a_kcontig == AKV && b_kcontig == BKV)                                                \
      return launch_split_full<64, 64, AKV, BKV>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, \
                                                 ldc, work, splits);
    DNGD_SPLIT_CASE(true, true)
    DNGD_SPLIT_CASE(true, false)
    DNGD_SPLIT_CASE(false, true)
    DNGD_SPLIT_CASE(false, false)
#undef DNGD_SPLIT_CASE
  }
  const bool big = (cdiv(M, 128) * cdiv(N, 128)) >= 512;
#define DNGD_GEMM_CASE(AKV, BKV)                                                               \
  if (a_kcontig == AKV && b_kcontig == BKV) {                                                  \
    if (big)                                                                                   \
      return launch<128, 128, AKV, BKV, GEMM_FULL>(s, M, N, K, alpha, A, lda, B, ldb, beta, C, \
                                                   ldc, work, 1);                              \
    return launch<64, 64, AKV, BKV, GEMM_FULL>(s, M, N, K, alpha, A, lda, B, ldb, beta, C,     \
                                               ldc, work, 1);                                  \
  }
  DNGD_GEMM_CASE(true, true)
  DNGD_GEMM_CASE(true, false)
  DNGD_GEMM_CASE(false, true)
  DNGD_GEMM_CASE(false, false)
#undef DNGD_GEMM_CASE
  return -1;
}

// FP64 products of an FP32 matrix: the K-contiguous kernel (widening at the
// LDS read) when A is 16-byte aligned with lda % 4 == 0, else the generic one.
// Both write the same partial-tile layout (lower 128 x 128 tiles by split).
int gemm_f64_syrk_partial_f32(hipStream_t s, int64_t M, int64_t K, const float* A, int64_t lda,
                              double* work, int splits) {
  if (M <= 0) return 0;
  if (lda % 4 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0)
    return launch_nt<128, GEMM_PARTIAL_LOWER, 32, float>(s, M, M, K, 1.0, A, lda, A, lda, 0.0,
                                                         nullptr, 0, work, splits);
  return gemm_f64_syrk_partial_f32_generic(s, M, K, A, lda, work, splits);
}

}  // namespace dngd
