// Dense dual solver (Section 4.1): Cholesky factorisation of
// K~ = K + lambda I and the forward / backward substitutions.
//
// Factorisation: right-looking, block width 64.
//   panel kernel  one 256-thread workgroup per 64 rows of the current block
//                 column. Every workgroup factors the 64 x 64 diagonal block
//                 in LDS (8-column groups: a parallel update, then an 8-step
//                 substitution inside one wave), workgroup 0 writes L11 and
//                 the reciprocal pivots, the others solve their rows of
//                 L21 = A21 L11^-T in the same groups, alongside.
//   update        A22 -= L21 L21^T on the FP64 matrix cores (lower tiles).
// A non-positive or non-finite pivot records its 1-based column in *info
// (first failure wins) and poisons the rest of the factor with NaN.
//
// Solves: blocked forward / backward substitution with inverted diagonal
// blocks (see chol_prepare_solve below); every kernel is independent of the
// others' progress (no inter-workgroup waiting).
#include "common.h"

namespace dngd {

namespace {

constexpr int NB = 64;
// CUs kept free of the look-ahead's trailing update beyond one per panel
// workgroup (more leave the main stream's block-column update short of CUs)
constexpr int kSideFreeExtra = 0;

// Grouped right-to-left elimination of one 64-wide panel, 8 columns at a
// time. For group g (columns c0 .. c0+7):
//   update  the group's columns of every row with the finished columns
//           k < c0 (a 64 x 8 x c0 product on the FP64 matrix cores), then
//   finish  the 8 columns by substitution inside wave 0 (lane i = row i,
//           8 dependent steps with no workgroup barrier; LDS accesses of one
//           wave complete in order).
// Two barriers per group instead of two per column.
constexpr int GW = 8;  // columns per group

typedef double f64x4_t __attribute__((ext_vector_type(4)));

// For the group's 8 columns c0 .. c0+7, subtract the finished columns k < c0:
//   Ld[i][c0 + j] -= sum_k Ld[i][k] Ld[c0 + j][k]   (diagonal block, rows i >= c0)
//   X[i][c0 + j]  -= sum_k X[i][k]  Ld[c0 + j][k]   (this workgroup's L21 rows)
// on the FP64 matrix cores. Wave w owns rows 16 w .. 16 w + 15 (a 16 x 16
// tile whose columns 8..15 are padding); k advances by 8 as two independent
// v_mfma_f64_16x16x4f64 chains per matrix (A lane l = (row l % 16, k l / 16),
// B lane l = (k l / 16, col l % 16), D element v of lane l = (row l / 16 + 4 v,
// col l % 16)), so the dependent chains are a quarter of c0 / 4 long.
__device__ inline void group_update(double (*Ld)[NB + 1], double (*X)[NB + 1], int c0,
                                    bool has_x) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ar = 16 * wave + (lane & 15), kq = lane >> 4, bc = lane & 15;
  const bool has_d = 16 * wave + 15 >= c0;  // this wave holds diagonal rows still open
  f64x4_t d0 = {0.0, 0.0, 0.0, 0.0}, d1 = d0, x0 = d0, x1 = d0;
  for (int k0 = 0; k0 < c0; k0 += 8) {
    const double b0 = (bc < GW) ? Ld[c0 + bc][k0 + kq] : 0.0;
    const double b1 = (bc < GW) ? Ld[c0 + bc][k0 + 4 + kq] : 0.0;
    if (has_d) {
      d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ld[ar][k0 + kq], b0, d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Ld[ar][k0 + 4 + kq], b1, d1, 0, 0, 0);
    }
    if (has_x) {
      x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(X[ar][k0 + kq], b0, x0, 0, 0, 0);
      x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(X[ar][k0 + 4 + kq], b1, x1, 0, 0, 0);
    }
  }
  if (bc < GW) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * wave + kq + 4 * v;
      if (has_d && r >= c0) Ld[r][c0 + bc] -= d0[v] + d1[v];
      if (has_x) X[r][c0 + bc] -= x0[v] + x1[v];
    }
  }
}

// 1 / sqrt(d) for a positive finite d: the hardware estimate refined by two
// Newton steps r <- r (3/2 - d r^2 / 2) (quadratic convergence from the
// estimate's ~2^-22 relative error to FP64 rounding).
__device__ inline double rsqrt_f64(double d) {
  double r = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  r = r * __builtin_fma(-h * r, r, 1.5);
  r = r * __builtin_fma(-h * r, r, 1.5);
  return r;
}

// Value of v held by lane `lane` (uniform), broadcast to the wave.
__device__ inline double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Every workgroup reads the diagonal block from K, so workgroup 0 must not
// overwrite it while others may still be loading it (workgroups of a launch
// can start at any time): L11 goes to `lbuf` (64 x 64, row-major) and is
// copied into K by diag_writeback_kernel after the last panel (nothing reads
// the factored diagonal blocks before that).
__global__ __launch_bounds__(256) void potrf_panel_kernel(int64_t m, double* __restrict__ K,
                                                          int64_t ldK, int64_t j0,
                                                          int64_t* __restrict__ info,
                                                          double* __restrict__ dinv,
                                                          double* __restrict__ lbuf) {
  // Ld: the diagonal block, factored in place (lower part). X: this
  // workgroup's 64 panel rows below it (workgroups >= 1), solved
  // X L11^T = A21 alongside, group by group.
  __shared__ double Ld[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ double rinv[NB];
  __shared__ int sbad;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int nb = (int)min<int64_t>(NB, m - j0);
  const bool has_x = blockIdx.x > 0;
  const int64_t r0 = j0 + (int64_t)blockIdx.x * NB;

  // ---- load the diagonal block (identity padding beyond m) and this
  //      workgroup's rows of the panel, coalesced
  {
    // every load unconditional, from a clamped in-bounds address, and both
    // blocks' loads in flight together (a conditional load is waited for
    // before the next one is issued); workgroup 0 reads its X rows (the
    // diagonal block's) and drops them
    double v[16], w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = q * 256 + t, i = e / NB, k = e % NB;
      v[q] = K[(j0 + min(i, nb - 1)) * ldK + j0 + min(k, nb - 1)];
      w[q] = K[min(r0 + i, m - 1) * ldK + j0 + min(k, nb - 1)];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = q * 256 + t, i = e / NB, k = e % NB;
      if (!(i < nb && k <= i)) v[q] = (i >= nb && k == i) ? 1.0 : 0.0;
      if (!(r0 + i < m && k < nb)) w[q] = 0.0;
      Ld[i][k] = v[q];
      if (has_x) X[i][k] = w[q];
    }
  }
  __syncthreads();
  // ---- per group: the update, then the substitution in wave 0:
  //      L_jj = sqrt(a_jj - sum_k L_jk^2),  L_ij = (a_ij - sum_k L_ik L_jk) / L_jj
  //      for the diagonal block's rows i and this workgroup's rows alike
  int bad = -1;  // wave 0: first failing pivot column of the block (uniform)
#pragma unroll
  for (int c0 = 0; c0 < NB; c0 += GW) {
    if (c0 > 0) group_update(Ld, X, c0, has_x);
    __syncthreads();
    if (wave == 0) {
      // lane i holds row i of the group (diagonal block: x, panel rows: y)
      // in registers; row c0 + j of L (the multipliers of step j) is read
      // from lane c0 + j of x
      const int i = lane;
      double x[GW], y[GW];
#pragma unroll
      for (int j = 0; j < GW; ++j) {
        x[j] = Ld[i][c0 + j];
        y[j] = has_x ? X[i][c0 + j] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < GW; ++j) {
        const int pj = c0 + j;
        double sij = x[j], yij = y[j];
#pragma unroll
        for (int k = 0; k < j; ++k) {
          const double l = lane_value(x[k], pj);  // L[pj][c0 + k], uniform
          sij -= x[k] * l;
          yij -= y[k] * l;
        }
        const double d = lane_value(sij, pj);  // the pivot, uniform
        double inv, ljj;
        if (d > 0.0 && __builtin_isfinite(d)) {
          inv = rsqrt_f64(d);
          ljj = d * inv;
        } else {
          if (bad < 0) bad = pj;
          inv = ljj = __builtin_nan("");
        }
        x[j] = (i == pj) ? ljj : ((i > pj) ? sij * inv : x[j]);
        y[j] = yij * inv;
        if (i == 0) rinv[pj] = inv;
      }
#pragma unroll
      for (int j = 0; j < GW; ++j) {
        if (i >= c0 + j) Ld[i][c0 + j] = x[j];
        if (has_x) X[i][c0 + j] = y[j];
      }
    }
    __syncthreads();
  }

  if (wave == 0 && lane == 0) sbad = bad;
  __syncthreads();
  if (!has_x) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = q * 256 + t;
      lbuf[e] = Ld[e / NB][e % NB];
    }
    if (t < nb && dinv) dinv[j0 + t] = rinv[t];
    if (t == 0 && sbad >= 0 && sbad < nb) {
      unsigned long long* p = reinterpret_cast<unsigned long long*>(info);
      atomicCAS(p, 0ull, (unsigned long long)(j0 + sbad + 1));
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = q * 256 + t, i = e / NB, k = e % NB;
    if (r0 + i < m && k < nb) K[(r0 + i) * ldK + j0 + k] = X[i][k];
  }
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) { *p = v; }

// K's diagonal 64 x 64 blocks (lower part) <- the factored blocks in lbuf
__global__ __launch_bounds__(256) void diag_writeback_kernel(int64_t m, double* __restrict__ K,
                                                             int64_t ldK,
                                                             const double* __restrict__ lbuf) {
  const int64_t j0 = (int64_t)blockIdx.x * NB;
  const double* src = lbuf + (int64_t)blockIdx.x * NB * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, k = e % NB;
    if (j0 + i < m && k <= i) K[(j0 + i) * ldK + j0 + k] = src[e];
  }
}

// ---------------------------------------------------------------------------
// Solves with the factor: L and L^T are applied block by block with explicit
// inverses of their NBI x NBI diagonal blocks (D_q = L_qq^{-1}), so every step
// is a bandwidth-bound matrix-vector product:
//   forward   y_q = D_q b_q ;  b_{>q} -= L_{>q,q} y_q
//   backward  x_q = D_q^T y_q ;  y_{<q} -= L_{q,<q}^T x_q
// The D_q are built after the factorisation: 64 x 64 diagonal blocks are
// inverted directly, then doubled up with
//   inv([A 0; B C]) = [A^{-1} 0; -C^{-1} (B A^{-1}) C^{-1}]
// (two batched FP64-MFMA GEMMs per doubling level).

// D_q <- lower part of L_qq, identity beyond m and zero above the diagonal.
__global__ void blkdiag_copy_kernel(int64_t m, const double* __restrict__ L, int64_t ldL,
                                    int64_t nbi, double* __restrict__ D) {
  const int64_t q = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nbi * nbi) return;
  const int64_t i = e / nbi, k = e % nbi;
  const int64_t gi = q * nbi + i, gk = q * nbi + k;
  double v;
  if (gi < m) v = (k <= i) ? L[gi * ldL + gk] : 0.0;
  else v = (i == k) ? 1.0 : 0.0;
  D[q * nbi * nbi + e] = v;
}

// dst[j][i] = src[i][j] for a batch of rows x cols matrices (64 x 64 tiles
// through LDS, both sides coalesced). lower_only: only src entries with
// j < i (strict lower) are moved.
__global__ __launch_bounds__(256) void transpose_kernel(int64_t rows, int64_t cols,
                                                        const double* __restrict__ src,
                                                        int64_t lds, int64_t sstride,
                                                        double* __restrict__ dst, int64_t ldd,
                                                        int64_t dstride, int lower_only) {
  __shared__ double tile[64][65];
  const int64_t b = blockIdx.z;
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  if (lower_only && j0 > i0 + 63) return;  // tile entirely above the diagonal
  src += b * sstride;
  dst += b * dstride;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int64_t i = i0 + r, j = j0 + tx;
    tile[r][tx] = (i < rows && j < cols) ? src[i * lds + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t j = j0 + r, i = i0 + tx;  // dst row j, column i
    if (j < cols && i < rows && (!lower_only || j < i)) dst[j * ldd + i] = tile[tx][r];
  }
}

// In-place inverse of every 64 x 64 diagonal block of the D_q: lane c
// computes column c by forward substitution.
__global__ __launch_bounds__(64) void tri_inv64_kernel(int64_t nbi, double* __restrict__ D) {
  __shared__ double Lb[NB][NB + 1];
  __shared__ double Xb[NB][NB + 1];
  const int c = threadIdx.x;
  const int64_t q = blockIdx.y, p = blockIdx.x;
  double* base = D + q * nbi * nbi + p * NB * (nbi + 1);
  for (int i = 0; i < NB; ++i) Lb[i][c] = base[i * nbi + c];
  __syncthreads();
  for (int i = 0; i < NB; ++i) {
    double x;
    if (i < c) {
      x = 0.0;
    } else if (i == c) {
      x = 1.0 / Lb[c][c];
    } else {
      double s0 = 0.0, s1 = 0.0;
      int k = c;
      for (; k + 1 < i; k += 2) {
        s0 += Lb[i][k] * Xb[k][c];
        s1 += Lb[i][k + 1] * Xb[k + 1][c];
      }
      if (k < i) s0 += Lb[i][k] * Xb[k][c];
      x = -(s0 + s1) / Lb[i][i];
    }
    Xb[i][c] = x;
  }
  for (int i = 0; i < NB; ++i) base[i * nbi + c] = Xb[i][c];
}

// y[r] = alpha * sum_k A[r][k] x[k] + beta * y[r]   (r < M; 4 rows per workgroup)
// Each thread loads 4 consecutive doubles of every row per 1024-column chunk,
// so a 1024-wide row segment is one round of loads for the whole workgroup.
constexpr int GR_ROWS = 4;
__global__ __launch_bounds__(256) void gemv_rows_kernel(int64_t M, int64_t K,
                                                        const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ x, double alpha,
                                                        double beta, double* __restrict__ y) {
  __shared__ double red[4][GR_ROWS];
  const int64_t r0 = (int64_t)blockIdx.x * GR_ROWS;
  double acc[GR_ROWS];
#pragma unroll
  for (int q = 0; q < GR_ROWS; ++q) acc[q] = 0.0;
  // loads are unconditional, from clamped in-bounds addresses, and masked
  // afterwards (a conditional load is waited for before the next one)
  for (int64_t k0 = 0; k0 < K; k0 += 1024) {
    const int64_t k = k0 + (int64_t)threadIdx.x * 4;
    double xv[4], av[GR_ROWS][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) xv[e] = x[min(k + e, K - 1)];
#pragma unroll
    for (int q = 0; q < GR_ROWS; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) av[q][e] = A[min(r0 + q, M - 1) * lda + min(k + e, K - 1)];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (k + e < K) {
#pragma unroll
        for (int q = 0; q < GR_ROWS; ++q) acc[q] += av[q][e] * xv[e];
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < GR_ROWS; ++q) {
    double v = acc[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < GR_ROWS && r0 + threadIdx.x < M) {
    const int q = threadIdx.x;
    const double v = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    y[r0 + q] = (beta == 0.0) ? alpha * v : alpha * v + beta * y[r0 + q];
  }
}

// X_q = L_qq^{-1} B_q for the 64-row block q of B, all N columns; one lane
// per column (64 per workgroup), L_qq and the columns staged in LDS.
__global__ __launch_bounds__(64) void trsm_diag_kernel(int64_t ell, const double* __restrict__ L,
                                                       int64_t ldL, int64_t q, int64_t N,
                                                       double* __restrict__ B, int64_t ldB) {
  __shared__ double Lq[NB][NB + 1];
  __shared__ double X[NB][NB + 1];  // X[i][lane]
  const int lane = threadIdx.x;
  const int64_t r0 = q * NB;
  const int nb = (int)min<int64_t>(NB, ell - r0);
  for (int e = lane; e < NB * NB; e += 64) {
    const int i = e / NB, k = e % NB;
    Lq[i][k] = (i < nb && k <= i) ? L[(r0 + i) * ldL + r0 + k] : (i == k ? 1.0 : 0.0);
  }
  const int64_t col = (int64_t)blockIdx.x * 64 + lane;
  const bool cok = col < N;
  for (int i = 0; i < NB; ++i) X[i][lane] = (cok && i < nb) ? B[(r0 + i) * ldB + col] : 0.0;
  __syncthreads();
  for (int i = 0; i < NB; ++i) {
    double sx = X[i][lane];
    for (int k = 0; k < i; ++k) sx -= Lq[i][k] * X[k][lane];
    X[i][lane] = sx / Lq[i][i];
  }
  if (cok)
    for (int i = 0; i < nb; ++i) B[(r0 + i) * ldB + col] = X[i][lane];
}

}  // namespace

int gemv_rows(hipStream_t s, int64_t M, int64_t K, const double* A, int64_t lda, const double* x,
              double alpha, double beta, double* y) {
  if (M <= 0) return 0;
  hipLaunchKernelGGL(gemv_rows_kernel, dim3((unsigned)cdiv(M, GR_ROWS)), dim3(256), 0, s, M, K, A, lda,
                     x, alpha, beta, y);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int trsm_lower_left(hipStream_t s, int64_t ell, const double* L, int64_t ldL, int64_t N, double* B,
                    int64_t ldB) {
  const int64_t nblk = cdiv(ell, NB);
  for (int64_t q = 0; q < nblk; ++q) {
    hipLaunchKernelGGL(trsm_diag_kernel, dim3((unsigned)cdiv(N, 64)), dim3(64), 0, s, ell, L,
                       ldL, q, N, B, ldB);
    DNGD_LAUNCH_CHECK();
    const int64_t rest = ell - (q + 1) * NB;
    if (rest > 0) {
      // B[(q+1)64:, :] -= L[(q+1)64:, q-block] X_q
      int rc = gemm_f64(s, GEMM_FULL, true, false, rest, N, NB, -1.0, L + (q + 1) * NB * ldL + q * NB,
                        ldL, B + q * NB * ldB, ldB, 1.0, B + (q + 1) * NB * ldB, ldB);
      if (rc) return rc;
    }
  }
  return 0;
}

size_t chol_workspace_bytes(int64_t m) { return (size_t)cdiv(m, NB) * NB * NB * sizeof(double); }

int chol_factor(hipStream_t s, int64_t m, double* K, int64_t ldK, int64_t* dinfo, double* work,
                double* dinv, hipStream_t side, hipEvent_t ev_panel, hipEvent_t ev_trail) {
  DNGD_REQUIRE(work != nullptr, "chol_factor: needs chol_workspace_bytes(m) of scratch");
  // Block columns of width NB2 = 4 NB. Inside one, each 64-wide panel is
  // factored (diagonal block + the rows below) and applied to the remaining
  // columns of the same block column. The block column's update of the
  // trailing matrix is split: the next block column (on `s`, needed by the
  // next panels) and the rest (on `side` when given, overlapping the next
  // block columns' panels). The side stream updates block b + 2's columns
  // first and records ev_trail; `s` waits for that before it updates block
  // b + 2's columns itself. The remainder (block b + 3 on) is done before
  // the side stream's next update, which `s` waits for in turn.
  constexpr int NB2 = 4 * NB;
  const bool ahead = side != nullptr && ev_panel != nullptr && ev_trail != nullptr;
  bool side_busy = false, side_used = false;
  int ncu = 0;
  if (ahead) {
    int dev = 0;
    DNGD_HIP(hipGetDevice(&dev));
    DNGD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  }
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, s, dinfo, (int64_t)0);
  DNGD_LAUNCH_CHECK();
  for (int64_t jb = 0; jb < m; jb += NB2) {
    const int64_t jend = std::min<int64_t>(m, jb + NB2);
    for (int64_t j0 = jb; j0 < jend; j0 += NB) {
      const int64_t rows = m - j0;
      const unsigned nblk = (unsigned)cdiv(rows, NB);
      hipLaunchKernelGGL(potrf_panel_kernel, dim3(nblk), dim3(256), 0, s, m, K, ldK, j0, dinfo,
                         dinv, work + (j0 / NB) * NB * NB);
      DNGD_LAUNCH_CHECK();
      const int64_t c0 = j0 + NB;            // first column still to update in this block
      if (c0 < jend) {
        // A[c0:m, c0:jend] -= L[c0:m, j0:j0+NB] L[c0:jend, j0:j0+NB]^T  (lower part)
        int rc = gemm_f64(s, GEMM_FULL_LOWER, true, true, m - c0, jend - c0, NB, -1.0,
                          K + c0 * ldK + j0, ldK, K + c0 * ldK + j0, ldK, 1.0, K + c0 * ldK + c0,
                          ldK);
        if (rc) return rc;
      }
    }
    const int64_t rest = m - jend;
    if (rest <= 0) break;
    const double* L21 = K + jend * ldK + jb;
    double* A22 = K + jend * ldK + jend;
    const int64_t kb = jend - jb;
    if (!ahead) {
      int rc = gemm_f64(s, GEMM_SYRK_LOWER, true, true, rest, rest, kb, -1.0, L21, ldK, L21, ldK,
                        1.0, A22, ldK);
      if (rc) return rc;
      continue;
    }
    // (i) the next block column, rows jend..m (lower part), on s; the
    //     previous side update covered its columns first, so wait for that
    if (side_busy) DNGD_HIP(hipStreamWaitEvent(s, ev_trail, 0));
    const int64_t nxt = std::min<int64_t>(NB2, rest);
    int rc = gemm_f64(s, GEMM_FULL_LOWER, true, true, rest, nxt, kb, -1.0, L21, ldK, L21, ldK,
                      1.0, A22, ldK);
    if (rc) return rc;
    // (ii) everything right of it, on the side stream once this block's
    //      panels are final: first the block column after next (what s
    //      waits for before its next update there), then the remainder
    const int64_t r2 = rest - nxt;
    if (r2 > 0) {
      DNGD_HIP(hipEventRecord(ev_panel, s));
      DNGD_HIP(hipStreamWaitEvent(side, ev_panel, 0));
      const int64_t nx2 = std::min<int64_t>(NB2, r2);
      rc = gemm_f64(side, GEMM_FULL_LOWER, true, true, r2, nx2, kb, -1.0, L21 + nxt * ldK, ldK,
                    L21 + nxt * ldK, ldK, 1.0, A22 + nxt * ldK + nxt, ldK);
      if (rc) return rc;
      DNGD_HIP(hipEventRecord(ev_trail, side));
      side_busy = side_used = true;
      const int64_t r3 = r2 - nx2, o3 = nxt + nx2;
      if (r3 > 0) {
        // on CUs of its own: the FP64 VALU chain of a panel workgroup runs
        // at half speed beside an update workgroup, so the remainder leaves
        // one CU free per workgroup of the next panel (plus kSideFreeExtra),
        // where the next block columns' panels and in-block updates run
        const int64_t busy = cdiv(rest, NB) + kSideFreeExtra;
        const int own = (int)std::max<int64_t>(ncu / 2, ncu - busy);
        rc = gemm_f64(side, GEMM_SYRK_LOWER, true, true, r3, r3, kb, -1.0, L21 + o3 * ldK, ldK,
                      L21 + o3 * ldK, ldK, 1.0, A22 + o3 * ldK + o3, ldK, nullptr, 1, own);
        if (rc) return rc;
      }
    } else {
      side_busy = false;
    }
  }
  if (side_used) {  // everything on the side stream, the last remainder included
    DNGD_HIP(hipEventRecord(ev_trail, side));
    DNGD_HIP(hipStreamWaitEvent(s, ev_trail, 0));
  }
  hipLaunchKernelGGL(diag_writeback_kernel, dim3((unsigned)cdiv(m, NB)), dim3(256), 0, s, m, K,
                     ldK, work);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int64_t chol_solve_block(int64_t m) {
  int64_t nbi = NB;
  while (nbi < m && nbi < 1024) nbi *= 2;
  return nbi;
}

// Solve workspace: D (nb inverted diagonal blocks), their transposes, a
// vector of m, and U = L^T (m x m, strict upper part used), so that both
// substitutions are row-wise matrix-vector products.
size_t chol_solve_aux_bytes(int64_t m) {
  const int64_t nbi = chol_solve_block(m), nb = cdiv(m, nbi);
  return std::max((size_t)(2 * nb * nbi * nbi + m + m * m) * sizeof(double),
                  chol_workspace_bytes(m));
}

int chol_prepare_solve(hipStream_t s, int64_t m, const double* L, int64_t ldL, double* aux) {
  const int64_t nbi = chol_solve_block(m), nb = cdiv(m, nbi);
  double* D = aux;
  double* T = aux + nb * nbi * nbi;
  double* U = T + nb * nbi * nbi + m;
  hipLaunchKernelGGL(blkdiag_copy_kernel, dim3((unsigned)cdiv(nbi * nbi, 256), (unsigned)nb),
                     dim3(256), 0, s, m, L, ldL, nbi, D);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(tri_inv64_kernel, dim3((unsigned)(nbi / NB), (unsigned)nb), dim3(64), 0, s,
                     nbi, D);
  DNGD_LAUNCH_CHECK();
  for (int64_t sz = NB; sz < nbi; sz *= 2) {
    const int64_t pairs = nbi / (2 * sz);
    const int64_t in = 2 * sz * (nbi + 1), out = nbi * nbi;
    // T = B A^{-1}   (B: rows [sz, 2sz) x cols [0, sz) of the pair)
    int rc = gemm_f64_batched(s, true, false, sz, sz, sz, 1.0, D + sz * nbi, nbi, out, in, D, nbi,
                              out, in, 0.0, T + sz * nbi, nbi, out, in, nb, pairs);
    if (rc) return rc;
    // X = -C^{-1} T  written over B
    rc = gemm_f64_batched(s, true, false, sz, sz, sz, -1.0, D + sz * (nbi + 1), nbi, out, in,
                          T + sz * nbi, nbi, out, in, 0.0, D + sz * nbi, nbi, out, in, nb, pairs);
    if (rc) return rc;
  }
  // T_q = D_q^T and U = L^T (strict upper)
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)(nbi / 64), (unsigned)(nbi / 64), (unsigned)nb),
                     dim3(256), 0, s, nbi, nbi, D, nbi, nbi * nbi, T, nbi, nbi * nbi, 0);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)cdiv(m, 64), (unsigned)cdiv(m, 64), 1u),
                     dim3(256), 0, s, m, m, L, ldL, (int64_t)0, U, m, (int64_t)0, 1);
  DNGD_LAUNCH_CHECK();
  return 0;
}

// forward  y_q = D_q b_q ;        b_{>q} -= L_{>q,q} y_q
// backward x_q = D_q^T y_q ;      y_{<q} -= U_{<q,q} x_q   (U = L^T)
int chol_solve(hipStream_t s, int64_t m, const double* L, int64_t ldL, const double* aux,
               double* b) {
  const int64_t nbi = chol_solve_block(m), nb = cdiv(m, nbi);
  const double* D = aux;
  const double* T = aux + nb * nbi * nbi;
  double* y = const_cast<double*>(aux) + 2 * nb * nbi * nbi;
  const double* U = y + m;
  int rc = 0;
  for (int64_t q = 0; q < nb && !rc; ++q) {
    const int64_t r0 = q * nbi, mq = std::min(nbi, m - r0), rest = m - r0 - mq;
    rc = gemv_rows(s, mq, mq, D + q * nbi * nbi, nbi, b + r0, 1.0, 0.0, y + r0);
    if (!rc && rest > 0)
      rc = gemv_rows(s, rest, mq, L + (r0 + mq) * ldL + r0, ldL, y + r0, -1.0, 1.0, b + r0 + mq);
  }
  for (int64_t q = nb - 1; q >= 0 && !rc; --q) {
    const int64_t r0 = q * nbi, mq = std::min(nbi, m - r0);
    rc = gemv_rows(s, mq, mq, T + q * nbi * nbi, nbi, y + r0, 1.0, 0.0, b + r0);
    if (!rc && r0 > 0) rc = gemv_rows(s, r0, mq, U + r0, m, b + r0, -1.0, 1.0, y);
  }
  return rc;
}

}  // namespace dngd
