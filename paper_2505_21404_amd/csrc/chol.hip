// Dense dual solver (Section 4.1): Cholesky factorisation of
// K~ = K + lambda I and the forward / backward substitutions.
//
// Factorisation: right-looking, block width 64.
//   panel kernel  one wave per 64 rows of the current block column. Every
//                 wave factors the 64 x 64 diagonal block in LDS (left-looking
//                 by columns, lane i owns row i), wave 0 writes L11, the others
//                 solve their rows of L21 = A21 L11^-T by substitution.
//   update        A22 -= L21 L21^T on the FP64 matrix cores (lower tiles).
// A non-positive or non-finite pivot records its 1-based column in *info
// (first failure wins) and poisons the rest of the factor with NaN.
//
// Substitutions: one kernel per triangle. Workgroup q owns the 64-row block q.
// It accumulates L[q, k] y_k for every earlier block k as soon as block k has
// published y_k (a per-block flag set with release semantics after the data
// is written), then solves its 64 x 64 diagonal block in one wave with
// readlane broadcasts and publishes y_q. Workgroup q only ever waits on
// workgroups with a smaller index, which are dispatched first; the grid is at
// most m/64 workgroups. Every wait is bounded: after ~2^24 polls the
// workgroup records DNGD_ETIMEOUT in *status, still publishes its flag (so the
// rest of the grid drains) and the host reports the failure.
#include "common.h"

namespace dngd {

namespace {

constexpr int NB = 64;

__device__ inline double readlane_d(double x, int lane) {
  union {
    double d;
    int i[2];
  } u, o;
  u.d = x;
  o.i[0] = __builtin_amdgcn_readlane(u.i[0], lane);
  o.i[1] = __builtin_amdgcn_readlane(u.i[1], lane);
  return o.d;
}

__global__ __launch_bounds__(64) void potrf_panel_kernel(int64_t m, double* __restrict__ K,
                                                         int64_t ldK, int64_t j0,
                                                         int64_t* __restrict__ info) {
  // Ld: the diagonal block, factored in place (lower part). X: this
  // workgroup's 64 panel rows below it (workgroups >= 1).
  __shared__ double Ld[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int lane = threadIdx.x;
  const int nb = (int)min<int64_t>(NB, m - j0);

  // ---- load the diagonal block (identity padding beyond m)
  for (int k = 0; k < NB; ++k) {
    double v = 0.0;
    if (lane < nb && k <= lane && k < nb) v = K[(j0 + lane) * ldK + j0 + k];
    if (lane >= nb && k == lane) v = 1.0;
    Ld[lane][k] = v;
  }
  __syncthreads();
  // ---- left-looking factorisation, lane i owns row i:
  //      s_i = A_ij - sum_{k<j} L_ik L_jk ;  L_jj = sqrt(s_j) ;  L_ij = s_i / L_jj
  int bad = -1;
  for (int j = 0; j < NB; ++j) {
    double sij = Ld[lane][j];
    for (int k = 0; k < j; ++k) sij -= Ld[lane][k] * Ld[j][k];
    const double d = __shfl(sij, j);
    double ljj;
    if (d > 0.0 && __builtin_isfinite(d)) {
      ljj = sqrt(d);
    } else {
      if (bad < 0) bad = j;
      ljj = __builtin_nan("");
    }
    if (lane == j) Ld[lane][j] = ljj;
    else if (lane > j) Ld[lane][j] = sij / ljj;
    __syncthreads();
  }

  if (blockIdx.x == 0) {
    if (lane < nb)
      for (int k = 0; k <= lane; ++k) K[(j0 + lane) * ldK + j0 + k] = Ld[lane][k];
    if (lane == 0 && bad >= 0 && bad < nb) {
      unsigned long long* p = reinterpret_cast<unsigned long long*>(info);
      atomicCAS(p, 0ull, (unsigned long long)(j0 + bad + 1));
    }
    return;
  }

  // ---- L21 rows: x L11^T = a  (forward substitution; lane owns one row)
  const int64_t row = j0 + (int64_t)blockIdx.x * NB + lane;
  const bool rok = row < m;
  for (int k = 0; k < NB; ++k) X[lane][k] = (rok && k < nb) ? K[row * ldK + j0 + k] : 0.0;
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    double sx = X[lane][j];
    for (int k = 0; k < j; ++k) sx -= X[lane][k] * Ld[j][k];
    X[lane][j] = sx / Ld[j][j];
  }
  if (rok)
    for (int k = 0; k < nb; ++k) K[row * ldK + j0 + k] = X[lane][k];
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) { *p = v; }

// ---------------------------------------------------------------------------
// chained substitutions

__device__ inline bool wait_flag(const unsigned* f, unsigned epoch, int* status) {
  unsigned spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > (1u << 24)) {
      atomicOr(status, 1);
      return false;
    }
  }
  return true;
}

__device__ inline void publish(unsigned* f, unsigned epoch) {
  __hip_atomic_store(f, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// L y = b, b overwritten by y. 256 threads; block q = blockIdx.x.
__global__ __launch_bounds__(256) void trsv_lower_kernel(int64_t m, const double* __restrict__ L,
                                                         int64_t ldL, double* b, unsigned* flags,
                                                         unsigned epoch, int* status) {
  __shared__ double part[4][NB];
  const int t = threadIdx.x;
  const int64_t q = blockIdx.x;
  const int i = t >> 2, quarter = t & 3;
  const int64_t row = q * NB + i;
  const bool rok = row < m;
  double acc = 0.0;
  for (int64_t k = 0; k < q; ++k) {
    wait_flag(flags + k, epoch, status);
    const double* lp = L + (rok ? row : 0) * ldL + k * NB + quarter * 16;
    const double* yp = b + k * NB + quarter * 16;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc += (rok ? lp[e] : 0.0) * yp[e];
  }
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  if (quarter == 0) part[0][i] = acc;
  __syncthreads();
  if (t < 64) {
    const int lane = t;
    const int64_t r = q * NB + lane;
    const bool ok = r < m;
    double rhs = ok ? (b[r] - part[0][lane]) : 0.0;
    double rowv[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int64_t c = q * NB + k;
      rowv[k] = (ok && k <= lane && c < m) ? L[r * ldL + c] : ((!ok && k == lane) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const double yj = readlane_d(rhs, j) / readlane_d(rowv[j], j);
      if (lane == j) rhs = yj;
      else if (lane > j) rhs -= rowv[j] * yj;
    }
    if (ok) b[r] = rhs;
    __threadfence();
    if (lane == 0) publish(flags + q, epoch);
  }
}

// L^T x = y, y overwritten by x. Workgroup w handles block q = nblk-1-w.
__global__ __launch_bounds__(256) void trsv_upper_kernel(int64_t m, const double* __restrict__ L,
                                                         int64_t ldL, double* b, unsigned* flags,
                                                         unsigned epoch, int* status) {
  __shared__ double part[4][NB];
  const int64_t nblk = (m + NB - 1) / NB;
  const int t = threadIdx.x;
  const int64_t q = nblk - 1 - blockIdx.x;
  const int j = t & 63, wave = t >> 6;
  const int64_t col = q * NB + j;
  const bool cok = col < m;
  double acc = 0.0;
  for (int64_t k = nblk - 1; k > q; --k) {
    wait_flag(flags + k, epoch, status);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t r = k * NB + wave * 16 + e;
      if (r < m) {
        const double xv = b[r];
        acc += (cok ? L[r * ldL + col] : 0.0) * xv;
      }
    }
  }
  part[wave][j] = acc;
  __syncthreads();
  if (t < 64) {
    const int lane = t;
    const int64_t r = q * NB + lane;
    const bool ok = r < m;
    double rhs = ok ? (b[r] - (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]))
                    : 0.0;
    double colv[NB];  // colv[k] = L[q*NB + k][q*NB + lane]
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int64_t rr = q * NB + k;
      colv[k] = (ok && k >= lane && rr < m) ? L[rr * ldL + r] : ((!ok && k == lane) ? 1.0 : 0.0);
    }
#pragma unroll
    for (int jj = NB - 1; jj >= 0; --jj) {
      const double xj = readlane_d(rhs, jj) / readlane_d(colv[jj], jj);
      if (lane == jj) rhs = xj;
      else if (lane < jj) rhs -= colv[jj] * xj;
    }
    if (ok) b[r] = rhs;
    __threadfence();
    if (lane == 0) publish(flags + q, epoch);
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

size_t chol_workspace_bytes(int64_t) { return 0; }

int chol_factor(hipStream_t s, int64_t m, double* K, int64_t ldK, int64_t* dinfo, void*) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(1), 0, s, dinfo, (int64_t)0);
  DNGD_LAUNCH_CHECK();
  for (int64_t j0 = 0; j0 < m; j0 += NB) {
    const int64_t rows = m - j0;
    const unsigned nblk = (unsigned)cdiv(rows, NB);
    hipLaunchKernelGGL(potrf_panel_kernel, dim3(nblk), dim3(64), 0, s, m, K, ldK, j0, dinfo);
    DNGD_LAUNCH_CHECK();
    const int64_t rest = rows - NB;
    if (rest > 0) {
      double* A21 = K + (j0 + NB) * ldK + j0;
      double* A22 = K + (j0 + NB) * ldK + j0 + NB;
      int rc = gemm_f64(s, GEMM_SYRK_LOWER, true, true, rest, rest, NB, -1.0, A21, ldK, A21, ldK,
                        1.0, A22, ldK);
      if (rc) return rc;
    }
  }
  return 0;
}

int64_t chol_solve_flag_count(int64_t m) { return 2 * cdiv(m, NB); }

int chol_solve(hipStream_t s, int64_t m, const double* L, int64_t ldL, double* b, unsigned* flags,
               unsigned* epoch, int* dstatus, double*) {
  const int64_t nblk = cdiv(m, NB);
  const unsigned e1 = ++(*epoch);
  hipLaunchKernelGGL(trsv_lower_kernel, dim3((unsigned)nblk), dim3(256), 0, s, m, L, ldL, b, flags,
                     e1, dstatus);
  DNGD_LAUNCH_CHECK();
  const unsigned e2 = ++(*epoch);
  hipLaunchKernelGGL(trsv_upper_kernel, dim3((unsigned)nblk), dim3(256), 0, s, m, L, ldL, b,
                     flags + nblk, e2, dstatus);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
