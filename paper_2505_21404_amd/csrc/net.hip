// tanh-MLP kernels on the jet-row layout: the residual map and its
// derivatives (Section 2.2), with input Laplacians in forward mode.
//
// A point's jet is its value, input gradient and input Laplacian; through an
// affine layer each channel is multiplied by W (the bias only enters the
// value), and through tanh:
//   a.v = s0,  a.g = s1 z.g,  a.l = s1 z.l + s2 |z.g|^2_lap
// with s_k the k-th derivative of tanh at z.v and |.|^2_lap summing the
// Laplacian coordinates only. The layer products run on the FP64 matrix
// cores (gemm_f64.hip); the kernels here are the per-(point, neuron)
// elementwise stages, the output row dots and the Jacobian row writer.
#include "common.h"

namespace dngd {

namespace {

struct Tanh {
  double s0, s1, s2, s3, s4;
  __device__ inline Tanh(double z, int order) {
    s0 = tanh(z);
    s1 = 1.0 - s0 * s0;
    s2 = -2.0 * s0 * s1;
    s3 = (order >= 3) ? s1 * (6.0 * s0 * s0 - 2.0) : 0.0;
    s4 = (order >= 4) ? 8.0 * s0 * s1 * (2.0 - 3.0 * s0 * s0) : 0.0;
  }
};

// point p -> (first jet row, channel count)
__device__ inline void point_rows(const RowMap& rm, int64_t p, int64_t& base, int& C) {
  if (p < rm.n_int) {
    base = p * rm.C_int;
    C = rm.C_int;
  } else {
    base = rm.R_int + (p - rm.n_int);
    C = 1;
  }
}

// residual index of component comp of point p (-1 if the point's class has
// fewer components): classes in order interior, boundary, initial, each
// point-major (a point's components are consecutive)
__device__ inline int64_t residual_row(const RowMap& rm, int64_t p, int comp) {
  if (p < rm.n_int) return comp < rm.r_int ? p * rm.r_int + comp : -1;
  if (p < rm.n_int + rm.n_bdy)
    return comp < rm.r_bdy ? rm.res_bdy0 + (p - rm.n_int) * rm.r_bdy + comp : -1;
  return comp == 0 ? rm.res_init0 + (p - rm.n_int - rm.n_bdy) : -1;
}

__global__ void input_layer_kernel(RowMap rm, const double* __restrict__ xi,
                                   const double* __restrict__ xb, const double* __restrict__ x0,
                                   double* __restrict__ A0) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const int d = rm.d_in;
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  const double* x;
  if (p < rm.n_int) x = xi + p * d;
  else if (p < rm.n_int + rm.n_bdy) x = xb + (p - rm.n_int) * d;
  else x = x0 + (p - rm.n_int - rm.n_bdy) * d;
  for (int k = 0; k < d; ++k) A0[base * d + k] = x[k];
  if (C > 1) {
    for (int c = 0; c < d; ++c)
      for (int k = 0; k < d; ++k) A0[(base + 1 + c) * d + k] = (c == k) ? 1.0 : 0.0;
    for (int k = 0; k < d; ++k) A0[(base + 1 + d) * d + k] = 0.0;
  }
}

// forward jet activation: Z.v += b; A = tanh-jet(Z)
__global__ __launch_bounds__(256) void bias_act_kernel(RowMap rm, int w, const double* __restrict__ b,
                                                       double* __restrict__ Z,
                                                       double* __restrict__ A) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= npts * w) return;
  const int64_t p = idx / w;
  const int o = (int)(idx % w);
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  double* z = Z + base * w + o;
  double* a = A + base * w + o;
  const double zv = z[0] + (b ? b[o] : 0.0);
  z[0] = zv;
  const Tanh s(zv, 2);
  a[0] = s.s0;
  if (C > 1) {
    const int d = rm.d_in;
    double gg = 0.0;
    for (int k = 0; k < d; ++k) {
      const double g = z[(int64_t)(1 + k) * w];
      if (k < rm.nlap) gg += g * g;
      a[(int64_t)(1 + k) * w] = s.s1 * g;
    }
    const double zl = z[(int64_t)(1 + d) * w];
    a[(int64_t)(1 + d) * w] = s.s1 * zl + s.s2 * gg;
  }
}

// adjoint of the jet activation: Zbar from Abar and Z (with bias)
__global__ __launch_bounds__(256) void act_adjoint_kernel(RowMap rm, int w,
                                                          const double* __restrict__ Z,
                                                          const double* __restrict__ Ab,
                                                          double* __restrict__ Zb) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= npts * w) return;
  const int64_t p = idx / w;
  const int o = (int)(idx % w);
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  const double* z = Z + base * w + o;
  const double* ab = Ab + base * w + o;
  double* zb = Zb + base * w + o;
  const Tanh s(z[0], 3);
  if (C == 1) {
    zb[0] = ab[0] * s.s1;
    return;
  }
  const int d = rm.d_in;
  const double abl = ab[(int64_t)(1 + d) * w];
  const double zl = z[(int64_t)(1 + d) * w];
  double gg = 0.0, ag = 0.0;
  for (int k = 0; k < d; ++k) {
    const double g = z[(int64_t)(1 + k) * w];
    const double agk = ab[(int64_t)(1 + k) * w];
    if (k < rm.nlap) gg += g * g;
    ag += agk * g;
    zb[(int64_t)(1 + k) * w] = s.s1 * agk + ((k < rm.nlap) ? 2.0 * s.s2 * abl * g : 0.0);
  }
  zb[0] = ab[0] * s.s1 + s.s2 * ag + abl * (s.s2 * zl + s.s3 * gg);
  zb[(int64_t)(1 + d) * w] = s.s1 * abl;
}

// out[row * nout + o] = X[row] . wv_o + beta * Y[row] . wv2_o for the nout rows
// wv_o = wv + o * w of the output layer's weights (one wave per jet row)
__global__ __launch_bounds__(256) void rowdot_kernel(int64_t R, int w, int nout,
                                                     const double* __restrict__ X,
                                                     const double* __restrict__ wv, double beta,
                                                     const double* __restrict__ Y,
                                                     const double* __restrict__ wv2,
                                                     double* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= R) return;
  for (int o = 0; o < nout; ++o) {
    const double* w1 = wv + (int64_t)o * w;
    const double* w2 = Y ? wv2 + (int64_t)o * w : nullptr;
    double s = 0.0;
    for (int k = lane; k < w; k += 64) {
      s += X[row * w + k] * w1[k];
      if (Y) s += beta * Y[row * w + k] * w2[k];
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) out[row * nout + o] = s;
  }
}

// interior operator on an output jet: -lap u (Poisson) or u_t - kappa lap u (heat)
__device__ inline double interior_op(const RowMap& rm, const double* U, int64_t base) {
  const double lap = U[base + 1 + rm.d_in];
  if (rm.pde == 0) return -lap;
  return U[base + rm.d_in] - rm.kappa * lap;  // channel 1 + (d_in - 1) is d/dt
}

__global__ void residual_kernel(RowMap rm, const double* __restrict__ U,
                                const double* __restrict__ bias_p, const double* __restrict__ f,
                                const double* __restrict__ g, const double* __restrict__ g0,
                                double* __restrict__ r) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double bias = bias_p ? bias_p[0] : 0.0;  // output bias: value channel only
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  double v;
  if (p < rm.n_int) {
    v = rm.c_int * (interior_op(rm, U, base) - (f ? f[p] : 0.0));
  } else if (p < rm.n_int + rm.n_bdy) {
    v = rm.c_bdy * (U[base] + bias - (g ? g[p - rm.n_int] : 0.0));
  } else {
    v = rm.c_init * (U[base] + bias - (g0 ? g0[p - rm.n_int - rm.n_bdy] : 0.0));
  }
  r[p] = v;
}

// per-row backward seeds: d r_p / d (output channel) times p_p (1 if p == null)
__global__ void seeds_kernel(RowMap rm, const double* __restrict__ pv, double* __restrict__ seed) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double s = pv ? pv[p] : 1.0;
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  if (p < rm.n_int) {
    for (int c = 0; c < C; ++c) seed[base + c] = 0.0;
    if (rm.pde == 0) {
      seed[base + 1 + rm.d_in] = -rm.c_int * s;
    } else {
      seed[base + rm.d_in] = rm.c_int * s;
      seed[base + 1 + rm.d_in] = -rm.kappa * rm.c_int * s;
    }
  } else if (p < rm.n_int + rm.n_bdy) {
    seed[base] = rm.c_bdy * s;
  } else {
    seed[base] = rm.c_init * s;
  }
}

// Abar of the last hidden layer: Ab[row][j] = sum_o seed[row][o] W_L[o][j]
__global__ void outer_seed_kernel(int64_t R, int w, int nout, const double* __restrict__ seed,
                                  const double* __restrict__ wL, double* __restrict__ Ab) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= R * w) return;
  const int64_t row = idx / w;
  const int j = (int)(idx % w);
  double a = 0.0;
  for (int o = 0; o < nout; ++o) a += seed[row * nout + o] * wL[(int64_t)o * w + j];
  Ab[idx] = a;
}

// ---------------------------------------------------------------------------
// Steady incompressible Navier-Stokes residuals (vector-valued classes). The
// network outputs (u, v, p); an interior point's four jet rows (value, d/dx,
// d/dy, Laplacian) each hold the three outputs, and its three residuals are
//   x-momentum  u u_x + v u_y + p_x - nu lap u
//   y-momentum  u v_x + v v_y + p_y - nu lap v
//   continuity  u_x + v_y
// (nu = rm.kappa). A boundary point's three residuals are its outputs against
// the prescribed values. Residual rows are point-major within a class.

struct NSCh {
  double u, v, p, ux, uy, vx, vy, px, py, lu, lv;
};

// the operator's inputs at an interior point; bias (may be null) enters the values
__device__ inline NSCh ns_channels(const double* __restrict__ U, int64_t base,
                                   const double* __restrict__ bias) {
  const double* r = U + base * 3;
  NSCh c;
  c.u = r[0] + (bias ? bias[0] : 0.0);
  c.v = r[1] + (bias ? bias[1] : 0.0);
  c.p = r[2] + (bias ? bias[2] : 0.0);
  c.ux = r[3];
  c.vx = r[4];
  c.px = r[5];
  c.uy = r[6];
  c.vy = r[7];
  c.py = r[8];
  c.lu = r[9];
  c.lv = r[10];
  return c;
}

// derivative of the operator at a in the direction b
__device__ inline void ns_linear(const NSCh& a, const NSCh& b, double nu, double out[3]) {
  out[0] = a.u * b.ux + b.u * a.ux + a.v * b.uy + b.v * a.uy + b.px - nu * b.lu;
  out[1] = a.u * b.vx + b.u * a.vx + a.v * b.vy + b.v * a.vy + b.py - nu * b.lv;
  out[2] = b.ux + b.vy;
}

__global__ void ns_residual_kernel(RowMap rm, const double* __restrict__ U,
                                   const double* __restrict__ bias, const double* __restrict__ f,
                                   const double* __restrict__ g, double* __restrict__ r) {
  const int64_t npts = rm.n_int + rm.n_bdy;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double nu = rm.kappa;
  if (p < rm.n_int) {
    const NSCh c = ns_channels(U, p * rm.C_int, bias);
    const double* fp = f ? f + p * 3 : nullptr;
    r[p * 3 + 0] = rm.c_int * (c.u * c.ux + c.v * c.uy + c.px - nu * c.lu - (fp ? fp[0] : 0.0));
    r[p * 3 + 1] = rm.c_int * (c.u * c.vx + c.v * c.vy + c.py - nu * c.lv - (fp ? fp[1] : 0.0));
    r[p * 3 + 2] = rm.c_int * (c.ux + c.vy - (fp ? fp[2] : 0.0));
  } else {
    const int64_t pb = p - rm.n_int;
    const double* u = U + (rm.R_int + pb) * 3;
    for (int o = 0; o < 3; ++o)
      r[rm.res_bdy0 + pb * 3 + o] =
          rm.c_bdy * (u[o] + (bias ? bias[o] : 0.0) - (g ? g[pb * 3 + o] : 0.0));
  }
}

// t-derivatives of the residual along theta + t dir from the output jets'
// t-derivatives U0 (+ b0), U1 (+ c1), U2: order 1 gives J dir = DN(U0)[U1];
// order 2 gives f_vv = DN(U0)[U2] + 2 B(U1, U1), B the operator's quadratic part
__global__ void ns_tangent_kernel(RowMap rm, const double* __restrict__ U0,
                                  const double* __restrict__ b0, const double* __restrict__ U1,
                                  const double* __restrict__ c1, const double* __restrict__ U2,
                                  int order, double* __restrict__ out) {
  const int64_t npts = rm.n_int + rm.n_bdy;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double nu = rm.kappa;
  if (p < rm.n_int) {
    const int64_t base = p * rm.C_int;
    const NSCh a = ns_channels(U0, base, b0);
    const NSCh b = ns_channels(U1, base, c1);
    double o3[3];
    if (order == 1) {
      ns_linear(a, b, nu, o3);
    } else {
      const NSCh d = ns_channels(U2, base, nullptr);
      ns_linear(a, d, nu, o3);
      o3[0] += 2.0 * (b.u * b.ux + b.v * b.uy);
      o3[1] += 2.0 * (b.u * b.vx + b.v * b.vy);
    }
    for (int k = 0; k < 3; ++k) out[p * 3 + k] = rm.c_int * o3[k];
  } else {
    const int64_t pb = p - rm.n_int;
    const int64_t row = (rm.R_int + pb) * 3;
    for (int o = 0; o < 3; ++o) {
      const double x = (order == 1) ? U1[row + o] + (c1 ? c1[o] : 0.0) : U2[row + o];
      out[rm.res_bdy0 + pb * 3 + o] = rm.c_bdy * x;
    }
  }
}

// Reverse-pass seeds: d/dU of sum_k w_k r_k for each point's residuals, with
// w = pw (the weights of a vector-Jacobian product) or w_k = [k == comp] (one
// Jacobian row per point). seed is R x 3 like U.
__global__ void ns_seeds_kernel(RowMap rm, const double* __restrict__ U,
                                const double* __restrict__ bias, const double* __restrict__ pw,
                                int comp, double* __restrict__ seed) {
  const int64_t npts = rm.n_int + rm.n_bdy;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double nu = rm.kappa;
  if (p < rm.n_int) {
    const int64_t base = p * rm.C_int;
    const NSCh a = ns_channels(U, base, bias);
    double w[3];
    for (int k = 0; k < 3; ++k)
      w[k] = rm.c_int * (pw ? pw[p * 3 + k] : (k == comp ? 1.0 : 0.0));
    double* s0 = seed + base * 3;  // value row, then d/dx, d/dy, Laplacian rows
    s0[0] = w[0] * a.ux + w[1] * a.vx;
    s0[1] = w[0] * a.uy + w[1] * a.vy;
    s0[2] = 0.0;
    s0[3] = w[0] * a.u + w[2];
    s0[4] = w[1] * a.u;
    s0[5] = w[0];
    s0[6] = w[0] * a.v;
    s0[7] = w[1] * a.v + w[2];
    s0[8] = w[1];
    s0[9] = -nu * w[0];
    s0[10] = -nu * w[1];
    s0[11] = 0.0;
  } else {
    const int64_t pb = p - rm.n_int;
    double* s0 = seed + (rm.R_int + pb) * 3;
    for (int o = 0; o < 3; ++o)
      s0[o] = rm.c_bdy * (pw ? pw[rm.res_bdy0 + pb * 3 + o] : (o == comp ? 1.0 : 0.0));
  }
}

// ---------------------------------------------------------------------------
// Jacobian rows: J[p][W_l[o][k]] = sum_c Zbar_l[p,c][o] A_{l-1}[p,c][k],
// J[p][b_l[o]] = Zbar_l[p,value][o]. One workgroup per point; a thread owns
// 4 consecutive inputs k (its A values stay in registers) and walks the
// outputs o, with the point's adjoints staged in LDS chunk by chunk.

struct JacLayers {
  const double* A[kMaxLayers];     // A_{l-1}: R x w_{l-1}
  const double* Zb[kMaxLayers];    // Zbar_l:  R x w_l  (seed for the output layer)
  int win[kMaxLayers], wout[kMaxLayers];
  int64_t woff[kMaxLayers], boff[kMaxLayers];
  int L;
};

constexpr int JOC = 256;  // outputs per staged adjoint chunk

// FP32 J rows are written once and read back only after the whole matrix
// (far larger than the caches) is done: nontemporal stores, each wave's one
// contiguous KB. (The FP64 rows' two 16-byte halves per lane leave gaps in
// each store instruction; there the cached stores, merged in L2, are faster.)
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
__device__ inline void store4(float* p, const float (&v)[4]) {
  __builtin_nontemporal_store(f32x4_nt{v[0], v[1], v[2], v[3]}, reinterpret_cast<f32x4_nt*>(p));
}
__device__ inline void store4(double* p, const double (&v)[4]) {
  reinterpret_cast<double2*>(p)[0] = double2{v[0], v[1]};
  reinterpret_cast<double2*>(p)[1] = double2{v[2], v[3]};
}

template <typename T>
__global__ __launch_bounds__(256) void jacobian_rows_kernel(RowMap rm, JacLayers jl, T* __restrict__ J,
                                                            int64_t ldJ, int64_t n,
                                                            double* __restrict__ rownorm2,
                                                            const int64_t* __restrict__ pidx,
                                                            int comp) {
  __shared__ double red[4];
  const int64_t p = pidx ? pidx[blockIdx.x] : (int64_t)blockIdx.x;
  // the J row of residual component `comp` of point p (row q of a gathered
  // set when pidx is given); points without that component have no row
  int64_t jrow = blockIdx.x;
  if (!pidx) {
    jrow = residual_row(rm, p, comp);
    if (jrow < 0) return;  // uniform over the workgroup
  }
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  T* row = J + jrow * ldJ;
  const int t = threadIdx.x;
  double ss = 0.0;
  // the point's adjoints of a chunk of JOC outputs, staged in LDS (every
  // thread of a row group reads the same entries)
  __shared__ double zs[kMaxChannels][JOC];
  for (int l = 0; l < jl.L; ++l) {
    const int win = jl.win[l], wout = jl.wout[l];
    const double* A = jl.A[l] + base * win;
    const double* Zb = jl.Zb[l] + base * wout;
    const int nq = (win + 3) >> 2;
    int tpr = 1;
    while (tpr < nq && tpr < 256) tpr <<= 1;
    const int rpp = 256 / tpr;
    T* W = row + jl.woff[l];
    // 4 consecutive outputs per thread can be stored as one vector
    const bool vec = (win % 4 == 0) && (jl.woff[l] % 4 == 0);
    for (int q0 = 0; q0 < nq; q0 += tpr) {
      const int q = q0 + (t % tpr);
      const bool qok = q < nq;
      double a[kMaxChannels][4];
#pragma unroll
      for (int c = 0; c < kMaxChannels; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = 4 * q + e;
          a[c][e] = (qok && c < C && k < win) ? A[(int64_t)c * win + k] : 0.0;
        }
      for (int o0 = 0; o0 < wout; o0 += JOC) {
        const int oc = min(JOC, wout - o0);
        __syncthreads();
        for (int e = t; e < C * JOC; e += 256) {
          const int c = e / JOC, o = e % JOC;
          if (o < oc) zs[c][o] = Zb[(int64_t)c * wout + o0 + o];
        }
        __syncthreads();
        if (!qok) continue;
        for (int o = t / tpr; o < oc; o += rpp) {
          double v[4] = {0, 0, 0, 0};
#pragma unroll
          for (int c = 0; c < kMaxChannels; ++c) {
            if (c < C) {
              const double zc = zs[c][o];
#pragma unroll
              for (int e = 0; e < 4; ++e) v[e] += zc * a[c][e];
            }
          }
          T* w = W + (int64_t)(o0 + o) * win + 4 * q;
          T tv[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            tv[e] = (T)v[e];
            if (4 * q + e < win) {
              const double vr = (double)tv[e];
              ss += vr * vr;
            }
          }
          if (vec) {
            store4(w, tv);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (4 * q + e < win) w[e] = tv[e];
          }
        }
      }
    }
    T* B = row + jl.boff[l];
    for (int o = t; o < wout; o += 256) {
      const double v = Zb[o];
      B[o] = (T)v;
      const double vr = (double)(T)v;
      ss += vr * vr;
    }
  }
  for (int64_t k = n + t; k < ldJ; k += 256) row[k] = (T)0;
  if (rownorm2) {
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    if ((t & 63) == 0) red[t >> 6] = ss;
    __syncthreads();
    if (t == 0) rownorm2[jrow] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// t-tangent streams (f_vv and J u): given Z0 and the layer products
// Z1 = W a1 + V a0 (+ c on the value channel, added here) and Z2 = W a2 + 2 V a1,
//   a1 = s'(z0) z1,  a2 = s'(z0) z2 + s''(z0) z1 z1
// where s'(z0), s''(z0) are jets (function rule) and products follow the
// jet product rule.

template <int D>
struct Jet {
  double v, g[D], l;
};

template <int D>
__device__ inline void jet_load(Jet<D>& j, const double* z, int64_t w, int C) {
  j.v = z[0];
#pragma unroll
  for (int k = 0; k < D; ++k) j.g[k] = (C > 1) ? z[(int64_t)(1 + k) * w] : 0.0;
  j.l = (C > 1) ? z[(int64_t)(1 + D) * w] : 0.0;
}
template <int D>
__device__ inline void jet_store(const Jet<D>& j, double* a, int64_t w, int C) {
  a[0] = j.v;
  if (C > 1) {
#pragma unroll
    for (int k = 0; k < D; ++k) a[(int64_t)(1 + k) * w] = j.g[k];
    a[(int64_t)(1 + D) * w] = j.l;
  }
}
template <int D>
__device__ inline Jet<D> jet_mul(const Jet<D>& p, const Jet<D>& q, int nlap) {
  Jet<D> r;
  r.v = p.v * q.v;
  double cross = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    r.g[k] = p.v * q.g[k] + q.v * p.g[k];
    if (k < nlap) cross += p.g[k] * q.g[k];
  }
  r.l = p.v * q.l + q.v * p.l + 2.0 * cross;
  return r;
}
// jet of phi(z) given phi(z.v), phi'(z.v), phi''(z.v)
template <int D>
__device__ inline Jet<D> jet_fn(double f0, double f1, double f2, const Jet<D>& z, int nlap) {
  Jet<D> r;
  r.v = f0;
  double gg = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    r.g[k] = f1 * z.g[k];
    if (k < nlap) gg += z.g[k] * z.g[k];
  }
  r.l = f1 * z.l + f2 * gg;
  return r;
}

// Boundary / initial rows carry only the value channel; their gradient and
// Laplacian entries are zero in the jets above, so the same formulas apply.
template <int D>
__global__ __launch_bounds__(256) void tangent_act_kernel(RowMap rm, int w, const double* __restrict__ b1,
                                                          const double* __restrict__ Z0,
                                                          double* __restrict__ Z1,
                                                          const double* __restrict__ Z2,
                                                          double* __restrict__ A1,
                                                          double* __restrict__ A2, int order) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= npts * w) return;
  const int64_t p = idx / w;
  const int o = (int)(idx % w);
  int64_t base;
  int C;
  point_rows(rm, p, base, C);
  const int nl = rm.nlap;
  const int64_t off = base * w + o;
  Jet<D> z0, z1;
  jet_load(z0, Z0 + off, w, C);
  jet_load(z1, Z1 + off, w, C);
  if (b1) z1.v += b1[o];
  const Tanh s(z0.v, order >= 2 ? 4 : 3);
  const Jet<D> P = jet_fn(s.s1, s.s2, s.s3, z0, nl);  // jet of tanh'(z0)
  const Jet<D> a1 = jet_mul(P, z1, nl);
  jet_store(a1, A1 + off, w, C);
  if (order >= 2) {
    Jet<D> z2;
    jet_load(z2, Z2 + off, w, C);
    const Jet<D> Q = jet_fn(s.s2, s.s3, s.s4, z0, nl);  // jet of tanh''(z0)
    const Jet<D> t1 = jet_mul(P, z2, nl);
    const Jet<D> t2 = jet_mul(Q, jet_mul(z1, z1, nl), nl);
    Jet<D> a2;
    a2.v = t1.v + t2.v;
#pragma unroll
    for (int k = 0; k < D; ++k) a2.g[k] = t1.g[k] + t2.g[k];
    a2.l = t1.l + t2.l;
    jet_store(a2, A2 + off, w, C);
  }
}

// sum over the value rows of Zbar (bias gradients), deterministic 2 passes
__global__ __launch_bounds__(256) void colsum_partial_kernel(RowMap rm, int w,
                                                             const double* __restrict__ Zb,
                                                             int64_t pts_per,
                                                             double* __restrict__ part) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= w) return;
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int64_t p0 = (int64_t)blockIdx.y * pts_per;
  const int64_t p1 = min(npts, p0 + pts_per);
  double s = 0.0;
  for (int64_t p = p0; p < p1; ++p) {
    int64_t base;
    int C;
    point_rows(rm, p, base, C);
    s += Zb[base * w + o];
  }
  part[(int64_t)blockIdx.y * w + o] = s;
}

__global__ void colsum_reduce_kernel(int w, int S, const double* __restrict__ part,
                                     double* __restrict__ out) {
  const int o = blockIdx.x * 256 + threadIdx.x;
  if (o >= w) return;
  double s = 0.0;
  for (int k = 0; k < S; ++k) s += part[(int64_t)k * w + o];
  out[o] = s;
}

// ---------------------------------------------------------------------------
// Landmark columns of K without forming J (Nystrom construction): for an
// affine layer with input activations H (jet rows x w_in) and output
// adjoints G (jet rows x w_out), the layer's part of J_i . J_j is
//   sum_{c in rows(i), c' in rows(j)} (G_c . G_c') (H_c . H_c') + G_i0 . G_j0,
// the second term from the bias (value rows only). G G_I^T and H H_I^T are
// FP64 GEMMs; this kernel gathers the landmark rows and combines.

__global__ void gather_rows_kernel(int64_t nrows, int w, const int64_t* __restrict__ rows,
                                   const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nrows * w) return;
  const int64_t r = e / w, k = e % w;
  dst[e] = src[rows[r] * w + k];
}

// Mt[q][p] (=, or += when accumulate) for points p in [p0, p0 + np) and all
// landmarks q; Gp, Hp hold the rows of the chunk starting at jet row row0,
// one column per landmark jet row (ld = total landmark rows).
// lower != 0 (all points are landmarks, q = point q): write K[p0 + i][q]
// (row-major, ldM) for q <= p0 + i only, the lower triangle.
__global__ void nystrom_combine_kernel(RowMap rm, int64_t p0, int64_t np, int64_t row0,
                                       const double* __restrict__ Gp,
                                       const double* __restrict__ Hp, int64_t ld, int64_t ell,
                                       const int64_t* __restrict__ qoff, double* __restrict__ Mt,
                                       int64_t ldM, int accumulate, int lower) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= np * ell) return;
  const int64_t i = e / ell, q = e % ell;  // consecutive threads: consecutive landmarks
  if (lower && q > p0 + i) return;
  int64_t base;
  int C;
  point_rows(rm, p0 + i, base, C);
  const int64_t rb = base - row0;
  const int64_t o = qoff[q], Cq = qoff[q + 1] - o;
  double sum = Gp[rb * ld + o];  // bias: value rows
  for (int c = 0; c < C; ++c) {
    const double* g = Gp + (rb + c) * ld + o;
    const double* h = Hp + (rb + c) * ld + o;
    for (int64_t c2 = 0; c2 < Cq; ++c2) sum += g[c2] * h[c2];
  }
  double* out = lower ? Mt + (p0 + i) * ldM + q : Mt + q * ldM + p0 + i;
  *out = accumulate ? *out + sum : sum;
}

}  // namespace

RowMap row_map(const Geometry& g) {
  RowMap r;
  r.n_int = g.n_int;
  r.n_bdy = g.n_bdy;
  r.n_init = g.n_init;
  r.R_int = g.R_int;
  r.C_int = g.C_int;
  r.d_in = g.d_in;
  r.nlap = g.nlap;
  r.pde = g.pde;
  r.kappa = g.kappa;
  r.c_int = g.c_int;
  r.c_bdy = g.c_bdy;
  r.c_init = g.c_init;
  r.d_out = g.widths[g.L];
  r.r_int = g.r_int;
  r.r_bdy = g.r_bdy;
  r.res_bdy0 = g.n_int * g.r_int;
  r.res_init0 = r.res_bdy0 + g.n_bdy * g.r_bdy;
  return r;
}

static inline unsigned blocks_for(int64_t n, int bs = 256) { return (unsigned)cdiv(n, bs); }

int net_input_layer(hipStream_t s, const RowMap& rm, const double* xi, const double* xb,
                    const double* x0, double* A0, int) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  hipLaunchKernelGGL(input_layer_kernel, dim3(blocks_for(npts, 128)), dim3(128), 0, s, rm, xi, xb,
                     x0, A0);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_bias_act(hipStream_t s, const RowMap& rm, int w, const double* b, double* Z, double* A) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for(npts * w)), dim3(256), 0, s, rm, w, b, Z, A);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_act_adjoint(hipStream_t s, const RowMap& rm, int w, const double* Z, const double* Ab,
                    double* Zb) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  hipLaunchKernelGGL(act_adjoint_kernel, dim3(blocks_for(npts * w)), dim3(256), 0, s, rm, w, Z, Ab,
                     Zb);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_rowdot(hipStream_t s, int64_t R, int w, int nout, const double* X, const double* wv,
               double beta, const double* Y, const double* wv2, double* out) {
  hipLaunchKernelGGL(rowdot_kernel, dim3(blocks_for(R, 4)), dim3(256), 0, s, R, w, nout, X, wv,
                     beta, Y, wv2, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_residual(hipStream_t s, const RowMap& rm, const double* U, const double* bias,
                 const double* f, const double* g, const double* g0, double* r) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  if (rm.pde == kNavierStokes) {
    hipLaunchKernelGGL(ns_residual_kernel, dim3(blocks_for(npts)), dim3(256), 0, s, rm, U, bias, f,
                       g, r);
    DNGD_LAUNCH_CHECK();
    return 0;
  }
  hipLaunchKernelGGL(residual_kernel, dim3(blocks_for(npts)), dim3(256), 0, s, rm, U, bias, f, g,
                     g0, r);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_linear_residual(hipStream_t s, const RowMap& rm, const double* U, const double* bias,
                        double* out) {
  return net_residual(s, rm, U, bias, nullptr, nullptr, nullptr, out);
}

int net_seeds(hipStream_t s, const RowMap& rm, const double* U, const double* bias,
              const double* p, int comp, double* seed) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  if (rm.pde == kNavierStokes) {
    hipLaunchKernelGGL(ns_seeds_kernel, dim3(blocks_for(npts)), dim3(256), 0, s, rm, U, bias, p,
                       comp, seed);
    DNGD_LAUNCH_CHECK();
    return 0;
  }
  hipLaunchKernelGGL(seeds_kernel, dim3(blocks_for(npts)), dim3(256), 0, s, rm, p, seed);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_outer_seed(hipStream_t s, int64_t R, int w, int nout, const double* seed,
                   const double* wL, double* Ab) {
  hipLaunchKernelGGL(outer_seed_kernel, dim3(blocks_for(R * w)), dim3(256), 0, s, R, w, nout, seed,
                     wL, Ab);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_jacobian_rows(hipStream_t s, const Geometry& g, const RowMap& rm, const double* const* A,
                      const double* const* Zb, const double* seed, void* J, int64_t ldJ,
                      int j_dtype, double* rownorm2, const int64_t* pidx, int64_t nrows,
                      int comp) {
  JacLayers jl;
  jl.L = g.L;
  for (int l = 0; l < g.L; ++l) {
    jl.A[l] = A[l];
    jl.Zb[l] = (l == g.L - 1) ? seed : Zb[l];
    jl.win[l] = g.widths[l];
    jl.wout[l] = g.widths[l + 1];
    jl.woff[l] = g.w_off[l];
    jl.boff[l] = g.b_off[l];
  }
  dim3 grid((unsigned)(pidx ? nrows : g.n_int + g.n_bdy + g.n_init));
  if (grid.x == 0) return 0;
  if (j_dtype == 0)
    hipLaunchKernelGGL(jacobian_rows_kernel<double>, grid, dim3(256), 0, s, rm, jl,
                       static_cast<double*>(J), ldJ, g.n, rownorm2, pidx, comp);
  else
    hipLaunchKernelGGL(jacobian_rows_kernel<float>, grid, dim3(256), 0, s, rm, jl,
                       static_cast<float*>(J), ldJ, g.n, rownorm2, pidx, comp);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_ns_tangent(hipStream_t s, const RowMap& rm, const double* U0, const double* b0,
                   const double* U1, const double* c1, const double* U2, int order, double* out) {
  const int64_t npts = rm.n_int + rm.n_bdy;
  hipLaunchKernelGGL(ns_tangent_kernel, dim3(blocks_for(npts)), dim3(256), 0, s, rm, U0, b0, U1, c1,
                     U2, order, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_tangent_act(hipStream_t s, const RowMap& rm, int w, const double* b1, const double* Z0,
                    double* Z1, double* Z2, double* A1, double* A2, int order) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const dim3 grid(blocks_for(npts * w));
  switch (rm.d_in) {
#define DNGD_TANGENT_CASE(DV)                                                                  \
  case DV:                                                                                    \
    hipLaunchKernelGGL(tangent_act_kernel<DV>, grid, dim3(256), 0, s, rm, w, b1, Z0, Z1, Z2, A1, \
                       A2, order);                                                            \
    break;
    DNGD_TANGENT_CASE(1)
    DNGD_TANGENT_CASE(2)
    DNGD_TANGENT_CASE(3)
    DNGD_TANGENT_CASE(4)
    DNGD_TANGENT_CASE(5)
    DNGD_TANGENT_CASE(6)
    DNGD_TANGENT_CASE(7)
    DNGD_TANGENT_CASE(8)
#undef DNGD_TANGENT_CASE
    default:
      set_error("tangent: d_in %d unsupported", rm.d_in);
      return -1;
  }
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_colsum_value_rows(hipStream_t s, const RowMap& rm, int w, const double* Zb, double* out,
                          double* work) {
  const int64_t npts = rm.n_int + rm.n_bdy + rm.n_init;
  const int S = (int)std::min<int64_t>(64, std::max<int64_t>(1, cdiv(npts, 256)));
  const int64_t per = cdiv(npts, S);
  hipLaunchKernelGGL(colsum_partial_kernel, dim3(blocks_for(w), S), dim3(256), 0, s, rm, w, Zb,
                     per, work);
  DNGD_LAUNCH_CHECK();
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3(blocks_for(w)), dim3(256), 0, s, w, S, work, out);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd

namespace dngd {

int net_gather_rows(hipStream_t s, int64_t nrows, int w, const int64_t* rows, const double* src,
                    double* dst) {
  if (nrows * w <= 0) return 0;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(nrows * w)), dim3(256), 0, s, nrows, w,
                     rows, src, dst);
  DNGD_LAUNCH_CHECK();
  return 0;
}

int net_nystrom_combine(hipStream_t s, const RowMap& rm, int64_t p0, int64_t np, int64_t row0,
                        const double* Gp, const double* Hp, int64_t ld, int64_t ell,
                        const int64_t* qoff, double* Mt, int64_t ldM, int accumulate,
                        int lower) {
  if (np * ell <= 0) return 0;
  hipLaunchKernelGGL(nystrom_combine_kernel, dim3(blocks_for(np * ell)), dim3(256), 0, s, rm, p0,
                     np, row0, Gp, Hp, ld, ell, qoff, Mt, ldM, accumulate, lower);
  DNGD_LAUNCH_CHECK();
  return 0;
}

}  // namespace dngd
