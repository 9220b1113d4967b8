// C ABI of libdngd (declared in include/dngd.h): problem handles, workspace
// management and the D-NGD step pipelines built from the kernels in this
// directory.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <vector>

#include "../../include/dngd.h"
#include "common.h"

namespace dngd {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return (e == hipErrorOutOfMemory) ? DNGD_ENOMEM : DNGD_EHIP;
}

}  // namespace dngd

using namespace dngd;

// ---------------------------------------------------------------------------
// problem handle

// Nystrom preconditioner in Woodbury form (see dngd_nystrom_pcg)
struct Precond {
  double* Mt = nullptr;  // ell x m   (L_I^{-1} K_{I,:})
  double* G = nullptr;   // ell x ell (lambda I + Mt Mt^T, Cholesky factor)
  double* tl = nullptr;    // ell scratch vector
  double* Gaux = nullptr;  // solve workspace for chol(G)
  int64_t ldM = 0;
  double delta = 0;
  int64_t ell = 0;
  double lambda = 0;
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct dngd_problem {
  Geometry g;
  RowMap rm;
  int device = 0;
  std::vector<void*> owned;  // freed at destroy
  double *x_int = nullptr, *x_bdy = nullptr, *x_init = nullptr;
  double *f_int = nullptr, *g_bdy = nullptr, *g_init = nullptr;
  // forward activations (hidden layers h = 0..L-2)
  double* A0 = nullptr;
  double* Z[kMaxLayers] = {nullptr};
  double* A[kMaxLayers] = {nullptr};
  double* Zb[kMaxLayers] = {nullptr};
  double* Ab[2] = {nullptr, nullptr};
  double* WT = nullptr;  // one hidden layer's weights transposed (backward products)
  double* seed = nullptr;  // R x d_out reverse-pass seeds on the output jets
  double* U = nullptr;     // R x d_out output jets of the last forward pass
  double *U1 = nullptr, *U2 = nullptr;  // their t-derivatives (Navier-Stokes tangents)
  // tangent streams (lazy)
  double *Z1 = nullptr, *Z2 = nullptr, *A1[2] = {nullptr, nullptr}, *A2[2] = {nullptr, nullptr};
  // step / solver workspace (lazy, grown on demand)
  DevBuf J, Jt, K, vecs, work, gram_work, solve_aux, small, iter;
  DevBuf lp;  // buffers of the bf16 kernel-vector product (LowpBufs carves them)
  int J_dtype = -1;
  int64_t ldJ = 0, ldK = 0;
  hipEvent_t ev[10] = {nullptr};
  // side stream and events of the factorisation's look-ahead
  hipStream_t side = nullptr;
  hipEvent_t cev[2] = {nullptr, nullptr};
  // Nystrom preconditioner of the last PCG step (in K's buffer), its age in
  // steps; -1 when K's buffer holds something else
  Precond pc;
  int pc_age = -1;
  // Gram tier that the adaptive mixed step last escalated to, with the
  // damping and system (dual or primal) it escalated at: a later step on the
  // same system with damping at or below starts at that tier
  int gram_hint = 0;
  double gram_hint_lambda = 0.0;
  bool gram_hint_primal = false;
  // Device memory comes from the stream-ordered allocator on the stream of
  // the call in progress (astream), so that growing a buffer mid-job or
  // destroying a handle never waits for the whole device (other jobs'
  // queued work); last_use is recorded on each call's stream.
  hipStream_t astream = nullptr;
  hipEvent_t last_use = nullptr;
  bool last_use_valid = false;
  // pinned host staging of the small device-to-host readbacks (read_back)
  void* hstage = nullptr;
};

namespace {

int64_t act_bytes(const Geometry& g) { return g.R * (int64_t)g.max_width * (int64_t)sizeof(double); }
size_t wt_bytes(const Geometry& g) { return (size_t)g.max_width * g.max_width * sizeof(double); }

int dmalloc(dngd_problem* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMallocAsync(p, bytes, h->astream);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_fail(e, "hipMallocAsync", __FILE__, __LINE__);
  }
  h->owned.push_back(*p);
  return 0;
}

// Readback of several small device arrays with one wait: the copies land in
// the handle's pinned staging buffer (a copy into pageable memory holds the
// calling thread until it completes, one round trip per copy) and are moved
// to their destinations after the stream has been waited for.
constexpr size_t kHostStageBytes = 1024;
struct Readback {
  void* dst;
  const void* src;
  size_t bytes;
};

int read_back(dngd_problem* h, hipStream_t s, std::initializer_list<Readback> items) {
  char* stage = static_cast<char*>(h->hstage);
  size_t off = 0;
  for (const Readback& it : items) {
    DNGD_REQUIRE(off + it.bytes <= kHostStageBytes, "read_back: %zu bytes exceed the stage",
                 off + it.bytes);
    if (it.bytes) DNGD_HIP(hipMemcpyAsync(stage + off, it.src, it.bytes, hipMemcpyDeviceToHost, s));
    off += (it.bytes + 7) & ~size_t(7);
  }
  DNGD_HIP(hipStreamSynchronize(s));
  off = 0;
  for (const Readback& it : items) {
    if (it.bytes) std::memcpy(it.dst, stage + off, it.bytes);
    off += (it.bytes + 7) & ~size_t(7);
  }
  return 0;
}

int ensure(dngd_problem* h, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return 0;
  if (b.p) {
    for (auto& q : h->owned)
      if (q == b.p) q = nullptr;
    DNGD_HIP(hipFreeAsync(b.p, h->astream));  // after the work already queued on the stream
    b.p = nullptr;
    b.bytes = 0;
  }
  int rc = dmalloc(h, &b.p, bytes);
  if (rc) return rc;
  b.bytes = bytes;
  return 0;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// Every entry point that takes a handle and a stream opens one: allocations
// of the call go to that stream, and the stream's last use of the handle is
// recorded for dngd_problem_destroy.
struct CallScope {
  dngd_problem* h;
  hipStream_t s;
  CallScope(dngd_problem* h_, hipStream_t s_) : h(h_), s(s_) { h->astream = s; }
  ~CallScope() {
    if (h->last_use && hipEventRecord(h->last_use, s) == hipSuccess) h->last_use_valid = true;
  }
};

const double* Wp(const dngd_problem* h, const double* th, int l) { return th + h->g.w_off[l]; }
const double* Bp(const dngd_problem* h, const double* th, int l) { return th + h->g.b_off[l]; }

// activation input of affine layer l
const double* act_in(const dngd_problem* h, int l) { return l == 0 ? h->A0 : h->A[l - 1]; }

// Forward pass on jets: activations of all hidden layers, output rows U, residual r.
int forward(dngd_problem* h, const double* theta, double* r, hipStream_t s) {
  const Geometry& g = h->g;
  int rc = net_input_layer(s, h->rm, h->x_int, h->x_bdy, h->x_init, h->A0, g.d_in);
  if (rc) return rc;
  for (int l = 0; l < g.L - 1; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    rc = gemm_f64(s, GEMM_FULL, true, true, g.R, wout, win, 1.0, act_in(h, l), win, Wp(h, theta, l),
                  win, 0.0, h->Z[l], wout);
    if (rc) return rc;
    rc = net_bias_act(s, h->rm, wout, Bp(h, theta, l), h->Z[l], h->A[l]);
    if (rc) return rc;
  }
  const int l = g.L - 1;
  rc = net_rowdot(s, g.R, g.widths[l], g.d_out, act_in(h, l), Wp(h, theta, l), 0.0, nullptr,
                  nullptr, h->U);
  if (rc) return rc;
  if (r) rc = net_residual(s, h->rm, h->U, Bp(h, theta, l), h->f_int, h->g_bdy, h->g_init, r);
  return rc;
}

// Backward pass from per-residual weights p (null = the Jacobian rows of
// residual component comp of every point): fills seed and Zb[h] (adjoints of
// every hidden pre-activation). Requires forward() at theta.
int backward(dngd_problem* h, const double* theta, const double* p, hipStream_t s, int comp = 0) {
  const Geometry& g = h->g;
  int rc = net_seeds(s, h->rm, h->U, Bp(h, theta, g.L - 1), p, comp, h->seed);
  if (rc) return rc;
  if (g.L == 1) return 0;
  int cur = 0;
  rc = net_outer_seed(s, g.R, g.widths[g.L - 1], g.d_out, h->seed, Wp(h, theta, g.L - 1),
                      h->Ab[cur]);
  if (rc) return rc;
  for (int hl = g.L - 2; hl >= 0; --hl) {
    const int w = g.widths[hl + 1];
    rc = net_act_adjoint(s, h->rm, w, h->Z[hl], h->Ab[cur], h->Zb[hl]);
    if (rc) return rc;
    if (hl > 0) {
      const int win = g.widths[hl];
      // Abar_{hl-1} = Zb[hl] W_hl : (R x w) (w x win), with W_hl transposed
      // first so that both operands run along K (the faster product kernel)
      rc = transpose_rm(s, w, win, Wp(h, theta, hl), win, 0, h->WT, w);
      if (rc) return rc;
      rc = gemm_f64(s, GEMM_FULL, true, true, g.R, win, w, 1.0, h->Zb[hl], w, h->WT, w, 0.0,
                    h->Ab[cur ^ 1], win);
      if (rc) return rc;
      cur ^= 1;
    }
  }
  return 0;
}

int write_jacobian(dngd_problem* h, void* J, int64_t ldJ, int j_dtype, double* rownorm2,
                   hipStream_t s, const int64_t* pidx = nullptr, int64_t nrows = 0,
                   int comp = 0) {
  const Geometry& g = h->g;
  const double* A[kMaxLayers];
  const double* Zb[kMaxLayers];
  for (int l = 0; l < g.L; ++l) {
    A[l] = act_in(h, l);
    Zb[l] = (l < g.L - 1) ? h->Zb[l] : h->seed;
  }
  return net_jacobian_rows(s, g, h->rm, A, Zb, h->seed, J, ldJ, j_dtype, rownorm2, pidx, nrows,
                           comp);
}

// Every row of J (and its squared norm): one backward pass per residual
// component of a point (the d x d blocks of vector-valued classes), each
// writing its component's rows. Requires forward() at theta.
int jacobian_all(dngd_problem* h, const double* theta, void* J, int64_t ldJ, int j_dtype,
                 double* rownorm2, hipStream_t s) {
  const int ncomp = std::max(h->g.r_int, h->g.r_bdy);
  for (int c = 0; c < ncomp; ++c) {
    int rc = backward(h, theta, nullptr, s, c);
    if (!rc) rc = write_jacobian(h, J, ldJ, j_dtype, rownorm2, s, nullptr, 0, c);
    if (rc) return rc;
  }
  return 0;
}

int ensure_tangent(dngd_problem* h) {
  if (h->Z1) return 0;
  const size_t b = act_bytes(h->g);
  int rc = 0;
  rc |= dmalloc(h, (void**)&h->Z1, b);
  rc |= dmalloc(h, (void**)&h->Z2, b);
  rc |= dmalloc(h, (void**)&h->A1[0], b);
  rc |= dmalloc(h, (void**)&h->A1[1], b);
  rc |= dmalloc(h, (void**)&h->A2[0], b);
  rc |= dmalloc(h, (void**)&h->A2[1], b);
  if (h->g.pde == kNavierStokes) {
    rc |= dmalloc(h, (void**)&h->U1, (size_t)h->g.R * h->g.d_out * sizeof(double));
    rc |= dmalloc(h, (void**)&h->U2, (size_t)h->g.R * h->g.d_out * sizeof(double));
  }
  return rc ? DNGD_ENOMEM : 0;
}

// Forward t-tangent streams along direction dir (requires forward() at theta).
// order 1: out = J dir.  order 2: out = d^2/dt^2 r(theta + t dir).
int tangent(dngd_problem* h, const double* theta, const double* dir, int order, double* out,
            hipStream_t s, bool f32 = false) {
  const Geometry& g = h->g;
  int rc = ensure_tangent(h);
  if (rc) return rc;
  int cur = 0;
  const double* a1p = nullptr;  // tangent activations of the previous layer (null = 0)
  const double* a2p = nullptr;
  for (int l = 0; l < g.L - 1; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    const double* a0 = act_in(h, l);
    if (f32 && win >= 16) {
      // FP32 matrix-core products, each tangent order one launch:
      // Z1 = a0 V^T (+ a1 W^T), Z2 = a2 W^T + 2 a1 V^T
      const int64_t ld[2] = {win, win}, kk[2] = {win, win};
      const double one2[2] = {1.0, 1.0}, z2a[2] = {1.0, 2.0};
      const double* A1[2] = {a0, a1p};
      const double* B1[2] = {Wp(h, dir, l), Wp(h, theta, l)};
      rc = gemm_f32_nt(s, g.R, wout, a1p ? 2 : 1, A1, ld, B1, ld, kk, one2, 0.0, h->Z1, wout);
      if (rc) return rc;
      if (order >= 2) {
        if (a1p) {
          const double* A2[2] = {a2p, a1p};
          const double* B2[2] = {Wp(h, theta, l), Wp(h, dir, l)};
          rc = gemm_f32_nt(s, g.R, wout, 2, A2, ld, B2, ld, kk, z2a, 0.0, h->Z2, wout);
        } else {
          rc = fill(s, g.R * wout, 0.0, h->Z2);
        }
        if (rc) return rc;
      }
      rc = net_tangent_act(s, h->rm, wout, Bp(h, dir, l), h->Z[l], h->Z1, h->Z2, h->A1[cur],
                           h->A2[cur], order);
      if (rc) return rc;
      a1p = h->A1[cur];
      a2p = h->A2[cur];
      cur ^= 1;
      continue;
    }
    // Z1 = a1 W^T + a0 V^T
    rc = gemm_f64(s, GEMM_FULL, true, true, g.R, wout, win, 1.0, a0, win, Wp(h, dir, l), win, 0.0,
                  h->Z1, wout);
    if (rc) return rc;
    if (a1p) {
      rc = gemm_f64(s, GEMM_FULL, true, true, g.R, wout, win, 1.0, a1p, win, Wp(h, theta, l), win,
                    1.0, h->Z1, wout);
      if (rc) return rc;
    }
    if (order >= 2) {
      // Z2 = a2 W^T + 2 a1 V^T
      if (a1p) {
        rc = gemm_f64(s, GEMM_FULL, true, true, g.R, wout, win, 1.0, a2p, win, Wp(h, theta, l),
                      win, 0.0, h->Z2, wout);
        if (rc) return rc;
        rc = gemm_f64(s, GEMM_FULL, true, true, g.R, wout, win, 2.0, a1p, win, Wp(h, dir, l), win,
                      1.0, h->Z2, wout);
        if (rc) return rc;
      } else {
        rc = fill(s, g.R * wout, 0.0, h->Z2);
        if (rc) return rc;
      }
    }
    rc = net_tangent_act(s, h->rm, wout, Bp(h, dir, l), h->Z[l], h->Z1, h->Z2, h->A1[cur],
                         h->A2[cur], order);
    if (rc) return rc;
    a1p = h->A1[cur];
    a2p = h->A2[cur];
    cur ^= 1;
  }
  const int l = g.L - 1;
  const int win = g.widths[l];
  if (g.pde == kNavierStokes) {
    // the operator is nonlinear in the outputs: keep U (the forward's output
    // jets) and form U1 = a1 W^T + a0 V^T, U2 = a2 W^T + 2 a1 V^T beside it
    rc = net_rowdot(s, g.R, win, g.d_out, act_in(h, l), Wp(h, dir, l), a1p ? 1.0 : 0.0, a1p,
                    Wp(h, theta, l), h->U1);
    if (rc) return rc;
    if (order >= 2) {
      rc = a1p ? net_rowdot(s, g.R, win, g.d_out, a2p, Wp(h, theta, l), 2.0, a1p, Wp(h, dir, l),
                            h->U2)
               : fill(s, g.R * g.d_out, 0.0, h->U2);
      if (rc) return rc;
    }
    return net_ns_tangent(s, h->rm, h->U, Bp(h, theta, l), h->U1, Bp(h, dir, l), h->U2, order,
                          out);
  }
  if (order == 1) {
    // u1 = a1 W^T + a0 V^T (+ c on the value channel)
    rc = net_rowdot(s, g.R, win, 1, act_in(h, l), Wp(h, dir, l), a1p ? 1.0 : 0.0, a1p,
                    Wp(h, theta, l), h->U);
    if (rc) return rc;
    return net_linear_residual(s, h->rm, h->U, Bp(h, dir, l), out);
  }
  if (!a1p) {  // a single affine layer: r is affine in theta
    return fill(s, g.m, 0.0, out);
  }
  // u2 = a2 W^T + 2 a1 V^T (no bias term)
  rc = net_rowdot(s, g.R, win, 1, a2p, Wp(h, theta, l), 2.0, a1p, Wp(h, dir, l), h->U);
  if (rc) return rc;
  return net_linear_residual(s, h->rm, h->U, nullptr, out);
}

size_t vjp_work_bytes(const Geometry& g);

// theta-bar = J^T p, matrix-free (requires forward() at theta).
int vjp(dngd_problem* h, const double* theta, const double* p, double* gout, hipStream_t s) {
  const Geometry& g = h->g;
  int rc = backward(h, theta, p, s);
  if (rc) return rc;
  // workspace for the split-K weight-gradient GEMMs and the bias column sums
  const int64_t tiles = cdiv(g.max_width, 64) * cdiv(g.max_width, 64);
  int splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, cdiv(512, tiles)));
  splits = (int)std::min<int64_t>(splits, std::max<int64_t>(1, g.R / 256));
  rc = ensure(h, h->work, vjp_work_bytes(g));
  if (rc) return rc;
  double* work = static_cast<double*>(h->work.p);
  for (int l = 0; l < g.L; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    const double* zb = (l < g.L - 1) ? h->Zb[l] : h->seed;
    // W-bar_l = Zb_l^T A_in(l): (wout x R)(R x win)
    rc = gemm_f64(s, GEMM_FULL, false, false, wout, win, g.R, 1.0, zb, wout, act_in(h, l), win,
                  0.0, gout + g.w_off[l], win, work, splits);
    if (rc) return rc;
    rc = net_colsum_value_rows(s, h->rm, wout, zb, gout + g.b_off[l], work);
    if (rc) return rc;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// bf16 kernel-vector product (Definition 3.6 with bf16 GEMM operands and FP32
// accumulation). Per step (theta fixed), after forward(): FP32 copies of the
// hidden pre-activation jets (the jet rules run in FP32), bf16 copies of
// every layer's input activations, row-major (tangent products) and
// transposed with a value-row marker (weight and bias gradients), and bf16
// copies of the hidden weights and their transposes. Per product: the
// adjoint and tangent streams in FP32 (GEMM outputs) and bf16 (GEMM inputs).
// Row lengths of bf16 matrices are rounded up to 32 with zero padding; the
// transposed matrices have Rp = R rounded up to 32 columns.

int64_t ldw(int w) { return round_up(w, 32); }

struct LowpBufs {
  int64_t Rp = 0;
  float* Zf[kMaxLayers] = {nullptr};      // l = 0..L-2: R x w_{l+1}
  uint16_t* Hb[kMaxLayers] = {nullptr};   // l = 0..L-1: R x ldw(w_l)
  uint16_t* HbT[kMaxLayers] = {nullptr};  // l = 0..L-1: (w_l + 1) x Rp
  uint16_t* Wb[kMaxLayers] = {nullptr};   // l = 1..L-2: w_{l+1} x ldw(w_l)
  uint16_t* WTb[kMaxLayers] = {nullptr};  // l = 1..L-2: w_l x ldw(w_{l+1})
  uint16_t* Vb[kMaxLayers] = {nullptr};   // l = 0..L-2: direction blocks, w_{l+1} x ldw(w_l)
  uint16_t* seedT = nullptr;              // Rp
  uint16_t* Zb = nullptr;                 // R x ldw(max width)
  uint16_t* ZbT = nullptr;                // max width x Rp
  float* F = nullptr;                     // R x max width (adjoints, then tangents)
  uint16_t* A1 = nullptr;                 // R x ldw(max width)
  float* part = nullptr;                  // split-K partials of the weight gradients
  size_t part_bytes = 0;
};

// Carves the buffers from base (null: only sizes them); returns the bytes.
size_t lp_layout(const Geometry& g, LowpBufs& b, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* q = base ? base + off : nullptr;
    off += round_up((int64_t)bytes, 256);
    return q;
  };
  const int64_t R = g.R;
  b.Rp = round_up(R, 32);
  const int64_t wp = ldw(g.max_width);
  for (int l = 0; l < g.L; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    if (l < g.L - 1) b.Zf[l] = reinterpret_cast<float*>(take((size_t)R * wout * 4));
    b.Hb[l] = reinterpret_cast<uint16_t*>(take((size_t)R * ldw(win) * 2));
    b.HbT[l] = reinterpret_cast<uint16_t*>(take((size_t)(win + 1) * b.Rp * 2));
    if (l >= 1 && l < g.L - 1) {
      b.Wb[l] = reinterpret_cast<uint16_t*>(take((size_t)wout * ldw(win) * 2));
      b.WTb[l] = reinterpret_cast<uint16_t*>(take((size_t)win * ldw(wout) * 2));
    }
    if (l < g.L - 1) b.Vb[l] = reinterpret_cast<uint16_t*>(take((size_t)wout * ldw(win) * 2));
  }
  b.seedT = reinterpret_cast<uint16_t*>(take((size_t)b.Rp * 2));
  b.Zb = reinterpret_cast<uint16_t*>(take((size_t)R * wp * 2));
  b.ZbT = reinterpret_cast<uint16_t*>(take((size_t)g.max_width * b.Rp * 2));
  b.F = reinterpret_cast<float*>(take((size_t)R * g.max_width * 4));
  b.A1 = reinterpret_cast<uint16_t*>(take((size_t)R * wp * 2));
  size_t pb = 0;
  for (int l = 0; l < g.L; ++l)
    pb = std::max(pb, gemm_bf16_split_work_bytes(g.widths[l + 1], g.widths[l] + 1, b.Rp));
  b.part_bytes = pb;
  b.part = reinterpret_cast<float*>(take(pb));
  return off;
}

// The per-step copies (requires forward() at theta; scalar residual classes,
// L >= 2).
int lp_prepare(dngd_problem* h, const double* theta, LowpBufs& b, hipStream_t s) {
  const Geometry& g = h->g;
  DNGD_REQUIRE(g.L >= 2 && g.d_out == 1,
               "bf16 products: networks with a hidden layer and one output only");
  LowpBufs probe;
  int rc = ensure(h, h->lp, lp_layout(g, probe, nullptr));
  if (rc) return rc;
  lp_layout(g, b, static_cast<char*>(h->lp.p));
  for (int l = 0; l < g.L; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    if (l < g.L - 1) rc = lp_to_f32(s, g.R * wout, h->Z[l], b.Zf[l]);
    if (!rc) rc = lp_to_bf16_pad(s, g.R, win, act_in(h, l), win, b.Hb[l], ldw(win));
    if (!rc) rc = lp_transpose(s, h->rm, g.R, win, act_in(h, l), 0, win, b.HbT[l], b.Rp, b.Rp, 1);
    if (!rc && l >= 1 && l < g.L - 1) {
      rc = lp_to_bf16_pad(s, wout, win, Wp(h, theta, l), win, b.Wb[l], ldw(win));
      if (!rc)
        rc = lp_transpose(s, h->rm, wout, win, Wp(h, theta, l), 0, win, b.WTb[l], ldw(wout),
                          ldw(wout), 0);
    }
    if (rc) return rc;
  }
  return 0;
}

// w = J (J^T p) + lambda p with bf16 GEMMs (FP32 accumulation); t: n FP64
// scratch (receives J^T p). Requires lp_prepare() at theta.
int kvp_lp(dngd_problem* h, const double* theta, double lambda, const LowpBufs& b,
           const double* p, double* t, double* w, hipStream_t s) {
  const Geometry& g = h->g;
  const int L = g.L;
  // reverse pass: t = J^T p
  int rc = net_seeds(s, h->rm, h->U, Bp(h, theta, L - 1), p, 0, h->seed);
  if (!rc) rc = lp_seed_row(s, g.R, b.Rp, h->seed, b.seedT);
  if (rc) return rc;
  for (int hl = L - 2; hl >= 0; --hl) {
    const int w_ = g.widths[hl + 1], win = g.widths[hl];
    const int64_t ldz = ldw(w_);
    rc = lp_act_adjoint(s, h->rm, w_, ldz, b.Zf[hl], hl == L - 2 ? nullptr : b.F, h->seed,
                        Wp(h, theta, L - 1), b.Zb);
    if (!rc) rc = lp_transpose(s, h->rm, g.R, w_, b.Zb, 1, ldz, b.ZbT, b.Rp, b.Rp, 0);
    // W-bar_hl = Zb^T H_hl, with the bias gradient as the marker column
    if (!rc)
      rc = gemm_bf16_nt_split(s, w_, win + 1, b.ZbT, b.Rp, b.HbT[hl], b.Rp, b.Rp,
                              t + g.w_off[hl], win, win, t + g.b_off[hl], b.part, b.part_bytes);
    // A-bar of the layer below = Zb W_hl
    if (!rc && hl > 0)
      rc = gemm_bf16_nt(s, g.R, win, b.Zb, ldz, b.WTb[hl], ldz, ldz, nullptr, 0, nullptr, 0, 0,
                        b.F, win);
    if (rc) return rc;
  }
  const int wl = g.widths[L - 1];
  rc = gemm_bf16_nt_split(s, 1, wl + 1, b.seedT, b.Rp, b.HbT[L - 1], b.Rp, b.Rp, t + g.w_off[L - 1],
                          wl, wl, t + g.b_off[L - 1], b.part, b.part_bytes);
  if (rc) return rc;
  // forward tangent along t: w = J t
  for (int l = 0; l < L - 1; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    rc = lp_to_bf16_pad(s, wout, win, t + g.w_off[l], win, b.Vb[l], ldw(win));
    if (!rc)
      rc = (l == 0) ? gemm_bf16_nt(s, g.R, wout, b.Hb[0], ldw(win), b.Vb[0], ldw(win), ldw(win),
                                   nullptr, 0, nullptr, 0, 0, b.F, wout)
                    : gemm_bf16_nt(s, g.R, wout, b.Hb[l], ldw(win), b.Vb[l], ldw(win), ldw(win),
                                   b.A1, ldw(win), b.Wb[l], ldw(win), ldw(win), b.F, wout);
    if (!rc) rc = lp_tangent_act(s, h->rm, wout, ldw(wout), t + g.b_off[l], b.Zf[l], b.F, b.A1);
    if (rc) return rc;
  }
  rc = lp_rowdot(s, g.R, wl, ldw(wl), b.A1, Wp(h, theta, L - 1), b.Hb[L - 1], t + g.w_off[L - 1],
                 h->U);
  if (!rc) rc = net_linear_residual(s, h->rm, h->U, t + g.b_off[L - 1], w);
  if (!rc && lambda != 0.0) rc = axpy(s, g.m, lambda, p, w);
  return rc;
}

// ---------------------------------------------------------------------------
// step workspace: vectors of m and n doubles plus reduction scratch

struct StepVecs {
  double *r, *alpha, *s, *fvv, *beta, *tmpm, *rownorm2;  // m each
  double *v, *a, *t, *thtmp;                                      // n each
  double *pg, *px, *ps;  // n each: primal right-hand side, solution, refinement residual
  double* red;   // reduction scratch (256 doubles)
  double* scal;  // 64 device scalars
  double* gemv_work;
};

size_t step_vec_bytes(const Geometry& g) {
  // gemv_t scratch: J^T x (m rows, n columns) and the preconditioner's M x
  // (at most 64 row bands of m columns)
  // (primal step: J^T x and its transpose product, the same sizes swapped)
  const int64_t m1 = std::max<int64_t>(g.m, 1), n1 = std::max<int64_t>(g.n, 1);
  const size_t gw = std::max({gemv_t_workspace_bytes(m1, n1), gemv_t_workspace_bytes(n1, m1),
                              (size_t)64 * (size_t)m1 * sizeof(double)});
  // each of the 16 segments is padded to 32 doubles (256-byte aligned starts)
  return (size_t)(7 * g.m + 7 * g.n + 64 + 16 * 32) * sizeof(double) + kReduceWorkBytes + gw;
}

int carve_vecs(dngd_problem* h, StepVecs& v) {
  const Geometry& g = h->g;
  int rc = ensure(h, h->vecs, step_vec_bytes(g));
  if (rc) return rc;
  double* p = static_cast<double*>(h->vecs.p);
  auto take = [&](int64_t k) {  // segments start 256-byte aligned (vector loads, GEMM operands)
    double* q = p;
    p += round_up(k, 32);
    return q;
  };
  v.r = take(g.m);
  v.alpha = take(g.m);
  v.s = take(g.m);
  v.fvv = take(g.m);
  v.beta = take(g.m);
  v.tmpm = take(g.m);
  v.rownorm2 = take(g.m);
  v.v = take(g.n);
  v.a = take(g.n);
  v.t = take(g.n);
  v.thtmp = take(g.n);
  v.pg = take(g.n);
  v.px = take(g.n);
  v.ps = take(g.n);
  v.scal = take(64);
  v.red = take(256);
  v.gemv_work = p;
  return 0;
}

// small device block: Cholesky info and the GA acceptance flag
struct Small {
  int64_t* info;
  int* ga_flag;
};

int carve_small(dngd_problem* h, Small& sm) {
  int rc = ensure(h, h->small, 64);
  if (rc) return rc;
  char* p = static_cast<char*>(h->small.p);
  sm.info = reinterpret_cast<int64_t*>(p);
  sm.ga_flag = reinterpret_cast<int*>(p + 8);
  return 0;
}


// DNGD_ENAN unless ||r||^2 is finite (a non-finite theta, point or target);
// synchronises s
int check_finite_residual(const StepVecs& v, int64_t m, hipStream_t s) {
  int rc = sumsq(s, m, v.r, v.scal + 30, v.red);
  if (rc) return rc;
  double rr = 0.0;
  DNGD_HIP(hipMemcpyAsync(&rr, v.scal + 30, sizeof(double), hipMemcpyDeviceToHost, s));
  DNGD_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(rr)) {
    set_error("non-finite residual at theta (||r||^2 = %g)", rr);
    return DNGD_ENAN;
  }
  return 0;
}

// The dense solvers factor K = A A^T + lambda I for an operator A (M x N,
// row-major, FP32 or FP64): A = J for the dual step (M = m residuals, N = n
// parameters, Section 4.1) and A = J^T for the primal step (M = n, N = m,
// Proposition 3.1). tN (N entries) and sM (M entries) are refinement scratch.
struct DenseOp {
  const void* A;
  int64_t M, N, ldA;
  int jd;
  double* tN;
  double* sM;
};

// x = (K + lam I)^{-1} rhs with the factor in h->K, then ir_sweeps sweeps of
// refinement against the exact operator: s = rhs - (A (A^T x) + lam x), computed
// with FP32/FP64 A and FP64 accumulation; ||s||^2 of sweep k -> ir_out[k].
// One refinement sweep's residual: tN = A^T x, sM = rhs - (A tN + lam x).
int refine_residual(const DenseOp& op, const StepVecs& v, const double* rhs, const double* x,
                    double lambda, hipStream_t s) {
  int rc = gemv_t(s, op.M, op.N, op.A, op.ldA, op.jd, x, 1.0, op.tN, v.gemv_work);
  if (rc) return rc;
  return gemv_n_residual(s, op.M, op.N, op.A, op.ldA, op.jd, op.tN, rhs, x, lambda, op.sM);
}

// x += (K + lam I)^{-1} sM (the correction of a sweep, with the factor in h->K)
int refine_correct(dngd_problem* h, const DenseOp& op, double* x, hipStream_t s) {
  double* K = static_cast<double*>(h->K.p);
  const double* aux = static_cast<const double*>(h->solve_aux.p);
  int rc = chol_solve(s, op.M, K, h->ldK, aux, op.sM);
  if (rc) return rc;
  return axpy(s, op.M, 1.0, op.sM, x);
}

int dense_solve(dngd_problem* h, const DenseOp& op, const StepVecs& v, const double* rhs,
                double* x, double lambda, int ir_sweeps, double* ir_out, hipStream_t s) {
  double* K = static_cast<double*>(h->K.p);
  const double* aux = static_cast<const double*>(h->solve_aux.p);
  int rc = copy(s, op.M, rhs, x);
  if (rc) return rc;
  rc = chol_solve(s, op.M, K, h->ldK, aux, x);
  if (rc) return rc;
  for (int k = 0; k < ir_sweeps; ++k) {
    rc = refine_residual(op, v, rhs, x, lambda, s);
    if (rc) return rc;
    if (ir_out && k < 8) {
      rc = sumsq(s, op.M, op.sM, ir_out + k, v.red);
      if (rc) return rc;
    }
    rc = refine_correct(h, op, x, s);
    if (rc) return rc;
  }
  return 0;
}


// Checks a problem description; need_data == false skips the array pointers
// (footprint queries before any data is on the device).
int validate_desc(const dngd_problem_desc* d, bool need_data) {
  DNGD_REQUIRE(d->pde == DNGD_POISSON || d->pde == DNGD_HEAT || d->pde == DNGD_NAVIER_STOKES,
               "unknown pde %d", d->pde);
  DNGD_REQUIRE(d->n_layers >= 1 && d->n_layers <= kMaxLayers, "n_layers out of range");
  DNGD_REQUIRE(d->widths != nullptr, "widths is null");
  DNGD_REQUIRE(d->widths[0] >= 1 && d->widths[0] <= kMaxDin, "d_in must be in [1, %d]", kMaxDin);
  if (d->pde == DNGD_NAVIER_STOKES) {
    DNGD_REQUIRE(d->widths[0] == 2 && d->widths[d->n_layers] == 3,
                 "Navier-Stokes: the network maps (x, y) to (u, v, p)");
    DNGD_REQUIRE(d->n_init == 0, "Navier-Stokes: no initial points");
  } else {
    DNGD_REQUIRE(d->widths[d->n_layers] == 1, "the network must have one output");
  }
  for (int l = 1; l < d->n_layers; ++l)
    DNGD_REQUIRE(d->widths[l] >= 1 && d->widths[l] <= kMaxWidth, "hidden width out of range");
  DNGD_REQUIRE(d->n_int >= 0 && d->n_bdy >= 0 && d->n_init >= 0, "negative point count");
  DNGD_REQUIRE(d->n_int + d->n_bdy + d->n_init > 0, "no points");
  DNGD_REQUIRE(d->pde == DNGD_HEAT || d->n_init == 0, "initial points need the heat equation");
  DNGD_REQUIRE(d->pde == DNGD_POISSON || d->widths[0] >= 2, "heat needs d_in >= 2");
  DNGD_REQUIRE(!need_data || ((d->n_int == 0 || (d->x_int && d->f_int)) &&
                                (d->n_bdy == 0 || (d->x_bdy && d->g_bdy)) &&
                                (d->n_init == 0 || (d->x_init && d->g_init))),
               "null point or target array");
  DNGD_REQUIRE(std::isfinite(d->kappa), "kappa not finite");
  return 0;
}

void make_geometry(const dngd_problem_desc* d, Geometry& g) {
  g.pde = d->pde;
  g.L = d->n_layers;
  int64_t off = 0;
  g.max_width = 1;
  for (int l = 0; l <= g.L; ++l) g.widths[l] = d->widths[l];
  for (int l = 0; l < g.L; ++l) {
    g.w_off[l] = off;
    off += (int64_t)g.widths[l] * g.widths[l + 1];
    g.b_off[l] = off;
    off += g.widths[l + 1];
    if (l < g.L - 1) g.max_width = std::max(g.max_width, g.widths[l + 1]);
  }
  g.n = off;
  g.n_int = d->n_int;
  g.n_bdy = d->n_bdy;
  g.n_init = d->n_init;
  g.d_out = d->widths[g.L];
  g.r_int = (g.pde == DNGD_NAVIER_STOKES) ? 3 : 1;
  g.r_bdy = (g.pde == DNGD_NAVIER_STOKES) ? 3 : 1;
  g.m = d->n_int * g.r_int + d->n_bdy * g.r_bdy + d->n_init;
  g.d_in = d->widths[0];
  g.nlap = (g.pde == DNGD_HEAT) ? g.d_in - 1 : g.d_in;
  g.C_int = g.d_in + 2;
  g.R_int = g.n_int * g.C_int;
  g.R = g.R_int + g.n_bdy + g.n_init;
  g.kappa = d->kappa;
  g.c_int = g.n_int ? 1.0 / std::sqrt((double)g.n_int) : 0.0;
  g.c_bdy = g.n_bdy ? 1.0 / std::sqrt((double)g.n_bdy) : 0.0;
  g.c_init = g.n_init ? 1.0 / std::sqrt((double)g.n_init) : 0.0;
}

size_t vjp_work_bytes(const Geometry& g) {
  const int64_t tiles = cdiv(g.max_width, 64) * cdiv(g.max_width, 64);
  int splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, cdiv(512, tiles)));
  splits = (int)std::min<int64_t>(splits, std::max<int64_t>(1, g.R / 256));
  return std::max<size_t>((size_t)splits * tiles * 64 * 64 * sizeof(double),
                          (size_t)64 * kMaxWidth * sizeof(double));
}

// Jet rows per chunk of the Nystrom column build: the two FP64 products of a
// chunk against the RI landmark rows take at most ~8 GB.
int64_t nystrom_chunk_rows(const Geometry& g, int64_t RI) {
  const int64_t rows = (int64_t)(8e9 / (16.0 * (double)std::max<int64_t>(RI, 1)));
  return std::max<int64_t>(g.C_int, std::min<int64_t>(g.R, rows));
}

// Jet rows of ell landmark points, at most (all interior points)
int64_t nystrom_rows_bound(const Geometry& g, int64_t ell) {
  return std::min<int64_t>(ell, g.n_int) * g.C_int + std::max<int64_t>(0, ell - g.n_int);
}

// Device bytes a handle holds after a step with options o (activations,
// tangent streams, vectors, J, K, Gram and solve workspaces), excluding the
// copies of the point arrays.
size_t footprint_bytes(const Geometry& g, const dngd_step_opts* o) {
  dngd_step_opts def;
  dngd_step_opts_default(&def);
  if (!o) o = &def;
  size_t b = 0;
  b += (size_t)g.R * g.d_in * 8 + 2 * (size_t)act_bytes(g) + 2 * (size_t)g.R * g.d_out * 8 +
       wt_bytes(g);
  for (int l = 0; l < g.L - 1; ++l) b += 3 * (size_t)g.R * g.widths[l + 1] * 8;
  if (o->ga || o->solver == DNGD_PCG) b += 6 * (size_t)act_bytes(g);
  if (o->ga && g.pde == DNGD_NAVIER_STOKES) b += 2 * (size_t)g.R * g.d_out * 8;
  b += step_vec_bytes(g) + vjp_work_bytes(g) + (size_t)g.n * 8 + 256;
  if (o->solver == DNGD_STRUCTURED) {
    // K, solve workspace, point offsets and the two chunk products (no J)
    const int64_t RC = nystrom_chunk_rows(g, g.R);
    b += (size_t)g.m * g.m * 8 + chol_solve_aux_bytes(g.m);
    b += (size_t)round_up(g.m + 1, 32) * 8 + 2 * (size_t)RC * g.R * 8;
  } else if (o->solver != DNGD_PCG) {
    const int jd = (o->precision == DNGD_PLAIN) ? DNGD_F64 : DNGD_F32;
    const size_t esz = (jd == DNGD_F64) ? 8 : 4;
    const int64_t ldJ = round_up(g.n, 256);
    b += (size_t)g.m * ldJ * esz;
    const bool primal =
        o->solver == DNGD_PRIMAL || (o->solver == DNGD_DENSE_AUTO && g.n < g.m);
    if (primal) {
      // J^T, and K, Gram and solve workspaces of the n x n system
      b += (size_t)g.n * round_up(g.m, 256) * esz;
      b += (size_t)g.n * g.n * 8 + chol_solve_aux_bytes(g.n);
      b += gram_workspace_bytes(g.n, g.m, jd, 3, nullptr);
    } else {
      b += (size_t)g.m * g.m * 8 + chol_solve_aux_bytes(g.m);
      b += gram_workspace_bytes(g.m, g.n, jd, 3, nullptr);
    }
  } else {
    const int64_t ell = std::max<int64_t>(1, o->n_landmarks);
    const int64_t ldM = round_up(g.m, 4);
    const int64_t RI = nystrom_rows_bound(g, ell);
    const int64_t RC = nystrom_chunk_rows(g, RI);
    b += (size_t)round_up(RI + ell + 1, 32) * 8 + 2 * (size_t)round_up(RI * g.max_width, 32) * 8 +
         2 * (size_t)round_up(RC * RI, 32) * 8;
    b += (size_t)ell * ldM * 8 + (size_t)ell * ell * 8 + 2 * (size_t)ell * 8 +
         chol_solve_aux_bytes(ell);
    b += gram_workspace_bytes(ell, g.m, DNGD_F64, 1, nullptr);
    if (o->pcg_kvp == DNGD_BF16) {
      LowpBufs lb;
      b += lp_layout(g, lb, nullptr);
    }
  }
  return b;
}

// losses[k] = 0.5 ||r(theta + etas[k] dtheta)||^2 (host array); synchronises s
int losses_impl(dngd_problem* h, const double* theta, const double* dtheta, int n_eta,
                const double* etas, double* losses, hipStream_t s);

// Dense Cholesky solve shared by dngd_cholesky_solve and its allocation-free
// variant. buf: device scratch of cholesky_solve_scratch_bytes(m) bytes (the
// info word, then the factor's and the solves' workspace); every byte the
// call reads is written by the call first.
int cholesky_solve_check(int64_t m, const double* K, int64_t ldK, int64_t nrhs, const double* B,
                         int64_t ldB, const int64_t* info) {
  DNGD_REQUIRE(K && info, "dngd_cholesky_solve: null pointer");
  DNGD_REQUIRE(m > 0 && ldK >= m && nrhs >= 0 && (nrhs == 0 || (B && ldB >= m)),
               "dngd_cholesky_solve: bad sizes");
  return 0;
}

size_t cholesky_solve_scratch_bytes(int64_t m) { return 256 + chol_solve_aux_bytes(m); }

int cholesky_solve_impl(int64_t m, double* K, int64_t ldK, int32_t factored, int64_t nrhs,
                        double* B, int64_t ldB, int64_t* info, hipStream_t s, char* buf) {
  *info = 0;
  int64_t* dinfo = reinterpret_cast<int64_t*>(buf);
  double* aux = reinterpret_cast<double*>(buf + 256);
  int rc = 0;
  if (!factored) {
    rc = chol_factor(s, m, K, ldK, dinfo, aux, nullptr);  // clears *dinfo first
    if (!rc) {
      hipError_t e = hipMemcpyAsync(info, dinfo, sizeof(int64_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) rc = hip_fail(e, "info readback", __FILE__, __LINE__);
    }
  }
  if (!rc && *info == 0 && nrhs > 0) {
    rc = chol_prepare_solve(s, m, K, ldK, aux);
    for (int64_t j = 0; j < nrhs && !rc; ++j) rc = chol_solve(s, m, K, ldK, aux, B + j * ldB);
  }
  if (rc) return rc;
  if (*info != 0) {
    set_error("Cholesky: non-positive pivot at column %lld", (long long)*info);
    return DNGD_ENOTPD;
  }
  return DNGD_OK;
}

}  // namespace

// Scratch of dngd_cholesky_solve_noalloc: a static device array, one copy on
// every device the library is loaded on, held until the process ends. Host
// code never uses the array's name as an address (on the host it is only a
// stand-in for the symbol): noalloc_scratch() looks up each device's address
// once, with that device current, and every launch takes that address.
constexpr int kNoAllocMaxM = 2048;
constexpr size_t kNoAllocScratchBytes = (size_t)65 << 20;  // >= 256 + chol_solve_aux_bytes(2048)
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {nullptr};

int noalloc_scratch(char** out) {
  int dev = 0;
  DNGD_HIP(hipGetDevice(&dev));
  DNGD_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* dngd_last_error(void) { return g_err; }
const char* dngd_version(void) { return "libdngd 0.1 (gfx950)"; }

void dngd_step_opts_default(dngd_step_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = DNGD_MIXED;
  o->solver = DNGD_DENSE;
  o->ga = 1;
  o->ir_sweeps = 2;
  o->gram_passes = 0;
  o->eps_norm = 0.0;
  o->pcg_tol = 1e-6;
  o->pcg_maxit = 500;
  o->ir_tol = 1e-5;
}

int dngd_problem_create(const dngd_problem_desc* d, dngd_problem** out) {
  DNGD_REQUIRE(d && out, "dngd_problem_create: null argument");
  *out = nullptr;
  int vrc = validate_desc(d, true);
  if (vrc) return vrc;

  dngd_problem* h = new dngd_problem();
  Geometry& g = h->g;
  make_geometry(d, g);
  h->rm = row_map(g);
  if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;

  int rc = 0;
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
    h->side = nullptr;
    rc = DNGD_EHIP;
  }
  if (!rc && hipEventCreateWithFlags(&h->last_use, hipEventDisableTiming) != hipSuccess) {
    h->last_use = nullptr;
    rc = DNGD_EHIP;
  }
  h->astream = h->side;  // creation's allocations and copies run on the side stream
  // A device-to-device hipMemcpy does not wait for the copy before it
  // returns, and the caller may free or reuse the source arrays as soon as
  // this call returns: enqueue the copies, then wait for them.
  auto dup = [&](double** dst, const double* src, int64_t cnt) {
    if (rc) return;
    rc = dmalloc(h, (void**)dst, (size_t)std::max<int64_t>(cnt, 1) * sizeof(double));
    if (!rc && cnt > 0) {
      hipError_t e = hipMemcpyAsync(*dst, src, (size_t)cnt * sizeof(double), hipMemcpyDefault,
                                    h->side);
      if (e != hipSuccess) rc = hip_fail(e, "hipMemcpyAsync", __FILE__, __LINE__);
    }
  };
  dup(&h->x_int, d->x_int, g.n_int * g.d_in);
  dup(&h->x_bdy, d->x_bdy, g.n_bdy * g.d_in);
  dup(&h->x_init, d->x_init, g.n_init * g.d_in);
  dup(&h->f_int, d->f_int, g.n_int * g.r_int);
  dup(&h->g_bdy, d->g_bdy, g.n_bdy * g.r_bdy);
  dup(&h->g_init, d->g_init, g.n_init);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(h->side);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
  }
  if (!rc) rc = dmalloc(h, (void**)&h->A0, (size_t)g.R * g.d_in * sizeof(double));
  for (int l = 0; l < g.L - 1 && !rc; ++l) {
    const size_t b = (size_t)g.R * g.widths[l + 1] * sizeof(double);
    rc |= dmalloc(h, (void**)&h->Z[l], b);
    if (!rc) rc = dmalloc(h, (void**)&h->A[l], b);
    if (!rc) rc = dmalloc(h, (void**)&h->Zb[l], b);
  }
  if (!rc) rc = dmalloc(h, (void**)&h->Ab[0], act_bytes(g));
  if (!rc) rc = dmalloc(h, (void**)&h->Ab[1], act_bytes(g));
  if (!rc) rc = dmalloc(h, (void**)&h->WT, wt_bytes(g));
  if (!rc) rc = dmalloc(h, (void**)&h->seed, (size_t)g.R * g.d_out * sizeof(double));
  if (!rc) rc = dmalloc(h, (void**)&h->U, (size_t)g.R * g.d_out * sizeof(double));
  for (int e = 0; e < 10 && !rc; ++e)
    if (hipEventCreate(&h->ev[e]) != hipSuccess) rc = DNGD_EHIP;
  for (int e = 0; e < 2 && !rc; ++e)
    if (hipEventCreateWithFlags(&h->cev[e], hipEventDisableTiming) != hipSuccess) rc = DNGD_EHIP;
  if (!rc && hipHostMalloc(&h->hstage, kHostStageBytes, hipHostMallocDefault) != hipSuccess) {
    h->hstage = nullptr;
    rc = DNGD_EHIP;
  }
  if (!rc) {  // the activation buffers are allocated once creation returns
    hipError_t e = hipStreamSynchronize(h->side);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize", __FILE__, __LINE__);
  }
  if (rc) {
    dngd_problem_destroy(h);
    return rc;
  }
  *out = h;
  return DNGD_OK;
}

int dngd_problem_destroy(dngd_problem* h) {
  if (!h) return DNGD_OK;
  // wait for this handle's own work only (its last call's stream and the
  // side stream), then return its memory to the stream-ordered pool
  if (h->last_use_valid) hipEventSynchronize(h->last_use);
  if (h->side) hipStreamSynchronize(h->side);
  for (void* p : h->owned)
    if (p) hipFreeAsync(p, h->side);
  if (h->side) hipStreamSynchronize(h->side);
  if (h->last_use) hipEventDestroy(h->last_use);
  for (auto& e : h->ev)
    if (e) hipEventDestroy(e);
  for (auto& e : h->cev)
    if (e) hipEventDestroy(e);
  if (h->side) hipStreamDestroy(h->side);
  if (h->hstage) hipHostFree(h->hstage);
  delete h;
  return DNGD_OK;
}

int64_t dngd_num_params(const dngd_problem* h) { return h ? h->g.n : -1; }
int64_t dngd_num_residuals(const dngd_problem* h) { return h ? h->g.m : -1; }
int64_t dngd_jacobian_ld(const dngd_problem* h) { return h ? round_up(h->g.n, 256) : -1; }

int dngd_footprint(const dngd_problem* h, const dngd_step_opts* o, size_t* bytes) {
  DNGD_REQUIRE(h && bytes, "dngd_footprint: null argument");
  *bytes = footprint_bytes(h->g, o);
  return DNGD_OK;
}

int dngd_footprint_desc(const dngd_problem_desc* d, const dngd_step_opts* o, size_t* bytes) {
  DNGD_REQUIRE(d && bytes, "dngd_footprint_desc: null argument");
  int rc = validate_desc(d, false);
  if (rc) return rc;
  Geometry g;
  make_geometry(d, g);
  *bytes = footprint_bytes(g, o) + (size_t)(g.n_int * (g.d_in + g.r_int) +
                                            g.n_bdy * (g.d_in + g.r_bdy) +
                                            g.n_init * (g.d_in + 1)) * sizeof(double);
  return DNGD_OK;
}

int dngd_residual_jacobian(dngd_problem* h, const double* theta, double* r, void* J, int64_t ldJ,
                           int32_t j_dtype, void* stream) {
  DNGD_REQUIRE(h && theta, "dngd_residual_jacobian: null argument");
  if (J) {
    DNGD_REQUIRE(j_dtype == DNGD_F64 || j_dtype == DNGD_F32, "bad j_dtype");
    DNGD_REQUIRE(ldJ >= h->g.n && ldJ % 4 == 0, "ldJ must be >= n and a multiple of 4");
  }
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  int rc = forward(h, theta, r, s);
  if (rc) return rc;
  if (!J) return DNGD_OK;
  return jacobian_all(h, theta, J, ldJ, j_dtype, nullptr, s);
}

int dngd_gram(int64_t m, int64_t n, const void* J, int64_t ldJ, int32_t j_dtype, int32_t passes,
              double lambda, double* K, int64_t ldK, void* stream) {
  DNGD_REQUIRE(J && K, "dngd_gram: null pointer");
  DNGD_REQUIRE(m > 0 && n > 0 && ldJ >= n && ldK >= m, "dngd_gram: bad sizes");
  DNGD_REQUIRE(j_dtype == DNGD_F64 || j_dtype == DNGD_F32, "dngd_gram: bad j_dtype");
  DNGD_REQUIRE(j_dtype == DNGD_F64 || passes == 1 || passes == 3 || passes == 4 ||
                   passes == DNGD_GRAM_F64,
               "dngd_gram: passes 1, 3, 4 or DNGD_GRAM_F64");
  DNGD_REQUIRE(std::isfinite(lambda), "dngd_gram: lambda not finite");
  DNGD_REQUIRE(j_dtype == DNGD_F64 || ldJ % 4 == 0, "dngd_gram: FP32 J needs ldJ %% 4 == 0");
  hipStream_t s = S(stream);
  const size_t wb = gram_workspace_bytes(m, n, j_dtype, passes, nullptr);
  void* work = nullptr;
  DNGD_HIP(hipMallocAsync(&work, wb, s));
  int rc = gram_launch(s, m, n, J, ldJ, j_dtype, passes, lambda, K, ldK, work, wb);
  hipError_t e = hipFreeAsync(work, s);
  if (rc) return rc;
  DNGD_HIP(e);
  return DNGD_OK;
}

int dngd_cholesky_solve(int64_t m, double* K, int64_t ldK, int32_t factored, int64_t nrhs,
                        double* B, int64_t ldB, int64_t* info, void* stream) {
  int rc = cholesky_solve_check(m, K, ldK, nrhs, B, ldB, info);
  if (rc) return rc;
  hipStream_t s = S(stream);
  char* buf = nullptr;
  DNGD_HIP(hipMallocAsync((void**)&buf, cholesky_solve_scratch_bytes(m), s));
  rc = cholesky_solve_impl(m, K, ldK, factored, nrhs, B, ldB, info, s, buf);
  hipFreeAsync(buf, s);
  return rc;
}

int dngd_cholesky_solve_noalloc(int64_t m, double* K, int64_t ldK, int32_t factored,
                                int64_t nrhs, double* B, int64_t ldB, int64_t* info,
                                void* stream) {
  int rc = cholesky_solve_check(m, K, ldK, nrhs, B, ldB, info);
  if (rc) return rc;
  const size_t need = cholesky_solve_scratch_bytes(m);
  DNGD_REQUIRE(need <= kNoAllocScratchBytes,
               "dngd_cholesky_solve_noalloc: m = %lld needs %zu bytes of scratch, the static "
               "array holds %zu (m <= %d)",
               (long long)m, need, kNoAllocScratchBytes, kNoAllocMaxM);
  char* buf = nullptr;
  rc = noalloc_scratch(&buf);
  if (rc) return rc;
  return cholesky_solve_impl(m, K, ldK, factored, nrhs, B, ldB, info, S(stream), buf);
}

int dngd_cholesky_solve_refine(int64_t m, double* K, int64_t ldK, int32_t factored,
                               int64_t nrhs, double* B, int64_t ldB, const dngd_refine* refine,
                               double* rel_res, int64_t* info, void* stream) {
  int rc = cholesky_solve_check(m, K, ldK, nrhs, B, ldB, info);
  if (rc) return rc;
  DNGD_REQUIRE(refine != nullptr && refine->J != nullptr,
               "dngd_cholesky_solve_refine: refine and refine->J must not be null");
  const dngd_refine R = *refine;
  DNGD_REQUIRE(R.j_dtype == DNGD_F32 || R.j_dtype == DNGD_F64,
               "dngd_cholesky_solve_refine: j_dtype must be DNGD_F32 or DNGD_F64");
  DNGD_REQUIRE(R.n >= 1 && R.ldJ >= R.n && R.ldJ % 4 == 0 &&
                   reinterpret_cast<uintptr_t>(R.J) % 16 == 0,
               "dngd_cholesky_solve_refine: J needs n >= 1, ldJ >= n, ldJ %% 4 == 0 and a "
               "16-byte aligned base");
  DNGD_REQUIRE(R.sweeps >= 0 && R.sweeps <= 16, "dngd_cholesky_solve_refine: sweeps in 0..16");
  DNGD_REQUIRE(std::isfinite(R.lambda) && R.lambda >= 0.0,
               "dngd_cholesky_solve_refine: lambda must be finite and >= 0");
  hipStream_t s = S(stream);
  // scratch: the Cholesky call's, then (256-byte aligned) b, s (m each),
  // J^T x (n), the sums of squares, the reduction and gemv_t workspaces
  const int64_t nss = (int64_t)std::max<int64_t>(1, nrhs) * (R.sweeps + 1);
  const size_t base = round_up((int64_t)cholesky_solve_scratch_bytes(m), 256);
  const size_t vec = (size_t)(2 * round_up(m, 32) + round_up(R.n, 32) + round_up(nss, 32)) *
                     sizeof(double);
  const size_t bytes = base + vec + kReduceWorkBytes + gemv_t_workspace_bytes(m, R.n);
  char* buf = nullptr;
  DNGD_HIP(hipMallocAsync((void**)&buf, bytes, s));
  double* bcopy = reinterpret_cast<double*>(buf + base);
  double* sres = bcopy + round_up(m, 32);
  double* tN = sres + round_up(m, 32);
  double* ss = tN + round_up(R.n, 32);
  double* red = ss + round_up(nss, 32);
  double* gw = red + kReduceWorkBytes / sizeof(double);
  // factor (and read info back), then the solves with refinement
  rc = cholesky_solve_impl(m, K, ldK, factored, 0, B, ldB, info, s, buf);
  double* aux = reinterpret_cast<double*>(buf + 256);
  if (!rc && nrhs > 0) rc = chol_prepare_solve(s, m, K, ldK, aux);
  for (int64_t j = 0; j < nrhs && !rc; ++j) {
    double* x = B + j * ldB;
    double* ssj = ss + j * (R.sweeps + 1);
    rc = copy(s, m, x, bcopy);
    if (!rc) rc = sumsq(s, m, bcopy, ssj, red);
    if (!rc) rc = chol_solve(s, m, K, ldK, aux, x);
    for (int k = 0; k < R.sweeps && !rc; ++k) {
      rc = gemv_t(s, m, R.n, R.J, R.ldJ, R.j_dtype, x, 1.0, tN, gw);
      if (!rc) rc = gemv_n_residual(s, m, R.n, R.J, R.ldJ, R.j_dtype, tN, bcopy, x, R.lambda, sres);
      if (!rc) rc = sumsq(s, m, sres, ssj + 1 + k, red);
      if (!rc) rc = chol_solve(s, m, K, ldK, aux, sres);
      if (!rc) rc = axpy(s, m, 1.0, sres, x);
    }
  }
  std::vector<double> hss;
  if (!rc && rel_res && nrhs > 0 && R.sweeps > 0) {
    hss.resize((size_t)nss);
    hipError_t e = hipMemcpyAsync(hss.data(), ss, nss * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) rc = hip_fail(e, "rel_res readback", __FILE__, __LINE__);
  }
  hipError_t e = hipFreeAsync(buf, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (rc) return rc;
  DNGD_HIP(e);
  for (int64_t j = 0; j < (int64_t)hss.size() / (R.sweeps + 1); ++j) {
    const double bb = hss[j * (R.sweeps + 1)];
    for (int k = 0; k < R.sweeps; ++k)
      rel_res[j * R.sweeps + k] = bb > 0.0 ? std::sqrt(hss[j * (R.sweeps + 1) + 1 + k] / bb) : 0.0;
  }
  return DNGD_OK;
}

int dngd_fvv(dngd_problem* h, const double* theta, const double* v, double* fvv, void* stream) {
  DNGD_REQUIRE(h && theta && v && fvv, "dngd_fvv: null argument");
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  int rc = forward(h, theta, nullptr, s);
  if (rc) return rc;
  return tangent(h, theta, v, 2, fvv, s);
}

int dngd_jvp(dngd_problem* h, const double* theta, const double* u, double* w, void* stream) {
  DNGD_REQUIRE(h && theta && u && w, "dngd_jvp: null argument");
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  int rc = forward(h, theta, nullptr, s);
  if (rc) return rc;
  return tangent(h, theta, u, 1, w, s);
}

int dngd_vjp(dngd_problem* h, const double* theta, const double* p, double* gout, void* stream) {
  DNGD_REQUIRE(h && theta && p && gout, "dngd_vjp: null argument");
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  int rc = forward(h, theta, nullptr, s);
  if (rc) return rc;
  return vjp(h, theta, p, gout, s);
}

int dngd_losses(dngd_problem* h, const double* theta, const double* dtheta, int32_t n_eta,
                const double* etas, double* losses, void* stream) {
  DNGD_REQUIRE(h && theta && dtheta && etas && losses && n_eta > 0 && n_eta <= 48,
               "dngd_losses: bad argument");
  CallScope scope(h, S(stream));
  return losses_impl(h, theta, dtheta, n_eta, etas, losses, S(stream));
}

}  // extern "C"

namespace {

int losses_impl(dngd_problem* h, const double* theta, const double* dtheta, int n_eta,
                const double* etas, double* losses, hipStream_t s) {
  StepVecs v;
  int rc = carve_vecs(h, v);
  if (rc) return rc;
  for (int k = 0; k < n_eta && !rc; ++k) {
    rc = copy(s, h->g.n, theta, v.thtmp);
    if (!rc) rc = axpy(s, h->g.n, etas[k], dtheta, v.thtmp);
    if (!rc) rc = forward(h, v.thtmp, v.tmpm, s);
    if (!rc) rc = sumsq(s, h->g.m, v.tmpm, v.scal + k, v.red);
  }
  if (rc) return rc;
  DNGD_HIP(hipMemcpyAsync(losses, v.scal, sizeof(double) * n_eta, hipMemcpyDeviceToHost, s));
  DNGD_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < n_eta; ++k) losses[k] *= 0.5;
  return DNGD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Nystrom-PCG (Sections 3.3, 4.2)
//
// The preconditioner is the paper's P^{-1} = U (L^ + lam I)^{-1} U^T +
// (I - U U^T)/lam with U L^ U^T = K^ = K_{:,I} K_II^+ K_{I,:}. Since
// P^{-1} = (K^ + lam I)^{-1}, it is applied here in Woodbury form without an
// eigendecomposition: with K_II + delta I = L_I L_I^T and M^T = L_I^{-1} K_{I,:}
// (so K^ = M M^T), P^{-1} x = (x - M (lam I + M^T M)^{-1} M^T x) / lam.
// delta = ell * eps * max_i (K_II)_ii plays the role of the paper's "positive
// eigenvalues" cut; it is doubled until the Cholesky of K_II succeeds.

namespace {

// K (m x m, lower triangle, row-major ldK) = J J^T + lam I without forming J.
// Per affine layer l with adjoints G_l and inputs H_l (R jet rows), the rows
// of J for point i are sum_c G_l[c] (x) H_l[c] over its jet rows c, so
//   J_i . J_j = sum_l sum_{c of i, c' of j} (G_l[c] . G_l[c']) (H_l[c] . H_l[c'])
//               + G_l[i value] . G_l[j value]   (bias)
// (the per-layer structured form the paper builds its kernel from, Section 4).
// Jet rows are taken in chunks; a chunk's G and H rows are multiplied (FP64
// MFMA) by the rows of all points up to the chunk's last one, and the combine
// kernel sums the channel pairs into K[p][q], q <= p.
int structured_gram(dngd_problem* h, const double* theta, double lambda, double* K,
                    int64_t ldK, hipStream_t s) {
  const Geometry& g = h->g;
  std::vector<int64_t> qoff(g.m + 1, 0);
  for (int64_t p = 0; p < g.m; ++p) qoff[p + 1] = qoff[p] + (p < g.n_int ? g.C_int : 1);
  const int64_t R = qoff[g.m];
  const int64_t RC = nystrom_chunk_rows(g, R);
  // work (h->J): point row offsets, then the chunk products Gp, Hp (RC x R)
  const size_t bOff = (size_t)round_up(g.m + 1, 32) * 8;
  int rc = ensure(h, h->J, bOff + 2 * (size_t)RC * R * 8);
  if (rc) return rc;
  int64_t* dQoff = static_cast<int64_t*>(h->J.p);
  double* Gp = reinterpret_cast<double*>(static_cast<char*>(h->J.p) + bOff);
  double* Hp = Gp + (size_t)RC * R;
  DNGD_HIP(hipMemcpyAsync(dQoff, qoff.data(), (g.m + 1) * 8, hipMemcpyHostToDevice, s));
  rc = backward(h, theta, nullptr, s);
  if (rc) return rc;
  for (int l = 0; l < g.L; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    const double* Gl = (l < g.L - 1) ? h->Zb[l] : h->seed;
    const double* Hl = act_in(h, l);
    for (int64_t p0 = 0; p0 < g.m;) {
      int64_t p1 = p0;
      if (p0 < g.n_int) p1 = std::min<int64_t>(g.n_int, p0 + std::max<int64_t>(1, RC / g.C_int));
      else p1 = std::min<int64_t>(g.m, p0 + RC);
      const int64_t row0 = qoff[p0], row1 = qoff[p1], nr = row1 - row0;
      rc = gemm_f64(s, GEMM_FULL, true, true, nr, row1, wout, 1.0, Gl + row0 * wout, wout, Gl,
                    wout, 0.0, Gp, R);
      if (!rc)
        rc = gemm_f64(s, GEMM_FULL, true, true, nr, row1, win, 1.0, Hl + row0 * win, win, Hl, win,
                      0.0, Hp, R);
      if (!rc)
        rc = net_nystrom_combine(s, h->rm, p0, p1 - p0, row0, Gp, Hp, R, p1, dQoff, K, ldK,
                                 l > 0 ? 1 : 0, 1);
      if (rc) return rc;
      p0 = p1;
    }
  }
  return add_diag(s, g.m, K, ldK, lambda);
}

// G = lam I + Mt Mt^T, factorised and prepared for solves (the Woodbury
// form's small system; redone alone when only lambda changes)
int pcg_factor_G(dngd_problem* h, Precond& P, double lambda, hipStream_t s) {
  const Geometry& g = h->g;
  StepVecs v;
  int rc = carve_vecs(h, v);
  if (rc) return rc;
  const int64_t ell = P.ell;
  const size_t gw = gram_workspace_bytes(ell, g.m, DNGD_F64, 1, nullptr);
  rc = ensure(h, h->gram_work, gw);
  if (rc) return rc;
  rc = gram_launch(s, ell, g.m, P.Mt, P.ldM, DNGD_F64, 1, lambda, P.G, ell, h->gram_work.p, gw);
  if (rc) return rc;
  rc = chol_factor(s, ell, P.G, ell, reinterpret_cast<int64_t*>(v.scal), P.Gaux, nullptr);
  if (rc) return rc;
  int64_t hinfo = 1;
  DNGD_HIP(hipMemcpyAsync(&hinfo, v.scal, 8, hipMemcpyDeviceToHost, s));
  DNGD_HIP(hipStreamSynchronize(s));
  DNGD_REQUIRE(hinfo == 0, "Nystrom: lam I + M^T M not positive definite");
  P.lambda = lambda;
  return chol_prepare_solve(s, ell, P.G, ell, P.Gaux);
}

// chunk_rows: jet rows per chunk of the landmark-column products (0 = sized
// for about 8 GB of products)
int pcg_build(dngd_problem* h, const double* theta, double lambda, const int64_t* I, int64_t ell,
              Precond& P, hipStream_t s, int64_t chunk_rows = 0) {
  const Geometry& g = h->g;
  // landmark indices: validated on the host before any kernel reads them
  std::vector<int64_t> hI(ell);
  DNGD_HIP(hipMemcpyAsync(hI.data(), I, ell * 8, hipMemcpyDeviceToHost, s));
  DNGD_HIP(hipStreamSynchronize(s));
  for (int64_t q = 0; q < ell; ++q) {
    DNGD_REQUIRE(hI[q] >= 0 && hI[q] < g.m, "landmark index %lld out of range", (long long)hI[q]);
    DNGD_REQUIRE(q == 0 || hI[q] > hI[q - 1], "landmarks must be sorted and distinct");
  }
  // jet rows of the landmark points (a residual is one point)
  std::vector<int64_t> rowsI, qoff(ell + 1, 0);
  for (int64_t q = 0; q < ell; ++q) {
    const int64_t p = hI[q];
    const int64_t base = p < g.n_int ? p * g.C_int : g.R_int + (p - g.n_int);
    const int C = p < g.n_int ? g.C_int : 1;
    for (int c = 0; c < C; ++c) rowsI.push_back(base + c);
    qoff[q + 1] = qoff[q] + C;
  }
  const int64_t RI = qoff[ell];
  const int64_t ldM = round_up(g.m, 4);
  const int64_t RC = chunk_rows > 0 ? std::max<int64_t>(chunk_rows, g.C_int)
                                    : nystrom_chunk_rows(g, RI);
  // work (h->J): landmark row lists, gathered G_I and H_I, chunk products Gp, Hp
  // the gathered rows start 256-byte aligned (the faster product kernel needs
  // 16-byte aligned operands)
  const size_t bRows = (size_t)round_up(RI + ell + 1, 32) * 8;
  const int64_t gath = round_up(RI * g.max_width, 32), prod = round_up(RC * RI, 32);
  const size_t bGath = 2 * (size_t)gath * 8;
  const size_t bProd = 2 * (size_t)prod * 8;
  int rc = ensure(h, h->J, bRows + bGath + bProd);
  if (rc) return rc;
  int64_t* dRows = static_cast<int64_t*>(h->J.p);
  int64_t* dQoff = dRows + RI;
  double* GI = reinterpret_cast<double*>(dRows + round_up(RI + ell + 1, 32));
  double* HI = GI + gath;
  double* Gp = HI + gath;
  double* Hp = Gp + prod;
  // Mt (ell x ldM), G (ell x ell), index scratch, ell vector, solve workspace
  const size_t bMt = (size_t)ell * ldM * 8, bG = (size_t)ell * ell * 8;
  rc = ensure(h, h->K, bMt + bG + (size_t)ell * 8 + (size_t)ell * 8 + chol_solve_aux_bytes(ell));
  if (rc) return rc;
  P.Mt = static_cast<double*>(h->K.p);
  P.ldM = ldM;
  P.G = P.Mt + (size_t)ell * ldM;
  int64_t* idx = reinterpret_cast<int64_t*>(P.G + (size_t)ell * ell);
  P.tl = reinterpret_cast<double*>(idx + ell);
  P.Gaux = P.tl + ell;
  P.ell = ell;
  P.lambda = lambda;
  StepVecs v;
  rc = carve_vecs(h, v);
  if (rc) return rc;
  DNGD_HIP(hipMemcpyAsync(dRows, rowsI.data(), RI * 8, hipMemcpyHostToDevice, s));
  DNGD_HIP(hipMemcpyAsync(dQoff, qoff.data(), (ell + 1) * 8, hipMemcpyHostToDevice, s));
  DNGD_HIP(hipMemcpyAsync(idx, hI.data(), ell * 8, hipMemcpyHostToDevice, s));

  // K_{I,:} = J_I J^T layer by layer from the Jacobian-seeded adjoints
  rc = backward(h, theta, nullptr, s);
  if (rc) return rc;
  const int64_t npts = g.m;
  for (int l = 0; l < g.L; ++l) {
    const int win = g.widths[l], wout = g.widths[l + 1];
    const double* Gl = (l < g.L - 1) ? h->Zb[l] : h->seed;
    const double* Hl = act_in(h, l);
    rc = net_gather_rows(s, RI, wout, dRows, Gl, GI);
    if (!rc) rc = net_gather_rows(s, RI, win, dRows, Hl, HI);
    if (rc) return rc;
    for (int64_t p0 = 0; p0 < npts;) {
      // points [p0, p1) whose jet rows fit in one chunk
      const int64_t row0 = p0 < g.n_int ? p0 * g.C_int : g.R_int + (p0 - g.n_int);
      int64_t p1 = p0;
      if (p0 < g.n_int) p1 = std::min<int64_t>(g.n_int, p0 + std::max<int64_t>(1, RC / g.C_int));
      else p1 = std::min<int64_t>(npts, p0 + RC);
      const int64_t row1 = p1 < g.n_int ? p1 * g.C_int : g.R_int + (p1 - g.n_int);
      const int64_t nr = row1 - row0;
      rc = gemm_f64(s, GEMM_FULL, true, true, nr, RI, wout, 1.0, Gl + row0 * wout, wout, GI, wout,
                    0.0, Gp, RI);
      if (!rc)
        rc = gemm_f64(s, GEMM_FULL, true, true, nr, RI, win, 1.0, Hl + row0 * win, win, HI, win,
                      0.0, Hp, RI);
      if (!rc)
        rc = net_nystrom_combine(s, h->rm, p0, p1 - p0, row0, Gp, Hp, RI, ell, dQoff, P.Mt, ldM,
                                 l > 0 ? 1 : 0);
      if (rc) return rc;
      p0 = p1;
    }
  }
  // K_II (landmark columns of K_{I,:}), shifted by delta and factorised; the
  // shift grows until the factorisation succeeds
  double* LI = P.G;  // G's storage holds L_I until M^T is formed
  rc = gather_cols(s, ell, P.Mt, ldM, I, LI);
  if (rc) return rc;
  std::vector<double> Kii((size_t)ell * ell);
  DNGD_HIP(hipMemcpyAsync(Kii.data(), LI, Kii.size() * 8, hipMemcpyDeviceToHost, s));
  DNGD_HIP(hipStreamSynchronize(s));
  double dmax = 0.0;
  for (int64_t i = 0; i < ell; ++i) dmax = std::max(dmax, Kii[(size_t)i * ell + i]);
  double delta = (double)ell * 2.220446049250313e-16 * dmax;
  if (!(delta > 0.0)) delta = 1e-300;
  int64_t hinfo = 1;
  for (int attempt = 0; attempt < 40 && hinfo != 0; ++attempt) {
    std::vector<double> A(Kii);
    for (int64_t i = 0; i < ell; ++i) A[(size_t)i * ell + i] += delta;
    DNGD_HIP(hipMemcpyAsync(LI, A.data(), A.size() * 8, hipMemcpyHostToDevice, s));
    rc = chol_factor(s, ell, LI, ell, reinterpret_cast<int64_t*>(v.scal), P.Gaux, nullptr);
    if (rc) return rc;
    DNGD_HIP(hipMemcpyAsync(&hinfo, v.scal, 8, hipMemcpyDeviceToHost, s));
    DNGD_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) delta *= 4.0;
  }
  DNGD_REQUIRE(hinfo == 0, "Nystrom: K_II could not be factorised");
  P.delta = delta;
  // Mt = L_I^{-1} K_{I,:}
  rc = trsm_lower_left(s, ell, LI, ell, g.m, P.Mt, ldM);
  if (rc) return rc;
  return pcg_factor_G(h, P, lambda, s);
}

// z = P^{-1} x
int precond_apply(dngd_problem* h, const Precond& P, const StepVecs& v, const Small& sm,
                  const double* x, double* z, double* tl, hipStream_t s) {
  const Geometry& g = h->g;
  // tl = -(M^T x)
  int rc = gemv_n_residual(s, P.ell, g.m, P.Mt, P.ldM, DNGD_F64, x, nullptr, nullptr, 0.0, tl);
  if (rc) return rc;
  rc = chol_solve(s, P.ell, P.G, P.ell, P.Gaux, tl);
  if (rc) return rc;
  // z = M tl = -(M (lam + M^T M)^{-1} M^T x); finish: z = (x + z_neg...) handled by sign
  rc = gemv_t(s, P.ell, g.m, P.Mt, P.ldM, DNGD_F64, tl, -1.0, z, v.gemv_work);
  if (rc) return rc;
  return woodbury_finish(s, g.m, x, 1.0 / P.lambda, z);
}

int kvp(dngd_problem* h, const double* theta, double lambda, const StepVecs& v, const double* p,
        double* w, hipStream_t s) {
  int rc = vjp(h, theta, p, v.t, s);
  if (rc) return rc;
  rc = tangent(h, theta, v.t, 1, w, s);
  if (rc) return rc;
  return axpy(s, h->g.m, lambda, p, w);
}

int read_scalars(double* host, const double* dev, int n, hipStream_t s) {
  DNGD_HIP(hipMemcpyAsync(host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  DNGD_HIP(hipStreamSynchronize(s));
  return 0;
}

struct PcgResult {
  int iters = 0;          // kernel-vector products of the iteration (either precision)
  double relres = 1.0;    // final ||r|| / ||b||: the true residual when one was formed last
  int kvp_f64 = 0;        // FP64 products (true residuals and FP64 iterations)
  int replacements = 0;   // recursive residuals replaced by true ones
  int escalated = 0;      // 1: the bf16 products stopped reducing the true residual
};

// PCG (appendix algorithm) on (J J^T + lam I) y = b from y = 0.
// Work vectors: y -> x (output); r = v.s; z = v.tmpm; p = v.rownorm2; Ap = v.alpha;
// the kernel-vector product uses v.t. b is read by every true residual.
//
// With lp (bf16 products), the recursion runs on the bf16 operator, whose
// error (~2^-8 of ||K|| per product) the recursive residual does not see.
// So whenever the recursive residual reaches tol (or has fallen 2^10-fold
// since the last replacement), the true residual b - A y is formed with the
// FP64 product; if it meets tol the solve has converged, else it replaces the
// recursive one and the recursion restarts from y (residual replacement).
// When a replacement shows that the true residual fell less than 8-fold
// since the previous one, the bf16 error (about 2^-8 ||K|| per product)
// dominates at this damping (lambda small against 2^-8 ||K||: the components
// of the residual along K's small eigenvalues are not reduced) and the
// remaining iterations use the FP64 product, which at such a rate of
// contraction needs fewer FP64 products than further replacements would.
int pcg_solve(dngd_problem* h, const double* theta, const Precond& P, const StepVecs& v,
              const Small& sm, const double* b, double* x, double tol, int64_t maxit,
              PcgResult* res, hipStream_t s, const LowpBufs* lp = nullptr) {
  const Geometry& g = h->g;
  double* r = v.s;
  double* z = v.tmpm;
  double* p = v.rownorm2;
  double* Ap = v.alpha;
  double* tlv = P.tl;
  *res = PcgResult();
  int rc = fill(s, g.m, 0.0, x);
  if (!rc) rc = copy(s, g.m, b, r);
  if (!rc) rc = sumsq(s, g.m, b, v.scal + 1, v.red);
  if (rc) return rc;
  double nb2;
  rc = read_scalars(&nb2, v.scal + 1, 1, s);
  if (rc) return rc;
  const double nb = std::sqrt(nb2);
  if (nb == 0.0) {
    res->relres = 0.0;
    return DNGD_OK;
  }
  bool f64 = (lp == nullptr);
  double last_true = nb;  // norm of the last true (or initial) residual
  double rho = 0.0;
  auto restart = [&]() -> int {
    int e = precond_apply(h, P, v, sm, r, z, tlv, s);
    if (!e) e = copy(s, g.m, z, p);
    if (!e) e = dot(s, g.m, r, z, v.scal + 0, v.red);
    if (!e) e = read_scalars(&rho, v.scal + 0, 1, s);
    return e;
  };
  rc = restart();
  if (rc) return rc;
  for (int64_t j = 0; j < maxit; ++j) {
    rc = f64 ? kvp(h, theta, P.lambda, v, p, Ap, s)
             : kvp_lp(h, theta, P.lambda, *lp, p, v.t, Ap, s);
    if (!rc) rc = dot(s, g.m, p, Ap, v.scal + 2, v.red);
    if (rc) return rc;
    if (f64) ++res->kvp_f64;
    double pAp;
    rc = read_scalars(&pAp, v.scal + 2, 1, s);
    if (rc) return rc;
    if (!(pAp > 0.0) || !std::isfinite(pAp)) return DNGD_ENOCONV;
    const double a = rho / pAp;
    rc = axpy(s, g.m, a, p, x);
    if (!rc) rc = axpy(s, g.m, -a, Ap, r);
    if (!rc) rc = sumsq(s, g.m, r, v.scal + 3, v.red);
    if (rc) return rc;
    double rr;
    rc = read_scalars(&rr, v.scal + 3, 1, s);
    if (rc) return rc;
    res->iters = (int)(j + 1);
    const double rn = std::sqrt(rr);
    res->relres = rn / nb;
    if (!f64 && (rn <= tol * nb || rn <= last_true * 0x1p-10)) {
      // true residual with the FP64 product: r = b - A x
      rc = kvp(h, theta, P.lambda, v, x, Ap, s);
      if (!rc) rc = copy(s, g.m, b, r);
      if (!rc) rc = axpy(s, g.m, -1.0, Ap, r);
      if (!rc) rc = sumsq(s, g.m, r, v.scal + 3, v.red);
      if (!rc) rc = read_scalars(&rr, v.scal + 3, 1, s);
      if (rc) return rc;
      ++res->kvp_f64;
      const double tn = std::sqrt(rr);
      res->relres = tn / nb;
      if (tn <= tol * nb) return DNGD_OK;
      if (!(tn < 0.125 * last_true)) {
        f64 = true;
        res->escalated = 1;
      }
      last_true = tn;
      ++res->replacements;
      rc = restart();
      if (rc) return rc;
      continue;
    }
    if (rn <= tol * nb) return DNGD_OK;
    rc = precond_apply(h, P, v, sm, r, z, tlv, s);
    if (!rc) rc = dot(s, g.m, r, z, v.scal + 4, v.red);
    if (rc) return rc;
    double rho_new;
    rc = read_scalars(&rho_new, v.scal + 4, 1, s);
    if (rc) return rc;
    if (!(rho > 0.0) || !std::isfinite(rho_new)) return DNGD_ENOCONV;
    rc = xpby(s, g.m, z, rho_new / rho, p);
    if (rc) return rc;
    rho = rho_new;
  }
  return DNGD_ENOCONV;
}

}  // namespace

extern "C" {

int dngd_nystrom_pcg(dngd_problem* h, const double* theta, double lambda, const int64_t* landmarks,
                     int64_t ell, double tol, int64_t maxit, const double* b, double* x,
                     dngd_step_stats* stats, void* stream) {
  DNGD_REQUIRE(h && theta && landmarks && b && x, "dngd_nystrom_pcg: null argument");
  DNGD_REQUIRE(ell >= 1 && ell <= h->g.m, "dngd_nystrom_pcg: ell out of range");
  DNGD_REQUIRE(h->g.pde != DNGD_NAVIER_STOKES,
               "dngd_nystrom_pcg: scalar residual classes only (one residual per point)");
  DNGD_REQUIRE(lambda > 0.0 && std::isfinite(lambda), "dngd_nystrom_pcg: lambda must be > 0");
  DNGD_REQUIRE(tol >= 0.0 && maxit >= 0, "dngd_nystrom_pcg: bad tol/maxit");
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  StepVecs v;
  Small sm;
  int rc = carve_vecs(h, v);
  if (!rc) rc = carve_small(h, sm);
  if (!rc) rc = forward(h, theta, nullptr, s);
  if (rc) return rc;
  h->pc_age = -1;  // K's buffer is rebuilt here
  Precond P;
  rc = pcg_build(h, theta, lambda, landmarks, ell, P, s);
  if (rc) return rc;
  PcgResult pr;
  const int st = pcg_solve(h, theta, P, v, sm, b, x, tol, maxit, &pr, s);
  if (st < 0) return st;
  DNGD_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->pcg_iterations = pr.iters;
    stats->pcg_converged = (st == DNGD_OK);
    stats->pcg_rel_residual = pr.relres;
    stats->nystrom_shift = P.delta;
    stats->nystrom_reused = 0;
    stats->pcg_kvp_f64 = pr.kvp_f64;
    stats->pcg_replacements = 0;  // FP64 products: the recursive residual is the true one
    stats->pcg_escalated = 0;
  }
  return st;
}

int dngd_kvp(dngd_problem* h, const double* theta, double lambda, const double* p, double* w,
             int32_t dtype, void* stream) {
  DNGD_REQUIRE(h && theta && p && w, "dngd_kvp: null argument");
  DNGD_REQUIRE(p != w, "dngd_kvp: w must not alias p");
  DNGD_REQUIRE(dtype == DNGD_F64 || dtype == DNGD_BF16, "dngd_kvp: dtype DNGD_F64 or DNGD_BF16");
  DNGD_REQUIRE(std::isfinite(lambda), "dngd_kvp: lambda must be finite");
  DNGD_REQUIRE(h->g.pde != DNGD_NAVIER_STOKES || dtype == DNGD_F64,
               "dngd_kvp: bf16 products for scalar residual classes only");
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  StepVecs v;
  int rc = carve_vecs(h, v);
  if (!rc) rc = forward(h, theta, nullptr, s);
  if (rc) return rc;
  if (dtype == DNGD_F64) return kvp(h, theta, lambda, v, p, w, s);
  LowpBufs b;
  rc = lp_prepare(h, theta, b, s);
  if (rc) return rc;
  return kvp_lp(h, theta, lambda, b, p, v.t, w, s);
}

int dngd_step(dngd_problem* h, const double* theta, double lambda, const dngd_step_opts* opts,
              double* dtheta, dngd_step_stats* stats, void* stream) {
  DNGD_REQUIRE(h && theta && dtheta, "dngd_step: null argument");
  DNGD_REQUIRE(lambda > 0.0 && std::isfinite(lambda), "dngd_step: lambda must be > 0");
  dngd_step_opts def;
  dngd_step_opts_default(&def);
  const dngd_step_opts& o = opts ? *opts : def;
  DNGD_REQUIRE(o.precision == DNGD_PLAIN || o.precision == DNGD_MIXED, "bad precision");
  DNGD_REQUIRE(o.solver == DNGD_DENSE || o.solver == DNGD_PCG || o.solver == DNGD_PRIMAL ||
                   o.solver == DNGD_DENSE_AUTO || o.solver == DNGD_STRUCTURED,
               "bad solver");
  DNGD_REQUIRE(o.ir_sweeps >= 0 && o.ir_sweeps <= 8, "ir_sweeps must be in [0, 8]");
  DNGD_REQUIRE(o.nystrom_chunk_rows >= 0 && o.nystrom_reuse >= 0, "bad Nystrom options");
  DNGD_REQUIRE(o.pcg_kvp == DNGD_F64 || o.pcg_kvp == DNGD_BF16,
               "pcg_kvp must be DNGD_F64 or DNGD_BF16");
  DNGD_REQUIRE(o.gram_passes == 0 || o.gram_passes == 1 || o.gram_passes == 3 ||
                   o.gram_passes == 4 || o.gram_passes == DNGD_GRAM_F64,
               "bad gram_passes");
  const Geometry& g = h->g;
  DNGD_REQUIRE(g.pde != DNGD_NAVIER_STOKES || o.solver == DNGD_DENSE || o.solver == DNGD_PRIMAL ||
                   o.solver == DNGD_DENSE_AUTO,
               "vector-valued residuals: dense solvers only (DNGD_DENSE, DNGD_PRIMAL, "
               "DNGD_DENSE_AUTO)");
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  StepVecs v;
  Small sm;
  int rc = carve_vecs(h, v);
  if (!rc) rc = carve_small(h, sm);
  if (rc) return rc;
  dngd_step_stats st;
  std::memset(&st, 0, sizeof(st));
  DNGD_HIP(hipEventRecord(h->ev[0], s));

  if (o.solver == DNGD_PCG) {
    DNGD_REQUIRE(o.landmarks && o.n_landmarks >= 1 && o.n_landmarks <= g.m, "PCG needs landmarks");
    rc = forward(h, theta, v.r, s);
    if (!rc) rc = check_finite_residual(v, g.m, s);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[1], s));
    // the Nystrom factors of an earlier PCG step on this handle are reused for
    // up to nystrom_reuse further steps (only G is refactored when lambda
    // changes); otherwise they are rebuilt from this step's landmarks
    const bool reuse = o.nystrom_reuse > 0 && h->pc_age >= 0 && h->pc_age < o.nystrom_reuse &&
                       h->pc.ell == o.n_landmarks;
    if (reuse) {
      if (h->pc.lambda != lambda) rc = pcg_factor_G(h, h->pc, lambda, s);
      ++h->pc_age;
    } else {
      h->pc_age = -1;
      rc = pcg_build(h, theta, lambda, o.landmarks, o.n_landmarks, h->pc, s,
                     o.nystrom_chunk_rows);
      if (!rc) h->pc_age = 0;
    }
    if (rc) return rc;
    const Precond& P = h->pc;
    st.nystrom_shift = P.delta;
    st.nystrom_reused = reuse ? 1 : 0;
    DNGD_HIP(hipEventRecord(h->ev[2], s));
    // bf16 products: the per-step copies of the activations and weights
    LowpBufs lpb;
    const LowpBufs* lp = nullptr;
    if (o.pcg_kvp == DNGD_BF16) {
      rc = lp_prepare(h, theta, lpb, s);
      if (rc) return rc;
      lp = &lpb;
    }
    // the dual solution alpha goes to v.fvv (pcg_solve works in s, tmpm, rownorm2, alpha)
    PcgResult pr, pr_ga;
    const int pst =
        pcg_solve(h, theta, P, v, sm, v.r, v.fvv, o.pcg_tol, o.pcg_maxit, &pr, s, lp);
    if (pst < 0) return pst;
    if (o.alpha_out) {
      rc = copy(s, g.m, v.fvv, o.alpha_out);
      if (rc) return rc;
    }
    // v = -J^T alpha (matrix-free reverse pass); dtheta = v unless GA is accepted
    rc = vjp(h, theta, v.fvv, v.t, s);
    if (!rc) rc = fill(s, g.n, 0.0, v.v);
    if (!rc) rc = axpy(s, g.n, -1.0, v.t, v.v);
    if (!rc) rc = copy(s, g.n, v.v, dtheta);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[3], s));
    // GA (Section 3.2, with the same preconditioner, Remark 3.5): f_vv along v,
    // beta from a second PCG solve, a = -J^T beta, combined as in the dense path
    int pst_ga = DNGD_OK;
    if (o.ga) {
      rc = tangent(h, theta, v.v, 2, v.fvv, s);
      if (!rc && o.fvv_out) rc = copy(s, g.m, v.fvv, o.fvv_out);
      if (rc) return rc;
      DNGD_HIP(hipEventRecord(h->ev[5], s));
      pst_ga = pcg_solve(h, theta, P, v, sm, v.fvv, v.beta, o.pcg_tol, o.pcg_maxit, &pr_ga, s,
                         lp);
      if (pst_ga < 0 && pst_ga != DNGD_ENOCONV) return pst_ga;
      if (pst_ga == DNGD_OK) {
        rc = vjp(h, theta, v.beta, v.t, s);
        if (!rc) rc = fill(s, g.n, 0.0, v.a);
        if (!rc) rc = axpy(s, g.n, -1.0, v.t, v.a);
        if (!rc) rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
        if (!rc) rc = sumsq(s, g.n, v.a, v.scal + 1, v.red);
        if (!rc) rc = ga_combine(s, g.n, v.v, v.a, v.scal, o.eps_norm, dtheta, sm.ga_flag);
        if (rc) return rc;
      }
    } else {
      DNGD_HIP(hipEventRecord(h->ev[5], s));
    }
    if (!o.ga || pst_ga != DNGD_OK) {
      // no correction: dtheta = v as copied above
      rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
      if (!rc) rc = fill(s, 1, 0.0, v.scal + 1);
      if (rc) return rc;
    }
    DNGD_HIP(hipEventRecord(h->ev[7], s));
    double nv[2] = {0, 0};
    int gaf = 0;
    rc = read_back(h, s, {{nv, v.scal, sizeof(nv)},
                          {&gaf, sm.ga_flag, (o.ga && pst_ga == DNGD_OK) ? sizeof(int) : 0}});
    if (rc) return rc;
    float ms = 0;
    hipEventElapsedTime(&ms, h->ev[0], h->ev[7]);
    st.ms_total = ms;
    hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
    st.ms_residual_jacobian = ms;
    hipEventElapsedTime(&ms, h->ev[1], h->ev[2]);
    st.ms_factor = ms;
    hipEventElapsedTime(&ms, h->ev[2], h->ev[3]);
    st.ms_solve_v = ms;
    if (o.ga) {
      hipEventElapsedTime(&ms, h->ev[3], h->ev[5]);
      st.ms_fvv = ms;
      hipEventElapsedTime(&ms, h->ev[5], h->ev[7]);
      st.ms_solve_a = ms;
    }
    st.vnorm = std::sqrt(nv[0]);
    st.anorm = std::sqrt(nv[1]);
    st.ga_accepted = (o.ga && pst_ga == DNGD_OK) ? gaf : 0;
    st.pcg_iterations = pr.iters;
    st.pcg_iterations_ga = pr_ga.iters;
    st.pcg_converged = (pst == DNGD_OK);
    st.pcg_rel_residual = pr.relres;
    st.pcg_kvp_f64 = pr.kvp_f64 + pr_ga.kvp_f64;
    st.pcg_replacements = pr.replacements + pr_ga.replacements;
    st.pcg_escalated = (pr.escalated || pr_ga.escalated) ? 1 : 0;
    if (stats) *stats = st;
    if (pst == DNGD_OK && (!std::isfinite(st.vnorm) || !std::isfinite(st.anorm))) {
      set_error("non-finite step");
      return DNGD_ENAN;
    }
    return pst;
  }

  // ---------------- dense dual solver on the structured FP64 kernel (J never formed) ------
  if (o.solver == DNGD_STRUCTURED) {
    rc = forward(h, theta, v.r, s);
    if (!rc) rc = check_finite_residual(v, g.m, s);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[1], s));
    h->pc_age = -1;  // K's buffer no longer holds a Nystrom preconditioner
    rc = ensure(h, h->K, (size_t)g.m * g.m * 8);
    if (!rc) rc = ensure(h, h->solve_aux, chol_solve_aux_bytes(g.m));
    if (rc) return rc;
    h->ldK = g.m;
    double* K = static_cast<double*>(h->K.p);
    DNGD_HIP(hipEventRecord(h->ev[8], s));
    rc = structured_gram(h, theta, lambda, K, g.m, s);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[9], s));
    DNGD_HIP(hipEventRecord(h->ev[2], s));
    double* aux = static_cast<double*>(h->solve_aux.p);
    rc = o.no_lookahead ? chol_factor(s, g.m, K, g.m, sm.info, aux, nullptr)
                        : chol_factor(s, g.m, K, g.m, sm.info, aux, nullptr, h->side, h->cev[0],
                                      h->cev[1]);
    if (!rc) rc = chol_prepare_solve(s, g.m, K, g.m, aux);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[3], s));
    // alpha = (K + lam I)^{-1} r; v = -J^T alpha (matrix-free reverse pass)
    rc = copy(s, g.m, v.r, v.alpha);
    if (!rc) rc = chol_solve(s, g.m, K, g.m, aux, v.alpha);
    if (!rc && o.alpha_out) rc = copy(s, g.m, v.alpha, o.alpha_out);
    if (!rc) rc = vjp(h, theta, v.alpha, v.t, s);
    if (!rc) rc = fill(s, g.n, 0.0, v.v);
    if (!rc) rc = axpy(s, g.n, -1.0, v.t, v.v);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[4], s));
    if (o.ga) {
      rc = tangent(h, theta, v.v, 2, v.fvv, s);
      if (!rc && o.fvv_out) rc = copy(s, g.m, v.fvv, o.fvv_out);
      if (rc) return rc;
      DNGD_HIP(hipEventRecord(h->ev[5], s));
      rc = copy(s, g.m, v.fvv, v.beta);
      if (!rc) rc = chol_solve(s, g.m, K, g.m, aux, v.beta);
      if (!rc) rc = vjp(h, theta, v.beta, v.t, s);
      if (!rc) rc = fill(s, g.n, 0.0, v.a);
      if (!rc) rc = axpy(s, g.n, -1.0, v.t, v.a);
      if (!rc) rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
      if (!rc) rc = sumsq(s, g.n, v.a, v.scal + 1, v.red);
      if (!rc) rc = ga_combine(s, g.n, v.v, v.a, v.scal, o.eps_norm, dtheta, sm.ga_flag);
      if (rc) return rc;
    } else {
      DNGD_HIP(hipEventRecord(h->ev[5], s));
      rc = copy(s, g.n, v.v, dtheta);
      if (!rc) rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
      if (rc) return rc;
    }
    DNGD_HIP(hipEventRecord(h->ev[6], s));
    double sc[2] = {0, 0};
    int gaf = 0;
    int64_t info = 0;
    rc = read_back(h, s, {{sc, v.scal, sizeof(sc)}, {&info, sm.info, 8},
                          {&gaf, sm.ga_flag, sizeof(int)}});
    if (rc) return rc;
    float ms = 0;
    hipEventElapsedTime(&ms, h->ev[0], h->ev[6]);
    st.ms_total = ms;
    hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
    st.ms_residual_jacobian = ms;
    hipEventElapsedTime(&ms, h->ev[1], h->ev[2]);
    st.ms_gram = ms;
    hipEventElapsedTime(&ms, h->ev[8], h->ev[9]);
    st.ms_gram_kernel = ms;
    hipEventElapsedTime(&ms, h->ev[2], h->ev[3]);
    st.ms_factor = ms;
    hipEventElapsedTime(&ms, h->ev[3], h->ev[4]);
    st.ms_solve_v = ms;
    hipEventElapsedTime(&ms, h->ev[4], h->ev[5]);
    st.ms_fvv = ms;
    hipEventElapsedTime(&ms, h->ev[5], h->ev[6]);
    st.ms_solve_a = ms;
    st.vnorm = std::sqrt(sc[0]);
    st.anorm = o.ga ? std::sqrt(sc[1]) : 0.0;
    st.ga_accepted = o.ga ? gaf : 0;
    st.gram_passes_used = DNGD_GRAM_F64;
    st.gram_attempts = 1;
    if (stats) *stats = st;
    if (info != 0) {
      set_error("Cholesky of K + lambda I: non-positive pivot at column %lld", (long long)info);
      return DNGD_ENOTPD;
    }
    if (!std::isfinite(st.vnorm) || !std::isfinite(st.anorm)) {
      set_error("non-finite step");
      return DNGD_ENAN;
    }
    return DNGD_OK;
  }

  // ---------------- dense solvers: dual (Section 4.1) or primal (Proposition 3.1) --------
  const int jd = (o.precision == DNGD_PLAIN) ? DNGD_F64 : DNGD_F32;
  const size_t esz = (jd == DNGD_F64) ? 8 : 4;
  // the primal system is n x n, the dual m x m: same step, the smaller solve
  const bool primal = o.solver == DNGD_PRIMAL || (o.solver == DNGD_DENSE_AUTO && g.n < g.m);
  const int64_t ldJ = round_up(g.n, 256);
  rc = ensure(h, h->J, (size_t)g.m * ldJ * esz);
  if (rc) return rc;
  h->ldJ = ldJ;
  h->J_dtype = jd;
  void* J = h->J.p;

  // residual + Jacobian (Section 2.2); ||r||^2 flags a non-finite theta or point
  rc = forward(h, theta, v.r, s);
  if (!rc) rc = sumsq(s, g.m, v.r, v.scal + 30, v.red);
  if (!rc) rc = jacobian_all(h, theta, J, ldJ, jd, v.rownorm2, s);
  if (rc) return rc;

  // the operator of K = A A^T + lam I and the first system K x = b:
  // dual A = J, b = r, x = alpha; primal A = J^T, b = J^T r, x = -v
  DenseOp op;
  const double* rhs1;
  double* x1;
  const double* diag;  // ||A_i||^2, the diagonal of K
  if (primal) {
    const int64_t ldJt = round_up(g.m, 256);
    rc = ensure(h, h->Jt, (size_t)g.n * ldJt * esz);
    if (!rc) rc = transpose_rm(s, g.m, g.n, J, ldJ, jd, h->Jt.p, ldJt);
    if (!rc) rc = rownorm2(s, g.n, g.m, h->Jt.p, ldJt, jd, v.ps);
    if (!rc) rc = gemv_t(s, g.m, g.n, J, ldJ, jd, v.r, 1.0, v.pg, v.gemv_work);
    if (rc) return rc;
    op = DenseOp{h->Jt.p, g.n, g.m, ldJt, jd, v.tmpm, v.ps};
    rhs1 = v.pg;
    x1 = v.px;
    diag = v.ps;
  } else {
    op = DenseOp{J, g.m, g.n, ldJ, jd, v.t, v.s};
    rhs1 = v.r;
    x1 = v.alpha;
    diag = v.rownorm2;
  }
  DNGD_HIP(hipEventRecord(h->ev[1], s));

  // Gram K = A A^T + lam I
  int passes = 1;
  if (jd == DNGD_F32) {
    passes = o.gram_passes;
    // D = max_i ||A_i||^2 (reduced on the device): decides the bf16 split when
    // passes == 0 (auto); it and ||r||^2 come back in one read
    rc = vmax(s, op.M, diag, v.scal + 31, v.red);
    if (rc) return rc;
    double rd[2];
    {
      const int rb_ = read_back(h, s, {{rd, v.scal + 30, sizeof(rd)}});
      if (rb_) return rb_;
    }
    const double dmax = std::max(rd[1], 0.0);
    st.max_row_norm2 = rd[1];
    if (!std::isfinite(rd[0]) || !std::isfinite(rd[1])) {
      if (stats) *stats = st;
      set_error("non-finite residual or Jacobian at theta (||r||^2 = %g, max ||J_i||^2 = %g)",
                rd[0], rd[1]);
      return DNGD_ENAN;
    }
    if (passes == 0) {
      // bf16 unit roundoff 2^-8 times sqrt(D / lam) estimates the refinement
      // contraction of a 1-pass Gram; split when it would exceed 1/50. The
      // split without lo lo^T is indefinite by ~2^-16 D: keep it only while
      // that is below lam / 10, else add the fourth product.
      if (std::ldexp(1.0, -8) * std::sqrt(dmax / lambda) <= 0.02) passes = 1;
      else if (std::ldexp(1.0, -16) * dmax <= 0.1 * lambda) passes = 3;
      else passes = 4;
    }
  }
  h->pc_age = -1;  // K's buffer no longer holds a Nystrom preconditioner
  rc = ensure(h, h->K, (size_t)op.M * op.M * 8);
  if (!rc) rc = ensure(h, h->solve_aux, chol_solve_aux_bytes(op.M));
  if (rc) return rc;
  h->ldK = op.M;
  double* K = static_cast<double*>(h->K.p);
  const int ir = (jd == DNGD_F32) ? o.ir_sweeps : 0;
  const bool adaptive = (jd == DNGD_F32 && o.gram_passes == 0);
  if (adaptive && h->gram_hint != 0) {
    // tiers are ordered 1 < 3 < 4 < DNGD_GRAM_F64 by value; a smaller damping
    // only makes the system harder, a larger one drops the memory
    if (h->gram_hint_primal == primal && lambda <= h->gram_hint_lambda)
      passes = std::max(passes, h->gram_hint);
    else
      h->gram_hint = 0;
  }
  st.gram_start_passes = passes;
  int64_t info = 0;
  int attempts = 0;
  for (;;) {
    ++attempts;
    const size_t gw = gram_workspace_bytes(op.M, op.N, jd, passes, nullptr);
    rc = ensure(h, h->gram_work, gw);
    if (!rc)
      rc = gram_launch(s, op.M, op.N, op.A, op.ldA, jd, passes, lambda, K, op.M,
                       h->gram_work.p, gw, h->ev[8], h->ev[9]);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[2], s));
    // Cholesky of K + lam I
    double* cwork = static_cast<double*>(h->solve_aux.p);  // reused by the solves after
    rc = o.no_lookahead ? chol_factor(s, op.M, K, op.M, sm.info, cwork, nullptr)
                        : chol_factor(s, op.M, K, op.M, sm.info, cwork, nullptr, h->side,
                                      h->cev[0], h->cev[1]);
    if (rc) return rc;
    const bool can_escalate = adaptive && passes != DNGD_GRAM_F64;
    if (can_escalate) {
      {
        const int rb_ = read_back(h, s, {{&info, sm.info, 8}});
        if (rb_) return rb_;
      }
      if (info != 0) {  // K~ + lam I not positive definite in this precision
        passes = (passes == 4) ? DNGD_GRAM_F64 : 4;
        continue;
      }
    }
    rc = chol_prepare_solve(s, op.M, K, op.M, static_cast<double*>(h->solve_aux.p));
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[3], s));

    // x = (K + lam I)^{-1} b (+ refinement)
    rc = dense_solve(h, op, v, rhs1, x1, lambda, ir, v.scal + 16, s);
    if (rc) return rc;
    if (can_escalate && ir > 0) {
      // refinement did not bring the residual below ir_tol: the Gram is too
      // coarse for this damping
      double sc2[9];
      rc = sumsq(s, op.M, rhs1, v.scal + 15, v.red);
      if (rc) return rc;
      {
        const int rb_ = read_back(h, s, {{sc2, v.scal + 15, sizeof(sc2)}});
        if (rb_) return rb_;
      }
      const double nr = std::sqrt(sc2[0]);
      const double last = nr > 0 ? std::sqrt(sc2[1 + std::min(ir, 8) - 1]) / nr : 0.0;
      if (!(last <= o.ir_tol)) {
        passes = DNGD_GRAM_F64;
        continue;
      }
    }
    break;
  }
  st.gram_passes_used = passes;
  st.gram_attempts = attempts;
  if (adaptive && attempts > 1) {
    h->gram_hint = passes;
    h->gram_hint_lambda = lambda;
    h->gram_hint_primal = primal;
  }
  // v = -J^T alpha (dual) or v = -x (primal)
  if (primal) {
    rc = fill(s, g.n, 0.0, v.v);
    if (!rc) rc = axpy(s, g.n, -1.0, x1, v.v);
  } else {
    rc = gemv_t(s, g.m, g.n, J, ldJ, jd, x1, -1.0, v.v, v.gemv_work);
    if (!rc && o.alpha_out) rc = copy(s, g.m, x1, o.alpha_out);
  }
  if (rc) return rc;
  DNGD_HIP(hipEventRecord(h->ev[4], s));

  if (o.ga) {
    // f_vv along v (Section 3.2); a = -J^T (K + lam I)^{-1} f_vv (dual) or
    // a = -(J^T J + lam I)^{-1} J^T f_vv (primal). The mixed step takes the
    // hidden layers' products in FP32 on the matrix cores (jet rules in FP64).
    rc = tangent(h, theta, v.v, 2, v.fvv, s, jd == DNGD_F32);
    if (!rc && o.fvv_out) rc = copy(s, g.m, v.fvv, o.fvv_out);
    if (rc) return rc;
    DNGD_HIP(hipEventRecord(h->ev[5], s));
    bool combined = false;  // dtheta and the GA flag already written
    if (primal) {
      rc = gemv_t(s, g.m, g.n, J, ldJ, jd, v.fvv, 1.0, v.t, v.gemv_work);
      if (!rc) rc = dense_solve(h, op, v, v.t, v.px, lambda, ir, nullptr, s);
      if (!rc) rc = fill(s, g.n, 0.0, v.a);
      if (!rc) rc = axpy(s, g.n, -1.0, v.px, v.a);
    } else if (ir > 0) {
      combined = true;
      const double* aux = static_cast<const double*>(h->solve_aux.p);
      // beta in stages. With beta0 the unrefined solve, t = J^T beta0 (so
      // a0 = -t) and s0 = f_vv - (J t + lam beta0) -- the first refinement
      // sweep's residual -- the refined a satisfies
      //   ||a - a0|| = ||J^T (K + lam I)^{-1} s0|| <= ||s0|| / (2 sqrt(lam))
      // (max over singular values of sigma / (sigma^2 + lam)). When even
      // ||a0|| minus that bound fails the acceptance test, the correction is
      // rejected for certain: the rest of its refinement is skipped and
      // dtheta = v, as the full computation would give.
      rc = copy(s, g.m, v.fvv, v.beta);
      if (!rc) rc = chol_solve(s, g.m, K, g.m, aux, v.beta);
      if (!rc) rc = refine_residual(op, v, v.fvv, v.beta, lambda, s);
      if (!rc) rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
      if (!rc) rc = sumsq(s, g.n, op.tN, v.scal + 1, v.red);
      if (!rc) rc = sumsq(s, g.m, op.sM, v.scal + 2, v.red);
      if (rc) return rc;
      double nr[3];
      {
        const int rb_ = read_back(h, s, {{nr, v.scal, sizeof(nr)}});
        if (rb_) return rb_;
      }
      const double nv = std::sqrt(nr[0]);
      const double a_low = std::sqrt(nr[1]) - std::sqrt(nr[2]) / (2.0 * std::sqrt(lambda));
      if (nv > o.eps_norm && 2.0 * a_low > 0.5 * nv) {
        st.ga_early_reject = 1;  // scal[1] holds ||a0||^2: the combine rejects, dtheta = v
        rc = ga_combine(s, g.n, v.v, v.a, v.scal, o.eps_norm, dtheta, sm.ga_flag);
        if (rc) return rc;
      } else {
        rc = refine_correct(h, op, v.beta, s);
        for (int k = 1; k < ir && !rc; ++k) {
          rc = refine_residual(op, v, v.fvv, v.beta, lambda, s);
          if (!rc) rc = refine_correct(h, op, v.beta, s);
        }
        if (!rc) rc = gemv_t(s, g.m, g.n, J, ldJ, jd, v.beta, -1.0, v.a, v.gemv_work);
        if (!rc) rc = sumsq(s, g.n, v.a, v.scal + 1, v.red);
        if (!rc) rc = ga_combine(s, g.n, v.v, v.a, v.scal, o.eps_norm, dtheta, sm.ga_flag);
        if (rc) return rc;
      }
    } else {
      rc = dense_solve(h, op, v, v.fvv, v.beta, lambda, ir, nullptr, s);
      if (!rc) rc = gemv_t(s, g.m, g.n, J, ldJ, jd, v.beta, -1.0, v.a, v.gemv_work);
    }
    if (!combined) {
      if (!rc) rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
      if (!rc) rc = sumsq(s, g.n, v.a, v.scal + 1, v.red);
      if (!rc) rc = ga_combine(s, g.n, v.v, v.a, v.scal, o.eps_norm, dtheta, sm.ga_flag);
    }
    if (rc) return rc;
  } else {
    DNGD_HIP(hipEventRecord(h->ev[5], s));
    rc = copy(s, g.n, v.v, dtheta);
    if (!rc) rc = sumsq(s, g.n, v.v, v.scal + 0, v.red);
    if (rc) return rc;
  }
  if (ir > 0) {
    rc = sumsq(s, op.M, rhs1, v.scal + 15, v.red);
    if (rc) return rc;
  }
  DNGD_HIP(hipEventRecord(h->ev[6], s));

  double sc[32];
  int gaf = 0;
  rc = read_back(h, s, {{sc, v.scal, sizeof(sc)}, {&info, sm.info, 8},
                        {&gaf, sm.ga_flag, sizeof(int)}});
  if (rc) return rc;
  float ms = 0;
  hipEventElapsedTime(&ms, h->ev[0], h->ev[6]);
  st.ms_total = ms;
  hipEventElapsedTime(&ms, h->ev[0], h->ev[1]);
  st.ms_residual_jacobian = ms;
  hipEventElapsedTime(&ms, h->ev[1], h->ev[2]);
  st.ms_gram = ms;
  hipEventElapsedTime(&ms, h->ev[8], h->ev[9]);
  st.ms_gram_kernel = ms;
  hipEventElapsedTime(&ms, h->ev[2], h->ev[3]);
  st.ms_factor = ms;
  hipEventElapsedTime(&ms, h->ev[3], h->ev[4]);
  st.ms_solve_v = ms;
  hipEventElapsedTime(&ms, h->ev[4], h->ev[5]);
  st.ms_fvv = ms;
  hipEventElapsedTime(&ms, h->ev[5], h->ev[6]);
  st.ms_solve_a = ms;
  st.vnorm = std::sqrt(sc[0]);
  st.anorm = o.ga ? std::sqrt(sc[1]) : 0.0;
  st.ga_accepted = o.ga ? gaf : 0;
  st.primal = primal ? 1 : 0;
  if (ir > 0) {
    const double nr = std::sqrt(sc[15]);
    for (int k = 0; k < ir && k < 8; ++k) st.ir_residual[k] = nr > 0 ? std::sqrt(sc[16 + k]) / nr : 0;
  }
  if (stats) *stats = st;
  if (!std::isfinite(sc[30])) {
    set_error("non-finite residual at theta (||r||^2 = %g)", sc[30]);
    return DNGD_ENAN;
  }
  if (info != 0) {
    set_error("Cholesky of K + lambda I: non-positive pivot at column %lld", (long long)info);
    return DNGD_ENOTPD;
  }
  if (!std::isfinite(st.vnorm) || !std::isfinite(st.anorm)) {
    set_error("non-finite step");
    return DNGD_ENAN;
  }
  return DNGD_OK;
}


// One iteration of the D-NGD workflow (damping rule, step, grid line search,
// update), see include/dngd.h.
int dngd_iterate(dngd_problem* h, double* theta, double lambda_cap, double lambda_fixed,
                 const dngd_step_opts* opts, int32_t n_eta, const double* etas, double* dtheta,
                 dngd_iter_stats* stats, void* stream) {
  DNGD_REQUIRE(h && theta && etas && n_eta > 0 && n_eta <= 48, "dngd_iterate: bad argument");
  DNGD_REQUIRE((lambda_fixed > 0.0 && std::isfinite(lambda_fixed)) ||
                   (lambda_fixed == 0.0 && lambda_cap > 0.0 && std::isfinite(lambda_cap)),
               "dngd_iterate: need lambda_fixed > 0, or lambda_fixed == 0 and lambda_cap > 0");
  for (int k = 0; k < n_eta; ++k)
    DNGD_REQUIRE(std::isfinite(etas[k]), "dngd_iterate: non-finite step length");
  const Geometry& g = h->g;
  hipStream_t s = S(stream);
  CallScope scope(h, s);
  int rc = ensure(h, h->iter, (size_t)g.n * sizeof(double));
  if (rc) return rc;
  double* dth = static_cast<double*>(h->iter.p);
  StepVecs v;
  rc = carve_vecs(h, v);
  if (rc) return rc;

  // L(theta_k) and the damping lambda_k = min(L(theta_k), cap)
  rc = forward(h, theta, v.tmpm, s);
  if (!rc) rc = sumsq(s, g.m, v.tmpm, v.scal + 56, v.red);
  if (rc) return rc;
  double rr = 0.0;
  {
    const int rb_ = read_back(h, s, {{&rr, v.scal + 56, 8}});
    if (rb_) return rb_;
  }
  const double L0 = 0.5 * rr;
  DNGD_REQUIRE(std::isfinite(L0), "dngd_iterate: non-finite loss at theta");
  double lam = (lambda_fixed > 0.0) ? lambda_fixed : std::min(L0, lambda_cap);
  lam = std::max(lam, 1e-300);  // L = 0 exactly: any positive damping gives dtheta = 0

  dngd_iter_stats st;
  std::memset(&st, 0, sizeof(st));
  const int sst = dngd_step(h, theta, lam, opts, dth, &st.step, stream);
  if (sst < 0) return sst;

  // grid line search: the first minimiser wins ties; NaN losses never win
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> L(n_eta);
  rc = losses_impl(h, theta, dth, n_eta, etas, L.data(), s);
  if (rc) return rc;
  int best = -1;
  for (int k = 0; k < n_eta; ++k)
    if (std::isfinite(L[k]) && (best < 0 || L[k] < L[best])) best = k;
  DNGD_REQUIRE(best >= 0, "dngd_iterate: every line-search loss is non-finite");
  rc = axpy(s, g.n, etas[best], dth, theta);
  if (!rc && dtheta) rc = copy(s, g.n, dth, dtheta);
  if (rc) return rc;
  DNGD_HIP(hipStreamSynchronize(s));
  st.ms_line_search =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  st.loss = L0;
  st.lambda = lam;
  st.eta = etas[best];
  st.eta_index = best;
  st.loss_new = L[best];
  st.step_status = sst;
  if (stats) *stats = st;
  return sst;
}

}  // extern "C"
