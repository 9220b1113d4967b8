"""Oracle: the PINN residual map of a tanh MLP and its derivatives (FP64 CPU).

Test infrastructure only (see ``oracle/__init__.py``).

Residuals follow Section 2.2 (residuals and Jacobian): for interior points
``r_i = N_int^{-1/2} (L u(x_i) - f(x_i))`` and for boundary / initial points
``r_j = N^{-1/2} (u(x_j) - g(x_j))``, concatenated interior, boundary, initial.
``L u = -lap u`` (Poisson) or ``u_t - kappa lap_xy u`` (heat). The input
Laplacian is taken in forward (Taylor) mode, as the experiments section says
the derivatives are: each activation carries a *spatial jet* (value, input
gradient, input Laplacian).

Jet rules used throughout (plain calculus):
  product:   (pq).v = p.v q.v,  (pq).g = p.v q.g + q.v p.g,
             (pq).l = p.v q.l + q.v p.l + 2 <p.g, q.g>_lap
  function:  phi(s) = (phi(s.v), phi'(s.v) s.g, phi'(s.v) s.l + phi''(s.v) |s.g|^2_lap)
where ``<.,.>_lap`` sums over the Laplacian coordinates only.

Parameter layout: per layer ``W`` row-major ``[out][in]`` then ``b[out]``.

All functions accept complex ``theta`` (complex-step differentiation pins the
Jacobian), so nothing here forces a float dtype.
"""
from __future__ import annotations

import numpy as np

POISSON = 0
HEAT = 1
NAVIER_STOKES = 2   # vector-valued residual classes: oracle/navier_stokes.py


def _ns():
    from . import navier_stokes
    return navier_stokes


# ----------------------------------------------------------------------------
# parameters


def unpack(theta, widths):
    """Split flat theta into [(W_l, b_l)] (views)."""
    out, o = [], 0
    for l in range(len(widths) - 1):
        fin, fout = widths[l], widths[l + 1]
        W = theta[o:o + fin * fout].reshape(fout, fin)
        o += fin * fout
        b = theta[o:o + fout]
        o += fout
        out.append((W, b))
    assert o == theta.shape[0], (o, theta.shape)
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def n_params(widths):
    return sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1))


# ----------------------------------------------------------------------------
# tanh and its derivatives, written in terms of a = tanh(z)


def tanh_derivs(z, order):
    """[tanh(z), tanh'(z), ..., tanh^(order)(z)]."""
    a = np.tanh(z)
    s1 = 1.0 - a * a
    ds = [a, s1]
    if order >= 2:
        ds.append(-2.0 * a * s1)
    if order >= 3:
        ds.append(s1 * (6.0 * a * a - 2.0))
    if order >= 4:
        ds.append(8.0 * a * s1 * (2.0 - 3.0 * a * a))
    return ds[:order + 1]


# ----------------------------------------------------------------------------
# spatial jets: (v, g, l) with v (N, w), g (N, d, w), l (N, w)


class Jet:
    """Value, input gradient and input Laplacian of a batch of fields.

    ``nlap`` = number of leading input coordinates the Laplacian sums over.
    """

    def __init__(self, v, g, l, nlap):
        self.v, self.g, self.l, self.nlap = v, g, l, nlap

    def glap_dot(self, other):
        return np.einsum("ndw,ndw->nw", self.g[:, :self.nlap], other.g[:, :self.nlap])

    def __add__(self, o):
        return Jet(self.v + o.v, self.g + o.g, self.l + o.l, self.nlap)

    def scale(self, c):
        return Jet(c * self.v, c * self.g, c * self.l, self.nlap)

    def mul(self, o):
        """Jet of the pointwise product (product rule, Laplacian cross term)."""
        return Jet(self.v * o.v,
                   self.v[:, None] * o.g + o.v[:, None] * self.g,
                   self.v * o.l + o.v * self.l + 2.0 * self.glap_dot(o),
                   self.nlap)

    def affine(self, W, b=None):
        """Jet of x -> W x + b (b enters the value only)."""
        v = self.v @ W.T
        if b is not None:
            v = v + b
        return Jet(v, self.g @ W.T, self.l @ W.T, self.nlap)


def apply_fn(derivs_at_v, s: Jet) -> Jet:
    """phi(s) from [phi(s.v), phi'(s.v), phi''(s.v)] (chain rule for value,
    gradient and Laplacian)."""
    p0, p1, p2 = derivs_at_v
    gg = np.einsum("ndw,ndw->nw", s.g[:, :s.nlap], s.g[:, :s.nlap])
    return Jet(p0, p1[:, None] * s.g, p1 * s.l + p2 * gg, s.nlap)


def input_jet(x, nlap):
    """Jet of the identity map on the inputs: value x, gradient e_k, Laplacian 0."""
    N, d = x.shape
    g = np.broadcast_to(np.eye(d, dtype=x.dtype), (N, d, d)).copy()
    return Jet(x.copy(), g, np.zeros_like(x), nlap)


def nlap_of(problem):
    return problem.d_in - 1 if problem.pde == HEAT else problem.d_in


# ----------------------------------------------------------------------------
# forward pass and residual (Section 2.2)


def forward(theta, widths, x, nlap, keep=False):
    """MLP forward on jets. Returns the output jet (width 1) and, if ``keep``,
    the per-layer (pre-activation jet z_l, post-activation jet a_l) list."""
    layers = unpack(theta, widths)
    a = input_jet(x, nlap)
    tape = [(None, a)]
    for li, (W, b) in enumerate(layers):
        z = a.affine(W, b)
        if li == len(layers) - 1:
            tape.append((z, z))
            return (z, tape) if keep else z
        a = apply_fn(tanh_derivs(z.v, 2), z)
        tape.append((z, a))


def class_scales(problem):
    """c_gamma = N_gamma^{-1/2} for interior, boundary, initial."""
    return tuple((1.0 / np.sqrt(n)) if n > 0 else 0.0
                 for n in (problem.n_int, problem.n_bdy, problem.n_init))


def interior_operator(problem, u: Jet):
    """L u at interior points: -lap u (Poisson) or u_t - kappa lap_xy u (heat)."""
    if problem.pde == POISSON:
        return -u.l[:, 0]
    return u.g[:, problem.d_in - 1, 0] - problem.kappa * u.l[:, 0]


def residual(problem, theta):
    """r(theta) in R^m, order interior, boundary, initial (Section 2.2)."""
    if problem.pde == NAVIER_STOKES:
        return _ns().residual(problem, theta)
    ci, cb, c0 = class_scales(problem)
    nl = nlap_of(problem)
    parts = []
    if problem.n_int:
        u = forward(theta, problem.widths, problem.x_int, nl)
        parts.append(ci * (interior_operator(problem, u) - problem.f_int))
    if problem.n_bdy:
        u = forward(theta, problem.widths, problem.x_bdy, nl)
        parts.append(cb * (u.v[:, 0] - problem.g_bdy))
    if problem.n_init:
        u = forward(theta, problem.widths, problem.x_init, nl)
        parts.append(c0 * (u.v[:, 0] - problem.g_init))
    return np.concatenate(parts)


def loss(problem, theta):
    r = residual(problem, theta)
    return 0.5 * float(np.real(r @ r))


def u_value(theta, widths, x):
    """Network output u_theta(x) (no derivatives)."""
    a = x
    layers = unpack(theta, widths)
    for li, (W, b) in enumerate(layers):
        a = a @ W.T + b
        if li < len(layers) - 1:
            a = np.tanh(a)
    return a[:, 0]


def relative_l2(problem, theta, x_eval, u_exact):
    u = u_value(theta, problem.widths, x_eval)
    return float(np.linalg.norm(u - u_exact) / np.linalg.norm(u_exact))


# ----------------------------------------------------------------------------
# Jacobian J = d r / d theta by reverse mode over the jets (Section 2.2)


def _tanh_jet_adjoint(z: Jet, abar: Jet) -> Jet:
    """Adjoint of a = phi(z) (the jet function rule above) for phi = tanh:
    returns zbar given abar. Derived term by term from
      a.v = s0, a.g = s1 z.g, a.l = s1 z.l + s2 |z.g|^2_lap."""
    s0, s1, s2, s3 = tanh_derivs(z.v, 3)
    nl = z.nlap
    gg = np.einsum("ndw,ndw->nw", z.g[:, :nl], z.g[:, :nl])
    # d/dz.v of each output channel, contracted with its adjoint
    vbar = (abar.v * s1
            + s2 * np.einsum("ndw,ndw->nw", abar.g, z.g)
            + abar.l * (s2 * z.l + s3 * gg))
    gbar = s1[:, None] * abar.g
    gbar[:, :nl] += 2.0 * (abar.l * s2)[:, None] * z.g[:, :nl]
    lbar = abar.l * s1
    return Jet(vbar, gbar, lbar, nl)


def _tape_class(theta, widths, x, nlap, seed_v, seed_g, seed_l):
    """Reverse pass over the jets of one point class: for every affine layer l,
    its input jet a_{l-1} and the adjoint zbar_l of its output jet, where the
    output jet's adjoint is the seed. A row of J is then, per layer,
    W_l-bar = sum over channels of zbar_l (x) a_{l-1} and b_l-bar = zbar_l.v.
    Seeds are per-point arrays: (N,), (N, d), (N,) for one output, or with a
    trailing output axis (N, o), (N, d, o), (N, o) for o outputs."""
    layers = unpack(theta, widths)
    _, tape = forward(theta, widths, x, nlap, keep=True)
    if seed_v.ndim == 1:
        seed_v, seed_g, seed_l = seed_v[:, None], seed_g[:, :, None], seed_l[:, None]
    # adjoint of the output jet
    zbar = Jet(seed_v.astype(theta.dtype), seed_g.astype(theta.dtype),
               seed_l.astype(theta.dtype), nlap)
    out = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        out[li] = (tape[li][1], zbar)
        if li == 0:
            break
        abar = Jet(zbar.v @ W, zbar.g @ W, zbar.l @ W, nlap)
        zbar = _tanh_jet_adjoint(tape[li][0], abar)
    return out


def _layer_rows(a_prev: Jet, zbar: Jet, o0=0, o1=None):
    """J's columns of W_l rows o0..o1 (row-major [out][in]) and of b_l[o0:o1]
    for the points of one class: z = a_prev W^T + b on every channel, so
    W-bar[o][i] = sum_ch zbar_ch[o] a_prev_ch[i] and b-bar = zbar.v."""
    zv, zg, zl = zbar.v[:, o0:o1], zbar.g[:, :, o0:o1], zbar.l[:, o0:o1]
    Wbar = (np.einsum("no,ni->noi", zv, a_prev.v)
            + np.einsum("ndo,ndi->noi", zg, a_prev.g)
            + np.einsum("no,ni->noi", zl, a_prev.l))
    return Wbar.reshape(Wbar.shape[0], -1), zv.copy()


def _jacobian_class(theta, widths, x, nlap, seed_v, seed_g, seed_l):
    """Rows d r_i / d theta for one point class, where r_i is the linear
    functional seed_v*u.v + <seed_g, u.g> + seed_l*u.l of the output jet at x_i
    (seed shapes as in _tape_class). Returns (N, n)."""
    tape = _tape_class(theta, widths, x, nlap, seed_v, seed_g, seed_l)
    return np.concatenate([np.concatenate(_layer_rows(a, z), axis=1) for a, z in tape], axis=1)


def _class_seeds(problem, c, N):
    """Output-jet seeds of the residuals of class c (0 interior, 1 boundary,
    2 initial) at N points, scalar residual families: r_i is c_gamma times a
    linear functional of the output jet (Section 2.2)."""
    ci, cb, c0 = class_scales(problem)
    d = problem.d_in
    sv, sg, sl = np.zeros(N), np.zeros((N, d)), np.zeros(N)
    if c == 0 and problem.pde == POISSON:
        sl[:] = -ci
    elif c == 0:
        sg[:, d - 1] = ci
        sl[:] = -ci * problem.kappa
    else:
        sv[:] = cb if c == 1 else c0
    return sv, sg, sl


def jacobian(problem, theta, chunk=512):
    """J = d r / d theta in R^{m x n}, rows in residual order, columns in the
    flat parameter layout."""
    if problem.pde == NAVIER_STOKES:
        return _ns().jacobian(problem, theta)
    nl = nlap_of(problem)
    rows = []
    for c, (N, x) in enumerate(((problem.n_int, problem.x_int), (problem.n_bdy, problem.x_bdy),
                                (problem.n_init, problem.x_init))):
        if not N:
            continue
        sv, sg, sl = _class_seeds(problem, c, N)
        for s0 in range(0, N, chunk):
            e = slice(s0, s0 + chunk)
            rows.append(_jacobian_class(theta, problem.widths, x[e], nl, sv[e], sg[e], sl[e]))
    return np.concatenate(rows, axis=0)


# ----------------------------------------------------------------------------
# Jacobians too large to form (FP64 J of the heat workload is 207 GB): the
# same reverse pass, kept per layer for all residuals, gives column blocks of J
# and the product J^T p without the whole matrix.


def layer_tapes(problem, theta, weights=None):
    """Per class, the reverse pass's (a_{l-1}, zbar_l) of every layer
    (``_tape_class``), scalar residual families. With ``weights`` (m) the seeds
    of residual i are multiplied by weights[i] (the adjoints of J^T weights)."""
    nl = nlap_of(problem)
    out, off = [], 0
    for c, (N, x) in enumerate(((problem.n_int, problem.x_int), (problem.n_bdy, problem.x_bdy),
                                (problem.n_init, problem.x_init))):
        if not N:
            continue
        sv, sg, sl = _class_seeds(problem, c, N)
        if weights is not None:
            w = weights[off:off + N]
            sv, sg, sl = sv * w, sg * w[:, None], sl * w
        out.append(_tape_class(theta, problem.widths, x, nl, sv, sg, sl))
        off += N
    return out


def jacobian_block(tapes, l, o0, o1):
    """Columns of J for W_l rows o0..o1 (contiguous in theta) and for
    b_l[o0:o1] (contiguous), all m rows: (m x (o1-o0) w_{l-1}, m x (o1-o0))."""
    parts = [_layer_rows(t[l][0], t[l][1], o0, o1) for t in tapes]
    return (np.concatenate([p[0] for p in parts], axis=0),
            np.concatenate([p[1] for p in parts], axis=0))


def vjp(problem, theta, p):
    """J^T p without forming J: the reverse pass with residual i's seed scaled
    by p_i, its weight gradients summed over the points (Section 2.2, where
    the loss gradient is J^T r)."""
    if problem.pde == NAVIER_STOKES:
        return jacobian(problem, theta).T @ p
    tapes = layer_tapes(problem, theta, weights=p)
    grads = []
    for l in range(len(problem.widths) - 1):
        Wg, bg = 0.0, 0.0
        for t in tapes:
            a, z = t[l]
            Wg = Wg + z.v.T @ a.v + np.einsum("ndo,ndi->oi", z.g, a.g) + z.l.T @ a.l
            bg = bg + z.v.sum(axis=0)
        grads.append(np.concatenate([np.ravel(Wg), bg]))
    return np.concatenate(grads)


def _class_of(problem, idx):
    """(class, point) for residual indices idx (order interior, boundary, initial)."""
    idx = np.asarray(idx, dtype=np.int64)
    b0, b1 = problem.n_int, problem.n_int + problem.n_bdy
    cls = np.where(idx < b0, 0, np.where(idx < b1, 1, 2))
    pt = np.where(cls == 0, idx, np.where(cls == 1, idx - b0, idx - b1))
    return cls, pt


def _class_points(problem, c):
    return (problem.x_int, problem.x_bdy, problem.x_init)[c]


def residual_rows(problem, theta, idx):
    """Entries idx of r(theta), each computed from its own point only (a
    residual depends on one collocation point)."""
    ci, cb, c0 = class_scales(problem)
    nl = nlap_of(problem)
    cls, pt = _class_of(problem, idx)
    out = np.empty(len(cls), dtype=np.result_type(theta, np.float64))
    for c, scale in ((0, ci), (1, cb), (2, c0)):
        sel = np.nonzero(cls == c)[0]
        if not len(sel):
            continue
        u = forward(theta, problem.widths, _class_points(problem, c)[pt[sel]], nl)
        if c == 0:
            out[sel] = scale * (interior_operator(problem, u) - problem.f_int[pt[sel]])
        else:
            tgt = problem.g_bdy if c == 1 else problem.g_init
            out[sel] = scale * (u.v[:, 0] - tgt[pt[sel]])
    return out


def jacobian_rows(problem, theta, idx):
    """Rows idx of J, each from its own point (seeds as in ``jacobian``)."""
    nl = nlap_of(problem)
    cls, pt = _class_of(problem, idx)
    out = np.empty((len(cls), n_params(problem.widths)))
    for c in (0, 1, 2):
        sel = np.nonzero(cls == c)[0]
        if not len(sel):
            continue
        sv, sg, sl = _class_seeds(problem, c, len(sel))
        out[sel] = _jacobian_class(theta, problem.widths, _class_points(problem, c)[pt[sel]], nl,
                                   sv, sg, sl)
    return out


# ----------------------------------------------------------------------------
# f_vv = d^2/dt^2 r(theta + t v) at t = 0 (Section 3.2, geodesic acceleration)


def _jet_fn_jet(dd, z: Jet) -> Jet:
    """The jet of phi^(k)(z) given dd = [phi^(k), phi^(k+1), phi^(k+2)] at z.v."""
    return apply_fn(dd, z)


def fvv_output(theta, v, widths, x, nlap):
    """Second t-derivative of the output jet along theta + t v (see t_jets)."""
    return t_jets(theta, v, widths, x, nlap)[2]


def t_jets(theta, v, widths, x, nlap):
    """The output jet and its first and second t-derivatives along theta + t v.

    Each layer carries the t-Taylor coefficients (as derivatives) z0, z1, z2 of
    its pre-activation, each a spatial jet. With W(t) = W + tV, b(t) = b + tc:
      z0 = W a0 + b,  z1 = W a1 + V a0 + c,  z2 = W a2 + 2 V a1,
      a0 = s(z0),     a1 = s'(z0) z1,        a2 = s'(z0) z2 + s''(z0) z1 z1,
    with s'(z0), s''(z0) themselves jets (function rule) and products by the
    jet product rule."""
    lay = unpack(theta, widths)
    vl = unpack(v, widths)
    a0 = input_jet(x, nlap)
    zero = Jet(np.zeros_like(a0.v), np.zeros_like(a0.g), np.zeros_like(a0.l), nlap)
    a1, a2 = zero, zero
    L = len(lay)
    for li in range(L):
        (W, b), (V, c) = lay[li], vl[li]
        z0 = a0.affine(W, b)
        z1 = a1.affine(W) + a0.affine(V, c)
        z2 = a2.affine(W) + a1.affine(V).scale(2.0)
        if li == L - 1:
            return z0, z1, z2
        d = tanh_derivs(z0.v, 4)
        s_1 = _jet_fn_jet(d[1:4], z0)   # jet of tanh'(z0)
        s_2 = _jet_fn_jet(d[2:5], z0)   # jet of tanh''(z0)
        a0 = apply_fn(d[0:3], z0)
        a1 = s_1.mul(z1)
        a2 = s_1.mul(z2) + s_2.mul(z1.mul(z1))


def fvv(problem, theta, v):
    """f_vv in R^m: the residual's second directional derivative along v.
    Targets f, g drop out (they do not depend on theta)."""
    if problem.pde == NAVIER_STOKES:
        return _ns().fvv(problem, theta, v)
    ci, cb, c0 = class_scales(problem)
    nl = nlap_of(problem)
    parts = []
    if problem.n_int:
        u2 = fvv_output(theta, v, problem.widths, problem.x_int, nl)
        parts.append(ci * interior_operator(problem, u2))
    for N, x, c in ((problem.n_bdy, problem.x_bdy, cb), (problem.n_init, problem.x_init, c0)):
        if N:
            u2 = fvv_output(theta, v, problem.widths, x, nl)
            parts.append(c * u2.v[:, 0])
    return np.concatenate(parts)


def fvv_rows(problem, theta, v, idx):
    """Entries idx of f_vv, each from its own point."""
    ci, cb, c0 = class_scales(problem)
    nl = nlap_of(problem)
    cls, pt = _class_of(problem, idx)
    out = np.empty(len(cls))
    for c, scale in ((0, ci), (1, cb), (2, c0)):
        sel = np.nonzero(cls == c)[0]
        if not len(sel):
            continue
        u2 = fvv_output(theta, v, problem.widths, _class_points(problem, c)[pt[sel]], nl)
        out[sel] = scale * (interior_operator(problem, u2) if c == 0 else u2.v[:, 0])
    return out
