"""Oracle: vector-valued residual classes for the steady incompressible
Navier-Stokes equations (FP64 CPU).

Test infrastructure only (see ``oracle/__init__.py``).

The network maps a point (x, y) to three outputs (u, v, p). Section 5.3
(Kovasznay flow) states the equations: the momentum balance
(u . grad) u + grad p - nu lap u = 0 and the continuity equation div u = 0.
A residual class gamma contributes N_gamma points of output dimension d_gamma
(the residual-space size m = sum_gamma N_gamma d_gamma of the abstract and the
class split of the AssembleGramian algorithm):

  interior point i (d = 3, scale c = N_int^{-1/2}):
      r_i0 = c (u u_x + v u_y + p_x - nu (u_xx + u_yy) - f_i0)   x-momentum
      r_i1 = c (u v_x + v v_y + p_y - nu (v_xx + v_yy) - f_i1)   y-momentum
      r_i2 = c (u_x + v_y - f_i2)                                continuity
  boundary point j (d = 3, scale N_bdy^{-1/2}):
      r_jk = c (out_k(x_j) - g_jk),  out = (u, v, p)             prescribed values

Rows are point-major inside a class (the d x d blocks of the KernelEntry
algorithm), interior class first. The source f is zero for Kovasznay flow and
kept as an input for generality.

How each piece is computed (no hand-derived derivative of the operator):
  * the output jets (value, gradient, Laplacian of u, v, p) come from the
    forward jets of ``network.forward`` with three outputs;
  * the operator N above is written once, in ``operator``, for any arithmetic
    with +, - and *;
  * J's rows: by the chain rule, d r_ik / d theta = sum_ch (d N_k / d U_ch)
    (d U_ch / d theta). The derivatives d N_k / d U_ch of the polynomial N are
    taken by complex step on ``operator`` (exact to rounding for a
    polynomial), and contracted with d U / d theta by the reverse pass over the
    jets (``network._jacobian_class``, pinned by complex step on theta);
  * f_vv = d^2/dt^2 r(theta + t v): the output jets' t-derivatives z0, z1, z2
    along the line (``network.t_jets``) enter ``operator`` as truncated
    Taylor numbers z0 + t z1 + t^2/2 z2; f_vv is twice the t^2 coefficient.
"""
from __future__ import annotations

import numpy as np

from . import network

NAVIER_STOKES = network.NAVIER_STOKES
D_INT = 3   # residual components per interior point
D_BDY = 3   # residual components per boundary point
N_OUT = 3   # network outputs (u, v, p)


def operator(ch, nu):
    """(x-momentum, y-momentum, continuity) from the output channels ``ch``:
    a dict with u, v, p_x, p_y, u_x, u_y, v_x, v_y, lap_u, lap_v (any type with
    +, - and *)."""
    mx = ch["u"] * ch["u_x"] + ch["v"] * ch["u_y"] + ch["p_x"] - nu * ch["lap_u"]
    my = ch["u"] * ch["v_x"] + ch["v"] * ch["v_y"] + ch["p_y"] - nu * ch["lap_v"]
    cont = ch["u_x"] + ch["v_y"]
    return mx, my, cont


# channel name -> (kind, spatial index, output index) in an output jet
CHANNELS = {
    "u": ("v", None, 0), "v": ("v", None, 1), "p": ("v", None, 2),
    "u_x": ("g", 0, 0), "u_y": ("g", 1, 0),
    "v_x": ("g", 0, 1), "v_y": ("g", 1, 1),
    "p_x": ("g", 0, 2), "p_y": ("g", 1, 2),
    "lap_u": ("l", None, 0), "lap_v": ("l", None, 1), "lap_p": ("l", None, 2),
}


def channels(U: network.Jet):
    """The operator's inputs from an output jet with three outputs."""
    out = {}
    for name, (kind, k, o) in CHANNELS.items():
        if kind == "v":
            out[name] = U.v[:, o]
        elif kind == "g":
            out[name] = U.g[:, k, o]
        else:
            out[name] = U.l[:, o]
    return out


def class_scales(problem):
    return tuple((1.0 / np.sqrt(n)) if n > 0 else 0.0 for n in (problem.n_int, problem.n_bdy))


def _interior_jet(problem, theta):
    return network.forward(theta, problem.widths, problem.x_int, 2)


def _boundary_jet(problem, theta):
    return network.forward(theta, problem.widths, problem.x_bdy, 2)


def residual(problem, theta):
    """r(theta) in R^m (m = 3 N_int + 3 N_bdy), point-major per class."""
    ci, cb = class_scales(problem)
    nu = problem.kappa
    parts = []
    if problem.n_int:
        N = np.stack(operator(channels(_interior_jet(problem, theta)), nu), axis=1)
        parts.append((ci * (N - problem.f_int.reshape(-1, D_INT))).ravel())
    if problem.n_bdy:
        U = _boundary_jet(problem, theta)
        parts.append((cb * (U.v - problem.g_bdy.reshape(-1, D_BDY))).ravel())
    return np.concatenate(parts)


def operator_partials(U: network.Jet, nu, h=1e-30):
    """d N_k / d (channel) at every point, by complex step on ``operator``:
    returns for k = 0, 1, 2 the seeds (seed_v (N, 3), seed_g (N, 2, 3),
    seed_l (N, 3)) of the linear functional sum_ch dN_k/dU_ch U_ch."""
    base = {k: x.astype(np.complex128) for k, x in channels(U).items()}
    Npts = U.v.shape[0]
    seeds = [(np.zeros((Npts, N_OUT)), np.zeros((Npts, 2, N_OUT)), np.zeros((Npts, N_OUT)))
             for _ in range(D_INT)]
    for name, (kind, k, o) in CHANNELS.items():
        ch = dict(base)
        ch[name] = base[name] + 1j * h
        out = operator(ch, nu)
        for comp in range(D_INT):
            d = np.imag(out[comp]) / h
            sv, sg, sl = seeds[comp]
            if kind == "v":
                sv[:, o] = d
            elif kind == "g":
                sg[:, k, o] = d
            else:
                sl[:, o] = d
    return seeds


def jacobian(problem, theta, chunk=256):
    """J = d r / d theta (m x n), rows in residual order."""
    ci, cb = class_scales(problem)
    nu = problem.kappa
    n = network.n_params(problem.widths)
    blocks = []
    for s0 in range(0, problem.n_int, chunk):
        x = problem.x_int[s0:s0 + chunk]
        U = network.forward(theta, problem.widths, x, 2)
        rows = np.empty((x.shape[0], D_INT, n))
        for k, (sv, sg, sl) in enumerate(operator_partials(U, nu)):
            rows[:, k] = network._jacobian_class(theta, problem.widths, x, 2,
                                                 ci * sv, ci * sg, ci * sl)
        blocks.append(rows.reshape(-1, n))
    for s0 in range(0, problem.n_bdy, chunk):
        x = problem.x_bdy[s0:s0 + chunk]
        Nx = x.shape[0]
        rows = np.empty((Nx, D_BDY, n))
        for k in range(D_BDY):
            sv = np.zeros((Nx, N_OUT))
            sv[:, k] = cb
            rows[:, k] = network._jacobian_class(theta, problem.widths, x, 2, sv,
                                                 np.zeros((Nx, 2, N_OUT)), np.zeros((Nx, N_OUT)))
        blocks.append(rows.reshape(-1, n))
    return np.concatenate(blocks, axis=0)


class Taylor2:
    """Truncated Taylor number a0 + a1 t + a2 t^2 (arrays; products drop t^3)."""

    def __init__(self, a0, a1, a2):
        self.a = (a0, a1, a2)

    @staticmethod
    def _lift(x):
        return x if isinstance(x, Taylor2) else Taylor2(x, 0.0, 0.0)

    def __add__(self, o):
        o = Taylor2._lift(o)
        return Taylor2(*(p + q for p, q in zip(self.a, o.a)))

    __radd__ = __add__

    def __sub__(self, o):
        o = Taylor2._lift(o)
        return Taylor2(*(p - q for p, q in zip(self.a, o.a)))

    def __rsub__(self, o):
        return Taylor2._lift(o) - self

    def __mul__(self, o):
        if not isinstance(o, Taylor2):
            return Taylor2(*(o * p for p in self.a))
        a, b = self.a, o.a
        return Taylor2(a[0] * b[0], a[0] * b[1] + a[1] * b[0],
                       a[0] * b[2] + a[1] * b[1] + a[2] * b[0])

    __rmul__ = __mul__


def fvv(problem, theta, v):
    """f_vv = d^2/dt^2 r(theta + t v) at t = 0 (Section 3.2)."""
    ci, cb = class_scales(problem)
    nu = problem.kappa
    parts = []
    if problem.n_int:
        z0, z1, z2 = network.t_jets(theta, v, problem.widths, problem.x_int, 2)
        c0, c1, c2 = channels(z0), channels(z1), channels(z2)
        ch = {k: Taylor2(c0[k], c1[k], 0.5 * c2[k]) for k in c0}
        out = operator(ch, nu)
        parts.append((ci * np.stack([2.0 * o.a[2] for o in out], axis=1)).ravel())
    if problem.n_bdy:
        _, _, z2 = network.t_jets(theta, v, problem.widths, problem.x_bdy, 2)
        parts.append((cb * z2.v).ravel())
    return np.concatenate(parts)


def velocity_relative_l2(theta, widths, x, uv_exact):
    """||(u, v)_theta - (u, v)*|| / ||(u, v)*|| over the points x."""
    a = x
    layers = network.unpack(theta, widths)
    for li, (W, b) in enumerate(layers):
        a = a @ W.T + b
        if li < len(layers) - 1:
            a = np.tanh(a)
    return float(np.linalg.norm(a[:, :2] - uv_exact) / np.linalg.norm(uv_exact))
