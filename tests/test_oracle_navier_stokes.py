"""Pins for the oracle's vector-valued residual classes (steady incompressible
Navier-Stokes, Section 5.3): Kovasznay's closed-form solution makes the
operator vanish, torch autograd reproduces the residual map, complex step
reproduces J, a Richardson second difference in t reproduces f_vv, a
direction that moves only the pressure output gives f_vv = 0, and the dual
step equals the primal one (push-through identity)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import navier_stokes as NS
from oracle import network as N
from oracle import step as S

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def kovasznay_channels(x, nu):
    """Closed-form value, gradient and Laplacian channels of Kovasznay's
    (u, v, p), differentiated by hand: with E = e^{l x}, C = cos 2 pi y,
    S = sin 2 pi y, k = 2 pi:
      u = 1 - E C:       u_x = -l E C,      u_y = k E S,      lap u = -(l^2 - k^2) E C
      v = l/k E S:       v_x = l^2/k E S,   v_y = l E C,      lap v = l/k (l^2 - k^2) E S
      p = (1 - E^2)/2:   p_x = -l E^2,      p_y = 0."""
    lam = 0.5 / nu - math.sqrt(0.25 / nu ** 2 + 4.0 * math.pi ** 2)
    k = 2.0 * math.pi
    E = np.exp(lam * x[:, 0])
    C, Sn = np.cos(k * x[:, 1]), np.sin(k * x[:, 1])
    return {
        "u": 1.0 - E * C, "v": lam / k * E * Sn, "p": 0.5 * (1.0 - E * E),
        "u_x": -lam * E * C, "u_y": k * E * Sn,
        "v_x": lam * lam / k * E * Sn, "v_y": lam * E * C,
        "p_x": -lam * E * E, "p_y": np.zeros_like(E),
        "lap_u": -(lam * lam - k * k) * E * C, "lap_v": lam / k * (lam * lam - k * k) * E * Sn,
        "lap_p": -2.0 * lam * lam * E * E,
    }


def test_hand_derivatives_of_kovasznay_match_finite_differences():
    """The closed-form channels above (the pin's own input) against fourth-order
    central differences of the workload's solution."""
    nu = 1.0 / 40.0
    x = W._rect_interior(np.random.default_rng(0), 50, W.KOVASZNAY_BOX)
    ch = kovasznay_channels(x, nu)
    f = lambda y: W.kovasznay_fields(y, nu)  # noqa: E731
    h = 1e-3
    for j, name in enumerate("uvp"):
        assert np.allclose(f(x)[:, j], ch[name], rtol=0, atol=1e-14)
    grads, laps = {}, 0.0
    for d, ax in enumerate("xy"):
        e = np.zeros(2)
        e[d] = h
        d1 = (-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * h)
        d2 = (-f(x + 2 * e) + 16 * f(x + e) - 30 * f(x) + 16 * f(x - e) - f(x - 2 * e)) / (12 * h * h)
        grads[ax] = d1
        laps = laps + d2
    for j, name in enumerate("uvp"):
        for ax in "xy":
            ref = ch[f"{name}_{ax}"]
            assert np.max(np.abs(grads[ax][:, j] - ref)) <= 1e-7 * (1 + np.max(np.abs(ref)))
        ref = ch[f"lap_{name}"]
        assert np.max(np.abs(laps[:, j] - ref)) <= 1e-5 * (1 + np.max(np.abs(ref)))


def test_operator_vanishes_on_kovasznay_flow():
    """Kovasznay's flow solves the steady equations exactly, term by term large:
    every equation's residual is at rounding level while its terms are O(1).
    A dropped term, a wrong sign or a swapped index fails this."""
    nu = 1.0 / 40.0
    x = W._rect_interior(np.random.default_rng(1), 200, W.KOVASZNAY_BOX)
    ch = kovasznay_channels(x, nu)
    mx, my, cont = NS.operator(ch, nu)
    scale = max(np.max(np.abs(ch[k])) for k in ch)
    for r in (mx, my, cont):
        assert np.max(np.abs(r)) <= 1e-13 * scale
    # the terms themselves are not small (the check is not vacuous)
    assert np.max(np.abs(ch["u"] * ch["u_x"])) > 1.0 and np.max(np.abs(ch["v"] * ch["u_y"])) > 0.1
    assert np.max(np.abs(ch["p_x"])) > 1.0 and np.max(np.abs(nu * ch["lap_v"])) > 0.1
    # and a different viscosity does not solve it
    assert np.max(np.abs(NS.operator(ch, 1.1 * nu)[0])) > 1e-2


def _torch_mlp(theta, widths, x):
    layers = N.unpack(theta, widths)
    a = x
    for li, (Wl, bl) in enumerate(layers):
        a = a @ Wl.T + bl
        if li < len(layers) - 1:
            a = torch.tanh(a)
    return a


def _torch_residual(problem, theta):
    """The same residual map with torch autograd for the input derivatives."""
    th = torch.tensor(theta, dtype=torch.float64)
    nu = problem.kappa
    x = torch.tensor(problem.x_int, dtype=torch.float64, requires_grad=True)
    out = _torch_mlp(th, problem.widths, x)
    g = [torch.autograd.grad(out[:, j].sum(), x, create_graph=True)[0] for j in range(3)]
    lap = [sum(torch.autograd.grad(g[j][:, d].sum(), x, create_graph=True)[0][:, d]
               for d in range(2)) for j in range(2)]
    u, v = out[:, 0], out[:, 1]
    mx = u * g[0][:, 0] + v * g[0][:, 1] + g[2][:, 0] - nu * lap[0]
    my = u * g[1][:, 0] + v * g[1][:, 1] + g[2][:, 1] - nu * lap[1]
    cont = g[0][:, 0] + g[1][:, 1]
    ri = torch.stack([mx, my, cont], 1) - torch.tensor(problem.f_int)
    rb = _torch_mlp(th, problem.widths, torch.tensor(problem.x_bdy)) - torch.tensor(problem.g_bdy)
    ci, cb = problem.n_int ** -0.5, problem.n_bdy ** -0.5
    return torch.cat([(ci * ri).reshape(-1), (cb * rb).reshape(-1)]).detach().numpy()


def test_residual_matches_torch_autograd():
    p = W.kovasznay(widths=[2, 16, 16, 3], n_int=60, n_bdy=40)
    th = W.glorot_theta(p.widths, 2)
    r = N.residual(p, th)
    assert r.shape == (3 * 60 + 3 * 40,)
    assert rel(r, _torch_residual(p, th)) <= 1e-13


def test_jacobian_matches_complex_step_all_columns():
    p = W.kovasznay(widths=[2, 5, 4, 3], n_int=7, n_bdy=5)
    th = W.glorot_theta(p.widths, 3)
    J = N.jacobian(p, th)
    n = th.size
    h = 1e-30
    Jcs = np.empty_like(J)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1j * h
        Jcs[:, j] = np.imag(N.residual(p, th + e)) / h
    assert J.shape == (3 * 7 + 3 * 5, n)
    assert np.max(np.abs(J - Jcs)) <= 1e-13 * np.max(np.abs(Jcs))


def test_jacobian_sampled_columns_at_full_size():
    """The Kovasznay network itself (n = 7953, m = 2400): complex-step columns."""
    p = W.kovasznay()
    th = W.glorot_theta(p.widths, 0)
    J = N.jacobian(p, th)
    cols = np.random.default_rng(9).choice(th.size, 12, replace=False)
    cols = np.concatenate([cols, [0, th.size - 1, th.size - 4]])  # first weight, last biases
    for j in cols:
        e = np.zeros(th.size, dtype=np.complex128)
        e[j] = 1e-30j
        col = np.imag(N.residual(p, th + e)) / 1e-30
        assert np.max(np.abs(J[:, j] - col)) <= 1e-12 * max(np.max(np.abs(col)), 1e-300)


def test_fvv_second_difference_and_invariants():
    p = W.kovasznay(widths=[2, 12, 12, 3], n_int=40, n_bdy=30)
    th = W.glorot_theta(p.widths, 4)
    v = W.random_direction(th.size, 5, 0.3)
    f = N.fvv(p, th, v)

    def d2(h):
        return (N.residual(p, th + h * v) - 2 * N.residual(p, th) + N.residual(p, th - h * v)) / h ** 2

    rich = (4 * d2(5e-4) - d2(1e-3)) / 3
    assert rel(f, rich) <= 1e-7
    assert rel(N.fvv(p, th, 2.0 * v), 4.0 * f) <= 1e-14
    # moving only the pressure output (last layer's row 2 and bias 2) moves r
    # affinely: p, p_x, p_y enter the equations linearly, so f_vv = 0
    L = len(p.widths) - 1
    wlast = p.widths[L - 1]
    vp = np.zeros_like(v)
    off = th.size - (3 * wlast + 3)
    vp[off + 2 * wlast: off + 3 * wlast] = v[: wlast]
    vp[-1] = 0.7
    assert np.max(np.abs(N.fvv(p, th, vp))) <= 1e-13
    # ... while the velocity outputs do not (the convective term is quadratic)
    vu = np.zeros_like(v)
    vu[off: off + wlast] = v[: wlast]
    assert np.max(np.abs(N.fvv(p, th, vu))) > 1e-6


@pytest.mark.parametrize("lam", [1e-3, 1e-5])
def test_dual_step_equals_primal_step(lam):
    """Push-through identity on a Navier-Stokes problem with n > m (dual) ..."""
    p = W.kovasznay(widths=[2, 20, 20, 3], n_int=60, n_bdy=40)
    th = W.glorot_theta(p.widths, 6)
    res = S.dense_step(p, th, lam, ga=True)
    assert res.J.shape == (300, th.size) and th.size > 300
    pr = S.primal_dense_step(p, th, lam, ga=True)
    assert rel(res.v, pr.v) <= 1e-9
    assert rel(res.a, pr.a) <= 1e-9
    assert res.accepted == pr.accepted
