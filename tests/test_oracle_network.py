"""Pins for the oracle's residual map, Jacobian and f_vv against things other
than the oracle itself: closed forms, complex-step and finite-difference
derivatives, torch's autograd (an independent library AD) and exact
invariants of the second directional derivative (Section 3.2)."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N


def tiny_poisson(widths=(2, 5, 4, 1), n_int=7, n_bdy=5, seed=3):
    return W.poisson_problem(list(widths), n_int, n_bdy, "sinsin", seed)


def tiny_heat(widths=(3, 6, 5, 1), seed=4):
    return W.heat_problem(list(widths), 6, 4, 3, 0.1, seed)


def rand_theta(widths, seed, scale=1.0):
    # nonzero biases so every term of the chain rule is exercised
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(N.n_params(widths))


# ----------------------------------------------------------------------------
# residual / Laplacian


def test_one_hidden_layer_closed_form():
    """u = sum_j c_j tanh(w_j.x + b_j) + b0  =>  lap u = sum_j c_j tanh''(z_j) |w_j|^2,
    grad u = sum_j c_j tanh'(z_j) w_j (direct differentiation)."""
    rng = np.random.default_rng(0)
    d, h = 4, 9
    W1 = rng.standard_normal((h, d))
    b1 = rng.standard_normal(h)
    c = rng.standard_normal((1, h))
    b0 = rng.standard_normal(1)
    theta = N.pack([(W1, b1), (c, b0)])
    x = rng.uniform(size=(13, d))
    u = N.forward(theta, [d, h, 1], x, nlap=d)
    z = x @ W1.T + b1
    t = np.tanh(z)
    lap = ((c[0] * (-2 * t * (1 - t * t))) * (W1 ** 2).sum(1)).sum(1)
    grad = ((c[0] * (1 - t * t))[:, :, None] * W1[None]).sum(1)
    val = (c[0] * t).sum(1) + b0
    assert np.allclose(u.v[:, 0], val, rtol=0, atol=1e-13)
    assert np.allclose(u.g[:, :, 0], grad, rtol=0, atol=1e-13)
    assert np.allclose(u.l[:, 0], lap, rtol=0, atol=1e-12)
    # partial Laplacian over the first 2 coordinates only (heat layout)
    u2 = N.forward(theta, [d, h, 1], x, nlap=2)
    lap2 = ((c[0] * (-2 * t * (1 - t * t))) * (W1[:, :2] ** 2).sum(1)).sum(1)
    assert np.allclose(u2.l[:, 0], lap2, rtol=0, atol=1e-12)


def test_zero_hidden_layers_has_zero_laplacian():
    rng = np.random.default_rng(1)
    theta = rng.standard_normal(4)
    u = N.forward(theta, [3, 1], rng.uniform(size=(5, 3)), nlap=3)
    assert np.all(u.l == 0.0)


def test_residual_assembly_constant_network():
    """All weights zero => u = b_out: r_int = c(-0 - f), r_bdy = c(b_out - g)."""
    p = tiny_poisson()
    th = np.zeros(N.n_params(p.widths))
    th[-1] = 0.7
    r = N.residual(p, th)
    ci, cb = 1 / np.sqrt(p.n_int), 1 / np.sqrt(p.n_bdy)
    assert np.allclose(r[:p.n_int], -ci * p.f_int, atol=1e-15)
    assert np.allclose(r[p.n_int:], cb * (0.7 - p.g_bdy), atol=1e-15)
    h = tiny_heat()
    th = np.zeros(N.n_params(h.widths))
    th[-1] = -0.3
    r = N.residual(h, th)
    assert r.shape == (h.m,)
    assert np.allclose(r[:h.n_int], 0.0)
    c0 = 1 / np.sqrt(h.n_init)
    assert np.allclose(r[h.n_int + h.n_bdy:], c0 * (-0.3 - h.g_init))


def _torch_u_derivs(theta, widths, x, nlap):
    """Value, gradient and Laplacian by torch autograd (hessian trace)."""
    torch = pytest.importorskip("torch")
    th = torch.tensor(theta, dtype=torch.float64)
    xs = torch.tensor(x, dtype=torch.float64)

    def u(xi):
        a = xi
        o = 0
        L = len(widths) - 1
        for l in range(L):
            fin, fout = widths[l], widths[l + 1]
            Wl = th[o:o + fin * fout].reshape(fout, fin)
            o += fin * fout
            bl = th[o:o + fout]
            o += fout
            a = Wl @ a + bl
            if l < L - 1:
                a = torch.tanh(a)
        return a[0]

    vals = torch.stack([u(xi) for xi in xs])
    grads = torch.stack([torch.func.grad(u)(xi) for xi in xs])
    laps = torch.stack([torch.diagonal(torch.func.hessian(u)(xi))[:nlap].sum() for xi in xs])
    return vals.numpy(), grads.numpy(), laps.numpy()


def test_deep_jets_match_torch_autograd():
    widths = [3, 8, 7, 6, 1]
    th = rand_theta(widths, 5, 0.6)
    x = np.random.default_rng(6).uniform(size=(9, 3))
    for nlap in (3, 2):
        u = N.forward(th, widths, x, nlap)
        v, g, l = _torch_u_derivs(th, widths, x, nlap)
        assert np.allclose(u.v[:, 0], v, atol=1e-13)
        assert np.allclose(u.g[:, :, 0], g, atol=1e-13)
        assert np.allclose(u.l[:, 0], l, atol=1e-12)


def test_laplacian_central_differences():
    widths = [2, 32, 32, 1]
    th = W.glorot_theta(widths, 0)
    x = np.random.default_rng(2).uniform(size=(6, 2))
    u = N.forward(th, widths, x, 2)

    def lap_fd(h):
        tot = 0
        for k in range(2):
            e = np.zeros(2)
            e[k] = h
            tot = tot + (N.u_value(th, widths, x + e) - 2 * N.u_value(th, widths, x)
                         + N.u_value(th, widths, x - e)) / h ** 2
        return tot

    rich = (4 * lap_fd(1e-3) - lap_fd(2e-3)) / 3
    assert np.allclose(u.l[:, 0], rich, rtol=1e-6, atol=1e-7)


# ----------------------------------------------------------------------------
# Jacobian


def _complex_step_jacobian(p, th, h=1e-30):
    n = th.size
    J = np.zeros((p.m, n))
    for k in range(n):
        tc = th.astype(np.complex128)
        tc[k] += 1j * h
        J[:, k] = np.imag(N.residual(p, tc)) / h
    return J


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_jacobian_complex_step(kind):
    p = tiny_poisson() if kind == "poisson" else tiny_heat()
    th = rand_theta(p.widths, 11, 0.7)
    J = N.jacobian(p, th)
    Jc = _complex_step_jacobian(p, th)
    scale = np.abs(Jc).max()
    assert np.abs(J - Jc).max() <= 1e-13 * scale


def test_jacobian_torch_jacrev_config0():
    torch = pytest.importorskip("torch")
    p = W.config(0)
    th = W.glorot_theta(p.widths, 0)
    J = N.jacobian(p, th)
    widths = p.widths
    xi = torch.tensor(p.x_int)
    xb = torch.tensor(p.x_bdy)
    f = torch.tensor(p.f_int)
    g = torch.tensor(p.g_bdy)

    def u_of(thv, x):
        a = x
        o = 0
        L = len(widths) - 1
        for l in range(L):
            fin, fout = widths[l], widths[l + 1]
            Wl = thv[o:o + fin * fout].reshape(fout, fin)
            o += fin * fout
            bl = thv[o:o + fout]
            o += fout
            a = Wl @ a + bl
            if l < L - 1:
                a = torch.tanh(a)
        return a[0]

    def res(thv):
        lap = torch.vmap(lambda x: torch.func.hessian(u_of, argnums=1)(thv, x).diagonal().sum())(xi)
        ub = torch.vmap(lambda x: u_of(thv, x))(xb)
        return torch.cat([(-lap - f) / np.sqrt(p.n_int), (ub - g) / np.sqrt(p.n_bdy)])

    Jt = torch.func.jacrev(res)(torch.tensor(th)).numpy()
    assert np.abs(J - Jt).max() <= 1e-12 * np.abs(Jt).max()


def test_jacobian_central_fd_sampled_columns():
    p = W.config(0)
    th = W.glorot_theta(p.widths, 0)
    J = N.jacobian(p, th)
    cols = np.random.default_rng(7).choice(th.size, 12, replace=False)
    for k in cols:
        e = np.zeros_like(th)
        h = 1e-5
        e[k] = h
        fd = (N.residual(p, th + e) - N.residual(p, th - e)) / (2 * h)
        assert np.allclose(J[:, k], fd, rtol=1e-6, atol=1e-8 * np.abs(J).max())


# ----------------------------------------------------------------------------
# f_vv


def _fd_fvv(p, th, v, h):
    return (N.residual(p, th + h * v) - 2 * N.residual(p, th) + N.residual(p, th - h * v)) / h ** 2


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_fvv_second_difference(kind):
    p = tiny_poisson((2, 6, 5, 1)) if kind == "poisson" else tiny_heat()
    th = rand_theta(p.widths, 21, 0.6)
    v = rand_theta(p.widths, 22, 0.3)
    f = N.fvv(p, th, v)
    rich = (4 * _fd_fvv(p, th, v, 1e-3) - _fd_fvv(p, th, v, 2e-3)) / 3
    assert np.allclose(f, rich, rtol=1e-6, atol=1e-7 * np.abs(f).max())


def test_fvv_matches_torch_nested_jvp():
    torch = pytest.importorskip("torch")
    p = tiny_heat((3, 5, 4, 1))
    th = rand_theta(p.widths, 31, 0.6)
    v = rand_theta(p.widths, 32, 0.4)
    widths = p.widths

    def u_of(thv, x):
        a = x
        o = 0
        L = len(widths) - 1
        for l in range(L):
            fin, fout = widths[l], widths[l + 1]
            Wl = thv[o:o + fin * fout].reshape(fout, fin)
            o += fin * fout
            bl = thv[o:o + fout]
            o += fout
            a = Wl @ a + bl
            if l < L - 1:
                a = torch.tanh(a)
        return a[0]

    X = torch.tensor(p.x_int)
    k = p.kappa

    def r_int(thv):
        out = []
        for x in X:
            H = torch.func.hessian(u_of, argnums=1)(thv, x)
            gt = torch.func.grad(u_of, argnums=1)(thv, x)[2]
            out.append(gt - k * (H[0, 0] + H[1, 1]))
        return torch.stack(out) / np.sqrt(p.n_int)

    tt = torch.tensor(th)
    vt = torch.tensor(v)
    first = lambda t_: torch.func.jvp(r_int, (t_,), (vt,))[1]
    second = torch.func.jvp(first, (tt,), (vt,))[1].numpy()
    f = N.fvv(p, th, v)[:p.n_int]
    assert np.allclose(f, second, atol=1e-12 * max(1.0, np.abs(second).max()))


def test_fvv_invariants():
    p = tiny_poisson((2, 6, 5, 1))
    th = rand_theta(p.widths, 41, 0.6)
    v = rand_theta(p.widths, 42, 0.3)
    f = N.fvv(p, th, v)
    # homogeneity of degree 2
    assert np.allclose(N.fvv(p, th, 2.5 * v), 6.25 * f, rtol=1e-13, atol=1e-15)
    # v = 0
    assert np.all(N.fvv(p, th, np.zeros_like(v)) == 0.0)
    # v supported on the output layer only: r is affine along v -> f_vv = 0
    vo = np.zeros_like(v)
    nlast = p.widths[-2] * 1 + 1
    vo[-nlast:] = v[-nlast:]
    assert np.abs(N.fvv(p, th, vo)).max() <= 1e-14


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_row_subsets_match_full_oracle(kind):
    """residual_rows / jacobian_rows / fvv_rows (point by point, used at sizes
    where the full arrays do not fit) equal the rows of the full results."""
    if kind == "poisson":
        p = W.config(0, scale=dict(widths=[2, 9, 7, 1], n_int=30, n_bdy=12))
    else:
        p = W.heat_problem([3, 8, 6, 1], 25, 9, 7, 0.3, 4)
    th = 0.6 * np.random.default_rng(1).standard_normal(N.n_params(p.widths))
    v = np.random.default_rng(2).standard_normal(N.n_params(p.widths))
    idx = np.array([p.m - 1, 0, 3, p.n_int, p.n_int + 1, p.m - 2, 5])
    assert np.array_equal(N.residual_rows(p, th, idx), N.residual(p, th)[idx])
    assert np.allclose(N.jacobian_rows(p, th, idx), N.jacobian(p, th)[idx], rtol=0, atol=1e-14)
    assert np.allclose(N.fvv_rows(p, th, v, idx), N.fvv(p, th, v)[idx], rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("kind", ["poisson", "heat"])
def test_jacobian_blocks_and_vjp_match_the_jacobian(kind):
    """The streamed forms used where J cannot be held (column blocks of J per
    layer, J^T p from the weighted reverse pass) against J itself (pinned by
    complex step above), on Poisson and heat nets."""
    if kind == "poisson":
        p = W.config(0, scale=dict(widths=[2, 7, 6, 1], n_int=20, n_bdy=9))
    else:
        p = W.heat_problem([3, 6, 5, 1], 15, 6, 4, 0.1, 0)
    th = W.glorot_theta(p.widths, 2)
    J = N.jacobian(p, th)
    tapes = N.layer_tapes(p, th)
    Jb = np.full_like(J, np.nan)
    off = 0
    for l in range(len(p.widths) - 1):
        win, wout = p.widths[l], p.widths[l + 1]
        for o0 in range(0, wout, 2):
            o1 = min(wout, o0 + 2)
            Wc, bc = N.jacobian_block(tapes, l, o0, o1)
            Jb[:, off + o0 * win: off + o1 * win] = Wc
            Jb[:, off + wout * win + o0: off + wout * win + o1] = bc
        off += wout * win + wout
    assert off == th.size
    assert np.max(np.abs(Jb - J)) <= 1e-15 * np.max(np.abs(J))
    pv = W.random_direction(p.m, 3)
    g = N.vjp(p, th, pv)
    assert np.linalg.norm(g - J.T @ pv) <= 1e-13 * np.linalg.norm(J.T @ pv)
