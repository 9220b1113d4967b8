"""Pins for the oracle's dense dual step against the primal normal equations
(push-through identity, Prop. 3.1 / Thm. 3.2), the paper's literal recovery
formulas, first-order optimality of the LM subproblem, the minimum-norm
least-squares limit and the Gramian's defining properties."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N
from oracle import step as S


@pytest.fixture(scope="module")
def c0():
    p = W.config(0)
    th = W.glorot_theta(p.widths, 0)
    return p, th, N.residual(p, th), N.jacobian(p, th)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("lam", [1e-2, 1e-4, 1e-6])
def test_dual_equals_primal_config0(c0, lam):
    """Config 0 (n = 1185) is small enough to solve the n x n primal system."""
    p, th, r, J = c0
    res = S.dense_step(p, th, lam, ga=True, J=J, r=r)
    vp = S.primal_step(J, r, lam)
    assert rel(res.v, vp) <= 1e-9
    ap = S.primal_accel(J, res.fvv, lam)
    assert rel(res.a, ap) <= 1e-9


def test_literal_dual_form_agrees(c0):
    p, th, r, J = c0
    lam = 1e-2
    res = S.dense_step(p, th, lam, ga=True, J=J, r=r)
    v_lit, a_lit = S.literal_dual_step(J, r, lam, res.fvv)
    assert rel(res.v, v_lit) <= 1e-9
    assert rel(res.a, a_lit) <= 1e-8


def test_optimality_and_descent(c0):
    p, th, r, J = c0
    for lam in (1e-3, 1e-6):
        v = S.dense_step(p, th, lam, ga=False, J=J, r=r).v
        g = J.T @ r
        kkt = J.T @ (r + J @ v) + lam * v
        assert np.linalg.norm(kkt) <= 1e-9 * np.linalg.norm(g)
        assert g @ v < 0


def test_min_norm_limit():
    """m < n, full row rank: as lam -> 0 the step tends to -pinv(J) r."""
    rng = np.random.default_rng(0)
    J = rng.standard_normal((30, 80))
    r = rng.standard_normal(30)
    K = S.gram(J)
    ch = S.cholesky(K, 1e-10)
    v = -(J.T @ S.solve(ch, r))
    ls = np.linalg.lstsq(J, -r, rcond=None)[0]
    assert rel(v, ls) <= 1e-8


def test_gramian_properties(c0):
    p, th, r, J = c0
    K = S.gram(J)
    assert np.array_equal(K, K.T) or np.abs(K - K.T).max() <= 1e-15 * np.abs(K).max()
    assert np.allclose(np.diag(K), (J * J).sum(1), rtol=1e-13)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -K.shape[0] * np.finfo(float).eps * ev.max()


def test_ga_rule_cases():
    v = np.array([3.0, 4.0])
    assert S.ga_accept(v, np.array([0.6, 0.8]))        # 2*1/5 = 0.4
    assert S.ga_accept(v, np.array([0.0, 1.25]))       # exactly 0.5: inclusive
    assert not S.ga_accept(v, np.array([0.0, 1.3]))
    assert not S.ga_accept(np.zeros(2), np.zeros(2))   # ||v|| = 0 -> plain step


def test_line_search_ties_pick_largest_eta():
    p = W.config(0)
    th = W.glorot_theta(p.widths, 0)
    eta, losses = S.line_search(p, th, np.zeros_like(th))
    assert eta == 1.0 and np.all(losses == losses[0])


@pytest.mark.slow
def test_config0_training_gate():
    """Config 0: 20 steps with GA at lam = 1e-8. Loss never increases (the grid
    contains 2^-30) and the relative L2 error reaches the 1e-2 gate."""
    p = W.config(0)
    th0 = W.glorot_theta(p.widths, 0)
    th, hist = S.train(p, th0, 20, lam_cap=1e-8, ga=True, fixed_lambda=1e-8)
    losses = [h["loss"] for h in hist] + [hist[-1]["loss_after"]]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(losses, losses[1:]))
    xe = W.eval_points(p, 10_000, 0)
    err = N.relative_l2(p, th, xe, W.exact_solution("sinsin", xe))
    print("config0 relative L2 after 20 steps:", err, "loss", losses[-1])
    assert err <= 1e-2


@pytest.mark.parametrize("widths,n_int,n_bdy,lam", [([2, 8, 1], 60, 20, 1e-3),
                                                   ([2, 6, 6, 1], 90, 30, 1e-6)])
def test_primal_dense_step_equals_dual_step(widths, n_int, n_bdy, lam):
    """The whole primal step (n x n systems, n < m here) equals the dual step
    (m x m systems): the same v, f_vv, a, acceptance and dtheta."""
    p = W.config(0, scale=dict(widths=widths, n_int=n_int, n_bdy=n_bdy))
    th = W.glorot_theta(p.widths, 3)
    n = sum(a * b + b for a, b in zip(widths[:-1], widths[1:]))
    assert n < p.m
    pr = S.primal_dense_step(p, th, lam)
    du = S.dense_step(p, th, lam)
    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    assert rel(pr.v, du.v) <= 1e-9
    assert rel(pr.fvv, du.fvv) <= 1e-9
    assert rel(pr.a, du.a) <= 1e-8
    assert pr.accepted == du.accepted
    assert rel(pr.dtheta, du.dtheta) <= 1e-8


def test_lm_lambda_is_the_smaller_of_loss_and_cap():
    """Damping rule of the hyper-parameter tables, lam_k = min(L(theta_k), cap):
    the cap binds above it and the loss below it (a max/min slip fails one)."""
    assert S.lm_lambda(3.0, 1e-5) == 1e-5
    assert S.lm_lambda(2e-7, 1e-5) == 2e-7
    assert S.lm_lambda(1e-5, 1e-5) == 1e-5


def test_backward_error_matches_its_defining_perturbation():
    """The normwise backward error eta of x for A x = b (Rigal-Gaches) is the
    smallest eps with (A + dA) x = b + db, ||dA|| <= eps ||A||, ||db|| <= eps ||b||.
    The minimising perturbation is dA = c ||A|| r x^T / ||x||, db = -c ||b|| r with
    r = b - A x and c = 1 / (||A|| ||x|| + ||b||); check both the equation and the
    norms, plus a diagonal case by hand."""
    rng = np.random.default_rng(7)
    m = 40
    B = rng.standard_normal((m, m))
    K = B @ B.T
    lam = 0.3
    A = K + lam * np.eye(m)
    b = rng.standard_normal(m)
    x = np.linalg.solve(A, b) + 1e-3 * rng.standard_normal(m)
    eta = S.backward_error(K, lam, x, b)
    r = b - A @ x
    nA, nx, nb = np.linalg.norm(A, 2), np.linalg.norm(x), np.linalg.norm(b)
    c = 1.0 / (nA * nx + nb)
    dA = c * nA * np.outer(r, x) / nx
    db = -c * nb * r
    assert np.linalg.norm((A + dA) @ x - (b + db)) <= 1e-13 * nb
    assert np.isclose(np.linalg.norm(dA, 2), eta * nA, rtol=1e-12)
    assert np.isclose(np.linalg.norm(db), eta * nb, rtol=1e-12)
    # diag(1, 4), x = (1, 1), b = 0: ||A x|| = sqrt(17), ||A|| = 4, ||x|| = sqrt(2)
    assert np.isclose(S.backward_error(np.diag([1.0, 4.0]), 0.0, np.ones(2), np.zeros(2)),
                      np.sqrt(17.0) / (4.0 * np.sqrt(2.0)), rtol=1e-15)
    # the exact solution has backward error at rounding level
    assert S.backward_error(K, lam, np.linalg.solve(A, b), b) <= 1e-15


def test_line_search_unique_minimiser_inside_the_grid():
    """Along a direction supported on the output layer the residual is affine,
    so L(theta + eta d) = 0.5 ||r0 + eta q||^2 with q = r(theta + d) - r(theta),
    minimised at eta* = -r0.q / q.q. Scaling d so that eta* = 0.3 makes 0.25 the
    grid's unique minimiser (|0.25 - 0.3| < |0.5 - 0.3|, and the quadratic is
    symmetric about eta*); doubling d halves it to 0.125."""
    p = W.config(0, scale=dict(widths=[2, 6, 1], n_int=30, n_bdy=10))
    th = W.glorot_theta(p.widths, 3)
    n = th.size
    d = np.zeros(n)
    d[n - 7:] = np.random.default_rng(4).standard_normal(7)  # W_2 (6) and b_2 (1)
    r0 = N.residual(p, th)
    q = N.residual(p, th + d) - r0
    assert np.allclose(N.residual(p, th + 0.5 * d), r0 + 0.5 * q, rtol=0, atol=1e-13)
    d = d * (-(r0 @ q) / (q @ q)) / 0.3  # now eta* = 0.3
    eta, losses = S.line_search(p, th, d)
    assert eta == 0.25
    assert np.sum(losses == losses.min()) == 1
    eta2, _ = S.line_search(p, th, 2.0 * d)
    assert eta2 == 0.125
