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
