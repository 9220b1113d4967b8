"""Oracle: the dense dual D-NGD step and its workflow (FP64 CPU, SciPy LAPACK).

Test infrastructure only (see ``oracle/__init__.py``).

The Levenberg-Marquardt subproblem (Section 3) has the unique minimiser
    dtheta = -(J^T J + lam I_n)^{-1} J^T r                        (primal, Prop. 3.1)
           = -J^T (J J^T + lam I_m)^{-1} r                        (dual, Thm. 3.2)
The second line is the dual system with the recovery formula rewritten as
``alpha = (K + lam I)^{-1} r``, ``dtheta = -J^T alpha`` ("alpha form"): with
the paper's ``y* = -(K+lam I)^{-1} K r`` one has ``y* + r = lam alpha``, so the
two are the same vector, and the alpha form avoids the cancellation in
``-(J^T y* + grad L)/lam`` at small lam. ``literal_dual_step`` keeps the
paper's printed form for the pins.

Geodesic acceleration (Section 3.2, Prop. 3.4): ``a = -J^T (K + lam I)^{-1} f_vv``,
reusing the factorisation; accepted when ``||v|| > eps`` and
``2 ||a|| / ||v|| <= 0.5`` (dense dual solver, Appendix algorithm).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from . import network


def gram(J):
    """Residual Gramian K = J J^T (Definition 3.3)."""
    return J @ J.T


def cholesky(K, lam):
    """Lower Cholesky factor of K + lam I (dense dual solver)."""
    return sla.cho_factor(K + lam * np.eye(K.shape[0]), lower=True, check_finite=True)


def solve(chol, b):
    return sla.cho_solve(chol, b, check_finite=True)


def primal_step(J, r, lam):
    """Primal normal equations (Prop. 3.1): (J^T J + lam I_n) x = -J^T r."""
    n = J.shape[1]
    G = J.T @ J + lam * np.eye(n)
    return -sla.solve(G, J.T @ r, assume_a="pos")


def primal_accel(J, fvv, lam):
    """Primal geodesic acceleration (Prop. 3.4): (J^T J + lam I) a = -J^T f_vv."""
    return primal_step(J, fvv, lam)


def literal_dual_step(J, r, lam, fvv=None):
    """The dual system and recovery formula as printed (Thm. 3.2, Prop. 3.4):
    (K + lam I) y = -J g, dtheta = -(J^T y + g)/lam with g = J^T r;
    (K + lam I) y_a = -K f_vv, a = -J^T (y_a + f_vv)/lam."""
    K = gram(J)
    g = J.T @ r
    A = K + lam * np.eye(K.shape[0])
    y = np.linalg.solve(A, -(J @ g))
    v = -(J.T @ y + g) / lam
    if fvv is None:
        return v
    ya = np.linalg.solve(A, -(K @ fvv))
    a = -(J.T @ (ya + fvv)) / lam
    return v, a


def ga_accept(v, a, eps_norm=0.0):
    """Acceptance rule of the dense dual solver: ||v|| > eps and 2||a||/||v|| <= 1/2."""
    nv = float(np.linalg.norm(v))
    if not nv > eps_norm:
        return False
    return 2.0 * float(np.linalg.norm(a)) / nv <= 0.5


@dataclasses.dataclass
class StepResult:
    r: np.ndarray
    J: np.ndarray
    K: np.ndarray
    alpha: np.ndarray
    v: np.ndarray
    fvv: np.ndarray | None
    beta: np.ndarray | None
    a: np.ndarray | None
    accepted: bool
    dtheta: np.ndarray


def dense_step(problem, theta, lam, ga=True, eps_norm=0.0, J=None, r=None):
    """One dense dual D-NGD step (Section 4.1 and its appendix algorithm),
    alpha form: K = J J^T; L L^T = K + lam I; alpha = L^-T L^-1 r; v = -J^T alpha;
    f_vv along v; beta = L^-T L^-1 f_vv; a = -J^T beta; dtheta = v (+ a/2)."""
    if r is None:
        r = network.residual(problem, theta)
    if J is None:
        J = network.jacobian(problem, theta)
    K = gram(J)
    ch = cholesky(K, lam)
    alpha = solve(ch, r)
    v = -(J.T @ alpha)
    if not ga:
        return StepResult(r, J, K, alpha, v, None, None, None, False, v.copy())
    f = network.fvv(problem, theta, v)
    beta = solve(ch, f)
    a = -(J.T @ beta)
    acc = ga_accept(v, a, eps_norm)
    dtheta = v + 0.5 * a if acc else v.copy()
    return StepResult(r, J, K, alpha, v, f, beta, a, acc, dtheta)


def primal_dense_step(problem, theta, lam, ga=True, eps_norm=0.0):
    """One D-NGD step through the primal normal equations (Prop. 3.1): v from
    (J^T J + lam I_n) v = -J^T r, f_vv along v, a from (J^T J + lam I_n) a =
    -J^T f_vv (Prop. 3.4), the same acceptance rule. K holds J^T J; alpha and
    beta are not formed."""
    r = network.residual(problem, theta)
    J = network.jacobian(problem, theta)
    v = primal_step(J, r, lam)
    if not ga:
        return StepResult(r, J, J.T @ J, None, v, None, None, None, False, v.copy())
    f = network.fvv(problem, theta, v)
    a = primal_accel(J, f, lam)
    acc = ga_accept(v, a, eps_norm)
    dtheta = v + 0.5 * a if acc else v.copy()
    return StepResult(r, J, J.T @ J, None, v, f, None, a, acc, dtheta)


def backward_error(K, lam, x, b):
    """Normwise backward error ||(K+lam I)x - b|| / (||K+lam I|| ||x|| + ||b||)."""
    A = K + lam * np.eye(K.shape[0])
    return float(np.linalg.norm(A @ x - b) /
                 (np.linalg.norm(A, 2) * np.linalg.norm(x) + np.linalg.norm(b)))


# ----------------------------------------------------------------------------
# workflow (D-NGD workflow algorithm): lam rule, line search, update


ETA_GRID = np.array([2.0 ** -k for k in range(31)])


def line_search(problem, theta, dtheta, etas=ETA_GRID):
    """eta = argmin over the grid of L(theta + eta dtheta); the first minimum
    (largest eta) wins ties. Returns (eta, losses)."""
    losses = np.array([network.loss(problem, theta + e * dtheta) for e in etas])
    k = int(np.argmin(losses))
    return float(etas[k]), losses


def lm_lambda(loss_value, cap):
    """lam_k = min(L(theta_k), cap) (hyper-parameter tables)."""
    return min(float(loss_value), float(cap))


def train(problem, theta0, steps, lam_cap, ga=True, fixed_lambda=None, callback=None):
    """Run the D-NGD workflow for ``steps`` dense steps; returns (theta, history)."""
    theta = theta0.copy()
    hist = []
    for k in range(steps):
        L0 = network.loss(problem, theta)
        lam = fixed_lambda if fixed_lambda is not None else lm_lambda(L0, lam_cap)
        res = dense_step(problem, theta, lam, ga=ga)
        eta, losses = line_search(problem, theta, res.dtheta)
        theta = theta + eta * res.dtheta
        rec = dict(step=k, loss=L0, lam=lam, eta=eta, loss_after=float(losses.min()),
                   accepted=res.accepted, vnorm=float(np.linalg.norm(res.v)))
        hist.append(rec)
        if callback:
            callback(k, theta, rec)
    return theta, hist
