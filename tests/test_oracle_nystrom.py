"""Pins for the oracle's Nystrom preconditioner and PCG (Sections 3.3, 4.2)
against the algebraic identities the construction must satisfy and a dense
Cholesky solve."""
import numpy as np

import workloads as W
from oracle import network as N
from oracle import nystrom as NY
from oracle import step as S


def small_problem():
    p = W.config(1, scale=dict(widths=[5, 24, 24, 1], n_int=160, n_bdy=40))
    th = W.glorot_theta(p.widths, 0)
    return p, th, N.residual(p, th), N.jacobian(p, th)


def test_nystrom_identities():
    p, th, r, J = small_problem()
    K = S.gram(J)
    I = W.landmarks(p.m, 60, 0)
    U, lh = NY.nystrom(K[:, I], I)
    # orthonormal basis
    assert np.abs(U.T @ U - np.eye(U.shape[1])).max() <= 1e-10
    Khat = (U * lh) @ U.T
    # Khat = K_{:,I} K_II^+ K_{I,:}
    Kii = K[np.ix_(I, I)]
    ref = K[:, I] @ np.linalg.pinv(Kii, rcond=1e-13, hermitian=True) @ K[I, :]
    assert np.abs(Khat - ref).max() <= 1e-7 * np.abs(K).max()
    # interpolation of the landmark columns
    assert np.abs(Khat[:, I] - K[:, I]).max() <= 1e-7 * np.abs(K).max()


def test_preconditioner_is_inverse_of_regularised_nystrom():
    p, th, r, J = small_problem()
    K = S.gram(J)
    I = W.landmarks(p.m, 50, 1)
    U, lh = NY.nystrom(K[:, I], I)
    lam = 1e-3
    x = np.random.default_rng(0).standard_normal(p.m)
    z = NY.precond_apply(U, lh, lam, x)
    A = (U * lh) @ U.T + lam * np.eye(p.m)
    assert np.linalg.norm(A @ z - x) <= 1e-10 * np.linalg.norm(x)


def test_full_landmarks_converge_in_one_iteration():
    p, th, r, J = small_problem()
    lam = 1e-4
    I = np.arange(p.m)
    dth, alpha, its, ok = NY.pcg_step(J, r, lam, I, tol=1e-10, maxit=50)
    assert ok and its <= 2
    ref = S.dense_step(p, th, lam, ga=False, J=J, r=r)
    assert np.linalg.norm(dth - ref.v) <= 1e-8 * np.linalg.norm(ref.v)


def test_pcg_matches_cholesky():
    p, th, r, J = small_problem()
    lam = 1e-5
    I = W.landmarks(p.m, 80, 2)
    dth, alpha, its, ok = NY.pcg_step(J, r, lam, I, tol=1e-10, maxit=500)
    assert ok
    ref = S.dense_step(p, th, lam, ga=False, J=J, r=r)
    K = ref.K
    # true residual of the dual system in FP64
    assert np.linalg.norm((K + lam * np.eye(p.m)) @ alpha - r) <= 1e-9 * np.linalg.norm(r)
    assert np.linalg.norm(dth - ref.v) <= 1e-6 * np.linalg.norm(ref.v)


def test_unpreconditioned_cg_terminates():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((12, 12))
    A = B @ B.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    y, its, ok, _ = NY.pcg(lambda v: A @ v, b, lambda v: v, 1e-12, 40)
    assert ok and its <= 14
    assert np.allclose(A @ y, b, atol=1e-10)


def test_pcg_maxit_and_breakdown_flags():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((30, 30))
    A = B @ B.T + np.eye(30)
    b = rng.standard_normal(30)
    y, its, ok, _ = NY.pcg(lambda v: A @ v, b, lambda v: v, 1e-14, 1)
    assert not ok and its == 1
    # indefinite operator -> <p, Ap> <= 0 stops the iteration
    y, its, ok, _ = NY.pcg(lambda v: -v, b, lambda v: v, 1e-10, 10)
    assert not ok and its == 0


def test_nystrom_is_exact_when_landmarks_span_the_range():
    """If K has rank r and K_II has the same rank, the Nystrom approximation
    reproduces K exactly (its columns span K's range), and P^{-1} = (K + lam I)^{-1}."""
    rng = np.random.default_rng(3)
    m, r = 90, 12
    B = rng.standard_normal((m, r))
    K = B @ B.T
    I = np.sort(rng.choice(m, 20, replace=False))
    Khat, rank = NY.nystrom_approx(K[:, I], I)
    assert rank == r
    assert np.abs(Khat - K).max() <= 1e-10 * np.abs(K).max()
    U, lh = NY.nystrom(K[:, I], I)
    assert U.shape == (m, r) and np.all(lh > 0)
    lam = 1e-2
    x = rng.standard_normal(m)
    z = NY.precond_apply(U, lh, lam, x)
    assert np.linalg.norm((K + lam * np.eye(m)) @ z - x) <= 1e-9 * np.linalg.norm(x)
    # with fewer landmarks than the rank, K_II is nonsingular and the shifted
    # form tends to the pseudo-inverse form as the shift vanishes
    I2 = I[:10]
    K0, rank2 = NY.nystrom_approx(K[:, I2], I2)
    Kd, _ = NY.nystrom_approx(K[:, I2], I2, delta=1e-10 * np.abs(K).max())
    assert rank2 == 10
    assert np.abs(Kd - K0).max() <= 1e-7 * np.abs(K).max()
