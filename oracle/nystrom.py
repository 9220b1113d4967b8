"""Oracle: Nystrom spectral preconditioner and preconditioned CG on the dual
system (FP64 CPU).

Test infrastructure only (see ``oracle/__init__.py``).

Section 3.3 approximates the residual Gramian K from its landmark columns
K_{:,I} (index set I, passed in; how it is drawn is the caller's business) by
the Nystrom approximation K^ = K_{:,I} K_II^+ K_{I,:}, written here as that
product with the pseudo-inverse of K_II (eigenvalues at or below a positivity
threshold dropped), and takes K^'s nonzero eigenpairs (U, Lambda^). The
spectral preconditioner is then
    P^{-1} = U (Lambda^ + lam I)^{-1} U^T + (I - U U^T) / lam,
which equals (K^ + lam I)^{-1}. PCG (appendix algorithm) runs on the alpha
form of the dual system, (K + lam I) alpha = r, and the step is dtheta = -J^T alpha.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def positive_threshold(Kii, ell_factor=None):
    """Eigenvalues kept as 'positive': > ell * u * lambda_max(K_II), u the FP64
    unit roundoff (the paper does not fix the threshold)."""
    ell = Kii.shape[0] if ell_factor is None else ell_factor
    lmax = float(np.max(np.abs(np.linalg.eigvalsh(Kii)))) if Kii.size else 0.0
    return ell * np.finfo(np.float64).eps * 0.5 * lmax


def nystrom_approx(K_cols, I, delta=None):
    """(K^, rank) with K^ = K_{:,I} K_II^+ K_{I,:} from the m x ell block
    K[:, I]. K_II^+ is the pseudo-inverse keeping the eigenvalues above
    ``positive_threshold``; with ``delta`` it is (K_II + delta I)^{-1} instead
    (the shifted form a Cholesky-based construction uses), evaluated as M M^T
    with M = K_{:,I} L^{-T}, L L^T = K_II + delta I (the product with the
    explicit inverse loses ~ ||K|| / delta digits when K_II is singular)."""
    Kii = K_cols[I, :]
    Kii = 0.5 * (Kii + Kii.T)
    if delta is None:
        lam_q, Q = np.linalg.eigh(Kii)
        keep = lam_q > positive_threshold(Kii)
        inv = (Q[:, keep] / lam_q[keep]) @ Q[:, keep].T
        return K_cols @ inv @ K_cols.T, int(keep.sum())
    L = np.linalg.cholesky(Kii + delta * np.eye(len(I)))
    M = sla.solve_triangular(L, K_cols.T, lower=True).T
    return M @ M.T, len(I)


def nystrom(K_cols, I):
    """(U, Lambda^): the eigenpairs of K^ with its `rank` largest eigenvalues
    (the others are zero up to rounding), U with orthonormal columns."""
    Khat, rank = nystrom_approx(K_cols, I)
    w, V = np.linalg.eigh(0.5 * (Khat + Khat.T))
    order = np.argsort(w)[::-1][:rank]
    return V[:, order], w[order]


def precond_apply(U, lam_hat, lam, x):
    """P^{-1} x for the spectral preconditioner."""
    ux = U.T @ x
    return U @ (ux / (lam_hat + lam)) + (x - U @ ux) / lam


def pcg(apply_A, b, apply_Pinv, tol, maxit):
    """Preconditioned CG (appendix algorithm) from y = 0. Stops on
    <p, Ap> <= 0, ||r|| <= tol ||b||, rho <= 0 or non-finite values.
    Returns (y, iterations, converged, residual history)."""
    y = np.zeros_like(b)
    r = b.copy()
    z = apply_Pinv(r)
    p = z.copy()
    rho = float(r @ z)
    nb = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r))]
    if hist[0] <= tol * nb:
        return y, 0, True, hist
    for j in range(maxit):
        Ap = apply_A(p)
        pAp = float(p @ Ap)
        if not (pAp > 0.0) or not np.isfinite(pAp):
            return y, j, False, hist
        a = rho / pAp
        y = y + a * p
        r = r - a * Ap
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= tol * nb:
            return y, j + 1, True, hist
        z = apply_Pinv(r)
        rho_new = float(r @ z)
        if not (rho > 0.0) or not np.isfinite(rho_new):
            return y, j + 1, False, hist
        p = z + (rho_new / rho) * p
        rho = rho_new
    return y, maxit, False, hist


def pcg_step(J, r, lam, I, tol, maxit):
    """Matrix-free PCG step: kvp(p) = J (J^T p) + lam p (Definition 3.6),
    Nystrom preconditioner from landmarks I. Returns (dtheta, alpha, its, ok)."""
    K_cols = J @ J[I, :].T
    U, lh = nystrom(K_cols, I)

    def kvp(p):
        return J @ (J.T @ p) + lam * p

    alpha, its, ok, _ = pcg(kvp, r, lambda x: precond_apply(U, lh, lam, x), tol, maxit)
    return -(J.T @ alpha), alpha, its, ok
