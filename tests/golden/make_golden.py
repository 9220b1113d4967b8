"""Write the stored oracle results used by the GPU parity tests.

Calls only ``oracle`` and ``workloads`` (seeded inputs): every stored value is
the FP64 CPU oracle's. Run from the repository root:
    python tests/golden/make_golden.py            # config 1 (about 3 minutes)
    python tests/golden/make_golden.py config2    # heat workload (about 15 minutes, 16 GB)
Output: tests/golden/config1_step.npz, tests/golden/config2_step.npz
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import network as N  # noqa: E402
from oracle import step as S  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def config1():
    p = W.config(1)
    th = W.glorot_theta(p.widths, 0)
    t0 = time.perf_counter()
    r = N.residual(p, th)
    lam = min(0.5 * float(r @ r), W.LAMBDA_CAP[1])
    J = N.jacobian(p, th)
    res = S.dense_step(p, th, lam, ga=True, J=J, r=r)
    # sampled Gram rows for a direct check of K
    rows = np.random.default_rng(123).choice(p.m, 16, replace=False)
    Krows = J[rows] @ J.T
    np.savez_compressed(os.path.join(OUT, "config1_step.npz"), lam=lam, r=r, alpha=res.alpha,
                        v=res.v, fvv=res.fvv, beta=res.beta, a=res.a, dtheta=res.dtheta,
                        accepted=res.accepted, K_rows_idx=rows, K_rows=Krows,
                        rownorm2=(J * J).sum(1))
    print(f"config1 golden written in {time.perf_counter() - t0:.1f} s, lam={lam:g}, "
          f"accepted={res.accepted}")


def config2(rows_per_block=16):
    """The heat workload at full size (n = 3,153,921, m = 8192) at the Glorot
    start, lambda = min(L, 1e-3), dense step with GA. Its FP64 J (207 GB) is
    never formed: K = sum_b J_b J_b^T over column blocks J_b of the reverse
    pass (LAPACK dsyrk, FP64), J^T alpha and J^T beta by the weighted reverse
    pass. dtheta is stored in FP32 (relative rounding 6e-8, far below the 1e-4
    bar it is compared at); the m-vectors in FP64."""
    import scipy.linalg.blas as blas
    p = W.config(2)
    th = W.glorot_theta(p.widths, 0)
    t0 = time.perf_counter()
    r = N.residual(p, th)
    lam = min(0.5 * float(r @ r), W.LAMBDA_CAP[2])
    tapes = N.layer_tapes(p, th)
    K = np.zeros((p.m, p.m), order="F")
    nb = 0
    for l in range(len(p.widths) - 1):
        wout = p.widths[l + 1]
        for o0 in range(0, wout, rows_per_block):
            Wc, bc = N.jacobian_block(tapes, l, o0, min(wout, o0 + rows_per_block))
            A = np.concatenate([Wc, bc], axis=1)  # m x cols, C order: A.T is Fortran
            K = blas.dsyrk(1.0, A.T, beta=1.0, c=K, trans=1, lower=1, overwrite_c=1)
            nb += A.shape[1]
        print(f"  layer {l}: {nb} columns, {time.perf_counter() - t0:.0f} s", flush=True)
    assert nb == th.size
    del tapes
    K = np.tril(K) + np.tril(K, -1).T
    ch = S.cholesky(K, lam)
    alpha = S.solve(ch, r)
    be = S.backward_error(K, lam, alpha, r)
    v = -N.vjp(p, th, alpha)
    f = N.fvv(p, th, v)
    beta = S.solve(ch, f)
    a = -N.vjp(p, th, beta)
    acc = S.ga_accept(v, a)
    dtheta = v + 0.5 * a if acc else v
    np.savez_compressed(os.path.join(OUT, "config2_step.npz"), lam=lam, r=r, alpha=alpha, fvv=f,
                        beta=beta, vnorm=np.linalg.norm(v), anorm=np.linalg.norm(a),
                        accepted=acc, dtheta32=dtheta.astype(np.float32),
                        dtheta_norm=np.linalg.norm(dtheta), K_diag=np.diag(K).copy(),
                        alpha_backward_error=be)
    print(f"config2 golden written in {time.perf_counter() - t0:.1f} s, lam={lam:g}, "
          f"accepted={acc}, |v|={np.linalg.norm(v):.6g}, |a|={np.linalg.norm(a):.6g}, "
          f"alpha backward error {be:.2e}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["config1"]
    for name in which:
        {"config1": config1, "config2": config2}[name]()
