"""Write the stored oracle results used by the GPU parity tests.

Calls only ``oracle`` and ``workloads`` (seeded inputs): every stored value is
the FP64 CPU oracle's. Run from the repository root:
    python tests/golden/make_golden.py            # config 1 (about 3 minutes)
Output: tests/golden/config1_step.npz
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


if __name__ == "__main__":
    config1()
