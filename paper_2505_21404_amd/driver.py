"""D-NGD training loop (the workflow algorithm of Section 4): per iteration
the damping rule lambda_k = min(L(theta_k), cap), one D-NGD step, the
31-point grid line search eta in {2^-k : k = 0..30} and the update
theta <- theta + eta dtheta. Each iteration is one call of dngd_iterate; this
module only keeps the history.
"""
from __future__ import annotations

import time
from typing import Callable, List, Optional, Tuple

import torch

from . import dngd as D

ETA_GRID = [2.0 ** -k for k in range(31)]


def train(prob: "D.Problem", theta0, steps: int, lam_cap: float = 0.0,
          fixed_lambda: float = 0.0, opts: Optional["D.StepOpts"] = None,
          etas=ETA_GRID, callback: Optional[Callable] = None, stream=None
          ) -> Tuple[torch.Tensor, List[dict]]:
    """Run ``steps`` iterations from theta0 and return (theta, history).

    Exactly one of ``lam_cap`` (damping rule) or ``fixed_lambda`` must be
    positive. Each history record holds the loss before the step, lambda,
    eta, the loss after, the step statistics and the iteration wall time."""
    if (lam_cap > 0) == (fixed_lambda > 0):
        raise ValueError("give exactly one of lam_cap > 0 or fixed_lambda > 0")
    theta = prob._theta(theta0).clone()
    hist = []
    for k in range(steps):
        t0 = time.perf_counter()
        st = prob.iterate(theta, etas, lam_cap=lam_cap, fixed_lambda=fixed_lambda, opts=opts,
                          stream=stream)
        rec = st.as_dict()
        rec["iter"] = k
        rec["ms_iter"] = (time.perf_counter() - t0) * 1e3
        hist.append(rec)
        if callback is not None:
            callback(k, theta, rec)
    return theta, hist
