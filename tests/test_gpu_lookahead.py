"""The dense step's Cholesky with look-ahead, at sizes that reach each of its
branches, against the FP64 oracle. The factorisation works in block columns
of 256; after each, the next block column is updated on the main stream and
the rest of the trailing matrix on a side stream: first the block column
after next, then the remainder as a persistent update on CUs of its own
(64-wide tiles below 1024 rows, 128-wide above). The sizes:

  m =  300  no side-stream update at all (one block column and a ragged one)
  m =  700  side update of the block column after next only (no remainder)
  m =  769  a remainder of a single row
  m = 1500  remainders below 1024 rows only
  m = 2100  remainders above and below 1024 rows, ragged last panel

Each plain (FP64) step's alpha, returned through alpha_out, must solve
(J J^T + lambda I) alpha = r to a backward error near rounding (computed with
the oracle's J and r), and its update must match the oracle's dense step."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N
from oracle import step as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("m", [300, 700, 769, 1500, 2100])
def test_dense_step_lookahead_branches(m):
    d = D()
    n_bdy = m // 5
    p = W.poisson_problem([2, 16, 16, 1], m - n_bdy, n_bdy, "sinsin", 11)
    assert p.m == m
    th = W.glorot_theta(p.widths, 3)
    lam = 1e-3
    print(f"case look-ahead m={m} n={p.n_params}", flush=True)
    ref = S.dense_step(p, th, lam, ga=True)
    prob = d.Problem.from_workload(p)
    alpha = torch.empty(m, dtype=torch.float64, device="cuda")
    dth, st = prob.step(th, lam, d.step_opts(precision=d.PLAIN, ga=True, alpha_out=alpha))
    a = alpha.cpu().numpy()
    be = S.backward_error(ref.K, lam, a, ref.r)
    e_alpha = rel(a, ref.alpha)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    print(f"  backward error {be:.2e}, alpha rel err {e_alpha:.2e}, dtheta rel err {e:.2e}",
          flush=True)
    assert be <= 1e-13
    assert e <= 1e-10
    assert st.ga_accepted == int(ref.accepted)
    prob.close()
