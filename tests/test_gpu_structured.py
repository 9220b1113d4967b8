"""The dense dual step on the structured FP64 kernel (K assembled per layer
from activations and adjoints, J never formed; v and a by the matrix-free
reverse pass) against the oracle's dense step, which forms J."""
import numpy as np
import pytest

import workloads as W
from oracle import step as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# (config, scale, lam): 2-D Poisson, 5-D Poisson (7 jet rows per interior
# point), heat (5 jet rows, initial points); the last 5-D case has 25,000 jet
# rows, so the Gram runs in two row chunks with a ragged boundary
CASES = [
    (0, dict(widths=[2, 32, 32, 1], n_int=400, n_bdy=100), 1e-4),
    (1, dict(widths=[5, 48, 48, 1], n_int=300, n_bdy=100), 1e-4),
    (2, dict(widths=[3, 40, 40, 1], n_int=192, n_bdy=48, n_init=48), 1e-3),
    (1, dict(widths=[5, 32, 32, 1], n_int=3500, n_bdy=500), 1e-3),
]


@pytest.mark.parametrize("idx,scale,lam", CASES)
def test_structured_step_matches_oracle(idx, scale, lam):
    d = D()
    p = W.config(idx, scale=scale)
    th = W.glorot_theta(p.widths, idx + 7)
    prob = d.Problem.from_workload(p)
    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    fvv = torch.empty(p.m, dtype=torch.float64, device="cuda")
    dth, st = prob.step(th, lam, d.step_opts(solver=d.STRUCTURED, ga=True, alpha_out=alpha,
                                              fvv_out=fvv))
    ref = S.dense_step(p, th, lam, ga=True)
    cond = np.linalg.cond(ref.K + lam * np.eye(p.m))
    tol = max(1e-10, 100 * np.finfo(float).eps * cond)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    say("case structured config", idx, scale["widths"], "m", p.m, "cond", f"{cond:.2e}",
        "err", e, "alpha", rel(alpha.cpu().numpy(), ref.alpha), "accepted", st.ga_accepted,
        ref.accepted, "ms gram", st.ms_gram_kernel)
    assert st.ga_accepted == int(ref.accepted)
    assert rel(alpha.cpu().numpy(), ref.alpha) <= tol
    assert rel(fvv.cpu().numpy(), ref.fvv) <= tol
    assert e <= tol
    prob.close()


def test_structured_equals_plain_dense_step():
    """The same FP64 step as the plain J path on the GPU, up to rounding."""
    d = D()
    p = W.config(1, scale=dict(widths=[5, 64, 64, 64, 1], n_int=400, n_bdy=100))
    th = W.glorot_theta(p.widths, 3)
    prob = d.Problem.from_workload(p)
    a, sa = prob.step(th, 1e-4, d.step_opts(solver=d.STRUCTURED, ga=True))
    b, sb = prob.step(th, 1e-4, d.step_opts(precision=d.PLAIN, solver=d.DENSE, ga=True))
    say("case structured vs plain J path: rel", rel(a.cpu().numpy(), b.cpu().numpy()))
    assert sa.ga_accepted == sb.ga_accepted
    assert rel(a.cpu().numpy(), b.cpu().numpy()) <= 1e-9
    prob.close()
