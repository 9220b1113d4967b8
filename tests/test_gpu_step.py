"""Full-size step parity: the dense D-NGD step on the GPU against the FP64
oracle, at the workload sizes and in the launch configuration bench.py
times (5-D Poisson, m = 5000, n = 133377) and on the 2-D Poisson workload
(m = 500, n = 1185, lambda = 1e-8)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import network as N
from oracle import step as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "config1_step.npz")


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def c1():
    d = D()
    p = W.config(1)
    th = W.glorot_theta(p.widths, 0)
    prob = d.Problem.from_workload(p)
    g = np.load(GOLD)
    yield d, p, th, prob, g
    prob.close()


def test_config1_residual_and_gram_rows(c1):
    d, p, th, prob, g = c1
    say("case config1 residual / J row norms / K rows")
    r, J = prob.residual_jacobian(th, d.F64)
    assert rel(r.cpu().numpy(), g["r"]) <= 1e-12
    rn = (J[:, :prob.n] ** 2).sum(1).cpu().numpy()
    assert rel(rn, g["rownorm2"]) <= 1e-12
    idx = g["K_rows_idx"]
    Krows = (J[torch.tensor(idx, device=J.device)] @ J.T).cpu().numpy()
    assert np.abs(Krows - g["K_rows"]).max() <= 1e-12 * np.abs(g["K_rows"]).max()
    # the FP64 Gram kernel on the same J: sampled rows of the lower triangle
    K = d.gram(J, prob.n, 0.0).cpu().numpy()
    for q, i in enumerate(idx):
        ref = g["K_rows"][q][: i + 1]
        assert np.abs(K[i, : i + 1] - ref).max() <= 1e-12 * np.abs(ref).max()
    del J


def test_config1_plain_step(c1):
    d, p, th, prob, g = c1
    lam = float(g["lam"])
    say("case config1 plain step, lam", lam)
    dth, st = prob.step(th, lam, d.step_opts(precision=d.PLAIN, ga=True))
    assert st.ga_accepted == int(g["accepted"])
    assert rel(dth.cpu().numpy(), g["dtheta"]) <= 1e-10


def test_config1_mixed_step(c1):
    d, p, th, prob, g = c1
    lam = float(g["lam"])
    say("case config1 mixed step (auto gram passes, 2 refinement sweeps)")
    dth, st = prob.step(th, lam, d.step_opts(precision=d.MIXED, ga=True, ir_sweeps=2))
    e = rel(dth.cpu().numpy(), g["dtheta"])
    say("mixed rel err", e, "passes", st.gram_passes_used, "ir", list(st.ir_residual)[:2])
    assert st.ga_accepted == int(g["accepted"])
    assert e <= 1e-4


def test_config1_mixed_is_deterministic(c1):
    d, p, th, prob, g = c1
    lam = float(g["lam"])
    o = d.step_opts(precision=d.MIXED, ga=True)
    a, _ = prob.step(th, lam, o)
    b, _ = prob.step(th, lam, o)
    assert torch.equal(a, b)


def test_config0_steps_match_oracle():
    d = D()
    p = W.config(0)
    th = W.glorot_theta(p.widths, 0)
    prob = d.Problem.from_workload(p)
    # tight check at moderate damping; the lam = 1e-8 case is conditioning-limited
    for lam, tol in ((1e-6, 1e-10), (1e-8, 1e-7)):
        ref = S.dense_step(p, th, lam, ga=True)
        say("case config0 plain step lam", lam)
        dth, st = prob.step(th, lam, d.step_opts(precision=d.PLAIN, ga=True))
        assert rel(dth.cpu().numpy(), ref.dtheta) <= tol
        assert st.ga_accepted == int(ref.accepted)
    prob.close()
