"""The primal Gauss-Newton solver (Proposition 3.1: v = -(J^T J + lam I)^{-1}
J^T r, a = -(J^T J + lam I)^{-1} J^T f_vv) and the dense solver's automatic
primal/dual choice, on the GPU against the oracle's primal step (which the
CPU tests pin to the dual step)."""
import numpy as np
import pytest

import workloads as W
from oracle import step as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

# (widths, n_int, n_bdy): n < m, from one to several Gram tiles (ragged)
CASES = [([2, 8, 1], 60, 20), ([2, 16, 16, 1], 300, 100), ([2, 32, 32, 1], 900, 300)]


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(widths, n_int, n_bdy, seed=0):
    p = W.config(0, scale=dict(widths=widths, n_int=n_int, n_bdy=n_bdy))
    return p, W.glorot_theta(p.widths, seed)


def n_params(widths):
    return sum(a * b + b for a, b in zip(widths[:-1], widths[1:]))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("lam", [1e-3, 1e-6])
def test_primal_plain_matches_oracle(case, lam):
    d = D()
    p, th = problem(*case)
    assert n_params(case[0]) < p.m
    prob = d.Problem.from_workload(p)
    fvv = torch.empty(p.m, dtype=torch.float64, device="cuda")
    dth, st = prob.step(th, lam, d.step_opts(precision=d.PLAIN, solver=d.PRIMAL, ga=True,
                                              fvv_out=fvv))
    ref = S.primal_dense_step(p, th, lam)
    cond = np.linalg.cond(ref.K + lam * np.eye(ref.K.shape[0]))
    tol = max(1e-10, 100 * np.finfo(float).eps * cond)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    say("case primal plain", case[0], "m", p.m, "lam", lam, "cond", f"{cond:.2e}", "err", e,
        "accepted", st.ga_accepted, ref.accepted)
    assert st.primal == 1
    assert st.ga_accepted == int(ref.accepted)
    assert rel(fvv.cpu().numpy(), ref.fvv) <= tol
    assert e <= tol
    prob.close()


@pytest.mark.parametrize("case", CASES)
def test_primal_mixed_matches_oracle(case):
    """FP32 J^T, bf16 Gram of J^T (auto passes and escalation), FP64 Cholesky
    and two refinement sweeps against the exact operator."""
    d = D()
    p, th = problem(*case, seed=1)
    lam = 1e-4
    prob = d.Problem.from_workload(p)
    dth, st = prob.step(th, lam, d.step_opts(precision=d.MIXED, solver=d.PRIMAL, ga=True))
    ref = S.primal_dense_step(p, th, lam)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    say("case primal mixed", case[0], "passes", st.gram_passes_used, "ir",
        list(st.ir_residual)[:2], "err", e)
    assert st.primal == 1 and st.gram_passes_used in (1, 3, 4, d.GRAM_F64)
    assert st.ga_accepted == int(ref.accepted)
    assert e <= 1e-4
    prob.close()


def test_dense_auto_takes_primal_when_n_lt_m():
    d = D()
    p, th = problem(*CASES[1])
    prob = d.Problem.from_workload(p)
    o_auto = d.step_opts(precision=d.PLAIN, solver=d.DENSE_AUTO, ga=True)
    o_prim = d.step_opts(precision=d.PLAIN, solver=d.PRIMAL, ga=True)
    a, sa = prob.step(th, 1e-4, o_auto)
    b, sb = prob.step(th, 1e-4, o_prim)
    say("case auto n < m: primal", sa.primal)
    assert sa.primal == 1 and torch.equal(a, b)
    prob.close()


def test_dense_auto_takes_dual_when_n_ge_m_and_forced_primal_agrees():
    """n = 65 > m = 40: the auto choice is the dual solver; the primal solver
    forced on the same problem (a 65 x 65 system) gives the same step."""
    d = D()
    p, th = problem([2, 16, 1], 30, 10, seed=2)
    assert n_params([2, 16, 1]) > p.m
    prob = d.Problem.from_workload(p)
    lam = 1e-3
    a, sa = prob.step(th, lam, d.step_opts(precision=d.PLAIN, solver=d.DENSE_AUTO, ga=True))
    b, sb = prob.step(th, lam, d.step_opts(precision=d.PLAIN, solver=d.DENSE, ga=True))
    c, sc = prob.step(th, lam, d.step_opts(precision=d.PLAIN, solver=d.PRIMAL, ga=True))
    ref = S.dense_step(p, th, lam, ga=True)
    say("case auto n > m: primal", sa.primal, "forced primal err", rel(c.cpu().numpy(), ref.dtheta))
    assert sa.primal == 0 and torch.equal(a, b)
    assert sc.primal == 1 and sc.ga_accepted == int(ref.accepted)
    assert rel(c.cpu().numpy(), ref.dtheta) <= 1e-9
    prob.close()
