"""GPU parity of the vector-valued residual classes (steady Navier-Stokes,
Kovasznay flow of Section 5.3) against the FP64 oracle: the residual map, the
Jacobian (FP64 and FP32), f_vv, J u and J^T p at a ragged small size and at the
paper's size ([2, 50 x 4, 3], 400 + 400 points, m = 2400, n = 7953); the
dense step (plain, mixed, primal); five workflow iterations; and the solvers
that are refused."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N
from oracle import step as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U64 = np.finfo(np.float64).eps / 2


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


SMALL = dict(widths=[2, 8, 8, 3], n_int=13, n_bdy=9)
CASES = [("small", SMALL), ("kovasznay", {})]


def _problem(kind):
    p = W.kovasznay(**SMALL) if kind == "small" else W.kovasznay()
    return p, W.glorot_theta(p.widths, 1 if kind == "small" else 0)


@pytest.mark.parametrize("kind,_", CASES)
def test_residual_and_jacobian(kind, _):
    d = D()
    p, th = _problem(kind)
    say("case NS residual/J", kind, "m", p.m, "n", th.size)
    prob = d.Problem.from_workload(p)
    assert prob.m == p.m == 3 * (p.n_int + p.n_bdy) and prob.n == th.size
    r_ref, J_ref = N.residual(p, th), N.jacobian(p, th)
    r, J = prob.residual_jacobian(th, d.F64)
    assert rel(r.cpu().numpy(), r_ref) <= 1e-12
    Jg = J[:, :prob.n].cpu().numpy()
    assert np.abs(Jg - J_ref).max() <= 1e-12 * np.abs(J_ref).max()
    assert torch.all(J[:, prob.n:] == 0)
    _, J32 = prob.residual_jacobian(th, d.F32)
    J32 = J32[:, :prob.n].cpu().numpy().astype(np.float64)
    # each FP32 entry is the FP64 value rounded once
    assert np.all(np.abs(J32 - J_ref) <= 2.0 ** -24 * np.abs(J_ref) + 1e-30)
    prob.close()


@pytest.mark.parametrize("kind,_", CASES)
def test_fvv_jvp_vjp(kind, _):
    d = D()
    p, th = _problem(kind)
    prob = d.Problem.from_workload(p)
    J = N.jacobian(p, th)
    u = W.random_direction(th.size, 7, 0.2)
    pw = W.random_direction(p.m, 8)
    say("case NS f_vv / J u / J^T p", kind)
    f_ref = N.fvv(p, th, u)
    assert rel(prob.fvv(th, u).cpu().numpy(), f_ref) <= 1e-11
    assert rel(prob.jvp(th, u).cpu().numpy(), J @ u) <= 1e-12
    assert rel(prob.vjp(th, pw).cpu().numpy(), J.T @ pw) <= 1e-12
    prob.close()


def test_dense_step_kovasznay():
    """One dense D-NGD step with GA at the paper's Kovasznay size, lambda =
    min(L(theta_0), 1e-5) (the experiment's damping rule): plain within
    max(1e-10, 10 u64 cond) with the alpha backward error <= m u64, mixed within
    1e-4, the primal solver within the same bar as plain."""
    d = D()
    p, th = _problem("kovasznay")
    lam = S.lm_lambda(N.loss(p, th), 1e-5)
    ref = S.dense_step(p, th, lam, ga=True)
    cond = np.linalg.cond(ref.K + lam * np.eye(p.m))
    prob = d.Problem.from_workload(p)
    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    say("case NS plain step, lam", lam, "u64 * cond", U64 * cond)
    dth, st = prob.step(th, lam, d.step_opts(precision=d.PLAIN, ga=True, alpha_out=alpha))
    be = S.backward_error(ref.K, lam, alpha.cpu().numpy(), ref.r)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    say(f"  plain: rel err {e:.2e}, backward error {be:.2e}, GA accepted {st.ga_accepted}")
    assert be <= p.m * U64
    assert e <= max(1e-10, 10 * U64 * cond)
    assert st.ga_accepted == int(ref.accepted)
    dm, sm = prob.step(th, lam, d.step_opts(precision=d.MIXED, ga=True))
    em = rel(dm.cpu().numpy(), ref.dtheta)
    say(f"  mixed: rel err {em:.2e}, passes {sm.gram_passes_used}, ir {list(sm.ir_residual)[:2]}")
    assert em <= 1e-4
    assert sm.ga_accepted == int(ref.accepted)
    dp, sp = prob.step(th, lam, d.step_opts(precision=d.PLAIN, solver=d.PRIMAL, ga=True))
    ep = rel(dp.cpu().numpy(), ref.dtheta)
    say(f"  primal: rel err {ep:.2e}")
    assert sp.primal == 1 and ep <= max(1e-10, 10 * U64 * cond)
    prob.close()


@pytest.mark.parametrize("precision,bar", [("PLAIN", None), ("MIXED", 1e-4)])
def test_kovasznay_iterations_match_oracle(precision, bar):
    """Five workflow iterations (damping min(L, 1e-5), GA, 31-point line
    search): the loss never increases and each step matches the oracle's at
    the GPU's own iterate."""
    d = D()
    p, th0 = _problem("kovasznay")
    prob = d.Problem.from_workload(p)
    theta = torch.tensor(th0, device="cuda")
    dbuf = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    prev = None
    for k in range(5):
        th_k = theta.cpu().numpy().copy()
        st = prob.iterate(theta, S.ETA_GRID, lam_cap=1e-5,
                          opts=d.step_opts(precision=getattr(d, precision), ga=True),
                          dtheta_out=dbuf)
        ref = S.dense_step(p, th_k, st.lam, ga=True)
        e = rel(dbuf.cpu().numpy(), ref.dtheta)
        cond = np.linalg.cond(ref.K + st.lam * np.eye(p.m))
        say(f"iter {k} {precision}: loss {st.loss:.6e} lam {st.lam:.2e} eta {st.eta:.3g} "
            f"rel err {e:.2e} (u64 cond {U64 * cond:.2e})")
        assert e <= (bar if bar else max(1e-10, 10 * U64 * cond))
        assert abs(st.loss - N.loss(p, th_k)) <= 1e-12 * st.loss
        assert st.loss_new <= st.loss
        if prev is not None:
            assert st.loss <= prev * (1 + 1e-12)
        prev = st.loss_new
    prob.close()


def test_scalar_only_solvers_refuse_vector_residuals():
    d = D()
    p, th = _problem("small")
    prob = d.Problem.from_workload(p)
    lm = torch.tensor(W.landmarks(p.m, 10, 0), device="cuda")
    for solver in (d.PCG, d.STRUCTURED):
        with pytest.raises(d.DngdError) as e:
            prob.step(th, 1e-4, d.step_opts(precision=d.PLAIN, solver=solver, landmarks=lm))
        assert e.value.status == d.EINVAL and "dense solvers only" in str(e.value)
    with pytest.raises(d.DngdError) as e:
        prob.nystrom_pcg(th, 1e-4, lm, np.ones(p.m))
    assert e.value.status == d.EINVAL
    prob.close()
