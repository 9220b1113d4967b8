"""Failure paths forced from the host: a non-finite parameter vector gives
DNGD_ENAN on every solver, PCG stopped at maxit gives DNGD_ENOCONV with a
finite last iterate, and the serving loop queues jobs when the memory budget
admits one at a time and rejects jobs that can never fit. Every kernel runs
to its normal end in these cases. A step that fails (a Gram precision fixed
too low for the damping: DNGD_ENOTPD) leaves the handle usable: the next
step is finite and the same as on a fresh handle."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def _small():
    p = W.config(0, scale=dict(widths=[2, 12, 12, 1], n_int=120, n_bdy=40))
    return p, W.glorot_theta(p.widths, 11)


@pytest.mark.parametrize("solver,precision", [("DENSE", "PLAIN"), ("DENSE", "MIXED"),
                                              ("PRIMAL", "MIXED"), ("STRUCTURED", "PLAIN"),
                                              ("PCG", "PLAIN")])
def test_non_finite_theta_gives_enan(solver, precision):
    d = D()
    p, th = _small()
    prob = d.Problem.from_workload(p)
    bad = th.copy()
    bad[5] = np.nan
    lm = torch.tensor(W.landmarks(p.m, 20, 0), device="cuda")
    opts = d.step_opts(precision=getattr(d, precision), solver=getattr(d, solver), ga=True,
                       landmarks=lm if solver == "PCG" else None)
    say("case NaN theta", solver, precision)
    with pytest.raises(d.DngdError) as e:
        prob.step(bad, 1e-4, opts)
    assert e.value.status == d.ENAN, str(e.value)
    # the handle stays usable: a finite theta steps normally afterwards
    dth, _ = prob.step(th, 1e-4, opts)
    assert torch.isfinite(dth).all()
    prob.close()


def test_iterate_rejects_non_finite_loss():
    d = D()
    p, th = _small()
    prob = d.Problem.from_workload(p)
    theta = torch.tensor(th, device="cuda")
    theta[0] = float("inf")
    with pytest.raises(d.DngdError) as e:
        prob.iterate(theta, [1.0, 0.5], lam_cap=1e-3)
    assert e.value.status == d.EINVAL and "non-finite loss" in str(e.value)
    prob.close()


def test_pcg_maxit_gives_enoconv_with_finite_iterate():
    d = D()
    p, th = _small()
    prob = d.Problem.from_workload(p)
    lam = 1e-4
    r = N.residual(p, th)
    lm = torch.tensor(W.landmarks(p.m, 8, 0), device="cuda")
    say("case PCG maxit 1 via dngd_nystrom_pcg")
    x, st, rc = prob.nystrom_pcg(th, lam, lm, r, tol=1e-12, maxit=1)
    assert rc == d.ENOCONV
    assert st.pcg_iterations == 1 and st.pcg_converged == 0
    xh = x.cpu().numpy()
    assert np.all(np.isfinite(xh))
    # the reported residual is the true one of the returned iterate (oracle K)
    J = N.jacobian(p, th)
    true_rel = np.linalg.norm(r - (J @ (J.T @ xh) + lam * xh)) / np.linalg.norm(r)
    # (one iteration minimises the error in the A-norm; the residual's 2-norm
    # need not fall below ||b||)
    assert 0.0 < st.pcg_rel_residual < np.inf
    assert abs(st.pcg_rel_residual - true_rel) <= 1e-8 * max(true_rel, 1.0)
    say("case PCG maxit 1 via dngd_step")
    opts = d.step_opts(precision=d.PLAIN, solver=d.PCG, ga=False, landmarks=lm, pcg_tol=1e-12,
                       pcg_maxit=1)
    dth, st2 = prob.step(th, lam, opts)
    assert st2.pcg_converged == 0 and st2.pcg_iterations == 1
    assert torch.isfinite(dth).all()
    prob.close()


def _small_stream(n=4, steps=2):
    from paper_2505_21404_amd import serving as SV
    jobs = W.serving_jobs(n_jobs=n, rate=40.0, steps=steps, m_range=(600, 1400),
                          widths_choice=(32,), depth=3)
    return SV.specs_from_workloads(jobs)


def test_serving_budget_forces_queueing_and_rejection():
    from paper_2505_21404_amd import serving as SV
    specs = _small_stream()
    fp, _ = SV.gpu_executor()
    fps = sorted(fp(s) for s in specs)
    # room for the largest job but never for two: strictly one at a time
    budget = max(fps[-1], 1)
    assert fps[0] + fps[1] > budget
    srv = SV.Server(budget_bytes=budget, max_slots=4)
    rep = srv.run(specs, realtime=False)
    say("queued run", {k: v for k, v in rep.items() if k != "results"})
    assert rep["rejected"] == 0 and not rep["errors"]
    assert srv.peak_slots == 1 and srv.peak_bytes <= budget
    assert rep["steps"] == sum(s.steps for s in specs)
    # below the smallest footprint every job is rejected and nothing runs
    srv = SV.Server(budget_bytes=fps[0] - 1, max_slots=4)
    rep = srv.run(specs, realtime=False)
    assert rep["rejected"] == len(specs) and rep["steps"] == 0


def test_failed_step_leaves_the_handle_usable():
    """A stiff 2-D Poisson job of the serving stream (m = 5742, width 256):
    a mixed step with the 3-pass Gram fixed (indefinite by about 2^-16
    max ||J_i||^2, far above lambda) fails to factor (DNGD_ENOTPD) and
    runs to its end with a non-finite factor. The next automatic step on the
    handle (whose GA correction is rejected before the acceleration is
    formed) must be finite and equal, bit for bit, to the same step on a
    fresh handle, which escalates to the same Gram tier."""
    from paper_2505_21404_amd import serving as SV
    d = D()
    sp = SV.specs_from_workloads(W.serving_jobs(n_jobs=8, rate=4.0, steps=200))[4]
    p = sp.problem
    assert p.pde == 0 and p.m == 5742
    auto = d.step_opts(precision=d.MIXED, ga=True, no_lookahead=True)
    prob = d.Problem.from_workload(p)
    th = torch.tensor(sp.theta0, device="cuda")
    st = prob.iterate(th, SV.ETA_GRID, lam_cap=sp.lam_cap, opts=auto)
    lam = st.lam
    with pytest.raises(d.DngdError) as err:
        prob.step(th, lam, d.step_opts(precision=d.MIXED, ga=True, no_lookahead=True,
                                       gram_passes=3))
    assert err.value.status == d.ENOTPD
    d1, s1 = prob.step(th, lam, auto)
    fresh = d.Problem.from_workload(p)
    d2, s2 = fresh.step(th, lam, auto)
    say(f"after the failed step: finite {bool(torch.isfinite(d1).all())}, tier "
        f"{s1.gram_passes_used} (fresh handle {s2.gram_passes_used}), early GA rejection "
        f"{s1.ga_early_reject}")
    assert torch.isfinite(d1).all()
    assert s1.gram_passes_used == s2.gram_passes_used and torch.equal(d1, d2)
    fresh.close()
    prob.close()
