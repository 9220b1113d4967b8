"""GPU parity of the workflow layers above the step: the D-NGD training loop
(dngd_iterate: damping rule, line search, update), the autograd.Function of
the residual map, and the Nystrom-PCG solver, each against the FP64 oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N
from oracle import nystrom as NY
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


# --------------------------------------------------------------------------
# training loop (a9)

def test_config0_training_20_steps():
    """Config 0 (2-D Poisson, m = 500, plain FP64, lambda = 1e-8, GA): 20
    iterations. The step is checked against the oracle at the GPU's own
    iterates (line-search ties may differ), the line search against the
    oracle's losses, the loss must not increase, and the final relative L2
    error against u* = sin(pi x) sin(pi y) must reach the 1e-2 gate."""
    from paper_2505_21404_amd import driver
    d = D()
    p = W.config(0)
    th0 = W.glorot_theta(p.widths, 0)
    prob = d.Problem.from_workload(p)
    thetas, dirs = [], []
    dbuf = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    theta = torch.tensor(th0, device="cuda")
    hist = []
    for k in range(20):
        thetas.append(theta.cpu().numpy().copy())
        st = prob.iterate(theta, driver.ETA_GRID, fixed_lambda=1e-8,
                          opts=d.step_opts(precision=d.PLAIN, ga=True), dtheta_out=dbuf)
        dirs.append(dbuf.cpu().numpy().copy())
        hist.append(st.as_dict())
        say(f"iter {k} loss {st.loss:.6e} eta {st.eta:.3g} -> {st.loss_new:.6e}")
    thT = theta.cpu().numpy()
    losses = [h["loss"] for h in hist] + [hist[-1]["loss_new"]]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(losses, losses[1:]))
    u64 = np.finfo(np.float64).eps / 2
    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    for k in (0, 7, 19):
        for lam in (1e-8, 1e-6):
            # both sides are backward stable: the GPU's alpha at this iterate
            # has a normwise backward error <= m u64 against the oracle's K
            # and r, and the forward error of the step is bounded by
            # ~ u64 cond(K + lambda I) (conditioning-limited at 1e-8)
            ref = S.dense_step(p, thetas[k], lam, ga=True)
            cond = np.linalg.cond(ref.K + lam * np.eye(p.m))
            dk, _ = prob.step(thetas[k], lam,
                              d.step_opts(precision=d.PLAIN, ga=True, alpha_out=alpha))
            be = S.backward_error(ref.K, lam, alpha.cpu().numpy(), ref.r)
            e = rel(dirs[k] if lam == 1e-8 else dk.cpu().numpy(), ref.dtheta)
            say(f"step {k} lambda {lam:g}: backward error {be:.2e}, rel err vs oracle {e:.2e},"
                f" u64 * cond {u64 * cond:.2e}")
            assert be <= p.m * u64  # backward stability: O(m u64), 5.6e-14 at m = 500
            assert e <= max(1e-10, 10 * u64 * cond)
            if lam == 1e-8:
                assert rel(dk.cpu().numpy(), dirs[k]) == 0.0  # the iterate's own step
                assert hist[k]["step"]["ga_accepted"] == int(ref.accepted)
        # the line search at this iterate against the oracle's losses
        eta, ls = S.line_search(p, thetas[k], dirs[k])
        assert abs(ls.min() - hist[k]["loss_new"]) <= 1e-10 * ls.min() + 1e-300
        assert np.isclose(ls[hist[k]["eta_index"]], ls.min(), rtol=1e-9, atol=0)
    # the update itself: theta_{k+1} = theta_k + eta dtheta
    k = 19
    assert rel(thT, thetas[k] + hist[k]["eta"] * dirs[k]) <= 1e-15
    xe = W.eval_points(p, 10_000, 0)
    l2 = N.relative_l2(p, thT, xe, W.exact_solution("sinsin", xe))
    say("relative L2 after 20 iterations", l2)
    assert l2 <= 1e-2
    prob.close()


@pytest.mark.parametrize("solver", ["PRIMAL", "DENSE_AUTO", "STRUCTURED"])
def test_iterate_with_other_dense_solvers(solver):
    """Five iterations of the workflow (damping rule, GA step, line search,
    update) with the primal, automatic and structured solvers (plain FP64) on
    a problem with n < m: the loss never increases and every step matches the
    oracle's dense step at the GPU's own iterate."""
    d = D()
    p = W.config(0, scale=dict(widths=[2, 16, 16, 1], n_int=300, n_bdy=100))
    theta = torch.tensor(W.glorot_theta(p.widths, 5), device="cuda")
    prob = d.Problem.from_workload(p)
    assert prob.n < prob.m
    opts = d.step_opts(precision=d.PLAIN, solver=getattr(d, solver), ga=True)
    dbuf = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    prev = None
    u64 = np.finfo(np.float64).eps / 2
    for k in range(5):
        th_k = theta.cpu().numpy().copy()
        st = prob.iterate(theta, [2.0 ** -j for j in range(31)], lam_cap=1e-3, opts=opts,
                          dtheta_out=dbuf)
        ref = S.dense_step(p, th_k, st.lam, ga=True)
        cond = np.linalg.cond(ref.K + st.lam * np.eye(p.m))
        e = rel(dbuf.cpu().numpy(), ref.dtheta)
        say("solver", solver, "iter", k, "loss", st.loss, "lam", st.lam, "err", e,
            "primal", st.step.primal)
        assert e <= max(1e-10, 100 * u64 * cond)
        assert st.step.ga_accepted == int(ref.accepted)
        assert st.step.primal == (1 if solver != "STRUCTURED" else 0)
        assert st.loss_new <= st.loss * (1 + 1e-12)
        if prev is not None:
            assert abs(st.loss - prev) <= 1e-12 * prev
        prev = st.loss_new
        eta, ls = S.line_search(p, th_k, dbuf.cpu().numpy())
        assert abs(ls.min() - st.loss_new) <= 1e-10 * ls.min()
    prob.close()


def test_driver_train_damping_rule():
    """driver.train with the damping rule lambda_k = min(L(theta_k), cap):
    the lambda it reports is min(loss, cap) and theta moves as recorded."""
    from paper_2505_21404_amd import driver
    d = D()
    p = W.config(1, scale=dict(widths=[5, 24, 24, 1], n_int=300, n_bdy=80))
    th0 = W.glorot_theta(p.widths, 3)
    prob = d.Problem.from_workload(p)
    theta, hist = driver.train(prob, th0, 4, lam_cap=1e-5, opts=d.step_opts(precision=d.MIXED))
    for h in hist:
        assert h["lam"] == min(h["loss"], 1e-5)
        assert h["loss_new"] <= h["loss"]
    assert abs(hist[0]["loss"] - N.loss(p, th0)) <= 1e-12 * hist[0]["loss"]
    assert abs(N.loss(p, theta.cpu().numpy()) - hist[-1]["loss_new"]) <= 1e-10 * hist[-1]["loss_new"]
    prob.close()


# --------------------------------------------------------------------------
# autograd.Function (a13)

def test_autograd_gradcheck_and_oracle_gradient():
    from paper_2505_21404_amd import autograd as AG
    d = D()
    p = W.heat_problem([3, 6, 5, 1], 9, 4, 3, 0.2, 11)
    prob = d.Problem.from_workload(p)
    th0 = 0.8 * np.random.default_rng(2).standard_normal(p.n_params)
    th = torch.tensor(th0, device="cuda", requires_grad=True)
    say("case gradcheck heat", p.widths, p.m)
    assert torch.autograd.gradcheck(lambda t: AG.residual(prob, t), (th,), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)
    # backward against the oracle's J^T r_bar, and the loss gradient J^T r
    rbar = np.random.default_rng(3).standard_normal(p.m)
    r = AG.residual(prob, th)
    (g,) = torch.autograd.grad(r, th, torch.tensor(rbar, device="cuda"))
    J = N.jacobian(p, th0)
    assert rel(g.cpu().numpy(), J.T @ rbar) <= 1e-12
    th.grad = None
    AG.loss(prob, th).backward()
    assert rel(th.grad.cpu().numpy(), J.T @ N.residual(p, th0)) <= 1e-12
    prob.close()


def test_autograd_backward_directional_fd_heat_full_size():
    """The heat workload at full size (MLP 3-1024x4-1, n = 3,153,921,
    m = 8192): the backward of the autograd.Function (theta_bar = J^T r_bar,
    dngd_vjp) against central differences of r_bar . r(theta + eps u) along
    three directions: the gradient's own direction (where the derivative is
    ||J^T r_bar||) and two random ones. A full gradcheck (n forward passes) is
    out of reach at this size; directional derivatives test the same map."""
    from paper_2505_21404_amd import autograd as AG
    d = D()
    p = W.config(2)
    th0 = W.glorot_theta(p.widths, 0)
    say("case autograd directional FD, heat full size: n", th0.size, "m", p.m)
    prob = d.Problem.from_workload(p)
    th = torch.tensor(th0, device="cuda", requires_grad=True)
    rbar = torch.tensor(W.random_direction(p.m, 5), device="cuda")
    r = AG.residual(prob, th)
    (g,) = torch.autograd.grad(r, th, rbar)
    g = g.detach()
    gn = float(torch.linalg.norm(g))
    base = th.detach()
    dirs = [g / gn] + [torch.tensor(W.random_direction(th0.size, 20 + k), device="cuda")
                       for k in range(2)]
    def central(u, eps):
        fp = float(rbar @ prob.residual(base + eps * u))
        fm = float(rbar @ prob.residual(base - eps * u))
        return (fp - fm) / (2 * eps)

    for k, u in enumerate(dirs):
        u = u / torch.linalg.norm(u)
        # Richardson extrapolation of two central differences: truncation O(eps^4),
        # cancellation ~1e-16 |r_bar . r| / eps, both far below 1e-6 ||J^T r_bar||
        eps = 2e-4
        fd = (4.0 * central(u, eps / 2) - central(u, eps)) / 3.0
        an = float(g @ u)
        say(f"  direction {k}: extrapolated central difference {fd:.12g}, J^T r_bar . u "
            f"{an:.12g}, difference / ||J^T r_bar|| {abs(fd - an) / gn:.2e}")
        assert abs(fd - an) <= 1e-6 * gn
    assert abs(float(g @ dirs[0]) - gn) <= 1e-12 * gn
    prob.close()


# --------------------------------------------------------------------------
# Nystrom-PCG (a10 - a12)

def _pcg_case(ell, lam, tol, seed=0):
    d = D()
    p = W.config(1, scale=dict(widths=[5, 32, 32, 1], n_int=240, n_bdy=60))
    th = W.glorot_theta(p.widths, seed)
    prob = d.Problem.from_workload(p)
    r = N.residual(p, th)
    J = N.jacobian(p, th)
    I = W.landmarks(p.m, ell, seed)
    x, st, rc = prob.nystrom_pcg(th, lam, torch.tensor(I), r, tol=tol, maxit=500)
    return d, p, th, prob, r, J, I, x.cpu().numpy(), st, rc


@pytest.mark.parametrize("ell", [30, 120])
def test_pcg_matches_dense_solution(ell):
    lam, tol = 1e-4, 1e-10
    d, p, th, prob, r, J, I, x, st, rc = _pcg_case(ell, lam, tol)
    say("case pcg ell", ell, "iters", st.pcg_iterations, "rel res", st.pcg_rel_residual)
    assert rc == d.OK and st.pcg_converged
    K = J @ J.T
    alpha = S.solve(S.cholesky(K, lam), r)
    # the true residual in FP64 and the distance to the dense solution
    true_res = np.linalg.norm((K + lam * np.eye(p.m)) @ x - r) / np.linalg.norm(r)
    assert true_res <= 10 * tol
    cond = np.linalg.cond(K + lam * np.eye(p.m))
    assert rel(x, alpha) <= 10 * tol * cond
    # iteration count against the oracle's PCG with the same landmarks
    _, _, its_o, ok_o = NY.pcg_step(J, r, lam, I, tol, 500)
    say("iterations gpu", st.pcg_iterations, "oracle", its_o)
    assert ok_o and abs(st.pcg_iterations - its_o) <= max(2, its_o // 5)
    prob.close()


def test_pcg_all_landmarks_converges_at_once():
    """ell = m: the preconditioner is (K + lam I)^{-1} up to the K_II shift,
    so PCG stops after one or two iterations."""
    d, p, th, prob, r, J, I, x, st, rc = _pcg_case(300, 1e-3, 1e-8)
    say("case pcg ell = m, iters", st.pcg_iterations)
    assert rc == d.OK and st.pcg_iterations <= 2
    prob.close()


def test_pcg_step_matches_oracle_step():
    """dngd_step with the PCG solver (no GA) against the oracle's dense step."""
    d = D()
    p = W.config(1, scale=dict(widths=[5, 32, 32, 1], n_int=240, n_bdy=60))
    th = W.glorot_theta(p.widths, 1)
    lam = 1e-4
    prob = d.Problem.from_workload(p)
    I = torch.tensor(W.landmarks(p.m, 60, 1))
    o = d.step_opts(solver=d.PCG, ga=False, landmarks=I.cuda(), pcg_tol=1e-10, pcg_maxit=500)
    dth, st = prob.step(th, lam, o)
    ref = S.dense_step(p, th, lam, ga=False)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    say("pcg step rel err", e, "iters", st.pcg_iterations)
    assert st.pcg_converged and e <= 1e-6
    prob.close()


@pytest.mark.parametrize("ell,seed", [(60, 1), (300, 2), (120, 5)])
def test_pcg_step_with_ga_matches_oracle_step(ell, seed):
    """dngd_step with the PCG solver and GA: f_vv along the PCG step v, a
    second PCG solve with the same Nystrom preconditioner for beta, a =
    -J^T beta and the acceptance test, against the oracle's dense GA step
    (same mathematics, exact solves)."""
    d = D()
    p = W.config(1, scale=dict(widths=[5, 32, 32, 1], n_int=240, n_bdy=60))
    th = W.glorot_theta(p.widths, seed)
    lam = 1e-4
    prob = d.Problem.from_workload(p)
    I = torch.tensor(W.landmarks(p.m, ell, seed))
    fvv = torch.empty(p.m, dtype=torch.float64, device="cuda")
    o = d.step_opts(solver=d.PCG, ga=True, landmarks=I.cuda(), pcg_tol=1e-10, pcg_maxit=500,
                    fvv_out=fvv)
    dth, st = prob.step(th, lam, o)
    ref = S.dense_step(p, th, lam, ga=True)
    e = rel(dth.cpu().numpy(), ref.dtheta)
    say("pcg+ga ell", ell, "seed", seed, "iters", st.pcg_iterations, st.pcg_iterations_ga,
        "accepted", st.ga_accepted, "oracle", ref.accepted, "rel err", e)
    assert st.pcg_converged and st.pcg_iterations_ga >= 1
    assert st.ga_accepted == int(ref.accepted)
    assert rel(fvv.cpu().numpy(), ref.fvv) <= 1e-6
    assert abs(st.anorm - np.linalg.norm(ref.a)) <= 1e-6 * np.linalg.norm(ref.a)
    assert abs(st.vnorm - np.linalg.norm(ref.v)) <= 1e-8 * np.linalg.norm(ref.v)
    assert e <= 1e-6
    prob.close()


# --------------------------------------------------------------------------
# mixed precision on a stiff serving job: the adaptive Gram

def test_mixed_step_escalates_on_stiff_job():
    """A 2-D Poisson job of the serving stream (width 128, m = 1100,
    lambda = 1e-5) whose bf16 Gram is too coarse after the first update: the
    mixed step must escalate (4 products, then FP64 products) and still
    match the oracle's step to the mixed tolerance at every iterate."""
    from paper_2505_21404_amd import serving as SV
    d = D()
    spec = SV.specs_from_workloads(W.serving_jobs(n_jobs=37, rate=4.0, steps=3))[36]
    p = spec.problem
    assert p.pde == 0 and p.widths[1] == 128 and p.m == 1100
    prob = d.Problem.from_workload(p)
    theta = torch.tensor(spec.theta0, device="cuda")
    dbuf = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    for k in range(3):
        th_k = theta.cpu().numpy().copy()
        st = prob.iterate(theta, SV.ETA_GRID, lam_cap=spec.lam_cap,
                          opts=d.step_opts(precision=d.MIXED, ga=True), dtheta_out=dbuf)
        ref = S.dense_step(p, th_k, st.lam, ga=True)
        e = rel(dbuf.cpu().numpy(), ref.dtheta)
        say(f"iter {k} lam {st.lam:.3g} passes {st.step.gram_passes_used} attempts "
            f"{st.step.gram_attempts} ir {list(st.step.ir_residual)[:2]} rel err {e:.3e}")
        assert e <= 1e-4
    prob.close()


def test_stiff_job_remembers_its_gram_tier():
    """The handle remembers the Gram tier its adaptive step escalated to and
    the damping it escalated at. On the same stiff serving job: once a step
    has escalated, later steps at that damping or below start at the
    remembered tier (one attempt for the FP64 tier) and still match the
    oracle; the step equals a fresh handle's step bit for bit when both end
    on the same tier; a larger damping clears the memory."""
    from paper_2505_21404_amd import serving as SV
    d = D()
    spec = SV.specs_from_workloads(W.serving_jobs(n_jobs=37, rate=4.0, steps=3))[36]
    p = spec.problem
    prob = d.Problem.from_workload(p)
    theta = torch.tensor(spec.theta0, device="cuda")
    dbuf = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    opts = d.step_opts(precision=d.MIXED, ga=True)
    hint, hint_lam = 0, 0.0
    for k in range(4):
        th_k = theta.cpu().numpy().copy()
        st = prob.iterate(theta, SV.ETA_GRID, lam_cap=spec.lam_cap, opts=opts, dtheta_out=dbuf)
        s_ = st.step
        say(f"iter {k} lam {st.lam:.3g} start {s_.gram_start_passes} used {s_.gram_passes_used} "
            f"attempts {s_.gram_attempts}")
        if hint and st.lam <= hint_lam:
            assert s_.gram_start_passes == hint
            if hint == d.GRAM_F64:
                assert s_.gram_attempts == 1
            e = rel(dbuf.cpu().numpy(), S.dense_step(p, th_k, st.lam, ga=True).dtheta)
            say(f"  remembered tier, rel err {e:.2e}")
            assert e <= 1e-4
        if s_.gram_attempts > 1:
            hint, hint_lam = s_.gram_passes_used, st.lam
    assert hint != 0, "the job did not escalate"
    # a fresh handle at the same theta and damping: same step when the tier agrees
    d1, st1 = prob.step(theta, hint_lam, opts)
    fresh = d.Problem.from_workload(p)
    d2, st2 = fresh.step(theta, hint_lam, opts)
    say(f"hinted: start {st1.gram_start_passes} used {st1.gram_passes_used} attempts "
        f"{st1.gram_attempts}; fresh: start {st2.gram_start_passes} used "
        f"{st2.gram_passes_used} attempts {st2.gram_attempts}")
    assert st1.gram_start_passes == hint and st2.gram_start_passes <= hint
    if st2.gram_passes_used == st1.gram_passes_used:
        assert torch.equal(d1, d2)
    fresh.close()
    # a larger damping starts from the auto choice and clears the memory
    st3 = prob.step(theta, 1e3 * hint_lam, opts)[1]
    if st3.gram_attempts == 1:
        st4 = prob.step(theta, hint_lam, opts)[1]
        assert st4.gram_start_passes == st2.gram_start_passes
    prob.close()


@pytest.mark.parametrize("m,n,ld", [(300, 7001, 7004), (129, 5, 8), (700, 33, 36), (1, 64, 64),
                                    (257, 3000, 3000)])
def test_gram_f64_products_of_fp32_jacobian(m, n, ld):
    """dngd_gram with FP32 J and passes = DNGD_GRAM_F64: the exact Gram of the
    FP32 values up to FP64 rounding, on the K-contiguous kernel that widens
    FP32 at the LDS read (ragged 128-row tiles, K below one 32-element stage,
    a partial last stage, a single row). An FP32 J whose row stride is not a
    multiple of 4 is rejected."""
    d = D()
    rng = np.random.default_rng(4 + m)
    J = (rng.standard_normal((m, n)) * rng.uniform(0.1, 3.0, size=(m, 1))).astype(np.float32)
    Jp = np.zeros((m, ld), dtype=np.float32)
    Jp[:, :n] = J
    K = d.gram(torch.tensor(Jp, device="cuda"), n, 0.5, passes=d.GRAM_F64).cpu().numpy()
    J64 = J.astype(np.float64)
    ref = J64 @ J64.T + 0.5 * np.eye(m)
    low = np.tril_indices(m)
    assert np.abs(K[low] - ref[low]).max() <= 1e-13 * np.abs(ref).max()
    if n % 4:
        with pytest.raises(d.DngdError) as err:
            d.gram(torch.tensor(J, device="cuda"), n, 0.5, passes=d.GRAM_F64)
        assert err.value.status == d.EINVAL


def test_pcg_heat_all_landmarks_and_partial():
    """Heat problem (three residual classes, 5 jet rows per interior point):
    with every residual a landmark the preconditioner inverts K + lam I, and
    with a subset PCG still reaches the dense solution."""
    d = D()
    p = W.heat_problem([3, 24, 24, 1], 180, 40, 40, 0.2, 12)
    th = W.glorot_theta(p.widths, 2)
    prob = d.Problem.from_workload(p)
    r = N.residual(p, th)
    J = N.jacobian(p, th)
    lam = 1e-3
    alpha = S.solve(S.cholesky(J @ J.T, lam), r)
    for ell, max_it in ((p.m, 2), (60, 500)):
        I = W.landmarks(p.m, ell, 4)
        x, st, rc = prob.nystrom_pcg(th, lam, torch.tensor(I), r, tol=1e-10, maxit=500)
        say("heat pcg ell", ell, "iters", st.pcg_iterations)
        assert rc == d.OK and st.pcg_iterations <= max_it
        assert rel(x.cpu().numpy(), alpha) <= 1e-6
    prob.close()
