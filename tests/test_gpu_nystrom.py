"""GPU parity of the Nystrom preconditioner and the PCG path (Section 3.3, the
Nystrom construction and PCGStep algorithms) beyond iteration counts:

* the applied preconditioner, element by element: one PCG iteration from
  y = 0 returns y1 = (b.z / z.Az) z with z = P^{-1} b, so the GPU's y1 is
  compared with the oracle's (K^ + lam I)^{-1} b built with the GPU's K_II
  shift delta (reading: the shift keeps K_II factorisable), at ell = m and
  ell < m;
* the landmark-column build split into several chunks of jet rows (as the
  large workload runs it) against one chunk and against the oracle, on a
  small problem and on the 5-D Poisson workload (m = 5000, width 256);
* reuse of the Nystrom factors across steps (built once, reused);
* the large matrix-free workload at full size (m = 50,000, n = 12.6M): the
  FP64 true residual of the PCG solution and sampled r and f_vv rows."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import network as N
from oracle import nystrom as NY
from oracle import step as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD1 = os.path.join(os.path.dirname(__file__), "golden", "config1_step.npz")


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small():
    p = W.config(1, scale=dict(widths=[5, 32, 32, 1], n_int=240, n_bdy=60))
    return p, W.glorot_theta(p.widths, 1)


@pytest.mark.parametrize("ell", [300, 60])
def test_preconditioner_applied_elementwise(ell):
    d = D()
    p, th = small()
    lam = 1e-4
    prob = d.Problem.from_workload(p)
    r = N.residual(p, th)
    I = W.landmarks(p.m, ell, 2)
    x, st, rc = prob.nystrom_pcg(th, lam, torch.tensor(I), r, tol=0.0, maxit=1)
    assert rc == d.ENOCONV and st.pcg_iterations == 1
    delta = st.nystrom_shift
    J = N.jacobian(p, th)
    K = J @ J.T
    Khat, _ = NY.nystrom_approx(K[:, I], I, delta=delta)
    A = K + lam * np.eye(p.m)
    z = np.linalg.solve(Khat + lam * np.eye(p.m), r)
    y1 = (r @ z) / (z @ (A @ z)) * z
    e = rel(x.cpu().numpy(), y1)
    say(f"ell {ell}: delta {delta:.3e}, P^-1 b (scaled) rel err {e:.2e}")
    assert delta > 0 and e <= 1e-9
    if ell == p.m:
        # all landmarks: P^{-1} = (K + lam I)^{-1} up to the shift
        alpha = np.linalg.solve(A, r)
        assert rel(z, alpha) <= 10 * delta / lam
    prob.close()


def test_chunked_landmark_columns_small():
    """The landmark-column products in chunks of 500 jet rows (4 chunks of the
    1740 rows) give the same step as one chunk, and the oracle's step."""
    d = D()
    p, th = small()
    lam = 1e-4
    prob = d.Problem.from_workload(p)
    I = torch.tensor(W.landmarks(p.m, 60, 1)).cuda()
    out = []
    for rows in (0, 500):
        o = d.step_opts(precision=d.PLAIN, solver=d.PCG, ga=True, landmarks=I, pcg_tol=1e-10,
                        nystrom_chunk_rows=rows)
        dth, st = prob.step(th, lam, o)
        say(f"chunk rows {rows}: iterations {st.pcg_iterations}/{st.pcg_iterations_ga}")
        out.append((dth.cpu().numpy(), st))
    assert rel(out[1][0], out[0][0]) <= 1e-12
    assert out[1][1].pcg_iterations == out[0][1].pcg_iterations
    ref = S.dense_step(p, th, lam, ga=True)
    assert rel(out[1][0], ref.dtheta) <= 1e-6
    prob.close()


def test_chunked_pcg_step_5d_poisson_m5000():
    """The 5-D Poisson workload (m = 5000, width 256, n = 133,377), PCG with
    GA and 1000 landmarks, landmark columns in three chunks of jet rows,
    against the stored oracle dense step (tests/golden/config1_step.npz)."""
    d = D()
    p = W.config(1)
    th = W.glorot_theta(p.widths, 0)
    g = np.load(GOLD1)
    lam = float(g["lam"])
    prob = d.Problem.from_workload(p)
    I = torch.tensor(W.landmarks(p.m, 1000, 0)).cuda()
    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    R = 4000 * 7 + 1000
    o = d.step_opts(precision=d.PLAIN, solver=d.PCG, ga=True, landmarks=I, pcg_tol=1e-10,
                    pcg_maxit=2000, nystrom_chunk_rows=R // 3 + 1, alpha_out=alpha)
    dth, st = prob.step(th, lam, o)
    e = rel(dth.cpu().numpy(), g["dtheta"])
    ea = rel(alpha.cpu().numpy(), g["alpha"])
    say(f"m=5000 PCG+GA: iterations {st.pcg_iterations}/{st.pcg_iterations_ga}, rel res "
        f"{st.pcg_rel_residual:.2e}, dtheta rel err {e:.2e}, alpha rel err {ea:.2e}, "
        f"accepted {st.ga_accepted} (oracle {int(g['accepted'])}), {st.ms_total:.0f} ms")
    assert st.pcg_converged and st.ga_accepted == int(g["accepted"])
    assert e <= 1e-6
    prob.close()


def test_nystrom_reuse_across_steps():
    """nystrom_reuse = 2: the first PCG step builds the factors, the next two
    reuse them (only the small system is refactored when lambda changes), the
    fourth rebuilds. Every step still converges to the dense solution. The
    parameters move by 1% of the step between calls: factors from far away
    (half a Gauss-Newton step at the Glorot start) leave K's new leading
    directions unpreconditioned and PCG needs thousands of iterations."""
    d = D()
    p, th = small()
    prob = d.Problem.from_workload(p)
    I = torch.tensor(W.landmarks(p.m, 80, 3)).cuda()
    theta = th.copy()
    flags = []
    for k, lam in enumerate((1e-4, 1e-4, 3e-4, 1e-4)):
        o = d.step_opts(precision=d.PLAIN, solver=d.PCG, ga=False, landmarks=I, pcg_tol=1e-10,
                        pcg_maxit=3000, nystrom_reuse=2)
        dth, st = prob.step(theta, lam, o)
        ref = S.dense_step(p, theta, lam, ga=False)
        e = rel(dth.cpu().numpy(), ref.dtheta)
        say(f"step {k}: lam {lam:g} reused {st.nystrom_reused} iterations {st.pcg_iterations}"
            f" rel err {e:.2e}")
        flags.append(st.nystrom_reused)
        assert st.pcg_converged and e <= 1e-6
        theta = theta + 0.01 * dth.cpu().numpy()
    assert flags == [0, 1, 1, 0]
    # a dense step on the handle invalidates the stored factors
    prob.step(theta, 1e-4, d.step_opts(precision=d.PLAIN, ga=False))
    _, st = prob.step(theta, 1e-4, d.step_opts(precision=d.PLAIN, solver=d.PCG, ga=False,
                                               landmarks=I, nystrom_reuse=2))
    assert st.nystrom_reused == 0
    prob.close()


def test_large_pcg_workload_full_size():
    """5-D Poisson, MLP 5-2048x4-1 (n = 12,603,393), m = 50,000, 2000
    landmarks, tolerance 1e-6, with GA. The FP64 true residual of the PCG
    solution, ||(J J^T + lam I) alpha - r|| / ||r||, from the matrix-free FP64
    products (dngd_vjp then dngd_jvp), is within 10 tol; r and f_vv on sampled
    residuals match the oracle's per-point values."""
    d = D()
    p = W.config(3)
    th = W.glorot_theta(p.widths, 0)
    say("case large PCG workload: m", p.m, "n", p.n_params)
    prob = d.Problem.from_workload(p)
    thd = torch.tensor(th, device="cuda")
    r = prob.residual(thd)
    r_np = r.cpu().numpy()
    rng = np.random.default_rng(7)
    idx = np.sort(np.concatenate([rng.choice(p.n_int, 12, replace=False),
                                  p.n_int + rng.choice(p.n_bdy, 12, replace=False)]))
    assert rel(r_np[idx], N.residual_rows(p, th, idx)) <= 1e-12
    lam = min(0.5 * float(r_np @ r_np), W.LAMBDA_CAP[3])
    tol = 1e-6
    I = torch.tensor(W.landmarks(p.m, 2000, 0)).cuda()
    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    fvv = torch.empty(p.m, dtype=torch.float64, device="cuda")
    o = d.step_opts(precision=d.PLAIN, solver=d.PCG, ga=True, landmarks=I, pcg_tol=tol,
                    pcg_maxit=500, alpha_out=alpha, fvv_out=fvv)
    dth, st = prob.step(thd, lam, o)
    say(f"step {st.ms_total / 1e3:.2f} s: iterations {st.pcg_iterations}/{st.pcg_iterations_ga}"
        f", recursive rel res {st.pcg_rel_residual:.2e}, shift {st.nystrom_shift:.2e}")
    assert st.pcg_converged
    u = prob.jvp(thd, prob.vjp(thd, alpha))
    true_res = float(torch.linalg.norm(u + lam * alpha - r) / torch.linalg.norm(r))
    say(f"FP64 true residual {true_res:.2e} (tol {tol:g})")
    assert true_res <= 10 * tol
    v64 = (-prob.vjp(thd, alpha)).cpu().numpy()
    f_o = N.fvv_rows(p, th, v64, idx)
    e_f = rel(fvv.cpu().numpy()[idx], f_o)
    say(f"f_vv rows vs oracle {e_f:.2e}")
    assert e_f <= 1e-10
    assert np.all(np.isfinite(dth.cpu().numpy()))
    prob.close()
