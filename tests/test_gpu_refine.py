"""The dense dual solve with iterative refinement through J
(dngd_cholesky_solve_refine; Section 4.1, the DenseDualSolve algorithm):
B <- (J J^T + lam I)^{-1} B with a reduced-precision Gram's Cholesky factor as
the inner solver, against the oracle's FP64 solve with the same J.

* FP32 J, 1- and 3-pass bf16 Gram: the refined solution reaches the FP64
  solution within a small multiple of u64 kappa, the per-sweep residuals
  shrink, and more sweeps help where the factor is crude.
* FP64 J and FP64 Gram: two sweeps, same bar.
* several right-hand sides (one zero), ragged n, an already factored K,
  sweeps = 0 against dngd_cholesky_solve bit for bit, and a K that is not
  positive definite (DNGD_ENOTPD with the failing column)."""
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


def setup(dtype, lam_rel, seed=0):
    """J (FP32 or FP64, m x ldJ zero-padded, ldJ a multiple of 4) of a small
    5-D Poisson problem with a ragged n, the FP64 operator it stands for, the
    damping lam = lam_rel max_i ||J_i||^2 and the condition number of
    J J^T + lam I. The damping keeps the reduced-precision factor a
    contraction (its error times kappa below 1)."""
    p = W.config(1, scale=dict(widths=[5, 24, 24, 1], n_int=400, n_bdy=130))
    th = W.glorot_theta(p.widths, seed)
    J = N.jacobian(p, th)
    m, n = J.shape
    Jd = J.astype(np.float32).astype(np.float64) if dtype == torch.float32 else J
    ldJ = (n + 3) // 4 * 4 + 4
    Jp = np.zeros((m, ldJ))
    Jp[:, :n] = Jd
    lam = lam_rel * float(np.max(np.sum(Jd * Jd, axis=1)))
    kappa = float(np.linalg.cond(S.gram(Jd) + lam * np.eye(m)))
    return p, th, torch.tensor(Jp, dtype=dtype, device="cuda"), Jd, n, lam, kappa


# (passes, sweeps, damping relative to max ||J_i||^2): an FP64 simulation of
# the refinement with bf16-rounded operands reaches the bar after 4 and 6
# sweeps in these two cases (8e-12 against 3e-10, 5e-12 against 3e-11)
@pytest.mark.parametrize("passes,sweeps,lam_rel", [(3, 4, 1e-3), (1, 8, 1e-2)])
def test_refined_solve_fp32_j_reaches_fp64_solution(passes, sweeps, lam_rel):
    d = D()
    p, th, Jt, Jd, n, lam, kappa = setup(torch.float32, lam_rel)
    m = Jd.shape[0]
    say(f"case refine FP32 J passes {passes} sweeps {sweeps}: m {m} n {n} lam {lam:.2e} "
        f"kappa {kappa:.2e}")
    r = N.residual(p, th)
    b = np.stack([r, W.random_direction(m, 5)])
    ref = np.stack([S.solve(S.cholesky(S.gram(Jd), lam), bj) for bj in b])
    K = d.gram(Jt, n, lam, passes=passes)
    B0 = torch.tensor(b, device="cuda")
    Kc = K.clone()
    info = d.cholesky_solve(Kc, B0.clone())
    assert info == 0
    B = B0.clone()
    info, res = d.cholesky_solve_refine(K, B, Jt, n, lam, sweeps)
    assert info == 0 and res.shape == (2, sweeps)
    X = B.cpu().numpy()
    # without refinement (the factor alone)
    B_plain = B0.clone()
    assert d.cholesky_solve(Kc, B_plain, factored=True) == 0
    e0 = max(rel(B_plain.cpu().numpy()[j], ref[j]) for j in range(2))
    e = max(rel(X[j], ref[j]) for j in range(2))
    bar = max(1e-13, 20 * U64 * kappa)
    say(f"  factor alone {e0:.2e}, refined {e:.2e} (bar {bar:.2e}); rel residuals {res.tolist()}")
    assert e <= bar
    assert e0 >= 10 * e
    for j in range(2):
        assert res[j, -1] < res[j, 0]
        # the reported residual is the exact residual of the iterate before the last correction
        assert res[j, -1] <= 1e-6
    # the backward error of the returned solution in the FP64 operator
    for j in range(2):
        assert S.backward_error(S.gram(Jd), lam, X[j], b[j]) <= 1e-14


def test_refined_solve_fp64_j():
    d = D()
    p, th, Jt, Jd, n, lam, kappa = setup(torch.float64, 1e-6, seed=2)
    m = Jd.shape[0]
    say(f"case refine FP64 J: m {m} n {n} kappa {kappa:.2e}")
    b = W.random_direction(m, 9)
    ref = S.solve(S.cholesky(S.gram(Jd), lam), b)
    K = d.gram(Jt, n, lam, passes=1)
    B = torch.tensor(b, device="cuda")
    info, res = d.cholesky_solve_refine(K, B, Jt, n, lam, 2)
    e = rel(B.cpu().numpy(), ref)
    bar = max(1e-13, 20 * U64 * kappa)
    say(f"  refined {e:.2e} (bar {bar:.2e}); rel residuals {res.tolist()}")
    assert info == 0 and e <= bar


def test_refined_solve_edge_cases():
    d = D()
    p, th, Jt, Jd, n, lam, kappa = setup(torch.float32, 1e-3, seed=4)
    m = Jd.shape[0]
    say(f"case refine edge cases: m {m} n {n}")
    K = d.gram(Jt, n, lam, passes=3)
    b = W.random_direction(m, 3)
    # sweeps = 0 is dngd_cholesky_solve, bit for bit
    Ka, Kb = K.clone(), K.clone()
    Ba = torch.tensor(b, device="cuda")
    Bb = Ba.clone()
    assert d.cholesky_solve(Ka, Ba) == 0
    info, res = d.cholesky_solve_refine(Kb, Bb, Jt, n, lam, 0)
    assert info == 0 and res.shape == (1, 0)
    assert torch.equal(Ka, Kb) and torch.equal(Ba, Bb)
    # an already factored K gives the same refined solution as factoring here
    B1 = torch.tensor(b, device="cuda")
    B2 = B1.clone()
    Kc = K.clone()
    assert d.cholesky_solve_refine(Kc, B1, Jt, n, lam, 3)[0] == 0
    assert d.cholesky_solve_refine(Kc, B2, Jt, n, lam, 3, factored=True)[0] == 0
    assert torch.equal(B1, B2)
    # a zero right-hand side stays zero with zero reported residuals
    Bz = torch.zeros(2, m, dtype=torch.float64, device="cuda")
    Bz[1] = torch.tensor(b, device="cuda")
    info, res = d.cholesky_solve_refine(Kc, Bz, Jt, n, lam, 3, factored=True)
    assert info == 0 and torch.count_nonzero(Bz[0]) == 0 and np.all(res[0] == 0.0)
    assert torch.equal(Bz[1], B2)
    # not positive definite: a negative diagonal entry at column 7
    Kn = K.clone()
    Kn[6, 6] = -1.0
    info, res = d.cholesky_solve_refine(Kn, torch.tensor(b, device="cuda"), Jt, n, lam, 2)
    assert info == 7 and res is None


def test_refined_solve_composes_the_mixed_step_at_full_size():
    """At the 5-D Poisson workload (m = 5000, n = 133,377): residual and
    FP32 J, the 3-pass bf16 Gram and the refined solve with 2 sweeps give the
    dual solution of dngd_step (same Gram passes and sweeps, no look-ahead)
    bit for bit, since they run the same kernels in the same order."""
    d = D()
    p = W.config(1)
    th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
    say("case refine composed vs step: m", p.m, "n", p.n_params)
    prob = d.Problem.from_workload(p)
    lam = 1e-5
    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    o = d.step_opts(precision=d.MIXED, ga=False, gram_passes=3, ir_sweeps=2, no_lookahead=True,
                    alpha_out=alpha)
    _, st = prob.step(th, lam, o)
    r, J = prob.residual_jacobian(th, d.F32)
    K = d.gram(J, prob.n, lam, passes=3)
    x = r.clone()
    info, res = d.cholesky_solve_refine(K, x, J, prob.n, lam, 2)
    say(f"  step IR residuals {list(st.ir_residual)[:2]}, refined solve {res.tolist()}")
    assert info == 0
    assert torch.equal(x, alpha)
    for k in range(2):  # the same per-sweep residuals, ||s_k|| / ||r||
        assert abs(res[0, k] - st.ir_residual[k]) <= 1e-12 * st.ir_residual[k]
    prob.close()


def test_refined_solve_degenerate_sizes():
    """No right-hand sides (factor only, nothing else written) and a single
    residual (m = 1: K = ||J_1||^2 + lam, x = b / K) with FP32 and FP64 J."""
    d = D()
    p, th, Jt, Jd, n, lam, kappa = setup(torch.float32, 1e-3, seed=6)
    m = Jd.shape[0]
    say("case refine degenerate sizes: m", m, "n", n)
    K = d.gram(Jt, n, lam, passes=3)
    K0 = K.clone()
    info, res = d.cholesky_solve_refine(K, torch.empty(0, m, dtype=torch.float64, device="cuda"),
                                        Jt, n, lam, 2)
    assert info == 0 and res.shape == (0, 2)
    Kf = K0.clone()
    assert d.cholesky_solve(Kf, torch.empty(0, m, dtype=torch.float64, device="cuda")) == 0
    assert torch.equal(torch.tril(K), torch.tril(Kf))  # the same factor, lower triangle
    for dt in (torch.float32, torch.float64):
        J1 = Jt[:1].to(dt).contiguous()
        k11 = float((J1[0, :n].double() ** 2).sum()) + lam
        K1 = d.gram(J1, n, lam, passes=3 if dt == torch.float32 else 1)
        b = torch.tensor([0.7], dtype=torch.float64, device="cuda")
        info, res = d.cholesky_solve_refine(K1, b, J1, n, lam, 3)
        say(f"  m = 1 ({dt}): x {float(b[0]):.17g} against {0.7 / k11:.17g}, residuals {res.tolist()}")
        assert info == 0
        assert abs(float(b[0]) - 0.7 / k11) <= 1e-14 * abs(0.7 / k11)
