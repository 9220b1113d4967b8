"""The heat workload at full size (2+1-D heat, MLP 3-1024x4-1, n = 3,153,921,
m = 8192 with 6144 interior, 1024 boundary, 1024 initial points; FP32 J of
103 GB materialised), mixed-precision step with GA.

The step is compared with the oracle's step stored in
tests/golden/config2_step.npz (written by tests/golden/make_golden.py, which
forms K from column blocks of the FP64 J on the host): dtheta within the mixed
bar 1e-4, the GA decision, alpha and f_vv. Also checked: r and f_vv on sampled
residuals, each from its own point, and properties that hold at any size (the
dual solution satisfies (J J^T + lambda I) alpha = r when the products are
taken in FP64 by the matrix-free kernel-vector product, Definition 3.6)."""
import os
import time

import numpy as np
import pytest

import workloads as W
from oracle import network as N

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config2_step.npz")


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sample_rows(p, k, seed=5):
    rng = np.random.default_rng(seed)
    parts = [rng.choice(p.n_int, k, replace=False),
             p.n_int + rng.choice(p.n_bdy, k, replace=False),
             p.n_int + p.n_bdy + rng.choice(p.n_init, k, replace=False)]
    return np.sort(np.concatenate(parts))


def test_config2_full_size_mixed_step():
    from paper_2505_21404_amd import dngd as D
    p = W.config(2)
    th = W.glorot_theta(p.widths, 0)
    say("case config2 full size: m", p.m, "n", p.n_params)
    prob = D.Problem.from_workload(p)
    thd = torch.tensor(th, device="cuda")
    idx = sample_rows(p, 16)

    r = prob.residual(thd)
    r_np = r.cpu().numpy()
    t0 = time.perf_counter()
    r_o = N.residual_rows(p, th, idx)
    say(f"oracle residual rows: {time.perf_counter() - t0:.1f} s")
    assert rel(r_np[idx], r_o) <= 1e-12
    L0 = 0.5 * float(r_np @ r_np)
    lam = min(L0, W.LAMBDA_CAP[2])

    alpha = torch.empty(p.m, dtype=torch.float64, device="cuda")
    fvv = torch.empty(p.m, dtype=torch.float64, device="cuda")
    opts = D.step_opts(precision=D.MIXED, ga=True, alpha_out=alpha, fvv_out=fvv)
    dth, st = prob.step(thd, lam, opts)
    say(f"mixed step: {st.ms_total:.1f} ms (J {st.ms_residual_jacobian:.1f}, Gram "
        f"{st.ms_gram:.1f}, factor {st.ms_factor:.1f}, v {st.ms_solve_v:.1f}, fvv {st.ms_fvv:.1f},"
        f" a {st.ms_solve_a:.1f}); passes {st.gram_passes_used} attempts {st.gram_attempts}; "
        f"ir {list(st.ir_residual)[:2]}; D {st.max_row_norm2:.4g} lam {lam:.3g}; "
        f"GA accepted {st.ga_accepted}")
    gram_flops = float(p.m) * (p.m + 1) * p.n_params
    say(f"Gram kernel {st.ms_gram_kernel:.1f} ms = {gram_flops / st.ms_gram_kernel / 1e9:.1f} TF/s")

    # dual residual with FP64 matrix-free products
    a = alpha
    u = prob.jvp(thd, prob.vjp(thd, a))
    res = (u + lam * a - r).cpu().numpy()
    dual_res = float(np.linalg.norm(res) / np.linalg.norm(r_np))
    say("dual residual (FP64 products)", dual_res)
    assert dual_res <= 1e-4

    # v = -J^T alpha against the FP64 reverse pass; f_vv at v on sampled rows
    v64 = (-prob.vjp(thd, a)).cpu().numpy()
    dth_v, st_v = prob.step(thd, lam, D.step_opts(precision=D.MIXED, ga=False))
    e_v = rel(dth_v.cpu().numpy(), v64)
    say("v vs -J^T alpha (FP64)", e_v)
    assert e_v <= 1e-5
    t0 = time.perf_counter()
    f_o = N.fvv_rows(p, th, v64, idx)
    say(f"oracle f_vv rows: {time.perf_counter() - t0:.1f} s")
    e_f = rel(fvv.cpu().numpy()[idx], f_o)
    say("f_vv rows vs oracle", e_f)
    assert e_f <= 1e-5
    assert np.all(np.isfinite(dth.cpu().numpy()))

    # against the oracle's step (Theorem 3.2 recovery, dense dual solve)
    g = np.load(GOLD)
    assert abs(lam - float(g["lam"])) <= 1e-14 * lam
    assert rel(r_np, g["r"]) <= 1e-12
    e_dth = rel(dth.cpu().numpy(), g["dtheta32"])
    e_alpha = rel(alpha.cpu().numpy(), g["alpha"])
    e_fvv = rel(fvv.cpu().numpy(), g["fvv"])
    say(f"vs oracle step: dtheta {e_dth:.2e}, alpha {e_alpha:.2e}, f_vv {e_fvv:.2e}, "
        f"|v| {st.vnorm:.6g} (oracle {float(g['vnorm']):.6g}), |a| {st.anorm:.6g} "
        f"(oracle {float(g['anorm']):.6g}), accepted {st.ga_accepted} (oracle "
        f"{int(g['accepted'])})")
    assert st.ga_accepted == int(g["accepted"])
    assert st.ga_early_reject == 0  # accepted: the f_vv solve was refined in full
    assert e_dth <= 1e-4
    # f_vv is quadratic in v: its relative error is about twice v's
    assert e_fvv <= 1e-4
    prob.close()
