#!/usr/bin/env python3
"""D-NGD step benchmark on one MI355X.

Workload: the 5-D Poisson problem -lap u = f on [0,1]^5 with
u* = sum_i sin(pi x_i / 2), tanh MLP 5-256-256-256-1 (133,377 parameters),
4,000 interior + 1,000 boundary uniform points (m = 5,000), Glorot init,
lambda = min(L(theta_0), 1e-5). Inputs are seeded synthetic data built by
``workloads`` and are resident in HBM before timing starts.

A step is one call of the dense dual solver with geodesic acceleration
(dngd_step): residual and Jacobian, Gram, Cholesky, solves with refinement,
velocity, f_vv, acceleration and the acceptance rule. ``value`` is mixed
precision steps/s (FP32 J, BF16-MFMA Gram, FP64 Cholesky + 2 refinement
sweeps); the plain FP64 path is timed on the same GPU and reported beside it,
as are the 31-point line search and the resulting optimiser iterations/s.

Prints one JSON line. ``--gpus N`` with N > 1 is refused: the library runs the
step on one GPU (there is no multi-GPU path).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bf16
MFMA_F64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--gram-passes", type=int, default=0)
    ap.add_argument("--ir-sweeps", type=int, default=2)
    ap.add_argument("--only-mixed", action="store_true", help="profiling: mixed steps only")
    ap.add_argument("--only-plain", action="store_true", help="profiling: plain steps only")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="profiling: 3 device copies of 1 GiB (calibrates the HBM byte counters)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-stream run")
    ap.add_argument("--serving-jobs", type=int, default=8,
                    help="jobs of the serving stream (its first N; the stream has 64)")
    ap.add_argument("--serving-steps", type=int, default=200,
                    help="iterations per serving job (the stream's jobs ask for 200)")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-budget-gb", type=float, default=0.0,
                    help="serving memory budget in GB (default: 80%% of free device memory)")
    ap.add_argument("--serving-lookahead", action="store_true",
                    help="serving jobs factor with the look-ahead (default off)")
    ap.add_argument("--serving-only", action="store_true",
                    help="instead: only the serving stream, one JSON line")
    ap.add_argument("--pcg", action="store_true",
                    help="instead: one Nystrom-PCG step on the 5-D Poisson MLP 5-2048x4-1, m=50000")
    ap.add_argument("--pcg-landmarks", type=int, default=2000)
    ap.add_argument("--pcg-maxit", type=int, default=500)
    ap.add_argument("--pcg-tol", type=float, default=1e-6)
    ap.add_argument("--pcg-iters", type=int, default=0,
                    help="with --pcg: also run this many optimiser iterations (PCG steps + line search)")
    ap.add_argument("--pcg-ga", action="store_true",
                    help="with --pcg: geodesic acceleration (second PCG solve for f_vv)")
    ap.add_argument("--pcg-kvp", choices=["f64", "bf16"], default="f64",
                    help="with --pcg: kernel-vector products in FP64 or with bf16 GEMM operands "
                         "(FP32 accumulation, FP64 true residuals)")
    ap.add_argument("--factor-compare", action="store_true",
                    help="instead: time the dense Cholesky beside the vendor library's dpotrf")
    ap.add_argument("--kvp", type=int, default=-1, metavar="CFG",
                    help="instead: time the kernel-vector product (FP64 and bf16) on workload CFG")
    ap.add_argument("--pcg-reuse", type=int, default=0,
                    help="with --pcg-iters: reuse the Nystrom factors for up to R further steps")
    ap.add_argument("--config0", action="store_true",
                    help="instead: the plain FP64 dense step with GA on the 2-D Poisson workload "
                         "(MLP 2-32-32-1, m = 500, lambda = 1e-8)")
    ap.add_argument("--kovasznay", action="store_true",
                    help="instead: the dense step on the Kovasznay flow (vector-valued residuals, "
                         "[2,50x4,3], 400 + 400 points, m = 2400): mixed and plain, GA")
    ap.add_argument("--landmark-study", type=str, default="", metavar="L1,L2,...",
                    help="instead: --pcg runs with --pcg-iters optimiser iterations (default 6) "
                         "for each landmark count; PCG iterations per step over training")
    ap.add_argument("--structured", type=int, default=-1, metavar="CFG",
                    help="instead: the dense step on the structured FP64 kernel (no J) against "
                         "the mixed J step, on workload CFG (1: 5-D Poisson, 2: heat)")
    ap.add_argument("--regime-map", action="store_true",
                    help="instead: primal vs dual dense step times over m x n shapes "
                         "(2-D Poisson, hidden width 50, FP64, GA)")
    return ap.parse_args()


def copy_calibration(torch):
    x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": x.numel() * 8, "launches": 3}))


def timed_steps(prob, th, lam, opts, steps, warmup, torch):
    for _ in range(warmup):
        prob.step(th, lam, opts)
    torch.cuda.synchronize()
    walls, stats = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        s0 = time.perf_counter()
        dth, st = prob.step(th, lam, opts)   # synchronises its stream before returning
        walls.append((time.perf_counter() - s0) * 1e3)
        stats.append(st.as_dict())
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return total, walls, stats, dth


def p99(xs):
    xs = sorted(xs)
    k = max(0, min(len(xs) - 1, int(round(0.99 * (len(xs) - 1)))))
    return xs[k]


def cpu_baseline(seed_theta, lam):
    """The oracle (unchanged) timed on the host cores: one whole dense step
    with geodesic acceleration on the benchmark workload itself (m = 5000,
    n = 133,377, same parameters and damping), nothing scaled or extrapolated.
    The phases are timed separately and reported beside the total."""
    from threadpoolctl import threadpool_info
    import workloads as W
    from oracle import network as N, step as S
    p = W.config(1)
    th = seed_theta
    t = {}

    def clock(name, fn):
        t0 = time.perf_counter()
        out = fn()
        t[name] = time.perf_counter() - t0
        return out

    r = clock("residual", lambda: N.residual(p, th))
    J = clock("jacobian", lambda: N.jacobian(p, th))
    K = clock("gram", lambda: S.gram(J))
    ch = clock("cholesky", lambda: S.cholesky(K, lam))
    alpha = clock("solve_v", lambda: S.solve(ch, r))
    v = clock("jt_v", lambda: -(J.T @ alpha))
    f = clock("fvv", lambda: N.fvv(p, th, v))
    beta = clock("solve_a", lambda: S.solve(ch, f))
    clock("jt_a", lambda: -(J.T @ beta))
    total = sum(t.values())
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": 1.0 / total, "unit": "steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"one whole oracle dense step with GA (r, J, K, Cholesky, v, f_vv, a) on "
                      f"the benchmark workload (m={p.m}, n=133377), measured, not scaled: "
                      f"{total:.1f} s; phases { {k: round(x, 3) for k, x in t.items()} } s"}


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "gram_bf16_kernel_poisson5d_m5000.traffic.txt")


def serving_run(n_jobs, steps, slots, torch, budget_gb=0.0, lookahead=False):
    """The serving stream (Poisson arrivals at 4 jobs/s, uneven m and widths)
    with ``steps`` iterations per job, admitted by footprint into 80% of the
    free device memory (or ``budget_gb`` GB)."""
    import workloads as W
    from paper_2505_21404_amd import serving as SV
    specs = SV.specs_from_workloads(W.serving_jobs(n_jobs=n_jobs, rate=4.0, steps=steps))
    free, _ = torch.cuda.mem_get_info()
    budget = int(budget_gb * 2 ** 30) if budget_gb > 0 else int(0.8 * free)
    fp, rj = SV.gpu_executor(lookahead=lookahead)
    t0 = time.perf_counter()

    def run_job(spec, res):  # the executor, plus a progress line per finished job
        rj(spec, res)
        progress(f"serving job {spec.job_id} done at {time.perf_counter() - t0:.1f} s "
                 f"(m {spec.problem.m}, {len(res.step_ms)} steps, median "
                 f"{statistics.median(res.step_ms):.1f} ms)")

    srv = SV.Server(budget_bytes=budget, max_slots=slots, run_job=run_job, footprint=fp)
    rep = srv.run(specs, realtime=True)
    out = {k: v for k, v in rep.items() if k not in ("results", "errors")}
    out["errors"] = len(rep["errors"])
    out["jobs_requested"] = n_jobs
    out["steps_per_job"] = steps
    out["slots"] = slots
    out["budget_bytes"] = srv.budget
    out["lookahead"] = lookahead
    return out


def progress(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def structured_run(cfg, torch, steps=3):
    """Dense dual step with GA on workload `cfg`: the structured FP64 kernel
    (per-layer products of activations and adjoints, J never formed) against
    the mixed step on the materialised FP32 J; median step times, phases and
    the relative difference of the two steps."""
    import workloads as W
    from paper_2505_21404_amd import dngd as D
    p = W.config(cfg)
    th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
    prob = D.Problem.from_workload(p)
    r = prob.residual(th)
    lam = min(0.5 * float((r * r).sum()), W.LAMBDA_CAP[cfg])
    out = {"metric": "dense D-NGD step, structured FP64 kernel vs mixed J", "unit": "ms",
           "n_gpus": 1, "data": "synthetic",
           "config": {"workload": W.CONFIG_NAMES[cfg], "m": prob.m, "n": prob.n, "lambda": lam}}
    dths = {}
    for name, o in (("structured", D.step_opts(solver=D.STRUCTURED, ga=True)),
                    ("mixed", D.step_opts(precision=D.MIXED, ga=True))):
        prob.step(th, lam, o)
        ws, sts = [], []
        for _ in range(steps):
            t0 = time.perf_counter()
            dth, st = prob.step(th, lam, o)
            ws.append((time.perf_counter() - t0) * 1e3)
            sts.append(st.as_dict())
        dths[name] = dth.clone()
        out[name] = {"ms_per_step": statistics.median(ws),
                     "phase_ms": {k: statistics.median(x[k] for x in sts) for k in (
                         "ms_residual_jacobian", "ms_gram", "ms_gram_kernel", "ms_factor",
                         "ms_solve_v", "ms_fvv", "ms_solve_a")},
                     "footprint_bytes": prob.footprint(o) if hasattr(prob, "footprint") else None}
        progress(f"structured run {name}: {out[name]['ms_per_step']:.1f} ms/step")
        torch.cuda.empty_cache()
    out["rel_diff_structured_vs_mixed"] = float(
        ((dths["structured"] - dths["mixed"]).norm() / dths["structured"].norm()).item())
    prob.close()
    return out


def regime_map(torch, ms=(300, 1300, 3300, 6300), ks=(0, 1, 2, 4), steps=3):
    """Primal (n x n) against dual (m x m) dense FP64 steps with GA on 2-D
    Poisson networks 2-50-...-50-1 with k + 1 hidden layers (n = 201 + 2550 k)
    and m residuals (4:1 interior to boundary); median ms over `steps` steps
    after one warmup, and the solver the cost rule (primal iff n < m) picks."""
    import workloads as W
    from paper_2505_21404_amd import dngd as D
    rows = []
    for k in ks:
        widths = [2] + [50] * (k + 1) + [1]
        for m in ms:
            p = W.config(0, scale=dict(widths=widths, n_int=4 * m // 5, n_bdy=m - 4 * m // 5))
            th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
            prob = D.Problem.from_workload(p)
            t = {}
            for name, solver in (("primal", D.PRIMAL), ("dual", D.DENSE)):
                o = D.step_opts(precision=D.PLAIN, solver=solver, ga=True)
                prob.step(th, 1e-4, o)
                ws = []
                for _ in range(steps):
                    t0 = time.perf_counter()
                    prob.step(th, 1e-4, o)
                    ws.append((time.perf_counter() - t0) * 1e3)
                t[name] = statistics.median(ws)
            auto = "primal" if prob.n < prob.m else "dual"
            rows.append({"m": prob.m, "n": prob.n, "ms_primal": t["primal"], "ms_dual": t["dual"],
                         "faster": min(t, key=t.get), "auto": auto})
            progress(f"regime m={prob.m} n={prob.n}: primal {t['primal']:.2f} ms, dual {t['dual']:.2f} ms")
            prob.close()
    agree = sum(r["faster"] == r["auto"] for r in rows)
    return {"metric": "dense D-NGD step time, primal vs dual (FP64, GA)", "unit": "ms",
            "n_gpus": 1, "data": "synthetic", "rows": rows,
            "auto_picks_faster": f"{agree}/{len(rows)}"}


def kovasznay_run(torch, steps=20, warmup=3):
    """Dense D-NGD step with GA on the Kovasznay flow (steady Navier-Stokes,
    vector-valued residual classes): [2, 50 x 4, 3] tanh MLP, 400 interior and
    400 boundary points (m = 2400, n = 7953), lambda = min(L, 1e-5)."""
    import workloads as W
    from paper_2505_21404_amd import dngd as D
    p = W.kovasznay()
    th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
    prob = D.Problem.from_workload(p)
    r = prob.residual(th)
    lam = min(0.5 * float((r * r).sum()), 1e-5)
    out = {"metric": "dense D-NGD step, Kovasznay flow (vector-valued residuals)",
           "unit": "steps/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": p.name, "m": prob.m, "n": prob.n, "lambda": lam}}
    for name, o in (("mixed", D.step_opts(precision=D.MIXED, ga=True)),
                    ("plain", D.step_opts(precision=D.PLAIN, ga=True)),
                    ("primal_plain", D.step_opts(precision=D.PLAIN, solver=D.PRIMAL, ga=True))):
        tot, walls, stats, _ = timed_steps(prob, th, lam, o, steps, warmup, torch)
        out[name] = {"steps_per_s": steps / tot, "p50_step_ms": statistics.median(walls),
                     "gram_passes": stats[-1]["gram_passes_used"],
                     "phase_ms_median": {k: statistics.median(x[k] for x in stats) for k in (
                         "ms_residual_jacobian", "ms_gram", "ms_factor", "ms_solve_v", "ms_fvv",
                         "ms_solve_a")}}
        progress(f"kovasznay {name}: {out[name]['p50_step_ms']:.2f} ms/step")
    prob.close()
    return out


def pcg_run(a, torch):
    """One matrix-free Nystrom-PCG step (GA with --pcg-ga) on the large 5-D Poisson
    workload: n = 12.6M parameters, m = 50,000 residuals (45,000 interior,
    5,000 boundary), FP64 kernel-vector products."""
    import numpy as np
    import workloads as W
    from paper_2505_21404_amd import dngd as D
    p = W.config(3)
    th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
    prob = D.Problem.from_workload(p)
    r = prob.residual(th)
    L0 = 0.5 * float((r * r).sum())
    lam = min(L0, W.LAMBDA_CAP[3])
    I = torch.tensor(W.landmarks(p.m, a.pcg_landmarks, 0), device="cuda")
    alpha = torch.empty(prob.m, dtype=torch.float64, device="cuda")
    kvp_dtype = D.BF16 if a.pcg_kvp == "bf16" else D.F64
    opts = D.step_opts(solver=D.PCG, ga=a.pcg_ga, landmarks=I, pcg_tol=a.pcg_tol,
                       pcg_maxit=a.pcg_maxit, alpha_out=alpha, pcg_kvp=kvp_dtype)
    progress(f"PCG step: n={prob.n} m={prob.m} landmarks={a.pcg_landmarks}")
    t0 = time.perf_counter()
    dth, st = prob.step(th, lam, opts)
    wall = time.perf_counter() - t0
    # true dual residual with one more FP64 matrix-free product, timed alone
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ka = prob.jvp(th, prob.vjp(th, alpha))
    torch.cuda.synchronize()
    kvp_ms = (time.perf_counter() - t1) * 1e3
    true_res = float(((ka + lam * alpha - r).norm() / r.norm()).item())
    its = max(st.pcg_iterations, 1)
    out = {
        "metric": "D-NGD PCG step (matrix-free, Nystrom preconditioner)", "unit": "s",
        "value": wall, "higher_is_better": False, "n_gpus": 1,
        "config": {"workload": "poisson5d_mlp5-2048x4-1_m50000_pcg" + ("_ga" if a.pcg_ga else ""),
                   "n": prob.n, "m": prob.m,
                   "landmarks": a.pcg_landmarks, "tol": a.pcg_tol, "maxit": a.pcg_maxit,
                   "lambda": lam, "kvp": a.pcg_kvp},
        "pcg_kvp_f64": st.pcg_kvp_f64, "pcg_replacements": st.pcg_replacements,
        "pcg_escalated": st.pcg_escalated,
        "pcg_iterations": st.pcg_iterations, "pcg_converged": bool(st.pcg_converged),
        "pcg_rel_residual": st.pcg_rel_residual, "true_rel_residual": true_res,
        "ms_forward": st.ms_residual_jacobian, "ms_nystrom_build": st.ms_factor,
        "ms_pcg_and_recovery": st.ms_solve_v, "ms_per_pcg_iteration": st.ms_solve_v / its,
        "ms_kvp_alone_incl_forward": kvp_ms, "dtheta_norm": float(dth.norm()),
    }
    if a.pcg_ga:
        out.update({"ms_fvv": st.ms_fvv, "ms_ga_pcg_and_recovery": st.ms_solve_a,
                    "pcg_iterations_ga": st.pcg_iterations_ga, "ga_accepted": st.ga_accepted,
                    "vnorm": st.vnorm, "anorm": st.anorm})
    if a.pcg_iters > 0:
        # optimiser iterations: fresh landmarks per step (seed + 3 + k), damping rule
        etas = [2.0 ** -k for k in range(31)]
        hist = []
        for k in range(a.pcg_iters):
            Ik = torch.tensor(W.landmarks(p.m, a.pcg_landmarks, 0, step=k), device="cuda")
            ok = D.step_opts(solver=D.PCG, ga=a.pcg_ga, landmarks=Ik, pcg_tol=a.pcg_tol,
                             pcg_maxit=a.pcg_maxit, nystrom_reuse=a.pcg_reuse,
                             pcg_kvp=kvp_dtype)
            t0 = time.perf_counter()
            it = prob.iterate(th, etas, lam_cap=W.LAMBDA_CAP[3], opts=ok)
            hist.append({"loss": it.loss, "lam": it.lam, "eta": it.eta,
                         "pcg_iterations": it.step.pcg_iterations,
                         "pcg_iterations_ga": it.step.pcg_iterations_ga,
                         "ga_accepted": it.step.ga_accepted,
                         "pcg_rel_residual": it.step.pcg_rel_residual,
                         "pcg_kvp_f64": it.step.pcg_kvp_f64,
                         "pcg_escalated": it.step.pcg_escalated,
                         "nystrom_reused": it.step.nystrom_reused,
                         "s_nystrom_build": it.step.ms_factor / 1e3,
                         "s_step": it.step.ms_total / 1e3, "s_line_search": it.ms_line_search / 1e3,
                         "s_iteration": time.perf_counter() - t0})
            progress(f"PCG iteration {k}: loss {it.loss:.4g} pcg its {it.step.pcg_iterations}")
        out["iterations"] = hist
    prob.close()
    return out


def kvp_run(cfg, a, torch):
    """The kernel-vector product w = J (J^T p) + lam p (Definition 3.6) on
    workload cfg, FP64 and bf16 products: wall ms per dngd_kvp call (forward
    pass included; bf16 also includes the per-step bf16/FP32 copies) and the
    forward pass alone, medians over --steps calls after --warmup."""
    import numpy as np
    import workloads as W
    from paper_2505_21404_amd import dngd as D
    p = W.config(cfg)
    th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
    prob = D.Problem.from_workload(p)
    pv = torch.tensor(W.random_direction(p.m, 1), device="cuda")
    lam = W.LAMBDA_CAP[cfg]

    def timed(fn):
        ts = []
        for k in range(a.warmup + a.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            if k >= a.warmup:
                ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts)), out

    progress(f"kvp: workload {cfg}, n={prob.n} m={prob.m}")
    t_fwd, r = timed(lambda: prob.residual(th))
    t64, w64 = timed(lambda: prob.kvp(th, lam, pv, D.F64))
    progress("kvp: FP64 products timed")
    t16, w16 = timed(lambda: prob.kvp(th, lam, pv, D.BF16))
    progress("kvp: bf16 products timed")
    err = float(((w16 - w64).norm() / w64.norm()).item())
    prob.close()
    return {"metric": "kernel-vector product ms (dngd_kvp, forward pass included)",
            "unit": "ms", "value": t16, "higher_is_better": False, "n_gpus": 1,
            "config": {"workload": p.name, "n": int(prob.n), "m": int(prob.m), "lambda": lam},
            "ms_forward_only": t_fwd, "ms_kvp_f64": t64, "ms_kvp_bf16": t16,
            "ms_product_f64": t64 - t_fwd, "ms_product_bf16_incl_copies": t16 - t_fwd,
            "bf16_vs_f64_rel_err": err}


def factor_compare_run(a, torch):
    """The dense factorisation K = L L^T (the Cholesky step of the dense dual
    solve) through dngd_cholesky_solve (factor only, no right-hand side),
    beside the vendor library's dpotrf (rocSOLVER, loaded with ctypes for
    this comparison only; the step never calls it), on the same SPD matrices
    (diagonal m, off-diagonal 1 / (1 + i + j)): median ms over --steps after
    --warmup. K is symmetric, so row-major lower and column-major lower hold
    the same factor."""
    import ctypes as C
    import numpy as np
    from paper_2505_21404_amd import dngd as D
    roc = None
    try:
        rb = C.CDLL("librocblas.so")
        rs = C.CDLL("librocsolver.so")
        handle = C.c_void_p()
        if rb.rocblas_create_handle(C.byref(handle)) == 0:
            roc = (rb, rs, handle)
    except OSError:
        pass
    out = {"metric": "dense Cholesky factorisation ms", "unit": "ms", "higher_is_better": False,
           "n_gpus": 1, "sizes": {}}
    for m in (2000, 5000, 8192):
        i = torch.arange(m, device="cuda", dtype=torch.float64)
        K0 = 1.0 / (1.0 + i[:, None] + i[None, :])
        K0.diagonal().fill_(float(m))
        K = torch.empty_like(K0)
        B = torch.empty((0, m), dtype=torch.float64, device="cuda")
        ts, tr = [], []
        info = C.c_int32()
        dinfo = torch.zeros(1, dtype=torch.int32, device="cuda")
        for k in range(a.warmup + a.steps):
            K.copy_(K0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            assert D.cholesky_solve(K, B) == 0
            torch.cuda.synchronize()
            if k >= a.warmup:
                ts.append((time.perf_counter() - t0) * 1e3)
            if roc is not None:
                rb, rs, handle = roc
                K.copy_(K0)
                rb.rocblas_set_stream(handle, C.c_void_p(torch.cuda.current_stream().cuda_stream))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = rs.rocsolver_dpotrf(handle, 122, m, C.c_void_p(K.data_ptr()), m,
                                         C.c_void_p(dinfo.data_ptr()))
                torch.cuda.synchronize()
                if st != 0 or int(dinfo.item()) != 0:
                    raise RuntimeError(f"rocsolver_dpotrf status {st}, info {int(dinfo.item())}")
                if k >= a.warmup:
                    tr.append((time.perf_counter() - t0) * 1e3)
        out["sizes"][m] = {"dngd_ms": float(np.median(ts)),
                           "rocsolver_dpotrf_ms": float(np.median(tr)) if tr else None}
        progress(f"factor m={m}: {out['sizes'][m]}")
    out["value"] = out["sizes"][5000]["dngd_ms"]
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: --gpus {a.gpus} refused: libdngd runs the D-NGD step on one GPU "
              "only (no multi-GPU path).", file=sys.stderr)
        return 2
    import numpy as np
    import torch
    if a.copy_calibration:
        copy_calibration(torch)
        return 0
    if a.landmark_study:
        rows = []
        for ell in (int(x) for x in a.landmark_study.split(",")):
            a.pcg_landmarks = ell
            a.pcg_iters = a.pcg_iters or 6
            out = pcg_run(a, torch)
            rows.append({"landmarks": ell, "first_step_s": out["value"],
                         "ms_nystrom_build": out["ms_nystrom_build"],
                         "ms_per_pcg_iteration": out["ms_per_pcg_iteration"],
                         "iterations": out["iterations"]})
        print(json.dumps({"metric": "PCG iterations per D-NGD step vs landmark count",
                          "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": "poisson5d_mlp5-2048x4-1_m50000_pcg",
                                     "tol": a.pcg_tol, "iterations": a.pcg_iters},
                          "rows": rows}), flush=True)
        return 0
    if a.factor_compare:
        print(json.dumps(factor_compare_run(a, torch)), flush=True)
        return
    if a.kvp >= 0:
        print(json.dumps(kvp_run(a.kvp, a, torch)), flush=True)
        return
    if a.pcg:
        print(json.dumps(pcg_run(a, torch)), flush=True)
        return 0
    if a.kovasznay:
        print(json.dumps(kovasznay_run(torch)), flush=True)
        return 0
    if a.config0:
        import workloads as W
        from paper_2505_21404_amd import dngd as D
        p = W.config(0)
        th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
        prob = D.Problem.from_workload(p)
        o = D.step_opts(precision=D.PLAIN, ga=True)
        tot, walls, stats, _ = timed_steps(prob, th, W.LAMBDA[0], o, a.steps, a.warmup, torch)
        etas = [2.0 ** -k for k in range(31)]
        ls = []
        for _ in range(5):
            t0 = time.perf_counter()
            prob.iterate(th.clone(), etas, fixed_lambda=W.LAMBDA[0], opts=o)
            ls.append((time.perf_counter() - t0) * 1e3)
        print(json.dumps({"metric": "D-NGD plain FP64 steps/s, 2-D Poisson", "unit": "steps/s",
                          "value": a.steps / tot, "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": W.CONFIG_NAMES[0], "m": prob.m, "n": prob.n,
                                     "lambda": W.LAMBDA[0]},
                          "p50_step_ms": statistics.median(walls), "p99_step_ms": p99(walls),
                          "optimizer_iteration_ms": statistics.median(ls),
                          "phase_ms_median": {k: statistics.median(x[k] for x in stats) for k in (
                              "ms_residual_jacobian", "ms_gram", "ms_factor", "ms_solve_v",
                              "ms_fvv", "ms_solve_a")}}), flush=True)
        prob.close()
        return 0
    if a.regime_map:
        print(json.dumps(regime_map(torch)), flush=True)
        return 0
    if a.structured >= 0:
        print(json.dumps(structured_run(a.structured, torch)), flush=True)
        return 0
    if a.serving_only:
        rep = serving_run(a.serving_jobs, a.serving_steps, a.serving_slots, torch,
                          a.serving_budget_gb, a.serving_lookahead)
        print(json.dumps({"metric": "serving stream: steps/s, p50/p99 step ms",
                          "value": rep["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
                          "higher_is_better": True, "data": "synthetic",
                          "config": {"workload": "serving_stream_poisson_heat",
                                     "jobs": a.serving_jobs, "steps_per_job": a.serving_steps,
                                     "slots": a.serving_slots}, "serving": rep}), flush=True)
        return 0
    import workloads as W
    from paper_2505_21404_amd import dngd as D

    p = W.config(1)
    th0 = W.glorot_theta(p.widths, 0)
    prob = D.Problem.from_workload(p)
    th = torch.tensor(th0, device="cuda")
    r0 = prob.residual(th)
    L0 = 0.5 * float((r0 * r0).sum())
    lam = min(L0, W.LAMBDA_CAP[1])

    if a.only_plain:
        plain = D.step_opts(precision=D.PLAIN, ga=True)
        tot, _, _, _ = timed_steps(prob, th, lam, plain, a.steps, a.warmup, torch)
        print(json.dumps({"steps": a.steps, "ms_per_step": tot * 1e3 / a.steps}))
        return 0
    mixed = D.step_opts(precision=D.MIXED, ga=True, ir_sweeps=a.ir_sweeps,
                        gram_passes=a.gram_passes)
    tot, walls, stats, dth_mixed = timed_steps(prob, th, lam, mixed, a.steps, a.warmup, torch)
    progress(f"mixed steps done: {tot * 1e3 / a.steps:.2f} ms/step")
    if a.only_mixed:
        print(json.dumps({"steps": a.steps, "ms_per_step": tot * 1e3 / a.steps}))
        return 0

    m, n = prob.m, prob.n
    gram_flops = float(m) * (m + 1) * n       # algorithmic: lower-triangle syrk
    gk = [s["ms_gram_kernel"] for s in stats]
    gk_avg = sum(gk) / len(gk)
    achieved = gram_flops / (gk_avg * 1e-3) / 1e12

    out = {
        "metric": "D-NGD steps/s (mixed vs FP64 plain, same GPU); Gram TFLOP/s; p99 step ms",
        "value": a.steps / tot,
        "unit": "steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": tot * 1e3 / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-mfma/f32-J/f64-solve",
        "data": "synthetic (seeded uniform collocation points, Glorot init)",
        "config": {"workload": "poisson5d_mlp5-256x3-1_m5000_dense_ga", "m": m, "n": n,
                   "lambda": lam, "gram_passes": stats[-1]["gram_passes_used"],
                   "ir_sweeps": a.ir_sweeps},
        "p50_step_ms": statistics.median(walls),
        "p99_step_ms": p99(walls),
        "gram_tflops": achieved,
        "phase_ms_median": {k: statistics.median(s[k] for s in stats) for k in (
            "ms_residual_jacobian", "ms_gram", "ms_gram_kernel", "ms_factor", "ms_solve_v",
            "ms_fvv", "ms_solve_a")},
        "ir_residual": stats[-1]["ir_residual"][:a.ir_sweeps],
        "ga_accepted": stats[-1]["ga_accepted"],
        "roofline": {"bound": "mfma", "kernel": "gram_bf16_kernel", "achieved": achieved,
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_BF16_PEAK_TFLOPS, "traffic": None,
                     "flops_per_launch": gram_flops, "avg_launch_ms": gk_avg},
    }
    from paper_2505_21404_amd.profiling import read_traffic
    tr = read_traffic(TRAFFIC_RECORD, ROOT)
    if tr is not None and int(tr.get("gram_passes", "-1")) == stats[-1]["gram_passes_used"]:
        out["roofline"]["traffic"] = float(tr["traffic_bytes_per_dispatch"])
        out["roofline"]["traffic_unit"] = ("bytes per launch (FETCH_SIZE + WRITE_SIZE, "
                                           "copy-calibrated; L2 misses, memory-side cache "
                                           "hits included)")
    # what the contraction must move: J read once, the lower triangle of K written
    out["roofline"]["algorithmic_bytes"] = float(4 * m * n + 8 * m * (m + 1) // 2)

    if not a.no_plain:
        plain = D.step_opts(precision=D.PLAIN, ga=True)
        ptot, pwalls, pstats, dth_plain = timed_steps(prob, th, lam, plain, a.plain_steps, 1,
                                                      torch)
        pg = statistics.median(s["ms_gram_kernel"] for s in pstats)
        out["plain"] = {"steps_per_s": a.plain_steps / ptot, "p50_step_ms": statistics.median(pwalls),
                        "p99_step_ms": p99(pwalls),
                        "gram_tflops": gram_flops / (pg * 1e-3) / 1e12,
                        "gram_frac_of_f64_peak": gram_flops / (pg * 1e-3) / 1e12 / MFMA_F64_PEAK_TFLOPS,
                        "phase_ms_median": {k: statistics.median(s[k] for s in pstats) for k in (
                            "ms_residual_jacobian", "ms_gram", "ms_factor", "ms_solve_v",
                            "ms_fvv", "ms_solve_a")}}
        out["speedup_mixed_vs_plain"] = out["value"] / out["plain"]["steps_per_s"]
        progress("plain steps done")
        dm, dp = dth_mixed.cpu().numpy(), dth_plain.cpu().numpy()
        out["mixed_vs_plain_rel_err"] = float(np.linalg.norm(dm - dp) / np.linalg.norm(dp))

    # line search (31 points, D-NGD workflow) and full optimiser iterations/s
    etas = [2.0 ** -k for k in range(31)]
    ls = []
    for _ in range(3):
        t0 = time.perf_counter()
        prob.losses(th, dth_mixed, etas)
        ls.append((time.perf_counter() - t0) * 1e3)
    out["line_search_ms"] = statistics.median(ls)
    out["optimizer_iters_per_s"] = 1e3 / (out["ms_per_step"] + out["line_search_ms"])

    # parity against the stored oracle step of this workload (tests/golden)
    gold = os.path.join(ROOT, "tests", "golden", "config1_step.npz")
    if os.path.exists(gold):
        g = np.load(gold)
        if abs(float(g["lam"]) - lam) <= 1e-12 * lam:
            ref = g["dtheta"]
            dm = dth_mixed.cpu().numpy()
            out["mixed_vs_oracle_rel_err"] = float(np.linalg.norm(dm - ref) / np.linalg.norm(ref))
            if "plain" in out:
                dp = dth_plain.cpu().numpy()
                out["plain_vs_oracle_rel_err"] = float(np.linalg.norm(dp - ref)
                                                       / np.linalg.norm(ref))

    if not a.no_serving:
        progress("serving stream ...")
        out["serving"] = serving_run(a.serving_jobs, a.serving_steps, a.serving_slots, torch,
                                     a.serving_budget_gb, a.serving_lookahead)
        progress("serving done")

    if not a.no_cpu:
        progress("CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(th0, lam)
    print(json.dumps(out), flush=True)
    prob.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
