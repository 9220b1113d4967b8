"""Serving loop: the scheduler's admission rules on the CPU with a fake
executor, and on the GPU that every job's result is the same alone and in
the mix."""
import threading
import time

import numpy as np
import pytest

import workloads as W
from paper_2505_21404_amd import serving as SV


def _fake(durations):
    live = {"n": 0, "max": 0}
    lock = threading.Lock()

    def run_job(spec, res):
        with lock:
            live["n"] += 1
            live["max"] = max(live["max"], live["n"])
        for _ in range(spec.steps):
            t0 = time.perf_counter()
            time.sleep(durations[spec.job_id])
            res.step_ms.append((time.perf_counter() - t0) * 1e3)
        res.theta = np.array([spec.job_id], dtype=float)
        with lock:
            live["n"] -= 1
    return run_job, live


def _specs(fps, arrivals, steps=2):
    return [SV.JobSpec(j, a, problem=None, theta0=None, steps=steps)
            for j, a in enumerate(arrivals)], {j: f for j, f in enumerate(fps)}


def test_scheduler_respects_slots_and_budget():
    specs, fps = _specs([4, 3, 5, 2, 6, 1], [0.0, 0.0, 0.01, 0.02, 0.02, 0.03])
    run_job, live = _fake({j: 0.02 for j in fps})
    srv = SV.Server(budget_bytes=9, max_slots=2, run_job=run_job,
                    footprint=lambda s: fps[s.job_id])
    rep = srv.run(specs)
    assert rep["jobs"] == 6 and not rep["errors"]
    assert srv.peak_bytes <= 9 and srv.peak_slots <= 2 and live["max"] <= 2
    for t, kind, j, in_use, active in srv.events:
        assert in_use <= 9 and active <= 2
    # first come, first served: admission order = arrival order
    admits = [j for _, kind, j, _, _ in srv.events if kind == "admit"]
    assert admits == sorted(admits, key=lambda j: (specs[j].arrival, j))
    for r in rep["results"].values():
        assert r.admitted >= r.arrival - 1e-9 and r.finished >= r.admitted
        assert len(r.step_ms) == 2
    assert rep["steps"] == 12 and rep["p99_step_ms"] >= rep["p50_step_ms"] > 0


def test_scheduler_queues_on_memory_and_overlaps_when_it_fits():
    # two jobs that together exceed the budget run one after the other ...
    specs, fps = _specs([6, 6], [0.0, 0.0])
    run_job, live = _fake({0: 0.05, 1: 0.05})
    srv = SV.Server(budget_bytes=10, max_slots=4, run_job=run_job,
                    footprint=lambda s: fps[s.job_id])
    rep = srv.run(specs)
    assert live["max"] == 1 and rep["results"][1].admitted >= rep["results"][0].finished - 1e-6
    # ... and overlap when both fit
    specs, fps = _specs([5, 5], [0.0, 0.0])
    run_job, live = _fake({0: 0.05, 1: 0.05})
    srv = SV.Server(budget_bytes=10, max_slots=4, run_job=run_job,
                    footprint=lambda s: fps[s.job_id])
    srv.run(specs)
    assert live["max"] == 2


def test_scheduler_rejects_job_larger_than_budget():
    """A job that can never fit is rejected at arrival; the others are served."""
    specs, fps = _specs([11, 4, 12, 6], [0.0, 0.0, 0.01, 0.02])
    run_job, live = _fake({j: 0.01 for j in fps})
    srv = SV.Server(budget_bytes=10, run_job=run_job, footprint=lambda s: fps[s.job_id])
    rep = srv.run(specs)
    assert rep["jobs"] == 4 and rep["rejected"] == 2
    assert sorted(rep["errors"]) == [0, 2]
    assert all(e.startswith("rejected") for e in rep["errors"].values())
    assert not rep["results"][0].step_ms and len(rep["results"][1].step_ms) == 2
    assert rep["steps"] == 4 and srv.peak_bytes <= 10


def test_footprint_query_is_host_only():
    from paper_2505_21404_amd import dngd as D
    p = W.config(1)
    b = D.footprint_of(p.pde, p.widths, p.n_int, p.n_bdy, p.n_init)
    # at least J (FP32, m x ldJ) and K (FP64, m x m)
    ldJ = -(-p.n_params // 256) * 256
    assert b >= p.m * ldJ * 4 + p.m * p.m * 8
    b64 = D.footprint_of(p.pde, p.widths, p.n_int, p.n_bdy, p.n_init,
                         D.step_opts(precision=D.PLAIN))
    assert b64 >= p.m * ldJ * 8 + p.m * p.m * 8


def small_jobs(n=8, steps=3):
    """A short job stream like the serving workload, scaled down (m 900-2600,
    width 32-64: several Cholesky block columns per job) so that it runs in
    seconds while jobs overlap on the device."""
    jobs = W.serving_jobs(n_jobs=n, rate=40.0, steps=steps, m_range=(900, 2600),
                          widths_choice=(32, 64), depth=3)
    return SV.specs_from_workloads(jobs)


@pytest.mark.gpu
def test_results_identical_alone_and_in_mix():
    """Every job's parameters after its iterations are bitwise the same alone
    and in the mix (deterministic kernels, no state shared between jobs, and
    no dependence on when a workgroup is scheduled: a mixed stream delays
    workgroups of one job behind another job's kernels)."""
    torch = pytest.importorskip("torch")
    specs = small_jobs()
    alone = {s.job_id: SV.run_alone(s) for s in specs}
    free, _ = torch.cuda.mem_get_info()
    srv = SV.Server(budget_bytes=int(0.5 * free), max_slots=4)
    rep = srv.run(specs, realtime=True)
    print("serving", {k: v for k, v in rep.items() if k != "results"}, flush=True)
    assert not rep["errors"], rep["errors"]
    assert srv.peak_slots >= 2   # the jobs did overlap
    for s in specs:
        a, b = alone[s.job_id].theta, rep["results"][s.job_id].theta
        assert np.array_equal(a, b), (s.job_id, np.abs(a - b).max())


def test_scheduler_assigns_distinct_slots():
    """Jobs that run at the same time hold distinct slot indices in
    [0, max_slots) (JobResult.slot)."""
    active = {}
    lock = threading.Lock()
    clash = []

    def run_job(spec, res):
        with lock:
            if res.slot in active.values() or not (0 <= res.slot < 3):
                clash.append((spec.job_id, res.slot, dict(active)))
            active[spec.job_id] = res.slot
        time.sleep(0.02)
        with lock:
            del active[spec.job_id]
        res.step_ms = [1.0]

    specs = [SV.JobSpec(i, 0.0, None, None, 1) for i in range(12)]
    srv = SV.Server(budget_bytes=10 ** 9, max_slots=3, run_job=run_job, footprint=lambda s: 1)
    rep = srv.run(specs, realtime=False)
    assert not clash, clash
    assert srv.peak_slots == 3 and rep["steps"] == 12
    assert {r.slot for r in rep["results"].values()} == {0, 1, 2}



def test_tail_with_and_without_changes_of_company():
    """A job's step time that depends only on how many jobs run beside it
    has a tail over its own median (company changes as jobs come and go)
    but none over the median of steps taken beside the same jobs."""
    live = set()
    lock = threading.Lock()

    def run_job(spec, res):
        with lock:
            live.add(spec.job_id)
        for _ in range(spec.steps):
            # start time and company read together: a job joins `live` after
            # its admission time and leaves it before its finish time, so a
            # step can only see less company than its interval says (ratio < 1)
            with lock:
                res.step_start.append(res.now())
                k = len(live)
            time.sleep(0.004 * k)
            res.step_ms.append(4.0 * k)  # the step's nominal time: 4 ms per resident job
        with lock:
            live.discard(spec.job_id)

    # job 0 runs alone, then beside the two jobs arriving after it
    specs = [SV.JobSpec(0, 0.0, None, None, 40), SV.JobSpec(1, 0.06, None, None, 5),
             SV.JobSpec(2, 0.06, None, None, 5)]
    srv = SV.Server(budget_bytes=10, max_slots=3, run_job=run_job, footprint=lambda s: 1)
    rep = srv.run(specs, realtime=True)
    assert all(len(r.step_start) == len(r.step_ms) for r in rep["results"].values())
    assert rep["p99_over_job_median"] >= 2.0
    assert rep["p99_over_same_company_median"] <= 1.5


@pytest.mark.gpu
def test_serving_stream_jobs_identical_alone_and_in_mix():
    """The first six jobs of the serving stream itself (heat and Poisson,
    widths 64-256, m 2199-5742), three iterations each, arriving 4 per second
    (compressed 10-fold so that they overlap): every job's parameters are
    bitwise the same alone and in the mix."""
    torch = pytest.importorskip("torch")
    jobs = W.serving_jobs(n_jobs=6, rate=4.0, steps=3)
    for j in jobs:
        j.arrival *= 0.1
    specs = SV.specs_from_workloads(jobs)
    alone = {s.job_id: SV.run_alone(s) for s in specs}
    free, _ = torch.cuda.mem_get_info()
    srv = SV.Server(budget_bytes=int(0.5 * free), max_slots=4)
    rep = srv.run(specs, realtime=True)
    print("serving stream jobs", {k: v for k, v in rep.items() if k != "results"}, flush=True)
    assert not rep["errors"], rep["errors"]
    assert srv.peak_slots >= 2
    for s in specs:
        a, b = alone[s.job_id].theta, rep["results"][s.job_id].theta
        assert np.array_equal(a, b), (s.job_id, np.abs(a - b).max())
