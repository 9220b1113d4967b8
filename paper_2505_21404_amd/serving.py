"""Continuous-batching serving loop for independent D-NGD jobs.

Each job is one PINN instance (points, network, initial parameters) that runs
a fixed number of D-NGD workflow iterations (dngd_iterate: damping rule,
mixed-precision step with geodesic acceleration, line search, update).
Jobs arrive over time. A job waiting at the head of the queue is admitted
as soon as a slot is free and its device footprint (dngd_footprint_desc:
activations, J, K and workspaces) fits in what is left of the memory budget;
admitted jobs run concurrently, each on its own HIP stream driven by its own
host thread (the library calls release the GIL), so their kernels overlap on
the device. A finished job frees its memory and slot, which admits the next.

A job whose footprint exceeds the whole budget is rejected when it arrives
(recorded as an error); the others are served. Per-step latencies (also split
into each job's first step, which allocates the handle's workspace, and the
steady state), admission waits and throughput are recorded; results do
not depend on what else runs (every kernel is deterministic and a job touches
only its own handle and stream).
"""
from __future__ import annotations

import statistics
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

ETA_GRID = [2.0 ** -k for k in range(31)]


@dataclass
class JobSpec:
    """A serving request. ``problem`` has the attributes of a PINN instance
    (pde, widths, x_int, x_bdy, x_init, f_int, g_bdy, g_init, kappa)."""
    job_id: int
    arrival: float          # seconds after the start of the run
    problem: object
    theta0: object          # n FP64 (host array)
    steps: int
    lam_cap: float = 1e-5


@dataclass
class JobResult:
    job_id: int
    arrival: float
    admitted: float
    finished: float
    footprint: int
    step_ms: List[float] = field(default_factory=list)
    losses: List[float] = field(default_factory=list)
    theta: object = None
    error: Optional[str] = None
    slot: int = -1          # the slot the job ran in (0 .. max_slots-1)
    # start of each step in seconds after the start of the run, read from
    # ``now`` (the server's clock, set at admission) by the executor
    step_start: List[float] = field(default_factory=list)
    now: Optional[Callable[[], float]] = None


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = max(0, min(len(xs) - 1, int(round(q * (len(xs) - 1)))))
    return xs[k]


class Server:
    """Admission by slots and memory budget, first come first served.

    ``run_job(spec, result)`` executes a job (it fills result.step_ms,
    result.losses, result.theta) and ``footprint(spec)`` returns its device
    bytes; both default to the HIP library (see ``gpu_executor``) and can be
    replaced, e.g. to test the scheduler without a device."""

    def __init__(self, budget_bytes: int, max_slots: int = 4,
                 run_job: Optional[Callable] = None, footprint: Optional[Callable] = None,
                 clock: Callable[[], float] = time.perf_counter):
        if max_slots < 1:
            raise ValueError("max_slots must be >= 1")
        self.budget = int(budget_bytes)
        self.max_slots = max_slots
        if run_job is None or footprint is None:
            fp, rj = gpu_executor()
            run_job = run_job or rj
            footprint = footprint or fp
        self._run_job = run_job
        self._footprint = footprint
        self._clock = clock
        self._lock = threading.Condition()
        self.peak_bytes = 0
        self.peak_slots = 0
        self.events: List[tuple] = []   # (time, "admit"/"finish", job_id, bytes_in_use, active)

    def run(self, jobs: List[JobSpec], realtime: bool = True) -> Dict:
        """Serve ``jobs``; with ``realtime`` a job becomes eligible at its
        arrival time, otherwise all are eligible at once (in arrival order)."""
        fps = {j.job_id: int(self._footprint(j)) for j in jobs}
        results: Dict[int, JobResult] = {}
        # a job that can never fit is rejected when it arrives; the rest are served
        rejected = [j for j in jobs if fps[j.job_id] > self.budget]
        for j in rejected:
            results[j.job_id] = JobResult(
                j.job_id, j.arrival, j.arrival, j.arrival, fps[j.job_id],
                error=f"rejected: footprint {fps[j.job_id]} B exceeds the budget {self.budget} B")
        pending = sorted((j for j in jobs if fps[j.job_id] <= self.budget),
                         key=lambda j: (j.arrival, j.job_id))
        in_use = 0
        active = 0
        free_slots = list(range(self.max_slots))
        threads = []
        t_start = self._clock()

        def worker(spec: JobSpec, res: JobResult):
            nonlocal in_use, active
            try:
                self._run_job(spec, res)
            except Exception as e:  # recorded, the loop goes on
                res.error = f"{type(e).__name__}: {e}"
            with self._lock:
                res.finished = self._clock() - t_start
                in_use -= res.footprint
                active -= 1
                free_slots.append(res.slot)
                free_slots.sort()
                self.events.append((res.finished, "finish", spec.job_id, in_use, active))
                self._lock.notify_all()

        queue: List[JobSpec] = []
        i = 0
        with self._lock:
            while i < len(pending) or queue or active:
                now = self._clock() - t_start
                while i < len(pending) and (not realtime or pending[i].arrival <= now):
                    queue.append(pending[i])
                    i += 1
                # admit from the head while the head fits
                while queue and active < self.max_slots and \
                        in_use + fps[queue[0].job_id] <= self.budget:
                    spec = queue.pop(0)
                    res = JobResult(spec.job_id, spec.arrival, now, 0.0, fps[spec.job_id])
                    res.slot = free_slots.pop(0)
                    res.now = lambda: self._clock() - t_start
                    results[spec.job_id] = res
                    in_use += res.footprint
                    active += 1
                    self.peak_bytes = max(self.peak_bytes, in_use)
                    self.peak_slots = max(self.peak_slots, active)
                    self.events.append((now, "admit", spec.job_id, in_use, active))
                    th = threading.Thread(target=worker, args=(spec, res), daemon=True)
                    threads.append(th)
                    th.start()
                # sleep until the next arrival or a job finishes
                timeout = None
                if i < len(pending) and realtime:
                    timeout = max(0.0, pending[i].arrival - (self._clock() - t_start))
                if i < len(pending) and not realtime:
                    timeout = 0.0
                if timeout is None or timeout > 0.0:
                    self._lock.wait(timeout=timeout if timeout is not None else 1.0)
        for th in threads:
            th.join()
        makespan = self._clock() - t_start
        return report(results, makespan, self)


def report(results: Dict[int, JobResult], makespan: float, server: Server) -> Dict:
    lat = [x for r in results.values() for x in r.step_ms]
    served = [r for r in results.values() if not (r.error or "").startswith("rejected")]
    waits = [r.admitted - r.arrival for r in served]
    first = [r.step_ms[0] for r in served if r.step_ms]
    steady = [x for r in served for x in r.step_ms[1:]]
    # each step against its own job's median: the tail that interference adds,
    # apart from the spread of job sizes
    norm = [x / statistics.median(r.step_ms) for r in served if r.step_ms for x in r.step_ms]
    steps = len(lat)
    # each step against the median of the same job's steps that ran beside the
    # same set of other jobs: the tail of interference alone, without the
    # changes of company as jobs finish and others are admitted
    same = float("nan")
    timed = [r for r in served if r.step_ms]
    if timed and all(len(r.step_start) == len(r.step_ms) for r in timed):
        span = {r.job_id: (r.admitted, r.finished) for r in served}
        ratios = []
        for r in timed:
            groups: Dict[tuple, List[float]] = {}
            for t, x in zip(r.step_start, r.step_ms):
                key = tuple(sorted(k for k, (a, f) in span.items()
                                   if k != r.job_id and a <= t < f))
                groups.setdefault(key, []).append(x)
            for xs in groups.values():
                med = statistics.median(xs)
                ratios += [x / med for x in xs]
        same = percentile(ratios, 0.99)
    return {
        "jobs": len(results),
        "rejected": len(results) - len(served),
        "errors": {r.job_id: r.error for r in results.values() if r.error},
        "steps": steps,
        "makespan_s": makespan,
        "steps_per_s": steps / makespan if makespan > 0 else float("nan"),
        "p50_step_ms": percentile(lat, 0.50),
        "p99_step_ms": percentile(lat, 0.99),
        "first_step_p50_ms": percentile(first, 0.50),
        "steady_p50_step_ms": percentile(steady, 0.50),
        "steady_p99_step_ms": percentile(steady, 0.99),
        "p99_over_job_median": percentile(norm, 0.99),
        "p99_over_same_company_median": same,
        "mean_step_ms": statistics.fmean(lat) if lat else float("nan"),
        "admission_wait_p50_s": percentile(waits, 0.50),
        "admission_wait_max_s": max(waits) if waits else float("nan"),
        "peak_bytes": server.peak_bytes,
        "peak_slots": server.peak_slots,
        "results": results,
    }


def specs_from_workloads(jobs, lam_cap_poisson: float = 1e-5, lam_cap_heat: float = 1e-3):
    """JobSpecs from workload jobs (objects with job_id, arrival, problem,
    theta0, steps); the damping cap follows the PDE (Poisson 1e-5, heat 1e-3)."""
    return [JobSpec(j.job_id, j.arrival, j.problem, j.theta0, j.steps,
                    lam_cap_heat if j.problem.pde == 1 else lam_cap_poisson) for j in jobs]


def gpu_executor(device: str = "cuda", opts_fn: Optional[Callable] = None,
                 lookahead: bool = False):
    """(footprint, run_job) backed by libdngd: each job gets its own handle,
    its own torch stream and the mixed-precision dense step with GA. The
    factorisation's look-ahead (a trailing update that reserves whole CUs
    beside the panels) is meant for a device with one job; with several
    resident jobs it is off unless ``lookahead``."""
    import torch

    from . import dngd as D

    def make_opts(spec):
        if opts_fn:
            return opts_fn(spec)
        return D.step_opts(precision=D.MIXED, ga=True, no_lookahead=not lookahead)

    def footprint(spec: JobSpec) -> int:
        p = spec.problem
        return D.footprint_of(p.pde, p.widths, len(p.x_int), len(p.x_bdy), len(p.x_init),
                              make_opts(spec))

    def run_job(spec: JobSpec, res: JobResult):
        stream = torch.cuda.Stream(device=device)
        with torch.cuda.stream(stream):
            prob = D.Problem.from_workload(spec.problem, device=device)
            try:
                theta = torch.tensor(spec.theta0, dtype=torch.float64, device=device)
                stream.synchronize()
                opts = make_opts(spec)
                for _ in range(spec.steps):
                    if res.now is not None:
                        res.step_start.append(res.now())
                    t0 = time.perf_counter()
                    st = prob.iterate(theta, ETA_GRID, lam_cap=spec.lam_cap, opts=opts,
                                      stream=stream)
                    res.step_ms.append((time.perf_counter() - t0) * 1e3)
                    res.losses.append(st.loss)
                res.theta = theta.cpu().numpy()
            finally:
                stream.synchronize()
                prob.close()

    return footprint, run_job


def run_alone(spec: JobSpec, device: str = "cuda", opts_fn: Optional[Callable] = None,
              lookahead: bool = False):
    """The same job on an idle device (reference for the mix)."""
    _, run_job = gpu_executor(device, opts_fn, lookahead)
    res = JobResult(spec.job_id, spec.arrival, 0.0, 0.0, 0)
    run_job(spec, res)
    return res
