"""Seeded synthetic inputs for the D-NGD step: network widths, Glorot-initialised
parameters, collocation points, PDE target values, landmark index sets and the
serving job stream.

This module is shared by the CPU oracle and the GPU path. It holds problem
*data* only (where points lie, what the source term and boundary values are),
none of the method's arithmetic: no residuals, derivatives, Gram matrices or
solves. Every draw comes from ``numpy.random.default_rng`` with a documented
seed offset so both sides see identical inputs.

Seeds: parameters ``seed``, points ``seed+1``, evaluation points ``seed+2``,
landmarks ``seed+3+k`` (outer step k), serving arrivals ``1000``, serving job j
``1001+j``.

The PDE families follow the paper's problem statement (Section 2.1, the PINN
loss): an interior operator class plus boundary (and, for the heat equation,
initial) classes, each sampled uniformly.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

POISSON = 0
HEAT = 1
NAVIER_STOKES = 2


@dataclasses.dataclass
class Problem:
    """One PINN instance: tanh MLP widths, PDE kind and the three point classes.

    Points are row-major ``(N, d_in)`` float64. For the heat equation the
    inputs are ordered ``(x, y, t)``: the Laplacian acts on the first
    ``d_in - 1`` coordinates and the time derivative on the last one.
    Targets: ``f_int`` is the interior source (Poisson: ``-lap u = f``; heat:
    zero), ``g_bdy`` the Dirichlet value, ``g_init`` the initial value.
    """

    pde: int
    widths: List[int]
    x_int: np.ndarray
    x_bdy: np.ndarray
    x_init: np.ndarray
    f_int: np.ndarray
    g_bdy: np.ndarray
    g_init: np.ndarray
    kappa: float = 0.0
    amplitude: float = 1.0
    name: str = ""
    solution: str = ""  # key into exact_solution()
    d_int: int = 1      # residual components per interior point (3 for Navier-Stokes)
    d_bdy: int = 1      # residual components per boundary point

    @property
    def d_in(self) -> int:
        return self.widths[0]

    @property
    def n_int(self) -> int:
        return self.x_int.shape[0]

    @property
    def n_bdy(self) -> int:
        return self.x_bdy.shape[0]

    @property
    def n_init(self) -> int:
        return self.x_init.shape[0]

    @property
    def m(self) -> int:
        """Residual-space size sum_gamma N_gamma d_gamma."""
        return self.n_int * self.d_int + self.n_bdy * self.d_bdy + self.n_init

    @property
    def n_params(self) -> int:
        return sum(self.widths[l + 1] * self.widths[l] + self.widths[l + 1]
                   for l in range(len(self.widths) - 1))


# ----------------------------------------------------------------------------
# parameters


def glorot_theta(widths, seed: int) -> np.ndarray:
    """Glorot-uniform weights ``U[-s, s]``, ``s = sqrt(6/(fan_in+fan_out))``,
    zero biases, drawn layer by layer; flat layout per layer: ``W`` row-major
    ``[out][in]`` then ``b[out]``."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        fin, fout = widths[l], widths[l + 1]
        s = math.sqrt(6.0 / (fin + fout))
        parts.append(rng.uniform(-s, s, size=(fout, fin)).ravel())
        parts.append(np.zeros(fout))
    return np.concatenate(parts).astype(np.float64)


def random_direction(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A seeded standard-normal vector (used as a test direction or adjoint)."""
    return scale * np.random.default_rng(seed).standard_normal(n)


# ----------------------------------------------------------------------------
# points


def _box_interior(rng, n, d):
    return rng.uniform(0.0, 1.0, size=(n, d))


def _box_boundary(rng, n, d):
    """Uniform on the surface of [0,1]^d: a face (all 2d faces have equal
    area) uniformly, then uniform on that face."""
    x = rng.uniform(0.0, 1.0, size=(n, d))
    face = rng.integers(0, 2 * d, size=n)
    dim = face // 2
    x[np.arange(n), dim] = (face % 2).astype(np.float64)
    return x


def _heat_boundary(rng, n):
    """Spatial boundary of [0,1]^2 times t ~ U[0,1]; columns (x, y, t)."""
    xy = _box_boundary(rng, n, 2)
    t = rng.uniform(0.0, 1.0, size=(n, 1))
    return np.hstack([xy, t])


def _heat_interior(rng, n):
    return rng.uniform(0.0, 1.0, size=(n, 3))


def _heat_initial(rng, n):
    xy = rng.uniform(0.0, 1.0, size=(n, 2))
    return np.hstack([xy, np.zeros((n, 1))])


# ----------------------------------------------------------------------------
# closed-form fields (problem data: exact solutions and the sources they imply)


def exact_solution(key: str, x: np.ndarray, kappa: float = 0.0, amplitude: float = 1.0):
    """Analytic solution used to build targets and to measure relative L2 error."""
    if key == "sinsin":  # u = A sin(pi x) sin(pi y) on [0,1]^2
        return amplitude * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1])
    if key == "sumsin_half":  # u = sum_i sin(pi x_i / 2)
        return np.sin(0.5 * np.pi * x).sum(axis=1)
    if key == "heat_sinsin":  # u = A exp(-2 pi^2 kappa t) sin(pi x) sin(pi y)
        return (amplitude * np.exp(-2.0 * np.pi ** 2 * kappa * x[:, 2])
                * np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]))
    if key == "kovasznay":  # (u, v, p) of Kovasznay flow, nu = kappa
        return kovasznay_fields(x, kappa)
    raise KeyError(key)


KOVASZNAY_BOX = ((-0.5, 1.0), (-0.5, 1.5))


def kovasznay_fields(x: np.ndarray, nu: float) -> np.ndarray:
    """Kovasznay's closed-form steady Navier-Stokes solution (u, v, p) at the
    points x (N, 2) for viscosity nu: with l = 1/(2 nu) - sqrt(1/(4 nu^2) + 4 pi^2),
    u = 1 - e^{l x} cos(2 pi y), v = l/(2 pi) e^{l x} sin(2 pi y),
    p = (1 - e^{2 l x}) / 2."""
    lam = 0.5 / nu - math.sqrt(0.25 / nu ** 2 + 4.0 * math.pi ** 2)
    ex = np.exp(lam * x[:, 0])
    c, sn = np.cos(2.0 * np.pi * x[:, 1]), np.sin(2.0 * np.pi * x[:, 1])
    return np.stack([1.0 - ex * c, lam / (2.0 * np.pi) * ex * sn, 0.5 * (1.0 - ex * ex)], axis=1)


def _rect_interior(rng, n, box):
    (x0, x1), (y0, y1) = box
    return np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], axis=1)


def _rect_boundary(rng, n, box):
    """Uniform in arc length on the rectangle's perimeter."""
    (x0, x1), (y0, y1) = box
    w, h = x1 - x0, y1 - y0
    s = rng.uniform(0.0, 2.0 * (w + h), n)
    out = np.empty((n, 2))
    for i, t in enumerate(s):
        if t < w:
            out[i] = (x0 + t, y0)
        elif t < w + h:
            out[i] = (x1, y0 + (t - w))
        elif t < 2 * w + h:
            out[i] = (x1 - (t - w - h), y1)
        else:
            out[i] = (x0, y1 - (t - 2 * w - h))
    return out


def kovasznay(seed: int = 0, widths=(2, 50, 50, 50, 50, 3), n_int: int = 400, n_bdy: int = 400,
              nu: float = 1.0 / 40.0) -> Problem:
    """Kovasznay flow at Re = 1/nu = 40 on [-0.5, 1.0] x [-0.5, 1.5]
    (Section 5.3 and its hyper-parameter table): a [2, 50 x 4, 3] tanh MLP for
    (u, v, p), N_int interior and N_bdy boundary points drawn uniformly (area and
    arc length). Interior targets f = 0 for the three equations; boundary values
    of u, v and p from the closed-form solution. m = 3 N_int + 3 N_bdy."""
    assert widths[0] == 2 and widths[-1] == 3
    rng = np.random.default_rng(seed + 1)
    xi = _rect_interior(rng, n_int, KOVASZNAY_BOX)
    xb = _rect_boundary(rng, n_bdy, KOVASZNAY_BOX)
    return Problem(
        pde=NAVIER_STOKES, widths=list(widths), x_int=xi, x_bdy=xb, x_init=np.zeros((0, 2)),
        f_int=np.zeros((n_int, 3)), g_bdy=kovasznay_fields(xb, nu), g_init=np.zeros(0),
        kappa=nu, name=f"kovasznay_re{round(1.0 / nu)}_m{3 * (n_int + n_bdy)}",
        solution="kovasznay", d_int=3, d_bdy=3)


def _source(key: str, x: np.ndarray, amplitude: float = 1.0):
    """Interior right-hand side f with -lap u* = f for the Poisson fields."""
    if key == "sinsin":
        return 2.0 * np.pi ** 2 * exact_solution(key, x, amplitude=amplitude)
    if key == "sumsin_half":
        return (np.pi ** 2 / 4.0) * np.sin(0.5 * np.pi * x).sum(axis=1)
    raise KeyError(key)


def poisson_problem(widths, n_int, n_bdy, solution, seed, amplitude=1.0, name=""):
    d = widths[0]
    rng = np.random.default_rng(seed + 1)
    xi = _box_interior(rng, n_int, d)
    xb = _box_boundary(rng, n_bdy, d)
    return Problem(
        pde=POISSON, widths=list(widths), x_int=xi, x_bdy=xb,
        x_init=np.zeros((0, d)), f_int=_source(solution, xi, amplitude),
        g_bdy=exact_solution(solution, xb, amplitude=amplitude),
        g_init=np.zeros(0), amplitude=amplitude, name=name, solution=solution)


def heat_problem(widths, n_int, n_bdy, n_init, kappa, seed, amplitude=1.0, name=""):
    assert widths[0] == 3
    rng = np.random.default_rng(seed + 1)
    xi = _heat_interior(rng, n_int)
    xb = _heat_boundary(rng, n_bdy)
    x0 = _heat_initial(rng, n_init)
    return Problem(
        pde=HEAT, widths=list(widths), x_int=xi, x_bdy=xb, x_init=x0,
        f_int=np.zeros(n_int), g_bdy=np.zeros(n_bdy),
        g_init=exact_solution("heat_sinsin", x0, kappa, amplitude),
        kappa=kappa, amplitude=amplitude, name=name, solution="heat_sinsin")


def eval_points(problem: Problem, n: int = 10_000, seed: int = 0):
    """Fresh uniform points in the (space-time) domain for relative L2 error."""
    rng = np.random.default_rng(seed + 2)
    if problem.pde == NAVIER_STOKES:
        return _rect_interior(rng, n, KOVASZNAY_BOX)
    return rng.uniform(0.0, 1.0, size=(n, problem.d_in))


def landmarks(m: int, ell: int, seed: int, step: int = 0) -> np.ndarray:
    """Nystrom landmark residual indices: uniform without replacement over all
    m residual components, sorted ascending (int64)."""
    rng = np.random.default_rng(seed + 3 + step)
    return np.sort(rng.choice(m, size=min(ell, m), replace=False)).astype(np.int64)


# ----------------------------------------------------------------------------
# the five workloads


CONFIG_NAMES = {
    0: "poisson2d_w32x2_m500_fp64",
    1: "poisson5d_w256x3_m5000",
    2: "heat2p1d_w1024x4_m8192",
    3: "poisson5d_w2048x4_m50000_pcg",
    4: "serving_stream_64jobs",
}

LAMBDA = {0: 1e-8}
LAMBDA_CAP = {0: 1e-8, 1: 1e-5, 2: 1e-3, 3: 1e-5}


def config(idx: int, seed: int = 0, scale: Optional[dict] = None) -> Problem:
    """Build workload ``idx`` (0-3). ``scale`` may override ``widths``,
    ``n_int``, ``n_bdy``, ``n_init`` to make a scaled mirror of the same
    structure."""
    s = dict(scale or {})
    if idx == 0:
        return poisson_problem(s.get("widths", [2, 32, 32, 1]), s.get("n_int", 400),
                               s.get("n_bdy", 100), "sinsin", seed, name=CONFIG_NAMES[0])
    if idx == 1:
        return poisson_problem(s.get("widths", [5, 256, 256, 256, 1]), s.get("n_int", 4000),
                               s.get("n_bdy", 1000), "sumsin_half", seed, name=CONFIG_NAMES[1])
    if idx == 2:
        return heat_problem(s.get("widths", [3, 1024, 1024, 1024, 1024, 1]),
                            s.get("n_int", 6144), s.get("n_bdy", 1024), s.get("n_init", 1024),
                            0.1, seed, name=CONFIG_NAMES[2])
    if idx == 3:
        return poisson_problem(s.get("widths", [5, 2048, 2048, 2048, 2048, 1]),
                               s.get("n_int", 45000), s.get("n_bdy", 5000), "sumsin_half",
                               seed, name=CONFIG_NAMES[3])
    raise ValueError(idx)


@dataclasses.dataclass
class Job:
    """One serving request: arrival time (s), problem, initial parameters."""
    job_id: int
    arrival: float
    problem: Problem
    theta0: np.ndarray
    steps: int


def serving_jobs(n_jobs: int = 64, rate: float = 4.0, steps: int = 200,
                 m_range=(500, 8000), widths_choice=(64, 128, 256), depth: int = 3):
    """Poisson-process job stream: exponential inter-arrival (mean 1/rate),
    PDE kind Bernoulli(1/2), kappa ~ U[0.05,0.5], amplitude ~ U[0.5,2],
    hidden width from ``widths_choice`` at ``depth`` hidden layers,
    m ~ U{m_range}. Class split 4:1 (Poisson) or 6:1:1 (heat)."""
    rng = np.random.default_rng(1000)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        heat = bool(rng.integers(0, 2))
        kappa = float(rng.uniform(0.05, 0.5))
        amp = float(rng.uniform(0.5, 2.0))
        w = int(rng.choice(widths_choice))
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        seed = 1001 + j
        if heat:
            n_b = m // 8
            n_0 = m // 8
            n_i = m - n_b - n_0
            prob = heat_problem([3] + [w] * depth + [1], n_i, n_b, n_0, kappa, seed,
                                amplitude=amp, name=f"job{j}_heat")
        else:
            n_b = m // 5
            n_i = m - n_b
            prob = poisson_problem([2] + [w] * depth + [1], n_i, n_b, "sinsin", seed,
                                   amplitude=amp, name=f"job{j}_poisson")
        jobs.append(Job(j, t, prob, glorot_theta(prob.widths, seed), steps))
    return jobs
