"""ctypes binding of libdngd (include/dngd.h): argument marshalling only.

Every computation runs in the HIP library; PyTorch provides device memory and
the current stream. If libdngd.so is missing this module raises at import;
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdngd.so")

OK, ENOCONV, EINVAL, ENOMEM, EHIP, ENOTPD, ENAN = 0, 1, -1, -2, -3, -4, -5
F64, F32, BF16 = 0, 1, 2
GRAM_F64 = 64   # gram_passes value: FP64-product Gram of an FP32 J
POISSON, HEAT, NAVIER_STOKES = 0, 1, 2
PLAIN, MIXED = 0, 1
DENSE, PCG, PRIMAL, DENSE_AUTO, STRUCTURED = 0, 1, 2, 3, 4

_STATUS = {ENOCONV: "DNGD_ENOCONV", EINVAL: "DNGD_EINVAL", ENOMEM: "DNGD_ENOMEM", EHIP: "DNGD_EHIP",
           ENOTPD: "DNGD_ENOTPD", ENAN: "DNGD_ENAN"}


class DngdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [("pde", C.c_int32), ("n_layers", C.c_int32), ("widths", C.POINTER(C.c_int32)),
                ("kappa", C.c_double), ("n_int", C.c_int64), ("n_bdy", C.c_int64),
                ("n_init", C.c_int64), ("x_int", C.c_void_p), ("x_bdy", C.c_void_p),
                ("x_init", C.c_void_p), ("f_int", C.c_void_p), ("g_bdy", C.c_void_p),
                ("g_init", C.c_void_p)]


class StepOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("solver", C.c_int32), ("ga", C.c_int32),
                ("ir_sweeps", C.c_int32), ("gram_passes", C.c_int32), ("no_lookahead", C.c_int32),
                ("eps_norm", C.c_double), ("n_landmarks", C.c_int64), ("landmarks", C.c_void_p),
                ("pcg_tol", C.c_double), ("pcg_maxit", C.c_int64), ("ir_tol", C.c_double),
                ("alpha_out", C.c_void_p), ("fvv_out", C.c_void_p),
                ("nystrom_chunk_rows", C.c_int64), ("nystrom_reuse", C.c_int32),
                ("pcg_kvp", C.c_int32)]


class Refine(C.Structure):
    _fields_ = [("J", C.c_void_p), ("n", C.c_int64), ("ldJ", C.c_int64), ("j_dtype", C.c_int32),
                ("sweeps", C.c_int32), ("lam", C.c_double)]


class StepStats(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_residual_jacobian", C.c_double),
                ("ms_gram", C.c_double), ("ms_factor", C.c_double), ("ms_solve_v", C.c_double),
                ("ms_fvv", C.c_double), ("ms_solve_a", C.c_double), ("vnorm", C.c_double),
                ("anorm", C.c_double), ("ga_accepted", C.c_int32),
                ("gram_passes_used", C.c_int32), ("pcg_iterations", C.c_int32),
                ("pcg_converged", C.c_int32), ("ir_residual", C.c_double * 8),
                ("max_row_norm2", C.c_double), ("pcg_rel_residual", C.c_double),
                ("ms_gram_kernel", C.c_double), ("gram_attempts", C.c_int32),
                ("pcg_iterations_ga", C.c_int32), ("primal", C.c_int32),
                ("ga_early_reject", C.c_int32), ("nystrom_shift", C.c_double),
                ("nystrom_reused", C.c_int32), ("pcg_kvp_f64", C.c_int32),
                ("pcg_replacements", C.c_int32), ("pcg_escalated", C.c_int32),
                ("gram_start_passes", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "ir_residual"}
        d["ir_residual"] = list(self.ir_residual)
        return d


class IterStats(C.Structure):
    _fields_ = [("loss", C.c_double), ("lam", C.c_double), ("eta", C.c_double),
                ("loss_new", C.c_double), ("ms_line_search", C.c_double),
                ("eta_index", C.c_int32), ("step_status", C.c_int32), ("step", StepStats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "step"}
        d["step"] = self.step.as_dict()
        return d


EXPORTS = [
    "dngd_last_error", "dngd_version", "dngd_step_opts_default", "dngd_problem_create",
    "dngd_problem_destroy", "dngd_num_params", "dngd_num_residuals", "dngd_jacobian_ld",
    "dngd_footprint", "dngd_residual_jacobian", "dngd_gram", "dngd_cholesky_solve", "dngd_fvv",
    "dngd_jvp", "dngd_vjp", "dngd_losses", "dngd_nystrom_pcg", "dngd_step", "dngd_iterate",
    "dngd_footprint_desc", "dngd_cholesky_solve_noalloc", "dngd_kvp",
    "dngd_cholesky_solve_refine",
]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it first (python -m paper_2505_21404_amd.build)")
    lib = C.CDLL(path)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    sig = {
        "dngd_last_error": (C.c_char_p, []),
        "dngd_version": (C.c_char_p, []),
        "dngd_step_opts_default": (None, [C.POINTER(StepOpts)]),
        "dngd_problem_create": (C.c_int, [C.POINTER(ProblemDesc), C.POINTER(vp)]),
        "dngd_problem_destroy": (C.c_int, [vp]),
        "dngd_num_params": (i64, [vp]),
        "dngd_num_residuals": (i64, [vp]),
        "dngd_jacobian_ld": (i64, [vp]),
        "dngd_footprint": (C.c_int, [vp, C.POINTER(StepOpts), C.POINTER(C.c_size_t)]),
        "dngd_footprint_desc": (C.c_int, [C.POINTER(ProblemDesc), C.POINTER(StepOpts),
                                          C.POINTER(C.c_size_t)]),
        "dngd_residual_jacobian": (C.c_int, [vp, vp, vp, vp, i64, i32, vp]),
        "dngd_gram": (C.c_int, [i64, i64, vp, i64, i32, i32, dbl, vp, i64, vp]),
        "dngd_cholesky_solve": (C.c_int, [i64, vp, i64, i32, i64, vp, i64, C.POINTER(i64), vp]),
        "dngd_cholesky_solve_noalloc": (C.c_int, [i64, vp, i64, i32, i64, vp, i64,
                                                  C.POINTER(i64), vp]),
        "dngd_cholesky_solve_refine": (C.c_int, [i64, vp, i64, i32, i64, vp, i64,
                                                 C.POINTER(Refine), vp, C.POINTER(i64), vp]),
        "dngd_fvv": (C.c_int, [vp, vp, vp, vp, vp]),
        "dngd_jvp": (C.c_int, [vp, vp, vp, vp, vp]),
        "dngd_vjp": (C.c_int, [vp, vp, vp, vp, vp]),
        "dngd_kvp": (C.c_int, [vp, vp, dbl, vp, vp, i32, vp]),
        "dngd_losses": (C.c_int, [vp, vp, vp, i32, C.POINTER(dbl), C.POINTER(dbl), vp]),
        "dngd_nystrom_pcg": (C.c_int, [vp, vp, dbl, vp, i64, dbl, i64, vp, vp,
                                       C.POINTER(StepStats), vp]),
        "dngd_step": (C.c_int, [vp, vp, dbl, C.POINTER(StepOpts), vp, C.POINTER(StepStats), vp]),
        "dngd_iterate": (C.c_int, [vp, vp, dbl, dbl, C.POINTER(StepOpts), i32, C.POINTER(dbl), vp,
                                   C.POINTER(IterStats), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = load_library()


def _check(rc: int, allow=(OK,)):
    if rc not in allow:
        raise DngdError(rc, _lib.dngd_last_error().decode())
    return rc


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(x, device) -> torch.Tensor:
    return torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()


def version() -> str:
    return _lib.dngd_version().decode()


def step_opts(precision=MIXED, solver=DENSE, ga=True, ir_sweeps=2, gram_passes=0, eps_norm=0.0,
              landmarks: Optional[torch.Tensor] = None, pcg_tol=1e-6, pcg_maxit=500,
              ir_tol: Optional[float] = None, alpha_out: Optional[torch.Tensor] = None,
              fvv_out: Optional[torch.Tensor] = None, nystrom_chunk_rows: int = 0,
              nystrom_reuse: int = 0, no_lookahead: bool = False, pcg_kvp: int = F64) -> StepOpts:
    o = StepOpts()
    _lib.dngd_step_opts_default(C.byref(o))
    o.precision, o.solver, o.ga = precision, solver, int(bool(ga))
    o.ir_sweeps, o.gram_passes, o.eps_norm = ir_sweeps, gram_passes, eps_norm
    if landmarks is not None:
        o.n_landmarks = landmarks.numel()
        o.landmarks = landmarks.data_ptr()
        o._landmarks_ref = landmarks   # the options hold a device pointer into it
    o.pcg_tol, o.pcg_maxit = pcg_tol, pcg_maxit
    o.nystrom_chunk_rows, o.nystrom_reuse = int(nystrom_chunk_rows), int(nystrom_reuse)
    o.no_lookahead = int(bool(no_lookahead))
    o.pcg_kvp = int(pcg_kvp)
    if ir_tol is not None:
        o.ir_tol = ir_tol
    for name, t in (("alpha_out", alpha_out), ("fvv_out", fvv_out)):
        if t is not None:
            assert t.dtype == torch.float64 and t.is_contiguous() and t.is_cuda
            setattr(o, name, t.data_ptr())
            setattr(o, "_" + name + "_ref", t)
    return o


class Problem:
    """A PINN instance resident on the GPU (wraps dngd_problem)."""

    def __init__(self, pde: int, widths: Sequence[int], x_int, x_bdy, x_init, f_int, g_bdy,
                 g_init, kappa: float = 0.0, device="cuda"):
        self.device = torch.device(device)
        self.widths = [int(w) for w in widths]
        arrs = [_dev_f64(a, self.device) for a in (x_int, x_bdy, x_init, f_int, g_bdy, g_init)]
        self._w = (C.c_int32 * len(self.widths))(*self.widths)
        d = ProblemDesc()
        d.pde, d.n_layers, d.widths, d.kappa = pde, len(self.widths) - 1, self._w, float(kappa)
        d.n_int, d.n_bdy, d.n_init = arrs[0].shape[0], arrs[1].shape[0], arrs[2].shape[0]
        d.x_int, d.x_bdy, d.x_init = [a.data_ptr() if a.numel() else None for a in arrs[:3]]
        d.f_int, d.g_bdy, d.g_init = [a.data_ptr() if a.numel() else None for a in arrs[3:]]
        # the device copies above were enqueued on the current stream; the
        # handle copies them with a synchronous call on the legacy stream
        torch.cuda.current_stream(self.device).synchronize()
        h = C.c_void_p()
        _check(_lib.dngd_problem_create(C.byref(d), C.byref(h)))
        self._h = h
        self.n = int(_lib.dngd_num_params(h))
        self.m = int(_lib.dngd_num_residuals(h))
        self.ldJ = int(_lib.dngd_jacobian_ld(h))

    @classmethod
    def from_workload(cls, p, device="cuda"):
        """Build from any object with the attributes of a PINN instance
        (pde, widths, x_int, x_bdy, x_init, f_int, g_bdy, g_init, kappa)."""
        return cls(p.pde, p.widths, p.x_int, p.x_bdy, p.x_init, p.f_int, p.g_bdy, p.g_init,
                   p.kappa, device)

    def close(self):
        if getattr(self, "_h", None):
            _lib.dngd_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _theta(self, theta):
        t = _dev_f64(theta, self.device)
        assert t.numel() == self.n, (t.numel(), self.n)
        return t

    def footprint(self, opts: Optional[StepOpts] = None) -> int:
        b = C.c_size_t()
        _check(_lib.dngd_footprint(self._h, C.byref(opts) if opts else None, C.byref(b)))
        return int(b.value)

    def residual(self, theta, stream=None) -> torch.Tensor:
        th = self._theta(theta)
        r = torch.empty(self.m, dtype=torch.float64, device=self.device)
        _check(_lib.dngd_residual_jacobian(self._h, _ptr(th), _ptr(r), None, 0, F64,
                                           _stream(stream)))
        return r

    def residual_jacobian(self, theta, j_dtype=F64, stream=None):
        th = self._theta(theta)
        r = torch.empty(self.m, dtype=torch.float64, device=self.device)
        dt = torch.float64 if j_dtype == F64 else torch.float32
        J = torch.empty(self.m, self.ldJ, dtype=dt, device=self.device)
        _check(_lib.dngd_residual_jacobian(self._h, _ptr(th), _ptr(r), _ptr(J), self.ldJ, j_dtype,
                                           _stream(stream)))
        return r, J

    def fvv(self, theta, v, stream=None) -> torch.Tensor:
        th, vv = self._theta(theta), self._theta(v)
        out = torch.empty(self.m, dtype=torch.float64, device=self.device)
        _check(_lib.dngd_fvv(self._h, _ptr(th), _ptr(vv), _ptr(out), _stream(stream)))
        return out

    def jvp(self, theta, u, stream=None) -> torch.Tensor:
        th, uu = self._theta(theta), self._theta(u)
        out = torch.empty(self.m, dtype=torch.float64, device=self.device)
        _check(_lib.dngd_jvp(self._h, _ptr(th), _ptr(uu), _ptr(out), _stream(stream)))
        return out

    def vjp(self, theta, p, stream=None) -> torch.Tensor:
        th = self._theta(theta)
        pp = _dev_f64(p, self.device)
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(_lib.dngd_vjp(self._h, _ptr(th), _ptr(pp), _ptr(out), _stream(stream)))
        return out

    def kvp(self, theta, lam: float, p, dtype: int = F64, stream=None) -> torch.Tensor:
        """w = J (J^T p) + lam p (dngd_kvp), FP64 or bf16 products."""
        th = self._theta(theta)
        pp = _dev_f64(p, self.device)
        out = torch.empty(self.m, dtype=torch.float64, device=self.device)
        _check(_lib.dngd_kvp(self._h, _ptr(th), float(lam), _ptr(pp), _ptr(out), int(dtype),
                             _stream(stream)))
        return out

    def losses(self, theta, dtheta, etas, stream=None):
        th, dth = self._theta(theta), self._theta(dtheta)
        etas = [float(e) for e in etas]
        ea = (C.c_double * len(etas))(*etas)
        la = (C.c_double * len(etas))()
        _check(_lib.dngd_losses(self._h, _ptr(th), _ptr(dth), len(etas), ea, la, _stream(stream)))
        return list(la)

    def step(self, theta, lam: float, opts: Optional[StepOpts] = None, out=None, stream=None):
        th = self._theta(theta)
        dth = out if out is not None else torch.empty(self.n, dtype=torch.float64,
                                                      device=self.device)
        st = StepStats()
        _check(_lib.dngd_step(self._h, _ptr(th), float(lam), C.byref(opts) if opts else None,
                              _ptr(dth), C.byref(st), _stream(stream)), allow=(OK, ENOCONV))
        return dth, st

    def iterate(self, theta: torch.Tensor, etas, lam_cap: float = 0.0, fixed_lambda: float = 0.0,
                opts: Optional[StepOpts] = None, dtheta_out=None, stream=None) -> IterStats:
        """One D-NGD workflow iteration; ``theta`` (device FP64, contiguous) is
        updated in place."""
        assert theta.dtype == torch.float64 and theta.is_contiguous() and theta.numel() == self.n
        etas = [float(e) for e in etas]
        ea = (C.c_double * len(etas))(*etas)
        st = IterStats()
        _check(_lib.dngd_iterate(self._h, _ptr(theta), float(lam_cap), float(fixed_lambda),
                                 C.byref(opts) if opts else None, len(etas), ea, _ptr(dtheta_out),
                                 C.byref(st), _stream(stream)), allow=(OK, ENOCONV))
        return st

    def nystrom_pcg(self, theta, lam, landmarks: torch.Tensor, b, tol=1e-6, maxit=500,
                    stream=None):
        th = self._theta(theta)
        bb = _dev_f64(b, self.device)
        I = landmarks.to(self.device, torch.int64).contiguous()
        x = torch.empty(self.m, dtype=torch.float64, device=self.device)
        st = StepStats()
        rc = _check(_lib.dngd_nystrom_pcg(self._h, _ptr(th), float(lam), _ptr(I), I.numel(),
                                          float(tol), int(maxit), _ptr(bb), _ptr(x), C.byref(st),
                                          _stream(stream)), allow=(OK, ENOCONV))
        return x, st, rc


def footprint_of(pde: int, widths: Sequence[int], n_int: int, n_bdy: int, n_init: int = 0,
                 opts: Optional[StepOpts] = None) -> int:
    """Device bytes a problem of this shape holds after a step with ``opts``
    (dngd_footprint_desc); host-only, allocates nothing."""
    w = (C.c_int32 * len(widths))(*[int(x) for x in widths])
    d = ProblemDesc()
    d.pde, d.n_layers, d.widths, d.kappa = pde, len(widths) - 1, w, 0.0
    d.n_int, d.n_bdy, d.n_init = int(n_int), int(n_bdy), int(n_init)
    b = C.c_size_t()
    _check(_lib.dngd_footprint_desc(C.byref(d), C.byref(opts) if opts else None, C.byref(b)))
    return int(b.value)


def gram(J: torch.Tensor, n: int, lam: float, passes: int = 1, stream=None) -> torch.Tensor:
    """K = J J^T + lam I (lower triangle; the upper is zero-filled here)."""
    m, ldJ = J.shape
    jd = F64 if J.dtype == torch.float64 else F32
    K = torch.zeros(m, m, dtype=torch.float64, device=J.device)
    _check(_lib.dngd_gram(m, n, _ptr(J), ldJ, jd, passes, float(lam), _ptr(K), m,
                          _stream(stream)))
    return K


def cholesky_solve_refine(K: torch.Tensor, B: torch.Tensor, J: torch.Tensor, n: int, lam: float,
                          sweeps: int, factored: bool = False, stream=None):
    """B <- (J J^T + lam I)^{-1} B with the Cholesky factor of K (lower
    triangle, factored in place unless ``factored``) as the inner solver and
    ``sweeps`` refinement sweeps against J (m x ldJ, FP32 or FP64). B is
    (nrhs, m) or (m,) FP64. Returns (info, rel_res) with rel_res an
    (nrhs, sweeps) array of ||b - A x|| / ||b|| per sweep."""
    m = K.shape[0]
    assert B.dtype == torch.float64 and B.is_contiguous() and J.is_contiguous()
    nrhs, ldB = (1, m) if B.dim() == 1 else (B.shape[0], B.shape[1])
    jd = F64 if J.dtype == torch.float64 else F32
    R = Refine(_ptr(J), int(n), J.shape[1], jd, int(sweeps), float(lam))
    rel = (C.c_double * max(1, nrhs * sweeps))()
    info = C.c_int64()
    rc = _lib.dngd_cholesky_solve_refine(m, _ptr(K), K.stride(0), int(factored), nrhs, _ptr(B),
                                         ldB, C.byref(R), rel, C.byref(info), _stream(stream))
    if rc == ENOTPD:
        return int(info.value), None
    _check(rc)
    return 0, np.array(rel[:nrhs * sweeps], dtype=np.float64).reshape(nrhs, sweeps)


def cholesky_solve(K: torch.Tensor, B: torch.Tensor, factored: bool = False, stream=None,
                   noalloc: bool = False):
    """Factor K (lower triangle, in place) and overwrite B (m x nrhs, column
    blocks contiguous: pass B as an (nrhs, m) tensor) with K^{-1} B.
    ``noalloc`` calls dngd_cholesky_solve_noalloc (static scratch, m <= 2048).
    Returns info (0 on success)."""
    m = K.shape[0]
    assert B.dtype == torch.float64 and B.is_contiguous()
    nrhs, ldB = (1, m) if B.dim() == 1 else (B.shape[0], B.shape[1])
    info = C.c_int64()
    fn = _lib.dngd_cholesky_solve_noalloc if noalloc else _lib.dngd_cholesky_solve
    rc = fn(m, _ptr(K), K.stride(0), int(factored), nrhs, _ptr(B), ldB, C.byref(info),
            _stream(stream))
    if rc == ENOTPD:
        return int(info.value)
    _check(rc)
    return 0
