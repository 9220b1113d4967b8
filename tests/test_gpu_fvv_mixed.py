"""f_vv inside the mixed step (Section 3.2): the hidden layers' tangent
products run in FP32 on the matrix cores (FP64 operands rounded to FP32, FP32
accumulation, FP64 jet rules). Checked against the oracle's f_vv along the
step's own v on ragged shapes (jet rows not a multiple of the 128-row tile,
widths not multiples of 16, one to three hidden layers, Poisson and heat),
and at the 5-D Poisson workload (m = 5000) against the FP64 dngd_fvv along
the same v.

FP32 rounding of the operands and FP32 sums over K <= 1024 terms put the
layer products within about 1e-6 of FP64; 1e-5 still fails any indexing or
segment mistake, which gives O(1) errors."""
import numpy as np
import pytest

import workloads as W
from oracle import network as N

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
BAR = 1e-5


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def mixed_fvv(prob, th, lam):
    """(v, f_vv) of one mixed step with GA: v is the step without GA (the
    same v the GA step computes), f_vv the step's own fvv_out."""
    d = D()
    v, _ = prob.step(th, lam, d.step_opts(precision=d.MIXED, ga=False))
    f = torch.empty(prob.m, dtype=torch.float64, device="cuda")
    prob.step(th, lam, d.step_opts(precision=d.MIXED, ga=True, fvv_out=f))
    return v, f


SHAPES = [
    ("poisson5d-40-24", lambda: W.config(1, scale=dict(widths=[5, 40, 24, 1], n_int=150,
                                                       n_bdy=47)), 1e-4),
    ("heat-48-33-20", lambda: W.config(2, scale=dict(widths=[3, 48, 33, 20, 1], n_int=131,
                                                     n_bdy=40, n_init=29)), 1e-3),
    ("poisson2d-3x64", lambda: W.config(0, scale=dict(widths=[2, 64, 64, 64, 1], n_int=300,
                                                      n_bdy=100)), 1e-4),
]


@pytest.mark.parametrize("name,make,lam", SHAPES, ids=[s[0] for s in SHAPES])
def test_mixed_step_fvv_against_oracle(name, make, lam):
    d = D()
    p = make()
    th = W.glorot_theta(p.widths, 2)
    say("case mixed f_vv", name, "m", p.m, "n", p.n_params)
    prob = d.Problem.from_workload(p)
    v, f = mixed_fvv(prob, th, lam)
    v64 = v.cpu().numpy()
    ref = N.fvv(p, th, v64)
    e = rel(f.cpu().numpy(), ref)
    e64 = rel(prob.fvv(th, v).cpu().numpy(), ref)
    say(f"  mixed step f_vv {e:.2e}, FP64 dngd_fvv {e64:.2e}")
    assert e64 <= 1e-11
    assert e <= BAR
    prob.close()


def test_mixed_step_fvv_5d_poisson_m5000():
    d = D()
    p = W.config(1)
    th = torch.tensor(W.glorot_theta(p.widths, 0), device="cuda")
    say("case mixed f_vv 5-D Poisson m", p.m)
    prob = d.Problem.from_workload(p)
    v, f = mixed_fvv(prob, th, 1e-5)
    f64 = prob.fvv(th, v)
    e = rel(f.cpu().numpy(), f64.cpu().numpy())
    say(f"  mixed step f_vv vs FP64 dngd_fvv {e:.2e}")
    assert e <= BAR
    prob.close()
