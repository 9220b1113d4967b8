"""One refinement sweep through J with a diagonal inner solver
(dngd_cholesky_solve_refine; Section 4.1, the DenseDualSolve algorithm).

With K~ = diag(d) the factor is exact, x0 = D^-1 b, and one sweep gives
    x1 = x0 + D^-1 (b - J (J^T x0) - lam x0),
so x1 and the sweep's ||s0|| / ||b|| are fixed by two FP64 matrix-vector
products computed here. Any mistake in the refinement residual (a dropped
column band, a wrong row, a sign) moves x1 by O(1); rounding moves it by
about 1e-15.

The shapes cover the J^T x and J t kernels' edges: column counts that leave
a partial 4-column group and a partial 1024-column workgroup, few columns
and many rows (J^T x split over many row bands, J t with one partial group),
many columns and few rows, M = 16384 with a 2 GB K, and tiny systems. A
repeat call must agree bit for bit (the reductions run in a fixed order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
BAR = 1e-12


def D():
    from paper_2505_21404_amd import dngd
    return dngd


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# (M, N, dtype)
SHAPES = [
    (777, 8205, torch.float32),      # a 13-column tail past the last 1024-column group
    (5000, 1000, torch.float64),     # one partial column workgroup, many row bands
    (40, 16391, torch.float64),      # few rows, a 3-column tail in the last 4-column group
    (16384, 300, torch.float32),     # many rows, few columns
    (16385, 64, torch.float32),      # a single row in the last 4-row group of J t
    (1, 5, torch.float64),
    (3, 1, torch.float32),
    (130, 33, torch.float32),        # one column past a 4-column group
]


@pytest.mark.parametrize("M,N,dtype", SHAPES,
                         ids=[f"{s[0]}x{s[1]}-{'f32' if s[2] == torch.float32 else 'f64'}"
                              for s in SHAPES])
def test_one_sweep_with_diagonal_factor(M, N, dtype):
    d = D()
    say(f"case refine residual M {M} N {N} {dtype}")
    rng = np.random.default_rng(M * 7919 + N)
    J = rng.standard_normal((M, N))
    if dtype == torch.float32:
        J = J.astype(np.float32).astype(np.float64)
    ldJ = (N + 3) // 4 * 4 + 4
    Jp = np.zeros((M, ldJ))
    Jp[:, :N] = J
    lam = 0.5
    # the Jacobi diagonal of J J^T + lam I, so s0 is of the size of b
    dg = np.sum(J * J, axis=1) + lam
    b = rng.standard_normal((2, M))
    x0 = b / dg
    s0 = b - (J @ (J.T @ x0.T)).T - lam * x0
    x1 = x0 + s0 / dg
    want_res = np.linalg.norm(s0, axis=1) / np.linalg.norm(b, axis=1)

    Jt = torch.tensor(Jp, dtype=dtype, device="cuda")
    out = []
    for rep in range(2):
        K = torch.diag(torch.tensor(dg, dtype=torch.float64, device="cuda"))
        B = torch.tensor(b, device="cuda")
        info, res = d.cholesky_solve_refine(K, B, Jt, N, lam, 1)
        assert info == 0
        out.append((B.cpu().numpy(), np.asarray(res)))
        del K
    X, res = out[0]
    e = max(rel(X[j], x1[j]) for j in range(2))
    # at M = 1 the diagonal is the whole matrix and s0 is rounding only
    say(f"  x1 {e:.2e}, ||s0||/||b|| {res[:, 0]} against {want_res}")
    assert e <= BAR
    assert np.all(np.abs(res[:, 0] - want_res) <= 1e-10 * want_res + 1e-14)
    assert np.array_equal(out[0][0], out[1][0])
