"""The allocation-free Cholesky entry point (dngd_cholesky_solve_noalloc)
against dngd_cholesky_solve: same kernels, so the factors and solutions must
agree bit for bit. Two calls in a row with the second smaller, the largest
accepted size, a failing pivot followed by a good call (nothing carries over
in the shared static scratch), and a pre-factored solve."""
import numpy as np
import pytest
import torch

from paper_2505_21404_amd import dngd as D

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _spd(m, seed, shift=1e-3):
    """Seeded SPD matrix J J^T / k + shift I (a Gram matrix like the step's)."""
    rng = np.random.default_rng(seed)
    k = m + 37
    A = rng.standard_normal((m, k))
    return A @ A.T / k + shift * np.eye(m)


def _rhs(m, nrhs, seed):
    return np.random.default_rng(seed + 1).standard_normal((nrhs, m))


def _both(Kh, Bh, factored=False, Lh=None):
    """(info, L, X) from both entry points on copies of the same inputs."""
    out = []
    for noalloc in (False, True):
        K = torch.tensor(Lh if factored else Kh, device=DEV)
        B = torch.tensor(Bh, device=DEV).contiguous()
        info = D.cholesky_solve(K, B, factored=factored, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append((info, torch.tril(K).cpu().numpy(), B.cpu().numpy()))
    return out


@pytest.mark.parametrize("sizes", [(1500, 700), (2048, 130)])
def test_noalloc_matches_allocating_entry_point_two_calls(sizes):
    for call, m in enumerate(sizes):
        print(f"noalloc call {call}: m={m}", flush=True)
        Kh, Bh = _spd(m, seed=10 + m), _rhs(m, 3 - call, seed=10 + m)
        (i0, L0, X0), (i1, L1, X1) = _both(Kh, Bh)
        assert i0 == 0 and i1 == 0
        assert np.array_equal(L0, L1), f"factor differs at m={m}"
        assert np.array_equal(X0, X1), f"solution differs at m={m}"
        # and the solution solves the system (FP64 backward error)
        for j in range(Bh.shape[0]):
            r = Kh @ X1[j] - Bh[j]
            be = np.linalg.norm(r) / (np.linalg.norm(Kh, 2) * np.linalg.norm(X1[j])
                                      + np.linalg.norm(Bh[j]))
            assert be <= 1e-14, (m, j, be)


def test_noalloc_failing_pivot_then_good_call():
    m = 300
    Kh = _spd(m, seed=3)
    Kh[200, 200] = -1.0  # the leading minor of order 201 is indefinite
    Bh = _rhs(m, 1, seed=3)
    (i0, _, _), (i1, _, _) = _both(Kh, Bh)
    assert i0 == i1 and i1 > 0, (i0, i1)
    # the next call on the same scratch starts from a cleared info word
    Kg = _spd(257, seed=4)
    Bg = _rhs(257, 2, seed=4)
    (j0, L0, X0), (j1, L1, X1) = _both(Kg, Bg)
    assert j0 == 0 and j1 == 0
    assert np.array_equal(X0, X1)


def test_noalloc_prefactored_solve():
    m = 1100
    Kh, Bh = _spd(m, seed=5), _rhs(m, 2, seed=5)
    (_, L0, _), _ = _both(Kh, Bh)
    (i0, _, X0), (i1, _, X1) = _both(Kh, Bh, factored=True, Lh=L0)
    assert i0 == 0 and i1 == 0
    assert np.array_equal(X0, X1)


def test_noalloc_rejects_sizes_beyond_the_static_scratch():
    m = 2049
    K = torch.zeros(m, m, dtype=torch.float64, device=DEV)
    B = torch.ones(m, dtype=torch.float64, device=DEV)
    with pytest.raises(D.DngdError) as e:
        D.cholesky_solve(K, B, noalloc=True)
    assert e.value.status == D.EINVAL and "2048" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(B == 1.0)
