"""Plain FP64 CPU oracle of the Dual Natural Gradient Descent (D-NGD) step.

TEST INFRASTRUCTURE ONLY. This package is the slow, obviously correct
reference that the GPU path is checked against. Only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may import it;
the product path never does, and it shares no code with the HIP library (both
sides read the same seeded inputs from ``workloads`` and nothing else).

Contents (each function cites the paper passage it follows):
  network  -- tanh-MLP forward jets (value, input gradient, input Laplacian),
              residual map r, Jacobian J (hand-written reverse mode), f_vv
              (nested t-jets), line-search losses.
  step     -- residual Gramian, dense dual solve, velocity and geodesic
              acceleration (dense dual solver of Section 4.1), primal solve,
              the paper's literal recovery formulas, the D-NGD workflow.
  nystrom  -- Nystrom construction, spectral preconditioner, PCG
              (Section 3.3 and Section 4.2).

Parity pins: every function is pinned in ``tests/test_oracle_*.py`` against
something other than itself (closed forms, complex-step and finite-difference
derivatives, a library AD, the primal normal equations, textbook identities).
"""
from . import network, step, nystrom  # noqa: F401
