"""CPU oracle for hierarchical multicontinuum homogenization (arXiv 2503.01276).

TEST INFRASTRUCTURE ONLY. This package is the independent FP64 reference that
the HIP path is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.

It is a plain assembled method: per cell, sparse Q1 assembly, Galerkin
restriction to the level-n space, and a SuperLU factorization of the KKT
matrix with one step of iterative refinement (cells.py); Algorithm 1 over the
macropoint hierarchy and the adjoint gradient (driver.py); the hierarchy of
macrogrids (hierarchy.py); element-level finite-element pieces (fem.py).

Pins: every function is checked in tests/test_oracle_*.py against closed forms,
exact invariances, the paper's worked hierarchy example, brute-force dense
solves and finite-difference / complex-step derivatives. Absolute values of
the effective tensors on the synthetic presets have no independent pin beyond
those checks ("parity unpinned" for the numbers themselves).
"""
from .driver import Forward, backward, forward, stack_A  # noqa: F401
