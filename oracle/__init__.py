"""Plain FP64 CPU oracle for the unitary-Fermi-gas fermion matrix (TEST INFRASTRUCTURE).

This package is test infrastructure only. It is a slow, obviously correct
numpy implementation of what the HIP library computes, written from the paper
(Ten, Drut, Laehde, "Preconditioning the non-relativistic many-fermion
problem", arXiv:1008.3647). Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does. It shares no code with the HIP library: the only thing both sides use is
the seeded input generator module ``synthetic``.

Conventions (0-based): time slice t = 0..Ntau-1 (the paper's j = t+1), spatial
site n = (z*Nx + y)*Nx + x, vectors shaped [Ntau][Nx][Nx][Nx] complex128.

Modules
  operator : fermion matrix M, its adjoint, M1, dense builders   (Sec. 1, Eq. MatrixM)
  freefield: M0^{-1} by the antiperiodic 4D Fourier transform    (Sec. 3)
  precond  : Chebyshev (Sec. 2), weak coupling + Euler (Sec. 3, 3.1),
             strong coupling (Sec. 4)
  solvers  : CG on the normal equations, two-step BiCGStab        (Sec. 1, Eqs. 1-3)
  force    : pseudofermion action, force, leapfrog MD             (Sec. 1)
  hmc      : heat bath, HMC trajectory, Metropolis step           (Sec. 1)
  costmodel: the paper's matrix-vector cost model                 (Sec. 5)

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against something other than itself (closed forms, dense linear algebra,
the paper's printed numbers, brute force on tiny lattices).
"""
from .operator import (  # noqa: F401
    coupling_A, momenta, kinetic_symbol, transfer_matrix_1d, apply_expK,
    field_b, apply_M, apply_Mdag, apply_M1, apply_M1dag, apply_Q,
    dense_M, dense_M1, dense_expK,
)
from .freefield import apply_M0inv, apply_M0inv_dag, free_spectrum  # noqa: F401
from . import precond, solvers, force, hmc, costmodel  # noqa: F401
