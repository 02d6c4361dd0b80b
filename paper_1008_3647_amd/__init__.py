"""MI355X (gfx950) library for the unitary-Fermi-gas fermion matrix and its
preconditioned Krylov solvers (Ten, Drut, Laehde, arXiv:1008.3647).

The computation lives in libufg.so (HIP, C ABI in include/ufg.h); this package
is the Python binding: `Lattice` wraps a handle and marshals torch tensors,
`Action` is the pseudofermion action as a torch.autograd.Function.
"""
from .lattice import Lattice, Precond, UfgError  # noqa: F401
from . import _lib  # noqa: F401

__all__ = ["Lattice", "Precond", "UfgError"]
