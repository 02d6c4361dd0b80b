"""The ctypes binding checks every buffer it hands to the C ABI.

The library receives bare device pointers and cannot check sizes, so a
mismatched out=, x0= or y must be rejected in Python before any library call:
each case below runs with the lattice's library handle replaced by a tripwire
that fails the test if it is touched. Correct buffers passed through out= and
x0= must give the same results as library-allocated ones.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.force  # noqa: F401
from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, to_dev, to_host, rel_err, TAU, G

pytestmark = pytest.mark.gpu


class Tripwire:
    def __getattr__(self, name):
        raise AssertionError(f"library function {name} called with an invalid buffer")


def _lattice(dtype=torch.complex128, nx=4, ntau=6):
    from paper_1008_3647_amd import Lattice
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma_field(nx, ntau, 880)))
    return L


def _rejects(L, exc, fn):
    lib = L._lib
    L._lib = Tripwire()
    try:
        with pytest.raises(exc):
            fn()
    finally:
        L._lib = lib


def test_operator_out_buffers_are_checked():
    require_gpu()
    from paper_1008_3647_amd import Precond
    L = _lattice()
    x = to_dev(gaussian_rhs(4, 6, [881, 882]))
    for apply in (L.apply_M, L.apply_Mdag):
        _rejects(L, TypeError, lambda: apply(x, out=torch.empty_like(x, dtype=torch.complex64)))
        _rejects(L, ValueError, lambda: apply(x, out=torch.empty_like(x[:1])))
        _rejects(L, ValueError, lambda: apply(x, out=torch.empty((2, 6, 4, 4, 8),
                                                                 dtype=x.dtype,
                                                                 device=x.device)[..., ::2]))
        _rejects(L, ValueError, lambda: apply(x, out=x))
        _rejects(L, TypeError, lambda: apply(x, out=torch.empty(x.shape, dtype=x.dtype)))
    pc = Precond("wce", wce_order=1)
    _rejects(L, ValueError, lambda: L.apply_precond(x, pc, "M", out=torch.empty_like(x[:1])))
    _rejects(L, TypeError, lambda: L.apply_precond(x, pc, "M",
                                                   out=torch.empty_like(x, dtype=torch.complex64)))
    _rejects(L, ValueError, lambda: L.apply_precond(x, pc, "X"))
    # valid out= buffers give the library-allocated results
    y = torch.empty_like(x)
    assert torch.equal(L.apply_M(x, out=y), L.apply_M(x))
    assert torch.equal(L.apply_precond(x, pc, "M", out=y), L.apply_precond(x, pc, "M"))


def test_solve_x0_is_checked():
    require_gpu()
    L = _lattice()
    b = to_dev(gaussian_rhs(4, 6, [883, 884]))
    # mixed solves write complex128 into x0: a complex64 x0 must be refused
    _rejects(L, TypeError, lambda: L.solve_bicgstab(b, "two_step", mixed=True,
                                                     x0=torch.zeros_like(b, dtype=torch.complex64)))
    _rejects(L, ValueError, lambda: L.solve_bicgstab(b, "M", x0=torch.zeros_like(b[:1])))
    _rejects(L, ValueError, lambda: L.solve_cg_normal(b, x0=torch.zeros_like(b[:1])))
    _rejects(L, ValueError, lambda: L.solve_bicgstab(b, "two_step", x0=b))
    _rejects(L, ValueError, lambda: L.solve_bicgstab(b, "bogus"))
    # a valid x0 (here the solution itself) is used as the starting vector
    x, st = L.solve_bicgstab(b, "M", tol=1e-12)
    x1, st1 = L.solve_bicgstab(b, "M", tol=1e-12, x0=x.clone())
    assert st1["iters"][0] <= 1
    assert rel_err(to_host(x1), to_host(x)) < 1e-10


def test_force_buffers_are_checked():
    require_gpu()
    L = _lattice()
    sigma = sigma_field(4, 6, 880)
    X = to_dev(gaussian_rhs(4, 6, [885, 886]))
    y = L.apply_M(X)
    _rejects(L, ValueError, lambda: L.force_dS_dsigma(X, y[:1]))
    _rejects(L, TypeError, lambda: L.force_dS_dsigma(X, y.to(torch.complex64)))
    _rejects(L, TypeError, lambda: L.force_dS_dsigma(
        X, y, out=torch.empty(L.shape, dtype=torch.float32, device=X.device)))
    _rejects(L, ValueError, lambda: L.force_dS_dsigma(
        X, y, out=torch.empty((6, 4, 4, 3), dtype=torch.float64, device=X.device)))
    g = torch.empty(L.shape, dtype=torch.float64, device=X.device)
    got = to_host(L.force_dS_dsigma(X, y, out=g))
    # y = M X here, so the sum of the oracle's per-rhs gradients is the reference
    ref = sum(oracle.force.gradient(to_host(X)[k], sigma, TAU, G) for k in range(2))
    assert rel_err(got, ref) < 1e-12
    assert np.array_equal(got, to_host(L.force_dS_dsigma(X, y)))


def test_empty_batches_are_rejected():
    """A batch of zero right-hand sides is an error raised in Python (the C
    ABI takes nrhs >= 1), for the operator, the preconditioners, the solvers,
    the norm, the force and the HMC calls."""
    require_gpu()
    from paper_1008_3647_amd import Precond
    L = _lattice()
    e = torch.empty((0,) + L.shape, dtype=L.dtype, device="cuda")
    s = to_dev(sigma_field(4, 6, 880))
    pi = torch.zeros(L.shape, dtype=torch.float64, device="cuda")
    for fn in (lambda: L.apply_M(e), lambda: L.apply_Mdag(e),
               lambda: L.apply_precond(e, Precond("wce", wce_order=1), "M"),
               lambda: L.solve_bicgstab(e, "M"), lambda: L.solve_cg_normal(e),
               lambda: L.norm2(e), lambda: L.force_dS_dsigma(e, e),
               lambda: L.hmc_trajectory(s, pi, e, 0.5, 0.1, 2)):
        _rejects(L, ValueError, fn)
