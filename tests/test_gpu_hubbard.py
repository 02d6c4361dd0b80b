"""The Hubbard-model dispersion (E = sum_i 1 - cos k_i, the extension named in
the paper's concluding section) through the C ABI (create_lattice_ex) against
the oracle with the same dispersion: both operators on the streaming (Nx = 8,
12, 16) and general (Nx = 4, 6) paths, preconditioned solves against dense LU,
the force contraction, and a batched solve mixing both dispersions.
Tolerances as for the free dispersion: 1e-13 (complex128) / 5e-6 (complex64)
relative to the largest output for the operators."""
import numpy as np
import pytest
import torch

import oracle
from oracle import operator as op
from oracle import solvers as osol
from oracle import force as oforce
from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu
H = "hubbard"


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 5e-6)])
@pytest.mark.parametrize("nx,ntau,nrhs", [(4, 7, 2), (6, 5, 1), (8, 9, 2), (12, 4, 1), (16, 5, 2)])
def test_operators_match_oracle(nx, ntau, nrhs, dtype, tol):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(nx, ntau, 950 + nx)
    x = gaussian_rhs(nx, ntau, range(960, 960 + nrhs))
    L = Lattice(nx, ntau, TAU, G, dtype, dispersion=H)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x, dtype)
    xr = to_host(xd).astype(np.complex128)
    y = to_host(L.apply_M(xd))
    yd = to_host(L.apply_Mdag(xd))
    for k in range(nrhs):
        assert rel_err(y[k], oracle.apply_M(xr[k], sigma, TAU, G, H)) < tol
        assert rel_err(yd[k], oracle.apply_Mdag(xr[k], sigma, TAU, G, H)) < tol
    # and it is not the free operator
    free = oracle.apply_M(xr[0], sigma, TAU, G)
    assert rel_err(y[0], free) > 1e-4


@pytest.mark.parametrize("nx", [4, 8])
def test_preconditioned_solves_match_dense_lu(nx):
    """WCE2 two-step BiCGStab (M0^{-1} through the eigenbasis of the Hubbard T)
    and Chebyshev CG reach the dense-LU solution of the Hubbard M."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    ntau = 8
    sigma = sigma_field(nx, ntau, 970 + nx)
    b = gaussian_rhs(nx, ntau, [971])
    L = Lattice(nx, ntau, TAU, G, torch.complex128, dispersion=H)
    L.set_aux_field(to_dev(sigma))
    Md = op.dense_M(sigma, TAU, G, H)
    ref = osol.dense_two_step(Md, b[0].ravel()).reshape(b[0].shape)
    x, st = L.solve_bicgstab(to_dev(b), "two_step", Precond("wce", wce_order=2), tol=1e-12)
    say(f"hubbard {nx}^3 x {ntau} WCE2: {st['iters']}")
    assert st["status"] == 0
    assert np.linalg.norm(to_host(x)[0] - ref) / np.linalg.norm(ref) < 1e-9
    x, st = L.solve_cg_normal(to_dev(b), Precond("cheb", degree=8, eps=1e-2, lam_max=-1.0),
                              tol=1e-12, maxit=5000)
    say(f"hubbard {nx}^3 x {ntau} Cheb8 CG: {st['iters']}")
    assert st["status"] == 0
    assert np.linalg.norm(to_host(x)[0] - ref) / np.linalg.norm(ref) < 1e-8


def test_force_matches_oracle():
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau = 8, 6
    sigma = sigma_field(nx, ntau, 980)
    X = gaussian_rhs(nx, ntau, [981, 982])
    y = np.stack([oracle.apply_M(Xi, sigma, TAU, G, H) for Xi in X])
    L = Lattice(nx, ntau, TAU, G, torch.complex128, dispersion=H)
    L.set_aux_field(to_dev(sigma))
    g = to_host(L.force_dS_dsigma(to_dev(X), to_dev(y)))
    ref = sum(oforce.gradient(Xi, sigma, TAU, G, H) for Xi in X)
    assert rel_err(g, ref) < 1e-12


def test_batched_mixes_dispersions():
    """One batched call over a free and a Hubbard lattice of the same size: each
    system reaches its own dense-LU solution (the two T factors form separate
    operator classes)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.lattice import solve_batched
    nx, ntau = 4, 9
    lats, bs, refs = [], [], []
    for i, disp in enumerate(("free", H)):
        sigma = sigma_field(nx, ntau, 990 + i)
        b = gaussian_rhs(nx, ntau, [995 + i])
        L = Lattice(nx, ntau, TAU, G, torch.complex128, dispersion=disp)
        L.set_aux_field(to_dev(sigma))
        lats.append(L)
        bs.append(to_dev(b))
        Md = op.dense_M(sigma, TAU, G, disp)
        refs.append(osol.dense_two_step(Md, b[0].ravel()).reshape(b[0].shape))
    xs, st = solve_batched(lats, bs, tol=1e-11, mixed=False)
    for x, s, ref in zip(xs, st, refs):
        assert s["status"] == 0
        assert np.linalg.norm(to_host(x)[0] - ref) / np.linalg.norm(ref) < 1e-8
