"""Parity of the preconditioners (apply_precond through the C ABI) with the oracle.

  SCA (Sec. 4): (L^dagger D L)^{-1} for alpha in {1, 1.5}
  WCE (Sec. 3, 3.1): W_d and W_d^T, d in {0, 1, 2, 4}, plain and Euler weights;
      W_d W_d^T for the CG (op Q) form
  Chebyshev (Sec. 2): P(Q/lam_max), degrees 8 and 16, bit-reversal order, and
      the BiCGStab extension P M^T / M P.
Tolerances (element-wise, relative to the largest output): complex128 1e-12
(WCE and Chebyshev chain up to 2d+2 operator applications), complex64 2e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import precond as pc
from synthetic import sigma_field, gaussian_rhs
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-12, torch.complex64: 2e-5}
SHAPES = [(4, 12, 2), (6, 9, 1), (8, 20, 3), (12, 7, 2), (16, 5, 1)]


def _setup(nx, ntau, nrhs, dtype, seed):
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(nx, ntau, seed)
    x = gaussian_rhs(nx, ntau, range(seed + 1, seed + 1 + nrhs))
    if dtype == torch.complex64:
        x = x.astype(np.complex64).astype(np.complex128)
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    return L, sigma, x, to_dev(x, dtype)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx,ntau,nrhs", SHAPES)
@pytest.mark.parametrize("alpha", [1.0, 1.5])
def test_sca(nx, ntau, nrhs, dtype, alpha):
    require_gpu()
    from paper_1008_3647_amd import Precond
    say(f"sca nx={nx} ntau={ntau} alpha={alpha} {dtype}")
    L, sigma, x, xd = _setup(nx, ntau, nrhs, dtype, 500)
    y = to_host(L.apply_precond(xd, Precond("sca", alpha=alpha), "Q"))
    D, Lb = pc.sca_setup(sigma, TAU, G, alpha)
    ref = np.stack([pc.sca_apply(xi, D, Lb) for xi in x])
    assert rel_err(y, ref) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx,ntau,nrhs", SHAPES)
@pytest.mark.parametrize("order,euler", [(0, False), (1, False), (2, False), (2, True), (4, True)])
def test_wce(nx, ntau, nrhs, dtype, order, euler):
    require_gpu()
    from paper_1008_3647_amd import Precond
    say(f"wce nx={nx} ntau={ntau} d={order} euler={euler} {dtype}")
    L, sigma, x, xd = _setup(nx, ntau, nrhs, dtype, 600)
    p = Precond("wce", wce_order=order, euler=euler)
    yM = to_host(L.apply_precond(xd, p, "M"))
    yT = to_host(L.apply_precond(xd, p, "Mdag"))
    refM = np.stack([pc.wce_apply(xi, sigma, TAU, G, order, euler) for xi in x])
    refT = np.stack([pc.wce_apply_dag(xi, sigma, TAU, G, order, euler) for xi in x])
    assert rel_err(yM, refM) < TOL[dtype]
    assert rel_err(yT, refT) < TOL[dtype]
    if order == 2 and dtype == torch.complex128:
        yQ = to_host(L.apply_precond(xd, p, "Q"))
        refQ = np.stack([pc.wce_apply(pc.wce_apply_dag(xi, sigma, TAU, G, order, euler),
                                      sigma, TAU, G, order, euler) for xi in x])
        assert rel_err(yQ, refQ) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx,ntau,nrhs", [(8, 16, 2), (8, 100, 2), (4, 333, 2), (4, 600, 2),
                                          (16, 40, 2), (16, 24, 4)])
def test_m0_inverse_on_device(nx, ntau, nrhs, dtype):
    """WCE of order 0 is M0^{-1}; M0 (g = 0) undoes it. The temporal solve
    splits each mode's time line into 8 chunks (here of 2, 13, 42 with a last
    one of 39, 75, 5 and 3 slices), 64 modes per workgroup.

    complex64 bound: the round trip chains nine 16-term line sums (U^T and U
    per axis around the temporal solve, then T per axis in M0), each with a
    rounding error of about sqrt(16) u relative to the largest entry for random
    signs (u = 2^-24), i.e. sqrt(9 * 16) u = 12 u, plus the first-order
    recurrence (|lam| <= 1, one rounding per slice, damped by 1 - lam except
    for the zero mode, whose antiperiodic sum cancels in M0); 2e-6 = 34 u
    leaves a factor ~3 on that estimate (measured 2.8e-7 to 5.4e-7 for Ntau
    from 16 to 600)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    say(f"m0 inverse nx={nx} ntau={ntau} nrhs={nrhs} {dtype}")
    x = gaussian_rhs(nx, ntau, range(650, 650 + nrhs))
    L0 = Lattice(nx, ntau, TAU, 0.0, dtype)
    xd = to_dev(x, dtype)
    tol = 1e-13 if dtype == torch.complex128 else 2e-6
    u = L0.apply_precond(xd, Precond("wce", wce_order=0), "M")
    back = to_host(L0.apply_M(u))
    e1 = rel_err(back, to_host(xd))
    ut = L0.apply_precond(xd, Precond("wce", wce_order=0), "Mdag")
    e2 = rel_err(to_host(L0.apply_Mdag(ut)), to_host(xd))
    say(f"m0 round trip nx={nx} ntau={ntau} {dtype}: {e1:.2e} {e2:.2e} (tol {tol:.1e})")
    assert e1 < tol and e2 < tol


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("degree", [8, 16])
def test_chebyshev(dtype, degree):
    require_gpu()
    from paper_1008_3647_amd import Precond
    nx, ntau, nrhs = 6, 10, 2
    say(f"cheb degree={degree} {dtype}")
    L, sigma, x, xd = _setup(nx, ntau, nrhs, dtype, 700)
    lam_max, eps = 7.0, 1e-2
    p = Precond("cheb", degree=degree, eps=eps, lam_max=lam_max)
    yQ = to_host(L.apply_precond(xd, p, "Q"))
    refQ = np.stack([pc.apply_cheb(xi, sigma, TAU, G, degree, eps, lam_max) for xi in x])
    tol = TOL[dtype] * (10 if dtype == torch.complex64 else 1)
    assert rel_err(yQ, refQ) < tol
    if dtype == torch.complex128:
        yM = to_host(L.apply_precond(xd, p, "M"))
        refM = np.stack([pc.apply_cheb(oracle.apply_Mdag(xi, sigma, TAU, G), sigma, TAU, G,
                                       degree, eps, lam_max) for xi in x])
        assert rel_err(yM, refM) < tol
        yT = to_host(L.apply_precond(xd, p, "Mdag"))
        refT = np.stack([oracle.apply_M(pc.apply_cheb(xi, sigma, TAU, G, degree, eps, lam_max),
                                        sigma, TAU, G) for xi in x])
        assert rel_err(yT, refT) < tol


def test_chebyshev_lam_max_estimates():
    """lam_max = 0 uses the bound (1 + max|b|)^2 >= ||Q|| exactly; lam_max < 0
    estimates it by power iteration, and PCG with it must still converge."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    from oracle import operator as op
    nx, ntau = 2, 8
    sigma = sigma_field(nx, ntau, 710)
    Md = op.dense_M(sigma, TAU, G)
    lam_true = np.linalg.eigvalsh(Md.T @ Md)[-1]
    b = oracle.field_b(sigma, oracle.coupling_A(TAU, G))
    bound = (1 + np.abs(b).max()) ** 2
    assert bound >= lam_true
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    x = gaussian_rhs(nx, ntau, [711])
    xd = to_dev(x)
    y = to_host(L.apply_precond(xd, Precond("cheb", degree=8, eps=1e-2, lam_max=0.0), "Q"))
    assert rel_err(y, pc.apply_cheb(x[0], sigma, TAU, G, 8, 1e-2, bound)[None]) < 1e-12
    sol, st = L.solve_cg_normal(xd, Precond("cheb", degree=8, eps=1e-2, lam_max=-1.0), tol=1e-10)
    assert st["status"] == 0 and st["relres"][0] <= 1e-10


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_chebyshev_degree32_streaming_nx16(dtype):
    """Degree 32 (the paper's largest) on an Nx = 16 lattice, where every
    factor runs on the streaming operator, element-wise against the oracle:
    P(Q^) and the BiCGStab extensions P M^T and M P. The constant is spread
    over the 32 factors, so the tolerance is that of degree 8 and 16 times two
    (twice the chained operator applications)."""
    require_gpu()
    from paper_1008_3647_amd import Precond
    nx, ntau, nrhs = 16, 4, 2
    say(f"cheb degree=32 nx=16 {dtype}")
    L, sigma, x, xd = _setup(nx, ntau, nrhs, dtype, 720)
    lam_max, eps = 6.5, 2e-3
    p = Precond("cheb", degree=32, eps=eps, lam_max=lam_max)
    tol = 2 * TOL[dtype] * (10 if dtype == torch.complex64 else 1)
    yQ = to_host(L.apply_precond(xd, p, "Q"))
    refQ = np.stack([pc.apply_cheb(xi, sigma, TAU, G, 32, eps, lam_max) for xi in x])
    assert rel_err(yQ, refQ) < tol
    yM = to_host(L.apply_precond(xd, p, "M"))
    refM = np.stack([pc.apply_cheb(oracle.apply_Mdag(xi, sigma, TAU, G), sigma, TAU, G,
                                   32, eps, lam_max) for xi in x])
    assert rel_err(yM, refM) < tol
    yT = to_host(L.apply_precond(xd, p, "Mdag"))
    refT = np.stack([oracle.apply_M(pc.apply_cheb(xi, sigma, TAU, G, 32, eps, lam_max),
                                    sigma, TAU, G) for xi in x])
    assert rel_err(yT, refT) < tol


@pytest.mark.parametrize("nx,ntau", [(2, 8), (4, 6), (4, 10)])
def test_power_iteration_lam_max_against_dense_spectrum(nx, ntau):
    """The power-iteration estimate (lam_max < 0) must bound the largest
    eigenvalue of Q = M^T M from above by at most its 5 % safety factor:
    lam_true <= estimate <= 1.05 lam_true (dense eigvalsh of Q); the
    preconditioner built with it matches the oracle's with the same lam_max at
    degree 32."""
    require_gpu()
    from paper_1008_3647_amd import Precond
    from oracle import operator as op
    L, sigma, x, xd = _setup(nx, ntau, 1, torch.complex128, 730 + nx + ntau)
    Md = op.dense_M(sigma, TAU, G)
    lam_true = np.linalg.eigvalsh(Md.T @ Md)[-1]
    p = Precond("cheb", degree=32, eps=1e-3, lam_max=-1.0)
    est = L.lam_max(p)
    say(f"{nx}^3 x {ntau}: lam_max dense {lam_true:.6f}, power iteration x 1.05 {est:.6f}")
    assert lam_true <= est <= 1.05 * lam_true * (1 + 1e-12)
    y = to_host(L.apply_precond(xd, p, "Q"))
    ref = pc.apply_cheb(x[0], sigma, TAU, G, 32, 1e-3, est)[None]
    assert rel_err(y, ref) < 2e-12


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx,ntau,nrhs", [(4, 12, 2), (8, 20, 1), (16, 5, 2)])
def test_sca_chebyshev_filter(nx, ntau, nrhs, dtype):
    """SCA with the Chebyshev filter (Sec. 4, closing remark): P_2n(S Q /
    lam_max) S element-wise against the oracle, for Q and (complex128) the
    BiCGStab extensions P M^T and M P; tolerance as for degree 8 Chebyshev
    (the SCA sweeps are first-order recurrences like those of M0^{-1})."""
    require_gpu()
    from paper_1008_3647_amd import Precond
    say(f"sca+cheb nx={nx} ntau={ntau} {dtype}")
    L, sigma, x, xd = _setup(nx, ntau, nrhs, dtype, 760)
    lam_max, eps, alpha = 3.0, 1e-2, 1.5
    p = Precond("sca_cheb", degree=8, eps=eps, lam_max=lam_max, alpha=alpha)
    tol = TOL[dtype] * (10 if dtype == torch.complex64 else 1)
    y = to_host(L.apply_precond(xd, p, "Q"))
    ref = np.stack([pc.apply_sca_cheb(xi, sigma, TAU, G, 8, eps, lam_max, alpha) for xi in x])
    assert rel_err(y, ref) < tol
    if dtype == torch.complex128:
        yM = to_host(L.apply_precond(xd, p, "M"))
        refM = np.stack([pc.apply_sca_cheb(oracle.apply_Mdag(xi, sigma, TAU, G), sigma, TAU, G,
                                           8, eps, lam_max, alpha) for xi in x])
        assert rel_err(yM, refM) < tol


def test_sca_chebyshev_lam_max_against_dense_spectrum():
    """lam_max < 0 estimates the largest eigenvalue of S Q by power iteration:
    lam_true <= estimate <= 1.05 lam_true, lam_true from the dense Hermitian
    S^{1/2} Q S^{1/2}."""
    require_gpu()
    from paper_1008_3647_amd import Precond
    from oracle import operator as op
    nx, ntau, alpha = 2, 8, 1.5
    L, sigma, x, xd = _setup(nx, ntau, 1, torch.complex128, 770)
    V, N = nx ** 3, nx ** 3 * ntau
    D, Lb = pc.sca_setup(sigma, TAU, G, alpha)
    S = np.zeros((N, N))
    for n in range(V):
        iz, iy, ix = np.unravel_index(n, (nx, nx, nx))
        Ld, Dd = pc.sca_dense_factors(D[:, iz, iy, ix], Lb[:, iz, iy, ix])
        idx = np.arange(ntau) * V + n
        S[np.ix_(idx, idx)] = np.linalg.inv(Ld @ Dd @ Ld.T)
    w, U = np.linalg.eigh(S)
    Sh = (U * np.sqrt(w)) @ U.T
    Md = op.dense_M(sigma, TAU, G)
    lam_true = np.linalg.eigvalsh(Sh @ (Md.T @ Md) @ Sh)[-1]
    est = L.lam_max(Precond("sca_cheb", degree=8, eps=1e-2, lam_max=-1.0, alpha=alpha))
    say(f"S Q: lam_max dense {lam_true:.6f}, power iteration x 1.05 {est:.6f}")
    assert lam_true <= est <= 1.05 * lam_true * (1 + 1e-12)
