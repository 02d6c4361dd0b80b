"""Lattices of spatial dimension 1 and 2 (create_lattice_dim) through the C ABI
against the oracle: the operator element by element (both dispersions, both
precisions, odd slice counts per workgroup and a ragged last workgroup), the
preconditioners, the solvers (BiCGStab, CG with every preconditioner and
split-preconditioned CG: dense LU on tiny lattices, the oracle's residual
elsewhere), the force, and a short HMC chain.

Tolerances as for three dimensions: operators 1e-13 (complex128) / 5e-6
(complex64), preconditioners 1e-12 / 2e-5, relative to the largest output
entry. A lower-dimensional slice is one or two 1D transforms of at most 16
terms, so the three-dimensional bounds hold a fortiori.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import force as fo
from oracle import hmc
from oracle import operator as op
from oracle import precond as pc
from synthetic import sigma_field, gaussian_rhs, gaussian_momenta, uniform_draws
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu

TOL_OP = {torch.complex128: 1e-13, torch.complex64: 5e-6}
TOL_PC = {torch.complex128: 1e-12, torch.complex64: 2e-5}

# (dim, nx, ntau): 1D slices of 16 sites (16 slices per workgroup, ntau = 37
# leaves a ragged last workgroup), 2D slices of 36 sites (7 slices per
# workgroup, 4 idle threads) and of 256 sites (one slice per workgroup)
SHAPES = [(1, 16, 37), (1, 2, 5), (1, 6, 12), (2, 6, 11), (2, 16, 9), (2, 2, 4), (2, 10, 5)]


def _lattice(dim, nx, ntau, dtype, g=G, disp="free", seed=800):
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(nx, ntau, seed, dim)
    L = Lattice(nx, ntau, TAU, g, dtype, dispersion=disp, dim=dim)
    L.set_aux_field(to_dev(sigma))
    return L, sigma


def _rhs(dim, nx, ntau, seeds, dtype):
    x = gaussian_rhs(nx, ntau, seeds, dim)
    if dtype == torch.complex64:
        x = x.astype(np.complex64).astype(np.complex128)
    return x, to_dev(x, dtype)


@pytest.mark.parametrize("disp", ["free", "hubbard"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("dim,nx,ntau", SHAPES)
def test_operator(dim, nx, ntau, dtype, disp):
    require_gpu()
    say(f"lowdim operator dim={dim} nx={nx} ntau={ntau} {dtype} {disp}")
    L, sigma = _lattice(dim, nx, ntau, dtype, disp=disp)
    assert L.shape == (ntau,) + (nx,) * dim
    x, xd = _rhs(dim, nx, ntau, [801, 802, 803], dtype)
    y = to_host(L.apply_M(xd))
    yd = to_host(L.apply_Mdag(xd))
    for k in range(3):
        assert rel_err(y[k], oracle.apply_M(x[k], sigma, TAU, G, disp)) < TOL_OP[dtype], k
        assert rel_err(yd[k], oracle.apply_Mdag(x[k], sigma, TAU, G, disp)) < TOL_OP[dtype], k


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("dim,nx,ntau", [(1, 8, 20), (2, 6, 11), (2, 16, 6)])
def test_preconditioners(dim, nx, ntau, dtype):
    require_gpu()
    from paper_1008_3647_amd import Precond
    say(f"lowdim preconditioners dim={dim} nx={nx} ntau={ntau} {dtype}")
    L, sigma = _lattice(dim, nx, ntau, dtype, seed=810)
    x, xd = _rhs(dim, nx, ntau, [811, 812], dtype)
    tol = TOL_PC[dtype]
    for order, euler in ((0, False), (2, False), (2, True)):
        p = Precond("wce", wce_order=order, euler=euler)
        yM = to_host(L.apply_precond(xd, p, "M"))
        yT = to_host(L.apply_precond(xd, p, "Mdag"))
        for k in range(2):
            assert rel_err(yM[k], pc.wce_apply(x[k], sigma, TAU, G, order, euler)) < tol
            assert rel_err(yT[k], pc.wce_apply_dag(x[k], sigma, TAU, G, order, euler)) < tol
    y = to_host(L.apply_precond(xd, Precond("sca", alpha=1.5), "Q"))
    D, Lb = pc.sca_setup(sigma, TAU, G, 1.5)
    for k in range(2):
        assert rel_err(y[k], pc.sca_apply(x[k], D, Lb)) < tol
    lam_max, eps = 7.0, 1e-2
    y = to_host(L.apply_precond(xd, Precond("cheb", degree=8, eps=eps, lam_max=lam_max), "Q"))
    for k in range(2):
        ref = pc.apply_cheb(x[k], sigma, TAU, G, 8, eps, lam_max)
        assert rel_err(y[k], ref) < tol * (10 if dtype == torch.complex64 else 1)


@pytest.mark.parametrize("dim,nx,ntau", [(1, 8, 6), (2, 4, 5)])
def test_solvers_against_dense_lu(dim, nx, ntau):
    require_gpu()
    from paper_1008_3647_amd import Precond
    L, sigma = _lattice(dim, nx, ntau, torch.complex128, seed=820)
    b, bd = _rhs(dim, nx, ntau, [821, 822], torch.complex128)
    Md = op.dense_M(sigma, TAU, G)
    for kind, pcd in (("M", None), ("Mdag", None), ("two_step", Precond("wce", wce_order=2))):
        x, st = L.solve_bicgstab(bd, kind, pcd, tol=1e-12)
        assert st["status"] == 0, (kind, st)
        A = Md if kind == "M" else Md.T if kind == "Mdag" else Md.T @ Md
        for k in range(2):
            ref = np.linalg.solve(A, b[k].ravel())
            assert rel_err(to_host(x)[k].ravel(), ref) < 1e-8, (kind, k)
    x, st = L.solve_cg_normal(bd, Precond("sca", alpha=2.0), tol=1e-12)
    assert st["status"] == 0
    for k in range(2):
        ref = np.linalg.solve(Md.T @ Md, b[k].ravel())
        assert rel_err(to_host(x)[k].ravel(), ref) < 1e-8


@pytest.mark.parametrize("dim,nx,ntau", [(1, 16, 64), (2, 16, 40)])
def test_fp32_refined_two_step(dim, nx, ntau):
    """FP32-refined two-step BiCGStab on a larger lower-dimensional lattice:
    the oracle's residual of each step and of M^T M x = b."""
    require_gpu()
    L, sigma = _lattice(dim, nx, ntau, torch.complex128, seed=830)
    b, bd = _rhs(dim, nx, ntau, [831, 832, 833], torch.complex128)
    x, st = L.solve_bicgstab(bd, "two_step", tol=1e-10, mixed=True)
    say(f"lowdim mixed two-step dim={dim}: iters {st['iters']} relres {st['relres']}")
    assert st["status"] == 0 and max(st["relres"]) <= 1e-10
    xh = to_host(x)
    for k in range(3):
        r = b[k] - oracle.apply_Q(xh[k], sigma, TAU, G)
        assert np.linalg.norm(r) / np.linalg.norm(b[k]) < 1e-7


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("dim,nx,ntau", [(1, 6, 9), (2, 4, 7), (2, 16, 3)])
def test_force(dim, nx, ntau, dtype):
    require_gpu()
    L, sigma = _lattice(dim, nx, ntau, dtype, seed=840)
    X, Xd = _rhs(dim, nx, ntau, [841, 842], dtype)
    y, yd = _rhs(dim, nx, ntau, [843, 844], dtype)
    g = to_host(L.force_dS_dsigma(Xd, yd))
    # the library's contraction: -2 A cos sigma s_t sum_r Re[X_t conj(T^d y_{t+1})],
    # the oracle's gradient with M X in place of y (force_dS_dsigma takes y)
    A = oracle.coupling_A(TAU, G)
    ref = np.zeros_like(sigma)
    for k in range(2):
        for t in range(ntau):
            s = 1.0 if t == ntau - 1 else -1.0
            Ty = op.apply_expK(y[k][(t + 1) % ntau], TAU, "free", dim)
            ref[t] += -2.0 * A * np.cos(sigma[t]) * s * np.real(X[k][t] * np.conj(Ty))
    tol = 1e-12 if dtype == torch.complex128 else 2e-5
    assert rel_err(g, ref) < tol
    # and with y = M X the contraction is the oracle's gradient
    if dtype == torch.complex128:
        MX = np.stack([oracle.apply_M(X[k], sigma, TAU, G) for k in range(2)])
        g2 = to_host(L.force_dS_dsigma(Xd, to_dev(MX)))
        ref2 = sum(fo.gradient(X[k], sigma, TAU, G) for k in range(2))
        assert rel_err(g2, ref2) < 1e-12


@pytest.mark.parametrize("dim,nx,ntau", [(1, 8, 8), (2, 4, 6)])
def test_hmc_chain_matches_oracle(dim, nx, ntau):
    """Three trajectories (dt = 0.1, 5 steps) with the same seeded momenta,
    pseudofermion sources and Metropolis draws as the oracle's dense chain:
    identical decisions, dH within the solver bound, the chain state within
    1e-10."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(nx, ntau, 850, dim)
    us = uniform_draws(851, 3)
    L = Lattice(nx, ntau, TAU, G, torch.complex128, dim=dim)
    s_o, s_g = sigma.copy(), to_dev(sigma)
    for k in range(3):
        pi = gaussian_momenta(nx, ntau, 852 + k, dim)
        eta = gaussian_rhs(nx, ntau, [860 + k], dim)
        ref = hmc.fermion_trajectory(s_o, pi, eta, us[k], 0.1, 5, TAU, G)
        s_g, p_g, info = L.hmc_trajectory(s_g, to_dev(pi), to_dev(eta), us[k], 0.1, 5,
                                          tol=1e-13)
        say(f"lowdim hmc dim={dim} traj {k}: dH gpu {info['dH']:+.10f} oracle "
            f"{ref['dH']:+.10f} accept {info['accept']}")
        kappa = np.linalg.cond(op.dense_M(s_o, TAU, G))
        assert info["status"] == 0 and info["accept"] == int(ref["accept"])
        assert abs(info["dH"] - ref["dH"]) <= 4 * kappa * 1e-13 * (ref["S0"] + ref["S1"]) + 1e-9
        assert rel_err(to_host(s_g), ref["sigma"]) < 1e-10
        s_o = ref["sigma"]


def test_batched_and_bad_dim_rejected():
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.lattice import UfgError, solve_batched
    L, _ = _lattice(2, 4, 6, torch.complex128, seed=870)
    _, bd = _rhs(2, 4, 6, [871], torch.complex128)
    with pytest.raises(UfgError):
        solve_batched([L], [bd], tol=1e-8)
    with pytest.raises(ValueError):
        Lattice(4, 6, TAU, G, torch.complex128, dim=4)
    with pytest.raises(ValueError):  # a 3D vector on a 2D lattice
        L.apply_M(to_dev(gaussian_rhs(4, 6, [872])))


@pytest.mark.parametrize("dim,nx,ntau", [(1, 8, 6), (2, 4, 5)])
def test_cg_variants_against_dense_lu(dim, nx, ntau):
    """CG on M^T M with the Chebyshev and SCA + Chebyshev preconditioners, and
    split-preconditioned CG with the weak-coupling W_1 (at g = 1, where the
    series converges in these dimensions), against dense LU."""
    require_gpu()
    from paper_1008_3647_amd import Precond
    b, bd = _rhs(dim, nx, ntau, [881, 882], torch.complex128)
    for g, solver, pcd in ((G, "cg", Precond("cheb", degree=8, eps=1e-2, lam_max=-1.0)),
                           (G, "cg", Precond("sca_cheb", degree=8, eps=1e-2, lam_max=-1.0)),
                           (1.0, "split", Precond("wce", wce_order=1))):
        L, sigma = _lattice(dim, nx, ntau, torch.complex128, g=g, seed=880)
        if solver == "cg":
            x, st = L.solve_cg_normal(bd, pcd, tol=1e-11)
        else:
            x, st = L.solve_cg_split(bd, pcd, tol=1e-11)
        say(f"lowdim {solver} {pcd.kind} dim={dim}: iters {st['iters']} status {st['status']}")
        assert st["status"] == 0, (solver, pcd.kind, st)
        Md = op.dense_M(sigma, TAU, g)
        for k in range(2):
            ref = np.linalg.solve(Md.T @ Md, b[k].ravel())
            assert rel_err(to_host(x)[k].ravel(), ref) < 1e-7, (solver, pcd.kind, k)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("dim,nx,ntau,nrhs", [(1, 16, 4000, 64), (2, 16, 1000, 8),
                                               (2, 8, 8000, 16)])
def test_operator_at_full_size(dim, nx, ntau, nrhs, dtype):
    """The lower-dimensional bandwidth workloads at their full size and right-hand
    side count, in the launch the bandwidth report times (library default):
    M and M^T element by element against the oracle for the first, a middle
    and the last rhs (1D: 64 slices per workgroup, 4000 = 62 x 64 + 32 leaves a
    ragged last workgroup; 2D, Nx = 8: 16 slices per workgroup)."""
    require_gpu()
    say(f"lowdim full-size operator dim={dim} nx={nx} ntau={ntau} nrhs={nrhs} {dtype}")
    L, sigma = _lattice(dim, nx, ntau, dtype, seed=890)
    seeds = list(range(891, 891 + nrhs))
    x, xd = _rhs(dim, nx, ntau, seeds, dtype)
    y = to_host(L.apply_M(xd))
    yd = to_host(L.apply_Mdag(xd))
    for k in (0, nrhs // 2, nrhs - 1):
        assert rel_err(y[k], oracle.apply_M(x[k], sigma, TAU, G)) < TOL_OP[dtype], k
        assert rel_err(yd[k], oracle.apply_Mdag(x[k], sigma, TAU, G)) < TOL_OP[dtype], k


@pytest.mark.parametrize("dim,ntau", [(1, (1 << 20) + 37), (2, (1 << 16) + 5)])
def test_operator_beyond_32bit_offsets(dim, ntau):
    """Nine complex128 right-hand sides of 16^d x ntau (2.4 GB): the last one
    starts beyond 2^31 bytes. Rhs 0 and 8 carry Gaussian vectors, the others
    zeros; sampled output slices of both (first, wrap-around, middle, last)
    against the oracle's slice formula (Sec. 1, Eq. MatrixM)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, nrhs = 16, 9
    say(f"lowdim 32-bit offsets dim={dim} ntau={ntau} nrhs={nrhs}")
    sigma = sigma_field(nx, ntau, 1300, dim)
    x0 = gaussian_rhs(nx, ntau, [1301], dim)[0]
    x8 = gaussian_rhs(nx, ntau, [1308], dim)[0]
    assert 8 * x8.nbytes >= (1 << 31)
    L = Lattice(nx, ntau, TAU, G, torch.complex128, dim=dim)
    L.set_aux_field(to_dev(sigma))
    xd = torch.zeros((nrhs,) + L.shape, dtype=torch.complex128, device="cuda")
    xd[0] = to_dev(x0)
    xd[8] = to_dev(x8)
    y = L.apply_M(xd)
    yd = L.apply_Mdag(xd)
    A = oracle.coupling_A(TAU, G)
    for r, x in ((0, x0), (8, x8)):
        for t in (0, 1, ntau // 2, ntau - 2, ntau - 1):
            tp, tn = (t - 1) % ntau, (t + 1) % ntau
            sp = 1.0 if tp == ntau - 1 else -1.0
            ref = x[t] + sp * op.apply_expK(oracle.field_b(sigma[tp], A) * x[tp], TAU, "free", dim)
            assert rel_err(to_host(y[r, t]), ref) < TOL_OP[torch.complex128], (r, t)
            st = 1.0 if t == ntau - 1 else -1.0
            refd = x[t] + st * oracle.field_b(sigma[t], A) * op.apply_expK(x[tn], TAU, "free", dim)
            assert rel_err(to_host(yd[r, t]), refd) < TOL_OP[torch.complex128], (r, t)
    assert float(y[4].abs().max()) == 0.0
    del xd, y, yd
    L.close()
    torch.cuda.empty_cache()
