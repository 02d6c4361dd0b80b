"""Parity of apply_M / apply_Mdag (HIP, through the C ABI) with the FP64 oracle.

Tolerance (element-wise, relative to the largest output magnitude):
  complex128: 1e-13 (a few ulps of the 3 x Nx-term sums and the FFT route)
  complex64 : 5e-6  (3 x 16-term FP32 sums, ~sqrt(48) * 6e-8, with margin)
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import operator as oracle_op
from synthetic import sigma_field, gaussian_rhs, WORKLOADS
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu

TOL = {torch.complex128: 1e-13, torch.complex64: 5e-6}

# (nx, ntau, nrhs): every supported Nx, slices-per-workgroup tails, the two
# smallest cases and the antiperiodic corner at Ntau = 2.
SHAPES = [(2, 2, 1), (2, 3, 2), (4, 40, 1), (4, 17, 2), (6, 9, 3), (8, 5, 2), (10, 3, 2),
          (12, 4, 1), (14, 3, 1), (16, 6, 2), (8, 160, 4), (16, 2, 1), (8, 9, 3), (12, 7, 2),
          (16, 13, 3)]


def _oracle(fn, x, sigma):
    return np.stack([fn(xi, sigma, TAU, G) for xi in x])


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx,ntau,nrhs", SHAPES)
def test_apply_matches_oracle(nx, ntau, nrhs, dtype):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    say(f"apply parity nx={nx} ntau={ntau} nrhs={nrhs} {dtype}")
    sigma = sigma_field(nx, ntau, 100 + nx + ntau)
    x = gaussian_rhs(nx, ntau, range(200, 200 + nrhs))
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x, dtype)
    y = to_host(L.apply_M(xd))
    yd = to_host(L.apply_Mdag(xd))
    ref = _oracle(oracle.apply_M, x.astype(np.complex64).astype(np.complex128)
                  if dtype == torch.complex64 else x, sigma)
    refd = _oracle(oracle.apply_Mdag, x.astype(np.complex64).astype(np.complex128)
                   if dtype == torch.complex64 else x, sigma)
    assert rel_err(y, ref) < TOL[dtype]
    assert rel_err(yd, refd) < TOL[dtype]


def test_adjoint_identity_on_device():
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau = 8, 24
    sigma = sigma_field(nx, ntau, 301)
    u, v = gaussian_rhs(nx, ntau, [302, 303])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    Mu = to_host(L.apply_M(to_dev(u[None])))[0]
    Mtv = to_host(L.apply_Mdag(to_dev(v[None])))[0]
    lhs, rhs = np.vdot(Mu, v), np.vdot(u, Mtv)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_full_size_lattice_16x400():
    """Full 16^3 x 400 lattice, 8 RHS, both precisions, in the launch the bench
    times: two right-hand sides (first and last) compared entry by entry."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    w = WORKLOADS["lattice_16x400"]
    nx, ntau = w["nx"], w["ntau"]
    sigma = sigma_field(nx, ntau, w["sigma_seed"])
    b = gaussian_rhs(nx, ntau, w["rhs_seeds"])
    for dtype in (torch.complex128, torch.complex64):
        say(f"full-size apply {dtype}")
        L = Lattice(nx, ntau, TAU, G, dtype)
        L.set_aux_field(to_dev(sigma))
        bd = to_dev(b, dtype)
        y = L.apply_M(bd)
        yd = L.apply_Mdag(bd)
        for k in (0, len(w["rhs_seeds"]) - 1):
            xk = b[k].astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else b[k]
            assert rel_err(to_host(y[k]), oracle.apply_M(xk, sigma, TAU, G)) < TOL[dtype]
            assert rel_err(to_host(yd[k]), oracle.apply_Mdag(xk, sigma, TAU, G)) < TOL[dtype]
        L.close()


def test_invalid_arguments_are_rejected():
    require_gpu()
    from paper_1008_3647_amd import Lattice, UfgError
    with pytest.raises(UfgError):
        Lattice(5, 8)
    with pytest.raises(UfgError):
        Lattice(4, 1)
    with pytest.raises(UfgError):
        Lattice(18, 4)
    L = Lattice(4, 4)
    with pytest.raises(TypeError):
        L.apply_M(torch.zeros((1, 4, 4, 4, 4), dtype=torch.complex64, device="cuda"))
    with pytest.raises(ValueError):
        L.apply_M(torch.zeros((1, 5, 4, 4, 4), dtype=torch.complex128, device="cuda"))
    with pytest.raises(UfgError):
        L.tune(slab=5)  # more slices per slab than Ntau
    with pytest.raises(UfgError):
        L.tune(nslab=5)  # more slabs than Ntau
    with pytest.raises(UfgError):
        L.tune(vec_blocks=5000)
    with pytest.raises(UfgError):
        L.tune(xcd_group=-2)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx", [8, 12, 16])
def test_apply_every_slab_size(nx, dtype):
    """The streaming kernel's slab size (slices per workgroup) changes the walk,
    the halo and the tail slab; every size from 1 to 6 must give the same
    operator, on a lattice whose Ntau (23) leaves a ragged last slab for all of
    them."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    ntau, nrhs = 23, 3
    sigma = sigma_field(nx, ntau, 410 + nx)
    x = gaussian_rhs(nx, ntau, range(420, 420 + nrhs))
    xin = x.astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else x
    ref = _oracle(oracle.apply_M, xin, sigma)
    refd = _oracle(oracle.apply_Mdag, xin, sigma)
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x, dtype)
    for slab in range(1, 7):
        say(f"slab parity nx={nx} slab={slab} {dtype}")
        L.tune(slab, 0)
        assert rel_err(to_host(L.apply_M(xd)), ref) < TOL[dtype], slab
        assert rel_err(to_host(L.apply_Mdag(xd)), refd) < TOL[dtype], slab
    # slab counts that do not divide Ntau (balanced partition), down to one
    # slab holding every slice
    for nslab in (1, 5, 7, 10, 17, 23):
        say(f"slab-count parity nx={nx} nslab={nslab} {dtype}")
        L.tune(0, 0, nslab=nslab)
        assert rel_err(to_host(L.apply_M(xd)), ref) < TOL[dtype], nslab
        assert rel_err(to_host(L.apply_Mdag(xd)), refd) < TOL[dtype], nslab


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("nx", [8, 16])
def test_apply_every_xcd_group(nx, dtype):
    """The workgroup numbering (slab groups per XCD, lattice_tune_order) only
    moves work between workgroups: every group size, with slab sizes that leave
    a partial last group and XCDs without work, must give the oracle's operator
    and bit-identical outputs for M, M^T and the basis changes of a WCE1
    application."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    ntau, nrhs = 23, 3
    sigma = sigma_field(nx, ntau, 440 + nx)
    x = gaussian_rhs(nx, ntau, range(450, 450 + nrhs))
    xin = x.astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else x
    ref = _oracle(oracle.apply_M, xin, sigma)
    refd = _oracle(oracle.apply_Mdag, xin, sigma)
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x, dtype)
    pc = Precond("wce", wce_order=1)
    first = None
    orders = [(0, False)] + [(g, ri) for g in (1, 2, 3, 5, 7, 23) for ri in (False, True)]
    for slab in (1, 2, 5):
        for group, ri in orders:
            say(f"xcd-group parity nx={nx} slab={slab} group={group} rhs_inner={ri} {dtype}")
            L.tune(slab, 0, xcd_group=group, rhs_inner=ri)
            y = to_host(L.apply_M(xd))
            yd = to_host(L.apply_Mdag(xd))
            w = to_host(L.apply_precond(xd, pc, "M"))
            assert rel_err(y, ref) < TOL[dtype], (slab, group)
            assert rel_err(yd, refd) < TOL[dtype], (slab, group)
            if first is None or first[0] != slab:
                first = (slab, y, yd, w)
            else:
                assert np.array_equal(y, first[1]) and np.array_equal(yd, first[2]), (slab, group)
                assert np.array_equal(w, first[3]), (slab, group)


@pytest.mark.parametrize("group,rhs_inner", [(0, False), (1, False), (4, False), (3, True)])
def test_solve_with_xcd_group(group, rhs_inner):
    """Fused reductions leave one partial per (rhs, slab) whatever workgroup
    computes it: two-step solves under each numbering converge to the oracle's
    residual bound."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau, nrhs = 8, 23, 2
    sigma = sigma_field(nx, ntau, 460)
    b = gaussian_rhs(nx, ntau, range(461, 461 + nrhs))
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    L.tune(1, 0, xcd_group=group, rhs_inner=rhs_inner)
    for mixed in (False, True):
        x, st = L.solve_bicgstab(to_dev(b), "two_step", tol=1e-10, mixed=mixed)
        assert st["status"] == 0, (group, mixed)
        xh = to_host(x)
        for i in range(nrhs):
            r = b[i] - oracle.apply_Q(xh[i], sigma, TAU, G)
            assert np.linalg.norm(r) / np.linalg.norm(b[i]) < 1e-9, (group, mixed, i)


@pytest.mark.parametrize("mixed", [False, True])
def test_solve_with_uneven_slab_count(mixed):
    """The fused reductions of the streaming kernel leave one partial per slab;
    a slab count that does not divide Ntau must still give converged solves of
    M x = b and M^T x = b (true residuals checked with the oracle operators)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau, nrhs = 8, 23, 2
    sigma = sigma_field(nx, ntau, 430)
    b = gaussian_rhs(nx, ntau, range(431, 431 + nrhs))
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    L.tune(0, 0, nslab=7)
    for op, fn in (("M", oracle.apply_M), ("Mdag", oracle.apply_Mdag)):
        x, st = L.solve_bicgstab(to_dev(b), op, tol=1e-10, mixed=mixed)
        assert st["status"] == 0, op
        xh = to_host(x)
        for i in range(nrhs):
            r = b[i] - fn(xh[i], sigma, TAU, G)
            assert np.linalg.norm(r) / np.linalg.norm(b[i]) < 2e-10, (op, i)


def test_device_copy_helper():
    """The copy used as the bandwidth reference moves bytes exactly."""
    require_gpu()
    from paper_1008_3647_amd.lattice import device_copy
    x = torch.randn(3 * 1024 * 1024 + 16, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    device_copy(x, y)
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def _slice_M(x, sigma, t, ntau):
    """Output slice t of y = M x from the oracle's pieces (Eq. MatrixM): the
    identity term plus the coupling of source slice t - 1."""
    tp = (t - 1) % ntau
    s = 1.0 if tp == ntau - 1 else -1.0
    b = oracle_op.field_b(sigma[tp], oracle_op.coupling_A(TAU, G))
    return x[t] + s * oracle_op.apply_expK(b * x[tp], TAU)


def _slice_Mdag(x, sigma, t, ntau):
    tn = (t + 1) % ntau
    s = 1.0 if t == ntau - 1 else -1.0
    b = oracle_op.field_b(sigma[t], oracle_op.coupling_A(TAU, G))
    return x[t] + s * b * oracle_op.apply_expK(x[tn], TAU)


@pytest.mark.parametrize("ntau", [32767, 32768])
def test_largest_rhs_blocks(ntau):
    """The streaming kernel addresses one right-hand side with 32-bit byte
    offsets, so it takes complex128 blocks below 2^31 bytes (16^3 x 32767) and
    larger ones (16^3 x 32768) go to the general slice kernel. Both must give
    the operator: sampled output slices (first, wrap-around, middle, last)
    against the oracle's slice formula."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx = 16
    say(f"largest blocks nx={nx} ntau={ntau}")
    sigma = sigma_field(nx, 32768, 470)[:ntau]
    x = gaussian_rhs(nx, 32768, [471])[0][:ntau]
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x[None])
    y = L.apply_M(xd)
    yd = L.apply_Mdag(xd)
    for t in (0, 1, ntau // 2, ntau - 2, ntau - 1):
        ref = _slice_M(x, sigma, t, ntau)
        assert rel_err(to_host(y[0, t]), ref) < TOL[torch.complex128], t
        refd = _slice_Mdag(x, sigma, t, ntau)
        assert rel_err(to_host(yd[0, t]), refd) < TOL[torch.complex128], t
    del y, yd, xd
    L.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("route", [1, 2])
@pytest.mark.parametrize("ntau,nrhs,slab", [(6, 2, 0), (23, 3, 2), (400, 8, 0)])
def test_transform_routes(ntau, nrhs, slab, route):
    """lattice_tune_transform: route 1 runs the y and x stages of T^3 as 16x16x4
    MFMA contractions, route 2 every stage as a 16-point DFT, the eigenvalues
    of T and the inverse DFT (complex64, Nx = 16). Each matches the oracle's
    operator within the complex64 tolerance on every slice (sampled slices of
    the full 16^3 x 400 launch), and the VALU route's output within 2e-6 (route
    1: one 16-term FP32 sum per axis in another order) or 1e-5 (route 2: six
    radix-4 DFT passes, each with an FP32 error of about log2(16) u relative to
    the line); route 0 is restored bit for bit afterwards."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx = 16
    sigma = sigma_field(nx, ntau, 470 + ntau)
    x = gaussian_rhs(nx, ntau, range(480, 480 + nrhs))
    L = Lattice(nx, ntau, TAU, G, torch.complex64)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x, torch.complex64)
    L.tune(slab, 0, transform=0)
    y0, yd0 = to_host(L.apply_M(xd)), to_host(L.apply_Mdag(xd))
    L.tune(slab, 0, transform=route)
    y1, yd1 = to_host(L.apply_M(xd)), to_host(L.apply_Mdag(xd))
    say(f"route {route} ntau={ntau}: |M diff| {rel_err(y1, y0):.1e}, "
        f"|M^T diff| {rel_err(yd1, yd0):.1e}")
    bound = 2e-6 if route == 1 else 1e-5
    assert rel_err(y1, y0) < bound and rel_err(yd1, yd0) < bound
    xin = x.astype(np.complex64).astype(np.complex128)
    ts = range(ntau) if ntau <= 23 else (0, 1, 199, 200, ntau - 1)
    for k in (range(nrhs) if ntau <= 23 else (0, nrhs - 1)):
        Mx = oracle.apply_M(xin[k], sigma, TAU, G)
        Mdx = oracle.apply_Mdag(xin[k], sigma, TAU, G)
        for t in ts:
            assert rel_err(y1[k, t], Mx[t]) < TOL[torch.complex64], (k, t)
            assert rel_err(yd1[k, t], Mdx[t]) < TOL[torch.complex64], (k, t)
    L.tune(slab, 0, transform=0)
    assert np.array_equal(to_host(L.apply_M(xd)), y0)
    with pytest.raises(Exception):
        L.tune(slab, 0, transform=3)


def test_dft_route_on_a_hubbard_lattice():
    """Route 2 takes the eigenvalues of T from T itself, so it holds for the
    Hubbard dispersion too (oracle within the complex64 tolerance)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau = 16, 7
    sigma = sigma_field(nx, ntau, 489)
    x = gaussian_rhs(nx, ntau, [490, 491])
    L = Lattice(nx, ntau, TAU, G, torch.complex64, dispersion="hubbard")
    L.set_aux_field(to_dev(sigma))
    L.tune(transform=2)
    y = to_host(L.apply_M(to_dev(x, torch.complex64)))
    xin = x.astype(np.complex64).astype(np.complex128)
    for k in range(2):
        assert rel_err(y[k], oracle.apply_M(xin[k], sigma, TAU, G, "hubbard")) < TOL[torch.complex64]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_tune_apply(dtype):
    """autotune.tune_apply: every (slab, numbering[, T^3 route]) candidate is
    timed on the plain operator, the best is applied, and apply_M / apply_Mdag
    under the chosen shape match the oracle on every slice."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.autotune import tune_apply, candidate_slabs, ORDERS
    nx, ntau, nrhs = 16, 12, 2
    sigma = sigma_field(nx, ntau, 490)
    x = gaussian_rhs(nx, ntau, [491, 492])
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    xd = to_dev(x, dtype)
    xs = [xd, xd.clone()]
    for dagger in (False, True):
        t = tune_apply(L, xs, dagger=dagger, launches=4, reps=1)
        nt = 3 if dtype == torch.complex64 else 1
        assert len(t["candidates"]) == len(candidate_slabs(L)) * len(ORDERS) * nt
        assert (t["xcd_group"], t["rhs_inner"]) in ORDERS and t["transform"] in range(nt)
        say(f"tune_apply {dtype} dagger={dagger}: "
            f"{ {k: t[k] for k in ('slab', 'xcd_group', 'rhs_inner', 'transform')} }")
        y = to_host(L.apply_Mdag(xd) if dagger else L.apply_M(xd))
        xin = x.astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else x
        for k in range(nrhs):
            ref = (oracle.apply_Mdag if dagger else oracle.apply_M)(xin[k], sigma, TAU, G)
            assert rel_err(y[k], ref) < TOL[dtype], (dagger, k)
