"""HMC force (paper, Sec. 1): the contraction kernel, the autograd Action, finite
differences, the oracle gradient on the 12^3 x 200 lattice, and 20 leapfrog steps.

Gradient target: ||g_gpu - g_oracle|| / ||g_oracle|| <= 1e-6 on sampled sites.
Finite differences use the Sherman-Morrison exact difference (oracle/force.py)
so that S ~ 3.5e5 does not cancel; its z = M^{-T} e comes from GPU solves.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import operator as op
from oracle import force as oforce
from synthetic import sigma_field, gaussian_rhs, gaussian_momenta, sample_sites, WORKLOADS
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(__file__)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-5)])
@pytest.mark.parametrize("nx,ntau,nrhs", [(4, 6, 1), (6, 10, 2), (16, 3, 1), (8, 5, 3)])
def test_force_kernel_matches_oracle(nx, ntau, nrhs, dtype, tol):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(nx, ntau, 800 + nx)
    X = gaussian_rhs(nx, ntau, range(810, 810 + nrhs))
    if dtype == torch.complex64:
        X = X.astype(np.complex64).astype(np.complex128)
    y = np.stack([oracle.apply_M(Xi, sigma, TAU, G) for Xi in X])
    if dtype == torch.complex64:
        y = y.astype(np.complex64).astype(np.complex128)
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    g = to_host(L.force_dS_dsigma(to_dev(X, dtype), to_dev(y, dtype)))
    ref = sum(oforce.gradient(Xi, sigma, TAU, G) for Xi in X)
    assert rel_err(g, ref) < tol


def test_autograd_action_tiny_dense():
    """S and dS/dsigma through torch.autograd vs dense linear algebra."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.action import action
    nx, ntau = 4, 6
    sigma = sigma_field(nx, ntau, 820) * 0.9
    eta = gaussian_rhs(nx, ntau, [821, 822])
    phi = np.stack([oracle.apply_Mdag(e, sigma, TAU, G) for e in eta])
    sigma2 = sigma + 0.2  # away from the heat-bath point
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    s = to_dev(sigma2).requires_grad_(True)
    S = action(s, to_dev(phi), L, tol=1e-13)
    S.backward()
    Md = op.dense_M(sigma2, TAU, G)
    Qd = Md.T @ Md
    S_ref = sum(np.vdot(p.ravel(), np.linalg.solve(Qd, p.ravel())).real for p in phi)
    assert S.item() == pytest.approx(S_ref, rel=1e-11)
    X = [np.linalg.solve(Qd, p.ravel()).reshape(sigma.shape) for p in phi]
    g_ref = sum(oforce.gradient(Xi, sigma2, TAU, G) for Xi in X)
    assert rel_err(to_host(s.grad), g_ref) < 1e-9
    # central differences of the dense action at a few sites
    flat = sigma2.reshape(-1)
    for i in (0, 17, 200, flat.size - 1):
        vals = []
        for h in (1e-5, -1e-5):
            sp = flat.copy()
            sp[i] += h
            Mp = op.dense_M(sp.reshape(sigma.shape), TAU, G)
            vals.append(sum(np.linalg.norm(np.linalg.solve(Mp.T, p.ravel())) ** 2 for p in phi))
        fd = (vals[0] - vals[1]) / 2e-5
        assert to_host(s.grad).reshape(-1)[i] == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.abs(g_ref).max())


@pytest.fixture(scope="module")
def lattice_12x200():
    require_gpu()
    from paper_1008_3647_amd import Lattice
    w = WORKLOADS["lattice_12x200"]
    nx, ntau = w["nx"], w["ntau"]
    sigma = sigma_field(nx, ntau, w["sigma_seed"])
    eta = gaussian_rhs(nx, ntau, [w["eta_seed"]])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    phi = L.apply_Mdag(to_dev(eta))
    return L, w, sigma, eta, phi


def test_force_12x200_against_oracle_and_exact_differences(lattice_12x200):
    from paper_1008_3647_amd import Precond
    from paper_1008_3647_amd.action import force
    L, w, sigma, eta, phi = lattice_12x200
    pc = Precond("wce", wce_order=2)
    S, g = force(to_dev(sigma), phi, L, pc, tol=1e-12)
    g = to_host(g)
    say(f"S = {S:.6f}, |eta|^2 = {np.vdot(eta, eta).real:.6f}")
    assert S == pytest.approx(np.vdot(eta, eta).real, rel=1e-10)
    ref = np.load(os.path.join(HERE, "golden", "lattice_12x200_reference.npz"))
    gs = g.reshape(-1)[ref["sites"]]
    err = np.linalg.norm(gs - ref["grad_sample"]) / np.linalg.norm(ref["grad_sample"])
    say(f"gradient vs oracle on {len(gs)} sites: {err:.2e}")
    assert err <= 1e-6
    # exact central differences at 32 sites (Sherman-Morrison, z = M^{-T} e by GPU solves)
    nx, ntau = w["nx"], w["ntau"]
    V = nx ** 3
    y, _ = L.solve_bicgstab(phi, "Mdag", pc, tol=1e-12)
    yh = to_host(y)[0]
    sites = sample_sites(V * ntau, 32, w["site_seed"])
    h = 1e-5
    fd, gg = [], []
    for flat in sites:
        t, n = int(flat // V), int(flat % V)
        e = np.zeros((1, ntau, nx, nx, nx), dtype=np.complex128)
        e[0, t].reshape(-1)[n] = 1.0
        z, st = L.solve_bicgstab(to_dev(e), "Mdag", pc, tol=1e-12)
        zh = to_host(z)[0].real

        def zf(site, zh=zh):
            return zh
        dp = oforce.exact_difference(yh, sigma, TAU, G, (t, n), h, zf)
        dm = oforce.exact_difference(yh, sigma, TAU, G, (t, n), -h, zf)
        fd.append((dp - dm) / (2 * h))
        gg.append(g.reshape(-1)[flat])
    fd, gg = np.array(fd), np.array(gg)
    err_fd = np.linalg.norm(gg - fd) / np.linalg.norm(fd)
    say(f"gradient vs exact central differences on 32 sites: {err_fd:.2e}")
    assert err_fd <= 1e-6


def test_leapfrog_20_steps(lattice_12x200):
    """20 leapfrog steps of the phi-algorithm MD (Sec. 1). The paper gives no
    step size; dt = 0.0025 is inside the integrator's stability limit for this
    stiff action (dt >= 0.01 diverges, dt = 0.005 gives |dH| ~ 3). Checks:
    |dH| small, reversibility (flip pi, integrate back), dH ~ dt^2."""
    from paper_1008_3647_amd import Precond
    from paper_1008_3647_amd.action import leapfrog, hamiltonian
    L, w, sigma, eta, phi = lattice_12x200
    pc = Precond("wce", wce_order=2, euler=True)
    pi0 = to_dev(gaussian_momenta(w["nx"], w["ntau"], w["momentum_seed"]))
    s0 = to_dev(sigma)
    dt = 0.0025
    s1, p1, S1 = leapfrog(s0, pi0, phi, L, dt, 20, pc, tol=1e-13)
    dH1 = hamiltonian(p1, S1[-1]) - hamiltonian(pi0, S1[0])
    say(f"dt {dt}: dH {dH1:.3e}")
    assert abs(dH1) < 0.1
    s2, p2, S2 = leapfrog(s1, -p1, phi, L, dt, 20, pc, tol=1e-13)
    rev = float((s2 - s0).abs().max().item())
    say(f"reversibility max|sigma - sigma0| = {rev:.2e}, max|pi + pi0| = "
        f"{float((p2 + pi0).abs().max().item()):.2e}")
    assert rev < 1e-8
    assert float((p2 + pi0).abs().max().item()) < 1e-8
    sh, ph, Sh = leapfrog(s0, pi0, phi, L, dt / 2, 40, pc, tol=1e-13)
    dH2 = hamiltonian(ph, Sh[-1]) - hamiltonian(pi0, Sh[0])
    ratio = abs(dH1) / abs(dH2)
    say(f"dt {dt / 2} (same trajectory length): dH {dH2:.3e}, |ratio| {ratio:.2f}")
    # second order: halving dt divides |dH| by ~4; at this trajectory length the
    # sign of dH still oscillates, so the magnitude ratio gets a wide band
    assert 2.0 < ratio < 8.0


def test_leapfrog_trajectory_matches_oracle():
    """The torch/HIP leapfrog (every force from two libufg solves and the force
    kernel) against the oracle's leapfrog with dense solves, same start, momenta,
    step and step count, on a tiny lattice: sigma and pi agree entry by entry
    (the GPU solves run to 1e-13, so each force carries ~cond x 1e-13 relative
    error; ten steps of dt = 0.02 keep sigma and pi within 1e-11; measured
    4e-15 and 4e-14)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.action import leapfrog, hamiltonian
    nx, ntau = 4, 6
    sigma = sigma_field(nx, ntau, 840)
    eta = gaussian_rhs(nx, ntau, [841])[0]
    phi = oracle.apply_Mdag(eta, sigma, TAU, G)
    pi0 = gaussian_momenta(nx, ntau, 842)
    dt, nsteps = 0.02, 10

    def grad_fn(s):
        Md = op.dense_M(s, TAU, G)
        X = np.linalg.solve(Md.T @ Md, phi.ravel()).reshape(phi.shape)
        return oforce.gradient(X, s, TAU, G)

    s_o, p_o = oforce.leapfrog(sigma, pi0, dt, nsteps, grad_fn)
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    s_g, p_g, S_g = leapfrog(to_dev(sigma), to_dev(pi0), to_dev(phi[None]), L, dt, nsteps,
                             None, tol=1e-13)
    es, ep = rel_err(to_host(s_g), s_o), rel_err(to_host(p_g), p_o)
    Md = op.dense_M(s_o, TAU, G)
    S_o = float(np.linalg.norm(np.linalg.solve(Md.T, phi.ravel())) ** 2)
    say(f"leapfrog vs oracle: sigma {es:.2e}, pi {ep:.2e}; S end {S_g[-1]:.12f} vs {S_o:.12f}")
    assert es < 1e-11 and ep < 1e-11
    assert S_g[-1] == pytest.approx(S_o, rel=1e-10)
    assert S_g[0] == pytest.approx(float(np.vdot(eta, eta).real), rel=1e-11)
