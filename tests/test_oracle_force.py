"""Pins for the oracle's action, force and leapfrog (paper, Sec. 1)."""
import numpy as np
import pytest

import oracle
from oracle import operator as op
from oracle import force
from synthetic import sigma_field, gaussian_rhs, gaussian_momenta

TAU, G = 0.05, 5.0


def _dense_action(sigma, phi):
    Md = op.dense_M(sigma, TAU, G)
    y = np.linalg.solve(Md.T, phi.ravel())
    return float(np.vdot(y, y).real)


def _setup(nx, ntau, seed):
    sigma = sigma_field(nx, ntau, seed)
    eta = gaussian_rhs(nx, ntau, [seed + 1])[0]
    phi = oracle.apply_Mdag(eta, sigma, TAU, G)
    return sigma, eta, phi


def test_action_at_heat_bath_point():
    # phi = M^T eta  =>  y = M^{-T} phi = eta and S = ||eta||^2
    sigma, eta, phi = _setup(2, 6, 61)
    assert _dense_action(sigma, phi) == pytest.approx(np.vdot(eta, eta).real, rel=1e-12)


def test_oracle_action_function_pinned():
    """oracle.force.action (S = phi^H Q^{-1} phi computed as ||y||^2 with
    M^T y = phi) against two values that do not use that route: at the
    heat-bath point phi = M^T eta, S = ||eta||^2 and y = eta (Sec. 1); for a
    general phi, the spectral sum sum_i |v_i^H phi|^2 / lambda_i over the
    eigenpairs of the dense Q = M^T M."""
    nx, ntau = 2, 6
    sigma, eta, phi = _setup(nx, ntau, 64)
    Md = op.dense_M(sigma, TAU, G)

    def solve_Mdag(r):
        return np.linalg.solve(Md.T, r.ravel()).reshape(r.shape)

    S, y = force.action(phi, sigma, TAU, G, solve_Mdag)
    assert isinstance(S, float)
    assert S == pytest.approx(np.vdot(eta, eta).real, rel=1e-12)
    assert np.max(np.abs(y - eta)) < 1e-12 * np.max(np.abs(eta))
    phi2 = gaussian_rhs(nx, ntau, [65])[0] * 1.7
    S2, _ = force.action(phi2, sigma + 0.4, TAU, G, lambda r: np.linalg.solve(
        op.dense_M(sigma + 0.4, TAU, G).T, r.ravel()).reshape(r.shape))
    Md2 = op.dense_M(sigma + 0.4, TAU, G)
    lam, V = np.linalg.eigh(Md2.T @ Md2)
    spectral = float(np.sum(np.abs(V.conj().T @ phi2.ravel()) ** 2 / lam))
    assert S2 == pytest.approx(spectral, rel=1e-10)


def test_gradient_against_central_differences():
    nx, ntau = 2, 5
    sigma, eta, phi = _setup(nx, ntau, 62)
    sigma = sigma + 0.3  # move away from the heat-bath point
    Md = op.dense_M(sigma, TAU, G)
    X = np.linalg.solve(Md.T @ Md, phi.ravel()).reshape(phi.shape)
    grad = force.gradient(X, sigma, TAU, G)
    h = 1e-5
    flat = sigma.reshape(-1)
    for i in range(flat.size):
        sp, sm = flat.copy(), flat.copy()
        sp[i] += h
        sm[i] -= h
        fd = (_dense_action(sp.reshape(sigma.shape), phi)
              - _dense_action(sm.reshape(sigma.shape), phi)) / (2 * h)
        assert grad.reshape(-1)[i] == pytest.approx(fd, rel=1e-6, abs=1e-7 * np.abs(grad).max())


def test_sherman_morrison_difference_is_exact():
    nx, ntau = 2, 6
    sigma, eta, phi = _setup(nx, ntau, 63)
    sigma = sigma - 0.2
    Md = op.dense_M(sigma, TAU, G)
    y = np.linalg.solve(Md.T, phi.ravel()).reshape(phi.shape)
    S0 = float(np.vdot(y, y).real)

    def z_of(site):
        t, n = site
        e = np.zeros(phi.shape)
        e[t].reshape(-1)[n] = 1.0
        return np.linalg.solve(Md.T, e.ravel()).reshape(phi.shape)

    for site in [(0, 3), (ntau - 1, 5), (2, 0)]:
        for h in (1e-5, 1e-2, 0.7):
            dS = force.exact_difference(y, sigma, TAU, G, site, h, z_of)
            sp = sigma.copy()
            sp[site[0]].reshape(-1)[site[1]] += h
            assert dS == pytest.approx(_dense_action(sp, phi) - S0, rel=1e-8, abs=1e-12 * S0)


def _dense_grad_fn(phi):
    def fn(sig):
        Md = op.dense_M(sig, TAU, G)
        X = np.linalg.solve(Md.T @ Md, phi.ravel()).reshape(phi.shape)
        return force.gradient(X, sig, TAU, G)
    return fn


def test_leapfrog_reversible_and_second_order():
    nx, ntau = 2, 4
    sigma, eta, phi = _setup(nx, ntau, 64)
    pi0 = gaussian_momenta(nx, ntau, 65)
    gfn = _dense_grad_fn(phi)
    H0 = force.hamiltonian(pi0, _dense_action(sigma, phi))
    s1, p1 = force.leapfrog(sigma, pi0, 0.05, 20, gfn)
    s2, p2 = force.leapfrog(s1, -p1, 0.05, 20, gfn)
    assert np.allclose(s2, sigma, atol=1e-10) and np.allclose(-p2, pi0, atol=1e-10)
    dH = []
    for dt, n in ((0.04, 10), (0.02, 20)):
        s, p = force.leapfrog(sigma, pi0, dt, n, gfn)
        dH.append(abs(force.hamiltonian(p, _dense_action(s, phi)) - H0))
    ratio = dH[0] / dH[1]
    assert 2.8 < ratio < 5.2  # ~4 for a second-order integrator
