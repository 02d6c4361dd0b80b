"""Pins of the oracle's HMC trajectory (oracle/hmc.py) against what the
mathematics fixes, independently of the oracle's own arithmetic:

* leapfrog on a harmonic action S = sum w^2 sigma^2 / 2 against its closed-form
  transfer matrix (Chebyshev powers), actions included;
* the Markov chain with Metropolis samples exp(-H) exactly: on the harmonic
  toy at a step where the leapfrog's shadow Hamiltonian is far from H, the
  chain's variance of sigma is 1 / w^2 (an always-accept or wrong-sign chain
  gives 1 / (w^2 (1 - dt^2 w^2 / 4)) or worse);
* the Metropolis rule against the acceptance probability min(1, exp(-dH));
* on tiny fermion lattices (dense solves): S_p at the heat-bath point equals
  ||eta||^2, dH shrinks as dt^2, the MD map is reversible and volume
  preserving (finite-difference Jacobian, det = 1), and the free case A = 0
  (g = 0) reduces to free streaming with dH = 0.
"""
import numpy as np
import pytest

from oracle import hmc
from oracle import operator as op
from synthetic import sigma_field, gaussian_rhs, gaussian_momenta, uniform_draws

TAU, G = 0.05, 5.0


def _harmonic(w2):
    def action_grad(s):
        return float(0.5 * np.sum(w2 * s * s)), w2 * s
    return action_grad


def test_leapfrog_matches_harmonic_closed_form():
    """One leapfrog step (kick-drift-kick, step h) on S = w^2 q^2 / 2 is the
    matrix T = [[c, h], [-h w^2 (1 - h^2 w^2 / 4), c]], c = 1 - h^2 w^2 / 2 = cos(th),
    det T = 1; T^n = [[cos n th, h s_n], [-h w^2 (1 - h^2 w^2 / 4) s_n, cos n th]]
    with s_n = sin(n th) / sin(th)."""
    rng = np.random.default_rng(1)
    w2 = rng.uniform(0.2, 3.0, size=50)
    q0, p0 = rng.standard_normal(50), rng.standard_normal(50)
    h, n = 0.3, 17
    q, p, actions = hmc.md(q0, p0, h, n, _harmonic(w2))
    c = 1.0 - 0.5 * h * h * w2
    th = np.arccos(c)

    def power(k):
        sk = np.sin(k * th) / np.sin(th)
        return np.cos(k * th), h * sk, -h * w2 * (1.0 - 0.25 * h * h * w2) * sk

    a, b, d = power(n)
    assert np.allclose(q, a * q0 + b * p0, rtol=0, atol=1e-12)
    assert np.allclose(p, d * q0 + a * p0, rtol=0, atol=1e-12)
    for k, S in enumerate(actions):
        ak, bk, _ = power(k)
        qk = ak * q0 + bk * p0
        assert S == pytest.approx(0.5 * np.sum(w2 * qk * qk), rel=1e-12)


def test_metropolis_rule():
    """accept iff u < exp(-dH): always for dH <= 0; on a uniform grid of u the
    accepted fraction is exp(-dH) for dH > 0."""
    u = (np.arange(100000) + 0.5) / 100000
    for dH in (-3.0, -1e-9, 0.0):
        assert all(hmc.metropolis(dH, x) for x in u[::997])
    for dH in (1e-3, 0.1, np.log(2.0), 2.5):
        frac = np.mean([hmc.metropolis(dH, x) for x in u[::7]])
        assert frac == pytest.approx(np.exp(-dH), abs=2e-4)
    assert hmc.metropolis(np.log(2.0), 0.4999) and not hmc.metropolis(np.log(2.0), 0.5001)


def test_chain_samples_exp_minus_H():
    """HMC chain on one harmonic mode (w = 1, dt = 1.2, 3 steps: acceptance ~ 0.7):
    the stationary law of sigma is N(0, 1 / w^2) only with a correct Metropolis
    step. Without it the chain samples the shadow Hamiltonian, variance
    1 / (1 - dt^2 / 4) = 1.5625 here."""
    w2 = np.array([1.0])
    ag = _harmonic(w2)
    rng = np.random.default_rng(7)
    n = 20000
    pis = rng.standard_normal(n)
    us = rng.random(n)
    s = np.array([0.0])
    xs, acc = np.empty(n), 0
    for i in range(n):
        out = hmc.trajectory(s, np.array([pis[i]]), us[i], 1.2, 3, ag)
        s = out["sigma"]
        acc += out["accept"]
        xs[i] = s[0]
    var = np.mean(xs[1000:] ** 2)
    assert 0.4 < acc / n < 0.95
    assert var == pytest.approx(1.0, abs=0.08)
    assert abs(np.mean(xs[1000:])) < 0.06


def _tiny(nx=2, ntau=4, seed=0, nphi=1):
    sigma = sigma_field(nx, ntau, 9100 + seed)
    pi = gaussian_momenta(nx, ntau, 9200 + seed)
    eta = gaussian_rhs(nx, ntau, [9300 + seed + 10 * k for k in range(nphi)])
    return sigma, pi, eta


@pytest.mark.parametrize("nphi", [1, 2])
def test_heat_bath_action_is_eta_norm(nphi):
    """S_p(sigma_0) = sum_r phi_r^H Q^{-1} phi_r = sum_r ||eta_r||^2 for phi = M^dagger eta.
    A heat bath with M in place of M^dagger breaks this (M is not normal)."""
    sigma, pi, eta = _tiny(4, 6, 1, nphi)
    phi = hmc.heat_bath(eta, sigma, TAU, G)
    S, _ = hmc.dense_action_grad(phi, TAU, G)(sigma)
    assert S == pytest.approx(float(np.sum(np.abs(eta) ** 2)), rel=1e-12)
    Md = op.dense_M(sigma, TAU, G)
    wrong = np.stack([(Md @ e.reshape(-1)).reshape(e.shape) for e in eta])
    Sw, _ = hmc.dense_action_grad(wrong, TAU, G)(sigma)
    assert abs(Sw / S - 1.0) > 1e-3


def test_dH_second_order_and_reversible():
    """dH(dt) / dH(dt/2) ~ 4 at fixed trajectory length; integrating back with
    flipped momenta returns to the start to rounding."""
    sigma, pi, eta = _tiny(2, 4, 2)
    phi = hmc.heat_bath(eta, sigma, TAU, G)
    ag = hmc.dense_action_grad(phi, TAU, G)
    dH = []
    for dt, n in ((0.02, 10), (0.01, 20), (0.005, 40)):
        out = hmc.trajectory(sigma, pi, 0.5, dt, n, ag)
        dH.append(out["dH"])
    assert abs(dH[0] / dH[1]) == pytest.approx(4.0, rel=0.1)
    assert abs(dH[1] / dH[2]) == pytest.approx(4.0, rel=0.05)
    out = hmc.trajectory(sigma, pi, 0.5, 0.02, 10, ag)
    s2, p2, _ = hmc.md(out["sigma_md"], -out["pi_md"], 0.02, 10, ag)
    assert np.max(np.abs(s2 - sigma)) < 1e-12
    assert np.max(np.abs(p2 + pi)) < 1e-12


def test_md_map_preserves_volume():
    """The leapfrog map (sigma, pi) -> (sigma', pi') is symplectic: the
    determinant of its Jacobian (central differences, h = 1e-6) is 1."""
    sigma, pi, eta = _tiny(2, 2, 3)
    phi = hmc.heat_bath(eta, sigma, TAU, G)
    ag = hmc.dense_action_grad(phi, TAU, G)
    n = sigma.size
    z0 = np.concatenate([sigma.ravel(), pi.ravel()])

    def flow(z):
        s, p, _ = hmc.md(z[:n].reshape(sigma.shape), z[n:].reshape(sigma.shape), 0.05, 6, ag)
        return np.concatenate([s.ravel(), p.ravel()])

    h = 1e-6
    J = np.empty((2 * n, 2 * n))
    for j in range(2 * n):
        e = np.zeros(2 * n)
        e[j] = h
        J[:, j] = (flow(z0 + e) - flow(z0 - e)) / (2 * h)
    assert np.linalg.det(J) == pytest.approx(1.0, abs=1e-6)
    # and the map is not trivially the identity or a free stream
    assert np.max(np.abs(J[n:, :n])) > 1e-3


def test_free_case_streams_freely():
    """g = 0 gives A = 0: M does not depend on sigma, the force vanishes, the MD
    is free streaming sigma' = sigma + T pi and dH = 0; every u < 1 accepts."""
    sigma, pi, eta = _tiny(2, 4, 4)
    out = hmc.fermion_trajectory(sigma, pi, eta, 0.999999, 0.1, 7, TAU, 0.0)
    assert np.allclose(out["sigma_md"], sigma + 0.7 * pi, rtol=0, atol=1e-13)
    assert np.array_equal(out["pi_md"], pi)
    assert abs(out["dH"]) < 1e-12 and out["accept"]


def test_reject_returns_start():
    """A draw above exp(-dH) rejects and the chain's next state is the start;
    a draw below it accepts the MD end point (seed 7: dH ~ +0.058)."""
    sigma, pi, eta = _tiny(2, 4, 7)
    out = hmc.fermion_trajectory(sigma, pi, eta, 0.0, 0.2, 5, TAU, G)
    assert out["dH"] > 0.01 and out["accept"]
    assert np.array_equal(out["sigma"], out["sigma_md"])
    u = np.exp(-out["dH"]) * 1.001
    rej = hmc.fermion_trajectory(sigma, pi, eta, u, 0.2, 5, TAU, G)
    assert not rej["accept"]
    assert np.array_equal(rej["sigma"], sigma) and np.array_equal(rej["pi"], pi)
    assert np.array_equal(rej["sigma_md"], out["sigma_md"])


def test_uniform_draws_range():
    u = uniform_draws(5005, 1000)
    assert u.min() >= 0.0 and u.max() < 1.0
