"""Pseudofermion action, fermion force and leapfrog MD (oracle; test infrastructure).

Paper, Sec. 1 (phi-algorithm):
  S_p[sigma] = phi^dagger Q^{-1} phi, Q = M^dagger M,
  H = sum pi^2 / 2 + S_p,
  the force involves phi^dagger Q^{-1} (dQ/dsigma) Q^{-1} phi.

Derivative (the plain definition written out): with X = Q^{-1} phi,
  dS/dsigma(n,t) = -X^dagger (dQ/dsigma(n,t)) X = -2 Re[(M X)^dagger (dM/dsigma(n,t)) X].
M depends on sigma(n,t) through the single column (n, t) of block (t+1, t):
  dM/dsigma(n,t) = s_t A cos sigma(n,t) e^{-tau K} e_n  placed in slice t+1,
so dS/dsigma(n,t) = -2 A cos sigma(n,t) s_t Re[X_t(n) conj((e^{-tau K} (M X)_{t+1})(n))].
Reading: the paper's F omits the sign; the MD equation used is
pi_dot = -dS/dsigma.
"""
from __future__ import annotations

import numpy as np

from .operator import apply_M, apply_Mdag, apply_expK, coupling_A, field_b


def action(phi, sigma, tau, g, solve_Mdag):
    """S = phi^H Q^{-1} phi = ||y||^2 with M^dagger y = phi.

    ``solve_Mdag(rhs)`` must return M^{-dagger} rhs (dense or iterative).
    """
    y = solve_Mdag(phi)
    return float(np.vdot(y, y).real), y


def gradient(X, sigma, tau, g, disp="free"):
    """dS/dsigma for X = Q^{-1} phi (formula in the module docstring); disp as
    in oracle.operator."""
    A = coupling_A(tau, g)
    ntau = sigma.shape[0]
    MX = apply_M(X, sigma, tau, g, disp)
    out = np.empty_like(sigma)
    for t in range(ntau):
        s = 1.0 if t == ntau - 1 else -1.0
        Ty = apply_expK(MX[(t + 1) % ntau], tau, disp, sigma.ndim - 1)
        out[t] = -2.0 * A * np.cos(sigma[t]) * s * np.real(X[t] * np.conj(Ty))
    return out


def exact_difference(phi_y, sigma, tau, g, site, h, solve_MdagT_unit):
    """S(sigma + h e) - S(sigma) without cancellation (Sherman-Morrison).

    Changing sigma at one site (n, t) changes one column of M:
    M' = M + a e^T with a = s_t (b'(n,t) - b(n,t)) e^{-tau K} e_n in slice t+1.
    With y = M^{-T} phi and z = M^{-T} e:
      y' = y - c z,  c = a^T y / (1 + a^T z),
      S' - S = -2 Re(conj(c) z^T y) + |c|^2 ||z||^2.
    ``solve_MdagT_unit(site)`` returns z (real). ``phi_y`` is y.
    """
    A = coupling_A(tau, g)
    ntau, nx, d = sigma.shape[0], sigma.shape[-1], sigma.ndim - 1
    t, n = site
    s = 1.0 if t == ntau - 1 else -1.0
    flat = sigma[t].reshape(-1)
    db = A * (np.sin(flat[n] + h) - np.sin(flat[n]))
    e_n = np.zeros(nx ** d)
    e_n[n] = 1.0
    col = apply_expK(e_n.reshape((nx,) * d), tau, "free", d).real.reshape(-1)
    a = np.zeros((ntau, nx ** d))
    a[(t + 1) % ntau] = s * db * col
    a = a.reshape(sigma.shape)
    z = solve_MdagT_unit(site)
    y = phi_y
    aty = np.sum(a * y)
    atz = np.sum(a * z)
    c = aty / (1.0 + atz)
    zy = np.sum(z * y)
    return float(-2.0 * np.real(np.conj(c) * zy) + abs(c) ** 2 * np.sum(z * z))


def leapfrog(sigma, pi, dt, nsteps, grad_fn):
    """Leapfrog (reversible, symplectic) integration of sigma_dot = pi,
    pi_dot = -dS/dsigma. ``grad_fn(sigma)`` returns dS/dsigma."""
    sigma = np.array(sigma, copy=True)
    pi = np.array(pi, copy=True)
    pi = pi - 0.5 * dt * grad_fn(sigma)
    for step in range(nsteps):
        sigma = sigma + dt * pi
        if step != nsteps - 1:
            pi = pi - dt * grad_fn(sigma)
    pi = pi - 0.5 * dt * grad_fn(sigma)
    return sigma, pi


def hamiltonian(pi, S):
    """H = sum pi^2 / 2 + S (paper, Sec. 1)."""
    return float(0.5 * np.sum(pi * pi) + S)


__all__ = ["action", "gradient", "exact_difference", "leapfrog", "hamiltonian",
           "apply_Mdag", "field_b"]
