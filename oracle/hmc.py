"""One HMC trajectory of the phi-algorithm (oracle; test infrastructure).

Paper, Sec. 1 (the phi-algorithm): the pseudofermion field phi is drawn from a
Gaussian heat bath and held fixed while the auxiliary field sigma and its
conjugate momentum pi follow the classical equations of motion of the MD
Hamiltonian H = sum pi^2 / 2 + S_p[sigma], S_p = phi^dagger Q^{-1} phi,
Q = M^dagger M, integrated by a reversible symplectic scheme; a Metropolis
accept/reject step at the end of the trajectory removes the step-size error.

Readings (the paper leaves these to the implementation):
  heat bath   phi_r = M^dagger eta_r with eta_r ~ exp(-eta^dagger eta): then
              phi ~ exp(-phi^dagger Q^{-1} phi) and S_p at the start equals
              sum_r ||eta_r||^2 exactly.
  integrator  leapfrog, kick-drift-kick with half kicks at both ends (the
              same scheme as oracle.force.leapfrog), pi_dot = -dS/dsigma.
  Metropolis  accept with probability min(1, exp(-dH)), dH = H_end - H_start:
              with u uniform on [0, 1), accept iff u < exp(-dH). On a reject
              the chain stays at the start (sigma and pi of the start are
              returned; pi is redrawn before the next trajectory anyway).
  inputs      every random number the method draws (eta, pi, u) is an input.
"""
from __future__ import annotations

import numpy as np

from .operator import apply_Mdag, dense_M
from .force import gradient


def heat_bath(eta, sigma, tau, g):
    """phi_r = M^dagger eta_r for every pseudofermion r (eta: [nphi][Ntau][Nx]^d)."""
    return np.stack([apply_Mdag(e, sigma, tau, g) for e in eta])


def dense_action_grad(phi, tau, g):
    """Returns action_grad(sigma) -> (S_p, dS/dsigma) by dense solves (tiny lattices):
    y_r = M^{-dagger} phi_r, S_p = sum_r ||y_r||^2, X_r = M^{-1} y_r = Q^{-1} phi_r,
    gradient from oracle.force.gradient."""
    shape = phi.shape[1:]

    def action_grad(sigma):
        Md = dense_M(sigma, tau, g)
        S = 0.0
        grad = np.zeros(shape[:1] + shape[1:], dtype=np.float64)
        for p in phi:
            y = np.linalg.solve(Md.T, p.reshape(-1))
            X = np.linalg.solve(Md, y)
            S += float(np.vdot(y, y).real)
            grad += gradient(X.reshape(shape), sigma, tau, g)
        return S, grad

    return action_grad


def kinetic(pi):
    """sum pi^2 / 2 (the momentum part of H, Sec. 1)."""
    return float(0.5 * np.sum(pi * pi))


def metropolis(dH, u):
    """Accept iff u < exp(-dH), u uniform on [0, 1): probability min(1, exp(-dH))."""
    return bool(u < np.exp(-dH))


def md(sigma, pi, dt, nsteps, action_grad):
    """Leapfrog trajectory of nsteps steps of size dt (nsteps + 1 forces).
    Returns sigma, pi at the end and the action at every force evaluation."""
    sigma = np.array(sigma, dtype=np.float64, copy=True)
    pi = np.array(pi, dtype=np.float64, copy=True)
    S, grad = action_grad(sigma)
    actions = [S]
    pi -= 0.5 * dt * grad
    for step in range(nsteps):
        sigma += dt * pi
        S, grad = action_grad(sigma)
        actions.append(S)
        pi -= (0.5 * dt if step == nsteps - 1 else dt) * grad
    return sigma, pi, actions


def trajectory(sigma, pi, u, dt, nsteps, action_grad):
    """One trajectory from (sigma, pi): MD, then Metropolis with the draw u.

    Returns a dict: sigma, pi (the chain's next state: the MD end point if
    accepted, else the start), sigma_md, pi_md (the MD end point), S0, S1, K0,
    K1, H0, H1, dH, accept, actions.
    """
    sigma_md, pi_md, actions = md(sigma, pi, dt, nsteps, action_grad)
    K0, K1 = kinetic(pi), kinetic(pi_md)
    S0, S1 = actions[0], actions[-1]
    H0, H1 = K0 + S0, K1 + S1
    dH = (K1 - K0) + (S1 - S0)
    acc = metropolis(dH, u)
    return dict(sigma=sigma_md if acc else np.array(sigma, dtype=np.float64, copy=True),
                pi=pi_md if acc else np.array(pi, dtype=np.float64, copy=True),
                sigma_md=sigma_md, pi_md=pi_md, S0=S0, S1=S1, K0=K0, K1=K1,
                H0=H0, H1=H1, dH=dH, accept=acc, actions=actions)


def fermion_trajectory(sigma, pi, eta, u, dt, nsteps, tau, g):
    """The phi-algorithm trajectory on a tiny lattice: heat bath phi = M^dagger eta
    at the starting sigma, then trajectory() with dense solves."""
    phi = heat_bath(eta, sigma, tau, g)
    out = trajectory(sigma, pi, u, dt, nsteps, dense_action_grad(phi, tau, g))
    out["phi"] = phi
    return out


__all__ = ["heat_bath", "dense_action_grad", "kinetic", "metropolis", "md", "trajectory",
           "fermion_trajectory"]
