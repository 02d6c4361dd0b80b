"""Pseudofermion action and HMC force (paper, Sec. 1, the phi-algorithm).

S[sigma] = sum_r phi_r^dagger (M^dagger M)^{-1} phi_r = sum_r ||y_r||^2, M^dagger y_r = phi_r.

`Action` is a torch.autograd.Function: forward solves M^dagger y = phi
(BiCGStab in libufg) and returns S; backward solves M X = y (the one extra
solve; then X = Q^{-1} phi and y = M X) and calls the library's force
contraction
    dS/dsigma(n,t) = -2 A cos sigma(n,t) s_t sum_r Re[X_t(n) conj((e^{-tau K} y_{t+1})(n))].
`leapfrog` integrates sigma_dot = pi, pi_dot = -dS/dsigma with a reversible
symplectic leapfrog (libufg hmc_leapfrog); `Lattice.hmc_trajectory` adds the
heat bath and the Metropolis step.
"""
from __future__ import annotations

import torch

from .lattice import Lattice, Precond


class Action(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, phi, lattice: Lattice, precond, tol, mixed):
        lattice.set_aux_field(sigma.detach().contiguous())
        y, st = lattice.solve_bicgstab(phi, "Mdag", precond=precond, tol=tol, mixed=mixed)
        if st["status"] != 0:
            raise RuntimeError(f"M^dagger y = phi did not converge: {st}")
        S = sum(lattice.norm2(y))
        ctx.lattice, ctx.precond, ctx.tol, ctx.mixed = lattice, precond, tol, mixed
        ctx.save_for_backward(sigma, y)
        ctx.stats = st
        return torch.tensor(S, dtype=torch.float64, device=sigma.device)

    @staticmethod
    def backward(ctx, grad_S):
        sigma, y = ctx.saved_tensors
        L = ctx.lattice
        L.set_aux_field(sigma.detach().contiguous())
        X, st = L.solve_bicgstab(y, "M", precond=ctx.precond, tol=ctx.tol, mixed=ctx.mixed)
        if st["status"] != 0:
            raise RuntimeError(f"M X = y did not converge: {st}")
        g = L.force_dS_dsigma(X, y)
        return grad_S * g, None, None, None, None, None


def action(sigma, phi, lattice: Lattice, precond: Precond | None = None, tol=1e-11,
           mixed=False):
    """S[sigma] as a differentiable scalar (float64 tensor)."""
    return Action.apply(sigma, phi, lattice, precond, tol, mixed)


def force(sigma, phi, lattice: Lattice, precond=None, tol=1e-11, mixed=False):
    """(S, dS/dsigma) at sigma through the autograd function."""
    s = sigma.detach().clone().requires_grad_(True)
    S = action(s, phi, lattice, precond, tol, mixed)
    (g,) = torch.autograd.grad(S, s)
    return float(S.item()), g


def heat_bath_phi(lattice: Lattice, eta):
    """phi = M^dagger eta (eta ~ exp(-eta^dagger eta)), Sec. 1."""
    return lattice.apply_Mdag(eta)


def leapfrog(sigma, pi, phi, lattice: Lattice, dt, nsteps, precond=None, tol=1e-11,
             mixed=False, chrono=True):
    """Leapfrog MD trajectory (libufg hmc_leapfrog: every solve, force and
    field update in the library); returns (sigma, pi, list of S at every force)."""
    s, p, actions, res = lattice.hmc_leapfrog(sigma.contiguous(), pi.contiguous(), phi, dt,
                                              nsteps, precond, tol=tol, mixed=mixed,
                                              chrono=chrono)
    if res["status"] != 0:
        raise RuntimeError(f"a solve of the MD trajectory did not converge: {res}")
    return s, p, actions


def hamiltonian(pi, S):
    """H = sum pi^2 / 2 + S (Sec. 1)."""
    return float(0.5 * torch.sum(pi * pi).item() + S)
