"""Krylov solvers of the paper (oracle; test infrastructure).

Paper, Sec. 1:
  Eq. (1) M^dagger M x = b solved by CG on the normal equations;
  Eq. (2) M^dagger y = b followed by M x = y, solved by BiCGStab;
  Eq. (3) preconditioning with P ~ (M^dagger M)^{-1} (left form for CG).

Readings (the paper names the methods but prints no variant):
  * CG with a Hermitian positive-definite P is textbook preconditioned CG.
  * BiCGStab is van der Vorst's method with shadow residual r^ = r_0 and
    right preconditioning (so the recursively updated residual is the
    residual of the original system); on a breakdown (rho = 0) it restarts
    with r^ = r.
  * Stop when ||r|| / ||b|| <= tol with x_0 = 0 (the paper's "reduction of
    the residual norm"); the returned residual is recomputed from scratch.
  * Iterations of the two-step BiCGStab are the sum over both solves.

Complex vectors use <a, b> = a^H b.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a, b)


def _norm(a):
    return float(np.sqrt(np.vdot(a, a).real))


def cg(apply_A, b, tol=1e-10, maxit=10000, precond=None, x0=None):
    """Preconditioned CG for a Hermitian positive-definite operator."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, copy=True)
    r = b - apply_A(x)
    z = precond(r) if precond else r
    p = z.copy()
    rz = _dot(r, z)
    bn = _norm(b)
    it = 0
    status = 1
    if _norm(r) <= tol * bn:
        status = 0
    while status and it < maxit:
        Ap = apply_A(p)
        alpha = rz / _dot(p, Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        it += 1
        if _norm(r) <= tol * bn:
            status = 0
            break
        z = precond(r) if precond else r
        rz_new = _dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, dict(iters=it, status=status,
                   relres=_norm(b - apply_A(x)) / bn)


def bicgstab(apply_A, b, tol=1e-10, maxit=10000, precond=None, x0=None):
    """Right-preconditioned BiCGStab (van der Vorst) for A x = b."""
    K = precond if precond else (lambda v: v)
    x = np.zeros_like(b) if x0 is None else np.array(x0, copy=True)
    r = b - apply_A(x)
    rhat = r.copy()
    rho_old = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    bn = _norm(b)
    it = 0
    status = 0 if _norm(r) <= tol * bn else 1
    while status and it < maxit:
        rho = _dot(rhat, r)
        if rho == 0:
            rhat = r.copy()
            rho = _dot(rhat, r)
            p = np.zeros_like(b)
            v = np.zeros_like(b)
            rho_old = alpha = omega = 1.0 + 0j
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        phat = K(p)
        v = apply_A(phat)
        alpha = rho / _dot(rhat, v)
        s = r - alpha * v
        it += 1
        if _norm(s) <= tol * bn:
            x = x + alpha * phat
            r = s
            status = 0
            break
        shat = K(s)
        t = apply_A(shat)
        omega = _dot(t, s) / _dot(t, t)
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        rho_old = rho
        if _norm(r) <= tol * bn:
            status = 0
    return x, dict(iters=it, status=status,
                   relres=_norm(b - apply_A(x)) / bn)


def solve_cg_normal(b, apply_M, apply_Mdag, tol=1e-10, maxit=10000, precond=None):
    """x = (M^dagger M)^{-1} b by (P)CG (paper, Eq. 1 and Eq. 3)."""
    Q = lambda v: apply_Mdag(apply_M(v))  # noqa: E731
    return cg(Q, b, tol, maxit, precond)


def solve_cg_split(b, apply_M, apply_Mdag, apply_E, apply_Edag, tol=1e-10, maxit=10000):
    """CG on the normal equations with split preconditioning (paper, Sec. 5,
    the remark after Table 2: (M0^dagger)^{-1} on the left and M0^{-1} on the
    right of M^dagger M). With E ~ M^{-1} (E = M0^{-1} in the paper, or any
    weak-coupling W_d) CG runs on the Hermitian positive-definite
    A' = E^dagger M^dagger M E with right-hand side b' = E^dagger b, and
    x = E z. The stop rule is CG's own residual, ||b' - A' z|| <= tol ||b'||;
    the residual of the original system is reported beside it."""
    Ap = lambda z: apply_Edag(apply_Mdag(apply_M(apply_E(z))))  # noqa: E731
    bp = apply_Edag(b)
    z, st = cg(Ap, bp, tol, maxit)
    x = apply_E(z)
    relq = _norm(b - apply_Mdag(apply_M(x))) / _norm(b)
    return x, dict(iters=st["iters"], status=st["status"], relres_split=st["relres"],
                   relres=relq)


def solve_two_step(b, apply_M, apply_Mdag, tol=1e-10, maxit=10000,
                   precond_M=None, precond_Mdag=None):
    """M^dagger y = b, then M x = y, each by BiCGStab (paper, Eq. 2)."""
    y, s1 = bicgstab(apply_Mdag, b, tol, maxit, precond_Mdag)
    x, s2 = bicgstab(apply_M, y, tol, maxit, precond_M)
    nb = _norm(b)
    relq = _norm(b - apply_Mdag(apply_M(x))) / nb
    return x, dict(iters=s1["iters"] + s2["iters"], iters_steps=(s1["iters"], s2["iters"]),
                   status=max(s1["status"], s2["status"]),
                   relres_steps=(s1["relres"], s2["relres"]), relres_normal=relq, y=y)


def dense_two_step(Md, b):
    """Dense LU route for tiny lattices: y = M^{-T} b, x = M^{-1} y."""
    y = np.linalg.solve(Md.T, b)
    return np.linalg.solve(Md, y)
