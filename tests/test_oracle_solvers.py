"""Pins for the oracle's solvers (paper, Sec. 1, Eqs. 1-3) and the paper tables."""
import csv
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle import operator as op
from oracle import precond as pc
from oracle import solvers, costmodel
from synthetic import sigma_field, gaussian_rhs, WORKLOADS

TAU, G = 0.05, 5.0
HERE = os.path.dirname(__file__)


def _ops(sigma):
    return (lambda v: oracle.apply_M(v, sigma, TAU, G),
            lambda v: oracle.apply_Mdag(v, sigma, TAU, G))


def test_lattice_4x40_against_dense_lu():
    w = WORKLOADS["lattice_4x40"]
    sigma = sigma_field(w["nx"], w["ntau"], w["sigma_seed"])
    b = gaussian_rhs(w["nx"], w["ntau"], w["rhs_seeds"])[0]
    Md = op.dense_M(sigma, TAU, G)
    x_lu = solvers.dense_two_step(Md, b.ravel()).reshape(b.shape)
    M, Mt = _ops(sigma)
    x_cg, st = solvers.solve_cg_normal(b, M, Mt, tol=1e-10)
    assert st["status"] == 0 and st["relres"] <= 1e-10
    x_bi, st2 = solvers.solve_two_step(b, M, Mt, tol=1e-10)
    assert st2["status"] == 0 and max(st2["relres_steps"]) <= 1e-10
    nrm = np.linalg.norm(x_lu)
    # forward error <= cond(Q) * relres; cond(Q) of this lattice is ~1e3-1e4
    assert np.linalg.norm(x_cg - x_lu) / nrm < 1e-6
    assert np.linalg.norm(x_bi - x_lu) / nrm < 1e-6
    x_tight, _ = solvers.solve_two_step(b, M, Mt, tol=1e-14, maxit=4000)
    assert np.linalg.norm(x_tight - x_lu) / nrm < 1e-10


def test_preconditioned_variants_reach_the_same_solution():
    nx, ntau = 4, 16
    sigma = sigma_field(nx, ntau, 51)
    b = gaussian_rhs(nx, ntau, [52])[0]
    M, Mt = _ops(sigma)
    Md = op.dense_M(sigma, TAU, G)
    x_ref = solvers.dense_two_step(Md, b.ravel()).reshape(b.shape)
    lam_max = 1.05 * np.linalg.eigvalsh(Md.T @ Md)[-1]
    D, L = pc.sca_setup(sigma, TAU, G, 1.0)
    variants = {
        "cheb8": lambda r: pc.apply_cheb(r, sigma, TAU, G, 8, 1e-2, lam_max),
        "sca": lambda r: pc.sca_apply(r, D, L),
        "wce_wwt": lambda r: pc.wce_apply(pc.wce_apply_dag(r, sigma, TAU, G, 1), sigma, TAU, G, 1),
    }
    it_plain = solvers.solve_cg_normal(b, M, Mt, tol=1e-12)[1]["iters"]
    for name, P in variants.items():
        x, st = solvers.solve_cg_normal(b, M, Mt, tol=1e-12, precond=P)
        assert st["status"] == 0, name
        assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8, name
        if name == "cheb8":
            assert st["iters"] < it_plain
    for d in (0, 1, 2):
        for eu in (False, True):
            x, st = solvers.solve_two_step(
                b, M, Mt, tol=1e-12,
                precond_M=lambda r: pc.wce_apply(r, sigma, TAU, G, d, eu),
                precond_Mdag=lambda r: pc.wce_apply_dag(r, sigma, TAU, G, d, eu))
            assert st["status"] == 0
            assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8


def test_wce_reduces_bicgstab_iterations():
    nx, ntau = 4, 40
    sigma = sigma_field(nx, ntau, 53)
    b = gaussian_rhs(nx, ntau, [54])[0]
    M, Mt = _ops(sigma)
    plain = solvers.solve_two_step(b, M, Mt, tol=1e-10)[1]["iters"]
    wce2 = solvers.solve_two_step(
        b, M, Mt, tol=1e-10,
        precond_M=lambda r: pc.wce_apply(r, sigma, TAU, G, 2),
        precond_Mdag=lambda r: pc.wce_apply_dag(r, sigma, TAU, G, 2))[1]["iters"]
    assert wce2 < plain


def test_scipy_gmres_cross_check():
    nx, ntau = 4, 12
    sigma = sigma_field(nx, ntau, 55)
    b = gaussian_rhs(nx, ntau, [56])[0]
    M, Mt = _ops(sigma)
    n = b.size
    Aop = spla.LinearOperator((n, n), dtype=np.complex128,
                              matvec=lambda v: M(v.reshape(b.shape)).ravel())
    x_g, info = spla.gmres(Aop, b.ravel(), rtol=1e-13, restart=200, maxiter=50)
    assert info == 0
    x_b, st = solvers.bicgstab(M, b, tol=1e-13)
    assert st["status"] == 0
    assert np.linalg.norm(x_b.ravel() - x_g) / np.linalg.norm(x_g) < 1e-10


def _read_table(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        rows = [r for r in csv.reader(line for line in f if not line.startswith("#"))]
    head, body = rows[0], rows[1:]
    return [dict(zip(head, r)) for r in body]


def test_paper_mv_table_follows_cost_model():
    # Table 2 = Table 1 x the MV-per-iteration model of Sec. 5
    t1 = _read_table("paper_table1_iterations.csv")
    t2 = _read_table("paper_table2_mv.csv")
    cols = [("cheb8", "cheb", 8), ("cheb16", "cheb", 16), ("cheb32", "cheb", 32),
            ("sca", "sca", 0), ("wce0", "wce", 0), ("wce1", "wce", 1), ("wce2", "wce", 2)]
    mismatches = []
    for r1, r2 in zip(t1, t2):
        for col, meth, deg in cols:
            if r1[col] == "-":
                assert r2[col] == "-"
                continue
            mv = costmodel.mv_count(meth, int(r1[col]), deg)
            if mv != int(r2[col]):
                mismatches.append((r1["nx"], r1["ntau"], col, mv, int(r2[col])))
        cg = [int(r2[c]) for c in ("cheb8", "cheb16", "cheb32", "sca") if r2[c] != "-"]
        assert int(r2["gain"]) == int(np.floor(min(cg) / int(r2["wce0"]) + 0.5))
    # the only mismatch is the printed 21,313 (model: 7,104 x 3 = 21,312)
    assert mismatches == [("10", "100", "sca", 21312, 21313)]


def test_split_cg_against_dense_lu_and_pcg_iterates():
    """solve_cg_split (E = M0^{-1} right, E^dagger left; Sec. 5 after Table 2):
    (i) its solution is the dense-LU solution of M^T M x = b; (ii) in exact
    arithmetic split CG is PCG with P = E E^dagger, so after k iterations both
    hold the same iterate x_k (k = 1..4, against the oracle's cg with that
    preconditioner) -- a missing E^dagger on the right-hand side or a missing E
    on the result changes the iterates. (M0 is normal, so E E^dagger =
    E^dagger E and the order of the two factors cannot be told apart here.)"""
    nx, ntau = 2, 8
    sigma = sigma_field(nx, ntau, 71)
    b = gaussian_rhs(nx, ntau, [72])[0]
    M, Mt = _ops(sigma)
    E = lambda v: oracle.apply_M0inv(v, TAU)  # noqa: E731
    Ed = lambda v: oracle.apply_M0inv_dag(v, TAU)  # noqa: E731
    Md = op.dense_M(sigma, TAU, G)
    x_lu = solvers.dense_two_step(Md, b.ravel()).reshape(b.shape)
    x, st = solvers.solve_cg_split(b, M, Mt, E, Ed, tol=1e-13, maxit=2000)
    assert st["status"] == 0
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-9
    Q = lambda v: Mt(M(v))  # noqa: E731
    for k in range(1, 5):
        xs, _ = solvers.solve_cg_split(b, M, Mt, E, Ed, tol=1e-30, maxit=k)
        xp, _ = solvers.cg(Q, b, tol=1e-30, maxit=k, precond=lambda r: E(Ed(r)))
        assert np.linalg.norm(xs - xp) / np.linalg.norm(xp) < 1e-11, k
    # without the final x = E z the iterate is z, not x
    Ap = lambda z: Ed(Mt(M(E(z))))  # noqa: E731
    z3, _ = solvers.cg(Ap, Ed(b), tol=1e-30, maxit=3)
    xs3, _ = solvers.solve_cg_split(b, M, Mt, E, Ed, tol=1e-30, maxit=3)
    assert np.linalg.norm(z3 - xs3) / np.linalg.norm(xs3) > 1e-3
    assert np.linalg.norm(E(z3) - xs3) / np.linalg.norm(xs3) < 1e-13
