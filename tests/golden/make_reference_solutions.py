"""Write oracle reference solutions for the GPU solve tests (calls only oracle/).

For each workload the oracle solves M^T y = b, M x = y by its own FP64
BiCGStab, right-preconditioned with its weak-coupling series (order 2), to a
relative residual of 1e-13 per step, and stores a seeded sample of entries of
x together with ||x|| and the achieved residuals:

  lattice_8x160  : all 4 right-hand sides
  lattice_16x400 : all 8 right-hand sides
  lattice_12x200 : the force workload: X = M^{-1} eta (so that Q^{-1} phi = X
                   for phi = M^T eta) and the oracle gradient at 64 sites
  batched_64     : both right-hand sides of 8 of the 64 problems (drawn with
                   sample_sites(64, 8, 4900)), 512 sampled entries each

Independent right-hand sides are solved in parallel worker processes.

Run from the repository root: python tests/golden/make_reference_solutions.py [name ...]
Output: tests/golden/<name>_reference.npz
"""
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import precond as pc, solvers as osol, force  # noqa: E402
from synthetic import (sigma_field, gaussian_rhs, sample_sites, batched_problem_shapes,  # noqa: E402
                       WORKLOADS)

TAU, G = 0.05, 5.0
HERE = os.path.dirname(os.path.abspath(__file__))
NSAMPLE = 2048


def two_step(sigma, b):
    M = lambda v: oracle.apply_M(v, sigma, TAU, G)  # noqa: E731
    Mt = lambda v: oracle.apply_Mdag(v, sigma, TAU, G)  # noqa: E731
    x, st = osol.solve_two_step(
        b, M, Mt, tol=1e-13, maxit=3000,
        precond_M=lambda r: pc.wce_apply(r, sigma, TAU, G, 2),
        precond_Mdag=lambda r: pc.wce_apply_dag(r, sigma, TAU, G, 2))
    return x, st


def _solve_one(args):
    """Worker: two-step oracle solve of one right-hand side; returns the
    sampled entries, the norm of x and the residuals."""
    tag, nx, ntau, sigma_seed, rhs_seed, idx = args
    sigma = sigma_field(nx, ntau, sigma_seed)
    b = gaussian_rhs(nx, ntau, [rhs_seed])[0]
    t0 = time.time()
    x, st = two_step(sigma, b)
    print(f"{tag}: iters {st['iters_steps']} relres {st['relres_steps']} "
          f"{time.time() - t0:.0f} s", flush=True)
    return (x.reshape(-1)[idx], np.linalg.norm(x), np.array(st["relres_steps"]),
            st["relres_normal"])


def _workers():
    return max(1, min(8, len(os.sched_getaffinity(0))))


def lattice(name, rhs_index):
    w = WORKLOADS[name]
    nx, ntau = w["nx"], w["ntau"]
    N = nx ** 3 * ntau
    idx = sample_sites(N, NSAMPLE, 7000 + nx)
    out = dict(sample_index=idx)
    jobs = [(f"{name} rhs {k}", nx, ntau, w["sigma_seed"], w["rhs_seeds"][k], idx)
            for k in rhs_index]
    with ProcessPoolExecutor(max_workers=_workers()) as ex:
        res = list(ex.map(_solve_one, jobs))
    for k, (xs, xn, rr, rn) in zip(rhs_index, res):
        out[f"x{k}_sample"] = xs
        out[f"x{k}_norm"] = xn
        out[f"x{k}_relres"] = rr
        out[f"x{k}_relres_normal"] = rn
    np.savez(os.path.join(HERE, f"{name}_reference.npz"), **out)


def batched_workload(nsample=512):
    w = WORKLOADS["batched_64"]
    shapes = batched_problem_shapes(w["count"], w["shape_seed"])
    probs = sample_sites(w["count"], 8, 4900)
    jobs, keys = [], []
    out = dict(problems=probs)
    for i in probs:
        nx, ntau = shapes[i]
        idx = sample_sites(nx ** 3 * ntau, nsample, 4950 + int(i))
        out[f"p{i}_sample_index"] = idx
        for k in range(w["nrhs"]):
            jobs.append((f"batched problem {i} ({nx}^3 x {ntau}) rhs {k}", nx, ntau,
                         w["sigma_seed0"] + int(i), w["rhs_seed0"] + w["nrhs"] * int(i) + k, idx))
            keys.append(f"p{i}_x{k}")
    with ProcessPoolExecutor(max_workers=_workers()) as ex:
        res = list(ex.map(_solve_one, jobs))
    for key, (xs, xn, rr, rn) in zip(keys, res):
        out[f"{key}_sample"] = xs
        out[f"{key}_norm"] = xn
        out[f"{key}_relres"] = rr
    np.savez(os.path.join(HERE, "batched_64_reference.npz"), **out)


def force_workload():
    w = WORKLOADS["lattice_12x200"]
    nx, ntau = w["nx"], w["ntau"]
    sigma = sigma_field(nx, ntau, w["sigma_seed"])
    eta = gaussian_rhs(nx, ntau, [w["eta_seed"]])[0]
    M = lambda v: oracle.apply_M(v, sigma, TAU, G)  # noqa: E731
    t0 = time.time()
    X, st = osol.bicgstab(M, eta, tol=1e-13, maxit=3000,
                          precond=lambda r: pc.wce_apply(r, sigma, TAU, G, 2))
    print(f"force X: iters {st['iters']} relres {st['relres']} {time.time() - t0:.0f} s", flush=True)
    grad = force.gradient(X, sigma, TAU, G)
    N = nx ** 3 * ntau
    sites = sample_sites(N, 64, w["site_seed"])
    np.savez(os.path.join(HERE, "lattice_12x200_reference.npz"), sites=sites,
             grad_sample=grad.reshape(-1)[sites], grad_norm=np.linalg.norm(grad),
             X_relres=st["relres"], action=float(np.vdot(eta, eta).real))


if __name__ == "__main__":
    names = sys.argv[1:] or ["lattice_8x160", "lattice_12x200", "lattice_16x400", "batched_64"]
    for n in names:
        if n == "lattice_8x160":
            lattice(n, [0, 1, 2, 3])
        elif n == "lattice_16x400":
            lattice(n, list(range(8)))
        elif n == "lattice_12x200":
            force_workload()
        elif n == "batched_64":
            batched_workload()
