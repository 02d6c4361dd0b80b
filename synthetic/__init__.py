"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This module holds no arithmetic of the method itself: it only draws the
random numbers the workloads are made of, so that the oracle and the HIP path
see bit-identical inputs.

Workload recipe (paper, Sec. 5 "Results"): the auxiliary field sigma is drawn
iid uniform on [-pi, pi] per space-time site; right-hand sides are complex
Gaussian vectors (Re and Im iid N(0, 1/2), the heat-bath law exp(-eta^H eta)).
All generators use numpy's PCG64 (``numpy.random.default_rng``).

Array layouts (C order), spatial dimension dim = 3 by default (1 and 2 for
the lower-dimensional lattices):
  sigma : float64 [ntau][nx]^dim
  rhs   : complex128 [nrhs][ntau][nx]^dim
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "sigma_field",
    "gaussian_rhs",
    "gaussian_momenta",
    "uniform_draws",
    "sweep_seeds",
    "batched_problem_shapes",
    "sample_sites",
    "WORKLOADS",
]


def sigma_field(nx: int, ntau: int, seed: int, dim: int = 3) -> np.ndarray:
    """Auxiliary field, iid uniform on [-pi, pi] per site (paper, Sec. 5)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=(ntau,) + (nx,) * dim)


def gaussian_rhs(nx: int, ntau: int, seeds, dim: int = 3) -> np.ndarray:
    """Complex Gaussian right-hand sides, one seed per RHS.

    Re and Im are iid N(0, 1/2) so that the density is proportional to
    exp(-|eta|^2), the pseudofermion heat-bath law (paper, Sec. 1).
    """
    seeds = list(seeds)
    shape = (ntau,) + (nx,) * dim
    out = np.empty((len(seeds),) + shape, dtype=np.complex128)
    for i, s in enumerate(seeds):
        rng = np.random.default_rng(s)
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        out[i] = (re + 1j * im) / np.sqrt(2.0)
    return out


def gaussian_momenta(nx: int, ntau: int, seed: int, dim: int = 3) -> np.ndarray:
    """MD momenta pi ~ N(0, 1) per site (paper, Sec. 1, MD Hamiltonian)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ntau,) + (nx,) * dim)


def uniform_draws(seed: int, count: int) -> np.ndarray:
    """Metropolis draws u, iid uniform on [0, 1) (paper, Sec. 1, accept/reject)."""
    rng = np.random.default_rng(seed)
    return rng.random(count)


def sweep_seeds(w, nx: int, ntau: int, k: int):
    """(sigma seed, rhs seed) of configuration k of the paper-sweep workload."""
    off = 10000 * k + 100 * nx + ntau // 10
    return w["sigma_seed0"] + off, w["rhs_seed0"] + off


def batched_problem_shapes(count: int = 64, seed: int = 4000):
    """Uneven lattice shapes for the batched workload.

    Nx drawn from {6, 8, 10, 12}, Ntau from {80, 120, ..., 320}.
    Returns a list of (nx, ntau) tuples.
    """
    rng = np.random.default_rng(seed)
    nxs = rng.choice([6, 8, 10, 12], size=count)
    nts = rng.choice(np.arange(80, 321, 40), size=count)
    return [(int(a), int(b)) for a, b in zip(nxs, nts)]


def sample_sites(n_sites: int, count: int, seed: int) -> np.ndarray:
    """Distinct flat site indices drawn without replacement."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_sites, size=count, replace=False))


# Named workloads (seeds and shapes); physics tau = 0.05, g = 5.0 throughout.
WORKLOADS = {
    # plain FP64 method, dense-LU checkable
    "lattice_4x40": dict(nx=4, ntau=40, sigma_seed=1001, rhs_seeds=[1002]),
    # preconditioner grid, 4 RHS
    "lattice_8x160": dict(nx=8, ntau=160, sigma_seed=2001,
                          rhs_seeds=[2002, 2003, 2004, 2005]),
    # precision comparison at Nx=16, Ntau=400, 8 RHS
    "lattice_16x400": dict(nx=16, ntau=400, sigma_seed=3001,
                           rhs_seeds=list(range(3002, 3010))),
    # 64 uneven lattices (shapes from batched_problem_shapes(64, 4000)), sigma
    # seed 4001 + i and right-hand-side seeds 4101 + 2 i, 4102 + 2 i for problem i
    "batched_64": dict(count=64, shape_seed=4000, sigma_seed0=4001, rhs_seed0=4101, nrhs=2),
    # force / molecular dynamics at Nx=12, Ntau=200
    "lattice_12x200": dict(nx=12, ntau=200, sigma_seed=5001, eta_seed=5002,
                           site_seed=5003, momentum_seed=5004, metropolis_seed=5005),
    # the paper's sweeps (Tables 1 and 3): 10 random sigma per lattice and
    # coupling, one random right-hand side each; sigma seed
    # sigma_seed0 + 10000 k + 100 nx + ntau / 10 for configuration k (rhs: rhs_seed0 + same)
    "paper_sweeps": dict(sigma_seed0=600000, rhs_seed0=700000, nsigma=10,
                         shapes=[(6, 50), (8, 50), (10, 50), (6, 100), (8, 100), (10, 100),
                                 (6, 200), (8, 200), (10, 200)]),
}
TAU = 0.05
G_COUPLING = 5.0
