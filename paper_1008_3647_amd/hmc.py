"""Markov chain of phi-algorithm HMC trajectories (paper, Sec. 1) with
checkpoint / resume and a JSON-lines log.

Every trajectory runs in the library (`Lattice.hmc_trajectory`: heat bath,
leapfrog, Metropolis); this module draws the trajectory's random inputs (MD
momenta, the pseudofermion source eta, the Metropolis draw u) from a numpy
PCG64 generator on the host and keeps the chain's bookkeeping. A checkpoint
(.npz) holds sigma, the trajectory index, the step size, the acceptance count
and the generator state, so a resumed chain continues bit for bit: the
library's kernels use fixed summation orders, and the draws resume where they
stopped.
"""
from __future__ import annotations

import json

import numpy as np
import torch

from .lattice import Lattice, Precond


class HMCChain:
    def __init__(self, lattice: Lattice, sigma, seed: int, dt: float, nsteps: int,
                 precond: Precond | None = None, tol: float = 1e-10, nphi: int = 1,
                 mixed: bool = False, log_path: str | None = None):
        self.L = lattice
        self.sigma = sigma.detach().clone().contiguous()
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.dt, self.nsteps, self.precond, self.tol = float(dt), int(nsteps), precond, tol
        self.nphi, self.mixed = int(nphi), bool(mixed)
        self.trajectory = 0
        self.accepted = 0
        self.log_path = log_path

    def _draws(self):
        shape = self.L.shape
        pi = self.rng.standard_normal(shape)
        eta = (self.rng.standard_normal((self.nphi,) + shape)
               + 1j * self.rng.standard_normal((self.nphi,) + shape)) / np.sqrt(2.0)
        u = float(self.rng.random())
        dev = self.sigma.device
        return (torch.from_numpy(pi).to(dev), torch.from_numpy(eta).to(dev, self.L.dtype), u)

    def step(self):
        """One trajectory; returns its result record (and appends it to the log)."""
        pi, eta, u = self._draws()
        self.sigma, _, info = self.L.hmc_trajectory(self.sigma, pi, eta, u, self.dt,
                                                    self.nsteps, self.precond, tol=self.tol,
                                                    mixed=self.mixed)
        if info["status"] != 0:
            raise RuntimeError(f"trajectory {self.trajectory}: solve status {info['status']}")
        self.trajectory += 1
        self.accepted += int(info["accept"])
        rec = {k: info[k] for k in ("dH", "S0", "S1", "K0", "K1", "accept", "solves", "iters",
                                    "seconds")}
        rec.update(trajectory=self.trajectory, dt=self.dt, u=u)
        if self.log_path:
            with open(self.log_path, "a") as f:
                f.write(json.dumps(rec) + "\n")
        return rec

    def run(self, ntraj: int):
        return [self.step() for _ in range(int(ntraj))]

    def save(self, path: str):
        state = json.dumps(self.rng.bit_generator.state)
        np.savez(path, sigma=self.sigma.cpu().numpy(), trajectory=self.trajectory,
                 accepted=self.accepted, dt=self.dt, nsteps=self.nsteps, nphi=self.nphi,
                 rng_state=np.array(state))

    def load(self, path: str):
        with np.load(path, allow_pickle=False) as d:
            if tuple(d["sigma"].shape) != self.L.shape:
                raise ValueError(f"checkpoint sigma has shape {d['sigma'].shape}, "
                                 f"lattice {self.L.shape}")
            self.sigma = torch.from_numpy(d["sigma"]).to(self.sigma.device)
            self.trajectory = int(d["trajectory"])
            self.accepted = int(d["accepted"])
            self.dt = float(d["dt"])
            self.nsteps = int(d["nsteps"])
            self.nphi = int(d["nphi"])
            self.rng.bit_generator.state = json.loads(str(d["rng_state"]))
        return self
