"""The phi-algorithm HMC trajectory through the C ABI (hmc_trajectory,
hmc_leapfrog) against the oracle's trajectory (oracle/hmc.py, dense solves).

Tiny lattice 4^3 x 6: a Markov chain of six trajectories (dt = 0.12, 5 steps;
the oracle accepts five and rejects the second) with the same seeded sigma,
momenta, eta and Metropolis draws on both sides. Per trajectory: the accept
decision is identical; dH agrees within 4 cond(M) tol (S0 + S1) + 1e-9 (each
S_p = ||y||^2 with y from a solve to relative residual tol carries at most
~2 cond(M) tol S relative error; the MD end points differ by far less); the
chain state (sigma, pi) agrees entry by entry within 1e-10; S0 equals ||eta||^2.
12^3 x 200: one trajectory with its acceptance and timing reported.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import hmc
from oracle import operator as op
from synthetic import (sigma_field, gaussian_rhs, gaussian_momenta, uniform_draws,
                       WORKLOADS)
from gpu_util import require_gpu, to_dev, to_host, rel_err, say, TAU, G

pytestmark = pytest.mark.gpu

NX, NT = 4, 6
DT, NSTEPS = 0.12, 5


def _chain_inputs(k):
    return (gaussian_momenta(NX, NT, 9410 + k), gaussian_rhs(NX, NT, [9420 + k]))


@pytest.mark.parametrize("mixed,chrono", [(False, True), (False, False), (True, True)])
def test_chain_matches_oracle(mixed, chrono):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    tol = 1e-12 if mixed else 1e-13
    sigma = sigma_field(NX, NT, 9400)
    us = uniform_draws(9401, 6)
    L = Lattice(NX, NT, TAU, G, torch.complex128)
    s_o, s_g = sigma.copy(), to_dev(sigma)
    decisions = []
    for k in range(6):
        pi, eta = _chain_inputs(k)
        ref = hmc.fermion_trajectory(s_o, pi, eta, us[k], DT, NSTEPS, TAU, G)
        s_g, p_g, info = L.hmc_trajectory(s_g, to_dev(pi), to_dev(eta), us[k], DT, NSTEPS,
                                          tol=tol, mixed=mixed, chrono=chrono)
        kappa = np.linalg.cond(op.dense_M(s_o, TAU, G))
        bound = 4 * kappa * tol * (ref["S0"] + ref["S1"]) + 1e-9
        say(f"traj {k}: dH gpu {info['dH']:+.10f} oracle {ref['dH']:+.10f} "
            f"(|diff| {abs(info['dH'] - ref['dH']):.1e}, bound {bound:.1e}) u {us[k]:.4f} "
            f"accept {info['accept']} iters {info['iters']} solves {info['solves']}")
        assert info["status"] == 0 and info["forces"] == NSTEPS + 1
        assert info["accept"] == int(ref["accept"])
        assert abs(info["dH"] - ref["dH"]) <= bound
        assert abs(us[k] - np.exp(-ref["dH"])) > 10 * bound  # the decision is not borderline
        assert info["S0"] == pytest.approx(float(np.sum(np.abs(eta) ** 2)), rel=1e-11)
        assert info["K0"] == pytest.approx(0.5 * float(np.sum(pi * pi)), rel=1e-14)
        assert np.allclose(info["actions"], ref["actions"], rtol=1e-10, atol=0)
        assert rel_err(to_host(s_g), ref["sigma"]) < 1e-10
        assert rel_err(to_host(p_g), ref["pi"]) < 1e-10
        decisions.append(info["accept"])
        s_o = ref["sigma"]
    assert decisions == [1, 0, 1, 1, 1, 1]


def test_two_pseudofermions_and_phi():
    """nphi = 2: S_p sums both; phi returned by the heat bath equals M^dagger eta."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(NX, NT, 9430)
    pi = gaussian_momenta(NX, NT, 9431)
    eta = gaussian_rhs(NX, NT, [9432, 9433])
    ref = hmc.fermion_trajectory(sigma, pi, eta, 0.3, 0.05, 6, TAU, G)
    L = Lattice(NX, NT, TAU, G, torch.complex128)
    s, p, info = L.hmc_trajectory(to_dev(sigma), to_dev(pi), to_dev(eta), 0.3, 0.05, 6,
                                  tol=1e-13, want_phi=True)
    say(f"nphi=2: dH gpu {info['dH']:+.3e} oracle {ref['dH']:+.3e}")
    assert rel_err(to_host(info["phi"]), ref["phi"]) < 1e-14
    assert info["accept"] == int(ref["accept"])
    assert abs(info["dH"] - ref["dH"]) < 1e-8
    assert rel_err(to_host(s), ref["sigma"]) < 1e-10


def test_reject_restores_start_and_field():
    """A draw just above exp(-dH) rejects: sigma and pi come back bit for bit and
    the installed field is the start's (apply_M after the call is M(sigma_0))."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    sigma = sigma_field(NX, NT, 9400)
    pi, eta = _chain_inputs(1)
    ref = hmc.fermion_trajectory(sigma, pi, eta, 0.0, DT, NSTEPS, TAU, G)
    assert ref["dH"] > 0.05
    u = float(np.exp(-ref["dH"]) * 1.01)
    L = Lattice(NX, NT, TAU, G, torch.complex128)
    s, p, info = L.hmc_trajectory(to_dev(sigma), to_dev(pi), to_dev(eta), u, DT, NSTEPS,
                                  tol=1e-13)
    assert info["accept"] == 0
    assert np.array_equal(to_host(s), sigma) and np.array_equal(to_host(p), pi)
    x = gaussian_rhs(NX, NT, [9440])
    y = to_host(L.apply_M(to_dev(x)))[0]
    assert rel_err(y, oracle.apply_M(x[0], sigma, TAU, G)) < 1e-14


def test_bad_arguments_raise():
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.lattice import UfgError
    sigma, (pi, eta) = sigma_field(NX, NT, 9400), _chain_inputs(0)
    L = Lattice(NX, NT, TAU, G, torch.complex128)
    args = (to_dev(sigma), to_dev(pi), to_dev(eta))
    for u, dt, n in ((1.0, 0.1, 2), (-0.1, 0.1, 2), (float("nan"), 0.1, 2), (0.5, 0.0, 2),
                     (0.5, float("inf"), 2), (0.5, 0.1, 0)):
        with pytest.raises(UfgError):
            L.hmc_trajectory(*args, u, dt, n)
    with pytest.raises(TypeError):
        L.hmc_trajectory(args[0].float(), args[1], args[2], 0.5, 0.1, 2)


def test_trajectory_12x200():
    """One trajectory on 12^3 x 200 (WCE2 + Euler preconditioned BiCGStab,
    tol 1e-12, dt = 0.0025, 20 steps): S0 = ||eta||^2, |dH| < 0.1, the decision
    is u < exp(-dH) and the returned state follows it; with and without
    chronological starting vectors the MD end points agree within 1e-9."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    w = WORKLOADS["lattice_12x200"]
    nx, ntau = w["nx"], w["ntau"]
    sigma = sigma_field(nx, ntau, w["sigma_seed"])
    eta = gaussian_rhs(nx, ntau, [w["eta_seed"]])
    pi = gaussian_momenta(nx, ntau, w["momentum_seed"])
    u = float(uniform_draws(w["metropolis_seed"], 1)[0])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    pc = Precond("wce", wce_order=2, euler=True)
    outs = {}
    for chrono in (True, False):
        s, p, info = L.hmc_trajectory(to_dev(sigma), to_dev(pi), to_dev(eta), u, 0.0025, 20,
                                      pc, tol=1e-12, chrono=chrono)
        say(f"12^3x200 chrono={chrono}: dH {info['dH']:+.4e} u {u:.4f} accept {info['accept']} "
            f"solves {info['solves']} iters {info['iters']} {info['seconds']:.2f}s "
            f"worst relres {info['worst_relres']:.1e}")
        assert info["status"] == 0
        assert info["S0"] == pytest.approx(float(np.vdot(eta, eta).real), rel=1e-10)
        assert abs(info["dH"]) < 0.1
        assert info["accept"] == int(u < np.exp(-info["dH"]))
        outs[chrono] = (to_host(s), to_host(p), info)
    (s1, p1, i1), (s0, p0, i0) = outs[True], outs[False]
    assert abs(i1["dH"] - i0["dH"]) < 1e-6
    if i1["accept"] and i0["accept"]:
        assert np.max(np.abs(s1 - s0)) < 1e-9 and np.max(np.abs(p1 - p0)) < 1e-9
    if not i1["accept"]:
        assert np.array_equal(s1, sigma)
    assert i1["iters"] < i0["iters"]  # chronological starting vectors save iterations


def test_chain_checkpoint_resume_is_bitwise(tmp_path):
    """HMCChain: a chain checkpointed after two trajectories and resumed in a
    fresh object (new lattice handle) continues bit for bit like the chain
    that ran straight through; the JSON-lines log holds one record per
    trajectory; every recorded decision equals u < exp(-dH)."""
    require_gpu()
    import json
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.hmc import HMCChain
    sigma = to_dev(sigma_field(NX, NT, 9450))
    log = tmp_path / "chain.jsonl"
    L = Lattice(NX, NT, TAU, G, torch.complex128)
    a = HMCChain(L, sigma, seed=9451, dt=DT, nsteps=NSTEPS, tol=1e-12, log_path=str(log))
    ra = a.run(4)
    b = HMCChain(Lattice(NX, NT, TAU, G, torch.complex128), sigma, seed=9451, dt=DT,
                 nsteps=NSTEPS, tol=1e-12)
    b.run(2)
    ck = tmp_path / "chain.npz"
    b.save(str(ck))
    c = HMCChain(Lattice(NX, NT, TAU, G, torch.complex128), sigma, seed=1, dt=0.5, nsteps=1,
                 tol=1e-12).load(str(ck))
    rc = c.run(2)
    assert c.trajectory == 4 and c.accepted == a.accepted
    assert torch.equal(c.sigma, a.sigma)
    assert [r["dH"] for r in rc] == [r["dH"] for r in ra[2:]]
    lines = [json.loads(x) for x in log.read_text().splitlines()]
    assert [r["trajectory"] for r in lines] == [1, 2, 3, 4]
    for r in lines:
        assert r["accept"] == int(r["u"] < np.exp(-r["dH"]))
