"""Batched two-step BiCGStab (solve_batched): many uneven lattices in one
persistent, graph-replayed pass. Each (problem, rhs) must reach the same
solution as the unbatched solve of that problem and meet the tolerance on the
residuals recomputed by the oracle's M.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import operator as op
from oracle import solvers as osol
from synthetic import sigma_field, gaussian_rhs, batched_problem_shapes, WORKLOADS
from gpu_util import require_gpu, to_dev, to_host, say, TAU, G

pytestmark = pytest.mark.gpu


def _problems(shapes, sigma_seed0, rhs_seed0, nrhs):
    out = []
    for i, (nx, ntau) in enumerate(shapes):
        sigma = sigma_field(nx, ntau, sigma_seed0 + i)
        b = gaussian_rhs(nx, ntau, [rhs_seed0 + nrhs * i + k for k in range(nrhs)])
        out.append((nx, ntau, sigma, b))
    return out


def _lattices(probs):
    from paper_1008_3647_amd import Lattice
    lats, bs = [], []
    for nx, ntau, sigma, b in probs:
        L = Lattice(nx, ntau, TAU, G, torch.complex128)
        L.set_aux_field(to_dev(sigma))
        lats.append(L)
        bs.append(to_dev(b))
    return lats, bs


@pytest.mark.parametrize("mixed", [True, False])
def test_tiny_uneven_batch_against_dense_lu(mixed):
    require_gpu()
    from paper_1008_3647_amd.lattice import solve_batched
    shapes = [(2, 2), (2, 7), (4, 3), (4, 12), (6, 5), (2, 16), (8, 4), (4, 9)]
    probs = _problems(shapes, 900, 950, 2)
    lats, bs = _lattices(probs)
    xs, st = solve_batched(lats, bs, tol=1e-10, mixed=mixed)
    for (nx, ntau, sigma, b), x, s in zip(probs, xs, st):
        say(f"{nx}x{ntau}: iters {s['iters']} relres {s['relres']}")
        assert s["status"] == 0 and max(s["relres"]) <= 1e-10
        Md = op.dense_M(sigma, TAU, G)
        xh = to_host(x)
        for k in range(b.shape[0]):
            ref = osol.dense_two_step(Md, b[k].ravel()).reshape(b[k].shape)
            assert np.linalg.norm(xh[k] - ref) / np.linalg.norm(ref) < 1e-7


def test_batched_64_against_unbatched_and_oracle():
    """The 64-lattice batch (Nx in {6,8,10,12}, Ntau in 80..320), 2 rhs each,
    complex64-refined: every system converges to 1e-10 per step; solutions
    agree with the unbatched mixed solve of the same problem within 1e-7
    (both are within ~cond(M) x 1e-10 of the exact solution); the oracle's M
    recomputes the residual of four problems."""
    require_gpu()
    from paper_1008_3647_amd.lattice import solve_batched
    w = WORKLOADS["batched_64"]
    shapes = batched_problem_shapes(w["count"], w["shape_seed"])
    probs = _problems(shapes, w["sigma_seed0"], w["rhs_seed0"], w["nrhs"])
    lats, bs = _lattices(probs)
    xs, st = solve_batched(lats, bs, tol=1e-10, mixed=True)
    say(f"batched: max iters {max(max(s['iters']) for s in st)}, wall {st[0]['seconds']:.3f}s")
    for s in st:
        assert s["status"] == 0 and max(s["relres"]) <= 1e-10
    for i in (0, 17, 40, 63):
        nx, ntau, sigma, b = probs[i]
        x1, s1 = lats[i].solve_bicgstab(bs[i], "two_step", tol=1e-10, mixed=True)
        a, c = to_host(xs[i]), to_host(x1)
        err = np.max(np.abs(a - c)) / np.max(np.abs(c))
        say(f"problem {i} ({nx}x{ntau}): batched vs unbatched {err:.2e}")
        assert err < 1e-7
        for k in range(b.shape[0]):
            r = b[k] - oracle.apply_Q(a[k], sigma, TAU, G)
            assert np.linalg.norm(r) / np.linalg.norm(b[k]) < 1e-7
