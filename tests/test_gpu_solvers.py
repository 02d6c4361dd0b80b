"""Parity of the HIP solvers with the oracle (paper, Eqs. 1-3).

The solution of M^T M x = b is unique, so every solver and preconditioner must
reach the same x; iteration counts are not compared. Checks:
  * true residual ||b - A x|| / ||b|| <= tol recomputed by the ORACLE's M;
  * forward error against the oracle's solution (dense LU on the 4^3 x 40
    lattice, the oracle's own BiCGStab to 1e-13 elsewhere) within
    cond-limited bounds stated per test.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import operator as op
from oracle import solvers as osol
from synthetic import sigma_field, gaussian_rhs, WORKLOADS
from gpu_util import require_gpu, to_dev, to_host, say, TAU, G

pytestmark = pytest.mark.gpu


def _relres_oracle(x, b, sigma, kind):
    """||b - A x|| / ||b|| with the oracle's operator (per rhs, worst)."""
    worst = 0.0
    for xi, bi in zip(x, b):
        if kind == "M":
            r = bi - oracle.apply_M(xi, sigma, TAU, G)
        elif kind == "Mdag":
            r = bi - oracle.apply_Mdag(xi, sigma, TAU, G)
        else:
            r = bi - oracle.apply_Q(xi, sigma, TAU, G)
        worst = max(worst, np.linalg.norm(r) / np.linalg.norm(bi))
    return worst


@pytest.fixture(scope="module")
def lattice_4x40():
    w = WORKLOADS["lattice_4x40"]
    sigma = sigma_field(w["nx"], w["ntau"], w["sigma_seed"])
    b = gaussian_rhs(w["nx"], w["ntau"], w["rhs_seeds"])
    Md = op.dense_M(sigma, TAU, G)
    x_lu = osol.dense_two_step(Md, b[0].ravel()).reshape(b[0].shape)
    y_lu = np.linalg.solve(Md.T, b[0].ravel()).reshape(b[0].shape)
    return sigma, b, x_lu, y_lu


@pytest.mark.parametrize("solver", ["cg", "bicgstab"])
@pytest.mark.parametrize("mixed", [False, True])
def test_lattice_4x40_against_dense_lu(lattice_4x40, solver, mixed):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    sigma, b, x_lu, y_lu = lattice_4x40
    say(f"4x40 {solver} mixed={mixed}")
    L = Lattice(4, 40, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    bd = to_dev(b)
    if solver == "cg":
        x, st = L.solve_cg_normal(bd, tol=1e-10, mixed=mixed)
    else:
        x, st = L.solve_bicgstab(bd, "two_step", tol=1e-10, mixed=mixed)
    x = to_host(x)
    say(st)
    assert st["status"] == 0
    assert max(st["relres"]) <= 1e-10 if solver == "bicgstab" else st["relres"][0] <= 1e-10
    if solver == "cg":
        assert _relres_oracle(x, b, sigma, "Q") <= 1.2e-10
    # forward error <= cond * residual: cond(M) ~ 1e2 per step here
    assert np.linalg.norm(x[0] - x_lu) / np.linalg.norm(x_lu) < 1e-6


@pytest.mark.parametrize("op_name", ["M", "Mdag"])
@pytest.mark.parametrize("dtype,mixed", [(torch.complex128, False), (torch.complex64, False),
                                         (torch.complex128, True)])
def test_single_system_bicgstab(op_name, dtype, mixed):
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau, nrhs = 6, 24, 3
    sigma = sigma_field(nx, ntau, 401)
    b = gaussian_rhs(nx, ntau, [402, 403, 404])
    say(f"bicgstab {op_name} {dtype} mixed={mixed}")
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    tol = 1e-10 if (dtype == torch.complex128) else 1e-5
    bd = to_dev(b, torch.complex128 if mixed else dtype)
    x, st = L.solve_bicgstab(bd, op_name, tol=tol, mixed=mixed)
    say(st)
    assert st["status"] == 0
    x = to_host(x).astype(np.complex128)
    bb = to_host(bd).astype(np.complex128)
    assert _relres_oracle(x, bb, sigma, op_name) <= 1.2 * tol


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("op_name", ["M", "Mdag"])
def test_bicgstab_check_interval(op_name, mixed):
    """On streaming lattices the unpreconditioned BiCGStab merges the x, r
    update of an iteration with the p update of the next one, and runs the
    separate update only in iterations that end at a check point. check_every
    = 1 gives the separate form only; 7 and 25 mostly the merged one (odd and
    long intervals change which p / v buffers are current at a check point).
    All must converge to the same solution with the true residual (oracle)
    within tol and comparable iteration counts."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau, nrhs = 8, 40, 2
    sigma = sigma_field(nx, ntau, 441)
    b = gaussian_rhs(nx, ntau, [442, 443])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    tol = 1e-10
    sols, iters = [], []
    for check in (1, 7, 25):
        say(f"bicgstab {op_name} mixed={mixed} check_every={check}")
        x, st = L.solve_bicgstab(to_dev(b), op_name, tol=tol, mixed=mixed, check_every=check)
        say(st)
        assert st["status"] == 0
        if not mixed:
            # the interval the loop issues after every rhs stopped (the host
            # reads check-point flags one interval late) is not counted: the
            # launched iterations end at the check point that confirmed
            n = max(st["iters"])
            assert st["mv"] == 2 * check * (-(-n // check))
        xh = to_host(x)
        assert _relres_oracle(xh, b, sigma, op_name) <= 1.2 * tol
        sols.append(xh)
        iters.append(max(st["iters"]))
    # every solution has a true residual <= tol: they differ by at most about
    # cond(M) tol (cond(M) of this lattice is far below 1e3)
    for xh in sols[1:]:
        assert np.max(np.abs(xh - sols[0])) / np.max(np.abs(sols[0])) < 1e-6
    # a check interval of c stops at most c - 1 iterations late
    assert max(iters) <= 1.25 * min(iters) + 25


@pytest.mark.parametrize("mixed", [True, False])
def test_lattice_16x400_against_oracle_reference(mixed):
    """Full-size two-step solve, 8 rhs, in the configuration bench.py times.
    Every right-hand side is compared with the oracle's reference solution
    (tests/golden/lattice_16x400_reference.npz: sampled entries of x solved by
    the oracle to ~1e-13 per step): forward error <= 1e-7, i.e. the per-step
    residual 1e-10 times cond(M) (~1e3 on this lattice) with margin, and the
    norm of x to 1e-8; and every rhs's residual of M^T M x = b is recomputed by
    the oracle's operators: b - M^T M x = (b - M^T y) + M^T (y - M x) with both
    steps <= 1e-10, so <= 1e-10 (1 + ||M^T|| ||y|| / ||b||), ||M^T|| <= 1 + max|b|,
    ||y|| ~ ||M x||, times 2 for the FP64 rounding of the recomputation."""
    require_gpu()
    import os
    from paper_1008_3647_amd import Lattice
    w = WORKLOADS["lattice_16x400"]
    nx, ntau = w["nx"], w["ntau"]
    sigma = sigma_field(nx, ntau, w["sigma_seed"])
    b = gaussian_rhs(nx, ntau, w["rhs_seeds"])
    say(f"16x400 two-step mixed={mixed}")
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    # check interval as bench.py times it
    x, st = L.solve_bicgstab(to_dev(b), "two_step", tol=1e-10, mixed=mixed, maxit=20000,
                             check_every=40)
    say(st)
    assert st["status"] == 0 and max(st["relres"]) <= 1e-10
    xh = to_host(x)
    bmax = np.abs(oracle.field_b(sigma, oracle.coupling_A(TAU, G))).max()
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "lattice_16x400_reference.npz"))
    idx = ref["sample_index"]
    for k in range(b.shape[0]):
        xs = xh[k].reshape(-1)[idx]
        rs = ref[f"x{k}_sample"]
        err = np.max(np.abs(xs - rs)) / np.max(np.abs(rs))
        mx = oracle.apply_M(xh[k], sigma, TAU, G)
        rq = np.linalg.norm(b[k] - oracle.apply_Mdag(mx, sigma, TAU, G)) / np.linalg.norm(b[k])
        bound = 2e-10 * (1 + (1 + bmax) * np.linalg.norm(mx) / np.linalg.norm(b[k]))
        say(f"rhs {k}: forward error vs oracle {err:.2e}, norm ratio "
            f"{np.linalg.norm(xh[k]) / ref[f'x{k}_norm']:.12f}, oracle residual {rq:.2e}")
        assert err < 1e-7, k
        assert np.linalg.norm(xh[k]) / ref[f"x{k}_norm"] == pytest.approx(1.0, abs=1e-8)
        assert rq < bound, (k, rq, bound)


@pytest.mark.parametrize("case", ["bicgstab_wce2", "bicgstab_nx6", "cg_cheb", "cg_sca_mixed"])
def test_graph_replay_matches_eager_launches(case):
    """Where the iteration is not fused into the streaming kernel, every check
    interval after the first replays a captured HIP graph. The replays (with
    check-point work and reliable updates between them) must give exactly the
    result of launching every kernel separately."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    nx, ntau = (6, 24) if case == "bicgstab_nx6" else (8, 16)
    sigma = sigma_field(nx, ntau, 460)
    b = gaussian_rhs(nx, ntau, [461, 462])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    bd = to_dev(b)
    mixed = case == "cg_sca_mixed"
    out = []
    for graph in (False, True):
        say(f"{case} graph={graph}")
        if case.startswith("bicgstab"):
            pc = Precond("wce", wce_order=2) if case == "bicgstab_wce2" else None
            x, st = L.solve_bicgstab(bd, "two_step", pc, tol=1e-11, check_every=3, graph=graph)
        else:
            pc = Precond("cheb", degree=8, eps=0.01) if case == "cg_cheb" else Precond("sca", alpha=2.0)
            x, st = L.solve_cg_normal(bd, pc, tol=1e-10, mixed=mixed, check_every=4, graph=graph)
        assert st["status"] == 0
        out.append((to_host(x), st["iters"], st["mv"]))
    (x0, it0, mv0), (x1, it1, mv1) = out
    assert it0 == it1 and mv0 == mv1
    assert np.array_equal(x0, x1)
    kind = "Q" if case.startswith("cg") else None
    if kind:
        assert _relres_oracle(x1, b, sigma, "Q") <= 1.5e-10


@pytest.mark.parametrize("op_name", ["M", "Mdag", "two_step"])
@pytest.mark.parametrize("mixed", [False, True])
def test_wce_bicgstab_fused_sources(op_name, mixed):
    """With the weak-coupling preconditioner on a streaming lattice, the first
    basis change of each application forms BiCGStab's p and s itself. The
    result must satisfy the oracle's residual for M, M^T and the two-step
    solve, in FP64 and FP32-refined; Nx = 12 with Ntau = 30 (uneven slabs)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    nx, ntau = 12, 30
    sigma = sigma_field(nx, ntau, 471)
    b = gaussian_rhs(nx, ntau, [472, 473])
    say(f"wce2 bicgstab {op_name} mixed={mixed}")
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    tol = 1e-10
    x, st = L.solve_bicgstab(to_dev(b), op_name, Precond("wce", wce_order=2), tol=tol,
                             mixed=mixed, check_every=7)
    say(st)
    assert st["status"] == 0
    xh = to_host(x)
    kind = "Q" if op_name == "two_step" else op_name
    # two-step: per-step residuals <= tol give ||b - Q x|| <~ cond(M) tol
    bound = 1.2 * tol if kind != "Q" else 1e-7
    assert _relres_oracle(xh, b, sigma, kind) <= bound


def test_autotune_with_preconditioner():
    """The autotuner times candidates on the preconditioned solve when given
    one; its choice is applied to the lattice and the solve still converges to
    the oracle's residual."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    from paper_1008_3647_amd.autotune import tune
    nx, ntau = 8, 24
    sigma = sigma_field(nx, ntau, 481)
    b = gaussian_rhs(nx, ntau, [482, 483])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    pc = Precond("wce", wce_order=2)
    bd = to_dev(b)
    t = tune(L, bd, mixed=True, op="M", iters=4, reps=1, vec_blocks=(0, 64), cache=None,
             precond=pc)
    from paper_1008_3647_amd.autotune import ORDERS
    say({k: t[k] for k in ("slab", "vec_blocks", "xcd_group", "rhs_inner")})
    # every (slab, numbering) at the default vector shape, then the other
    # vector shape for the best of them
    nslabs = len([s for s in (1, 2, 3, 4, 6, 8) if s <= ntau])
    assert len(t["candidates"]) == nslabs * len(ORDERS) + 1
    assert t["slab"] in (1, 2, 3, 4, 6, 8) and t["vec_blocks"] in (0, 64)
    assert (t["xcd_group"], t["rhs_inner"]) in ORDERS
    x, st = L.solve_bicgstab(bd, "M", pc, tol=1e-10, mixed=True)
    assert st["status"] == 0
    assert _relres_oracle(to_host(x), b, sigma, "M") <= 1.2e-10


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("check", [1, 4, 10])
def test_bicgstab_iteration_cap_then_fresh_solve(mixed, check):
    """A solve stopped by the iteration cap reports status 1 with the capped
    iteration count and its true residual (checked by the oracle), whatever
    the check interval (the host reads check-point flags one interval late).
    A following solve on the same lattice starts from a clean state and
    converges."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    nx, ntau = 8, 40
    sigma = sigma_field(nx, ntau, 491)
    b = gaussian_rhs(nx, ntau, [492, 493])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    say(f"cap mixed={mixed} check={check}")
    x, st = L.solve_bicgstab(to_dev(b), "M", tol=1e-12, maxit=15, mixed=mixed, check_every=check)
    say(st)
    assert st["status"] == 1
    assert st["iters"][0] == 15
    rel = _relres_oracle(to_host(x), b, sigma, "M")
    assert rel == pytest.approx(max(st["relres"]), rel=1e-6)
    assert rel > 1e-12
    x, st = L.solve_bicgstab(to_dev(b), "M", tol=1e-10, mixed=mixed, check_every=check)
    assert st["status"] == 0
    assert _relres_oracle(to_host(x), b, sigma, "M") <= 1.2e-10


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("order", [0, 2])
def test_split_cg_against_dense_lu(dtype, order):
    """solve_cg_split (W_d^T Q W_d z = W_d^T b, x = W_d z; Sec. 5 after Table 2)
    on tiny lattices against dense LU. The forward error is bounded by
    cond(Q) times the residual of M^T M x = b recomputed by the oracle (x2 for
    rounding). complex64 runs at tol 1e-4: FP32 CG cannot go much below
    cond x 2^-24 (cond(W_0^T Q W_0) ~ 200 here), and a tolerance below that
    is not reachable in the lattice's own precision (mixed solves are the
    route to smaller residuals)."""
    require_gpu()
    from paper_1008_3647_amd import Lattice, Precond
    from oracle import operator as op
    nx, ntau = 4, 12
    sigma = sigma_field(nx, ntau, 480 + order)
    b = gaussian_rhs(nx, ntau, [481, 482])
    L = Lattice(nx, ntau, TAU, G, dtype)
    L.set_aux_field(to_dev(sigma))
    tol = 1e-12 if dtype == torch.complex128 else 1e-4
    x, st = L.solve_cg_split(to_dev(b, dtype), Precond("wce", wce_order=order), tol=tol,
                             maxit=5000)
    say(f"split CG W{order} {dtype}: {st}")
    assert st["status"] == 0
    Md = op.dense_M(sigma, TAU, G)
    condQ = np.linalg.cond(Md.T @ Md)
    xh = to_host(x).astype(np.complex128)
    for k in range(2):
        ref = osol.dense_two_step(Md, b[k].ravel()).reshape(b[k].shape)
        err = np.linalg.norm(xh[k] - ref) / np.linalg.norm(ref)
        rq = np.linalg.norm(b[k] - oracle.apply_Q(xh[k], sigma, TAU, G)) / np.linalg.norm(b[k])
        say(f"rhs {k}: forward error {err:.2e}, oracle residual {rq:.2e}, cond(Q) {condQ:.0f}")
        assert err <= 2 * condQ * rq, (k, err)
        assert rq < (1e-10 if dtype == torch.complex128 else 1e-3), (k, rq)


def test_solve_log_json_lines(tmp_path):
    """Lattice(log_path=...): one JSON line per solve with the call, its
    parameters and the statistics the call returned."""
    require_gpu()
    import json
    from paper_1008_3647_amd import Lattice, Precond
    nx, ntau = 4, 8
    sigma = sigma_field(nx, ntau, 495)
    b = to_dev(gaussian_rhs(nx, ntau, [496, 497]))
    log = tmp_path / "solves.jsonl"
    L = Lattice(nx, ntau, TAU, G, torch.complex128, log_path=str(log))
    L.set_aux_field(to_dev(sigma))
    _, s1 = L.solve_bicgstab(b, "two_step", tol=1e-10, mixed=True)
    _, s2 = L.solve_cg_normal(b, Precond("sca", alpha=2.0), tol=1e-9)
    recs = [json.loads(x) for x in log.read_text().splitlines()]
    assert [r["call"] for r in recs] == ["solve_bicgstab", "solve_cg_normal"]
    assert recs[0]["op"] == "two_step" and recs[0]["mixed"] is True and recs[0]["nrhs"] == 2
    assert tuple(recs[0]["iters"]) == s1["iters"] and recs[0]["status"] == s1["status"]
    assert recs[1]["relres"][0] == s2["relres"][0] and "sca" in recs[1]["precond"]
    assert recs[0]["lattice"] == dict(nx=nx, ntau=ntau, dim=3, dtype="complex128",
                                      dispersion="free", tau=TAU, g=G)


def test_tune_picks_a_candidate_and_the_solve_converges():
    """autotune.tune on an 8^3 x 40 lattice (FP32-refined, 2 rhs; no cache):
    the short sweep over slab sizes, workgroup orders and vector workgroups,
    then the finalists over longer runs; the choice is one of the candidates,
    stays applied, and the two-step solve with it meets tol against the
    oracle's residual."""
    require_gpu()
    from paper_1008_3647_amd import Lattice
    from paper_1008_3647_amd.autotune import tune
    nx, ntau = 8, 40
    sigma = sigma_field(nx, ntau, 1400)
    b = gaussian_rhs(nx, ntau, [1401, 1402])
    L = Lattice(nx, ntau, TAU, G, torch.complex128)
    L.set_aux_field(to_dev(sigma))
    bd = to_dev(b)
    ch = tune(L, bd, mixed=True, cache=None, vec_blocks=(0, 64), finalists=2,
              refine_iters=20, refine_reps=2)
    say(f"tune choice {ch['slab']} {ch['vec_blocks']} {ch['xcd_group']} {ch['rhs_inner']} "
        f"refined {ch.get('refined_seconds')}")
    shapes = [(c["slab"], c["vec_blocks"], c["xcd_group"], c["rhs_inner"])
              for c in ch["candidates"]]
    assert (ch["slab"], ch["vec_blocks"], ch["xcd_group"], ch["rhs_inner"]) in shapes
    assert ch["refine_iters"] == 20 and ch["refined_seconds"] > 0
    x, st = L.solve_bicgstab(bd, "two_step", tol=1e-10, mixed=True)
    assert st["status"] == 0 and max(st["relres"]) <= 1e-10
    xh = to_host(x)
    for k in range(2):
        r = b[k] - oracle.apply_Q(xh[k], sigma, TAU, G)
        assert np.linalg.norm(r) / np.linalg.norm(b[k]) < 1e-7
