"""Autotuners for launch shapes.

tune(): per lattice, the slab size and workgroup numbering of the streaming
M / M^T kernels and the workgroups per right-hand side of the Krylov vector
kernels. tune_apply(): the launch shape of the plain operator (apply_M or
apply_Mdag) including the route of the T^3 transform. tune_batched():
the persistent launch shape of solve_batched for a set of problems.

The workgroup size of the streaming kernels is not a knob: one thread owns one
z-line of an Nx^3 slice (Nx^2 threads), which the transform's three stages are
built on. Right-hand sides per workgroup follow from the numbering: with
rhs_inner an XCD takes every rhs of a slab group in turn.

Each candidate is timed on the real workload: a BiCGStab run of a fixed number
of iterations (tolerance unreachable, so every candidate does identical work)
on the caller's right-hand sides. tune() applies the best pair with
Lattice.tune() and caches it in a JSON file keyed by device, lattice shape,
number of right-hand sides, dtype and precision mode.
"""
from __future__ import annotations

import itertools
import json
import os
import time

import torch

from .lattice import Lattice

DEFAULT_CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                             "ufg_mi355x", "tune.json")


def _key(L: Lattice, nrhs, mixed, precond=None):
    dev = torch.cuda.get_device_properties(L.device)
    arch = getattr(dev, "gcnArchName", dev.name)
    key = f"{arch}|{L.nx}|{L.ntau}|{nrhs}|{L.dtype}|{int(mixed)}"
    return key if precond is None else f"{key}|{precond!r}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def candidate_slabs(L: Lattice):
    if L.nx not in (8, 12, 16):
        return [0]
    return [s for s in (1, 2, 3, 4, 6, 8) if s <= L.ntau]


# workgroup numberings of the streaming kernels: (xcd_group, rhs_inner);
# (0, False) is the contiguous per-XCD numbering (see lattice_tune_order)
ORDERS = ((0, False), (5, False), (10, False), (5, True), (10, True))


def _time_solve(L, b, op, precond, mixed, iters, reps):
    L.solve_bicgstab(b, op, precond=precond, tol=1e-30, maxit=2, mixed=mixed)  # warm-up
    best_t = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.solve_bicgstab(b, op, precond=precond, tol=1e-30, maxit=iters, mixed=mixed,
                         check_every=iters)
        torch.cuda.synchronize()
        best_t = min(best_t, time.perf_counter() - t0)
    return best_t


def tune(L: Lattice, b: torch.Tensor, mixed=False, op="M", iters=16, reps=2,
         vec_blocks=(0, 32, 64, 128, 256, 512), orders=ORDERS,
         cache: str | None = DEFAULT_CACHE, force=False, verbose=False, precond=None,
         finalists=3, refine_iters=100, refine_reps=2):
    """Pick the launch shape for solves of `b` on `L` (with `precond`, whose
    basis-change launches follow the same slab choice): slices per slab and
    workgroup numbering of the streaming kernels first (vector kernels at their
    default), then the workgroups per rhs of the vector kernels for that
    choice; the `finalists` fastest of all are timed again over
    `refine_iters` iterations, `refine_reps` rounds in turn (the short runs
    cannot separate shapes a few tenths of a per cent apart). Returns a dict
    with the choice and the timings of every candidate."""
    nrhs = b.shape[0]
    key = "v3|" + _key(L, nrhs, mixed, precond)
    data = _load(cache) if cache else {}
    if not force and key in data:
        best = data[key]
        L.tune(best["slab"], best["vec_blocks"], xcd_group=best["xcd_group"],
               rhs_inner=best["rhs_inner"])
        return dict(best, cached=True)
    results = []

    def run(slab, vb, grp, ri):
        L.tune(slab, vb, xcd_group=grp, rhs_inner=ri)
        t = _time_solve(L, b, op, precond, mixed, iters, reps)
        results.append(dict(slab=slab, vec_blocks=vb, xcd_group=grp, rhs_inner=ri, seconds=t))
        if verbose:
            print(f"tune slab={slab} vec_blocks={vb} group={grp} rhs_inner={ri}: "
                  f"{t * 1e3:.2f} ms", flush=True)
        return results[-1]

    streaming = L.nx in (8, 12, 16)
    for slab in candidate_slabs(L):
        for grp, ri in (orders if streaming else ((0, False),)):
            run(slab, 0, grp, ri)
    first = min(results, key=lambda d: d["seconds"])
    for vb in vec_blocks:
        if vb != 0:
            run(first["slab"], vb, first["xcd_group"], first["rhs_inner"])
    final = sorted(results, key=lambda d: d["seconds"])[:max(1, finalists)]
    if len(final) > 1 and refine_reps > 0:
        for d in final:
            d["refined"] = float("inf")
        for _ in range(refine_reps):
            for d in final:
                L.tune(d["slab"], d["vec_blocks"], xcd_group=d["xcd_group"],
                       rhs_inner=d["rhs_inner"])
                d["refined"] = min(d["refined"], _time_solve(L, b, op, precond, mixed,
                                                             refine_iters, 1))
        if verbose:
            for d in final:
                print(f"tune refine slab={d['slab']} vec_blocks={d['vec_blocks']} "
                      f"group={d['xcd_group']} rhs_inner={d['rhs_inner']}: "
                      f"{d['refined'] * 1e3:.2f} ms", flush=True)
        best = min(final, key=lambda d: d["refined"])
    else:
        best = final[0]
    L.tune(best["slab"], best["vec_blocks"], xcd_group=best["xcd_group"],
           rhs_inner=best["rhs_inner"])
    choice = {k: best[k] for k in ("slab", "vec_blocks", "xcd_group", "rhs_inner", "seconds")}
    choice["iters"] = iters
    if "refined" in best:
        choice["refined_seconds"] = best["refined"]
        choice["refine_iters"] = refine_iters
    if cache:
        data[key] = choice
        _store(cache, data)
    return dict(choice, cached=False, candidates=results)


def tune_apply(L: Lattice, x, dagger=False, launches=100, reps=3, orders=ORDERS,
               transforms=None, verbose=False):
    """Pick the launch shape of the plain operator (apply_M, or apply_Mdag with
    dagger=True) on `x` (a tensor, or a list of tensors that the timed
    launches cycle through, e.g. to keep the operands out of the Infinity
    Cache): slices per slab, workgroup numbering and, for complex64 on
    Nx = 16, the transform route (0: VALU block form, 1: y and x stages on
    MFMA, 2: 16-point DFTs; see lattice_tune_transform). Each candidate is
    timed over `launches` back-to-back applications with HIP events on the
    lattice's stream (best of `reps`); the best is applied with Lattice.tune
    and returned with the timings of every candidate."""
    fn = L.apply_Mdag if dagger else L.apply_M
    xs = list(x) if isinstance(x, (list, tuple)) else [x]
    ys = [torch.empty_like(v) for v in xs]
    x = xs[0]
    if transforms is None:
        transforms = (0, 1, 2) if (x.dtype == torch.complex64 and L.nx == 16) else (0,)
    streaming = L.nx in (8, 12, 16)
    results = []
    for slab in candidate_slabs(L):
        for grp, ri in (orders if streaming else ((0, False),)):
            for tr in transforms:
                L.tune(slab, 0, xcd_group=grp, rhs_inner=ri, transform=tr)
                for i in range(len(xs)):  # warm-up
                    fn(xs[i], ys[i])
                best_t = float("inf")
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                for _ in range(reps):
                    e0.record(L.stream)  # on the stream the lattice launches on
                    for i in range(launches):
                        fn(xs[i % len(xs)], ys[i % len(xs)])
                    e1.record(L.stream)
                    torch.cuda.synchronize()
                    best_t = min(best_t, e0.elapsed_time(e1) * 1e-3 / launches)
                results.append(dict(slab=slab, xcd_group=grp, rhs_inner=ri, transform=tr,
                                    seconds=best_t))
                if verbose:
                    print(f"tune_apply slab={slab} group={grp} rhs_inner={ri} transform={tr}: "
                          f"{best_t * 1e6:.1f} us", flush=True)
    best = min(results, key=lambda d: d["seconds"])
    L.tune(best["slab"], 0, xcd_group=best["xcd_group"], rhs_inner=best["rhs_inner"],
           transform=best["transform"])
    choice = {k: best[k] for k in ("slab", "xcd_group", "rhs_inner", "transform", "seconds")}
    return dict(choice, candidates=results)


def tune_batched(lattices, bs, mixed=True, iters=10, reps=2, hop_blocks=(2, 4, 8),
                 vec_blocks=(8, 16), chunks=(4096, 16384), slabs=(1, 2, 4), finalists=3,
                 refine_iters=60, refine_reps=3, verbose=False):
    """Pick the launch shape of solve_batched (workgroups per CU of the
    persistent operator and vector launches, elements per vector work item,
    slices per slab of the batched operator) for
    this set of problems. Each candidate runs the batch for a fixed number of
    iterations per step (tolerance unreachable, identical work); the
    `finalists` fastest are timed again over `refine_iters` iterations per
    step, `refine_reps` rounds in turn (short runs cannot separate shapes a
    few per cent apart); the best is applied with solve_batched_tune and
    returned."""
    from .lattice import solve_batched, solve_batched_tune

    def run(shape, n):
        solve_batched_tune(*shape)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve_batched(lattices, bs, tol=1e-30, maxit=n, mixed=mixed, check_every=n)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    results = []
    for hb, vb, ch, sl in itertools.product(hop_blocks, vec_blocks, chunks, slabs):
        solve_batched_tune(hb, vb, ch, sl)
        solve_batched(lattices, bs, tol=1e-30, maxit=2, mixed=mixed, check_every=2)
        best_t = min(run((hb, vb, ch, sl), iters) for _ in range(reps))
        results.append(dict(hop_blocks_per_cu=hb, vec_blocks_per_cu=vb, chunk=ch, slab=sl,
                            seconds=best_t))
        if verbose:
            print(f"tune_batched {hb} {vb} {ch} {sl}: {best_t * 1e3:.2f} ms", flush=True)
    keys = ("hop_blocks_per_cu", "vec_blocks_per_cu", "chunk", "slab")
    final = sorted(results, key=lambda d: d["seconds"])[:max(1, finalists)]
    if len(final) > 1 and refine_reps > 0:
        for d in final:
            d["refined"] = float("inf")
        for _ in range(refine_reps):
            for d in final:
                d["refined"] = min(d["refined"], run(tuple(d[k] for k in keys), refine_iters))
        if verbose:
            for d in final:
                print(f"tune_batched refine {[d[k] for k in keys]}: "
                      f"{d['refined'] * 1e3:.2f} ms", flush=True)
        best = min(final, key=lambda d: d["refined"])
    else:
        best = final[0]
    solve_batched_tune(best["hop_blocks_per_cu"], best["vec_blocks_per_cu"], best["chunk"],
                       best["slab"])
    return {k: best[k] for k in ("hop_blocks_per_cu", "vec_blocks_per_cu", "chunk", "slab")}
