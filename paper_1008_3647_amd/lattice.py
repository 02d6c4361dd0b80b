"""Python handle over a libufg lattice: torch tensors in, torch tensors out.

Method names follow the C ABI (create_lattice / set_aux_field / apply_M /
apply_Mdag / apply_precond / solve_cg_normal / solve_bicgstab /
force_dS_dsigma); each one checks the dtype, shape, device and contiguity of
every tensor it passes (inputs, out=, x0=) before it makes exactly one
library call, since the C ABI receives bare pointers and cannot.
"""
from __future__ import annotations

import ctypes as C
import json
import time

import torch

from . import _lib as L
from ._lib import Precond, UfgError  # noqa: F401

_OPS = {"M": L.UFG_OP_M, "Mdag": L.UFG_OP_MDAG, "two_step": L.UFG_OP_TWO_STEP, "Q": L.UFG_OP_Q}


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Lattice:
    """Nx^3 x Ntau lattice with field sigma (paper, Sec. 1); Nx^dim x Ntau for
    dim = 1 or 2 (the lower dimensions of the paper's conclusions).

    dtype: torch.complex64 or torch.complex128 (the vector type of apply_* and
    of plain solves; mixed-precision solves need complex128).
    dispersion: "free" (E = k^2/2, the paper's) or "hubbard" (E = 1 - cos k per
    axis; C ABI create_lattice_ex).
    dim: spatial dimension (C ABI create_lattice_dim); vectors are
    [nrhs][Ntau][Nx]^dim.
    log_path: when set, every solve appends one JSON line (call, parameters,
    solve statistics) to this file.
    """

    def __init__(self, nx, ntau, tau=0.05, g=5.0, dtype=torch.complex128, stream=None,
                 dispersion="free", dim=3, log_path=None):
        self._lib = L.load()
        if dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        if dispersion not in L.DISPERSIONS:
            raise ValueError(f"dispersion must be one of {sorted(L.DISPERSIONS)}")
        if dim not in (1, 2, 3):
            raise ValueError("dim must be 1, 2 or 3")
        self.nx, self.ntau, self.tau, self.g, self.dtype = nx, ntau, tau, g, dtype
        self.dispersion = dispersion
        self.dim = int(dim)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        code = self._lib.create_lattice_dim(nx, ntau, self.dim, tau, g,
                                            L.UFG_C128 if dtype == torch.complex128 else L.UFG_C64,
                                            L.DISPERSIONS[dispersion], _stream_ptr(stream),
                                            C.byref(h))
        L.check(code, "create_lattice")
        self._h = h
        A = C.c_double()
        L.check(self._lib.lattice_info(h, None, None, None, C.byref(A)), "lattice_info")
        self.A = A.value
        self._sigma = None
        self.log_path = log_path

    # ------------------------------------------------------------------ utils
    @property
    def shape(self):
        return (self.ntau,) + (self.nx,) * self.dim

    def _vec(self, x, name, dtype=None):
        dtype = dtype or self.dtype
        if not isinstance(x, torch.Tensor) or x.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if x.dtype != dtype:
            raise TypeError(f"{name} must have dtype {dtype}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if x.dim() < len(self.shape) or tuple(x.shape[-len(self.shape):]) != self.shape:
            raise ValueError(f"{name} must end in shape {self.shape}, got {tuple(x.shape)}")
        n = x.numel() // (self.ntau * self.nx ** self.dim)
        if n == 0:
            raise ValueError(f"{name} holds no right-hand sides (shape {tuple(x.shape)})")
        return n

    def _like(self, t, ref, name):
        """`t` must be a contiguous CUDA tensor of ref's dtype, shape and device
        (the library writes through it as ref's layout)."""
        if not isinstance(t, torch.Tensor) or t.device != ref.device:
            raise TypeError(f"{name} must be a CUDA tensor on {ref.device}")
        if t.dtype != ref.dtype:
            raise TypeError(f"{name} must have dtype {ref.dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(ref.shape):
            raise ValueError(f"{name} must have shape {tuple(ref.shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _out(self, out, x, name="out"):
        if out is None:
            return torch.empty_like(x, memory_format=torch.contiguous_format)
        self._like(out, x, name)
        if out.data_ptr() == x.data_ptr():
            raise ValueError(f"{name} must not alias the input")
        return out

    def _log(self, call, stats, nrhs, **params):
        """Append one JSON line per solve to log_path (when set): the call, its
        parameters and the solve statistics (ufg_solve_stats)."""
        if not self.log_path:
            return
        rec = dict(call=call, lattice=dict(nx=self.nx, ntau=self.ntau, dim=self.dim,
                                           dtype=str(self.dtype).replace("torch.", ""),
                                           dispersion=self.dispersion, tau=self.tau, g=self.g),
                   nrhs=nrhs, time=time.time(), **params)
        rec.update({k: v for k, v in stats.items() if isinstance(v, (int, float, list, tuple))})
        with open(self.log_path, "a") as f:
            f.write(json.dumps(rec) + "\n")

    def new_vectors(self, nrhs, dtype=None):
        return torch.empty((nrhs,) + self.shape, dtype=dtype or self.dtype, device=self.device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.destroy_lattice(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        L.check(self._lib.set_lattice_stream(self._h, _stream_ptr(stream)), "set_lattice_stream")
        self.stream = stream if stream is not None else torch.cuda.current_stream()

    # ---------------------------------------------------------------- the ABI
    def set_aux_field(self, sigma: torch.Tensor):
        if sigma.dtype != torch.float64 or sigma.device.type != "cuda":
            raise TypeError("sigma must be a float64 CUDA tensor")
        if tuple(sigma.shape) != self.shape or not sigma.is_contiguous():
            raise ValueError(f"sigma must be contiguous with shape {self.shape}")
        L.check(self._lib.set_aux_field(self._h, C.c_void_p(sigma.data_ptr())), "set_aux_field")
        self._sigma = sigma

    def apply_M(self, x, out=None):
        n = self._vec(x, "x")
        y = self._out(out, x)
        L.check(self._lib.apply_M(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), n),
                "apply_M")
        return y

    def apply_Mdag(self, x, out=None):
        n = self._vec(x, "x")
        y = self._out(out, x)
        L.check(self._lib.apply_Mdag(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                     n), "apply_Mdag")
        return y

    def apply_precond(self, x, precond: Precond, op="M", out=None):
        n = self._vec(x, "x")
        if op not in _OPS:
            raise ValueError(f"op must be one of {sorted(_OPS)}")
        y = self._out(out, x)
        p = precond.to_c()
        L.check(self._lib.apply_precond(self._h, C.byref(p), _OPS[op], C.c_void_p(x.data_ptr()),
                                        C.c_void_p(y.data_ptr()), n), "apply_precond")
        return y

    def lam_max(self, precond: Precond):
        """lam_max the Chebyshev preconditioner normalises Q with (C ABI
        precond_lam_max; runs the power iteration when precond.lam_max < 0)."""
        p = precond.to_c()
        out = C.c_double()
        L.check(self._lib.precond_lam_max(self._h, C.byref(p), C.byref(out)), "precond_lam_max")
        return out.value

    def _solve_dtype(self, mixed):
        return torch.complex128 if mixed else self.dtype

    def solve_cg_normal(self, b, precond: Precond | None = None, tol=1e-10, maxit=10000,
                        mixed=False, delta=0.1, check_every=10, x0=None, graph=True):
        dt = self._solve_dtype(mixed)
        n = self._vec(b, "b", dt)
        x = self._out(x0, b, "x0") if x0 is not None else torch.empty_like(b)
        o = L.solve_opts(tol, maxit, mixed, delta, check_every, x0 is not None, not graph)
        st = L.ufg_solve_stats()
        p = precond.to_c() if precond else None
        code = self._lib.solve_cg_normal(self._h, C.byref(p) if p else None,
                                         C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), n,
                                         C.byref(o), C.byref(st))
        L.check(code, "solve_cg_normal")
        stats = st.as_dict()
        self._log("solve_cg_normal", stats, n, precond=repr(precond), tol=tol, maxit=maxit,
                  mixed=bool(mixed))
        return x, stats

    def solve_cg_split(self, b, precond: Precond, tol=1e-10, maxit=10000, check_every=10,
                       graph=True):
        """CG with split preconditioning E^T Q E z = E^T b, x = E z, E = W_d of
        the weak-coupling `precond` (C ABI solve_cg_split)."""
        n = self._vec(b, "b")
        x = torch.empty_like(b)
        o = L.solve_opts(tol, maxit, False, 0.1, check_every, False, not graph)
        st = L.ufg_solve_stats()
        p = precond.to_c()
        code = self._lib.solve_cg_split(self._h, C.byref(p), C.c_void_p(b.data_ptr()),
                                        C.c_void_p(x.data_ptr()), n, C.byref(o), C.byref(st))
        L.check(code, "solve_cg_split")
        stats = st.as_dict()
        self._log("solve_cg_split", stats, n, precond=repr(precond), tol=tol, maxit=maxit)
        return x, stats

    def solve_bicgstab(self, b, op="two_step", precond: Precond | None = None, tol=1e-10,
                       maxit=10000, mixed=False, delta=0.1, check_every=10, x0=None,
                       graph=True):
        dt = self._solve_dtype(mixed)
        n = self._vec(b, "b", dt)
        if op not in _OPS:
            raise ValueError(f"op must be one of {sorted(_OPS)}")
        x = self._out(x0, b, "x0") if x0 is not None else torch.empty_like(b)
        o = L.solve_opts(tol, maxit, mixed, delta, check_every, x0 is not None, not graph)
        st = L.ufg_solve_stats()
        p = precond.to_c() if precond else None
        code = self._lib.solve_bicgstab(self._h, C.byref(p) if p else None, _OPS[op],
                                        C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), n,
                                        C.byref(o), C.byref(st))
        L.check(code, "solve_bicgstab")
        stats = st.as_dict()
        self._log("solve_bicgstab", stats, n, op=op, precond=repr(precond), tol=tol,
                  maxit=maxit, mixed=bool(mixed))
        return x, stats

    def tune(self, slab=0, vec_blocks=0, nslab=0, xcd_group=-1, rhs_inner=False, transform=0):
        """Launch parameters (0 = library default, xcd_group -1 = default); see
        lattice_tune, lattice_tune_slabs, lattice_tune_order and
        lattice_tune_transform in ufg.h (nslab, when given, overrides slab)."""
        L.check(self._lib.lattice_tune(self._h, int(slab), int(vec_blocks)), "lattice_tune")
        L.check(self._lib.lattice_tune_slabs(self._h, int(nslab)), "lattice_tune_slabs")
        L.check(self._lib.lattice_tune_order(self._h, int(xcd_group), int(bool(rhs_inner))),
                "lattice_tune_order")
        L.check(self._lib.lattice_tune_transform(self._h, int(transform)),
                "lattice_tune_transform")

    def _real_field(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must have dtype torch.float64, got {t.dtype}")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}")
        return t

    def _hmc_args(self, sigma, pi, vec, name, dt, nsteps, tol, maxit, mixed, check_every,
                  chrono):
        self._real_field(sigma, "sigma")
        self._real_field(pi, "pi")
        if pi.device != sigma.device:
            raise TypeError("sigma and pi must be on one device")
        n = self._vec(vec, name, self._solve_dtype(mixed))
        if vec.device != sigma.device:
            raise TypeError(f"{name} must be on {sigma.device}")
        s = sigma.detach().clone()
        p = pi.detach().clone()
        o = L.ufg_hmc_opts(float(dt), int(nsteps), float(tol), int(maxit), int(bool(mixed)),
                           int(check_every), int(bool(chrono)))
        return n, s, p, o

    def hmc_leapfrog(self, sigma, pi, phi, dt, nsteps, precond: Precond | None = None,
                     tol=1e-11, maxit=10000, mixed=False, check_every=10, chrono=True):
        """Leapfrog MD of the phi-algorithm from (sigma, pi) with phi fixed
        (C ABI hmc_leapfrog). Returns new (sigma, pi) tensors, the action at
        every force evaluation and the result record."""
        n, s, p, o = self._hmc_args(sigma, pi, phi, "phi", dt, nsteps, tol, maxit, mixed,
                                    check_every, chrono)
        acts = (C.c_double * (int(nsteps) + 1))()
        res = L.ufg_hmc_result()
        pc = precond.to_c() if precond else None
        code = self._lib.hmc_leapfrog(self._h, C.byref(pc) if pc else None,
                                      C.c_void_p(s.data_ptr()), C.c_void_p(p.data_ptr()),
                                      C.c_void_p(phi.data_ptr()), n, C.byref(o), acts,
                                      C.byref(res))
        L.check(code, "hmc_leapfrog")
        self._sigma = s
        return s, p, list(acts), res.as_dict()

    def hmc_trajectory(self, sigma, pi, eta, u, dt, nsteps, precond: Precond | None = None,
                       tol=1e-11, maxit=10000, mixed=False, check_every=10, chrono=True,
                       want_phi=False):
        """One phi-algorithm trajectory (C ABI hmc_trajectory): heat bath
        phi = M^dagger eta at sigma, leapfrog, Metropolis with the draw u.
        Returns (sigma, pi, info): the chain's next state (MD end point if
        accepted, else the start) and the result record plus 'actions' (and
        'phi' when want_phi)."""
        n, s, p, o = self._hmc_args(sigma, pi, eta, "eta", dt, nsteps, tol, maxit, mixed,
                                    check_every, chrono)
        phi = torch.empty_like(eta) if want_phi else None
        acts = (C.c_double * (int(nsteps) + 1))()
        res = L.ufg_hmc_result()
        pc = precond.to_c() if precond else None
        code = self._lib.hmc_trajectory(self._h, C.byref(pc) if pc else None,
                                        C.c_void_p(s.data_ptr()), C.c_void_p(p.data_ptr()),
                                        C.c_void_p(eta.data_ptr()), n, float(u), C.byref(o),
                                        C.c_void_p(phi.data_ptr()) if phi is not None else None,
                                        acts, C.byref(res))
        L.check(code, "hmc_trajectory")
        self._sigma = s
        info = res.as_dict()
        info["actions"] = list(acts)
        if phi is not None:
            info["phi"] = phi
        return s, p, info

    def norm2(self, x):
        """||x_r||^2 per right-hand side (host list), FP64 accumulation."""
        n = self._vec(x, "x")
        out = (C.c_double * n)()
        L.check(self._lib.lattice_norm2(self._h, C.c_void_p(x.data_ptr()), n, out),
                "lattice_norm2")
        return list(out)

    def norm2_noalloc(self, x, out):
        """||x_r||^2 per right-hand side into the float64 CUDA tensor `out`
        (nrhs entries), asynchronously and without any allocation by the
        library (C ABI lattice_norm2_noalloc)."""
        n = self._vec(x, "x")
        if not isinstance(out, torch.Tensor) or out.device != x.device:
            raise TypeError(f"out must be a CUDA tensor on {x.device}")
        if out.dtype != torch.float64 or out.numel() != n or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float64 tensor of {n} entries")
        L.check(self._lib.lattice_norm2_noalloc(self._h, C.c_void_p(x.data_ptr()), n,
                                                C.c_void_p(out.data_ptr())),
                "lattice_norm2_noalloc")
        return out

    def force_dS_dsigma(self, X, y, out=None):
        n = self._vec(X, "X")
        self._like(y, X, "y")
        if out is None:
            g = torch.empty(self.shape, dtype=torch.float64, device=X.device)
        else:
            g = out
            if not isinstance(g, torch.Tensor) or g.device != X.device:
                raise TypeError(f"out must be a CUDA tensor on {X.device}")
            if g.dtype != torch.float64:
                raise TypeError(f"out must have dtype torch.float64, got {g.dtype}")
            if tuple(g.shape) != self.shape or not g.is_contiguous():
                raise ValueError(f"out must be contiguous with shape {self.shape}")
        L.check(self._lib.force_dS_dsigma(self._h, C.c_void_p(X.data_ptr()),
                                          C.c_void_p(y.data_ptr()), n, C.c_void_p(g.data_ptr())),
                "force_dS_dsigma")
        return g


# Host helpers (no GPU needed)
def cheb_roots(degree, eps):
    lib = L.load()
    out = (C.c_double * (2 * degree))()
    c = (C.c_double * 2)()
    L.check(lib.ufg_cheb_roots(degree, eps, out, c), "ufg_cheb_roots")
    roots = [complex(out[2 * i], out[2 * i + 1]) for i in range(degree)]
    return roots, complex(c[0], c[1])


def euler_weights(order, p=0.5):
    lib = L.load()
    out = (C.c_double * (order + 1))()
    L.check(lib.ufg_euler_weights(order, p, out), "ufg_euler_weights")
    return list(out)


def transfer_matrix(nx, tau):
    lib = L.load()
    out = (C.c_double * (nx * nx))()
    L.check(lib.ufg_transfer_matrix(nx, tau, out), "ufg_transfer_matrix")
    return [[out[i * nx + j] for j in range(nx)] for i in range(nx)]


def device_copy(src, dst):
    """Streaming device copy src -> dst (C ABI ufg_device_copy) on torch's current
    stream: the plain-copy reference rate for the streaming operator."""
    if src.nbytes != dst.nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("device_copy needs two device tensors of equal size")
    stream = torch.cuda.current_stream(src.device).cuda_stream
    L.check(L.load().ufg_device_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                     src.nbytes, C.c_void_p(stream)), "ufg_device_copy")


def solve_batched(lattices, bs, tol=1e-10, maxit=10000, mixed=True, delta=0.1, check_every=10):
    """Two-step BiCGStab for many lattices at once (C ABI solve_batched).

    lattices: list of complex128 Lattice objects (fields installed); bs: list of
    complex128 tensors [nrhs_i][Ntau_i][Nx_i]^3. Returns (xs, stats)."""
    lib = L.load()
    n = len(lattices)
    if n != len(bs) or n == 0:
        raise ValueError("need one right-hand-side tensor per lattice")
    xs, nr = [], []
    for lat, b in zip(lattices, bs):
        if lat.dtype != torch.complex128:
            raise TypeError("batched solves need complex128 lattices")
        nr.append(lat._vec(b, "b", torch.complex128))
        xs.append(torch.empty_like(b))
    handles = (C.c_void_p * n)(*[lat._h.value for lat in lattices])
    bp = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    xp = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    nrhs = (C.c_int * n)(*nr)
    o = L.solve_opts(tol, maxit, mixed, delta, check_every, False)
    st = (L.ufg_solve_stats * n)()
    L.check(lib.solve_batched(handles, n, bp, xp, nrhs, None, C.byref(o), st), "solve_batched")
    return xs, [s.as_dict() for s in st]


def solve_batched_tune(hop_blocks_per_cu=0, vec_blocks_per_cu=0, chunk=0, slab=0, sync_iters=0):
    """Launch shape of batched solves (0 = default); see ufg.h."""
    L.check(L.load().solve_batched_tune(int(hop_blocks_per_cu), int(vec_blocks_per_cu),
                                        int(chunk), int(slab), int(sync_iters)),
            "solve_batched_tune")
