"""ctypes binding of libufg.so (C ABI in include/ufg.h).

Argument marshalling only: every step of the computation runs in the HIP
library. The functions keep the C names; tensors supply device memory and
torch's current stream is the default stream of a lattice. There is no CPU
fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libufg.so")

UFG_C64, UFG_C128 = 0, 1
UFG_DISP_FREE, UFG_DISP_HUBBARD = 0, 1
DISPERSIONS = {"free": UFG_DISP_FREE, "hubbard": UFG_DISP_HUBBARD}
UFG_OP_M, UFG_OP_MDAG, UFG_OP_TWO_STEP, UFG_OP_Q = 0, 1, 2, 3
UFG_PC_NONE, UFG_PC_CHEB, UFG_PC_SCA, UFG_PC_WCE, UFG_PC_SCA_CHEB = 0, 1, 2, 3, 4
UFG_OK, UFG_EINVAL, UFG_ENOMEM, UFG_EHIP = 0, -1, -2, -3
UFG_NOT_CONVERGED, UFG_BREAKDOWN = 1, 2


class ufg_precond(C.Structure):
    _fields_ = [("kind", C.c_int), ("degree", C.c_int), ("eps", C.c_double),
                ("lam_max", C.c_double), ("alpha", C.c_double), ("wce_order", C.c_int),
                ("euler", C.c_int), ("euler_p", C.c_double)]


class ufg_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("mixed", C.c_int),
                ("delta", C.c_double), ("check_every", C.c_int), ("use_x0", C.c_int),
                ("eager", C.c_int)]


class ufg_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int * 2), ("mv", C.c_longlong), ("m0inv", C.c_longlong),
                ("sca_sweeps", C.c_longlong), ("reliable_updates", C.c_longlong),
                ("relres", C.c_double * 2), ("relres_normal", C.c_double),
                ("seconds", C.c_double), ("paper_mv", C.c_double), ("status", C.c_int),
                ("host_syncs", C.c_longlong), ("host_submits", C.c_longlong)]

    def as_dict(self):
        return dict(iters=(self.iters[0], self.iters[1]), mv=self.mv, m0inv=self.m0inv,
                    sca_sweeps=self.sca_sweeps, reliable_updates=self.reliable_updates,
                    relres=(self.relres[0], self.relres[1]), relres_normal=self.relres_normal,
                    seconds=self.seconds, paper_mv=self.paper_mv, status=self.status,
                    host_syncs=self.host_syncs, host_submits=self.host_submits)


class ufg_hmc_opts(C.Structure):
    _fields_ = [("dt", C.c_double), ("nsteps", C.c_int), ("tol", C.c_double),
                ("maxit", C.c_int), ("mixed", C.c_int), ("check_every", C.c_int),
                ("chrono", C.c_int)]


class ufg_hmc_result(C.Structure):
    _fields_ = [("S0", C.c_double), ("S1", C.c_double), ("K0", C.c_double),
                ("K1", C.c_double), ("dH", C.c_double), ("accept", C.c_int),
                ("status", C.c_int), ("forces", C.c_int), ("solves", C.c_longlong),
                ("iters", C.c_longlong), ("mv", C.c_longlong), ("worst_relres", C.c_double),
                ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_SIGNATURES = {
    "create_lattice_ex": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
                                    _P, C.POINTER(_P)]),
    "create_lattice_dim": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                     C.c_int, C.c_int, _P, C.POINTER(_P)]),
    "create_lattice": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _P,
                                 C.POINTER(_P)]),
    "destroy_lattice": (C.c_int, [_P]),
    "set_lattice_stream": (C.c_int, [_P, _P]),
    "set_aux_field": (C.c_int, [_P, _P]),
    "apply_M": (C.c_int, [_P, _P, _P, C.c_int]),
    "apply_Mdag": (C.c_int, [_P, _P, _P, C.c_int]),
    "apply_precond": (C.c_int, [_P, C.POINTER(ufg_precond), C.c_int, _P, _P, C.c_int]),
    "solve_cg_normal": (C.c_int, [_P, C.POINTER(ufg_precond), _P, _P, C.c_int,
                                  C.POINTER(ufg_solve_opts), C.POINTER(ufg_solve_stats)]),
    "solve_cg_split": (C.c_int, [_P, C.POINTER(ufg_precond), _P, _P, C.c_int,
                                 C.POINTER(ufg_solve_opts), C.POINTER(ufg_solve_stats)]),
    "solve_bicgstab": (C.c_int, [_P, C.POINTER(ufg_precond), C.c_int, _P, _P, C.c_int,
                                 C.POINTER(ufg_solve_opts), C.POINTER(ufg_solve_stats)]),
    "solve_batched": (C.c_int, [C.POINTER(_P), C.c_int, C.POINTER(_P), C.POINTER(_P),
                                C.POINTER(C.c_int), C.POINTER(ufg_precond),
                                C.POINTER(ufg_solve_opts), C.POINTER(ufg_solve_stats)]),
    "solve_batched_tune": (C.c_int, [C.c_int, C.c_int, C.c_longlong, C.c_int, C.c_int]),
    "force_dS_dsigma": (C.c_int, [_P, _P, _P, C.c_int, _P]),
    "lattice_tune": (C.c_int, [_P, C.c_int, C.c_int]),
    "lattice_tune_slabs": (C.c_int, [_P, C.c_int]),
    "lattice_tune_order": (C.c_int, [_P, C.c_int, C.c_int]),
    "lattice_tune_transform": (C.c_int, [_P, C.c_int]),
    "precond_lam_max": (C.c_int, [_P, C.POINTER(ufg_precond), C.POINTER(C.c_double)]),
    "hmc_leapfrog": (C.c_int, [_P, C.POINTER(ufg_precond), _P, _P, _P, C.c_int,
                               C.POINTER(ufg_hmc_opts), C.POINTER(C.c_double),
                               C.POINTER(ufg_hmc_result)]),
    "hmc_trajectory": (C.c_int, [_P, C.POINTER(ufg_precond), _P, _P, _P, C.c_int, C.c_double,
                                 C.POINTER(ufg_hmc_opts), _P, C.POINTER(C.c_double),
                                 C.POINTER(ufg_hmc_result)]),
    "lattice_norm2": (C.c_int, [_P, _P, C.c_int, C.POINTER(C.c_double)]),
    "lattice_norm2_noalloc": (C.c_int, [_P, _P, C.c_int, _P]),
    "ufg_device_copy": (C.c_int, [_P, _P, C.c_longlong, _P]),
    "lattice_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int),
                               C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "ufg_last_error": (C.c_char_p, []),
    "last_error": (C.c_char_p, []),
    "ufg_cheb_roots": (C.c_int, [C.c_int, C.c_double, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]),
    "ufg_euler_weights": (C.c_int, [C.c_int, C.c_double, C.POINTER(C.c_double)]),
    "ufg_transfer_matrix": (C.c_int, [C.c_int, C.c_double, C.POINTER(C.c_double)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libufg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1008_3647_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class UfgError(RuntimeError):
    def __init__(self, code, where):
        msg = load().ufg_last_error().decode(errors="replace")
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def check(code, where):
    if code < 0:
        raise UfgError(code, where)
    return code


@dataclass
class Precond:
    """Preconditioner description (mirrors ufg_precond)."""
    kind: str = "none"          # none | cheb | sca | wce | sca_cheb
    degree: int = 16
    eps: float = 1e-2
    lam_max: float = 0.0        # >0 given, 0 bound, <0 power iteration
    alpha: float = 2.0          # SCA shift (Sec. 4 leaves it to tuning)
    wce_order: int = 0
    euler: bool = False
    euler_p: float = 0.5

    def to_c(self):
        kinds = {"none": UFG_PC_NONE, "cheb": UFG_PC_CHEB, "sca": UFG_PC_SCA, "wce": UFG_PC_WCE,
                 "sca_cheb": UFG_PC_SCA_CHEB}
        return ufg_precond(kinds[self.kind], self.degree, self.eps, self.lam_max, self.alpha,
                           self.wce_order, int(self.euler), self.euler_p)


def solve_opts(tol=1e-10, maxit=10000, mixed=False, delta=0.1, check_every=10, use_x0=False,
               eager=False):
    return ufg_solve_opts(tol, maxit, int(mixed), delta, check_every, int(use_x0), int(eager))
