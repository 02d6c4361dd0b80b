"""Non-interacting matrix M0 = M|_{A=0} and its inverse (oracle; test infrastructure).

Paper, Sec. 3: M0^{-1} is diagonal in frequency-momentum space,
  [M0^{-1}]_{omega,k} = [1 - exp(-i omega - tau E(k))]^{-1},
with antiperiodic Matsubara frequencies omega = (2 n_tau + 1) pi / Ntau
("Fourier acceleration" through a 4D Fourier transform). The paper leaves a
constant normalisation open; it is fixed here by M0 M0^{-1} = 1.

The antiperiodic time direction is handled by the usual twist: with
u_t = exp(i pi t / Ntau) u~_t the twisted field u~ is periodic, so an ordinary
periodic FFT over t diagonalises the problem, and the periodic frequency
2 pi n / Ntau plus the twist pi / Ntau is exactly omega_n.
"""
from __future__ import annotations

import numpy as np

from .operator import kinetic_symbol


def _frequencies(ntau: int) -> np.ndarray:
    # periodic FFT frequency (numpy order) + antiperiodic twist = omega_n
    return 2.0 * np.pi * np.fft.fftfreq(ntau) + np.pi / ntau


def free_spectrum(nx: int, ntau: int, tau: float, dim: int = 3) -> np.ndarray:
    """Eigenvalues of M0: 1 - exp(-i omega) exp(-tau E(k)) on the (1 + dim)D grid."""
    lam = kinetic_symbol(nx, tau, "free", dim)
    w = _frequencies(ntau)
    return 1.0 - np.exp(-1j * w).reshape((ntau,) + (1,) * dim) * lam[None]


def _apply_symbol(v, tau, adjoint):
    ntau, nx, dim = v.shape[0], v.shape[-1], v.ndim - 1
    t = np.arange(ntau)
    twist = np.exp(-1j * np.pi * t / ntau).reshape((ntau,) + (1,) * dim)
    sym = free_spectrum(nx, ntau, tau, dim)
    if adjoint:
        # M0^T shifts the other way in time, u_t - e^{-tau K} u_{t+1}; under
        # the same twist its symbol is 1 - exp(+i omega) exp(-tau E(k)),
        # the complex conjugate of M0's symbol.
        sym = np.conj(sym)
    axes = tuple(range(dim + 1))
    vt = np.fft.fftn(v * twist, axes=axes)
    ut = np.fft.ifftn(vt / sym, axes=axes)
    return ut / twist


def apply_M0inv(v: np.ndarray, tau: float) -> np.ndarray:
    """u = M0^{-1} v via the antiperiodic (1 + d)-dimensional Fourier transform
    (paper, Sec. 3; 4D for d = 3); v is one vector [Ntau][Nx]^d."""
    return _apply_symbol(np.asarray(v, dtype=np.complex128), tau, adjoint=False)


def apply_M0inv_dag(v: np.ndarray, tau: float) -> np.ndarray:
    """u = M0^{-T} v (M0 is real, so its adjoint inverse is the transpose)."""
    return _apply_symbol(np.asarray(v, dtype=np.complex128), tau, adjoint=True)
