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


def free_spectrum(nx: int, ntau: int, tau: float) -> np.ndarray:
    """Eigenvalues of M0: 1 - exp(-i omega) exp(-tau E(k)) on the 4D grid."""
    lam = kinetic_symbol(nx, tau)
    w = _frequencies(ntau)
    return 1.0 - np.exp(-1j * w)[:, None, None, None] * lam[None]


def _apply_symbol(v, tau, adjoint):
    ntau, nx = v.shape[0], v.shape[-1]
    t = np.arange(ntau)
    twist = np.exp(-1j * np.pi * t / ntau)[:, None, None, None]
    sym = free_spectrum(nx, ntau, tau)
    if adjoint:
        # M0^T shifts the other way in time, u_t - e^{-tau K} u_{t+1}; under
        # the same twist its symbol is 1 - exp(+i omega) exp(-tau E(k)),
        # the complex conjugate of M0's symbol.
        sym = np.conj(sym)
    vt = np.fft.fftn(v * twist, axes=(0, 1, 2, 3))
    ut = np.fft.ifftn(vt / sym, axes=(0, 1, 2, 3))
    return ut / twist


def apply_M0inv(v: np.ndarray, tau: float) -> np.ndarray:
    """u = M0^{-1} v via the antiperiodic 4D Fourier transform (paper, Sec. 3)."""
    return _apply_symbol(np.asarray(v, dtype=np.complex128), tau, adjoint=False)


def apply_M0inv_dag(v: np.ndarray, tau: float) -> np.ndarray:
    """u = M0^{-T} v (M0 is real, so its adjoint inverse is the transpose)."""
    return _apply_symbol(np.asarray(v, dtype=np.complex128), tau, adjoint=True)
