"""Fermion matrix M[sigma] of the unitary Fermi gas (oracle; test infrastructure).

Definition (paper, Sec. 1, Eq. MatrixM and the text after it):
  * M is block cyclic over Ntau time slices: unit diagonal blocks, -B_j on the
    block sub-diagonal and +B_{Ntau} in the top-right corner (the sign that
    makes the time direction antiperiodic).
  * B_j = exp(-tau K) (1 + A sin sigma_j), sigma_j the diagonal matrix of the
    field on slice j, A = sqrt(2) sqrt(exp(tau g) - 1).
  * K is diagonal in momentum space with E(k) = k^2 / 2 (hbar = m = 1, lattice
    spacing 1), k_i = 2 pi n_i / Nx, n_i = -Nx/2 .. Nx/2-1.
  * disp="hubbard" (the other dispersion the concluding section names, that of
    the Hubbard model): E(k) = sum_i (1 - cos k_i), nearest-neighbour hopping of
    amplitude 1/2, equal to k^2 / 2 up to O(k^4). Everything else is unchanged.
  * M is real, so M^dagger = M^T.
  * Lower dimensions (the concluding section names them as an extension): a
    slice has Nx^d sites for d = 1, 2, 3 and E(k) sums over the d axes; the
    dimension of a vector or field is read off its number of axes (one time
    axis plus d spatial axes).

0-based restatement used everywhere: with b_t = 1 + A sin sigma(., t),
  (M x)_{t+1 mod Ntau} = x_{t+1} + s_t e^{-tau K}(b_t x_t),
  s_t = -1 for t < Ntau-1 and s_{Ntau-1} = +1,
  (M^T x)_t = x_t + s_t b_t e^{-tau K} x_{t+1 mod Ntau}.

exp(-tau K) is applied literally as its definition says: a d-dimensional
FFT of the slice, a multiplication by exp(-tau E(k)), and the inverse FFT.
"""
from __future__ import annotations

import numpy as np


def coupling_A(tau: float, g: float) -> float:
    """A = sqrt(2) sqrt(exp(tau g) - 1) (paper, Sec. 1, below Eq. MatrixM)."""
    return float(np.sqrt(2.0) * np.sqrt(np.exp(tau * g) - 1.0))


def momenta(nx: int) -> np.ndarray:
    """k = 2 pi n / Nx for n = -Nx/2 .. Nx/2-1 (paper, Sec. 1)."""
    n = np.arange(-(nx // 2), nx // 2)
    return 2.0 * np.pi * n / nx


def _fft_momenta(nx: int) -> np.ndarray:
    # the same set of momenta as momenta(), listed in numpy's FFT order
    return 2.0 * np.pi * np.fft.fftfreq(nx)


DISPERSIONS = ("free", "hubbard")


def dispersion(k, disp: str = "free"):
    """Per-axis kinetic energy: k^2 / 2 (hbar = m = 1, paper Sec. 1), or
    1 - cos k for the Hubbard-model dispersion."""
    k = np.asarray(k)
    if disp == "free":
        return 0.5 * k ** 2
    if disp == "hubbard":
        return 1.0 - np.cos(k)
    raise ValueError(f"unknown dispersion {disp!r}")


def kinetic_symbol(nx: int, tau: float, disp: str = "free", dim: int = 3) -> np.ndarray:
    """exp(-tau E(k)) on the dim-dimensional momentum grid, numpy FFT order,
    axes (z, y, x) for dim = 3 (the last dim of them for dim < 3)."""
    k = _fft_momenta(nx)
    grids = np.meshgrid(*([k] * dim), indexing="ij")
    return np.exp(-tau * sum(dispersion(ki, disp) for ki in grids))


def apply_expK(v: np.ndarray, tau: float, disp: str = "free", dim: int = 3) -> np.ndarray:
    """exp(-tau K) applied to every slice of v (its last `dim` axes).

    K is diagonal in momentum space, so: FFT, multiply, inverse FFT.
    """
    nx = v.shape[-1]
    sym = kinetic_symbol(nx, tau, disp, dim)
    axes = tuple(range(-dim, 0))
    return np.fft.ifftn(np.fft.fftn(v, axes=axes) * sym, axes=axes)


def spatial_dim(a: np.ndarray) -> int:
    """Spatial dimension of a field or vector [Ntau][Nx]^d."""
    return a.ndim - 1


def field_b(sigma: np.ndarray, A: float) -> np.ndarray:
    """Diagonal of the auxiliary-field factor 1 + A sin sigma (paper, Sec. 1)."""
    return 1.0 + A * np.sin(sigma)


def _sign(t: int, ntau: int) -> float:
    # block (t+1, t) carries -B; the corner block (0, Ntau-1) carries +B
    return 1.0 if t == ntau - 1 else -1.0


def apply_M(x: np.ndarray, sigma: np.ndarray, tau: float, g: float,
            disp: str = "free") -> np.ndarray:
    """y = M[sigma] x for one vector x shaped [Ntau][Nx]^d (d = 3: [Ntau][Nx][Nx][Nx])."""
    A = coupling_A(tau, g)
    b = field_b(sigma, A)
    ntau, d = x.shape[0], spatial_dim(sigma)
    y = np.array(x, dtype=np.complex128, copy=True)
    for t in range(ntau):
        y[(t + 1) % ntau] += _sign(t, ntau) * apply_expK(b[t] * x[t], tau, disp, d)
    return y


def apply_Mdag(x: np.ndarray, sigma: np.ndarray, tau: float, g: float,
               disp: str = "free") -> np.ndarray:
    """y = M^T x (M is real, paper Sec. 1)."""
    A = coupling_A(tau, g)
    b = field_b(sigma, A)
    ntau, d = x.shape[0], spatial_dim(sigma)
    y = np.array(x, dtype=np.complex128, copy=True)
    for t in range(ntau):
        y[t] += _sign(t, ntau) * b[t] * apply_expK(x[(t + 1) % ntau], tau, disp, d)
    return y


def apply_M1(x: np.ndarray, sigma: np.ndarray, tau: float) -> np.ndarray:
    """y = M1 x: the A-linear part of M, blocks C_j = exp(-tau K) sin sigma_j,
    zero diagonal (paper, Sec. 3, Eq. MatrixM_1)."""
    ntau, d = x.shape[0], spatial_dim(sigma)
    s = np.sin(sigma)
    y = np.zeros_like(x, dtype=np.complex128)
    for t in range(ntau):
        y[(t + 1) % ntau] += _sign(t, ntau) * apply_expK(s[t] * x[t], tau, "free", d)
    return y


def apply_M1dag(x: np.ndarray, sigma: np.ndarray, tau: float) -> np.ndarray:
    """y = M1^T x."""
    ntau, d = x.shape[0], spatial_dim(sigma)
    s = np.sin(sigma)
    y = np.zeros_like(x, dtype=np.complex128)
    for t in range(ntau):
        y[t] += _sign(t, ntau) * s[t] * apply_expK(x[(t + 1) % ntau], tau, "free", d)
    return y


def apply_Q(x, sigma, tau, g, disp="free"):
    """Q x = M^T M x (paper, Sec. 1, Eq. 1)."""
    return apply_Mdag(apply_M(x, sigma, tau, g, disp), sigma, tau, g, disp)


# ---------------------------------------------------------------------------
# Dense builders for tiny lattices (N <= a few thousand). These take a
# different route from the FFT above: exp(-tau K) in position space is the
# Kronecker product of d Nx x Nx matrices built from the cosine sum.


def transfer_matrix_1d(nx: int, tau: float, disp: str = "free") -> np.ndarray:
    """T_{xy} = (1/Nx) sum_m exp(-tau E(k_m)) exp(i k_m (x - y)), real.

    One-dimensional factor of exp(-tau K); K separates over the axes.
    """
    k = momenta(nx)
    x = np.arange(nx)
    d = x[:, None] - x[None, :]
    T = np.zeros((nx, nx))
    for km in k:
        T += np.exp(-tau * dispersion(km, disp)) * np.cos(km * d)
    return T / nx


def dense_expK(nx: int, tau: float, disp: str = "free", dim: int = 3) -> np.ndarray:
    T = transfer_matrix_1d(nx, tau, disp)
    out = T
    for _ in range(dim - 1):
        out = np.kron(T, out)  # site index (z*Nx + y)*Nx + x for dim = 3
    return out


def _dense_blocks(diag_fields, nx, tau, identity=True, disp="free"):
    ntau, d = diag_fields.shape[0], spatial_dim(diag_fields)
    V = nx ** d
    T3 = dense_expK(nx, tau, disp, d)
    Mx = np.eye(ntau * V) if identity else np.zeros((ntau * V, ntau * V))
    for t in range(ntau):
        r = (t + 1) % ntau
        blk = _sign(t, ntau) * T3 * diag_fields[t].reshape(-1)[None, :]
        Mx[r * V:(r + 1) * V, t * V:(t + 1) * V] += blk
    return Mx


def dense_M(sigma, tau, g, disp="free"):
    """Dense real M[sigma], index (t*V + n); tiny lattices only."""
    nx = sigma.shape[-1]
    return _dense_blocks(field_b(sigma, coupling_A(tau, g)), nx, tau, True, disp)


def dense_M1(sigma, tau):
    nx = sigma.shape[-1]
    return _dense_blocks(np.sin(sigma), nx, tau, False)
