"""Pins for the oracle's fermion matrix (paper, Sec. 1, Eq. MatrixM).

Each test checks the oracle against something other than itself: numbers the
paper prints, closed-form spectra and determinants, or a dense matrix built by
a different route (cosine-sum Kronecker product instead of FFTs).
"""
import os

import numpy as np
import pytest

import oracle
from oracle import operator as op
from synthetic import sigma_field, gaussian_rhs

HERE = os.path.dirname(__file__)
TAU, G = 0.05, 5.0


def test_coupling_matches_printed_values():
    # paper, Sec. 5: A ~ 0.52, 0.75, 0.95 for g = 2.5, 5, 7.5; A ~ 1.14 for g = 10
    rows = np.loadtxt(os.path.join(HERE, "golden", "paper_A_values.txt"))
    for g, a_printed, digits in rows:
        assert round(oracle.coupling_A(TAU, g), int(digits)) == pytest.approx(a_printed, abs=1e-12)


def test_momentum_grid_and_transfer_matrix():
    for nx in (2, 4, 6, 8):
        k = op.momenta(nx)
        assert len(k) == nx and k[0] == pytest.approx(-np.pi)
        T = op.transfer_matrix_1d(nx, TAU)
        assert np.allclose(T, T.T, atol=1e-15)
        # circulant: T[i, j] depends on (i - j) mod nx only
        for i in range(nx):
            assert np.allclose(np.roll(T[0], i), T[i], atol=1e-15)
        # eigenvalues are exp(-tau k^2 / 2) over the grid
        ev = np.sort(np.linalg.eigvalsh(T))
        assert np.allclose(ev, np.sort(np.exp(-TAU * k ** 2 / 2)), atol=1e-14)


def test_free_field_spectrum_closed_form():
    # Sec. 3: M0 is diagonal in (omega, k) with eigenvalues 1 - e^{-i omega} e^{-tau E(k)},
    # antiperiodic omega = (2n+1) pi / Ntau.
    nx, ntau = 4, 6
    sigma = sigma_field(nx, ntau, 11)
    M0 = op.dense_M(sigma, TAU, 0.0)
    ev = np.linalg.eigvals(M0)
    k = op.momenta(nx)
    E = (k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2).ravel() / 2
    w = (2 * np.arange(ntau) + 1) * np.pi / ntau
    closed = (1 - np.exp(-1j * w)[:, None] * np.exp(-TAU * E)[None, :]).ravel()
    # match as multisets
    key = lambda z: (np.round(z.real, 9), np.round(z.imag, 9))  # noqa: E731
    assert sorted(map(key, ev)) == sorted(map(key, closed))
    assert sorted(map(key, oracle.free_spectrum(nx, ntau, TAU).ravel())) == sorted(map(key, closed))


def test_free_determinant():
    # det M0 = prod_k (1 + exp(-tau Ntau E(k))) for the antiperiodic block-cyclic matrix
    nx, ntau = 4, 5
    M0 = op.dense_M(np.zeros((ntau, nx, nx, nx)), TAU, G)  # sigma = 0: b = 1, A drops out
    sign, logdet = np.linalg.slogdet(M0)
    k = op.momenta(nx)
    E = (k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2).ravel() / 2
    assert sign == 1.0
    assert logdet == pytest.approx(np.sum(np.log1p(np.exp(-TAU * ntau * E))), rel=1e-12)


def test_determinant_block_cyclic_identity():
    # det M = det(1 + B_{Ntau} ... B_1): the + sign pins the antiperiodic corner
    nx, ntau = 2, 5
    sigma = sigma_field(nx, ntau, 12)
    Md = op.dense_M(sigma, TAU, G)
    b = op.field_b(sigma, oracle.coupling_A(TAU, G))
    T3 = op.dense_expK(nx, TAU)
    prod = np.eye(nx ** 3)
    for t in range(ntau):
        prod = (T3 * b[t].reshape(-1)[None, :]) @ prod
    assert np.linalg.det(Md) == pytest.approx(np.linalg.det(np.eye(nx ** 3) + prod), rel=1e-10)
    # the periodic (wrong-sign) corner would give det(1 - prod) instead
    assert abs(np.linalg.det(np.eye(nx ** 3) - prod) - np.linalg.det(Md)) > 1e-3


@pytest.mark.parametrize("nx,ntau", [(2, 3), (4, 6), (4, 2)])
def test_matrix_free_equals_dense(nx, ntau):
    sigma = sigma_field(nx, ntau, 13)
    x = gaussian_rhs(nx, ntau, [14])[0]
    Md = op.dense_M(sigma, TAU, G)
    y = oracle.apply_M(x, sigma, TAU, G)
    assert np.allclose(y.ravel(), Md @ x.ravel(), atol=1e-13)
    yd = oracle.apply_Mdag(x, sigma, TAU, G)
    assert np.allclose(yd.ravel(), Md.T @ x.ravel(), atol=1e-13)
    M1 = op.dense_M1(sigma, TAU)
    assert np.allclose(oracle.apply_M1(x, sigma, TAU).ravel(), M1 @ x.ravel(), atol=1e-13)
    assert np.allclose(oracle.apply_M1dag(x, sigma, TAU).ravel(), M1.T @ x.ravel(), atol=1e-13)
    # M = M0 + A M1 (Sec. 3)
    M0 = op.dense_M(sigma, TAU, 0.0)
    assert np.allclose(Md, M0 + oracle.coupling_A(TAU, G) * M1, atol=1e-14)


def test_adjoint_identity():
    nx, ntau = 6, 8
    sigma = sigma_field(nx, ntau, 15)
    u, v = gaussian_rhs(nx, ntau, [16, 17])
    lhs = np.vdot(oracle.apply_M(u, sigma, TAU, G), v)
    rhs = np.vdot(u, oracle.apply_Mdag(v, sigma, TAU, G))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_zero_coupling_is_free_matrix():
    nx, ntau = 4, 6
    x = gaussian_rhs(nx, ntau, [18])[0]
    y1 = oracle.apply_M(x, sigma_field(nx, ntau, 19), TAU, 0.0)
    y2 = oracle.apply_M(x, sigma_field(nx, ntau, 20), TAU, 0.0)
    assert np.allclose(y1, y2, atol=1e-15)


def test_real_operator_does_not_mix_components():
    nx, ntau = 4, 4
    sigma = sigma_field(nx, ntau, 21)
    x = gaussian_rhs(nx, ntau, [22])[0]
    y = oracle.apply_M(x, sigma, TAU, G)
    yr = oracle.apply_M(x.real.astype(complex), sigma, TAU, G)
    assert np.allclose(y.real, yr.real, atol=1e-14) and np.allclose(yr.imag, 0, atol=1e-14)


def test_hubbard_transfer_is_matrix_exponential_of_hopping():
    """Hubbard-model dispersion (the extension the concluding section names):
    E(k) = 1 - cos k per axis is the symbol of H = 1 - (S+ + S-)/2 (S+- the
    periodic shifts), so the cosine-sum factor must equal expm(-tau H), computed
    here by scipy's Pade route; and E agrees with k^2/2 to O(k^4)."""
    from scipy.linalg import expm
    for nx in (2, 4, 6, 8, 12, 16):
        H = np.eye(nx)
        for i in range(nx):
            H[i, (i + 1) % nx] -= 0.5
            H[i, (i - 1) % nx] -= 0.5
        T = op.transfer_matrix_1d(nx, TAU, "hubbard")
        assert np.allclose(T, expm(-TAU * H), rtol=0, atol=1e-14), nx
        assert not np.allclose(T, op.transfer_matrix_1d(nx, TAU, "free"), atol=1e-6)
    k = np.linspace(-0.3, 0.3, 61)
    assert np.all(np.abs(op.dispersion(k, "hubbard") - k ** 2 / 2) <= k ** 4 / 24 + 1e-16)


@pytest.mark.parametrize("nx,ntau", [(2, 3), (4, 5)])
def test_hubbard_matrix_free_equals_dense(nx, ntau):
    """FFT route (symbol) against the Kronecker route (cosine sums) for the
    Hubbard dispersion, M and M^T, and the block-cyclic determinant identity."""
    sigma = sigma_field(nx, ntau, 15)
    x = gaussian_rhs(nx, ntau, [16])[0]
    Md = op.dense_M(sigma, TAU, G, "hubbard")
    assert np.allclose(oracle.apply_M(x, sigma, TAU, G, "hubbard").ravel(), Md @ x.ravel(),
                       atol=1e-13)
    assert np.allclose(oracle.apply_Mdag(x, sigma, TAU, G, "hubbard").ravel(),
                       Md.T @ x.ravel(), atol=1e-13)
    b = op.field_b(sigma, oracle.coupling_A(TAU, G))
    T3 = op.dense_expK(nx, TAU, "hubbard")
    prod = np.eye(nx ** 3)
    for t in range(ntau):
        prod = (T3 * b[t].reshape(-1)[None, :]) @ prod
    assert np.linalg.det(Md) == pytest.approx(np.linalg.det(np.eye(nx ** 3) + prod), rel=1e-10)
