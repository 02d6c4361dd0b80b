"""Pins for the oracle's M0^{-1} and preconditioners (paper, Secs. 2-4)."""
from math import log

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle
from oracle import operator as op
from oracle import precond as pc
from synthetic import sigma_field, gaussian_rhs

TAU, G = 0.05, 5.0


# ---------------------------------------------------------------- M0^{-1}

def test_m0inv_inverts_free_matrix():
    nx, ntau = 4, 10
    v = gaussian_rhs(nx, ntau, [31])[0]
    sig = sigma_field(nx, ntau, 32)
    u = oracle.apply_M0inv(v, TAU)
    assert np.allclose(oracle.apply_M(u, sig, TAU, 0.0), v, atol=1e-13)
    assert np.allclose(oracle.apply_M0inv(oracle.apply_M(v, sig, TAU, 0.0), TAU), v, atol=1e-13)
    ud = oracle.apply_M0inv_dag(v, TAU)
    assert np.allclose(oracle.apply_Mdag(ud, sig, TAU, 0.0), v, atol=1e-13)


def test_m0inv_matches_dense_inverse():
    nx, ntau = 2, 6
    v = gaussian_rhs(nx, ntau, [33])[0]
    M0 = op.dense_M(np.zeros((ntau, nx, nx, nx)), TAU, 0.0)
    assert np.allclose(oracle.apply_M0inv(v, TAU).ravel(), np.linalg.solve(M0, v.ravel()), atol=1e-13)
    assert np.allclose(oracle.apply_M0inv_dag(v, TAU).ravel(), np.linalg.solve(M0.T, v.ravel()), atol=1e-13)


# ---------------------------------------------------------------- Chebyshev

@pytest.mark.parametrize("degree", [8, 16, 32])
@pytest.mark.parametrize("eps", [1e-2, 1e-3])
def test_chebyshev_closed_form(degree, eps):
    # 1 - z P(z) = T_{2n+1}(x(z)) / T_{2n+1}(x(0)), x(z) = (1 + eps - 2 z) / (1 - eps):
    # the paper's roots are the non-zero roots of T_{2n+1}(x(z)) = T_{2n+1}(x(0)).
    z = np.linspace(eps, 1.0, 301)
    P = pc.cheb_scalar(z, degree, eps)
    assert np.max(np.abs(P.imag)) < 1e-9 * np.max(np.abs(P.real))
    coef = np.zeros(degree + 2)
    coef[-1] = 1.0
    x = lambda zz: (1 + eps - 2 * zz) / (1 - eps)  # noqa: E731
    closed = npcheb.chebval(x(z), coef) / npcheb.chebval(x(0.0), coef)
    assert np.allclose(1 - z * P.real, closed, atol=1e-11)
    # the paper's relative-error bound on [eps, 1]
    R = np.abs((P.real - 1 / z) * z)
    bound = 2 * ((1 - np.sqrt(eps)) / (1 + np.sqrt(eps))) ** (degree + 1)
    assert np.all(R <= bound * (1 + 1e-9))
    # normalisation: P((1+eps)/2) = 2/(1+eps), i.e. zP = 1 at the midpoint (T(0)=0)
    h = (1 + eps) / 2
    assert pc.cheb_scalar(h, degree, eps).real == pytest.approx(1 / h, rel=1e-10)


def test_chebyshev_positive_beyond_interval():
    z = np.concatenate([np.linspace(1e-6, 1e-3, 50), np.linspace(1, 3, 50)])
    assert np.all(pc.cheb_scalar(z, 16, 1e-2).real > 0)


def test_bit_reversal_order():
    assert list(pc.bit_reversal_order(8)) == [0, 4, 2, 6, 1, 5, 3, 7]
    assert sorted(pc.bit_reversal_order(32)) == list(range(32))
    with pytest.raises(ValueError):
        pc.bit_reversal_order(12)


def test_chebyshev_operator_via_eigendecomposition():
    nx, ntau = 2, 6
    sigma = sigma_field(nx, ntau, 34)
    v = gaussian_rhs(nx, ntau, [35])[0]
    Md = op.dense_M(sigma, TAU, G)
    Q = Md.T @ Md
    lam, V = np.linalg.eigh(Q)
    lam_max = 1.05 * lam[-1]
    deg, eps = 8, 1e-2
    ref = V @ (pc.cheb_scalar(lam / lam_max, deg, eps) * (V.T @ v.ravel()))
    out = pc.apply_cheb(v, sigma, TAU, G, deg, eps, lam_max)
    assert np.allclose(out.ravel(), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


# ---------------------------------------------------------------- SCA

def _dense_Mtilde_T_Mtilde(b):
    ntau = b.shape[0]
    Mt = np.eye(ntau)
    for t in range(ntau - 1):
        Mt[t + 1, t] = -b[t]
    Mt[0, ntau - 1] = b[ntau - 1]
    return Mt.T @ Mt


@pytest.mark.parametrize("alpha", [1.0, 1.5])
def test_sca_factorisation_and_fill(alpha):
    rng = np.random.default_rng(36)
    ntau = 7
    b = 1 + 0.75 * np.sin(rng.uniform(-np.pi, np.pi, ntau))
    D, L = pc.sca_factor(b, alpha)
    Ld, Dd = pc.sca_dense_factors(D, L)
    LDL = Ld @ Dd @ Ld.T
    ref = _dense_Mtilde_T_Mtilde(b) + (alpha - 1) * np.eye(ntau)
    fill = LDL - ref
    # the recursion reproduces M~^T M~ up to one symmetric fill-in pair at
    # (Ntau-1, 1) and (1, Ntau-1) (0-based), equal to -b_0 b_{Ntau-1} / D_0
    expect = np.zeros((ntau, ntau))
    expect[ntau - 1, 1] = expect[1, ntau - 1] = -b[0] * b[ntau - 1] / D[0]
    assert np.allclose(fill, expect, atol=1e-13)


def test_sca_exact_without_corner():
    rng = np.random.default_rng(37)
    ntau = 6
    b = 1 + 0.75 * np.sin(rng.uniform(-np.pi, np.pi, ntau))
    b[-1] = 0.0
    D, L = pc.sca_factor(b, 1.0)
    Ld, Dd = pc.sca_dense_factors(D, L)
    assert np.allclose(Ld @ Dd @ Ld.T, _dense_Mtilde_T_Mtilde(b), atol=1e-13)


def test_sca_apply_is_inverse_of_factorisation():
    nx, ntau = 2, 9
    sigma = sigma_field(nx, ntau, 38)
    v = gaussian_rhs(nx, ntau, [39])[0]
    D, L = pc.sca_setup(sigma, TAU, G, 1.25)
    x = pc.sca_apply(v, D, L)
    for n in range(nx ** 3):
        iz, iy, ix = np.unravel_index(n, (nx, nx, nx))
        Ld, Dd = pc.sca_dense_factors(D[:, iz, iy, ix], L[:, iz, iy, ix])
        ref = np.linalg.solve(Ld @ Dd @ Ld.T, v[:, iz, iy, ix])
        assert np.allclose(x[:, iz, iy, ix], ref, atol=1e-12)


# ---------------------------------------------------------------- WCE / Euler

def test_wce_order0_is_free_inverse():
    nx, ntau = 4, 8
    sigma = sigma_field(nx, ntau, 40)
    v = gaussian_rhs(nx, ntau, [41])[0]
    assert np.allclose(pc.wce_apply(v, sigma, TAU, G, 0), oracle.apply_M0inv(v, TAU), atol=1e-15)
    assert np.allclose(pc.wce_apply_dag(v, sigma, TAU, G, 0), oracle.apply_M0inv_dag(v, TAU), atol=1e-15)


@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_wce_truncation_identity(d):
    # M W_d = 1 - M0 (-A X)^{d+1} M0^{-1} exactly (fixes the signs and the order)
    nx, ntau = 2, 6
    sigma = sigma_field(nx, ntau, 42)
    v = gaussian_rhs(nx, ntau, [43])[0].ravel()
    Md = op.dense_M(sigma, TAU, G)
    M0 = op.dense_M(sigma, TAU, 0.0)
    M1 = op.dense_M1(sigma, TAU)
    A = oracle.coupling_A(TAU, G)
    X = np.linalg.solve(M0, M1)
    rhs = v - M0 @ np.linalg.matrix_power(-A * X, d + 1) @ np.linalg.solve(M0, v)
    W = pc.wce_apply(v.reshape(sigma.shape), sigma, TAU, G, d).ravel()
    assert np.allclose(Md @ W, rhs, atol=1e-12)
    # transpose: W_d^T M^T = 1 - M0^{-T} ((-A X)^T)^{d+1} M0^T
    WT = pc.wce_apply_dag(v.reshape(sigma.shape), sigma, TAU, G, d).ravel()
    Wd = np.linalg.matrix_power(-A * X, 0)
    Wd = sum(np.linalg.matrix_power(-A * X, m) for m in range(d + 1)) @ np.linalg.inv(M0)
    assert np.allclose(WT, Wd.T @ v, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 4])
def test_wce_euler_adjointness(d):
    nx, ntau = 4, 6
    sigma = sigma_field(nx, ntau, 44)
    u, v = gaussian_rhs(nx, ntau, [45, 46])
    for euler in (False, True):
        lhs = np.vdot(pc.wce_apply(u, sigma, TAU, G, d, euler), v)
        rhs = np.vdot(u, pc.wce_apply_dag(v, sigma, TAU, G, d, euler))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_euler_recursion_geometric_closed_form():
    # For S_{0,k} = sum_{n<=k} (-x)^n the recursion with p = 1/2 gives
    # S_{K,0} = [1 + x ((1 - x)/2)^K] / (1 + x)   (derived by hand).
    for x in (0.3, 0.8, 1.5):
        for K in (1, 2, 4, 7):
            partial = np.cumsum([(-x) ** n for n in range(K + 1)])
            est = pc.euler_estimate(list(partial), 0.5)
            assert est == pytest.approx((1 + x * ((1 - x) / 2) ** K) / (1 + x), rel=1e-13)


def test_euler_accelerates_alternating_series():
    # ln 2 = 1 - 1/2 + 1/3 - ...: Euler's estimate from 9 terms beats the raw sum
    partial = np.cumsum([(-1) ** n / (n + 1) for n in range(9)])
    raw_err = abs(partial[-1] - log(2))
    eul_err = abs(pc.euler_estimate(list(partial)) - log(2))
    assert eul_err < raw_err / 50


def test_euler_weights_closed_form():
    assert np.allclose(pc.euler_weights(2), [1, 3 / 4, 1 / 4])
    assert np.allclose(pc.euler_weights(4), [1, 15 / 16, 11 / 16, 5 / 16, 1 / 16])
    rng = np.random.default_rng(47)
    for d in range(0, 6):
        terms = rng.standard_normal(d + 1)
        est = pc.euler_estimate(list(np.cumsum(terms)))
        assert est == pytest.approx(np.dot(pc.euler_weights(d), terms), rel=1e-13)


@pytest.mark.parametrize("degree", [4, 8])
def test_sca_chebyshev_filter_via_eigendecomposition(degree):
    """apply_sca_cheb (P = P_2n(S Q / lam_max) S) against a dense route that
    does not use its factor sweep: S = (L^T D L)^{-1} assembled per site from
    the dense factors, H = S^{1/2} Q S^{1/2} = V diag(lam) V^H (Hermitian, similar
    to S Q), P = S^{1/2} V p(lam / lam_max) V^H S^{1/2} with the scalar
    polynomial p (cheb_scalar, pinned by the Chebyshev closed form). With
    lam_max above the largest lam, P is Hermitian positive definite."""
    nx, ntau, alpha, eps = 2, 6, 1.5, 1e-2
    V = nx ** 3
    N = V * ntau
    sigma = sigma_field(nx, ntau, 91)
    v = gaussian_rhs(nx, ntau, [92])[0]
    D, L = pc.sca_setup(sigma, TAU, G, alpha)
    S = np.zeros((N, N))
    for n in range(V):
        iz, iy, ix = np.unravel_index(n, (nx, nx, nx))
        Ld, Dd = pc.sca_dense_factors(D[:, iz, iy, ix], L[:, iz, iy, ix])
        Sn = np.linalg.inv(Ld @ Dd @ Ld.T)
        idx = np.arange(ntau) * V + n
        S[np.ix_(idx, idx)] = Sn
    Md = op.dense_M(sigma, TAU, G)
    w, U = np.linalg.eigh(S)
    assert w.min() > 0
    Sh = (U * np.sqrt(w)) @ U.T
    lam, Vh = np.linalg.eigh(Sh @ (Md.T @ Md) @ Sh)
    lam_max = 1.02 * lam[-1]
    p = pc.cheb_scalar(lam / lam_max, degree, eps)
    assert np.all(p.real > 0) and np.max(np.abs(p.imag)) < 1e-10 * np.max(np.abs(p))
    P = Sh @ (Vh * p) @ Vh.conj().T @ Sh
    got = pc.apply_sca_cheb(v, sigma, TAU, G, degree, eps, lam_max, alpha)
    ref = (P @ v.ravel()).reshape(v.shape)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))
