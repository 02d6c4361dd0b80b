"""Pins for the oracle's lattices of spatial dimension 1 and 2 (the lower
dimensions the paper's concluding section names as an extension; the
definitions of Sec. 1 with Nx^d sites per slice and E(k) summed over d axes).

Pinned against things other than the FFT route itself: the free spectrum and
determinant in closed form, the block-cyclic determinant identity, dense
matrices built from the cosine-sum Kronecker product, and the embedding of a
d-dimensional lattice into a (d+1)-dimensional one whose field and vector do
not depend on the extra axis (a momentum-k mode along that axis multiplies
the hopping blocks by exp(-tau E(k))), which ties both to the 3D operator.
"""
import numpy as np
import pytest

import oracle
from oracle import operator as op
from oracle import force as fo
from oracle import precond as pc
from synthetic import sigma_field, gaussian_rhs

TAU, G = 0.05, 5.0


def _E(nx, dim, disp="free"):
    k = op.momenta(nx)
    grids = np.meshgrid(*([k] * dim), indexing="ij")
    return sum(op.dispersion(g, disp) for g in grids).ravel()


@pytest.mark.parametrize("dim,nx,ntau", [(1, 6, 5), (2, 4, 5)])
def test_free_spectrum_and_determinant_closed_form(dim, nx, ntau):
    # Sec. 3: M0 is diagonal in (omega, k): 1 - e^{-i omega} e^{-tau E(k)},
    # omega = (2n+1) pi / Ntau; det M0 = prod_k (1 + e^{-tau Ntau E(k)})
    sigma = sigma_field(nx, ntau, 601, dim)
    M0 = op.dense_M(sigma, TAU, 0.0)
    assert M0.shape == (ntau * nx ** dim,) * 2
    E = _E(nx, dim)
    w = (2 * np.arange(ntau) + 1) * np.pi / ntau
    closed = (1 - np.exp(-1j * w)[:, None] * np.exp(-TAU * E)[None, :]).ravel()
    key = lambda z: (np.round(z.real, 9), np.round(z.imag, 9))  # noqa: E731
    assert sorted(map(key, np.linalg.eigvals(M0))) == sorted(map(key, closed))
    assert sorted(map(key, oracle.free_spectrum(nx, ntau, TAU, dim).ravel())) == \
        sorted(map(key, closed))
    sign, logdet = np.linalg.slogdet(M0)
    assert sign == 1.0
    assert logdet == pytest.approx(np.sum(np.log1p(np.exp(-TAU * ntau * E))), rel=1e-12)


@pytest.mark.parametrize("dim,nx", [(1, 4), (2, 2)])
def test_determinant_block_cyclic_identity(dim, nx):
    ntau = 5
    sigma = sigma_field(nx, ntau, 602, dim)
    Md = op.dense_M(sigma, TAU, G)
    b = op.field_b(sigma, oracle.coupling_A(TAU, G))
    Td = op.dense_expK(nx, TAU, "free", dim)
    prod = np.eye(nx ** dim)
    for t in range(ntau):
        prod = (Td * b[t].reshape(-1)[None, :]) @ prod
    assert np.linalg.det(Md) == pytest.approx(np.linalg.det(np.eye(nx ** dim) + prod), rel=1e-10)


@pytest.mark.parametrize("disp", ["free", "hubbard"])
@pytest.mark.parametrize("dim,nx,ntau", [(1, 8, 6), (1, 2, 3), (2, 4, 4), (2, 6, 3)])
def test_matrix_free_equals_dense(dim, nx, ntau, disp):
    sigma = sigma_field(nx, ntau, 603, dim)
    x = gaussian_rhs(nx, ntau, [604], dim)[0]
    Md = op.dense_M(sigma, TAU, G, disp)
    assert np.allclose(oracle.apply_M(x, sigma, TAU, G, disp).ravel(), Md @ x.ravel(), atol=1e-13)
    assert np.allclose(oracle.apply_Mdag(x, sigma, TAU, G, disp).ravel(), Md.T @ x.ravel(),
                       atol=1e-13)
    if disp == "free":
        M1 = op.dense_M1(sigma, TAU)
        assert np.allclose(oracle.apply_M1(x, sigma, TAU).ravel(), M1 @ x.ravel(), atol=1e-13)
        assert np.allclose(oracle.apply_M1dag(x, sigma, TAU).ravel(), M1.T @ x.ravel(),
                           atol=1e-13)


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_embedding_along_an_extra_axis(dim, m):
    """A (d+1)-dimensional vector e^{i k_m y} f with a field independent of y:
    M_{d+1} x = e^{i k_m y} [f + c (M_d f - f)], c = exp(-tau E(k_m)) with k_m
    folded into [-pi, pi) (the momentum grid of Sec. 1); at m = 0 the
    (d+1)-dimensional operator reduces to the d-dimensional one."""
    nx, ntau = 4, 5
    sig_d = sigma_field(nx, ntau, 605 + dim, dim)
    f = gaussian_rhs(nx, ntau, [606 + dim], dim)[0]
    # the extra axis is the slowest spatial axis (z for d + 1 = 3, y for 2)
    sig_up = np.repeat(sig_d[:, None], nx, axis=1)
    k = 2 * np.pi * m / nx
    phase = np.exp(1j * k * np.arange(nx)).reshape((1, nx) + (1,) * dim)
    x_up = phase * f[:, None]
    kf = 2 * np.pi * ((m + nx // 2) % nx - nx // 2) / nx  # the grid's momentum, in [-pi, pi)
    c = np.exp(-TAU * 0.5 * kf ** 2)
    for apply in (oracle.apply_M, oracle.apply_Mdag):
        lo = apply(f, sig_d, TAU, G)
        ref = phase * (f + c * (lo - f))[:, None]
        assert np.allclose(apply(x_up, sig_up, TAU, G), ref, atol=1e-13)


@pytest.mark.parametrize("dim,nx,ntau", [(1, 8, 10), (2, 4, 6)])
def test_m0inv_inverts_free_matrix(dim, nx, ntau):
    v = gaussian_rhs(nx, ntau, [607], dim)[0]
    sig = sigma_field(nx, ntau, 608, dim)
    assert np.allclose(oracle.apply_M(oracle.apply_M0inv(v, TAU), sig, TAU, 0.0), v, atol=1e-13)
    assert np.allclose(oracle.apply_Mdag(oracle.apply_M0inv_dag(v, TAU), sig, TAU, 0.0), v,
                       atol=1e-13)
    M0 = op.dense_M(np.zeros((ntau,) + (nx,) * dim), TAU, 0.0)
    assert np.allclose(oracle.apply_M0inv(v, TAU).ravel(), np.linalg.solve(M0, v.ravel()),
                       atol=1e-12)


@pytest.mark.parametrize("dim,nx", [(1, 6), (2, 2)])
def test_wce_series_converges_to_the_inverse(dim, nx):
    """Eq. WCE: the truncated series approaches M^{-1} v with the order at small A."""
    ntau = 6
    g = 0.5
    sigma = sigma_field(nx, ntau, 609, dim)
    v = gaussian_rhs(nx, ntau, [610], dim)[0]
    exact = np.linalg.solve(op.dense_M(sigma, TAU, g), v.ravel())
    errs = [np.linalg.norm(pc.wce_apply(v, sigma, TAU, g, d).ravel() - exact) for d in range(5)]
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:]))
    exact_t = np.linalg.solve(op.dense_M(sigma, TAU, g).T, v.ravel())
    assert np.linalg.norm(pc.wce_apply_dag(v, sigma, TAU, g, 4).ravel() - exact_t) < errs[4] * 10


@pytest.mark.parametrize("dim,nx", [(1, 4), (2, 2)])
def test_gradient_against_central_differences(dim, nx):
    ntau = 4
    sigma = sigma_field(nx, ntau, 611, dim)
    phi = gaussian_rhs(nx, ntau, [612], dim)[0]

    def action(s):
        y = np.linalg.solve(op.dense_M(s, TAU, G).T, phi.ravel())
        return float(np.vdot(y, y).real)

    Md = op.dense_M(sigma, TAU, G)
    y = np.linalg.solve(Md.T, phi.ravel())
    X = np.linalg.solve(Md, y).reshape(sigma.shape)
    grad = fo.gradient(X, sigma, TAU, G)
    h = 1e-5
    for idx in [(0,) + (0,) * dim, (ntau - 1,) + (nx - 1,) * dim, (1,) + (1,) * dim]:
        sp, sm = sigma.copy(), sigma.copy()
        sp[idx] += h
        sm[idx] -= h
        fd = (action(sp) - action(sm)) / (2 * h)
        assert grad[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)
