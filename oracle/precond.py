"""The paper's three preconditioners (oracle; test infrastructure).

Chebyshev  : paper Sec. 2 (Eq. ChebInv, its coefficient, roots and error bound)
Weak coupl.: paper Sec. 3 (M = M0 + A M1, Eq. WCE) and Sec. 3.1 (Euler, Eq. Euler)
Strong c.  : paper Sec. 4 (L^dagger D L factorisation and its recursions)

Readings where the paper is silent or ambiguous (all listed in the design notes):
  * Chebyshev spectrum normalisation: Q^ = Q / lam_max, lam_max is an input.
  * "Bit-reversal ordering": with 2n = 2^m factors and 0-based root index
    j = k-1, factor i (i = 0..2n-1) uses root j = bitrev_m(i).
  * SCA: the t = 1 recursion refers to an undefined D_0; it is read as
    D_1 = alpha + B_{0,1}^2 (the 0-based first slice).
  * Euler: the estimate is S_{kmax,0} of the recursion Eq. (Euler); the
    paper's b_n expression is the classical Euler transform of the infinite
    series, which does not equal that finite estimate, so the recursion is
    what is implemented.
"""
from __future__ import annotations

from math import comb

import numpy as np

from .operator import apply_M1, apply_M1dag, apply_Q, coupling_A, field_b
from .freefield import apply_M0inv, apply_M0inv_dag


# --------------------------------------------------------------------------
# Chebyshev polynomial approximation of 1/z (paper, Sec. 2)


def cheb_roots(degree: int, eps: float) -> np.ndarray:
    """z_{2n,k}, k = 1..2n, for a polynomial of degree 2n = ``degree``."""
    two_n = degree
    k = np.arange(1, two_n + 1)
    th = 2.0 * np.pi * k / (two_n + 1)
    return 0.5 * (1.0 + eps) * (1.0 - np.cos(th)) - 1j * np.sqrt(eps) * np.sin(th)


def cheb_constant(degree: int, eps: float) -> complex:
    """c_{2n} from c^{-1} = (1+eps)/2 prod_k ((1+eps)/2 - z_k)."""
    z = cheb_roots(degree, eps)
    h = 0.5 * (1.0 + eps)
    return 1.0 / (h * np.prod(h - z))


def cheb_scalar(z, degree: int, eps: float):
    """P(z) = c prod_k (z - z_k), evaluated on scalars/arrays."""
    roots = cheb_roots(degree, eps)
    z = np.asarray(z, dtype=np.complex128)
    out = np.full(z.shape, cheb_constant(degree, eps), dtype=np.complex128)
    for r in roots:
        out = out * (z - r)
    return out


def bit_reversal_order(degree: int) -> np.ndarray:
    """0-based root indices in the order the factors are applied."""
    m = int(round(np.log2(degree)))
    if 2 ** m != degree:
        raise ValueError("bit-reversal ordering needs a power-of-two degree")
    order = []
    for i in range(degree):
        r = 0
        for bit in range(m):
            if i >> bit & 1:
                r |= 1 << (m - 1 - bit)
        order.append(r)
    return np.array(order)


def apply_cheb(v, sigma, tau, g, degree, eps, lam_max):
    """P(Q^) v, Q^ = Q / lam_max, factors applied in bit-reversal order.

    The constant c is spread as c^{1/(2n)} over the factors (the product
    commutes, so only rounding depends on this choice).
    """
    roots = cheb_roots(degree, eps)
    c = cheb_constant(degree, eps)
    cf = c ** (1.0 / degree)
    y = np.array(v, dtype=np.complex128, copy=True)
    for j in bit_reversal_order(degree):
        y = cf * (apply_Q(y, sigma, tau, g) / lam_max - roots[j] * y)
    return y


def apply_sca_cheb(v, sigma, tau, g, degree, eps, lam_max, alpha=1.0):
    """Strong coupling with the Chebyshev polynomial as a secondary filter
    (paper, Sec. 4, closing remark; Sec. 2 for the polynomial).

    Reading: the strong-coupling inverse S = (L^dagger D L)^{-1} ~ Q^{-1} is
    applied first, and the Chebyshev approximation of 1/z then acts on the
    S-preconditioned operator: P v = P_2n(S Q / lam_max) S v, with lam_max the
    largest eigenvalue of S Q (real and positive: S Q is similar to the
    Hermitian S^{1/2} Q S^{1/2}), so P ~ (S Q)^{-1} S = Q^{-1}. Factors in
    bit-reversal order with c^{1/(2n)} each, as in apply_cheb.
    """
    D, L = sca_setup(sigma, tau, g, alpha)
    roots = cheb_roots(degree, eps)
    cf = cheb_constant(degree, eps) ** (1.0 / degree)
    y = sca_apply(v, D, L)
    for j in bit_reversal_order(degree):
        y = cf * (sca_apply(apply_Q(y, sigma, tau, g), D, L) / lam_max - roots[j] * y)
    return y


# --------------------------------------------------------------------------
# Strong-coupling approximation (paper, Sec. 4)


def sca_setup(sigma, tau, g, alpha=1.0):
    """Blocks D_t, L_t (per site) of M~^dagger M~ ~ L^dagger D L.

    M~ is M with B_j -> B_{0,j} = 1 + A sin sigma_j (diagonal in position).
    """
    return sca_factor(field_b(sigma, coupling_A(tau, g)), alpha)


def sca_factor(b, alpha=1.0):
    """The recursions of Sec. 4 for a given diagonal b_t (0-based):
      D_0 = alpha + b_0^2
      D_t = alpha + b_t^2 - b_{t-1}^2 / D_{t-1},                1 <= t <= Ntau-2
      D_{Ntau-1} = alpha + b^2 - b_{Ntau-2}^2 / D_{Ntau-2} - b_{Ntau-1}^2 / D_0
      L_t = b_t / D_t (t <= Ntau-2),  L_{Ntau-1} = b_{Ntau-1} / D_0 (corner).
    """
    ntau = b.shape[0]
    D = np.empty_like(b)
    L = np.empty_like(b)
    D[0] = alpha + b[0] ** 2
    for t in range(1, ntau):
        D[t] = alpha + b[t] ** 2 - b[t - 1] ** 2 / D[t - 1]
    D[ntau - 1] -= b[ntau - 1] ** 2 / D[0]
    for t in range(ntau - 1):
        L[t] = b[t] / D[t]
    L[ntau - 1] = b[ntau - 1] / D[0]
    return D, L


def sca_apply(v, D, L):
    """x = L^{-1} D^{-1} L^{dagger -1} v, per site (paper, Sec. 4).

    L^dagger is unit lower bidiagonal with -L_t below the diagonal and the
    corner L_{Ntau-1} in row Ntau-1, column 0; its inverse is the forward
    recursion printed in the paper. L^{-1} is the matching backward sweep.
    """
    ntau = v.shape[0]
    w = np.array(v, dtype=np.complex128, copy=True)
    for t in range(1, ntau):
        w[t] = v[t] + L[t - 1] * w[t - 1]
    w[ntau - 1] -= L[ntau - 1] * w[0]
    w = w / D
    x = np.empty_like(w)
    x[ntau - 1] = w[ntau - 1]
    for t in range(ntau - 2, 0, -1):
        x[t] = w[t] + L[t] * x[t + 1]
    x[0] = w[0] + L[0] * x[1] - L[ntau - 1] * x[ntau - 1] if ntau > 1 else w[0]
    return x


def sca_dense_factors(D, L):
    """Dense per-time matrices L^dagger and D for one site (tests only)."""
    ntau = D.shape[0]
    Ld = np.eye(ntau)
    for t in range(ntau - 1):
        Ld[t + 1, t] = -L[t]
    Ld[ntau - 1, 0] += L[ntau - 1]
    return Ld, np.diag(D)


# --------------------------------------------------------------------------
# Weak-coupling expansion (paper, Sec. 3) and Euler acceleration (Sec. 3.1)


def euler_estimate(partial_sums, p=0.5):
    """S_{kmax,0} from S_{j+1,k} = p S_{j,k} + (1-p) S_{j,k+1} (Eq. Euler).

    ``partial_sums`` is a list of S_{0,k}, k = 0..kmax (scalars or arrays).
    """
    S = list(partial_sums)
    while len(S) > 1:
        S = [p * S[k] + (1.0 - p) * S[k + 1] for k in range(len(S) - 1)]
    return S[0]


def wce_apply(v, sigma, tau, g, order, euler=False, p=0.5):
    """W_d v ~ M^{-1} v from Eq. (WCE): sum_{m<=d} (-A X)^m M0^{-1} v, X = M0^{-1} M1.

    With ``euler`` the partial sums S_{0,k} are accelerated by the Euler
    recursion and the estimate S_{d,0} is returned.
    """
    A = coupling_A(tau, g)
    u = apply_M0inv(v, tau)
    partial = [u.copy()]
    for _ in range(order):
        u = -A * apply_M0inv(apply_M1(u, sigma, tau), tau)
        partial.append(partial[-1] + u)
    if euler:
        return euler_estimate(partial, p)
    return partial[-1]


def wce_apply_dag(v, sigma, tau, g, order, euler=False, p=0.5):
    """W_d^T v ~ M^{-T} v: the transpose of the truncated series,
    sum_m M0^{-T} (-A M1^T M0^{-T})^m v, with the same (Euler) weighting."""
    A = coupling_A(tau, g)
    terms = [np.array(v, dtype=np.complex128, copy=True)]
    for _ in range(order):
        terms.append(-A * apply_M1dag(apply_M0inv_dag(terms[-1], tau), sigma, tau))
    partial = []
    acc = np.zeros_like(terms[0])
    for tm in terms:
        acc = acc + tm
        partial.append(apply_M0inv_dag(acc, tau))
    if euler:
        return euler_estimate(partial, p)
    return partial[-1]


def euler_weights(order, p=0.5):
    """Closed-form weights w_m with S_{d,0} = sum_m w_m u_m (derived from the
    recursion: S_{d,0} = sum_k C(d,k) p^{d-k} (1-p)^k S_{0,k})."""
    return np.array([sum(comb(order, k) * p ** (order - k) * (1 - p) ** k
                         for k in range(m, order + 1)) for m in range(order + 1)])
