"""Thermodynamics and exact linear theory of the method (part of the CPU oracle).

Everything here is written from the paper's equations (Lulli et al.,
arXiv:2212.07848) or from linear algebra on the linearised lattice update; none
of it calls the oracle's arithmetic.  Lattice units: n_c = 1, T = c_s^2 = 1/3,
psi = exp(-1/n), G = e^2/(3 T_hat).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import optimize, integrate

CS2 = 1.0 / 3.0


# ---------------------------------------------------------------------------
# Thermodynamics: reduced EoS, Eq. (7); compressibility, Eq. (8); spinodal and
# Maxwell coexistence.
# ---------------------------------------------------------------------------
def p_hat(n, T):
    """Reduced ("general") EoS, Eq. (7): p = 2 n T - exp(2 - 2/n)."""
    return 2.0 * n * T - np.exp(2.0 - 2.0 / n)


def dp_hat_dn(n, T):
    return 2.0 * T - 2.0 / n ** 2 * np.exp(2.0 - 2.0 / n)


def d2p_hat_dn2(n, T):
    e = np.exp(2.0 - 2.0 / n)
    return (4.0 / n ** 3 - 4.0 / n ** 4) * e


def kappa_T(n, T):
    """Eq. (8): kappa_T = (n/2) [n^2 T - exp(2 - 2/n)]^{-1}."""
    return 0.5 * n / (n ** 2 * T - np.exp(2.0 - 2.0 / n))


def spinodal(T):
    """(n_gas, n_liquid) where dp/dn = 0 on the isotherm T < 1."""
    g = lambda n: n ** 2 * T - math.exp(2.0 - 2.0 / n)
    return optimize.brentq(g, 0.05, 1.0), optimize.brentq(g, 1.0, 50.0)


def binodal(T):
    """Maxwell equal-area coexistence (n_gas, n_liquid, p_hat) on the isotherm T < 1.

    Equal areas are taken in the specific volume v = 1/n.
    """
    ns_g, ns_l = spinodal(T)
    p_lo = max(p_hat(ns_l, T), 1e-8)
    p_hi = p_hat(ns_g, T)

    def roots(p):
        ng = optimize.brentq(lambda n: p_hat(n, T) - p, 1e-9, ns_g)
        nl = optimize.brentq(lambda n: p_hat(n, T) - p, ns_l, 100.0)
        return ng, nl

    def area(p):
        ng, nl = roots(p)
        val, _ = integrate.quad(lambda v: p_hat(1.0 / v, T) - p, 1.0 / nl, 1.0 / ng,
                                epsabs=1e-14, epsrel=1e-13, limit=200)
        return val

    p0 = optimize.brentq(area, p_lo, p_hi - 1e-12, xtol=1e-15)
    ng, nl = roots(p0)
    return ng, nl, p0


def coupling(T_hat):
    return math.e ** 2 * CS2 / T_hat


# ---------------------------------------------------------------------------
# Exact static structure factor, Eqs. (15)-(16), in lattice units.
# ---------------------------------------------------------------------------
def sound_speed_sq(k, n0, G):
    """Eq. (15): c^2(k) = c^2_{s,0} - (1/2) G psi0 psi0' [cos k - 1]."""
    psi0 = math.exp(-1.0 / n0)
    dpsi0 = psi0 / n0 ** 2
    cs0 = CS2 - G * psi0 * dpsi0  # dp/dn of p = nT - (G/2) psi^2
    return cs0 - 0.5 * G * psi0 * dpsi0 * (np.cos(k) - 1.0)


def sk_exact(k, n0, G, kBT):
    """Eq. (16): S(k) = n0 kBT / c^2(k), along a lattice axis (E4 stencil)."""
    return n0 * kBT / sound_speed_sq(k, n0, G)


def sk_exact_order_k2(k, n0, G, kBT):
    """Eq. (16) with c^2(k) truncated at O(k^2) (the paper's dashed lines)."""
    psi0 = math.exp(-1.0 / n0)
    dpsi0 = psi0 / n0 ** 2
    cs0 = CS2 - G * psi0 * dpsi0
    return n0 * kBT / (cs0 + 0.25 * G * psi0 * dpsi0 * np.asarray(k) ** 2)


# ---------------------------------------------------------------------------
# Linearised lattice update around the homogeneous state and its per-k
# covariance recursion Sigma_{t+1} = A Sigma_t A^H + Qn, Sigma_0 = 0 (the
# homogeneous start).  S(k, t) = 1^T Sigma_t 1.
# ---------------------------------------------------------------------------
def d2q9():
    c = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    return c, w


def d3q19():
    c = [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
         [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
         [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]]
    c = np.array(c)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    return c, w


def stencil_set(D, kind):
    """Offsets and the weights of Eq. (1) normalised to sum_a w e_x^2 = 1."""
    if D == 2 and kind == 4:
        W = {1: 1 / 3, 2: 1 / 12}
        r = 1
    elif D == 2 and kind == 8:
        W = {1: 4 / 21, 2: 4 / 45, 4: 1 / 60, 5: 2 / 315, 8: 1 / 5040}
        r = 2
    elif D == 3 and kind == 4:
        W = {1: 1 / 6, 2: 1 / 12}
        r = 1
    else:
        raise ValueError
    E, Wt = [], []
    rng = range(-r, r + 1)
    for e in np.array(np.meshgrid(*([list(rng)] * D), indexing="ij")).reshape(D, -1).T:
        e2 = int((e ** 2).sum())
        if e2 in W:
            E.append(e)
            Wt.append(W[e2])
    return np.array(E), np.array(Wt)


def _basis_rows(D, c):
    """A moment basis orthogonal under the lattice weights (its span and class
    split are all the linear theory needs)."""
    x = c[:, 0].astype(float)
    y = c[:, 1].astype(float)
    if D == 2:
        c2 = x * x + y * y
        R = [np.ones_like(x), x, y, 3 * c2 - 2, x * x - y * y, x * y, (3 * c2 - 4) * x,
             (3 * c2 - 4) * y, 9 * c2 * c2 - 15 * c2 + 2]
        cls = [0, 0, 0, 1, 2, 2, 3, 3, 3]
    else:
        z = c[:, 2].astype(float)
        c2 = x * x + y * y + z * z
        R = [np.ones_like(x), x, y, z, c2 - 1, 3 * x * x - c2, y * y - z * z, x * y, y * z,
             z * x, (3 * c2 - 5) * x, (3 * c2 - 5) * y, (3 * c2 - 5) * z, x * (y * y - z * z),
             y * (z * z - x * x), z * (x * x - y * y), 3 * c2 * c2 - 6 * c2 + 1,
             (2 * c2 - 3) * (3 * x * x - c2), (2 * c2 - 3) * (y * y - z * z)]
        cls = [0, 0, 0, 0, 1, 2, 2, 2, 2, 2] + [3] * 9
    return np.array(R), np.array(cls)


def linear_operator(kvec, *, D=2, kind=4, n0, G, kBT, lam=(1.0, 1.0, 1.0)):
    """(A, Qn) of the linearised step at wave vector kvec (lattice units)."""
    c, w = d2q9() if D == 2 else d3q19()
    Q = len(w)
    E, We = stencil_set(D, kind)
    kvec = np.asarray(kvec, dtype=float)
    M, cls = _basis_rows(D, c)
    b = (M ** 2 * w).sum(axis=1)
    lam_a = np.array([1.0 if k == 0 else lam[k - 1] for k in cls])
    Minv = np.linalg.inv(M)
    psi0 = math.exp(-1.0 / n0)
    dpsi0 = psi0 / n0 ** 2
    g = (We[:, None] * E * np.exp(1j * (E @ kvec))[:, None]).sum(axis=0)  # sum_a w_a e_a e^{ik.e_a}
    ones = np.ones(Q)
    # delta n = 1^T f ; delta j = c^T f ; delta F = G psi0 psi0' g delta n
    Fop = G * psi0 * dpsi0 * np.outer(g, ones)           # D x Q
    uop = (c.T.astype(complex) + 0.5 * Fop) / n0         # D x Q
    feq = w[:, None] * (np.outer(ones, ones) + n0 * (c @ uop) / CS2)
    S = w[:, None] * (c @ Fop) / CS2
    L = np.diag(lam_a)
    I = np.eye(Q)
    Cop = I - Minv @ L @ M @ (I - feq) + Minv @ (I - 0.5 * L) @ M @ S
    P = np.diag(np.exp(-1j * (c @ kvec)))
    A = P @ Cop
    mu = kBT / CS2
    amp = np.sqrt(mu * n0 * b * (1.0 - (1.0 - lam_a) ** 2))
    amp[: D + 1] = 0.0
    B = Minv @ np.diag(amp)
    Qn = P @ (B @ B.T) @ P.conj().T
    return A, Qn


def sk_linear_stationary(kvec, doublings=48, **kw):
    """Stationary S(k) = 1^T X 1 with X = sum_j A^j Qn (A^j)^H, by repeated
    doubling (it stays well posed where A has an unexcited unit-modulus
    eigenvalue, e.g. k = pi on an axis at tau = 1)."""
    A, Qn = linear_operator(kvec, **kw)
    X = Qn.copy()
    Ak = A.copy()
    for _ in range(doublings):
        X = X + Ak @ X @ Ak.conj().T
        Ak = Ak @ Ak
    ones = np.ones(A.shape[0])
    return float(np.real(ones @ X @ ones))


def sk_linear_times(kvec, times, **kw):
    """Exact linear expectation S(k, t) at the given (sorted) times from Sigma_0 = 0."""
    A, Qn = linear_operator(kvec, **kw)
    ones = np.ones(A.shape[0])
    X = np.zeros_like(A)
    out = []
    t = 0
    for ts in times:
        while t < ts:
            X = A @ X @ A.conj().T + Qn
            t += 1
        out.append(float(np.real(ones @ X @ ones)))
    return np.array(out)


def sk_exact_axis(k, n0, G, kBT, *, D=2, kind=4):
    """On-axis exact S(k) for any stencil of Eq. (1).

    Summing the linearised force over the stencil gives
    c^2(k) = c^2_{s,0} + G psi0 psi0' [1 - h(k)] with
    h(k) = sum_a w_a e_ax sin(k e_ax) / (2 tan(k/2)); for E4, h = (1 + cos k)/2
    and this is Eq. (15)-(16) unchanged.
    """
    E, W = stencil_set(D, kind)
    k = np.atleast_1d(np.asarray(k, dtype=float))
    g = (W[None, :] * E[None, :, 0] * np.sin(k[:, None] * E[None, :, 0])).sum(axis=1)
    h = g / (2.0 * np.tan(k / 2.0))
    psi0 = math.exp(-1.0 / n0)
    dpsi0 = psi0 / n0 ** 2
    c2 = CS2 - G * psi0 * dpsi0 * h
    return n0 * kBT / c2
