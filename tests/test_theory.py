"""Pins of the closed forms in tests/theory.py against what the paper fixes."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import theory as T


def test_critical_point_is_1_1_1():
    # Reduced EoS, Eq. (7): critical point at n = p = T = 1, where the first
    # two density derivatives vanish.
    assert T.p_hat(1.0, 1.0) == pytest.approx(1.0, abs=1e-15)
    assert T.dp_hat_dn(1.0, 1.0) == pytest.approx(0.0, abs=1e-15)
    assert T.d2p_hat_dn2(1.0, 1.0) == pytest.approx(0.0, abs=1e-15)


def test_critical_constants_from_psi_scaling():
    # Eq. (4): psi = a exp(-b/n) with a = e sqrt(Tc nc), b = nc; with psi = exp(-1/n)
    # (b = 1 -> nc = 1) and G a^2 = G we have Tc = G/e^2; T = 1/3 gives the
    # coupling G = e^2/(3 T_hat), and p_c = nc Tc / 2 (Eq. 6 at the critical point).
    for T_hat in (0.6, 0.7, 0.8, 0.9, 0.99):
        G = T.coupling(T_hat)
        Tc = G / math.e ** 2
        assert (1.0 / 3.0) / Tc == pytest.approx(T_hat, rel=1e-14)
        # lattice EoS p = nT - (G/2) exp(-2/n) equals p_c * p_hat(n, T_hat)
        for n in (0.3, 1.0, 2.5):
            p = n / 3.0 - 0.5 * G * math.exp(-2.0 / n)
            assert p == pytest.approx(0.5 * Tc * T.p_hat(n, T_hat), rel=1e-13)


def test_spinodal_and_binodal_are_consistent():
    for T_hat in (0.6, 0.7, 0.8, 0.9, 0.95, 0.99):
        ns_g, ns_l = T.spinodal(T_hat)
        assert T.dp_hat_dn(ns_g, T_hat) == pytest.approx(0.0, abs=1e-11)
        assert T.dp_hat_dn(ns_l, T_hat) == pytest.approx(0.0, abs=1e-11)
        ng, nl, p0 = T.binodal(T_hat)
        assert ng < ns_g < 1.0 < ns_l < nl
        assert T.p_hat(ng, T_hat) == pytest.approx(p0, abs=1e-11)
        assert T.p_hat(nl, T_hat) == pytest.approx(p0, abs=1e-11)
        # equal areas in the specific volume
        area, _ = integrate.quad(lambda v: T.p_hat(1.0 / v, T_hat) - p0, 1.0 / nl, 1.0 / ng,
                                 epsabs=1e-13, limit=200)
        assert abs(area) < 1e-10
    # the binodal closes at the critical point
    ng, nl, _ = T.binodal(0.999)
    assert abs(ng - 1.0) < 0.1 and abs(nl - 1.0) < 0.1


def test_compressibility_closed_form():
    # Eq. (8) is 1/(n dp/dn) of Eq. (7).
    for T_hat, n in ((1.2, 1.0), (0.9, 0.5), (0.8, 2.5)):
        h = 1e-6
        dp = (T.p_hat(n + h, T_hat) - T.p_hat(n - h, T_hat)) / (2 * h)
        assert T.kappa_T(n, T_hat) == pytest.approx(1.0 / (n * dp), rel=1e-7)


def test_compressibility_exponents():
    # kappa_T ~ (T-1)^-1 at n = 1 (critical), and ~ (p - p_s)^-1/2 near the
    # spinodal along an isotherm, Eqs. (8)-(10).
    eps = np.array([1e-3, 1e-4])
    k = T.kappa_T(1.0, 1.0 + eps)
    slope = np.log(k[1] / k[0]) / np.log(eps[1] / eps[0])
    assert slope == pytest.approx(-1.0, abs=1e-3)
    T_hat = 0.8
    ns, _ = T.spinodal(T_hat)
    ps = T.p_hat(ns, T_hat)
    dn = np.array([1e-4, 1e-5])
    n = ns - dn  # stable gas side
    k = T.kappa_T(n, T_hat)
    dp = np.abs(T.p_hat(n, T_hat) - ps)
    slope = np.log(k[1] / k[0]) / np.log(dp[1] / dp[0])
    assert slope == pytest.approx(-0.5, abs=1e-3)
    # amplitudes of Eq. (10); on the gas branch p has a maximum at the
    # spinodal, so A < 0 and n - n_s < 0, and the magnitudes enter
    A = T.d2p_hat_dn2(ns, T_hat)
    assert A < 0
    assert k[1] == pytest.approx(1.0 / (A * ns) / (n[1] - ns), rel=1e-3)
    pred = 1.0 / (math.sqrt(2 * abs(A)) * ns) * dp[1] ** -0.5
    assert k[1] == pytest.approx(pred, rel=1e-3)


@pytest.mark.parametrize("D,kind", [(2, 4), (2, 8), (3, 4)])
def test_stencil_weights_isotropy(D, kind):
    # Eq. (1)'s weights: sum w e_x^2 = 1 (gives p = nT - G psi^2/2, Eq. 2) and
    # isotropic 4th (and for E8 6th) order moments.
    E, W = T.stencil_set(D, kind)
    ex, ey = E[:, 0].astype(float), E[:, 1].astype(float)
    assert (W * ex ** 2).sum() == pytest.approx(1.0, abs=1e-15)
    assert (W * ex ** 4).sum() == pytest.approx(3 * (W * ex ** 2 * ey ** 2).sum(), abs=1e-15)
    if kind == 8:
        assert (W * ex ** 6).sum() == pytest.approx(5 * (W * ex ** 4 * ey ** 2).sum(), abs=1e-15)
    assert len(W) == {(2, 4): 8, (2, 8): 24, (3, 4): 18}[(D, kind)]


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("T_hat,n0", [(0.9, 0.5), (0.8, 0.62), (0.9, 2.0), (0.6, 0.3)])
@pytest.mark.parametrize("lam", [(1.0, 1.0, 1.0), (0.7, 1.3, 1.8)])
def test_linear_theory_reproduces_exact_sk_on_axis(D, T_hat, n0, lam):
    # The linearised lattice update's stationary covariance equals the paper's
    # exact S(k), Eq. (16), along a lattice axis, for any collision rates.
    G = T.coupling(T_hat)
    for m in (1, 3, 8, 15, 16):
        k = 2 * math.pi * m / 32
        kv = np.zeros(D)
        kv[0] = k
        s = T.sk_linear_stationary(kv, D=D, kind=4, n0=n0, G=G, kBT=1.0, lam=lam)
        assert s == pytest.approx(T.sk_exact(k, n0, G, 1.0), rel=1e-10)


def test_linear_theory_e8_axis_form():
    G = T.coupling(0.7)
    for m in (1, 5, 16):
        k = 2 * math.pi * m / 32
        s = T.sk_linear_stationary([k, 0.0], D=2, kind=8, n0=0.4, G=G, kBT=1.0)
        assert s == pytest.approx(T.sk_exact_axis(k, 0.4, G, 1.0, kind=8)[0], rel=1e-10)
    # and the general form reduces to Eq. (16) for E4
    k = np.linspace(0.1, math.pi, 7)
    assert np.allclose(T.sk_exact_axis(k, 0.5, 2.5, 1.0, kind=4), T.sk_exact(k, 0.5, 2.5, 1.0),
                       rtol=1e-13)


def test_ideal_gas_limit_is_flat():
    # G = 0: S(k) = n0 kBT / T for every k (the fluctuating ideal gas).
    for kv in ([0.3, 0.0], [1.0, 2.0], [math.pi, math.pi]):
        s = T.sk_linear_stationary(kv, D=2, kind=4, n0=0.7, G=0.0, kBT=2.0)
        assert s == pytest.approx(0.7 * 2.0 * 3.0, rel=1e-10)


def test_k_to_zero_limit_is_compressibility():
    # S(0) c^2_{s,0} / (n0 kBT) = 1, i.e. S(0) ~ kappa_T.
    G = T.coupling(0.8)
    n0 = 0.6
    psi0 = math.exp(-1 / n0)
    cs0 = 1 / 3 - G * psi0 * psi0 / n0 ** 2
    assert T.sk_exact(1e-8, n0, G, 1.0) * cs0 / n0 == pytest.approx(1.0, rel=1e-12)


def test_order_k2_truncation_fails_beyond_half_pi():
    # Negative control: the O(k^2) truncation departs from Eq. (16) for k > pi/2.
    G = T.coupling(0.8)
    n0 = 0.62
    k = np.array([0.05, math.pi / 2, 3.0])
    ex = T.sk_exact(k, n0, G, 1.0)
    tr = T.sk_exact_order_k2(k, n0, G, 1.0)
    rel = np.abs(tr / ex - 1)
    assert rel[0] < 1e-3
    assert rel[1] > 0.02 and rel[2] > 0.1
