"""Host logic of the S(k -> 0) scaling study (paper_2212_07848_amd/scaling.py)
against the oracle's independent theory and against the exponents of
Eq. 8 and Eq. 10.  CPU only: the module's state-point algebra and fits are
plain numpy."""
import math

import numpy as np
import pytest

from oracle import theory as T
from paper_2212_07848_amd import scaling as SC


@pytest.mark.parametrize("Th", [0.6, 0.8, 0.9, 0.99])
def test_spinodal_and_binodal_agree_with_the_oracle(Th):
    assert np.allclose(SC.spinodal_densities(Th), T.spinodal(Th), rtol=1e-12)
    assert np.allclose(SC.binodal_densities(Th), T.binodal(Th), rtol=1e-9)


def test_binodal_matches_the_tabulated_coexistence_point():
    # T_hat = 0.8: gas 0.431328, liquid 2.378732, p_hat 0.618538
    ng, nl, p0 = SC.binodal_densities(0.8)
    assert ng == pytest.approx(0.431328, abs=2e-6)
    assert nl == pytest.approx(2.378732, abs=2e-6)
    assert p0 == pytest.approx(0.618538, abs=2e-6)


@pytest.mark.parametrize("side", ["gas", "liquid"])
def test_state_points_sit_at_the_requested_spinodal_distance(side):
    Th = 0.8
    ng_s, nl_s = T.spinodal(Th)
    ps = T.p_hat(ng_s if side == "gas" else nl_s, Th)
    ng_b, nl_b, _ = T.binodal(Th)
    for d in (0.1, 0.01, 0.001):
        n = SC.density_at_spinodal_distance(Th, d, side)
        assert abs(1.0 - T.p_hat(n, Th) / ps) == pytest.approx(d, rel=1e-9)
        lo, hi = (ng_b, ng_s) if side == "gas" else (nl_s, nl_b)
        assert lo < n < hi  # metastable branch


@pytest.mark.parametrize("stencil", [4, 8])
def test_axis_structure_factor_matches_the_oracle(stencil):
    k = 2 * np.pi * np.arange(1, 33) / 64
    for n0, Th in ((0.5, 0.9), (0.62, 0.8), (2.0, 0.9)):
        got = SC.sk_exact(k, n0, Th, 1e-13, stencil)
        ref = T.sk_exact_axis(k, n0, T.coupling(Th), 1e-13, D=2, kind=stencil)
        assert np.allclose(got, ref, rtol=1e-12)


def test_s0_is_n0_kbt_over_dp_dn():
    # S(0) = n0 kBT / (dp/dn), with dp/dn in lattice units = (T/(2 T_hat)) dp_hat/dn
    for n0, Th in ((0.5, 0.9), (0.62, 0.8), (1.8, 0.9)):
        dpdn = (1.0 / 3.0) / (2.0 * Th) * T.dp_hat_dn(n0, Th)
        assert SC.s0_exact(n0, Th, 1e-13) == pytest.approx(n0 * 1e-13 / dpdn, rel=1e-12)
        # the k -> 0 limit of Eq. 16
        assert SC.sk_exact(np.array([1e-6]), n0, Th, 1e-13)[0] == pytest.approx(
            SC.s0_exact(n0, Th, 1e-13), rel=1e-9)


def test_fit_recovers_s0_from_exact_low_k_modes():
    k = 2 * np.pi * np.arange(1, 7) / 64
    for n0, Th in ((0.5, 0.9), (0.64, 0.8), (2.0, 0.95)):
        S = SC.sk_exact(k, n0, Th, 1e-13)
        assert SC.fit_s0(k, S) == pytest.approx(SC.s0_exact(n0, Th, 1e-13), rel=1e-10)
    # near the spinodal the smallest mode is far below S(0): the extrapolation matters
    n0 = SC.density_at_spinodal_distance(0.8, 1e-3, "gas")
    S = SC.sk_exact(k, n0, 0.8, 1e-13)
    s0 = SC.s0_exact(n0, 0.8, 1e-13)
    assert SC.fit_s0(k, S) == pytest.approx(s0, rel=1e-9)
    assert S[0] < 0.96 * s0


def test_asymptotic_exponents_of_the_exact_s0():
    # Eq. 10: S(0) ~ (p - p_s)^(-1/2) on an isotherm; Eq. 8: ~ (1 - T)^(-1) on the binodal
    for side in ("gas", "liquid"):
        d = [1e-5, 3e-6, 1e-6]
        s0 = [SC.s0_exact(SC.density_at_spinodal_distance(0.8, x, side), 0.8, 1.0) for x in d]
        assert SC.fit_exponent(d, s0) == pytest.approx(-0.5, abs=5e-3)
        t = [1e-5, 4e-6, 1.6e-6]  # corrections to scaling are O(t^(1/2)) on the binodal
        s0 = [SC.s0_exact(SC.binodal_densities(1 - x)[0 if side == "gas" else 1], 1 - x, 1.0)
              for x in t]
        assert SC.fit_exponent(t, s0) == pytest.approx(-1.0, abs=1e-2)


def test_state_point_list():
    pts = SC.state_points()
    assert len(pts) == 2 * (len(SC.DEFAULT_SPINODAL_D) + len(SC.DEFAULT_BINODAL_T))
    for p in pts:
        assert p["rho0"] > 0 and 0 < p["T_hat"] < 1
