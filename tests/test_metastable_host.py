"""Host-side pins of the lifetime study: the linear growth rate against the
exact linearised step of the oracle, linear stability of the metastable
states, and the summaries and fits on synthetic first-passage data."""
import math

import numpy as np
import pytest

from oracle import theory as T
from paper_2212_07848_amd import metastable as M


def _max_growth(n0, T_hat, directions, ks):
    G = T.coupling(T_hat)
    best = 0.0
    for d in directions:
        d = np.asarray(d, dtype=float) / np.linalg.norm(d)
        for k in ks:
            A = T.linear_operator(k * d, D=2, kind=4, n0=n0, G=G, kBT=0.0)[0]
            best = max(best, float(np.max(np.abs(np.linalg.eigvals(A)))))
    return best


def test_growth_rate_matches_the_exact_linear_step_on_axis():
    n0 = M.state_points()["unstable"]
    s, k = M.growth_rate(n0, 0.8)
    ks = np.linspace(0.3, 0.7, 161)
    exact = math.log(_max_growth(n0, 0.8, [(1, 0)], ks))
    assert s == pytest.approx(exact, rel=0.02)
    assert 0.3 < k < 0.7


@pytest.mark.parametrize("n0", [0.62, 0.55, 1.8, 2.0])
def test_metastable_states_are_linearly_stable(n0):
    # between the binodal and the spinodal on the T_hat = 0.8 isotherm no
    # wave vector grows under the exact linearised step
    ng_b, nl_b, _ = M.binodal_densities(0.8)
    ng_s, nl_s = M.spinodal_densities(0.8)
    assert ng_b < n0 < ng_s or nl_s < n0 < nl_b
    ks = np.linspace(0.02, math.pi, 60)
    g = _max_growth(n0, 0.8, [(1, 0), (1, 1), (2, 1)], ks)
    assert g <= 1.0 + 1e-12
    assert M.growth_rate(n0, 0.8)[0] == 0.0


@pytest.mark.parametrize("frac", [0.05, 0.5, 0.95])
def test_unstable_states_grow(frac):
    ng_s, nl_s = M.spinodal_densities(0.8)
    n0 = ng_s + frac * (nl_s - ng_s)
    ks = np.linspace(0.05, 1.5, 30)
    assert _max_growth(n0, 0.8, [(1, 0)], ks) > 1.0
    assert M.growth_rate(n0, 0.8)[0] > 0.0


def test_summary_median_counts_survivors_as_late():
    r = M.summarize(1e-4, [100, 300, None, 200, None])
    assert r["separated"] == 3 and r["median"] == 300.0 and r["mean"] is None
    r = M.summarize(1e-4, [100, None, None, 200])
    assert r["median"] is None
    r = M.summarize(1e-4, [100, -50, 300])
    assert r["diverged"] == 1 and r["median"] is None and r["times"] == [100, None, 300]
    r = M.summarize(1e-4, [10, 20, 30, 40])
    assert r["mean"] == 25.0 and r["median"] == 25.0


def test_fits_recover_synthetic_laws():
    dF, a = 0.002, 3.0
    rows = [dict(kBT=k, median=math.exp(a + dF / k), mean=None) for k in (6e-4, 4e-4, 3e-4, 2.5e-4)]
    b, a2, r2 = M.barrier_fit(rows)
    assert b == pytest.approx(dF, rel=1e-9) and a2 == pytest.approx(a, rel=1e-9) and r2 > 0.999999
    rows = [dict(kBT=k, mean=40.0 + 6.5 * math.log(1.0 / k), median=None)
            for k in (1e-3, 1e-5, 1e-9, 1e-13)]
    # rows above the linear regime are left out
    rows[0]["mean"] = 0.0
    assert M.onset_slope(rows) == pytest.approx(6.5, rel=1e-9)
