"""The domain-growth study on a small deep quench (256^2 D2Q9 E8 FP32 at the
critical density, T_hat = 0.7): the recorded L(t) grows, and the phases reach
the coexisting densities of the Maxwell construction."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
from paper_2212_07848_amd import coarsening as CO  # noqa: E402
from paper_2212_07848_amd.scaling import binodal_densities  # noqa: E402


def test_small_quench_coarsens_towards_the_binodal():
    res = CO.run(n=256, steps=6000, every=500)
    assert res["bad"] == 0
    t, L = np.array(res["step"]), np.array(res["L"])
    assert list(t) == list(range(500, 6001, 500))
    # domains grow after the linear stage
    assert L[-1] > 1.5 * L[1] and np.all(np.diff(L[2:]) > -0.02 * L[2:-1])
    ng, nl, _ = binodal_densities(0.7)
    # the extremes of the phase-separated field sit near the coexisting densities
    assert abs(res["rho_min"] - ng) < 0.15 * ng and abs(res["rho_max"] - nl) < 0.15 * nl
    print(res["L"], res["rho_min"], res["rho_max"], CO.growth_exponent(t, L, 2000))
