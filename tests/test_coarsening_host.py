"""Host-side pieces of the domain-growth study (no GPU)."""
import numpy as np

from paper_2212_07848_amd.coarsening import growth_exponent


def test_growth_exponent_of_a_power_law():
    t = np.arange(500, 50001, 500)
    L = 3.0 * t ** 0.4
    assert abs(growth_exponent(t, L, 10000) - 0.4) < 1e-12
    # only the window counts: an early transient does not enter the fit
    L2 = np.where(t < 10000, 50.0, L)
    assert abs(growth_exponent(t, L2, 10000) - 0.4) < 1e-12
    assert growth_exponent(t, L, 60000) is None
