"""Reduced lifetime study on the GPU: an unstable state separates after a
time logarithmic in 1/k_B theta with the slope of the exact linear growth
rate; a metastable state's lifetime grows steeply as the noise falls and it
does not separate at k_B theta = 1e-13."""
import math

import numpy as np
import pytest

from oracle import theory as T

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
from paper_2212_07848_amd import metastable as M  # noqa: E402


def test_unstable_onset_is_logarithmic_in_the_noise():
    n0 = M.state_points()["unstable"]
    res = M.run(n0, [1e-5, 1e-9, 1e-13], seeds=4, n=64, max_steps=2000, check_every=5)
    for r in res["rows"]:
        print(r["kBT"], r["times"])
        assert r["separated"] == 4
    G = T.coupling(0.8)
    # fastest exact growth over the wave vectors of a 64^2 box near |k| = 0.5
    g = 0.0
    for m1 in range(0, 9):
        for m2 in range(0, 9):
            kv = 2 * math.pi * np.array([m1, m2]) / 64
            if 0.3 < np.linalg.norm(kv) < 0.7:
                A = T.linear_operator(kv, D=2, kind=4, n0=n0, G=G, kBT=0.0)[0]
                g = max(g, float(np.max(np.abs(np.linalg.eigvals(A)))))
    slope = M.onset_slope(res["rows"])
    print("slope", slope, "linear", 1 / (2 * math.log(g)))
    assert slope == pytest.approx(1.0 / (2.0 * math.log(g)), rel=0.12)


def test_metastable_lifetime_grows_as_the_noise_falls():
    res = M.run(0.62, [6e-4, 3e-4, 1e-13], seeds=8, n=128, max_steps=40000, check_every=100)
    fast, slow, zero = res["rows"]
    for r in res["rows"]:
        print(r["kBT"], r["times"])
        assert r["diverged"] == 0
    assert fast["separated"] == 8
    assert slow["median"] is not None and slow["median"] > 3.0 * fast["median"]
    assert zero["separated"] == 0
