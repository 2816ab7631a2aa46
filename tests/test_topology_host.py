"""The periodic topology classifier of paper_2212_07848_amd/topology.py on
synthetic fields whose answer is known: balls, tubes, slabs and their
complements, placed across the periodic faces, and a bicontinuous network."""
import numpy as np
import pytest

from paper_2212_07848_amd import topology as TP

N = 24


def _grid():
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    return z, y, x


def _pdist(a, c):
    d = np.abs(a - c)
    return np.minimum(d, N - d)


def _field(mask):
    return np.where(mask, 2.0, 0.4)


@pytest.mark.parametrize("centre", [(12, 12, 12), (0, 0, 0), (23, 1, 12)])
def test_ball_and_bubble(centre):
    z, y, x = _grid()
    r2 = _pdist(z, centre[0]) ** 2 + _pdist(y, centre[1]) ** 2 + _pdist(x, centre[2]) ** 2
    ball = r2 < 6 ** 2
    assert TP.classify(_field(ball), 1.2)["shape"] == "droplet"
    assert TP.classify(_field(~ball), 1.2)["shape"] == "bubble"


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_tubes(axis):
    z, y, x = _grid()
    a, b = [v for i, v in enumerate((z, y, x)) if i != axis]
    tube = _pdist(a, 0) ** 2 + _pdist(b, 5) ** 2 < 5 ** 2  # centred on a face
    c = TP.classify(_field(tube), 1.2)
    assert c["shape"] == "droplet-cylinder" and c["liquid_wraps"] == 1
    assert TP.classify(_field(~tube), 1.2)["shape"] == "bubble-cylinder"


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_slab(axis):
    v = _grid()[axis]
    slab = _pdist(v, 1) < 6  # straddles the face
    c = TP.classify(_field(slab), 1.2)
    assert c["shape"] == "flat" and (c["liquid_wraps"], c["gas_wraps"]) == (2, 2)


def test_bicontinuous_network_is_mixed():
    z, y, x = _grid()
    k = 2 * np.pi / N
    g = np.sin(k * x) * np.cos(k * y) + np.sin(k * y) * np.cos(k * z) + np.sin(k * z) * np.cos(k * x)
    c = TP.classify(_field(g > 0), 1.2)
    assert c["shape"] == "mixed" and c["liquid_wraps"] == 3 and c["gas_wraps"] == 3


def test_two_droplets_report_the_largest():
    z, y, x = _grid()
    a = _pdist(z, 5) ** 2 + _pdist(y, 5) ** 2 + _pdist(x, 5) ** 2 < 4 ** 2
    b = _pdist(z, 17) ** 2 + _pdist(y, 17) ** 2 + _pdist(x, 17) ** 2 < 3 ** 2
    c = TP.classify(_field(a | b), 1.2)
    assert c["shape"] == "droplet"
    assert c["largest_liquid"] == pytest.approx(a.mean())


def test_winding_through_a_chain_of_labels():
    # a tube broken by the box face into pieces with different labels along x,
    # closing only through the periodic face: still one wrap
    z, y, x = _grid()
    tube = (_pdist(z, 12) ** 2 + _pdist(y, 12) ** 2 < 4 ** 2) & (x != 12)
    tube |= (_pdist(z, 12) ** 2 + _pdist(y, 12) ** 2 < 2 ** 2)  # thin bridge at x = 12
    assert TP.wrapping(tube)[1] == 1


def test_default_densities_span_the_unstable_interval():
    d = TP.default_densities(0.8)
    assert 0.6454 < min(d) and max(d) < 1.6698 and len(d) == len(TP.DEFAULT_FRACTIONS)
    assert all(a < b for a, b in zip(d, d[1:]))
