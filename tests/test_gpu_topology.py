"""3D spinodal decomposition on the unstable branch of the T_hat = 0.8
isotherm (the paper's Fig. 1): the final interface topology runs from
droplets at low density through tubes and flat slabs to gas tubes and
bubbles near the liquid spinodal.  48^3 D3Q19, k_B theta = 1e-10, four noise
seeds per density, classified by the periodic wrapping of each phase."""
import pytest

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
from paper_2212_07848_amd import topology as TP  # noqa: E402


def _majority(counts):
    return max(counts, key=counts.get)


def test_topology_sequence_across_the_unstable_branch():
    dens = TP.default_densities(0.8, fractions=(0.03, 0.25, 0.5, 0.97))
    res = TP.run(dens, n=48, seeds=4, max_steps=40000, check_every=4000)
    c = [x["shapes"] for x in res["counts"]]
    print(c, res["lattice_seconds"])
    assert c[0] == {"droplet": 4}
    assert c[1].get("droplet-cylinder", 0) >= 1
    assert set(c[1]) <= {"droplet", "droplet-cylinder", "mixed"}
    assert _majority(c[2]) == "flat"
    assert sum(c[3].get(s, 0) for s in ("bubble", "bubble-cylinder")) == 4
    # the classified shapes never go backwards in the sequence as n0 rises
    idx = [[TP.ORDER.index(s) for s, k in cc.items() if s in TP.ORDER for _ in range(k)]
           for cc in c]
    means = [sum(v) / len(v) for v in idx]
    assert all(a <= b for a, b in zip(means, means[1:]))
