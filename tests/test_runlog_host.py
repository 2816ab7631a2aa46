"""The JSON-lines run log against a stand-in simulation object (host only)."""
import numpy as np

from paper_2212_07848_amd import runlog as RL


class _Lat:
    """Answers the calls the log makes of a Lattice."""

    def __init__(self):
        self.t = 0

    def stats(self, allow_diverged=False):
        assert allow_diverged
        return dict(mass=12.5, mom=np.array([1e-3, -2e-3]), rho_min=0.4, rho_max=0.6, bad=0,
                    nodes=64)

    def read_sk(self, kind):
        return np.ones((2, 3)), 2 * np.ones((2, 3)), np.full((2, 3), 4, dtype=np.int64)


class _Ens(_Lat):
    plist = [object(), object(), object()]
    n = 3

    def stats(self, r, allow_diverged=False):
        d = super().stats(allow_diverged)
        d["mass"] += r
        return d

    def read_sk(self, r, kind):
        return super().read_sk(kind)


def test_lattice_records_round_trip(tmp_path):
    sim = _Lat()
    path = tmp_path / "run.jsonl"
    with RL.RunLog(str(path), sim, sk_kind=0) as log:
        first = log.record(note="start")
        sim.t = 100
        log.record()
    recs = RL.read(str(path))
    assert [r["step"] for r in recs] == [0, 100]
    assert recs[0]["note"] == "start" and first["mlups"] is None
    assert recs[1]["mlups"] > 0  # 64 nodes x 100 steps over the elapsed time
    rep = recs[1]["replicas"][0]
    assert rep["replica"] is None and rep["mass"] == 12.5 and rep["mom"] == [1e-3, -2e-3]
    assert rep["sk_count"] == [[4, 4, 4], [4, 4, 4]]


def test_ensemble_records_every_replica_or_a_subset(tmp_path):
    sim = _Ens()
    with RL.RunLog(str(tmp_path / "a.jsonl"), sim) as log:
        rec = log.record()
    assert [r["replica"] for r in rec["replicas"]] == [0, 1, 2]
    assert [r["mass"] for r in rec["replicas"]] == [12.5, 13.5, 14.5]
    assert "sk_sum" not in rec["replicas"][0]
    with RL.RunLog(str(tmp_path / "b.jsonl"), sim, replicas=[2]) as log:
        rec = log.record()
    assert [r["replica"] for r in rec["replicas"]] == [2]
