"""The JSON-lines run log on a real lattice and ensemble (through the C ABI)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
from paper_2212_07848_amd import runlog as RL  # noqa: E402


def test_run_log_of_a_lattice_and_an_ensemble(tmp_path):
    p = fsc.make_params(D=2, nx=64, ny=64, stencil=fsc.FSC_E4, precision="fp32", T_hat=0.9,
                        rho0=0.5, kBT=1e-4, seed=5)
    path = tmp_path / "lat.jsonl"
    with fsc.Lattice(p) as lat, RL.RunLog(str(path), lat, sk_kind=fsc.FSC_SK_AXIS) as log:
        lat.init_uniform()
        log.record()
        for _ in range(3):
            lat.run(200, sk_every=20)
            log.record(phase="run")
    recs = RL.read(str(path))
    assert [r["step"] for r in recs] == [0, 200, 400, 600]
    mass0 = 0.5 * 64 * 64
    for r in recs:
        rep = r["replicas"][0]
        assert abs(rep["mass"] - mass0) < 1e-6 * mass0  # FP32 storage, FP64 sums
        assert rep["bad"] == 0 and rep["rho_min"] <= 0.5 <= rep["rho_max"]
    assert all(r["mlups"] > 0 for r in recs[1:])
    # ten samples per 200 steps, two axes, modes +-m
    counts = [np.array(r["replicas"][0]["sk_count"])[:, 1].sum() for r in recs]
    assert counts == [0, 40, 80, 120]

    plist = [fsc.make_params(D=2, nx=n, ny=n, stencil=fsc.FSC_E4, precision="fp32", T_hat=0.9,
                             rho0=0.5, kBT=1e-4, seed=5, replica=r)
             for r, n in enumerate((32, 64))]
    ens = fsc.Ensemble(plist)
    try:
        with RL.RunLog(str(tmp_path / "ens.jsonl"), ens) as log:
            ens.init_uniform()
            ens.run(100)
            rec = log.record()
    finally:
        ens.close()
    assert [r["replica"] for r in rec["replicas"]] == [0, 1]
    assert rec["step"] == 100 and rec["mlups"] > 0
    assert [round(r["mass"]) for r in rec["replicas"]] == [512, 2048]
