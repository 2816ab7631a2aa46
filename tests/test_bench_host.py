"""Host-side plumbing of bench.py (no GPU): the kernel names and launch sizes
it looks up in the committed counter summary, and the calibration that turns
rocprofv3's FETCH_SIZE / WRITE_SIZE readings into HBM bytes."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _profile():
    with open(os.path.join(ROOT, "profiles", "step_traffic.json")) as fh:
        return json.load(fh)


def test_kernel_names_match_the_profiler_names():
    names = {e["kernel"] for e in _profile()["entries"]}
    # the ensemble's two-step launch, and single-step kernels of both lattices
    two = dict(tx=256, ty=1, pf=1, blocks=741, steps=2)
    assert bench.kernel_name("StencilE4_2D", True, two) == "k_step2<StencilE4_2D, float, true, 256, 2, false>"
    assert bench.kernel_name("StencilE4_2D", True, two) in names
    one3 = dict(tx=64, ty=4, pf=0, blocks=512, steps=1)
    assert bench.kernel_name("StencilE4_3D", True, one3, "D3Q19") in names
    one2 = dict(tx=128, ty=1, pf=2, blocks=512, steps=1)
    assert bench.kernel_name("StencilE4_2D", True, one2) in names


def test_grid_threads_counts_the_edge_wave_of_the_two_step_kernel():
    assert bench.grid_threads(dict(tx=256, ty=1, pf=1, blocks=741, steps=2)) == 741 * 320
    assert bench.grid_threads(dict(tx=64, ty=4, pf=0, blocks=512, steps=1)) == 512 * 256
    # the tilings whose lanes hold the halo columns: 246 + 10 (E8), 250 + 6 (E4)
    hin = dict(tx=246, ty=1, pf=0, blocks=765, steps=2)
    assert bench.grid_threads(hin) == 765 * 256
    assert bench.kernel_name("StencilE8_2D", True, hin) == "k_step2<StencilE8_2D, float, true, 246, 1, true>"
    assert bench.grid_threads(dict(tx=250, ty=1, pf=1, blocks=10, steps=2)) == 10 * 256
    # the single-step partner of a 246-wide tiling has no edge wave
    assert bench.grid_threads(dict(tx=246, ty=1, pf=1, blocks=10, steps=1)) == 10 * 246
    # and the profile holds that kernel's launches under sizes of that form
    # (the march length, hence the block count, is the autotuner's choice)
    sizes = {e["grid_threads"] for e in _profile()["entries"]
             if e["kernel"] == "k_step2<StencilE4_2D, float, true, 256, 2, false>"}
    assert sizes and all(n % 320 == 0 for n in sizes)
    sizes = {e["grid_threads"] for e in _profile()["entries"]
             if e["kernel"] == "k_step2<StencilE8_2D, float, true, 246, 1, true>"}
    assert sizes and all(n % 256 == 0 for n in sizes)


def _write_csv(path, counter, rows):
    cols = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for name, grid, v in rows:
            w.writerow(dict(Kernel_Name=name, Grid_Size=grid, Counter_Name=counter, Counter_Value=v))


def test_ingest_scales_the_counters_by_the_copy_calibration(tmp_path):
    # FETCH_SIZE reads half the true bytes of a 1 GiB copy (as on this part),
    # WRITE_SIZE reads them exactly; a step kernel's readings scale alike
    copy = "void fsc::k_copy(uint4 const*, uint4*, long)"
    step = "void fsc::k_step2<fsc::StencilE4_2D, float, true, 256, 2, false>(fsc::RepDesc const*, int const*, int, int, unsigned long const*, unsigned int)"
    kib = float(1 << 20)  # 1 GiB in KiB
    f, w, v = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "v.csv"
    _write_csv(f, "FETCH_SIZE", [(copy, 1 << 26, kib / 2)] * 3 + [(step, 237120, 1000.0), (step, 237120, 1002.0)])
    _write_csv(w, "WRITE_SIZE", [(copy, 1 << 26, kib)] * 3 + [(step, 237120, 500.0)] * 2)
    _write_csv(v, "SQ_INSTS_VALU", [(step, 237120, 7.0e7)] * 2)
    out = tmp_path / "traffic.json"
    doc = bench.ingest_pmc(str(f), str(w), str(v), str(out))
    assert doc["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert doc["calibration"]["write_scale"] == pytest.approx(1.0)
    (e,) = doc["entries"]
    assert e["kernel"] == "k_step2<StencilE4_2D, float, true, 256, 2, false>" and e["grid_threads"] == 237120
    assert e["fetch_bytes"] == int(1001.0 * 1024 * 2.0)
    assert e["write_bytes"] == int(500.0 * 1024)
    assert e["bytes_per_launch"] == int(1001.0 * 1024 * 2.0 + 500.0 * 1024)
    assert e["valu_insts_per_launch"] == int(7.0e7)
    assert json.load(open(out))["entries"][0] == e


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stdout


def test_kernel_view_prices_a_launch_by_its_nodes():
    # one launch reads and writes every population of every node once, also
    # when it advances two steps: 72 B per node for D2Q9, 152 B for D3Q19
    q = dict(D=2, nx=4096, ny=4096, nz=1, stencil=8, precision="fp32")
    two = dict(tx=192, ty=1, pf=0, blocks=1012, steps=2)
    kv = bench.kernel_view(q, two, t_step=200e-6)
    assert kv["kernel"] == "k_step2<StencilE8_2D, float, true, 192, 1, false>"
    assert kv["nodes_per_launch"] == 4096 * 4096 and kv["lups_per_launch"] == 2 * 4096 * 4096
    assert kv["algorithmic_bytes_per_launch"] == 72 * 4096 * 4096
    assert kv["avg_launch_us"] == pytest.approx(400.0)
    assert kv["hbm_gbs"] == pytest.approx(72 * 4096 * 4096 / 400e-6 / 1e9)
    c4 = dict(D=3, nx=256, ny=256, nz=256, stencil=4, precision="fp32")
    one = dict(tx=64, ty=4, pf=0, blocks=512, steps=1)
    kv3 = bench.kernel_view(c4, one, t_step=565e-6)
    assert kv3["kernel"] == "k_step<D3Q19, StencilE4_3D, float, true, 64, 4, 0, false>"
    assert kv3["algorithmic_bytes_per_launch"] == 152 * 256 ** 3


def test_bench_defaults_time_the_whole_workload():
    # the default run is the deep quench's 50 000 steps in periods of 500
    # lattice steps, each ending in its S(k,t)/L(t) sample
    import fsc_inputs as I
    assert I.DEEP_QUENCH["sk_every"] == 500 and I.DEEP_QUENCH["steps"] == 50000
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'ap.add_argument("--steps", type=int, default=100)' in src
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--kernel-steps", "3"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "kernel-steps" in r.stdout
