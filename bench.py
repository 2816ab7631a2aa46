"""Throughput of the fluctuating Shan-Chen hot path on one MI355X.

Workload (the headline): the deep quench -- one 4096^2 D2Q9 lattice, E8 force
stencil, FP32 shifted populations, n0 = 1 (the critical density) at
T_hat = 0.7, kBT = 1e-4, quenched from the homogeneous state, with the radially
binned S(k, t) and the domain length L(t) recorded (FP64 bins) every 500 lattice
steps inside the replayed hipGraph chunks.  A bench "step" is one pass of the
whole hot path: 500 fused lattice time steps plus one S(k, t)/L(t) sample, so
every timed step carries its measurement; --steps K times K such periods
(500 K lattice steps; the default K = 100 is the workload's full 50 000 steps).
value = lattice updates per second (MLUPS) over the timed region.

The JSON line also carries: the metric's "% HBM roofline" (72 B per lattice
update times the update rate, against 8 TB/s: the bandwidth a kernel reading
and writing every population once per update would need); the roofline of
the dominant kernel, the two-step fused step (temporal blocking: one launch
advances two time steps with one read and one write of every population, 72 B
per node per launch), from HIP events on the lattice's stream and the
committed rocprofv3 counter summary; the other workloads as extra lines (the
64-replica ensemble, the 256^3 D3Q19 metastable lattice, each with its own
S(k) samples inside its timed region, and the noise-free quench); the
surrogate; and the FP64 CPU oracle timed on bounded samples of the workloads.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline (FP32 D2Q9 fluct. SC); surrogate speedup at 5% S(k) err"
HBM_PEAK_GBS = 8000.0
# FP32 vector issue: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz = 78.6 T
# operations/s (the published 157.3 TFLOP/s counts an FMA as two).  Integer
# and transcendental instructions issue at about 1/2 and 1/3.5 of that rate.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
KERNEL_SOURCES = ["paper_2212_07848_amd/csrc/fsc_step_kernel.h",
                  "paper_2212_07848_amd/csrc/fsc_step2_kernel.h",
                  "paper_2212_07848_amd/csrc/fsc_device.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_lup(D: int, precision: str) -> int:
    Q = 9 if D == 2 else 19
    return 2 * Q * (4 if precision == "fp32" else 8)


def kernel_name(stencil: str, noise: bool, tiling: dict, lattice: str = "D2Q9") -> str:
    """Name of the step kernel a tiling launches (as rocprofv3 reports it)."""
    n = "true" if noise else "false"
    if tiling.get("steps", 1) == 2:  # prefetch field 0/1: one or two barriers per row
        hin = "true" if in_tile_halo(tiling) else "false"
        return f"k_step2<{stencil}, float, {n}, {tiling['tx']}, {tiling['pf'] + 1}, {hin}>"
    # the last argument: buffers below 4 GiB (one buffer resource for all populations)
    return f"k_step<{lattice}, {stencil}, float, {n}, {tiling['tx']}, {tiling['ty']}, {tiling['pf']}, false>"


# two-step tile widths whose workgroups hold the halo columns in the tile's own
# lanes (tx + 4R + 2 = 256 lanes: E4 R = 1, E8 R = 2); the others add an edge wave
IN_TILE_HALO = {250: 6, 246: 10}


def in_tile_halo(tiling: dict) -> bool:
    return tiling.get("steps", 1) == 2 and tiling["tx"] in IN_TILE_HALO


def grid_threads(tiling: dict) -> int:
    if in_tile_halo(tiling):
        return tiling["blocks"] * (tiling["tx"] + IN_TILE_HALO[tiling["tx"]])
    extra = 64 if tiling.get("steps", 1) == 2 else 0  # the two-step kernel's edge wave
    return tiling["blocks"] * (tiling["tx"] * tiling["ty"] + extra)


def counters_from_profile(stencil: str, noise: bool, tiling: dict, lattice: str = "D2Q9"):
    """Counter measurements of the step kernel per launch (HBM bytes:
    FETCH_SIZE + WRITE_SIZE scaled by the counters' reading of a plain copy of
    known size; VALU wave-instructions: SQ_INSTS_VALU) from the committed
    rocprofv3 summary, for the same kernel source and launch shape (or the
    nearest shape of the same kernel); (entry, note) or None."""
    path = os.path.join(ROOT, "profiles", "step_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        doc = json.load(fh)
    if doc.get("kernel_hash") != kernel_hash():
        return None
    name = kernel_name(stencil, noise, tiling, lattice)
    threads = grid_threads(tiling)
    same = [e for e in doc["entries"] if e["kernel"].endswith(name)]
    for e in same:
        if e["grid_threads"] == threads:
            return e, "same kernel and launch shape"
    if same:  # the autotuner picked another march length than in the counter run
        e = min(same, key=lambda e: abs(e["grid_threads"] - threads))
        return e, f"same kernel, nearest launch shape ({e['grid_threads']} threads in the " \
                  f"counter run, {threads} here)"
    return None


COPY_BYTES = 1 << 30  # size of the calibration copy in copy_ceiling()
PMC_ARGS = "--steps 2 --warmup 1 --kernel-steps 16 --no-cpu-baseline --no-surrogate"


def ingest_pmc(fetch_csv: str, write_csv: str, valu_csv: str, out_path: str):
    """Builds profiles/step_traffic.json from three rocprofv3 counter runs of
    this script (FETCH_SIZE, WRITE_SIZE, SQ_INSTS_VALU).  FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) are scaled so that the plain 1 GiB copy of
    copy_ceiling() reads 1 GiB fetched and 1 GiB written; the step kernels'
    per-launch means are then HBM bytes per launch.  SQ_INSTS_VALU counts
    the VALU instructions the waves issue (each acts on up to 64 lanes)."""
    import csv
    from collections import defaultdict

    def load(path, counter, calibrate=True):
        sums, counts, copies = defaultdict(float), defaultdict(int), []
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                name, grid, v = r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])
                if "fsc::k_copy" in name:
                    copies.append((grid, v))
                elif "fsc::k_step<" in name or "fsc::k_step2<" in name:
                    key = (name.replace("void ", "").split("(")[0], grid)
                    sums[key] += v
                    counts[key] += 1
        if not calibrate:
            return {k: sums[k] / counts[k] for k in sums}, counts, 1.0
        # the calibration copy is the most frequent k_copy launch
        grids = defaultdict(list)
        for g, v in copies:
            grids[g].append(v)
        cal = max(grids.values(), key=len)
        scale = COPY_BYTES / (sum(cal) / len(cal) * 1024.0)
        return {k: sums[k] / counts[k] * 1024.0 * scale for k in sums}, counts, scale

    fetch, counts, fscale = load(fetch_csv, "FETCH_SIZE")
    write, _, wscale = load(write_csv, "WRITE_SIZE")
    valu, _, _ = load(valu_csv, "SQ_INSTS_VALU", calibrate=False)
    entries = []
    for key in sorted(fetch):
        if key not in write:
            continue
        entries.append(dict(kernel=key[0], grid_threads=key[1], launches=counts[key],
                            fetch_bytes=int(fetch[key]), write_bytes=int(write[key]),
                            bytes_per_launch=int(fetch[key] + write[key]),
                            valu_insts_per_launch=int(valu[key]) if key in valu else None))
    for e in entries:
        e["kernel"] = e["kernel"].replace("fsc::", "")
    # kept: of every kernel the launch shape with the most launches (the one
    # timed; the others are tuning trials), and of the two-step kernels with
    # noise also the shapes near the tuned march lengths (within a factor 2
    # of the timed one), where another box's autotuner may land
    best = {}
    for e in entries:
        if e["kernel"] not in best or e["launches"] > best[e["kernel"]]["launches"]:
            best[e["kernel"]] = e
    fams = ("k_step2<StencilE4_2D, float, true,", "k_step2<StencilE8_2D, float, true,")
    keep = set(id(e) for e in best.values())
    for e in entries:
        b = best[e["kernel"]]
        if e["kernel"].startswith(fams) and b["launches"] > 11 and \
                0.5 <= e["grid_threads"] / b["grid_threads"] <= 2.0:
            keep.add(id(e))
    entries = sorted((e for e in entries if id(e) in keep),
                     key=lambda e: (e["kernel"], e["grid_threads"]))
    doc = dict(kernel_hash=kernel_hash(),
               commands=[f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d <fetch_dir> -o run "
                         f"-- python3 bench.py {PMC_ARGS}",
                         f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d <write_dir> -o run "
                         f"-- python3 bench.py {PMC_ARGS}",
                         f"rocprofv3 --pmc SQ_INSTS_VALU --output-format csv -d <valu_dir> -o run "
                         f"-- python3 bench.py {PMC_ARGS}",
                         "python3 bench.py --ingest-pmc <fetch_dir>/run_counter_collection.csv "
                         "<write_dir>/run_counter_collection.csv "
                         "<valu_dir>/run_counter_collection.csv"],
               calibration=dict(note="plain 16-byte copy (fsc_copy) of 1 GiB; counter KiB x scale "
                                     "x 1024 = bytes", fetch_scale=round(fscale, 4),
                                write_scale=round(wscale, 4)),
               entries=entries)
    with open(out_path, "w") as fh:
        head = {k: v for k, v in doc.items() if k != "entries"}
        fh.write(json.dumps(head, indent=1)[:-2] + ',\n "entries": [\n')
        fh.write(",\n".join("  " + json.dumps(e) for e in entries) + "\n ]\n}\n")
    return doc


TRACE_ARGS = "--steps 4 --warmup 1 --kernel-steps 400 --no-cpu-baseline --no-surrogate"


def summarize_trace(trace_dir: str, log_path: str, out_path: str):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats --output-format
    csv` run of this script: rocprofv3's own per-kernel statistics, the
    per-launch-shape means of the step kernels from the dispatch trace, and
    the same run's HIP-event timing of the benchmarked launch shape."""
    import csv
    from collections import defaultdict
    with open(os.path.join(trace_dir, "run_kernel_stats.csv")) as fh:
        stats = list(csv.DictReader(fh))
    shapes = defaultdict(list)
    with open(os.path.join(trace_dir, "run_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            if "fsc::k_step<" in r["Kernel_Name"] or "fsc::k_step2<" in r["Kernel_Name"]:
                key = (r["Kernel_Name"].replace("void ", "").split("(")[0], int(r["Grid_Size_X"]))
                shapes[key].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    bench = None
    with open(log_path) as fh:
        for line in fh:
            if line.startswith('{"metric"'):
                bench = json.loads(line)
    lines = ["# Fused step kernels: rocprofv3 kernel trace of bench.py", "",
             "Command (repository root as working directory, TMPDIR=/tmp):", "",
             f"    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- "
             f"python3 bench.py {TRACE_ARGS} > <log>",
             f"    python3 bench.py --summarize-trace <dir> <log> <this file>", ""]
    if bench:
        rf = bench["roofline"]
        t = rf["tiling"]
        grid = grid_threads(t)
        kname = rf["kernel"]
        key = next((k for k in shapes if k[1] == grid and k[0].replace("fsc::", "").endswith(kname)),
                   None)
        lines += [f"## Benchmarked launch ({bench['config']['workload']}, {t.get('steps', 1)} "
                  f"step(s) per launch)", "",
                  f"- kernel: `{kname}`, {t['blocks']} blocks ({grid} threads)",
                  f"- HIP events in the same run: {rf['avg_launch_us']} us per launch"]
        if key:
            v = shapes[key]
            lines.append(f"- rocprofv3 dispatch trace: {sum(v) / len(v) / 1e3:.2f} us mean over "
                         f"{len(v)} dispatches (min {min(v) / 1e3:.2f}, max {max(v) / 1e3:.2f})")
        lines += [f"- algorithmic bytes per launch: {rf['nodes_per_launch']} nodes x "
                  f"{rf['algorithmic_bytes_per_node']} B (every population read and written "
                  f"once) = {rf['algorithmic_bytes_per_launch']} B", ""]
    lines += ["## Step kernels by launch shape (dispatch trace)", "",
              "| kernel | grid threads | dispatches | mean us |", "|---|---|---|---|"]
    for (name, grid), v in sorted(shapes.items(), key=lambda kv: -sum(kv[1]))[:16]:
        lines.append(f"| `{name.replace('fsc::', '')}` | {grid} | {len(v)} | "
                     f"{sum(v) / len(v) / 1e3:.2f} |")
    lines += ["", "## rocprofv3 kernel statistics (run_kernel_stats.csv, top 12)", "",
              "| kernel | calls | mean us | % of GPU time |", "|---|---|---|---|"]
    for r in stats[:12]:
        name = r["Name"].replace("void ", "").split("(")[0].replace("fsc::", "")
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{r['Percentage']} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


SUR_TRACE_ARGS = "--steps 1 --warmup 1 --kernel-steps 16 --no-cpu-baseline --no-extra"
BF16_PEAK_TFLOPS = 2500.0  # dense BF16 matrix-core peak of the part


def summarize_surrogate_trace(trace_dir: str, log_path: str, out_path: str):
    """Markdown summary of the surrogate's kernels in a `rocprofv3
    --kernel-trace --stats --output-format csv` run of this script: per
    kernel, the dispatches and mean duration; for the 32 -> 32 matrix-core
    layer (k_mid) the achieved BF16 rate per launch from the rollout's batch
    (the bench's held-out seeds, 128^2 pixels each)."""
    import csv
    import re
    from collections import defaultdict
    bench = None
    with open(log_path) as fh:
        for line in fh:
            if line.startswith('{"metric"'):
                bench = json.loads(line)
    per = defaultdict(list)
    with open(os.path.join(trace_dir, "run_kernel_trace.csv")) as fh:
        for r in csv.DictReader(fh):
            name = r["Kernel_Name"]
            m = re.match(r"_ZN3fsc(\d+)(\w+)", name)  # names rocprofv3 leaves mangled
            if m:
                ident = m.group(2)[:int(m.group(1))]
                rest = m.group(2)[int(m.group(1)):]
                args = re.findall(r"L([bi])(\d+)E", rest[:24])
                flag = ("<" + ", ".join(("true" if v == "1" else "false") if t == "b" else v
                                        for t, v in args) + ">") if args else ""
                short = ident + flag
            elif "fsc::k_" in name:
                short = name.replace("void ", "").split("(")[0].replace("fsc::", "")
            else:
                continue
            if short.split("<")[0] in ("k_input", "k_first", "k_mid", "k_mid_lds", "k_last",
                                       "k_img_part", "k_img_total", "k_pred"):
                per[short].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    lines = ["# Surrogate kernels: rocprofv3 kernel trace of bench.py (rollout part)", "",
             "Command (repository root as working directory, TMPDIR=/tmp):", "",
             f"    rocprofv3 --kernel-trace --stats --output-format csv -d <dir> -o run -- "
             f"python3 bench.py {SUR_TRACE_ARGS} > <log>",
             f"    python3 bench.py --summarize-surrogate-trace <dir> <log> <this file>", ""]
    batch = None
    models = {}
    if bench and "surrogate" in bench:
        su = bench["surrogate"]
        batch = su["held_out_seeds"]
        models = su["models"]
        for name, mo in models.items():
            lines.append(f"- {name}: {mo['model']}; rollout of {batch} images of 128^2 pixels: "
                         f"{mo['surrogate_s_per_stride'] * 1e6:.1f} us per stride (one captured "
                         f"graph per rollout) against {mo['lattice_s_per_stride'] * 1e3:.1f} ms of "
                         f"lattice (speedup {mo['speedup_at_5pct']}x), "
                         f"{mo['bf16_tflops_in_rollout']} TFLOP/s BF16 over the whole pass")
        lines.append("")
    lines += ["| kernel | dispatches | mean us | note |", "|---|---|---|---|"]
    means = {}
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        mean = sum(v) / len(v)
        means[name] = mean
        note = ""
        if name.startswith("k_mid") and batch:  # the generic and the LDS-staged forms
            flops = 2 * 9 * 32 * 32 * batch * 128 * 128
            tf = flops / (mean * 1e-9) / 1e12
            note = (f"{flops / 1e9:.2f} GFLOP per launch: {tf:.1f} TFLOP/s, "
                    f"{tf / BF16_PEAK_TFLOPS * 100:.1f}% of the BF16 peak")
        lines.append(f"| `{name}` | {len(v)} | {mean / 1e3:.2f} | {note} |")
    # kernel time of one inference pass of each model from the per-kernel means
    mid = means.get("k_mid_lds<false, false>") or means.get("k_mid<false, false>")
    for name, mo in models.items():
        K = 2 if "2ch" in name else 1
        layers = int(name.split("layer")[0])
        first = means.get(f"k_first<{K}, false, true>")
        if first and mid and "k_last" in means and "k_pred" in means:
            tot = first + (layers - 2) * mid + means["k_last"] + means["k_pred"]
            lines.append(f"\n{name}: kernel time per pass {tot / 1e3:.1f} us (k_first + "
                         f"{layers - 2} x k_mid_lds + k_last + k_pred); the rollout takes "
                         f"{mo['surrogate_s_per_stride'] * 1e6:.1f} us per pass in wall time.")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def time_steps(obj, steps: int, stream, torch):
    """Average duration of one lattice time step of the fused step kernel (HIP
    events on the library's stream), over `steps` steps without measurement."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    obj.run(steps, 0)
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / steps * 1e-3  # s per step


STENCIL_NAME = {(2, 4): "StencilE4_2D", (2, 8): "StencilE8_2D", (3, 4): "StencilE4_3D"}


def kernel_view(cfg, tiling, t_step, noise=True):
    """Kernel figures of a lattice's fused step: launch time, algorithmic bytes
    per launch (each launch reads and writes every population of every node
    once: 2 Q x 4 B per node, whether it advances one step or two), and the
    counters' bytes and VALU instructions for the same kernel and launch shape
    from the committed summary."""
    D = cfg["D"]
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    spl = tiling.get("steps", 1)
    t_launch = t_step * spl
    alg = n * bytes_per_lup(D, cfg["precision"])
    stencil = STENCIL_NAME[(D, cfg["stencil"])]
    lattice = "D2Q9" if D == 2 else "D3Q19"
    out = dict(kernel=kernel_name(stencil, noise, tiling, lattice), steps_per_launch=spl,
               nodes_per_launch=n, lups_per_launch=n * spl, avg_launch_us=round(t_launch * 1e6, 2),
               algorithmic_bytes_per_launch=alg,
               hbm_gbs=alg / t_launch / 1e9, traffic=None, valu_tops=None, counters=None)
    cnt = counters_from_profile(stencil, noise, tiling, lattice)
    if cnt and cfg["precision"] == "fp32":
        entry, note = cnt
        out["traffic"] = entry["bytes_per_launch"]
        out["measured_hbm_gbs"] = entry["bytes_per_launch"] / t_launch / 1e9
        if entry.get("valu_insts_per_launch"):
            out["valu_tops"] = entry["valu_insts_per_launch"] * 64 / t_launch / 1e12
        out["counters"] = note
    return out


def params_of(cfg, fsc, kBT=None):
    return fsc.make_params(D=cfg["D"], nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"],
                           stencil=cfg["stencil"], precision=cfg["precision"], T_hat=cfg["T_hat"],
                           rho0=cfg["rho0"], kBT=cfg["kBT"] if kBT is None else kBT,
                           seed=cfg["seed"])


def run_quench(args, torch, fsc, I):
    """The headline: the deep quench from the homogeneous state, K periods of
    `sk_every` lattice steps, each ending in one S(k, t)/L(t) sample, timed
    between two device synchronisations.  The warm-up periods (autotuning,
    graph capture) run first on the same lattice, which is then reset to the
    homogeneous state so the timed region is the workload from t = 0."""
    cfg = I.DEEP_QUENCH
    every = cfg["sk_every"]
    stream = torch.cuda.Stream()
    lat = fsc.Lattice(params_of(cfg, fsc), stream=stream)
    lat.init_uniform()
    lat.series_enable(args.warmup + 2)
    lat.run(max(args.warmup, 1) * every, every)
    lat.init_uniform()
    lat.series_enable(args.steps + 2)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    lat.run(args.steps * every, every)
    e1.record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gpu_dt = e0.elapsed_time(e1) * 1e-3
    ser = lat.read_series()
    st = lat.stats(allow_diverged=True)
    tiling = lat.tiling
    # kernel-only timing of the fused step in the same launch configuration
    t_step = time_steps(lat, args.kernel_steps, stream, torch)
    lat.close()
    L = [float(v) for v in ser["L"]]
    ok = (len(L) == args.steps and all(math.isfinite(v) and v > 0 for v in L)
          and list(ser["step"]) == [every * (k + 1) for k in range(args.steps)] and st["bad"] == 0)
    n = cfg["nx"] * cfg["ny"]
    return dict(cfg=cfg, lups=n * every * args.steps, dt=dt, gpu_dt=gpu_dt, t_step=t_step,
                tiling=tiling, samples=len(L), samples_ok=ok, L_first=L[0] if L else None,
                L_last=L[-1] if L else None, rho_range=(st["rho_min"], st["rho_max"]))


def run_ensemble(torch, fsc, I, steps=2000):
    """The 64-replica metastable ensemble (sides 128/256/512), `steps` steps with
    its S(k) sample of every replica every 100 steps inside the timed region."""
    reps = I.ensemble_replicas(n=64, seed=0, kBT=1e-13)
    plist = [fsc.make_params(**{k: v for k, v in r.items() if k != "precision"}, precision="fp32")
             for r in reps]
    lups = sum(r["nx"] * r["ny"] for r in reps)
    every = I.ENSEMBLE["sk_every"]
    stream = torch.cuda.Stream()
    ens = fsc.Ensemble(plist, stream=stream)
    ens.init_uniform()
    ens.run(4 * every, every)  # autotune, graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(steps, every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t_step = time_steps(ens, 400, stream, torch)
    tiling = ens.tiling
    ens.close()
    cfg = dict(D=2, nx=lups, ny=1, nz=1, stencil=4, precision="fp32")
    kv = kernel_view(cfg, tiling, t_step)
    return {"mlups": round(lups * steps / dt / 1e6, 1), "steps_timed": steps,
            "samples_timed": steps // every, "lattice_updates_per_step": lups,
            "sides": sorted({r["nx"] for r in reps}), "kBT": 1e-13,
            "metric_hbm_roofline_frac": round(72 * lups * steps / dt / 1e9 / HBM_PEAK_GBS, 4),
            "kernel": kv["kernel"], "avg_launch_us": kv["avg_launch_us"],
            "kernel_hbm_frac": round(kv["hbm_gbs"] / HBM_PEAK_GBS, 4),
            "kernel_valu_frac": None if kv["valu_tops"] is None else
            round(kv["valu_tops"] / VALU_PEAK_TOPS, 4),
            "tiling": tiling}


def run_lattice(cfg, torch, fsc, steps=None, every=None, kernel_steps=200, kBT=None):
    """One lattice of a workload: `steps` steps with an S(k) sample every
    `every` steps (wall clock), and the fused step alone (HIP events)."""
    stream = torch.cuda.Stream()
    lat = fsc.Lattice(params_of(cfg, fsc, kBT), stream=stream)
    lat.init_uniform()
    lat.run(64, 0)  # autotune, graph capture
    out = {}
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    if steps:
        lat.run(every, every)  # the measurement plan and its graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.run(steps, every)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.update(mlups=round(n * steps / dt / 1e6, 1), steps_timed=steps,
                   samples_timed=steps // every,
                   metric_hbm_roofline_frac=round(bytes_per_lup(cfg["D"], cfg["precision"]) * n
                                                  * steps / dt / 1e9 / HBM_PEAK_GBS, 4))
    t = time_steps(lat, kernel_steps, stream, torch)
    tiling = lat.tiling
    lat.close()
    kv = kernel_view(cfg, tiling, t, noise=(cfg["kBT"] if kBT is None else kBT) > 0)
    out.update(kernel=kv["kernel"], kernel_mlups=round(n / t / 1e6, 1),
               avg_launch_us=kv["avg_launch_us"],
               kernel_hbm_frac=round(kv["hbm_gbs"] / HBM_PEAK_GBS, 4),
               tiling=f"{tiling['tx']}x{tiling['ty']}/pf{tiling['pf']}/{tiling['blocks']}blk/"
                      f"{tiling['steps']}step")
    if kv["traffic"]:
        out["measured_bytes_per_node_launch"] = round(kv["traffic"] / n, 2)
        out["measured_hbm_gbs"] = round(kv["measured_hbm_gbs"], 1)
    if kv["valu_tops"]:
        out["kernel_valu_frac"] = round(kv["valu_tops"] / VALU_PEAK_TOPS, 4)
    return out


def copy_ceiling(torch, fsc, nbytes=1 << 30, reps=20):
    """Practical HBM read+write bandwidth: a plain 16-byte copy of 1 GiB."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.Stream()
    for _ in range(3):
        fsc.device_copy(a.data_ptr(), b.data_ptr(), nbytes, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fsc.device_copy(a.data_ptr(), b.data_ptr(), nbytes, stream)
    e1.record(stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del a, b
    return 2 * nbytes / t / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(I, budget_s: float):
    """The FP64 oracle on bounded samples of the workloads, all host threads
    (and one thread on the headline's lattice): whole lattices of the same
    size and parameters from the homogeneous state, a window of steps sized to
    the time budget (one step first, to size it).  Headline: the 4096^2 deep
    quench; windows of the 64-replica ensemble and the 256^3 D3Q19 lattice."""
    import oracle as O

    def window(cfg, budget, threads=None):
        if threads:
            O.set_threads(threads)
        G = O.coupling_from_reduced_temperature(cfg["T_hat"])
        shape = (cfg["ny"], cfg["nx"]) if cfg["D"] == 2 else (cfg["nz"], cfg["ny"], cfg["nx"])
        f = O.uniform_state(cfg["D"], shape, cfg["rho0"])
        kw = dict(G=G, kind=cfg["stencil"], kBT=cfg["kBT"], seed=cfg["seed"],
                  replica=cfg.get("replica", 0))
        t0 = time.perf_counter()
        f = O.step(f, 1, t0=0, **kw)
        t1 = time.perf_counter() - t0
        k = max(0, min(199, int(budget / max(t1, 1e-9)) - 1))
        t0 = time.perf_counter()
        if k:
            O.step(f, k, t0=1, **kw)
        tk = time.perf_counter() - t0
        n = f[0].size
        return (k + 1) * n, t1 + tk, k + 1

    threads = O.max_threads()
    q = I.DEEP_QUENCH
    lups, t, k = window(q, budget_s * 0.5)
    lups1, t1, k1 = window(q, 0.0, threads=1)
    O.set_threads(threads)
    out = dict(value=lups / t / 1e6, unit="MLUPS", cores=threads, kind="oracle", cpu=cpu_model(),
               single_core_value=round(lups1 / t1 / 1e6, 3),
               sample=f"the 4096^2 D2Q9 E8 deep quench (the headline lattice, same parameters) from "
                      f"the homogeneous state, {k} steps: {lups / 1e6:.0f} M lattice updates in "
                      f"{t:.1f} s on {threads} threads; single thread: {k1} step in {t1:.1f} s")
    windows = {}
    reps = I.ensemble_replicas(n=64, seed=0, kBT=1e-13)
    done, tt, nrep, steps = 0, 0.0, 0, 0
    for r in reps:
        if tt > budget_s * 0.25:
            break
        c = dict(r, nz=1)
        l, dt_, k = window(c, 0.25 * budget_s / 8)
        done, tt, nrep, steps = done + l, tt + dt_, nrep + 1, k
    windows[I.ENSEMBLE["name"]] = dict(mlups=round(done / tt / 1e6, 3), replicas=nrep,
                                       seconds=round(tt, 2))
    m3 = I.METASTABLE_3D
    l, dt_, k = window(m3, budget_s * 0.25)
    windows[m3["name"]] = dict(mlups=round(l / dt_ / 1e6, 3), steps=k, seconds=round(dt_, 2))
    out["windows"] = windows
    return out


def surrogate_flops(meta, pixels: int) -> int:
    """Multiply-add FLOPs of one network pass over `pixels` pixels (2 per MAC)."""
    C, K, L = 32, meta.get("in_ch", 2), meta["layers"]  # K: input channels
    per_pixel = 2 * 9 * (K * C + (L - 2) * C * C + C)
    return per_pixel * pixels


def run_surrogate(torch, seeds=16):
    """The learned surrogates on held-out seeds of the 1024^2 deep quench:
    rollouts from the lattice state at t = 2048, S(k, t) error per stride
    against the lattice, the horizon within 5%, and the wall-clock speedup over
    the lattice for the same strides on this GPU, without and with the lattice
    warm-up to the rollout's start.  Both the committed 9-layer two-channel
    network and the 5-layer one-channel network the workload names, on one
    set of lattice trajectories."""
    from paper_2212_07848_amd import surrogate as SU
    t0_snap, n_out = 8, 16
    snaps, t_lbm = SU.run_quench(torch, range(seeds), n=1024, n_snap=t0_snap + n_out,
                                 seed_base=1000)
    out = {"workload": "d2q9_1024x1024_fp32_e8_quench, 8x8 block means, stride 256 steps",
           "held_out_seeds": seeds, "t0": t0_snap * 256, "models": {}}
    for name, path in (("9layer_2ch", SU.MODEL_PATH), ("5layer_1ch", SU.MODEL_5X1_PATH)):
        if not os.path.exists(path):
            continue
        sur, meta = SU.load_model(path, max_batch=seeds)
        ev = SU.evaluate(torch, sur, range(seeds), n=1024, t0_snaps=(t0_snap,), n_out=n_out,
                         snaps=snaps, t_lbm=t_lbm)
        sur.close()
        st = ev["starts"][0]
        h = st["horizon_5pct"]
        out["models"][name] = {
            "model": f"{meta['layers']}-layer 3x3 conv, 32 channels, input "
                     + ("(rho_t, rho_t - rho_t-256)" if meta.get("in_ch", 2) == 2 else "rho_t")
                     + ", BF16 MFMA / FP32 accumulate",
            "train_seeds": meta.get("train_seeds"),
            "horizon_strides_at_5pct": h, "horizon_lattice_steps": h * ev["stride"],
            "persistence_horizon_strides": st["persistence_horizon_5pct"],
            "sk_rel_err_per_stride": [round(r["sk_rel_err"], 4) for r in st["rows"]],
            "speedup_at_5pct": round(st["speedup"], 1),
            "speedup_with_lattice_warmup": None if st["speedup_with_warmup"] is None
            else round(st["speedup_with_warmup"], 2),
            "bf16_tflops_in_rollout": round(surrogate_flops(meta, 128 * 128) * seeds * n_out
                                            / st["surrogate_seconds"] / 1e12, 1),
            "lattice_s_per_stride": round(st["lbm_seconds"] / n_out, 5),
            "surrogate_s_per_stride": round(st["surrogate_seconds"] / n_out, 7)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # bench steps: periods of 500 lattice steps each ending in one S(k,t)/L(t)
    # sample; 100 periods = the deep-quench workload's 50 000 steps (about 11 s)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-steps", type=int, default=1000)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--ingest-pmc", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "VALU_CSV"),
                    help="write profiles/step_traffic.json from three rocprofv3 counter runs")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TRACE_DIR", "LOG", "OUT_MD"),
                    help="write a markdown summary of a rocprofv3 kernel-trace run")
    ap.add_argument("--summarize-surrogate-trace", nargs=3, metavar=("TRACE_DIR", "LOG", "OUT_MD"),
                    help="write a markdown summary of the surrogate kernels of a kernel-trace run")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_surrogate_trace:
        summarize_surrogate_trace(*args.summarize_surrogate_trace)
        return
    if args.ingest_pmc:
        doc = ingest_pmc(*args.ingest_pmc, os.path.join(ROOT, "profiles", "step_traffic.json"))
        print(f"{len(doc['entries'])} step-kernel launch shapes, calibration {doc['calibration']}")
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.steps < 1 or args.kernel_steps < 2 or args.kernel_steps % 2:
        print(json.dumps({"error": "--steps must be >= 1 and --kernel-steps even and >= 2"}))
        sys.exit(2)

    import torch
    import fsc_inputs as I
    import paper_2212_07848_amd as fsc

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    r = run_quench(args, torch, fsc, I)
    cfg = r["cfg"]
    mlups = r["lups"] / r["dt"] / 1e6
    kv = kernel_view(cfg, r["tiling"], r["t_step"])
    hbm_view = {"bound": "hbm", "achieved": round(kv["hbm_gbs"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(kv["hbm_gbs"] / HBM_PEAK_GBS, 4),
                "traffic": kv["traffic"]}
    alu_view = None if kv["valu_tops"] is None else {
        "bound": "alu", "achieved": round(kv["valu_tops"], 2), "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "Tlane-op/s", "frac": round(kv["valu_tops"] / VALU_PEAK_TOPS, 4),
        "traffic": kv["traffic"]}
    # the binding roof is the one nearer its peak
    main_view, other = hbm_view, alu_view
    if alu_view and alu_view["frac"] > hbm_view["frac"]:
        main_view, other = alu_view, hbm_view
    every = cfg["sk_every"]
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["dt"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "lattice": [cfg["nx"], cfg["ny"]], "stencil": "E8",
                   "T_hat": cfg["T_hat"], "rho0": cfg["rho0"], "kBT": cfg["kBT"],
                   "collision": "MRT all rates 1 (BGK tau=1)",
                   "lattice_steps_per_step": every,
                   "lattice_steps_timed": every * args.steps,
                   "samples_timed": r["samples"],
                   "sample": "radial S(k,t) and L(t), FP64 bins, one per step (every 500 "
                             "lattice steps), recorded inside the replayed graphs",
                   "samples_ok": r["samples_ok"], "L_first": r["L_first"], "L_last": r["L_last"],
                   "gpu_event_seconds": round(r["gpu_dt"], 4)},
        # the metric's own "% HBM roofline": 72 B per lattice update x the update
        # rate / 8 TB/s -- the bandwidth a kernel moving every population once per
        # update would need; the two-step kernel moves half of it (roofline below)
        "metric_hbm_roofline_frac": round(72 * r["lups"] / r["dt"] / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": dict(main_view, **{
            "kernel": kv["kernel"],
            "traffic_source": kv["counters"] or "no counter run of this kernel source",
            "steps_per_launch": kv["steps_per_launch"],
            "nodes_per_launch": kv["nodes_per_launch"],
            "algorithmic_bytes_per_node": bytes_per_lup(2, "fp32"),
            "algorithmic_bytes_per_launch": kv["algorithmic_bytes_per_launch"],
            "avg_launch_us": kv["avg_launch_us"],
            "measured_hbm_gbs": None if kv["traffic"] is None else round(kv["measured_hbm_gbs"], 1),
            "other": other,
            "tiling": r["tiling"]}),
    }
    out["roofline"]["copy_ceiling_gbs"] = round(copy_ceiling(torch, fsc), 1)
    if not args.no_extra:
        extra = {I.ENSEMBLE["name"]: run_ensemble(torch, fsc, I)}
        m3 = I.METASTABLE_3D
        extra[m3["name"]] = run_lattice(m3, torch, fsc, steps=1000, every=m3["sk_every"])
        extra[cfg["name"] + "_noise_free_kernel"] = run_lattice(cfg, torch, fsc, kBT=0.0,
                                                                kernel_steps=600)
        out["extra"] = extra
    if not args.no_surrogate:
        out["surrogate"] = run_surrogate(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
