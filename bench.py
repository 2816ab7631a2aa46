"""Throughput of the fluctuating Shan-Chen hot path on one MI355X.

Workload (default): the batched metastable ensemble -- 64 D2Q9 replicas of
side 128/256/512 (seeded draw), FP32 shifted populations, E4 force stencil,
T_hat stratified over [0.6, 0.99], mean densities between binodal and
spinodal, kBT = 1e-13, one fused kernel launch per step over all replicas,
S(k) of every replica accumulated in FP64 every 100 steps, replayed as
captured hipGraphs.  A "step" advances every replica by one time step.

Prints one JSON line (value = MLUPS over the whole ensemble) with the
roofline of the fused step kernel (HIP events on the library's stream) and
the FP64 CPU oracle timed on a bounded sample of the same workload.

The step kernel is the one the autotuner picks: with the two-step kernel
(temporal blocking) a launch advances two time steps with one read and one
write of the populations, so its HBM traffic per lattice update halves and
the vector ALUs become the bound; the roofline object then reports the ALU
bound (VALU lane-instructions per launch from a counter run, over the live
launch time, against the issue peak) and the HBM view beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
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
        return f"k_step2<{stencil}, float, {n}, {tiling['tx']}, {tiling['pf'] + 1}>"
    # the last argument: buffers below 4 GiB (one buffer resource for all populations)
    return f"k_step<{lattice}, {stencil}, float, {n}, {tiling['tx']}, {tiling['ty']}, {tiling['pf']}, false>"


def grid_threads(tiling: dict) -> int:
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
PMC_ARGS = "--steps 64 --warmup 8 --kernel-steps 16 --no-cpu-baseline --no-surrogate"


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
    # kept: every launch shape (march length) of the ensemble's two-step kernels
    # (the roofline reads the autotuner's choice among them), and of every other
    # kernel the shape with the most launches (the one timed; the others are
    # tuning trials)
    ens = "k_step2<StencilE4_2D, float, true,"
    best = {}
    for e in entries:
        if not e["kernel"].startswith(ens):
            if e["kernel"] not in best or e["launches"] > best[e["kernel"]]["launches"]:
                best[e["kernel"]] = e
    entries = [e for e in entries if e["kernel"].startswith(ens)] + sorted(best.values(),
                                                                          key=lambda e: e["kernel"])
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


TRACE_ARGS = "--steps 400 --warmup 40 --kernel-steps 200 --no-cpu-baseline --no-surrogate"


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
        kname = kernel_name("StencilE4_2D", True, t)
        key = next((k for k in shapes if k[1] == grid and k[0].endswith(kname)), None)
        lines += [f"## Benchmarked launch (64-replica D2Q9 ensemble, {t.get('steps', 1)} step(s) "
                  f"per launch)", "",
                  f"- kernel: `{kname}`, {t['blocks']} blocks ({grid} threads)",
                  f"- HIP events in the same run: {rf['avg_launch_us']} us per launch"]
        if key:
            v = shapes[key]
            lines.append(f"- rocprofv3 dispatch trace: {sum(v) / len(v) / 1e3:.2f} us mean over "
                         f"{len(v)} dispatches (min {min(v) / 1e3:.2f}, max {max(v) / 1e3:.2f})")
        lines += [f"- algorithmic bytes per launch: {rf['lups_per_launch']} lattice updates "
                  f"x {rf['algorithmic_bytes_per_lup']} B", ""]
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


SUR_TRACE_ARGS = "--steps 40 --warmup 8 --kernel-steps 16 --no-cpu-baseline --no-extra"
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
                flags = re.findall(r"Lb([01])E", rest[:12])
                flag = "<" + ", ".join("true" if f == "1" else "false" for f in flags) + ">" if flags else ""
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
    if bench and "surrogate" in bench:
        su = bench["surrogate"]
        batch = su["held_out_seeds"]
        lines += [f"- model: {su['model']}",
                  f"- rollout of {batch} images of 128^2 pixels: {su['surrogate_s_per_stride'] * 1e3:.3f} ms "
                  f"per stride against {su['lattice_s_per_stride'] * 1e3:.1f} ms of lattice "
                  f"(speedup {su['speedup_at_5pct']}x), {su['bf16_tflops_in_rollout']} TFLOP/s "
                  f"BF16 over the whole pass", ""]
    lines += ["| kernel | dispatches | mean us | note |", "|---|---|---|---|"]
    for name, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        mean = sum(v) / len(v)
        note = ""
        if name.startswith("k_mid") and batch:  # the generic and the LDS-staged forms
            flops = 2 * 9 * 32 * 32 * batch * 128 * 128
            tf = flops / (mean * 1e-9) / 1e12
            note = (f"{flops / 1e9:.2f} GFLOP per launch: {tf:.1f} TFLOP/s, "
                    f"{tf / BF16_PEAK_TFLOPS * 100:.1f}% of the BF16 peak")
        lines.append(f"| `{name}` | {len(v)} | {mean / 1e3:.2f} | {note} |")
    total = sum(sum(v) / len(v) * (len(v) // max(1, len(per.get("k_pred", [1])))) for v in per.values())
    lines += ["", f"Kernel time per pass (sum of the means, counting each kernel's launches per "
              f"pass): {total / 1e3:.1f} us.  Each launch is small (8 images of 128^2), so the "
              f"rollout is bound by launch latency and the gaps between its kernels, not by the "
              f"matrix cores."]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def time_steps(obj, steps: int, stream, torch):
    """Average duration of one fused step launch (HIP events on the library's
    stream), over `steps` launches without measurement."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    obj.run(steps, 0)
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / steps * 1e-3  # s per step


def run_ensemble(args, torch, fsc, I):
    reps = I.ensemble_replicas(n=args.replicas, seed=0, kBT=1e-13)
    plist = [fsc.make_params(**{k: v for k, v in r.items() if k != "precision"}, precision="fp32")
             for r in reps]
    lups = sum(r["nx"] * r["ny"] for r in reps)
    stream = torch.cuda.Stream()
    ens = fsc.Ensemble(plist, stream=stream)
    ens.init_uniform()
    ens.run(args.warmup, I.ENSEMBLE["sk_every"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(args.steps, I.ENSEMBLE["sk_every"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # kernel-only timing of the fused step (same launch configuration)
    t_step = time_steps(ens, args.kernel_steps, stream, torch)
    st = ens.stats(0)
    tiling = ens.tiling
    ens.close()
    return dict(lups=lups, dt=dt, t_step=t_step, stats_ok=st["bad"] == 0,
                sides=sorted({r["nx"] for r in reps}), nrep=len(reps), tiling=tiling)


def run_single(cfg, steps, torch, fsc, kBT=None):
    p = fsc.make_params(D=cfg["D"], nx=cfg["nx"], ny=cfg["ny"], nz=cfg["nz"],
                        stencil=cfg["stencil"], precision=cfg["precision"], T_hat=cfg["T_hat"],
                        rho0=cfg["rho0"], kBT=cfg["kBT"] if kBT is None else kBT, seed=cfg["seed"])
    stream = torch.cuda.Stream()
    lat = fsc.Lattice(p, stream=stream)
    lat.init_uniform()
    lat.run(64, 0)
    t = time_steps(lat, steps, stream, torch)
    tiling = lat.tiling
    lat.close()
    n = cfg["nx"] * cfg["ny"] * cfg["nz"]
    # algorithmic bandwidth: one read and one write of every population per update
    out = dict(mlups=n / t / 1e6,
               algorithmic_gbs=n * bytes_per_lup(cfg["D"], cfg["precision"]) / t / 1e9,
               ms_per_step=t * 1e3, tiling=f"{tiling['tx']}x{tiling['ty']}/pf{tiling['pf']}"
                                             f"/{tiling['blocks']}blk/{tiling['steps']}step")
    # counter figures of the same kernel from the committed summary, if present
    stencil = {(2, 4): "StencilE4_2D", (2, 8): "StencilE8_2D", (3, 4): "StencilE4_3D"}[
        (cfg["D"], cfg["stencil"])]
    noise = (cfg["kBT"] if kBT is None else kBT) > 0
    cnt = counters_from_profile(stencil, noise, tiling, "D2Q9" if cfg["D"] == 2 else "D3Q19")
    if cnt and cfg["precision"] == "fp32":
        entry, note = cnt
        t_launch = t * tiling.get("steps", 1)
        lups = n * tiling.get("steps", 1)
        out["measured_bytes_per_lup"] = entry["bytes_per_launch"] / lups
        out["measured_hbm_gbs"] = entry["bytes_per_launch"] / t_launch / 1e9
        if entry.get("valu_insts_per_launch"):
            out["valu_issue_frac"] = entry["valu_insts_per_launch"] * 64 / t_launch / 1e12 / VALU_PEAK_TOPS
        out["counters"] = note
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
    """The FP64 oracle on a bounded sample of the ensemble workload: whole
    replicas of the same workload, stepped until the time budget is used, on
    all host threads and then on one."""
    import oracle as O
    reps = I.ensemble_replicas(n=64, seed=0, kBT=1e-13)
    nsteps = 40

    def run(budget):
        done_lups, t_used, nrep = 0, 0.0, 0
        for r in reps:
            if t_used > budget:
                break
            G = O.coupling_from_reduced_temperature(r["T_hat"])
            f = O.uniform_state(2, (r["ny"], r["nx"]), r["rho0"])
            t0 = time.perf_counter()
            O.step(f, nsteps, G=G, kind=4, kBT=r["kBT"], seed=r["seed"], replica=r["replica"])
            t_used += time.perf_counter() - t0
            done_lups += r["nx"] * r["ny"] * nsteps
            nrep += 1
        return done_lups, t_used, nrep

    threads = O.max_threads()
    lups, t_used, nrep = run(budget_s)
    O.set_threads(1)
    lups1, t1, nrep1 = run(budget_s / 4)
    O.set_threads(threads)
    return dict(value=lups / t_used / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                cpu=cpu_model(), single_core_value=round(lups1 / t1 / 1e6, 3),
                sample=f"the first {nrep} of the 64 ensemble replicas (sides 128-512) x {nsteps} "
                       f"steps each, {lups / 1e6:.0f} M lattice updates in {t_used:.1f} s on "
                       f"{threads} threads; single thread: {nrep1} replicas in {t1:.1f} s")


def surrogate_flops(meta, pixels: int) -> int:
    """Multiply-add FLOPs of one network pass over `pixels` pixels (2 per MAC)."""
    C, K, L = 32, meta.get("in_ch", 2), meta["layers"]
    per_pixel = 2 * 9 * (K * C + (L - 2) * C * C + C)
    return per_pixel * pixels


def run_surrogate(torch):
    """The committed coarse-grained surrogate on held-out seeds of the 1024^2
    deep quench: rollout from the lattice state at t = 2048, S(k, t) error per
    stride against the lattice, the horizon within 5%, and the wall-clock
    speedup over the lattice for the same strides on this GPU."""
    from paper_2212_07848_amd import surrogate as SU
    sur, meta = SU.load_model()
    ev = SU.evaluate(torch, sur, range(8), n=1024, t0_snaps=(8,), n_out=16, seed_base=1000)
    sur.close()
    st = ev["starts"][0]
    h = st["horizon_5pct"]
    return {"workload": "d2q9_1024x1024_fp32_e8_quench, 8x8 block means, stride 256 steps",
            "model": f"{meta['layers']}-layer 3x3 conv, 32 channels, input (rho_t, rho_t - "
                     f"rho_t-256), BF16 MFMA / FP32 accumulate",
            "held_out_seeds": len(ev["seeds"]), "t0": st["t0"],
            "horizon_strides_at_5pct": h, "horizon_lattice_steps": h * ev["stride"],
            "persistence_horizon_strides": st["persistence_horizon_5pct"],
            "sk_rel_err_per_stride": [round(r["sk_rel_err"], 4) for r in st["rows"]],
            "speedup_at_5pct": round(st["speedup"], 1),
            "bf16_tflops_in_rollout": round(surrogate_flops(meta, 128 * 128) * len(ev["seeds"])
                                            * ev["n_out"] / st["surrogate_seconds"] / 1e12, 1),
            "lattice_s_per_stride": round(st["lbm_seconds"] / ev["n_out"], 5),
            "surrogate_s_per_stride": round(st["surrogate_seconds"] / ev["n_out"], 6)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the ensemble workload's own length: 20 000 steps per replica (about 2 s)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=400)
    ap.add_argument("--kernel-steps", type=int, default=1000)
    ap.add_argument("--replicas", type=int, default=64)
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

    import torch
    import fsc_inputs as I
    import paper_2212_07848_amd as fsc

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    r = run_ensemble(args, torch, fsc, I)
    mlups = r["lups"] * args.steps / r["dt"] / 1e6
    bpl = bytes_per_lup(2, "fp32")
    tiling = r["tiling"]
    steps_per_launch = tiling.get("steps", 1)
    t_launch = r["t_step"] * steps_per_launch
    # algorithmic HBM bytes per launch: 72 B per lattice update (one read and
    # one write of every population), times the updates the launch makes; a
    # launch of the two-step kernel moves half of that (measured: `traffic`)
    lups_per_launch = r["lups"] * steps_per_launch
    hbm = lups_per_launch * bpl / t_launch / 1e9
    cnt = counters_from_profile("StencilE4_2D", True, tiling)
    traffic, valu, note = None, None, "no counter run of this kernel source"
    if cnt:
        entry, note = cnt
        traffic = entry["bytes_per_launch"]
        if entry.get("valu_insts_per_launch"):
            valu = entry["valu_insts_per_launch"] * 64 / t_launch / 1e12  # lane-ops, T/s
    hbm_view = {"bound": "hbm", "achieved": round(hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm / HBM_PEAK_GBS, 4), "traffic": traffic}
    alu_view = None if valu is None else {
        "bound": "alu", "achieved": round(valu, 2), "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "Tlane-op/s", "frac": round(valu / VALU_PEAK_TOPS, 4), "traffic": traffic}
    # the binding roofline is the one nearer its peak
    main_view, other = hbm_view, alu_view
    if alu_view and alu_view["frac"] > hbm_view["frac"]:
        main_view, other = alu_view, hbm_view
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["dt"] / args.steps * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": I.ENSEMBLE["name"], "replicas": r["nrep"], "sides": r["sides"],
                   "lattice_updates_per_step": r["lups"], "stencil": "E4", "sk_every": 100,
                   "kBT": 1e-13, "collision": "MRT all rates 1 (BGK tau=1)"},
        "roofline": dict(main_view, **{
            "traffic_source": note,
            "kernel": kernel_name("StencilE4_2D", True, tiling),
            "steps_per_launch": steps_per_launch,
            "lups_per_launch": lups_per_launch,
            "algorithmic_bytes_per_lup": bpl,
            "avg_launch_us": round(t_launch * 1e6, 2),
            # what the counters saw move through HBM (temporal blocking keeps
            # the intermediate step on chip)
            "measured_bytes_per_lup": None if traffic is None else round(traffic / lups_per_launch, 2),
            "measured_hbm_gbs": None if traffic is None else round(traffic / t_launch / 1e9, 1),
            "other": other,
            "tiling": tiling}),
    }
    out["roofline"]["copy_ceiling_gbs"] = round(copy_ceiling(torch, fsc), 1)
    if not args.no_extra:
        extra = {}
        for cfg, steps in ((I.DEEP_QUENCH, 300), (I.METASTABLE_3D, 200)):
            e = run_single(cfg, steps, torch, fsc)
            e["algorithmic_frac"] = round(e["algorithmic_gbs"] / HBM_PEAK_GBS, 4)
            extra[cfg["name"]] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in e.items()}
        e = run_single(I.DEEP_QUENCH, 300, torch, fsc, kBT=0.0)
        extra[I.DEEP_QUENCH["name"] + "_noise_free"] = {
            k: (round(v, 3) if isinstance(v, float) else v) for k, v in e.items()}
        out["extra"] = extra
    if not args.no_surrogate:
        out["surrogate"] = run_surrogate(torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(I, args.cpu_budget)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
