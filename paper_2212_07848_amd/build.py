"""Builds ``libfsc.so`` (the HIP library behind include/fsc.h) for gfx950.

Every translation unit is compiled with ``hipcc --offload-arch=gfx950`` in
parallel, then linked into the package directory.  Packed FP32 instructions
are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfsc.so")

SOURCES = [
    "fsc_api.hip",
    "fsc_step.hip",
    "fsc_step_d2e4_f32.hip",
    "fsc_step_d2e4_f64.hip",
    "fsc_step_d2e8_f32.hip",
    "fsc_step_d2e8_f64.hip",
    "fsc_step2_e4.hip",
    "fsc_step2_e8.hip",
    "fsc_step_d3e4_f32.hip",
    "fsc_step_d3e4_f64.hip",
    "fsc_measure.hip",
    "fsc_surrogate.hip",
    "fsc_linear.hip",
]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ROCM = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
ARCH = os.environ.get("FSC_OFFLOAD_ARCH", "gfx950")
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-result"]


def _newest_header() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(ROOT, "include", "fsc.h"))
    return max(os.path.getmtime(h) for h in hs)


# The fused step kernels must not spill vector registers or use scratch: a
# spill to scratch memory costs them a large part of their speed, and the
# FP64 D3Q19 form once gave wrong values next to the register limit.  Their
# translation units are compiled with the compiler's resource report, which is
# checked here; SGPR spills (to vector-register lanes) are logged.
STEP_SOURCES = [s for s in SOURCES if s.startswith("fsc_step") and s != "fsc_step.hip"]


def resource_report(stderr: str):
    """Per kernel: VGPRs, AGPRs, scratch bytes per lane, VGPR and SGPR spills,
    from the -Rpass-analysis=kernel-resource-usage remarks."""
    keys = {"VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
            "VGPRs Spill": "vgpr_spill", "SGPRs Spill": "sgpr_spill",
            "Occupancy [waves/SIMD]": "waves"}
    rows, cur = [], None
    for line in stderr.splitlines():
        if "remark:" not in line:
            continue
        body = line.split("remark:", 1)[1].strip()
        if body.startswith("Function Name:"):
            cur = {"name": body.split(":", 1)[1].split()[0]}
            rows.append(cur)
            continue
        if cur is None or ":" not in body:
            continue
        k, v = body.split(":", 1)
        v = v.split("[-Rpass")[0].strip()
        if k.strip() in keys and v.isdigit():
            cur[keys[k.strip()]] = int(v)
    return rows


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _newest_header():
            return obj
    check = src in STEP_SOURCES
    # step kernels: resource report, and no FP contraction beyond the written
    # fused multiply-adds (every kernel then rounds the same way)
    extra = ["-Rpass-analysis=kernel-resource-usage", "-ffp-contract=off"] if check else []
    cmd = [HIPCC, "-c", *CFLAGS, *extra, os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if check:
        rows = resource_report(r.stderr)
        bad = [k for k in rows if k.get("scratch", 0) > 0 or k.get("vgpr_spill", 0) > 0]
        with open(os.path.join(BUILD, os.path.splitext(src)[0] + ".resources.txt"), "w") as fh:
            for k in rows:
                fh.write(" ".join(f"{a}={k[a]}" for a in ("vgpr", "agpr", "scratch", "vgpr_spill",
                                                          "sgpr_spill", "waves") if a in k)
                         + f" {k['name']}\n")
        if bad:
            os.remove(obj)
            raise RuntimeError(f"{src}: step kernels with scratch or VGPR spills: "
                               + ", ".join(k["name"] for k in bad))
    return obj


def build(verbose: bool = False, jobs: int | None = None, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
           "-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects")
        worst = 0
        for src in STEP_SOURCES:
            path = os.path.join(BUILD, os.path.splitext(src)[0] + ".resources.txt")
            if os.path.exists(path):
                for line in open(path):
                    worst = max([worst] + [int(t.split("=")[1]) for t in line.split()
                                           if t.startswith("sgpr_spill=")])
        print(f"step kernels: no scratch, no VGPR spills; largest SGPR spill count {worst} "
              f"(per-kernel report in {BUILD}/*.resources.txt)")
    return LIB


def build_lds_poison(out: str | None = None) -> str:
    """Debug build with FSC_LDS_POISON: every kernel's LDS starts as NaN, so a
    read of a slot not yet written by the launch shows up in the results.
    Objects go to _build/lds_poison/; run the GPU tests on it with
    FSC_LIB=<out> (the binding then loads it instead of libfsc.so)."""
    out = out or os.path.join(BUILD, "libfsc_lds_poison.so")
    odir = os.path.join(BUILD, "lds_poison")
    os.makedirs(odir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def one(src):
        obj = os.path.join(odir, os.path.splitext(src)[0] + ".o")
        extra = ["-ffp-contract=off"] if src in STEP_SOURCES else []
        cmd = [HIPCC, "-c", *CFLAGS, *extra, "-DFSC_LDS_POISON", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as ex:
        objs = list(ex.map(one, srcs))
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", out,
           "-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    return out


if __name__ == "__main__":
    if "--lds-poison" in sys.argv:
        i = sys.argv.index("--lds-poison")
        print(build_lds_poison(sys.argv[i + 1] if i + 1 < len(sys.argv) else None))
    else:
        build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
