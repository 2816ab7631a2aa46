"""Domain growth after a deep quench into the unstable region: the 4096^2 D2Q9
E8 FP32 workload at the critical density and T_hat = 0.7, with the radially
binned S(k, t) and the domain length L(t) recorded every 500 steps inside the
hipGraph chunks (fsc_series_enable; L = 2 pi sum_k S / sum_k |k| S, the
inverse first moment of the structure factor).

After the linear instability has saturated, the domains coarsen and L grows
as a power of time; `growth_exponent` fits d ln L / d ln t over a late window.
The paper shows the final interface shapes of such quenches (its Fig. 1) but
no growth law, so the fit is reported, not compared.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import _lib as F


def growth_exponent(steps, L, t_min, t_max=None):
    """Least-squares slope of ln L against ln t over t_min <= t <= t_max."""
    t = np.asarray(steps, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    sel = (t >= t_min) & (t <= (t_max if t_max is not None else t.max())) & (L > 0)
    if sel.sum() < 2:
        return None
    A = np.stack([np.log(t[sel]), np.ones(sel.sum())], axis=1)
    coef, *_ = np.linalg.lstsq(A, np.log(L[sel]), rcond=None)
    return float(coef[0])


def run(n=4096, steps=50000, every=500, stencil=8, T_hat=0.7, rho0=1.0, kBT=1e-4, seed=0,
        stream=None):
    """One n^2 lattice from the homogeneous state; returns the recorded series
    (step, L, per-shell S) and the lattice wall time."""
    p = F.make_params(D=2, nx=n, ny=n, stencil=stencil, precision="fp32", T_hat=T_hat,
                      rho0=rho0, kBT=kBT, seed=seed)
    with F.Lattice(p, stream=stream) as lat:
        lat.init_uniform()
        lat.series_enable(steps // every + 1)
        t0 = time.perf_counter()
        lat.run(steps, every)
        st = lat.stats(allow_diverged=True)
        wall = time.perf_counter() - t0
        ser = lat.read_series()
        tiling = lat.tiling
    return dict(n=n, steps=steps, every=every, stencil=stencil, T_hat=T_hat, rho0=rho0, kBT=kBT,
                seed=seed, wall_seconds=wall, tiling=tiling, bad=int(st["bad"]),
                rho_min=float(st["rho_min"]), rho_max=float(st["rho_max"]),
                step=ser["step"].tolist(), L=ser["L"].tolist())


def main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="domain growth L(t) after a deep quench")
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--t-min", type=int, default=10000, help="start of the fit window")
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "coarsening.json"))
    a = ap.parse_args(argv)
    res = run(n=a.n, steps=a.steps, every=a.every)
    res["growth_exponent"] = growth_exponent(res["step"], res["L"], a.t_min)
    res["growth_exponent_window"] = [a.t_min, a.steps]
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    for s, L in zip(res["step"], res["L"]):
        if s in (500, 1000, 2000, 5000, 10000, 20000, 30000, 40000, 50000) or s == res["step"][-1]:
            print(f"t = {s:6d}: L = {L:8.2f}", flush=True)
    mlups = a.n * a.n * a.steps / res["wall_seconds"] / 1e6
    print(json.dumps(dict(growth_exponent=res["growth_exponent"], wall_seconds=round(res["wall_seconds"], 2),
                          mlups=round(mlups), tiling=res["tiling"], bad=res["bad"],
                          rho_range=[res["rho_min"], res["rho_max"]])), flush=True)


if __name__ == "__main__":
    main()
