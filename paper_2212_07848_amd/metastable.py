"""Lifetime of homogeneous states against the noise amplitude (the paper's
introduction and closing summary: unstable states separate at once, while in
the metastable region the time to phase separation grows without bound as
k_B theta goes to zero).

Replicas of one homogeneous state, each with its own k_B theta and noise seed,
run side by side on the ensemble path (one launch per step).  Every
`check_every` steps the FP64 reductions give each replica's density range; a
replica has phase-separated at the first check where that range exceeds half
of the binodal gap, n_max - n_min > (n_l - n_g) / 2 (a nucleus or domain of
the other phase exists; sub-critical fluctuations stay far below this).  The
first-passage step is recorded, or None if it never happens within
max_steps.  A replica whose density turns non-positive (noise far beyond the
fluctuating-hydrodynamics range) is counted as diverged, not separated.

What the two regimes predict:

* unstable (inside the spinodal): the fastest linear mode grows at a rate
  s_max from an amplitude ~ sqrt(k_B theta), so the onset time is
  t = a + ln(1/k_B theta) / (2 s_max): logarithmic in the noise.
* metastable (between binodal and spinodal): the state is linearly stable;
  a critical nucleus has to be formed by a fluctuation, so the lifetime grows
  like exp(Delta F / k_B theta) and is infinite at zero noise.

`growth_rate` gives s_max of the linearised continuum equations (Eq. 13 with
the lattice pressure of Eq. 15) for the on-axis modes, with the longitudinal
viscosity of the moment-space collision.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import _lib as F
from .scaling import (CS2, binodal_densities, coupling, density_at_spinodal_distance, h_axis,
                      spinodal_densities)


def growth_rate(n0, T_hat, lam_shear=1.0, lam_bulk=1.0, D=2, stencil=4, nk=4096):
    """Largest growth rate per step of a density mode along an axis, and its k:
    s^2 + nu_L k^2 s + c^2(k) k^2 = 0, with c^2(k) = c_s^2 - G psi0 psi0' h(k)
    and nu_L = 2 (D - 1)/D nu + zeta, nu = c_s^2 (1/lam_shear - 1/2),
    zeta = 2/D c_s^2 (1/lam_bulk - 1/2).  Zero if no mode grows."""
    G = coupling(T_hat)
    psi0 = math.exp(-1.0 / n0)
    nu = CS2 * (1.0 / lam_shear - 0.5)
    zeta = 2.0 / D * CS2 * (1.0 / lam_bulk - 0.5)
    nuL = 2.0 * (D - 1) / D * nu + zeta
    k = np.linspace(1e-4, math.pi, nk)
    c2 = CS2 - G * psi0 * psi0 / n0 ** 2 * h_axis(k, stencil)
    disc = (nuL * k * k / 2.0) ** 2 - c2 * k * k
    s = np.where(c2 < 0, -nuL * k * k / 2.0 + np.sqrt(np.maximum(disc, 0.0)), 0.0)
    i = int(np.argmax(s))
    return float(s[i]), float(k[i])


def run(n0, kBTs, seeds=4, n=128, T_hat=0.8, max_steps=200000, check_every=500, seed=7,
        stream=None, log=None):
    """First-passage steps to phase separation of n x n D2Q9 FP32 E4 lattices
    at density n0, `seeds` replicas per k_B theta.  Returns the per-replica
    times (None: not separated within max_steps) and their summary per
    k_B theta."""
    ng_b, nl_b, _ = binodal_densities(T_hat)
    gap = 0.5 * (nl_b - ng_b)
    kb = [float(k) for k in kBTs for _ in range(seeds)]
    plist = [F.make_params(D=2, nx=n, ny=n, stencil=4, precision="fp32", T_hat=T_hat, rho0=n0,
                           kBT=k, seed=seed, replica=i) for i, k in enumerate(kb)]
    ens = F.Ensemble(plist, stream=stream)
    ens.init_uniform()
    t_sep = [None] * len(kb)
    step = 0
    t0 = time.perf_counter()
    while step < max_steps and any(t is None for t in t_sep):
        ens.run(check_every, 0)
        step += check_every
        for i in range(len(kb)):
            if t_sep[i] is not None:
                continue
            st = ens.stats(i, allow_diverged=True)
            if st["bad"]:
                t_sep[i] = -step  # non-positive or non-finite density: noise too strong
            elif st["rho_max"] - st["rho_min"] > gap:
                t_sep[i] = step
        if log and step % (200 * check_every) == 0:
            log(f"step {step}: separated {sum(t is not None for t in t_sep)} of {len(kb)}")
    ens.close()
    rows = [summarize(k, t_sep[j * seeds:(j + 1) * seeds]) for j, k in enumerate(kBTs)]
    return dict(n0=float(n0), T_hat=T_hat, n=n, max_steps=max_steps, check_every=check_every,
                steps=step, seconds=time.perf_counter() - t0, rows=rows)


def summarize(kBT, ts):
    """One row of the study from the first-passage steps of its replicas
    (None: still homogeneous at the end; negative: diverged at that step)."""
    seeds = len(ts)
    done = [t for t in ts if t is not None and t > 0]
    bad = sum(1 for t in ts if t is not None and t < 0)
    # the median counts replicas still homogeneous at the end as later than any
    # separated one, so it exists once more than half have separated
    srt = sorted(done) + [math.inf] * (seeds - len(done) - bad)
    med = float(np.median(srt)) if bad == 0 and 2 * len(done) > seeds else None
    return dict(kBT=float(kBT), separated=len(done), diverged=bad, seeds=seeds,
                times=[None if t is None or t < 0 else t for t in ts],
                mean=(float(np.mean(done)) if len(done) == seeds else None), median=med)


def onset_slope(rows, kbt_max=1e-5):
    """Least-squares slope of the mean onset step against ln(1/k_B theta)
    over the rows where every replica separated and k_B theta <= kbt_max
    (larger noise starts the growth outside the linear regime)."""
    use = [r for r in rows if r["mean"] is not None and r["kBT"] <= kbt_max]
    x = [math.log(1.0 / r["kBT"]) for r in use]
    y = [r["mean"] for r in use]
    if len(x) < 2:
        return None
    return float(np.polyfit(x, y, 1)[0])


def barrier_fit(rows):
    """Arrhenius fit ln(median lifetime) = a + Delta F / k_B theta over the
    rows with a median; returns (Delta F, a, r^2) or None."""
    pts = [(1.0 / r["kBT"], math.log(r["median"])) for r in rows
           if r["median"] is not None and math.isfinite(r["median"])]
    if len(pts) < 3:
        return None
    x, y = np.array(pts).T
    b, a = np.polyfit(x, y, 1)
    r2 = 1.0 - np.sum((y - (a + b * x)) ** 2) / np.sum((y - y.mean()) ** 2)
    return float(b), float(a), float(r2)


def state_points(T_hat=0.8, d_meta=1.3e-3, frac_unstable=0.5):
    """The two homogeneous states of the study on one isotherm: a gas-side
    metastable density at |1 - p/p_s| = d_meta, and an unstable density at
    the given fraction of the interval between the spinodals."""
    ng, nl = spinodal_densities(T_hat)
    return dict(metastable=density_at_spinodal_distance(T_hat, d_meta, "gas"),
                unstable=ng + frac_unstable * (nl - ng))


def main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="lifetime of homogeneous states against k_B theta")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--d-meta", type=float, default=1.3e-3)
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--meta-kbt", default="6e-4,5e-4,4e-4,3.5e-4,3e-4,2.5e-4,1e-13",
                    help="comma-separated k_B theta values of the metastable state")
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "metastable_study.json"))
    a = ap.parse_args(argv)
    sp = state_points(d_meta=a.d_meta)
    say = lambda s: print(s, flush=True)
    uns = run(sp["unstable"], [1e-3, 1e-5, 1e-7, 1e-9, 1e-11, 1e-13], seeds=a.seeds, n=a.n,
              max_steps=4000, check_every=5, log=say)
    met = run(sp["metastable"], [float(v) for v in a.meta_kbt.split(",")], seeds=a.seeds,
              n=a.n, max_steps=a.max_steps, check_every=100, log=say)
    s, k = growth_rate(sp["unstable"], 0.8)
    res = dict(unstable=uns, metastable=met, growth_rate=s, k_fastest=k,
               onset_slope=onset_slope(uns["rows"]), onset_slope_linear=1.0 / (2.0 * s),
               barrier=barrier_fit(met["rows"]))
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    for name, r in (("unstable", uns), ("metastable", met)):
        for row in r["rows"]:
            say(f"{name} n0={r['n0']:.4f} kBT={row['kBT']:.1e}: {row['separated']}/{row['seeds']} "
                f"separated, mean {row['mean']}, median {row['median']}")
    say(json.dumps(dict(onset_slope=res["onset_slope"], linear=res["onset_slope_linear"],
                        barrier=res["barrier"])))


if __name__ == "__main__":
    main()
