"""Interface topology after spinodal decomposition in 3D (the paper's Fig. 1,
upper panel): on the unstable branch of the T_hat = 0.8 isotherm, the final
state of a periodic box is a droplet, a droplet-cylinder, a flat slab, a
bubble-cylinder or a bubble as the initial density rises.

The classification is topological.  For each phase (liquid: n above the
mid-point of the coexisting densities; gas: the rest) the largest connected
component of the periodic box is found together with the set of lattice
translations it wraps around; the number of independent wrapping directions
of liquid and gas identifies the shape:

    (0, 3) droplet          liquid ball in connected gas
    (1, 3) droplet-cylinder liquid tube
    (2, 2) flat             liquid slab
    (3, 1) bubble-cylinder  gas tube
    (3, 0) bubble           gas ball

Anything else (a still bicontinuous network, several domains) is "mixed".
The lattice runs on the ensemble path (D3Q19 FP32, E4, one replica per
density); host numpy/scipy does the labelling only.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import _lib as F
from .scaling import binodal_densities, spinodal_densities

SHAPES = {(0, 3): "droplet", (1, 3): "droplet-cylinder", (2, 2): "flat",
          (3, 1): "bubble-cylinder", (3, 0): "bubble"}
ORDER = ["droplet", "droplet-cylinder", "flat", "bubble-cylinder", "bubble"]


def wrapping(mask: np.ndarray):
    """Largest periodic connected component of a boolean 3D field (faces
    connect; periodic in every axis): returns (cells, rank) where rank is the
    number of independent lattice translations the component wraps around
    (0: a bounded blob, 1: a tube, 2: a sheet, 3: space-filling)."""
    from scipy import ndimage

    mask = np.asarray(mask, dtype=bool)
    lab, nlab = ndimage.label(mask)  # 6-connected, not periodic
    if nlab == 0:
        return 0, 0
    sizes = np.bincount(lab.ravel())[1:]
    # Union-find over labels with an offset (in box units) to the root: the
    # offset of label a relative to its root is off[a]; an edge a -> b that
    # crosses the face along axis k forward says pos(b) = pos(a) + e_k.
    parent = list(range(nlab + 1))
    off = [np.zeros(3, dtype=np.int64) for _ in range(nlab + 1)]
    windings = {}

    def root_off(i):
        path = []
        while parent[i] != i:
            path.append(i)
            i = parent[i]
        # compress, accumulating offsets from the top down
        acc = np.zeros(3, dtype=np.int64)
        for j in reversed(path):
            acc = acc + off[j]
            off[j] = acc.copy()
            parent[j] = i
        return i

    def union(a, b, shift):
        ra, rb = root_off(a), root_off(b)
        oa = off[a] if a != ra else np.zeros(3, dtype=np.int64)
        ob = off[b] if b != rb else np.zeros(3, dtype=np.int64)
        # position of b relative to ra through this edge: oa + shift; through rb: ob
        if ra == rb:
            w = oa + shift - ob
            if np.any(w):
                windings.setdefault(ra, []).append(w)
            return
        # attach rb under ra: pos(rb) = pos(ra) + oa + shift - ob
        parent[rb] = ra
        off[rb] = oa + shift - ob
        if rb in windings:
            windings.setdefault(ra, []).extend(windings.pop(rb))

    for k in range(3):
        e = np.zeros(3, dtype=np.int64)
        e[k] = 1
        last = np.take(lab, -1, axis=k)
        first = np.take(lab, 0, axis=k)
        both = (last > 0) & (first > 0)
        for a, b in set(zip(last[both].tolist(), first[both].tolist())):
            union(a, b, e)
    # sizes and windings per root
    tot = {}
    for lbl in range(1, nlab + 1):
        r = root_off(lbl)
        tot[r] = tot.get(r, 0) + int(sizes[lbl - 1])
    big = max(tot, key=tot.get)
    ws = windings.get(big, [])
    rank = int(np.linalg.matrix_rank(np.array(ws, dtype=np.float64))) if ws else 0
    return tot[big], rank


def classify(rho: np.ndarray, n_mid: float):
    liquid = rho > n_mid
    cl, rl = wrapping(liquid)
    cg, rg = wrapping(~liquid)
    return dict(shape=SHAPES.get((rl, rg), "mixed"), liquid_wraps=rl, gas_wraps=rg,
                liquid_fraction=float(liquid.mean()),
                largest_liquid=cl / liquid.size, largest_gas=cg / liquid.size)


DEFAULT_FRACTIONS = (0.03, 0.1, 0.25, 0.4, 0.5, 0.6, 0.75, 0.9, 0.97)


def default_densities(T_hat=0.8, fractions=DEFAULT_FRACTIONS):
    """Densities at the given fractions of the unstable interval between the
    gas and liquid spinodals of the isotherm."""
    ng, nl = spinodal_densities(T_hat)
    return [ng + f * (nl - ng) for f in fractions]


def run(densities, n=64, T_hat=0.8, kBT=1e-10, max_steps=60000, check_every=2000, seed=11,
        seeds=1, stream=None, log=None):
    """`seeds` replicas per density (n^3 D3Q19 FP32, E4, BGK tau = 1, noise
    seeds differing by replica), stepped until every replica has held the
    same classified shape for two checks in a row (or max_steps).  Returns the
    per-replica history and final shapes, and the shape counts per density."""
    ng_b, nl_b, _ = binodal_densities(T_hat)
    n_mid = 0.5 * (ng_b + nl_b)
    dens = [float(r) for r in densities for _ in range(seeds)]
    plist = [F.make_params(D=3, nx=n, ny=n, nz=n, stencil=4, precision="fp32", T_hat=T_hat,
                           rho0=r, kBT=kBT, seed=seed, replica=i)
             for i, r in enumerate(dens)]
    ens = F.Ensemble(plist, stream=stream)
    ens.init_uniform()
    hist = [[] for _ in dens]
    stable = [0] * len(dens)
    t0 = time.perf_counter()
    lattice_s = 0.0
    step = 0
    while step < max_steps and min(stable) < 2:
        t1 = time.perf_counter()
        ens.run(check_every, 0)
        ens.stats(0)  # synchronises
        lattice_s += time.perf_counter() - t1
        step += check_every
        for i in range(len(dens)):
            st = ens.stats(i)
            if st["bad"]:
                raise RuntimeError(f"density {dens[i]} diverged at step {step}")
            c = classify(ens.density(i), n_mid)
            c["step"] = step
            prev = hist[i][-1]["shape"] if hist[i] else None
            stable[i] = stable[i] + 1 if (c["shape"] == prev and c["shape"] != "mixed") else 0
            hist[i].append(c)
        if log:
            log(f"step {step}: " + ", ".join(h[-1]["shape"] for h in hist))
    ens.close()
    final = [dict(rho0=r, liquid_fraction_lever=(r - ng_b) / (nl_b - ng_b),
                  **{k: v for k, v in h[-1].items()}) for r, h in zip(dens, hist)]
    counts = []
    for j, r in enumerate(densities):
        shapes = [f["shape"] for f in final[j * seeds:(j + 1) * seeds]]
        counts.append(dict(rho0=float(r), liquid_fraction_lever=(float(r) - ng_b) / (nl_b - ng_b),
                           shapes={s: shapes.count(s) for s in sorted(set(shapes))}))
    return dict(n=n, T_hat=T_hat, kBT=kBT, seeds=seeds, steps=step, lattice_seconds=lattice_s,
                wall_seconds=time.perf_counter() - t0, counts=counts, final=final, history=hist)


def main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="3D interface topology on the unstable branch")
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--max-steps", type=int, default=80000)
    ap.add_argument("--check-every", type=int, default=2000)
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--seed", type=int, default=11, help="noise seed (replica ids 0, 1, ...)")
    ap.add_argument("--fractions", default=",".join(str(f) for f in DEFAULT_FRACTIONS),
                    help="comma-separated fractions of the interval between the spinodals")
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "topology_study.json"))
    a = ap.parse_args(argv)
    fr = tuple(float(f) for f in a.fractions.split(","))
    res = run(default_densities(fractions=fr), n=a.n, max_steps=a.max_steps,
              check_every=a.check_every, seed=a.seed, seeds=a.seeds,
              log=lambda s: print(s[:200], flush=True))
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    for c in res["counts"]:
        print(f"n0 = {c['rho0']:.4f} (lever fraction {c['liquid_fraction_lever']:.3f}): "
              f"{c['shapes']}", flush=True)
    print(json.dumps(dict(steps=res["steps"], lattice_seconds=round(res["lattice_seconds"], 1))))


if __name__ == "__main__":
    main()
