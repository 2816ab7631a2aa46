"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds no arithmetic of the method: it names the workloads (lattice
sizes, reduced temperatures, mean densities, noise energies, seeds) and draws
seeded random fields.  The mean densities of the metastable ensemble are read
from tests/golden/metastable_windows.json, which oracle/make_workloads.py
writes from the equation of state.

The paper uses no dataset: every run starts from a homogeneous density plus a
noise seed on a periodic lattice, which is exactly what these inputs are.
"""
from __future__ import annotations

import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
WINDOWS = os.path.join(_HERE, "tests", "golden", "metastable_windows.json")

# 64^2 D2Q9, E4, FP64, BGK tau = 1, T_hat = 0.9, stable gas n0 = 0.5 (below the
# binodal 0.5688), kBT = 1e-4, seed 0, 1000 steps, S(k) every 10 steps.
SMALL_PARITY = dict(name="d2q9_64x64_fp64_e4", D=2, nx=64, ny=64, nz=1, stencil=4,
                    precision="fp64", T_hat=0.9, rho0=0.5, kBT=1e-4, seed=0, steps=1000,
                    sk_every=10)

# 4096^2 D2Q9, E8, FP32-shifted, deep quench n0 = 1 at T_hat = 0.7, kBT = 1e-4,
# 50k steps, S(k, t) and L(t) every 500 steps.
DEEP_QUENCH = dict(name="d2q9_4096x4096_fp32_e8_quench", D=2, nx=4096, ny=4096, nz=1, stencil=8,
                   precision="fp32", T_hat=0.7, rho0=1.0, kBT=1e-4, seed=0, steps=50000,
                   sk_every=500)

# 256^3 D3Q19, E4, FP32-shifted, metastable gas n0 = 0.62 near the spinodal
# (0.6454) at T_hat = 0.8, kBT = 1e-13, 10k steps, radial S(k) every 500.
METASTABLE_3D = dict(name="d3q19_256cube_fp32_e4_metastable", D=3, nx=256, ny=256, nz=256,
                     stencil=4, precision="fp32", T_hat=0.8, rho0=0.62, kBT=1e-13, seed=0,
                     steps=10000, sk_every=500)


def load_windows():
    with open(WINDOWS) as fh:
        return json.load(fh)["windows"]


def ensemble_replicas(n: int = 64, seed: int = 0, kBT: float = 1e-13, sides=(128, 256, 512)):
    """The batched metastable ensemble: n D2Q9 E4 FP32 replicas.

    Side drawn uniformly from `sides`; T_hat stratified over [0.6, 0.99]; the
    mean density sits between binodal and spinodal at fraction theta in
    (0.25, 0.5, 0.75) (cycling), gas side for even replicas and liquid side for
    odd ones; noise seed `seed`, replica index r.
    """
    rng = np.random.default_rng(seed)
    side = rng.choice(np.asarray(sides), size=n)
    win = load_windows()
    reps = []
    for r in range(n):
        th = 0.6 + 0.39 * (r + 0.5) / n
        key = f"{th:.12f}"
        if key not in win:
            raise KeyError(f"no metastable window tabulated for T_hat={th}")
        w = win[key]
        theta = (0.25, 0.5, 0.75)[r % 3]
        if r % 2 == 0:
            n0 = w["binodal_gas"] + theta * (w["spinodal_gas"] - w["binodal_gas"])
        else:
            n0 = w["binodal_liquid"] + theta * (w["spinodal_liquid"] - w["binodal_liquid"])
        reps.append(dict(D=2, nx=int(side[r]), ny=int(side[r]), nz=1, stencil=4, precision="fp32",
                         T_hat=th, rho0=float(n0), kBT=kBT, seed=seed, replica=r))
    return reps


ENSEMBLE = dict(name="d2q9_ensemble64_mixed128-512_fp32_e4_metastable", steps=20000,
                sk_every=100)


def random_populations(Q: int, shape, rho0: float, amp: float, seed: int) -> np.ndarray:
    """Positive populations f_i(x) = rho0/Q (1 + amp U(-1, 1)), independent per
    population and node: a generic (non-equilibrium) input state."""
    rng = np.random.default_rng(seed)
    return (rho0 / Q) * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(Q,) + tuple(shape)))


def wide_density_populations(Q: int, shape, lo: float, hi: float, modes: int,
                             seed: int) -> np.ndarray:
    """Populations rho(x)/Q (with 2% independent jitter) where rho sweeps the
    whole range [lo, hi] in a few long waves: a state with the density
    contrast of a phase-separated lattice, gas and liquid both present."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    field = np.zeros(shape)
    for _ in range(modes):
        k = [2 * np.pi * rng.integers(1, 4) / s for s in shape]
        field = field + np.cos(sum(kk * g for kk, g in zip(k, grids)) + rng.uniform(0, 2 * np.pi))
    field = (field - field.min()) / (field.max() - field.min())
    rho = lo + (hi - lo) * field
    f = np.empty((Q,) + tuple(shape))
    for i in range(Q):
        f[i] = rho / Q * (1.0 + 0.02 * rng.uniform(-1, 1, size=shape))
    return f


def smooth_density_populations(Q: int, shape, rho0: float, amp: float, modes: int,
                               seed: int) -> np.ndarray:
    """Populations rho(x)/Q with rho a sum of a few random long-wave cosines of
    relative amplitude amp (a structured input with a ragged spectrum)."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    rho = np.full(shape, rho0)
    for _ in range(modes):
        k = [2 * np.pi * rng.integers(0, 4) / s for s in shape]
        ph = rng.uniform(0, 2 * np.pi)
        rho = rho + rho0 * amp / modes * np.cos(sum(kk * g for kk, g in zip(k, grids)) + ph)
    f = np.empty((Q,) + tuple(shape))
    for i in range(Q):
        f[i] = rho / Q * (1.0 + 0.02 * rng.uniform(-1, 1, size=shape))
    return f
