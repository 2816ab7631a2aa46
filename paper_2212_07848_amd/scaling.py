"""Scaling of the long-wavelength structure factor near the spinodal and the
critical point (the paper's Fig. 3), on the ensemble path.

S(k -> 0) = n0 k_B theta / (dp/dn) grows like the isothermal compressibility
(Eq. 8): as (p_hat - p_hat_s)^(-1/2) along an isotherm towards the spinodal
(Eq. 10), and as (1 - T_hat)^(-1) along the binodal towards the critical point
(Eq. 8 with n_hat -> 1).  This module picks the state points from the reduced
EoS (Eq. 7), runs one replica per (state point, seed) in a single ensemble at
k_B theta = 1e-13 (all lattice work in libfsc.so), and extrapolates S(0) from
the measured axis bins with the exact k-dependence of Eq. 16:

    1/S(k) = (T - G psi0 psi0' h(k)) / (n0 k_B theta),  h(k) -> 1 as k -> 0,

a straight line in h(k) whose value at h = 1 is 1/S(0).  The fitted S(0) of
each state point, its exact value, and the exponents fitted through both are
returned.  Host-side numpy does the state-point algebra and the fits only.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import _lib as F

CS2 = 1.0 / 3.0  # lattice temperature T = c_s^2 of the isothermal D2Q9 model


# ---------------------------------------------------------------------------
# Reduced EoS (Eq. 7) and its special points; psi = exp(-1/n), n_c = 1.
# ---------------------------------------------------------------------------
def p_hat(n, T):
    return 2.0 * n * T - np.exp(2.0 - 2.0 / n)


def dp_hat(n, T):
    return 2.0 * T - 2.0 * np.exp(2.0 - 2.0 / n) / n ** 2


def _bisect(f, a, b, tol=1e-15):
    fa = f(a)
    for _ in range(200):
        m = 0.5 * (a + b)
        fm = f(m)
        if (fm > 0) == (fa > 0):
            a, fa = m, fm
        else:
            b = m
        if b - a < tol * max(1.0, abs(m)):
            break
    return 0.5 * (a + b)


def spinodal_densities(T):
    """Gas and liquid spinodal densities (dp/dn = 0) at T_hat < 1: the roots of
    n^2 T = exp(2 - 2/n) on either side of the maximum of exp(2 - 2/n)/n^2
    at n = 1."""
    g = lambda n: n * n * T - math.exp(2.0 - 2.0 / n)
    return _bisect(g, 0.05, 1.0), _bisect(g, 1.0, 50.0)


def binodal_densities(T):
    """Coexisting gas and liquid densities at T_hat < 1: equal pressure and
    equal area in the specific volume v = 1/n (Maxwell's construction)."""
    ng_s, nl_s = spinodal_densities(T)

    def branch(p, lo, hi):
        return _bisect(lambda n: p_hat(n, T) - p, lo, hi)

    def area(p):
        ng = branch(p, 1e-6, ng_s)
        nl = branch(p, nl_s, 200.0)
        # int_{v_l}^{v_g} (p(v) - p) dv with v = 1/n, by Gauss-Legendre
        x, w = np.polynomial.legendre.leggauss(64)
        vl, vg = 1.0 / nl, 1.0 / ng
        v = 0.5 * (vg - vl) * x + 0.5 * (vg + vl)
        return float(np.sum(w * (p_hat(1.0 / v, T) - p)) * 0.5 * (vg - vl)), ng, nl

    p_lo = max(p_hat(nl_s, T), 1e-12)
    p_hi = p_hat(ng_s, T)
    p0 = _bisect(lambda p: area(p)[0], p_lo, p_hi, tol=1e-14)
    _, ng, nl = area(p0)
    return ng, nl, p0


def density_at_spinodal_distance(T, d, side):
    """Density on the metastable branch with |1 - p_hat/p_hat_s| = d."""
    ng_s, nl_s = spinodal_densities(T)
    ng_b, nl_b, _ = binodal_densities(T)
    if side == "gas":
        ps = p_hat(ng_s, T)
        return _bisect(lambda n: p_hat(n, T) - ps * (1.0 - d), ng_b, ng_s)
    ps = p_hat(nl_s, T)
    return _bisect(lambda n: p_hat(n, T) - ps * (1.0 + d), nl_s, nl_b)


def coupling(T_hat):
    """G of Eq. 1 for psi = exp(-1/n): T_c = G/e^2 and T = c_s^2."""
    return math.exp(2.0) * CS2 / T_hat


def h_axis(k, stencil=4):
    """h(k) of the on-axis sound speed, sum_a w_a e_x sin(k e_x) / (2 tan(k/2)),
    for the interaction sets (weights normalised to sum w e_x^2 = 1).  E4 gives
    the same h in 2D and 3D: the neighbours with e_x = 1 weigh 1/3 + 2/12 in 2D
    and 1/6 + 4/12 in 3D, 1/2 either way."""
    if stencil == 4:
        sets = [(1, 1.0 / 3.0 + 2.0 / 12.0)]  # e_x = 1: (1,0) and (1,+-1)
    else:
        # E8: |e|^2 = 1, 2, 4, 5, 8 with weights 4/21, 4/45, 1/60, 2/315, 1/5040
        w1, w2, w4, w5, w8 = 4 / 21, 4 / 45, 1 / 60, 2 / 315, 1 / 5040
        sets = [(1, w1 + 2 * w2 + 2 * w5), (2, w4 + 2 * w5 + 2 * w8)]
    k = np.asarray(k, dtype=np.float64)
    num = sum(2.0 * w * e * np.sin(k * e) for e, w in sets)
    return num / (2.0 * np.tan(k / 2.0))


def sk_exact(k, n0, T_hat, kBT, stencil=4):
    """Eq. 16 along a lattice axis: S(k) = n0 kBT / (T - G psi0 psi0' h(k))."""
    G = coupling(T_hat)
    psi0 = math.exp(-1.0 / n0)
    dpsi = psi0 / n0 ** 2
    return n0 * kBT / (CS2 - G * psi0 * dpsi * h_axis(k, stencil))


def s0_exact(n0, T_hat, kBT):
    G = coupling(T_hat)
    psi0 = math.exp(-1.0 / n0)
    return n0 * kBT / (CS2 - G * psi0 * psi0 / n0 ** 2)


# ---------------------------------------------------------------------------
# Extrapolation and exponent fits.
# ---------------------------------------------------------------------------
def fit_s0(k, S, stencil=4, weights=None):
    """S(0) from 1/S(k) = alpha - beta h(k) (least squares over the given
    modes, relative weights); returns S(0) = 1/(alpha - beta)."""
    h = h_axis(k, stencil)
    y = 1.0 / np.asarray(S, dtype=np.float64)
    w = np.ones_like(y) if weights is None else np.asarray(weights, dtype=np.float64)
    A = np.stack([np.ones_like(h), -h], axis=1) * w[:, None]
    coef, *_ = np.linalg.lstsq(A, y * w, rcond=None)
    return 1.0 / (coef[0] - coef[1])


def fit_exponent(x, y):
    """Slope of log y against log x (least squares)."""
    lx, ly = np.log(np.asarray(x, dtype=np.float64)), np.log(np.asarray(y, dtype=np.float64))
    A = np.stack([lx, np.ones_like(lx)], axis=1)
    coef, *_ = np.linalg.lstsq(A, ly, rcond=None)
    return float(coef[0])


# ---------------------------------------------------------------------------
# The study.
# ---------------------------------------------------------------------------
DEFAULT_SPINODAL_D = (0.1, 0.03, 0.01, 0.003, 0.001)
DEFAULT_BINODAL_T = (0.8, 0.9, 0.95, 0.97, 0.98, 0.99)


def state_points(T_spin=0.8, spin_d=DEFAULT_SPINODAL_D, bin_T=DEFAULT_BINODAL_T):
    pts = []
    for side in ("gas", "liquid"):
        for d in spin_d:
            pts.append(dict(kind="spinodal", side=side, T_hat=T_spin, d=d,
                            rho0=density_at_spinodal_distance(T_spin, d, side)))
        for T in bin_T:
            ng, nl, _ = binodal_densities(T)
            pts.append(dict(kind="binodal", side=side, T_hat=T, d=1.0 - T,
                            rho0=ng if side == "gas" else nl))
    return pts


def run(points, n=64, seeds=4, kBT=1e-13, burn=4000, steps=16000, sk_every=50, kfit=6,
        seed_base=7000, stream=None, D=2):
    """One ensemble of len(points) x seeds replicas of n^D FP32 lattices
    (D2Q9 or D3Q19, E4, BGK tau = 1).  After `burn` steps the S(k)
    accumulators are reset; then `steps` steps with a sample every
    `sk_every`.  Returns the points with the measured axis S(k) (mean over
    seeds, axes and +-k), the fitted and exact S(0), and the lattice wall
    time."""
    plist = []
    for i, p in enumerate(points):
        for s in range(seeds):
            plist.append(F.make_params(D=D, nx=n, ny=n, nz=n if D == 3 else 1, stencil=4,
                                       precision="fp32", T_hat=p["T_hat"], rho0=p["rho0"],
                                       kBT=kBT, seed=seed_base + i, replica=s))
    ens = F.Ensemble(plist, stream=stream)
    ens.init_uniform()
    t0 = time.perf_counter()
    ens.run(burn, 0)
    ens.sk_reset()
    ens.run(steps, sk_every)
    wall = time.perf_counter() - t0
    m = np.arange(1, n // 2 + 1)
    k = 2.0 * np.pi * m / n
    out = []
    for i, p in enumerate(points):
        tot = np.zeros(len(m))
        cnt = np.zeros(len(m))
        for s in range(seeds):
            st = ens.stats(i * seeds + s)
            if st["bad"]:
                raise RuntimeError(f"state point {i} replica {s} diverged")
            S, _, c = ens.read_sk(i * seeds + s)
            tot += S[:, 1:n // 2 + 1].sum(axis=0)
            cnt += c[:, 1:n // 2 + 1].sum(axis=0)
        Sk = tot / cnt
        ex = sk_exact(k, p["rho0"], p["T_hat"], kBT)
        q = dict(p)
        q.update(k=k.tolist(), S=Sk.tolist(), S_exact=ex.tolist(),
                 S0_fit=float(fit_s0(k[:kfit], Sk[:kfit])),
                 S0_exact=s0_exact(p["rho0"], p["T_hat"], kBT),
                 samples=int(cnt[0] / (2 * D * seeds)))
        out.append(q)
    ens.close()
    return out, wall


def exponents(results):
    """Exponents of S(0) (fitted from the lattice, and exact at the same
    state points) against |1 - pi_s| along the isotherm and 1 - T_hat along
    the binodal, per side; asymptotic values -1/2 and -1."""
    ex = {}
    for kind, asym in (("spinodal", -0.5), ("binodal", -1.0)):
        for side in ("gas", "liquid"):
            pts = [r for r in results if r["kind"] == kind and r["side"] == side]
            if len(pts) < 2:
                continue
            pts = sorted(pts, key=lambda r: r["d"])
            d = [r["d"] for r in pts]
            ex[f"{kind}_{side}"] = dict(
                measured=fit_exponent(d, [r["S0_fit"] for r in pts]),
                exact_same_points=fit_exponent(d, [r["S0_exact"] for r in pts]),
                # local slope between the two points closest to the singularity
                measured_closest=fit_exponent(d[:2], [r["S0_fit"] for r in pts[:2]]),
                exact_closest=fit_exponent(d[:2], [r["S0_exact"] for r in pts[:2]]),
                asymptotic=asym, points=len(pts))
    return ex


def main(argv=None):
    import argparse

    ap = argparse.ArgumentParser(description="S(k -> 0) scaling near the spinodal and the critical point")
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3))
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--seeds", type=int, default=32)
    ap.add_argument("--burn", type=int, default=4000)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--out", default=os.path.join(os.getcwd(), "scaling_study.json"))
    a = ap.parse_args(argv)
    pts = state_points()
    res, wall = run(pts, n=a.n, seeds=a.seeds, burn=a.burn, steps=a.steps, D=a.dim)
    ex = exponents(res)
    doc = dict(D=a.dim, n=a.n, seeds=a.seeds, burn=a.burn, steps=a.steps, kBT=1e-13,
               lattice_seconds=wall, exponents=ex, points=res)
    with open(a.out, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(dict(lattice_seconds=round(wall, 2), exponents=ex)), flush=True)
    for r in res:
        print(f"{r['kind']:8s} {r['side']:6s} T={r['T_hat']:.3f} d={r['d']:.4g} n0={r['rho0']:.5f} "
              f"S0 fit/exact = {r['S0_fit'] / r['S0_exact']:.4f}", flush=True)


if __name__ == "__main__":
    main()
