"""FP64 CPU oracle of the fluctuating Shan-Chen lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``; never by the product package.

The step itself lives in ``fsc_oracle.c`` (plain C, double precision); this
module loads it through ctypes and adds the structure-factor measurement in
numpy.  Paper: Lulli et al., arXiv:2212.07848.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle_fsc.so")
_lib = None

CS2 = 1.0 / 3.0  # isothermal lattice temperature T = c_s^2


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIBPATH)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    u32p = C.POINTER(C.c_uint32)
    lib.orc_lattice.argtypes = [C.c_int, ip, ip, dp]
    lib.orc_stencil.argtypes = [C.c_int, C.c_int, ip, ip, dp]
    lib.orc_basis.argtypes = [C.c_int, dp, dp, ip]
    lib.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_normals.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_uint64, C.c_uint32, dp]
    lib.orc_normals.restype = None
    lib.orc_density.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp]
    lib.orc_force_from_psi.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.c_double, dp]
    lib.orc_noise_matrix.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, dp]
    lib.orc_step.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                             C.c_double, C.c_double, C.c_double, C.c_double,
                             C.c_uint64, C.c_uint32, C.c_int64, C.c_int64]
    lib.orc_conserved.argtypes = [dp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
    lib.orc_max_threads.argtypes = []
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops."""
    _load().orc_set_threads(int(n))


# --------------------------------------------------------------------------
# Parameters.
# --------------------------------------------------------------------------
def coupling_from_reduced_temperature(T_hat: float) -> float:
    """G of Eq. (1) for psi = exp(-1/n) at reduced temperature T/T_c.

    With psi = a exp(-b/n), the critical-point conditions give a = e sqrt(T_c n_c),
    b = n_c (Eq. 4).  psi = exp(-1/n) is b = 1 (n_c = 1) with G a^2 = G, so
    T_c = G / e^2; the lattice is isothermal at T = c_s^2 = 1/3, hence
    G = e^2 / (3 T_hat).
    """
    return math.e ** 2 * CS2 / T_hat


def lattice(D: int):
    lib = _load()
    Q = C.c_int()
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    assert lib.orc_lattice(D, C.byref(Q), c.ctypes.data_as(C.POINTER(C.c_int)), _dp(w)) == 0
    return c[: Q.value].copy(), w[: Q.value].copy()


def stencil(D: int, kind: int):
    lib = _load()
    nf = C.c_int()
    e = np.zeros((24, 3), dtype=np.int32)
    w = np.zeros(24)
    rc = lib.orc_stencil(D, kind, C.byref(nf), e.ctypes.data_as(C.POINTER(C.c_int)), _dp(w))
    if rc != 0:
        raise ValueError(f"no stencil E{kind} in {D}D")
    return e[: nf.value].copy(), w[: nf.value].copy()


def basis(D: int):
    lib = _load()
    Q = 9 if D == 2 else 19
    M = np.zeros((Q, Q))
    b = np.zeros(Q)
    cls = np.zeros(Q, dtype=np.int32)
    assert lib.orc_basis(D, _dp(M), _dp(b), cls.ctypes.data_as(C.POINTER(C.c_int))) == 0
    return M, b, cls


def philox4x32_10(ctr, key):
    lib = _load()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    out = (C.c_uint32 * 4)()
    lib.orc_philox4x32_10(c, k, out)
    return [int(v) for v in out]


def normals(D: int, node: int, step: int, seed: int, replica: int) -> np.ndarray:
    lib = _load()
    Q = 9 if D == 2 else 19
    xi = np.zeros(Q - D - 1)
    lib.orc_normals(D, int(node), int(step), C.c_uint64(seed), C.c_uint32(replica), _dp(xi))
    return xi


def noise_matrix(D: int, n: float, kBT: float, lam_bulk=1.0, lam_shear=1.0, lam_ghost=1.0):
    lib = _load()
    Q = 9 if D == 2 else 19
    B = np.zeros((Q, Q - D - 1))
    assert lib.orc_noise_matrix(D, n, kBT, lam_bulk, lam_shear, lam_ghost, _dp(B)) == 0
    return B


def _dims(f: np.ndarray):
    if f.ndim == 3:
        return 2, 1, f.shape[1], f.shape[2]
    return 3, f.shape[1], f.shape[2], f.shape[3]


def uniform_state(D: int, shape, rho0: float) -> np.ndarray:
    """f_i = w_i rho0: the homogeneous initial condition of the runs."""
    _, w = lattice(D)
    f = np.empty((len(w),) + tuple(shape))
    for i, wi in enumerate(w):
        f[i] = wi * rho0
    return f


def density(f: np.ndarray) -> np.ndarray:
    lib = _load()
    D, nz, ny, nx = _dims(f)
    f = np.ascontiguousarray(f, dtype=np.float64)
    n = np.zeros(f.shape[1:])
    assert lib.orc_density(_dp(f), D, nx, ny, nz, _dp(n)) == 0
    return n


def force_from_psi(psi: np.ndarray, kind: int, G: float) -> np.ndarray:
    lib = _load()
    D = psi.ndim
    if D == 2:
        nz, (ny, nx) = 1, psi.shape
    else:
        nz, ny, nx = psi.shape
    psi = np.ascontiguousarray(psi, dtype=np.float64)
    F = np.zeros((D,) + psi.shape)
    assert lib.orc_force_from_psi(_dp(psi), D, nx, ny, nz, kind, G, _dp(F)) == 0
    return F


def step(f: np.ndarray, nsteps: int, *, G: float, kind: int = 4, kBT: float = 0.0,
         lam_bulk: float = 1.0, lam_shear: float = 1.0, lam_ghost: float = 1.0,
         seed: int = 0, replica: int = 0, t0: int = 0) -> np.ndarray:
    """Advances a copy of the state f (time t0) by nsteps; returns it."""
    lib = _load()
    D, nz, ny, nx = _dims(f)
    out = np.array(f, dtype=np.float64, order="C", copy=True)
    rc = lib.orc_step(_dp(out), D, nx, ny, nz, kind, G, lam_bulk, lam_shear, lam_ghost, kBT,
                      C.c_uint64(seed), C.c_uint32(replica), int(t0), int(nsteps))
    if rc != 0:
        raise RuntimeError(f"orc_step failed ({rc})")
    return out


def conserved(f: np.ndarray):
    lib = _load()
    D, nz, ny, nx = _dims(f)
    f = np.ascontiguousarray(f, dtype=np.float64)
    mass = C.c_double()
    mom = np.zeros(3)
    assert lib.orc_conserved(_dp(f), D, nx, ny, nz, C.byref(mass), _dp(mom)) == 0
    return mass.value, mom[:D].copy()


# --------------------------------------------------------------------------
# Structure factor S(k) = <|dn(k)|^2>, the paper's measured quantity.
# Normalisation |sum_x dn(x) e^{-i k.x}|^2 / N (per-node variance, so that the
# exact result reads S = n0 kBT / c^2(k) as in Eq. (16)); k = 0 is excluded.
# --------------------------------------------------------------------------
def radial_bin(msq: int) -> int:
    """Shell index round(sqrt(msq)) of an integer squared mode number, exactly."""
    b = math.isqrt(msq)
    if msq - b * b > b:
        b += 1
    return b


def sk_bins(shape):
    """Axis and radial bin counts for a lattice of the given (.., ny, nx) shape."""
    D = len(shape)
    n_axis = max(shape) // 2 + 1
    n_rad = None
    if all(s == shape[0] for s in shape):
        n_rad = radial_bin(D * (shape[0] // 2) ** 2) + 1
    return D, n_axis, n_rad


def radial_bins_of(msq: np.ndarray) -> np.ndarray:
    """Vectorised radial_bin: integer shell index of squared mode numbers."""
    msq = np.asarray(msq, dtype=np.int64)
    b = np.floor(np.sqrt(msq.astype(np.float64))).astype(np.int64)
    b = np.where(b * b > msq, b - 1, b)            # exact integer square root
    b = np.where((b + 1) * (b + 1) <= msq, b + 1, b)
    return np.where(msq - b * b > b, b + 1, b)       # round to nearest (no ties)


def sk_sample(rho: np.ndarray):
    """One sample of P(k) = |dn(k)|^2/N, binned (k = 0 excluded).

    Returns dict(axis=(sum, sumsq, count), radial=(sum, sumsq, count) or None).
    axis arrays are [D][n_axis]: row d collects the modes +-m along axis d
    (d = 0 is x, the fastest array index); radial arrays are [n_rad], shell
    b = round(|m|) over all modes, and only exist when all sides are equal.
    """
    rho = np.asarray(rho, dtype=np.float64)
    D, n_axis, n_rad = sk_bins(rho.shape)
    N = rho.size
    dn = rho - rho.mean()
    P = np.abs(np.fft.fftn(dn)) ** 2 / N
    a_sum = np.zeros((D, n_axis))
    a_sq = np.zeros((D, n_axis))
    a_cnt = np.zeros((D, n_axis), dtype=np.int64)
    for d in range(D):
        ax = rho.ndim - 1 - d
        L = rho.shape[ax]
        for q in range(1, L):
            m = q if q <= L // 2 else L - q
            idx = [0] * rho.ndim
            idx[ax] = q
            v = P[tuple(idx)]
            a_sum[d, m] += v
            a_sq[d, m] += v * v
            a_cnt[d, m] += 1
    rad = None
    if n_rad is not None:
        L = rho.shape[0]
        q = np.arange(L)
        msigned = np.where(q <= L // 2, q, q - L).astype(np.int64)
        grids = np.meshgrid(*([msigned] * D), indexing="ij")
        msq = sum(g * g for g in grids).ravel()
        keep = msq > 0
        b = radial_bins_of(msq[keep])
        v = P.ravel()[keep]
        rad = (np.bincount(b, weights=v, minlength=n_rad),
               np.bincount(b, weights=v * v, minlength=n_rad),
               np.bincount(b, minlength=n_rad).astype(np.int64))
    return dict(axis=(a_sum, a_sq, a_cnt), radial=rad)


def domain_length(rho: np.ndarray) -> float:
    """L = 2 pi sum_k P(k) / sum_k |k| P(k) over k != 0 (|k| exact per mode):
    the inverse first moment of the structure factor, used as the domain size
    of a phase-separating field."""
    rho = np.asarray(rho, dtype=np.float64)
    P = np.abs(np.fft.fftn(rho - rho.mean())) ** 2 / rho.size
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(s) for s in rho.shape], indexing="ij")
    kabs = np.sqrt(sum(k * k for k in ks))
    mask = kabs > 0
    return float(2 * np.pi * P[mask].sum() / (kabs[mask] * P[mask]).sum())


def shell_means(rho: np.ndarray) -> np.ndarray:
    """Mean of P(k) over each radial shell b = round(|m|) (equal sides only)."""
    s = sk_sample(rho)["radial"]
    tot, _, cnt = s
    return np.where(cnt > 0, tot / np.maximum(cnt, 1), 0.0)
