"""Dynamic structure factor S(k, omega) of density fluctuations (the
frequency-resolved form behind Eq. 16: integrating it over omega gives the
static S(k)).

An ensemble of stationary replicas records, every `every` lattice steps, the
complex amplitudes dn^(k, t) = sum_x (n(x) - n0) e^{-i k.x} of the lowest
axis modes (fsc_modes_enable; the lattice work and the FFT are libfsc.so's).
From them:

  C(k, tau)   = < dn^(k, t + tau) dn^(k, t)* > / N,    tau = 0, every, ...
  S(k, omega) = every * sum_tau C(k, tau) e^{-i omega tau}  (omega per lattice step)

estimated by averaging over replicas, axes and time origins (C) or over
Hann-windowed segments (S, Welch).  The exact values of the linearised step
come from fsc_linear_corr; the spectrum has its sound peaks near
omega = +-c(k) k with c^2(k) = T - G psi0 psi0' h(k) (Eq. 15 generalised).
"""
from __future__ import annotations

import math

import numpy as np

from . import _lib as F
from .scaling import coupling, h_axis

CS2 = 1.0 / 3.0


def record(params, nm=4, every=2, burn=3000, samples=2000, stream=None):
    """Runs an ensemble of the given replicas (a list of fsc_params, usually
    one state with different replica ids) to `burn` steps, then records
    `samples` rows of the axis modes 1..nm every `every` steps.  Returns the
    amplitudes as complex [replica][sample][D][nm]."""
    ens = F.Ensemble(list(params), stream=stream)
    ens.init_uniform()
    ens.run(burn, 0)
    ens.modes_enable(nm, samples)
    ens.run(samples * every, every)
    amps = np.stack([ens.read_modes(r) for r in range(len(params))])
    ens.close()
    return amps


def correlation(amps, N, max_lag):
    """C(k, tau) for tau = 0..max_lag samples: mean over replicas, axes and
    time origins of a(t + tau) a(t)* / N; returns complex [max_lag + 1][nm]."""
    R, T, D, nm = amps.shape
    out = np.zeros((max_lag + 1, nm), dtype=complex)
    for lag in range(max_lag + 1):
        prod = amps[:, lag:] * np.conj(amps[:, :T - lag])
        out[lag] = prod.mean(axis=(0, 1, 2)) / N
    return out


def spectrum(amps, N, every, seg=256):
    """Welch estimate of S(k, omega): Hann-windowed segments of `seg` samples
    (half overlap), |FFT|^2 scaled so that the mean over frequencies is C(k, 0);
    returns (omega [seg] in radians per lattice step, centred, S [seg][nm])."""
    R, T, D, nm = amps.shape
    w = np.hanning(seg)
    norm = (w ** 2).sum()
    acc = np.zeros((seg, nm))
    cnt = 0
    for s0 in range(0, T - seg + 1, seg // 2):
        x = amps[:, s0:s0 + seg] * w[None, :, None, None]
        P = np.abs(np.fft.fft(x, axis=1)) ** 2
        acc += P.sum(axis=(0, 2))
        cnt += R * D
    S = acc / cnt / norm / N * every
    omega = np.fft.fftfreq(seg, d=every) * 2.0 * math.pi
    order = np.argsort(omega)
    return omega[order], S[order]


def theory_correlation(p, n, nm, lags_steps):
    """Exact C(k, tau) of the linearised step for the axis modes 1..nm of an
    n-sided lattice at the given lags (lattice steps); complex [nlag][nm]."""
    k = 2.0 * math.pi * np.arange(1, nm + 1) / n
    kv = np.zeros((nm, p.D))
    kv[:, 0] = k
    return F.linear_corr(p, kv, np.asarray(lags_steps, dtype=np.int32)).T


def theory_spectrum(p, n, nm, every, omega, max_lag_steps):
    """S(k, omega) of the linearised step sampled every `every` steps:
    every * [C(0) + 2 sum_{tau >= 1} Re C(tau) cos(omega tau)] over the lags
    tau = every, 2 every, ... up to max_lag_steps."""
    lags = np.arange(0, max_lag_steps + 1, every)
    C = theory_correlation(p, n, nm, lags)
    om = np.asarray(omega)[:, None]
    S = C[0].real[None, :] + 2.0 * np.sum(
        C[1:].real[None, :, :] * np.cos(om[:, :, None] * lags[1:][None, :, None]), axis=1)
    return S * every


def theory_welch(p, n, nm, every, seg):
    """Expected value of `spectrum`'s estimate under the exact linear C(k, tau):
    the Hann window's lag product r(j) = sum_t w(t) w(t + j) multiplies the
    correlation, so  E[S(omega)] = every / sum w^2 * sum_{|j| < seg} r(j) C(j every)
    e^{-i omega j every}.  Returns (omega, S) on `spectrum`'s grid."""
    w = np.hanning(seg)
    r = np.correlate(w, w, mode="full")[seg - 1:]  # r[j], j = 0..seg-1
    C = theory_correlation(p, n, nm, np.arange(seg) * every)  # [seg][nm]
    omega = np.sort(np.fft.fftfreq(seg, d=every) * 2.0 * math.pi)
    j = np.arange(1, seg)
    ph = np.exp(-1j * omega[:, None] * (j * every)[None, :])  # [omega][j]
    pos = (ph * r[1:][None, :]) @ C[1:]  # sum over j >= 1
    S = r[0] * C[0].real[None, :] + 2.0 * pos.real
    return omega, S * every / (w ** 2).sum()


def sound_frequency(k, n0, T_hat, stencil=4):
    """omega = c(k) k with c^2(k) = T - G psi0 psi0' h(k) along an axis."""
    G = coupling(T_hat)
    psi0 = math.exp(-1.0 / n0)
    c2 = CS2 - G * psi0 * psi0 / n0 ** 2 * h_axis(k, stencil)
    return np.sqrt(c2) * k
