"""Host estimators of paper_2212_07848_amd/dynamic.py on a process with a
known answer: a complex AR(1) sequence a(t+1) = r a(t) + noise has
C(tau) = C(0) r^tau and S(omega) = (1 - |r|^2) C(0) / |1 - r e^{-i omega}|^2."""
import math

import numpy as np
import pytest

from paper_2212_07848_amd import dynamic as DY


def _ar1(rng, r, T, R=8, D=2, nm=2, sigma=1.0):
    a = np.zeros((R, T, D, nm), dtype=complex)
    x = np.zeros((R, D, nm), dtype=complex)
    for t in range(T + 200):
        x = r * x + sigma * (rng.normal(size=x.shape) + 1j * rng.normal(size=x.shape)) / math.sqrt(2)
        if t >= 200:
            a[:, t - 200] = x
    return a


def test_correlation_of_ar1():
    rng = np.random.default_rng(0)
    r = 0.9 * np.exp(0.2j)
    a = _ar1(rng, r, 20000)
    C = DY.correlation(a, N=1.0, max_lag=10)
    C0 = 1.0 / (1.0 - abs(r) ** 2)
    for lag in range(11):
        assert abs(C[lag, 0] - C0 * r ** lag) < 0.05 * C0


def test_spectrum_of_ar1_and_its_normalisation():
    rng = np.random.default_rng(1)
    r = 0.8 * np.exp(0.5j)
    a = _ar1(rng, r, 40000)
    every = 3
    om, S = DY.spectrum(a, N=1.0, every=every, seg=128)
    C0 = 1.0 / (1.0 - abs(r) ** 2)
    # mean over the frequency grid is C(0) (Parseval)
    assert abs(np.mean(S[:, 0]) / every - C0) < 0.03 * C0
    # shape: AR(1) spectrum per sample, omega in radians per lattice step
    ws = om * every
    ref = every * (1 - abs(r) ** 2) * C0 / np.abs(1 - r * np.exp(-1j * ws)) ** 2
    mid = np.abs(ws - 0.5) < 1.0
    assert np.max(np.abs(S[mid, 0] / ref[mid] - 1)) < 0.15
    # the peak sits at the AR phase
    assert abs(ws[np.argmax(S[:, 0])] - 0.5) < 2 * math.pi / 128 * 1.5


def test_sound_frequency_small_k_is_the_sound_speed():
    k = 1e-4
    n0, T = 0.5, 0.9
    G = math.exp(2) / (3 * T)
    psi0 = math.exp(-1 / n0)
    c0 = math.sqrt(1 / 3 - G * psi0 * psi0 / n0 ** 2)
    assert DY.sound_frequency(np.array([k]), n0, T)[0] / k == pytest.approx(c0, rel=1e-6)
