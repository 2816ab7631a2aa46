"""Recorded mode amplitudes and the dynamic structure factor on the GPU:
the recorder against a direct FFT of the density, the exact correlation
routine against the oracle's linear operator, and the measured C(k, tau)
and S(k, omega) against the exact linear values."""
import math

import numpy as np
import pytest

import fsc_inputs as I
import oracle as O
from oracle import theory as T

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
from paper_2212_07848_amd import dynamic as DY  # noqa: E402


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 2e-5)])
def test_recorder_matches_the_fft_of_the_density(precision, tol):
    ny, nx, nm = 24, 40, 5
    p = fsc.make_params(D=2, nx=nx, ny=ny, stencil=4, precision=precision, T_hat=0.9, rho0=0.5,
                        kBT=1e-4, seed=3)
    f = I.smooth_density_populations(9, (ny, nx), 0.5, 0.05, 4, seed=9)
    with fsc.Lattice(p) as lat:
        lat.set_populations(f, 0)
        lat.modes_enable(nm, 8)
        ref = []
        for _ in range(6):
            lat.measure_sk()
            d = np.fft.fft2(lat.density() - 0.5)
            ref.append(np.stack([d[0, 1:nm + 1], d[1:nm + 1, 0]]))
            lat.step(3)
        got = lat.read_modes()
    ref = np.array(ref)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("D,stencil", [(2, 4), (2, 8), (3, 4)])
def test_linear_correlation_matches_the_oracle(D, stencil):
    rng = np.random.default_rng(5)
    kv = rng.uniform(-math.pi, math.pi, size=(6, D))
    lags = [0, 1, 2, 5, 17, 60]
    lam = (0.9, 1.2, 1.5)
    p = fsc.make_params(D=D, nx=8, ny=8, nz=8 if D == 3 else 1, stencil=stencil, T_hat=0.85,
                        rho0=0.55, kBT=1e-4, lam=lam)
    got = fsc.linear_corr(p, kv, lags)
    for i, k in enumerate(kv):
        A, Qn = T.linear_operator(k, D=D, kind=stencil, n0=0.55, G=T.coupling(0.85), kBT=1e-4,
                                  lam=lam)
        X, Ak = Qn.copy(), A.copy()
        for _ in range(48):
            X = X + Ak @ X @ Ak.conj().T
            Ak = Ak @ Ak
        one = np.ones(A.shape[0])
        v = X @ one
        ref = []
        t = 0
        for lag in lags:
            while t < lag:
                v = A @ v
                t += 1
            ref.append(one @ v)
        ref = np.array(ref)
        assert np.max(np.abs(got[i] - ref)) < 1e-9 * abs(ref[0])
        assert np.max(np.abs(got[i].imag)) < 1e-9 * abs(ref[0])  # real by parity


def test_measured_correlation_and_spectrum_match_the_linear_theory():
    n, nm, every, R = 64, 3, 2, 32
    plist = [fsc.make_params(D=2, nx=n, ny=n, stencil=4, precision="fp32", T_hat=0.9, rho0=0.5,
                             kBT=1e-4, seed=21, replica=r) for r in range(R)]
    amps = DY.record(plist, nm=nm, every=every, burn=3000, samples=3000)
    N = n * n
    max_lag = 150  # samples = 300 steps
    C = DY.correlation(amps, N, max_lag)
    Cth = DY.theory_correlation(plist[0], n, nm, np.arange(0, max_lag + 1) * every)
    rho = C.real / C[0].real
    rho_th = Cth.real / Cth[0].real
    print("C(0) measured / exact", C[0].real / Cth[0].real)
    print("max |rho - rho_exact|", np.max(np.abs(rho - rho_th), axis=0))
    assert np.all(np.abs(C[0].real / Cth[0].real - 1) < 0.05)
    assert np.max(np.abs(rho - rho_th)) < 0.08
    # the spectrum: peaks at the sound frequency of each mode
    om, S = DY.spectrum(amps, N, every, seg=512)
    k = 2 * math.pi * np.arange(1, nm + 1) / n
    wB = DY.sound_frequency(k, 0.5, 0.9)
    dw = 2 * math.pi / (512 * every)
    for m in range(nm):
        pos = om > 0
        peak = om[pos][np.argmax(S[pos, m])]
        print("mode", m + 1, "peak", peak, "sound", wB[m])
        assert abs(peak - wB[m]) < 2.5 * dw
    # the whole estimate against its exact expectation under the linear theory
    om2, Sexp = DY.theory_welch(plist[0], n, nm, every, 512)
    assert np.allclose(om2, om)
    band = Sexp > 0.2 * Sexp.max(axis=0)
    rel = np.abs(S - Sexp) / Sexp
    print("band max rel", [float(rel[band[:, m], m].max()) for m in range(nm)],
          "band sum rel", (S * band).sum(0) / (Sexp * band).sum(0) - 1)
    assert np.all(np.abs((S * band).sum(0) / (Sexp * band).sum(0) - 1) < 0.06)
    assert max(rel[band[:, m], m].max() for m in range(nm)) < 0.35
    # normalisation: integrated over a frequency grid fine enough that no lag
    # aliases, the spectrum gives back C(k, 0)
    M = 8192
    omf = np.fft.fftfreq(M, d=every) * 2.0 * math.pi
    Sth = DY.theory_spectrum(plist[0], n, nm, every, omf, 6000)
    assert np.allclose(Sth.sum(axis=0) / (M * every), Cth[0].real, rtol=1e-9)
