"""The exact linear S(k) routine (fsc_linear_sk) against the oracle's own
per-k covariance (its Lyapunov doubling, written separately), against the
closed form of Eq. 16 on the axes, against brute force over every mode of
small lattices for the radial shells, and the lattice's measured 3D radial
S(k) against it."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import theory as T

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")


def _p(D, stencil, T_hat, rho0, kBT, lam=(1, 1, 1), n=16):
    return fsc.make_params(D=D, nx=n, ny=n, nz=n if D == 3 else 1, stencil=stencil, T_hat=T_hat,
                           rho0=rho0, kBT=kBT, lam=lam)


@pytest.mark.parametrize("D,stencil", [(2, 4), (2, 8), (3, 4)])
@pytest.mark.parametrize("lam", [(1.0, 1.0, 1.0), (0.8, 1.3, 1.7)])
def test_random_wave_vectors_match_the_oracle(D, stencil, lam):
    rng = np.random.default_rng(D * 10 + stencil)
    kv = rng.uniform(-math.pi, math.pi, size=(24, D))
    for T_hat, n0 in ((0.9, 0.5), (0.8, 2.2)):
        p = _p(D, stencil, T_hat, n0, 1e-4, lam)
        got = fsc.linear_sk(p, kv)
        ref = np.array([T.sk_linear_stationary(k, D=D, kind=stencil, n0=n0,
                                               G=T.coupling(T_hat), kBT=1e-4, lam=lam) for k in kv])
        assert np.allclose(got, ref, rtol=1e-9, atol=0), np.max(np.abs(got / ref - 1))


@pytest.mark.parametrize("D,stencil", [(2, 4), (2, 8), (3, 4)])
def test_axis_values_are_eq16(D, stencil):
    k = 2 * np.pi * np.arange(1, 33) / 64
    kv = np.zeros((len(k), D))
    kv[:, 0] = k
    for T_hat, n0 in ((0.9, 0.5), (0.8, 0.62), (0.95, 1.6)):
        got = fsc.linear_sk(_p(D, stencil, T_hat, n0, 1e-13), kv)
        ref = T.sk_exact_axis(k, n0, T.coupling(T_hat), 1e-13, D=D, kind=stencil)
        assert np.allclose(got, ref, rtol=1e-9, atol=0)


@pytest.mark.parametrize("D,n", [(2, 20), (3, 8)])
def test_radial_shells_match_brute_force(D, n):
    p = _p(D, 4, 0.85, 0.55, 1e-4, n=n)
    nb = O.radial_bin(D * (n // 2) ** 2) + 1
    mean, cnt = fsc.linear_sk_radial(p, nb)
    # every mode of the lattice, one by one
    m = np.arange(n)
    m = np.where(m > n // 2, m - n, m)
    grids = np.meshgrid(*([m] * D), indexing="ij")
    modes = np.stack([g.ravel() for g in grids], axis=1)
    modes = modes[np.any(modes != 0, axis=1)]
    S = fsc.linear_sk(p, 2 * np.pi * modes / n)
    b = O.radial_bins_of((modes ** 2).sum(axis=1))
    ref = np.bincount(b, weights=S, minlength=nb)[:nb] / np.maximum(np.bincount(b, minlength=nb)[:nb], 1)
    assert np.array_equal(cnt, np.bincount(b, minlength=nb)[:nb])
    assert np.allclose(mean, ref, rtol=1e-11, atol=0)
    # and a few modes through the oracle directly
    for i in range(0, len(modes), max(1, len(modes) // 7)):
        r = T.sk_linear_stationary(2 * np.pi * modes[i] / n, D=D, kind=4, n0=0.55,
                                   G=T.coupling(0.85), kBT=1e-4)
        assert S[i] == pytest.approx(r, rel=1e-9)


def test_measured_3d_radial_structure_factor_matches_the_linear_theory():
    # metastable gas at T_hat = 0.8 (between binodal 0.431 and spinodal 0.645)
    n, nrep, T_hat, n0, kBT = 24, 16, 0.8, 0.55, 1e-13
    plist = [fsc.make_params(D=3, nx=n, ny=n, nz=n, stencil=4, precision="fp32", T_hat=T_hat,
                             rho0=n0, kBT=kBT, seed=31, replica=r) for r in range(nrep)]
    ens = fsc.Ensemble(plist)
    ens.init_uniform()
    ens.run(3000, 0)
    ens.sk_reset()
    ens.run(12000, 40)
    tot = cnt = None
    for r in range(nrep):
        s, _, c = ens.read_sk(r, fsc.FSC_SK_RADIAL)
        tot = s if tot is None else tot + s
        cnt = c if cnt is None else cnt + c
    ens.close()
    meas = tot / np.maximum(cnt, 1)
    nb = len(meas)
    theory, _ = fsc.linear_sk_radial(plist[0], nb)
    rel = meas[1:] / theory[1:] - 1
    print("relative deviation per shell", np.round(rel, 4))
    assert np.max(np.abs(rel)) < 0.05
    assert abs(np.mean(rel)) < 0.01
