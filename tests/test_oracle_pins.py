"""Pins of the FP64 oracle to things other than itself.

Each test checks the oracle against a published value, a closed form, an
invariant the paper states, a textbook special case, or brute force, chosen so
that a dropped term, a wrong sign, index or transposition fails one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import theory as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- generator --
def test_philox_known_answers():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    assert len(rows) == 3
    for r in rows:
        assert O.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


def test_normals_are_standard_gaussian():
    # The noise must be Gaussian with unit variance per draw (the paper's
    # random stress is Gaussian, uncorrelated in space and time).
    z = np.concatenate([O.normals(2, node, step, seed=3, replica=1)
                        for node in range(3000) for step in (0, 1)])
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 4.0 * math.sqrt(96.0 / n)
    # the uniform map keeps u in (0, 1): |z| <= sqrt(-2 ln 2^-24)
    assert np.all(np.abs(z) <= math.sqrt(-2.0 * math.log(2.0 ** -24)))
    # distinct streams for distinct (node, step, seed, replica)
    a = O.normals(3, 5, 9, seed=1, replica=0)
    assert a.shape == (15,)
    assert not np.allclose(a, O.normals(3, 5, 9, seed=1, replica=1))
    assert not np.allclose(a, O.normals(3, 5, 10, seed=1, replica=0))
    assert not np.allclose(a, O.normals(3, 6, 9, seed=1, replica=0))
    assert not np.allclose(a, O.normals(3, 5, 9, seed=1 + (1 << 32), replica=0))


# ------------------------------------------------------- stencils and basis --
@pytest.mark.parametrize("D,kind", [(2, 4), (2, 8), (3, 4)])
def test_stencil_is_isotropic_and_normalised(D, kind):
    e, w = O.stencil(D, kind)
    ex, ey = e[:, 0].astype(float), e[:, 1].astype(float)
    assert (w * ex ** 2).sum() == pytest.approx(1.0, abs=1e-15)        # Eq. (2)
    assert np.abs((w[:, None] * e).sum(axis=0)).max() < 1e-16          # no net force
    assert (w * ex ** 4).sum() == pytest.approx(3 * (w * ex ** 2 * ey ** 2).sum(), abs=1e-15)
    if kind == 8:
        assert (w * ex ** 6).sum() == pytest.approx(5 * (w * ex ** 4 * ey ** 2).sum(), abs=1e-15)
    assert len(w) == {(2, 4): 8, (2, 8): 24, (3, 4): 18}[(D, kind)]


@pytest.mark.parametrize("D", [2, 3])
def test_basis_is_weight_orthogonal_with_hydrodynamic_rows(D):
    c, w = O.lattice(D)
    M, b, cls = O.basis(D)
    Q = len(w)
    assert M.shape == (Q, Q)
    Gm = M @ np.diag(w) @ M.T
    assert np.abs(Gm - np.diag(np.diag(Gm))).max() < 1e-14
    assert np.allclose(np.diag(Gm), b, rtol=1e-14)
    assert np.linalg.matrix_rank(M) == Q
    assert np.allclose(M[0], 1.0)
    for d in range(D):
        assert np.allclose(M[1 + d], c[:, d])
    assert list(cls[: D + 1]) == [0] * (D + 1)
    # lattice isotropy of the weights: sum w = 1, sum w c c = 1/3 delta
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose((w[:, None, None] * c[:, :, None] * c[:, None, :]).sum(0),
                       np.eye(3)[: 3, : 3] * (1 / 3) * (np.arange(3) < D)[:, None], atol=1e-15)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("lam", [1.0, 0.6, 1.7])
def test_noise_covariance_is_the_fluctuation_dissipation_form(D, lam):
    # With one rate lam for all non-conserved moments the noise covariance of
    # the populations is basis free:
    #   mu n (1 - (1-lam)^2) [W - w w^T - sum_a (w c_a)(w c_a)^T / c_s^2]
    # (zero on mass and momentum, diagonal in any weight-orthogonal basis).
    c, w = O.lattice(D)
    n, kBT = 0.73, 2.5e-3
    B = O.noise_matrix(D, n, kBT, lam, lam, lam)
    cov = B @ B.T
    mu = kBT * 3.0
    expect = np.diag(w) - np.outer(w, w)
    for d in range(D):
        wc = w * c[:, d]
        expect -= 3.0 * np.outer(wc, wc)
    expect *= mu * n * (1.0 - (1.0 - lam) ** 2)
    assert np.abs(cov - expect).max() < 1e-15 * max(1.0, np.abs(expect).max()) * 50
    # mass and momentum of the noise vanish
    assert np.abs(B.sum(axis=0)).max() < 1e-16
    assert np.abs(c[:, :D].T @ B).max() < 1e-16


def test_noise_unequal_rates_diagonal_in_moments():
    D = 2
    M, b, cls = O.basis(D)
    B = O.noise_matrix(D, 1.1, 1e-3, 0.8, 1.3, 1.9)
    cm = M @ (B @ B.T) @ M.T
    lam = np.array([0, 0, 0, 0.8, 1.3, 1.3, 1.9, 1.9, 1.9])
    expect = 3e-3 * 1.1 * b * (1 - (1 - lam) ** 2)
    expect[:3] = 0
    assert np.allclose(cm, np.diag(expect), atol=1e-18, rtol=1e-12)


# ------------------------------------------------------------------ force ----
def _force_by_fft(psi, D, kind, G):
    """Eq. (1) by FFT convolution with the paper-cited weights."""
    E, W = T.stencil_set(D, kind)
    # array axes are (z,) y, x; offsets are (x, y[, z])
    shape = psi.shape
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(s) for s in shape], indexing="ij")
    kvec = ks[::-1]  # (kx, ky[, kz])
    ph = np.fft.fftn(psi)
    out = []
    for d in range(D):
        g = np.zeros(shape, dtype=complex)
        for e, wa in zip(E, W):
            g += wa * e[d] * np.exp(1j * sum(e[q] * kvec[q] for q in range(D)))
        out.append(G * psi * np.real(np.fft.ifftn(g * ph)))
    return np.array(out)


@pytest.mark.parametrize("D,kind,shape", [(2, 4, (8, 8)), (2, 8, (10, 12)), (2, 4, (5, 7)),
                                          (3, 4, (6, 5, 8))])
def test_force_matches_fft_convolution(D, kind, shape):
    rng = np.random.default_rng(11)
    psi = rng.uniform(0.05, 0.6, size=shape)
    F = O.force_from_psi(psi, kind, G=2.9)
    F2 = _force_by_fft(psi, D, kind, 2.9)
    assert np.abs(F - F2).max() < 1e-14


# ------------------------------------------------------ one deterministic step
def _bgk_guo_step(f, D, kind, G, lam):
    """Textbook population-space BGK with Guo forcing and periodic streaming
    (equal rates, no noise), with the force of Eq. (1) by FFT convolution."""
    c, w = (T.d2q9() if D == 2 else T.d3q19())
    n = f.sum(axis=0)
    psi = np.exp(-1.0 / n)
    F = _force_by_fft(psi, D, kind, G)
    sp = f.shape[1:]
    cc = [c[:, d].reshape((-1,) + (1,) * len(sp)) for d in range(D)]
    j = [(f * cc[d]).sum(axis=0) for d in range(D)]
    u = [(j[d] + 0.5 * F[d]) / n for d in range(D)]
    uu = sum(ud * ud for ud in u)
    cu = sum(cc[d] * u[d] for d in range(D))
    cF = sum(cc[d] * F[d] for d in range(D))
    uF = sum(u[d] * F[d] for d in range(D))
    wv = w.reshape((-1,) + (1,) * len(sp))
    feq = wv * n * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
    S = wv * (3 * (cF - uF) + 9 * cu * cF)
    fs = f - lam * (f - feq) + (1 - 0.5 * lam) * S
    out = np.empty_like(fs)
    for i in range(len(w)):
        shift = tuple(int(c[i, d]) for d in range(D))[::-1]
        out[i] = np.roll(fs[i], shift, axis=tuple(range(len(sp))))
    return out


@pytest.mark.parametrize("D,kind,shape", [(2, 4, (8, 8)), (2, 8, (9, 11)), (3, 4, (5, 6, 4))])
@pytest.mark.parametrize("lam", [1.0, 0.8, 1.6])
def test_moment_collision_equals_bgk_at_equal_rates(D, kind, shape, lam):
    rng = np.random.default_rng(5)
    c, w = O.lattice(D)
    rho = rng.uniform(0.4, 1.6, size=shape)
    f = np.array([wi * rho for wi in w]) * rng.uniform(0.8, 1.2, size=(len(w),) + shape)
    G = T.coupling(0.85)
    got = O.step(f, 1, G=G, kind=kind, kBT=0.0, lam_bulk=lam, lam_shear=lam, lam_ghost=lam)
    ref = _bgk_guo_step(f, D, kind, G, lam)
    assert np.abs(got - ref).max() < 1e-14


def test_rates_of_conserved_moments_do_not_matter_and_classes_act_separately():
    # m*_a = m_a - lam_a (m_a - m^eq_a) + ...: changing only the ghost rate must
    # change only the ghost content (no mass or momentum change).
    rng = np.random.default_rng(2)
    f = O.uniform_state(2, (6, 6), 0.9) * rng.uniform(0.9, 1.1, size=(9, 6, 6))
    G = T.coupling(0.9)
    a = O.step(f, 1, G=G, lam_ghost=1.0)
    b = O.step(f, 1, G=G, lam_ghost=0.5)
    assert not np.allclose(a, b)
    ma, pa = O.conserved(a)
    mb, pb = O.conserved(b)
    assert ma == pytest.approx(mb, rel=1e-15)
    assert np.allclose(pa, pb, atol=1e-15)


# ------------------------------------------------------------- invariants ----
@pytest.mark.parametrize("D,shape,kind", [(2, (64, 64), 4), (2, (24, 40), 8), (3, (10, 12, 8), 4)])
def test_mass_and_momentum_conserved_with_noise(D, shape, kind):
    G = T.coupling(0.9)
    f0 = O.uniform_state(D, shape, 0.5)
    m0, p0 = O.conserved(f0)
    f = O.step(f0, 300, G=G, kind=kind, kBT=1e-4, seed=0)
    m1, p1 = O.conserved(f)
    assert abs(m1 - m0) / m0 < 1e-12
    assert np.abs(p1).max() / m0 < 1e-13
    # and the noise did act
    assert np.std(O.density(f)) > 1e-4


@pytest.mark.parametrize("T_hat,n0,kind", [(0.9, 0.5, 4), (0.7, 1.0, 8), (0.7, 1.0, 4)])
def test_noise_free_flat_state_stays_flat(T_hat, n0, kind):
    # Homogeneous densities are stationary without noise, even inside the
    # unstable region (n0 = 1 at T_hat = 0.7).
    f0 = O.uniform_state(2, (16, 16), n0)
    f = O.step(f0, 200, G=T.coupling(T_hat), kind=kind, kBT=0.0)
    assert np.abs(f - f0).max() < 1e-14


def test_unstable_state_phase_separates_with_noise():
    # Spinodal decomposition: inside the unstable region tiny noise grows.
    f0 = O.uniform_state(2, (32, 32), 1.0)
    f = O.step(f0, 400, G=T.coupling(0.7), kind=4, kBT=1e-10)
    n = O.density(f)
    assert n.max() - n.min() > 0.1


@pytest.mark.parametrize("T_hat,tol", [(0.9, 2e-5), (0.8, 1e-3)])
def test_flat_interface_coexistence_matches_maxwell(T_hat, tol):
    # Noise-free flat liquid slab in gas: the bulk densities relax to the
    # coexistence densities of the EoS, Eq. (2) (equal areas in 1/n because
    # psi = exp(-1/n)); lattice corrections grow as T_hat drops.  The lattice
    # normal pressure, Eq. (14), is constant through the interface.
    G = T.coupling(T_hat)
    ng, nl, _ = T.binodal(T_hat)
    nx = 96
    rho = np.full((1, nx), ng)
    rho[:, nx // 4: 3 * nx // 4] = nl
    c, w = O.lattice(2)
    f = np.array([wi * rho for wi in w])
    f = O.step(f, 16000, G=G)
    n = O.density(f)[0]
    assert abs(n[0] / ng - 1) < tol
    assert abs(n[nx // 2] / nl - 1) < tol
    psi = np.exp(-1.0 / n)
    PN = n / 3.0 - 0.25 * G * psi * (np.roll(psi, 1) + np.roll(psi, -1))
    assert (PN.max() - PN.min()) / PN.mean() < 10 * tol
    # the normal pressure is the bulk pressure of Eq. (2) in the bulk
    p_bulk = ng / 3.0 - 0.5 * G * math.exp(-2.0 / ng)
    assert PN.mean() == pytest.approx(p_bulk, rel=10 * tol)


# ----------------------------------------------------- structure factor -----
def test_sk_sample_normalisation_and_bins():
    # White noise of variance s2 has E[|dn(k)|^2]/N = s2 (k != 0).
    rng = np.random.default_rng(4)
    acc = None
    for _ in range(200):
        s = O.sk_sample(rng.normal(0.0, 0.3, size=(16, 16)))
        a_sum, _, a_cnt = s["axis"]
        r_sum, _, r_cnt = s["radial"]
        acc = (a_sum, r_sum) if acc is None else (acc[0] + a_sum, acc[1] + r_sum)
    assert a_cnt[0, 1] == 2 and a_cnt[0, 8] == 1 and a_cnt[0, 0] == 0
    assert r_cnt.sum() == 255 and r_cnt[0] == 0
    mean_ax = acc[0][:, 1:].sum() / (200 * a_cnt[:, 1:].sum())
    mean_rad = acc[1].sum() / (200 * 255)
    assert mean_ax == pytest.approx(0.09, rel=0.1)
    assert mean_rad == pytest.approx(0.09 * 256 / 255, rel=0.03)
    # brute-force DFT of one mode
    x = rng.normal(size=(6, 10))
    s = O.sk_sample(x)
    dn = x - x.mean()
    k = 2 * math.pi * 3 / 10
    X = sum(dn[y, xx] * np.exp(-1j * k * xx) for y in range(6) for xx in range(10))
    assert s["axis"][0][0, 3] == pytest.approx(2 * abs(X) ** 2 / 60, rel=1e-12)


def test_radial_bin_rule_is_exact_rounding():
    assert O.radial_bin(0) == 0
    for m in range(1, 5000):
        b = O.radial_bin(m)
        assert (b - 0.5) ** 2 <= m < (b + 0.5) ** 2
    assert np.array_equal(O.radial_bins_of(np.arange(5000)),
                          np.array([O.radial_bin(m) for m in range(5000)]))


def _mc_axis_sk(L, T_hat, n0, kBT, G=None, nsamp=800, every=10, seed=7):
    G = T.coupling(T_hat) if G is None else G
    f = O.uniform_state(2, (L, L), n0)
    out = []
    t = 0
    for _ in range(nsamp):
        f = O.step(f, every, G=G, kBT=kBT, seed=seed, t0=t)
        t += every
        a_sum, _, a_cnt = O.sk_sample(O.density(f))["axis"]
        out.append(a_sum.sum(axis=0) / np.maximum(a_cnt.sum(axis=0), 1))
    return np.array(out), G, every * np.arange(1, nsamp + 1)


@pytest.mark.slow
@pytest.mark.parametrize("T_hat,n0,G", [(0.9, 0.5, None), (0.9, 2.0, None), (None, 0.7, 0.0)])
def test_oracle_sk_matches_exact_linear_theory(T_hat, n0, G):
    # The measured S(k) agrees with the exact linear expectation at the
    # sampled times (which tends to Eq. (16)) within the statistical error,
    # estimated by batch means.  k_B theta is small so the linear theory holds.
    L, kBT = 32, 1e-6
    S, G, times = _mc_axis_sk(L, T_hat, n0, kBT, G=G)
    z = []
    for m in range(1, L // 2 + 1):
        k = 2 * math.pi * m / L
        th = T.sk_linear_times([k, 0.0], times, D=2, kind=4, n0=n0, G=G, kBT=kBT).mean()
        batches = S[:, m].reshape(40, -1).mean(axis=1)
        err = batches.std(ddof=1) / math.sqrt(len(batches))
        z.append((S[:, m].mean() - th) / err)
        assert abs(S[:, m].mean() / th - 1) < 0.12
    z = np.array(z)
    assert np.all(np.abs(z) < 4.0), z
    assert np.mean(z ** 2) < 2.5, z


def test_domain_length_of_single_modes():
    # a field made of one wave vector k0 (and its conjugate) has L = 2 pi/|k0|
    for shape, m in [((32, 32), (3, 0)), ((32, 32), (2, 5)), ((16, 16, 16), (1, 2, 2))]:
        grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
        k = [2 * np.pi * mm / s for mm, s in zip(m, shape)]
        rho = 1.0 + 0.1 * np.cos(sum(kk * g for kk, g in zip(k, grids)))
        assert O.domain_length(rho) == pytest.approx(2 * np.pi / np.sqrt(sum(kk * kk for kk in k)),
                                                     rel=1e-12)
    # two equal-power modes: the harmonic mean of their lengths
    g = np.arange(64)
    rho = np.cos(2 * np.pi * 2 * g / 64)[None, :] + np.cos(2 * np.pi * 8 * g / 64)[:, None]
    k1, k2 = 2 * np.pi * 2 / 64, 2 * np.pi * 8 / 64
    assert O.domain_length(rho) == pytest.approx(2 * np.pi * 2 / (k1 + k2), rel=1e-12)
