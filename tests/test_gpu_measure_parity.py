"""Parity of the measurement rows with the FP64 oracle, through the C ABI.

- The batched S(k) sample of an ensemble of uneven replicas (power-of-two
  sides on the FFT path, a ragged replica on the DFT path, a flat replica that
  only carries noise), element by element per bin, in the single-step and the
  two-step tilings, eager and replayed from captured graphs.
- The FP64 reductions (mass, momentum, density range, the count of bad nodes)
  against the oracle's sums of the same state, and the divergence report of a
  state holding a non-finite and a non-positive density.
- The thermal-noise increment of steps at k_B theta = 1e-13 (the metastable
  workloads' noise, Eq. 12), which is too small to show in population parity.

Tolerances: S(k) bins rtol 1e-4 (FP32) / 1e-10 (FP64) per bin, with a floor of
a millionth of the mean bin; reductions 1e-6 (FP32) / 1e-12 (FP64) of the
total mass; the noise increment within 1e-3 of the oracle's, relative to its
largest element.
"""
import ctypes

import numpy as np
import pytest

import fsc_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")

from test_gpu_parity import assert_bins_close, assert_pop_close  # noqa: E402


def _p(shape, precision, *, T_hat, rho0, kBT, replica, seed=31, lam=(1.0, 1.0, 1.0), stencil=4):
    if len(shape) == 2:
        (ny, nx), nz, D = shape, 1, 2
    else:
        (nz, ny, nx), D = shape, 3
    return fsc.make_params(D=D, nx=nx, ny=ny, nz=nz, stencil=stencil, precision=precision,
                           T_hat=T_hat, rho0=rho0, lam=lam, kBT=kBT, seed=seed, replica=replica)


# replica specs: (shape, T_hat, rho0, random start?)
MIXED_2D = [((128, 128), 0.9, 0.5, True), ((256, 256), 0.8, 2.0, True),
            ((512, 512), 0.85, 0.7, True), ((136, 200), 0.95, 0.8, True),
            ((256, 256), 0.9, 0.5, False)]
MIXED_3D = [((16, 16, 16), 0.9, 0.5, True), ((24, 24, 24), 0.8, 0.62, True),
            ((9, 10, 12), 0.95, 1.2, True), ((16, 16, 16), 0.9, 1.8, False)]


def _oracle_bins(f0, p, G, nsteps, every, lam):
    """Sum over the samples after every `every` steps of the oracle's bins."""
    acc = None
    f = f0
    t = 0
    while t < nsteps:
        f = O.step(f, every, G=G, kind=p.stencil, kBT=p.kBT, lam_bulk=lam[0], lam_shear=lam[1],
                   lam_ghost=lam[2], seed=p.seed, replica=p.replica, t0=t)
        t += every
        s = O.sk_sample(O.density(f))
        if acc is None:
            acc = s
        else:
            acc = dict(axis=tuple(a + b for a, b in zip(acc["axis"], s["axis"])),
                       radial=None if s["radial"] is None else
                       tuple(a + b for a, b in zip(acc["radial"], s["radial"])))
    return acc


@pytest.mark.parametrize("D,precision,tiling", [(2, "fp32", None), (2, "fp32", (256, 1, 1, 2)),
                                                (2, "fp64", None), (3, "fp32", None),
                                                (3, "fp64", None)])
def test_mixed_ensemble_sk_matches_oracle_per_bin(D, precision, tiling):
    specs = MIXED_2D if D == 2 else MIXED_3D
    lam = (0.9, 1.2, 1.5)
    Q = 9 if D == 2 else 19
    plist = [_p(sh, precision, T_hat=th, rho0=r0, kBT=1e-4, replica=k, lam=lam)
             for k, (sh, th, r0, _) in enumerate(specs)]
    ens = fsc.Ensemble(plist)
    ens.init_uniform()
    f0 = {}
    for k, (sh, th, r0, rnd) in enumerate(specs):
        f0[k] = (I.random_populations(Q, sh, r0, 0.3, seed=60 + k) if rnd
                 else O.uniform_state(D, sh, r0))
        if rnd:
            ens.set_populations(k, f0[k])
    nsteps, every = 4, 2
    if tiling is not None:
        # two steps per launch: a graph chunk holds an even number of launches,
        # so 8 steps with a sample every 2 replay two chunks of four steps
        ens.set_tiling(*tiling, target_blocks=256)
        nsteps = 8
    ens.run(nsteps, every)
    print("tiling", ens.tiling, flush=True)
    worst = 0.0
    for k, (sh, th, r0, rnd) in enumerate(specs):
        G = O.coupling_from_reduced_temperature(th)
        ref = _oracle_bins(f0[k], plist[k], G, nsteps, every, lam)
        s, q, c = ens.read_sk(k, fsc.FSC_SK_AXIS)
        rs, rq, rc = ref["axis"]
        assert np.array_equal(c, rc), k
        worst = max(worst, assert_bins_close(s, rs, precision))
        assert_bins_close(q, rq, precision, factor=2.0)
        rad = ens.read_sk(k, fsc.FSC_SK_RADIAL)
        if ref["radial"] is None:
            assert rad[0].size == 0
        else:
            rs, rq, rc = ref["radial"]
            assert np.array_equal(rad[2], rc), k
            worst = max(worst, assert_bins_close(rad[0], rs, precision))
            assert_bins_close(rad[1], rq, precision, factor=2.0)
    print(f"D={D} {precision} {tiling}: worst relative bin error {worst:.2e}")
    ens.close()


# ------------------------------------------------------------ reductions -----
@pytest.mark.parametrize("D,shape", [(2, (37, 150)), (2, (256, 256)), (3, (9, 17, 40))])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_stats_match_oracle_sums(D, shape, precision):
    Q = 9 if D == 2 else 19
    rho0 = 0.8
    f = I.random_populations(Q, shape, rho0, 0.3, seed=77)
    # a population field with nonzero momentum and a wide density range
    c, _ = O.lattice(D)
    f = f * (1.0 + 0.2 * c[:, 0].reshape((-1,) + (1,) * D))
    with fsc.Lattice(_p(shape, precision, T_hat=0.9, rho0=rho0, kBT=0.0, replica=0)) as lat:
        lat.set_populations(f, 5)
        st = lat.stats()
        # the boundary's names for the same reductions and the density read
        m2, p2 = lat.conserved()
        assert m2 == st["mass"] and np.array_equal(p2, st["mom"])
        rho_a = lat.density()
        rho_b = np.empty(shape)
        assert fsc.lib().fsc_read_density(
            lat._h, rho_b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
        assert np.array_equal(rho_a, rho_b)
    mass, mom = O.conserved(f)
    rho = O.density(f)
    tol = 1e-6 if precision == "fp32" else 1e-12
    assert abs(st["mass"] - mass) <= tol * mass
    assert np.abs(st["mom"] - mom).max() <= tol * mass
    assert abs(st["rho_min"] - rho.min()) <= tol * rho.min()
    assert abs(st["rho_max"] - rho.max()) <= tol * rho.max()
    assert st["bad"] == 0 and st["nodes"] == rho.size


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_divergence_is_reported(precision):
    D, shape, rho0 = 2, (20, 33), 0.6
    f = I.random_populations(9, shape, rho0, 0.2, seed=3)
    f[4, 7, 11] = np.nan                   # a non-finite density at (x 11, y 7)
    _, w = O.lattice(D)
    f[:, 15, 2] = -0.1 * w                 # a negative density at (x 2, y 15)
    rho = O.density(np.where(np.isnan(f), 0.0, f))
    good = np.ones(shape, dtype=bool)
    good[7, 11] = False
    with fsc.Lattice(_p(shape, precision, T_hat=0.9, rho0=rho0, kBT=1e-4, replica=0)) as lat:
        lat.set_populations(f, 0)
        with pytest.raises(fsc.FscError) as ei:
            lat.stats()
        assert ei.value.code == -4
        st = lat.stats(allow_diverged=True)
        assert st["bad"] == 2 and st["nodes"] == rho.size
        assert np.isnan(st["mass"])
        # the density range skips the non-finite node and shows the negative one
        tol = 1e-6 if precision == "fp32" else 1e-12
        assert st["rho_min"] == pytest.approx(rho[good].min(), abs=tol)
        assert st["rho_max"] == pytest.approx(rho[good].max(), rel=tol)
        # stepping carries the bad nodes on; the report stays
        lat.step(3)
        st = lat.stats(allow_diverged=True)
        assert st["bad"] >= 2
    # in an ensemble only the replica that diverged reports it
    plist = [_p((16, 16), precision, T_hat=0.9, rho0=0.5, kBT=1e-4, replica=r) for r in range(3)]
    ens = fsc.Ensemble(plist)
    ens.init_uniform()
    g = O.uniform_state(2, (16, 16), 0.5)
    g[0, 3, 3] = np.inf
    ens.set_populations(1, g)
    assert ens.stats(0)["bad"] == 0 and ens.stats(2)["bad"] == 0
    with pytest.raises(fsc.FscError) as ei:
        ens.stats(1)
    assert ei.value.code == -4
    assert ens.stats(1, allow_diverged=True)["bad"] == 1
    ens.close()


# ----------------------------------------------------------- noise size -----
def _increment_check(got, f0, nsteps, G, kind, kBT, seed, replica, t0, D, rho0, precision):
    """The state minus the noise-free oracle step equals the oracle's noise
    increment (noisy minus noise-free) to 1e-3 of its largest element."""
    ref = O.step(f0, nsteps, G=G, kind=kind, kBT=kBT, seed=seed, replica=replica, t0=t0)
    quiet = O.step(f0, nsteps, G=G, kind=kind, kBT=0.0, seed=seed, replica=replica, t0=t0)
    assert_pop_close(got, ref, D, rho0, precision)
    inc_ref = ref - quiet
    inc_got = got - quiet
    scale = np.abs(inc_ref).max()
    assert scale > 0
    err = np.abs(inc_got - inc_ref).max() / scale
    rms = np.sqrt(np.mean((inc_got - inc_ref) ** 2) / np.mean(inc_ref ** 2))
    print(f"noise increment: max |d| / max |inc| = {err:.2e}, rms ratio {rms:.2e}")
    return err, rms


def test_noise_increment_at_metastable_kbt_2d_ensemble():
    # the bench ensemble's noise (k_B theta = 1e-13) on a flat replica of each
    # side, in the ensemble's autotuned launch: the populations after two steps
    # carry nothing but the noise, which must be the oracle's
    reps = I.ensemble_replicas(n=64, seed=0, kBT=1e-13)
    plist = [fsc.make_params(**{k: v for k, v in r.items() if k != "precision"}, precision="fp32")
             for r in reps]
    ens = fsc.Ensemble(plist)
    ens.init_uniform()
    ens.autotune()
    ens.run(2, 0)
    for side in (128, 256, 512):
        k = next(r for r, rep in enumerate(reps) if rep["nx"] == side)
        rf = reps[k]
        f0 = O.uniform_state(2, (rf["ny"], rf["nx"]), rf["rho0"])
        err, _ = _increment_check(ens.get_populations(k), f0, 2,
                                  O.coupling_from_reduced_temperature(rf["T_hat"]), 4,
                                  rf["kBT"], 0, k, 0, 2, rf["rho0"], "fp32")
        assert err <= 1e-3
    ens.close()


@pytest.mark.parametrize("start", ["flat", "random"])
def test_noise_increment_at_metastable_kbt_3d(start):
    c = I.METASTABLE_3D
    shape = (40, 36, 70)  # the 3D metastable state point on a smaller, ragged box
    f0 = O.uniform_state(3, shape, c["rho0"])
    if start == "random":
        # near-equilibrium populations, 2% off w_i n0 node by node
        f0 = f0 * (1.0 + 0.02 * np.random.default_rng(8).uniform(-1, 1, size=f0.shape))
    with fsc.Lattice(_p(shape, "fp32", T_hat=c["T_hat"], rho0=c["rho0"], kBT=c["kBT"],
                        replica=0, seed=c["seed"])) as lat:
        lat.set_populations(f0, 900)
        lat.step(1)
        got = lat.get_populations()
        G = lat.G
    err, rms = _increment_check(got, f0, 1, G, 4, c["kBT"], c["seed"], 0, 900, 3, c["rho0"],
                                "fp32")
    if start == "flat":
        assert err <= 1e-3
    else:
        # FP32 storage rounds deviations of ~2e-2 w_i n0 to ~1e-11, a few parts
        # in 1e4 of the noise at 1e-13 (the CPU emulation of that rounding
        # gives 2e-4 max, 1e-4 rms)
        assert err <= 2e-3 and rms <= 1e-3


# --------------------------------------------------- the small workload -----
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_workload_sk_series_matches_oracle_and_linear_theory(precision):
    # 64^2 D2Q9 E4, T_hat 0.9, n0 0.5, kBT 1e-4, seed 0: 1000 steps with an axis
    # S(k) sample every 10 steps, as configured.  The accumulated bins equal the
    # oracle's own trajectory sampled alike (the run is stable, so the two
    # trajectories stay within the population tolerance), and the sample mean
    # of each axis mode agrees with the exact linear expectation at the sampled
    # times (Eq. 16 in the limit) within its statistical error.
    from oracle import theory as T
    c = I.SMALL_PARITY
    L, every, steps = c["nx"], c["sk_every"], c["steps"]
    p = _p((c["ny"], c["nx"]), precision, T_hat=c["T_hat"], rho0=c["rho0"], kBT=c["kBT"],
           replica=0, seed=c["seed"])
    with fsc.Lattice(p) as lat:
        lat.init_uniform()
        lat.run(steps, every)
        s, q, cnt = lat.read_sk(fsc.FSC_SK_AXIS)
        G = lat.G
    f = O.uniform_state(2, (c["ny"], c["nx"]), c["rho0"])
    ref_s = np.zeros_like(s)
    ref_c = np.zeros_like(cnt)
    for k in range(steps // every):
        f = O.step(f, every, G=G, kind=c["stencil"], kBT=c["kBT"], seed=c["seed"], t0=k * every)
        a_sum, _, a_cnt = O.sk_sample(O.density(f))["axis"]
        ref_s[:, : a_sum.shape[1]] += a_sum
        ref_c[:, : a_cnt.shape[1]] += a_cnt
    assert np.array_equal(cnt, ref_c)
    # the populations agree to 1e-11 (FP64) / 1e-5 (FP32) relative; P(k) of a
    # fluctuation field carries twice that relative error, more on low bins
    rtol = 1e-8 if precision == "fp64" else 5e-3
    nz = ref_s > 0
    assert np.all(np.abs(s[nz] - ref_s[nz]) <= rtol * ref_s[nz] + 1e-6 * ref_s[nz].mean())
    times = every * np.arange(1, steps // every + 1)
    z = []
    for m in range(1, L // 2):
        k = 2 * np.pi * m / L
        th = T.sk_linear_times([k, 0.0], times, D=2, kind=4, n0=c["rho0"], G=G,
                               kBT=c["kBT"]).mean()
        mean = s[:, m].sum() / cnt[:, m].sum()
        # 4 modes per sample (+-m on two axes), correlated over a few samples
        err = th / np.sqrt(cnt[:, m].sum() / 4.0)
        z.append((mean - th) / err)
    z = np.array(z)
    print(precision, "z-scores", np.round(z, 2))
    assert np.abs(z).max() < 5.0 and np.mean(z ** 2) < 4.0


# ------------------------------------------ the headline quench, early times -----
def test_quench_early_sk_growth_matches_exact_linear_theory():
    # The deep quench of the headline workload (D2Q9 E8, T_hat 0.7, n0 1,
    # kBT 1e-4, FP32) is linearly unstable: from the homogeneous start each
    # axis mode's S(k, t) follows the exact linear expectation (the linearised
    # step iterated on the noise covariance, Eq. 16 being its stationary limit
    # where one exists) until the amplitudes leave the linear regime.  16
    # replicas of 256^2 in the two-step tiling of the headline (192 lanes, one
    # barrier per row), sampled after 4, 8, 12 and 16 steps: the fastest
    # modes' S grows about 100-fold from the first sample to the last, while
    # the density still deviates by a few percent at most.
    from oracle import theory as T
    L, nrep, every, steps = 256, 16, 4, 16
    T_hat, n0, kBT = 0.7, 1.0, 1e-4
    plist = [_p((L, L), "fp32", T_hat=T_hat, rho0=n0, kBT=kBT, replica=r, seed=77, stencil=8)
             for r in range(nrep)]
    ens = fsc.Ensemble(plist)
    try:
        ens.init_uniform()
        ens.set_tiling(246, 1, 0, 2)  # the headline tiling (halo columns in the tile lanes)
        ens.run(steps, every)
        s = sum(ens.read_sk(r, fsc.FSC_SK_AXIS)[0] for r in range(nrep))
        cnt = sum(ens.read_sk(r, fsc.FSC_SK_AXIS)[2] for r in range(nrep))
        rmax = max(ens.stats(r)["rho_max"] for r in range(nrep))
        rmin = min(ens.stats(r)["rho_min"] for r in range(nrep))
    finally:
        ens.close()
    assert rmax - n0 < 0.2 and n0 - rmin < 0.2  # still close to the homogeneous state
    G = O.coupling_from_reduced_temperature(T_hat)
    times = every * np.arange(1, steps // every + 1)
    z, growth = [], []
    for m in range(1, L // 2):
        th_t = T.sk_linear_times([2 * np.pi * m / L, 0.0], times, D=2, kind=8, n0=n0, G=G,
                                 kBT=kBT)
        th = th_t.mean()
        growth.append(th_t[-1] / th_t[0])
        mean = s[:, m].sum() / cnt[:, m].sum()
        # per sample time: 2 independent modes per replica (+-m give the same
        # power of a real field); the four times are counted as one sample
        err = th / np.sqrt(2 * nrep)
        z.append((mean - th) / err)
    z = np.array(z)
    print("fastest theory growth over the run: %.0f-fold; z-scores max %.2f, mean z^2 %.2f"
          % (max(growth), np.abs(z).max(), np.mean(z ** 2)))
    assert max(growth) > 20  # the unstable band is resolved and growing
    assert np.abs(z).max() < 5.0 and np.mean(z ** 2) < 2.0


def test_3d_quench_early_sk_growth_matches_exact_linear_theory():
    # The same check for the D3Q19 kernel: E4, T_hat 0.8, n0 1 (between the
    # spinodal densities 0.645 and 1.670, so unstable), kBT 1e-4, FP32; 8
    # replicas of 48^3 sampled after 4, 8, 12 and 16 steps.
    from oracle import theory as T
    L, nrep, every, steps = 48, 8, 4, 16
    T_hat, n0, kBT = 0.8, 1.0, 1e-4
    plist = [_p((L, L, L), "fp32", T_hat=T_hat, rho0=n0, kBT=kBT, replica=r, seed=78)
             for r in range(nrep)]
    ens = fsc.Ensemble(plist)
    try:
        ens.init_uniform()
        ens.run(steps, every)
        s = sum(ens.read_sk(r, fsc.FSC_SK_AXIS)[0] for r in range(nrep))
        cnt = sum(ens.read_sk(r, fsc.FSC_SK_AXIS)[2] for r in range(nrep))
    finally:
        ens.close()
    G = O.coupling_from_reduced_temperature(T_hat)
    times = every * np.arange(1, steps // every + 1)
    z, growth = [], []
    for m in range(1, L // 2):
        th_t = T.sk_linear_times([2 * np.pi * m / L, 0.0, 0.0], times, D=3, kind=4, n0=n0, G=G,
                                 kBT=kBT)
        th = th_t.mean()
        growth.append(th_t[-1] / th_t[0])
        mean = s[:, m].sum() / cnt[:, m].sum()
        err = th / np.sqrt(3 * nrep)  # three axes per replica, +-m alike
        z.append((mean - th) / err)
    z = np.array(z)
    print("fastest theory growth over the run: %.0f-fold; z-scores max %.2f, mean z^2 %.2f"
          % (max(growth), np.abs(z).max(), np.mean(z ** 2)))
    assert max(growth) > 20
    assert np.abs(z).max() < 5.0 and np.mean(z ** 2) < 2.0
