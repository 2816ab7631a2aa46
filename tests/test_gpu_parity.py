"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: FP64 populations agree to 1e-11 relative; FP32-shifted populations
agree to 1e-5 relative, measured on the full f_i with a floor of w_i n0 (the
deviations f_i - w_i n0 themselves can be ~1e-7).  Integer work (Philox
words, node indexing, streaming) is compared bit for bit.
"""
import math
import os

import numpy as np
import pytest

import fsc_inputs as I
import oracle as O
from oracle import theory as T

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _params(D, shape, stencil, precision, T_hat=0.9, rho0=0.5, kBT=0.0, lam=(1, 1, 1), seed=0,
            replica=0):
    if D == 2:
        ny, nx = shape
        nz = 1
    else:
        nz, ny, nx = shape
    return fsc.make_params(D=D, nx=nx, ny=ny, nz=nz, stencil=stencil, precision=precision,
                           T_hat=T_hat, rho0=rho0, lam=lam, kBT=kBT, seed=seed, replica=replica)


def assert_pop_close(got, ref, D, rho0, precision):
    _, w = O.lattice(D)
    scale = np.maximum(np.abs(ref), (w * rho0).reshape((-1,) + (1,) * (ref.ndim - 1)))
    rel = np.abs(got - ref) / scale
    tol = 1e-11 if precision == "fp64" else 1e-5
    assert np.isfinite(got).all()
    assert rel.max() <= tol, f"max rel err {rel.max():.3e} > {tol:.0e}"
    return rel.max()


# --------------------------------------------------------------- generator --
def test_philox_bitexact_against_oracle_and_published_vectors():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(4096, 2), dtype=np.uint64).astype(np.uint32)
    ctr = np.vstack([np.array([r[0:4] for r in rows], dtype=np.uint32), ctr])
    key = np.vstack([np.array([r[4:6] for r in rows], dtype=np.uint32), key])
    got = fsc.philox(ctr, key)
    for k, r in enumerate(rows):
        assert list(got[k]) == r[6:10]
    ref = np.array([O.philox4x32_10(c, kk) for c, kk in zip(ctr[:600], key[:600])], dtype=np.uint32)
    assert np.array_equal(got[:600], ref)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("precision,atol", [("fp64", 1e-13), ("fp32", 4e-6)])
def test_normals_match_oracle(D, precision, atol):
    rng = np.random.default_rng(2)
    nodes = rng.integers(0, 2 ** 24, size=3000)
    steps = rng.integers(0, 2 ** 32, size=3000)
    seed = (7 << 32) | 12345
    got = fsc.normals(D, precision, seed, 3, nodes, steps)
    ref = np.array([O.normals(D, int(n), int(s), seed, 3) for n, s in zip(nodes, steps)])
    assert np.abs(got - ref).max() <= atol


# ------------------------------------------------------------ one step -------
CASES = [
    # D, shape (slow..fast), stencil
    (2, (37, 150), 4),     # ragged x tail (150 = 128 + 22), odd rows
    (2, (61, 300), 8),     # E8 halo of 2, three x tiles with a ragged tail
    (2, (1, 7), 4),        # single row: every neighbour wraps onto itself
    (2, (3, 5), 8),        # lattice smaller than the E8 halo
    (3, (9, 17, 40), 4),   # ragged in x (32 + 8) and y (8 + 8 + 1)
    (3, (2, 3, 1), 4),     # degenerate 3D
    (2, (7, 1), 8),        # single column under the E8 halo
    (2, (1, 1), 4),        # one node: every neighbour is the node itself, no force
    (3, (1, 1, 1), 4),
    (3, (3, 1, 5), 4),     # one row in y
]


@pytest.mark.parametrize("D,shape,stencil", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_steps_from_random_state(D, shape, stencil, precision):
    Q = 9 if D == 2 else 19
    rho0 = 0.8
    f0 = I.random_populations(Q, shape, rho0, 0.3, seed=11)
    lam = (0.9, 1.25, 1.6)
    kw = dict(T_hat=0.85, rho0=rho0, kBT=2e-4, lam=lam, seed=(3 << 32) | 5, replica=2)
    with fsc.Lattice(_params(D, shape, stencil, precision, **kw)) as lat:
        lat.set_populations(f0, step=17)
        lat.step(1)
        g1 = lat.get_populations()
        lat.step(2)
        g3 = lat.get_populations()
        assert lat.t == 20
        G = lat.G
    r1 = O.step(f0, 1, G=G, kind=stencil, kBT=2e-4, lam_bulk=lam[0], lam_shear=lam[1],
                lam_ghost=lam[2], seed=(3 << 32) | 5, replica=2, t0=17)
    r3 = O.step(r1, 2, G=G, kind=stencil, kBT=2e-4, lam_bulk=lam[0], lam_shear=lam[1],
                lam_ghost=lam[2], seed=(3 << 32) | 5, replica=2, t0=18)
    assert_pop_close(g1, r1, D, rho0, precision)
    assert_pop_close(g3, r3, D, rho0, precision)


@pytest.mark.parametrize("D,shape,stencil,precision,tiling", [
    (2, (37, 300), 8, "fp32", (246, 1, 0, 2)),   # the headline's two-step tiling
    (2, (37, 300), 8, "fp32", (128, 1, 1, 1)),
    (2, (29, 41), 4, "fp32", (250, 1, 1, 2)),
    (3, (9, 20, 37), 4, "fp32", (256, 4, 0, 1)),
    (2, (29, 41), 8, "fp64", None),
    (3, (9, 20, 37), 4, "fp64", None),
])
def test_phase_separated_densities_match_oracle(D, shape, stencil, precision, tiling):
    # densities from 0.3 to 2.5 around n0 = 1: the pseudopotential's argument
    # dn / (n0 n) runs from -2.3 to 0.6, through both branches of the FP32
    # kernels' expm1 (|x| < 1/2 and beyond) and both signs of the force
    Q = 9 if D == 2 else 19
    f0 = I.wide_density_populations(Q, shape, 0.3, 2.5, 3, seed=31)
    p = _params(D, shape, stencil, precision, T_hat=0.7, rho0=1.0, kBT=1e-4, seed=9)
    with fsc.Lattice(p) as lat:
        lat.set_populations(f0, 77)
        if tiling is not None:
            lat.set_tiling(*tiling, 1 << 20)
        lat.step(2)
        got = lat.get_populations()
        G = lat.G
    n0 = O.density(f0)
    assert n0.min() < 0.35 and n0.max() > 2.4
    ref = O.step(f0, 2, G=G, kind=stencil, kBT=1e-4, seed=9, t0=77)
    assert_pop_close(got, ref, D, 1.0, precision)


def test_coupling_from_reduced_temperature():
    with fsc.Lattice(_params(2, (8, 8), 4, "fp32", T_hat=0.8)) as lat:
        assert lat.G == pytest.approx(O.coupling_from_reduced_temperature(0.8), rel=1e-15)


# ------------------------------------------------------- long stable runs ----
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_small_parity_workload(precision):
    c = dict(I.SMALL_PARITY)
    p = _params(2, (c["ny"], c["nx"]), c["stencil"], precision, T_hat=c["T_hat"], rho0=c["rho0"],
                kBT=c["kBT"], seed=c["seed"])
    with fsc.Lattice(p) as lat:
        lat.init_uniform()
        lat.step(c["steps"])
        got = lat.get_populations()
        G = lat.G
        st = lat.stats()
    ref = O.step(O.uniform_state(2, (c["ny"], c["nx"]), c["rho0"]), c["steps"], G=G,
                 kind=c["stencil"], kBT=c["kBT"], seed=c["seed"])
    err = assert_pop_close(got, ref, 2, c["rho0"], precision)
    print(f"{precision}: max rel err {err:.3e}")
    m_ref, p_ref = O.conserved(ref)
    M0 = c["rho0"] * c["nx"] * c["ny"]
    assert abs(st["mass"] - M0) / M0 <= (1e-12 if precision == "fp64" else 1e-6)
    assert np.abs(st["mom"]).max() / M0 <= (1e-12 if precision == "fp64" else 1e-6)
    assert abs(m_ref - M0) / M0 < 1e-12


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("D,shape,stencil,T_hat,rho0",
                         [(2, (32, 64), 8, 0.7, 1.0), (2, (20, 30), 4, 0.9, 0.5),
                          (3, (8, 12, 16), 4, 0.8, 0.62)])
def test_noise_free_flat_state_is_bit_exact(precision, D, shape, stencil, T_hat, rho0):
    with fsc.Lattice(_params(D, shape, stencil, precision, T_hat=T_hat, rho0=rho0)) as lat:
        lat.init_uniform()
        lat.step(101)
        n = lat.density()
        f = lat.get_populations()
    assert np.all(n == rho0)
    assert np.array_equal(f, O.uniform_state(D, shape, rho0))


def test_fp32_mass_drift_over_long_run():
    p = _params(2, (128, 128), 4, "fp32", T_hat=0.9, rho0=0.5, kBT=1e-4)
    with fsc.Lattice(p) as lat:
        lat.init_uniform()
        lat.step(20000)
        st = lat.stats()
    M0 = 0.5 * 128 * 128
    drift = abs(st["mass"] - M0) / M0
    print(f"fp32 relative mass drift after 20000 steps: {drift:.3e}")
    assert drift <= 1e-6
    assert np.abs(st["mom"]).max() / M0 <= 1e-6
    assert st["bad"] == 0


def test_same_seed_is_bitwise_deterministic():
    p = _params(2, (64, 96), 8, "fp32", T_hat=0.75, rho0=1.0, kBT=1e-4, seed=9)
    out = []
    for _ in range(2):
        with fsc.Lattice(p) as lat:
            lat.init_uniform()
            lat.step(300)
            out.append(lat.get_populations())
    assert np.array_equal(out[0], out[1])
    p2 = _params(2, (64, 96), 8, "fp32", T_hat=0.75, rho0=1.0, kBT=1e-4, seed=10)
    with fsc.Lattice(p2) as lat:
        lat.init_uniform()
        lat.step(300)
        assert not np.array_equal(out[0], lat.get_populations())


def test_rejects_bad_parameters():
    with pytest.raises(fsc.FscError):
        fsc.Lattice(_params(3, (8, 8, 8), 8, "fp32"))
    with pytest.raises(fsc.FscError):
        fsc.Lattice(fsc.make_params(D=2, nx=8, ny=8, rho0=-1.0))
    with pytest.raises(fsc.FscError):
        fsc.Lattice(fsc.make_params(D=2, nx=8, ny=8, lam=(1.0, 2.5, 1.0)))
    with fsc.Lattice(_params(2, (8, 8), 4, "fp32")) as lat:
        lat.init_uniform()
        with pytest.raises(fsc.FscError):
            lat.step(-1)
    # S(k) of a side beyond the FFT limit is refused, again on a second request
    # (a refusal leaves no half-built sample buffers behind), and steps still run
    with fsc.Lattice(_params(2, (2, 8200), 4, "fp32")) as lat:
        lat.init_uniform()
        for _ in range(2):
            with pytest.raises(fsc.FscError, match="8192"):
                lat.measure_sk()
        lat.step(3)
        assert lat.stats()["bad"] == 0


def test_zero_steps_and_empty_requests():
    # zero steps leave the state and the step counter as they are, with and
    # without sampling; an ensemble of no replicas and an S(k) batch of no
    # fields are refused
    with fsc.Lattice(_params(2, (8, 8), 4, "fp32", kBT=1e-4, seed=2)) as lat:
        lat.set_populations(I.random_populations(9, (8, 8), 0.5, 0.3, seed=2), step=5)
        g0 = lat.get_populations()
        lat.step(0)
        lat.run(0, 10)
        assert lat.t == 5
        assert np.array_equal(lat.get_populations(), g0)
        lat.step(1)
        assert lat.t == 6 and not np.array_equal(lat.get_populations(), g0)
    with pytest.raises(fsc.FscError):
        fsc.Ensemble([])
    torch = pytest.importorskip("torch")
    fields = torch.ones((1, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(fsc.FscError):
        fsc.field_sk(fields, 0, 16)
    s, L = fsc.field_sk(fields, 1, 16)  # a flat field: no power anywhere
    assert np.all(s == 0.0)


# -------------------------------------------------------------- S(k) --------
def _sk_case(shape, precision, seed):
    D = len(shape)
    Q = 9 if D == 2 else 19
    # a white (random) density field: every bin carries power of the same order,
    # so the bins can be compared one by one with a relative tolerance
    f = I.random_populations(Q, shape, 0.7, 0.3, seed)
    p = _params(D, shape, 4, precision, rho0=0.7)
    with fsc.Lattice(p) as lat:
        lat.set_populations(f, 0)
        lat.measure_sk()
        lat.measure_sk()
        ax = lat.read_sk(fsc.FSC_SK_AXIS)
        rad = lat.read_sk(fsc.FSC_SK_RADIAL)
        rho_gpu = lat.density()
    ref = O.sk_sample(O.density(f))
    return ax, rad, ref, rho_gpu, O.density(f)


# Per-bin tolerance of the S(k) sums: FP64 is summed exactly up to rounding
# order; FP32 forms the density and its FFT in single precision (about
# log2(N) * 6e-8 of the rms amplitude per mode), accumulated in FP64.  The
# absolute floor is a millionth of the mean bin, far below any bin's own power.
SK_RTOL = {"fp64": 1e-10, "fp32": 1e-4}


def assert_bins_close(got, ref, precision, factor=1.0):
    """Element-wise |got - ref| <= rtol |ref| + floor; factor 2 for sums of squares."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    floor = 1e-6 * np.abs(ref[ref != 0]).mean() if np.any(ref != 0) else 0.0
    bad = np.abs(got - ref) > factor * SK_RTOL[precision] * np.abs(ref) + floor
    assert not bad.any(), (np.argwhere(bad)[:5], got[bad][:5], ref[bad][:5])
    nz = ref != 0
    return float((np.abs(got - ref)[nz] / np.abs(ref[nz])).max()) if nz.any() else 0.0


@pytest.mark.parametrize("shape", [(64, 64), (48, 80), (24, 40), (16, 16, 16), (12, 10, 9),
                                   # degenerate: no mode at all, single rows and columns,
                                   # sides of 2 (the Nyquist mode only) and 3
                                   (1, 1), (7, 1), (1, 7), (2, 2), (2, 3), (1, 1, 1), (2, 3, 1),
                                   (1, 2, 2), (2, 2, 2), (3, 3, 3)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_structure_factor_measurement_matches_oracle(shape, precision):
    ax, rad, ref, rho_gpu, rho_ref = _sk_case(shape, precision, seed=4)
    assert np.abs(rho_gpu - rho_ref).max() <= (1e-13 if precision == "fp64" else 1e-6)
    a_sum, a_sq, a_cnt = ax
    r_sum, r_sq, r_cnt = ref["axis"]
    assert np.array_equal(a_cnt, 2 * r_cnt[:, : a_cnt.shape[1]])
    # two identical samples: sums are twice the oracle's one-sample bins
    worst = assert_bins_close(a_sum[:, : r_sum.shape[1]], 2 * r_sum, precision)
    assert_bins_close(a_sq[:, : r_sq.shape[1]], 2 * r_sq, precision, factor=2.0)
    if ref["radial"] is not None:
        g_sum, g_sq, g_cnt = rad
        o_sum, o_sq, o_cnt = ref["radial"]
        assert np.array_equal(g_cnt, 2 * o_cnt)
        worst = max(worst, assert_bins_close(g_sum, 2 * o_sum, precision))
        assert_bins_close(g_sq, 2 * o_sq, precision, factor=2.0)
    else:
        assert rad[0].size == 0
    print(f"{shape} {precision}: worst relative bin error {worst:.2e}")


# ----------------------------------------------------- graph and ensemble ----
def test_graph_replay_equals_eager_steps():
    p = _params(2, (64, 64), 4, "fp32", T_hat=0.9, rho0=0.5, kBT=1e-4, seed=3)
    with fsc.Lattice(p) as a, fsc.Lattice(p) as b:
        a.init_uniform()
        b.init_uniform()
        a.run(400, sk_every=10)
        for _ in range(40):
            b.step(10)
            b.measure_sk()
        assert a.t == b.t == 400
        assert np.array_equal(a.get_populations(), b.get_populations())
        sa, qa, ca = a.read_sk()
        sb, qb, cb = b.read_sk()
        assert np.array_equal(ca, cb)
        assert np.allclose(sa, sb, rtol=1e-12, atol=0)
        ra = a.read_sk(fsc.FSC_SK_RADIAL)
        rb = b.read_sk(fsc.FSC_SK_RADIAL)
        assert np.allclose(ra[0], rb[0], rtol=1e-12, atol=0)
        # odd chunk and remainder handling
        a.run(37, sk_every=7)
        for _ in range(5):
            b.step(7)
            b.measure_sk()
        b.step(2)
        assert np.array_equal(a.get_populations(), b.get_populations())


def test_ensemble_replicas_equal_single_lattices_and_oracle():
    specs = [((64, 64), 0.9, 0.5), ((80, 96), 0.8, 2.0), ((128, 128), 0.7, 0.3), ((33, 47), 0.95, 0.8)]
    plist = [_params(2, sh, 4, "fp32", T_hat=th, rho0=r0, kBT=1e-4, seed=5, replica=k)
             for k, (sh, th, r0) in enumerate(specs)]
    ens = fsc.Ensemble(plist)
    ens.init_uniform()
    ens.run(130, sk_every=0)
    assert ens.t == 130
    for k, (sh, th, r0) in enumerate(specs):
        with fsc.Lattice(plist[k]) as lat:
            lat.init_uniform()
            lat.step(130)
            single = lat.get_populations()
            G = lat.G
        got = ens.get_populations(k)
        assert np.array_equal(got, single)
        ref = O.step(O.uniform_state(2, sh, r0), 130, G=G, kind=4, kBT=1e-4, seed=5, replica=k)
        assert_pop_close(got, ref, 2, r0, "fp32")
    ens.close()


def test_autotune_leaves_state_and_results_unchanged():
    p = _params(2, (200, 300), 8, "fp32", T_hat=0.75, rho0=1.0, kBT=1e-4, seed=4)
    with fsc.Lattice(p) as a, fsc.Lattice(p) as b:
        a.init_uniform()
        b.init_uniform()
        a.step(40)
        b.step(17)
        before = b.get_populations()
        b.autotune()
        assert np.array_equal(before, b.get_populations())
        b.step(23)
        assert np.array_equal(a.get_populations(), b.get_populations())
        t = b.tiling
        assert t["blocks"] > 0 and (t["tx"], t["ty"], t["pf"], t["steps"]) in fsc.tile_shapes(2, 8, "fp32")


def test_ensemble_autotune_restores_every_replica():
    # the autotuner's trial launches alternate the two buffers of every replica
    # on a copy of the state, which it puts back: uneven replicas at an odd step
    # (state in the second buffer) keep their populations, and continue exactly
    # as an untuned twin
    specs = [((96, 80), 0.8, 1.0), ((64, 200), 0.75, 1.2), ((130, 70), 0.9, 0.8)]
    plist = [_params(2, sh, 8, "fp32", T_hat=th, rho0=r0, kBT=1e-4, seed=11, replica=k)
             for k, (sh, th, r0) in enumerate(specs)]
    a, b = fsc.Ensemble(plist), fsc.Ensemble(plist)
    try:
        a.init_uniform()
        b.init_uniform()
        a.run(30, 0)
        b.run(13, 0)
        before = [b.get_populations(k) for k in range(len(specs))]
        b.autotune()
        for k in range(len(specs)):
            assert np.array_equal(before[k], b.get_populations(k)), k
        b.run(17, 0)
        for k in range(len(specs)):
            assert np.array_equal(a.get_populations(k), b.get_populations(k)), k
    finally:
        a.close()
        b.close()


def test_checkpoint_resume_is_bit_exact(tmp_path):
    specs = [((64, 64), 0.9, 0.5), ((40, 48), 0.8, 2.0)]
    plist = [_params(2, sh, 4, "fp32", T_hat=th, rho0=r0, kBT=1e-4, seed=9, replica=k)
             for k, (sh, th, r0) in enumerate(specs)]
    path = str(tmp_path / "ens.ckpt")
    a = fsc.Ensemble(plist)
    a.init_uniform()
    a.run(60, sk_every=10)
    a.save(path)
    a.run(50, sk_every=10)
    b = fsc.Ensemble(plist)
    b.load(path)
    assert b.t == 60
    b.run(50, sk_every=10)
    for k in range(len(specs)):
        assert np.array_equal(a.get_populations(k), b.get_populations(k))
        # S(k) bins are summed with FP64 atomics: equal up to the order of the
        # additions (last bits); the mode counts are exact
        kinds = [fsc.FSC_SK_AXIS] + ([fsc.FSC_SK_RADIAL] if k == 0 else [])
        for kind in kinds:
            (sb, qb, cb), (sa, qa, ca) = b.read_sk(k, kind), a.read_sk(k, kind)
            assert np.allclose(sb, sa, rtol=1e-12, atol=0) and np.allclose(qb, qa, rtol=1e-12, atol=0)
            assert np.array_equal(cb, ca)
    # another seed, a truncated file, a missing file: refused, state untouched
    other = fsc.Ensemble([plist[0], _params(2, specs[1][0], 4, "fp32", T_hat=0.8, rho0=2.0,
                                            kBT=1e-4, seed=10, replica=1)])
    other.init_uniform()
    with pytest.raises(fsc.FscError, match="invalid argument"):
        other.load(path)
    assert other.t == 0
    trunc = str(tmp_path / "trunc.ckpt")
    with open(path, "rb") as src, open(trunc, "wb") as dst:
        dst.write(src.read()[:4000])
    before = b.get_populations(1)
    with pytest.raises(fsc.FscError, match="file error"):
        b.load(trunc)
    with pytest.raises(fsc.FscError, match="file error"):
        b.load(str(tmp_path / "missing.ckpt"))
    assert b.t == 110 and np.array_equal(b.get_populations(1), before)
    for e in (a, b, other):
        e.close()
    # single lattice, FP64, D3Q19
    p3 = _params(3, (10, 12, 14), 4, "fp64", T_hat=0.9, rho0=0.5, kBT=1e-4, seed=2)
    with fsc.Lattice(p3) as x, fsc.Lattice(p3) as y:
        x.init_uniform()
        x.step(7)
        x.save(path)
        x.step(5)
        y.load(path)
        y.step(5)
        assert np.array_equal(x.get_populations(), y.get_populations())


# ------------------------------------------------ full-size sampled parity ---
@pytest.mark.parametrize("case", ["deep_quench_4096", "metastable_256cube"])
def test_full_size_one_step_matches_oracle(case):
    c = I.DEEP_QUENCH if case == "deep_quench_4096" else I.METASTABLE_3D
    D = c["D"]
    shape = (c["ny"], c["nx"]) if D == 2 else (c["nz"], c["ny"], c["nx"])
    Q = 9 if D == 2 else 19
    f0 = I.random_populations(Q, shape, c["rho0"], 0.1, seed=21)
    p = _params(D, shape, c["stencil"], c["precision"], T_hat=c["T_hat"], rho0=c["rho0"],
                kBT=c["kBT"], seed=c["seed"])
    with fsc.Lattice(p) as lat:
        lat.set_populations(f0, 1234)
        lat.step(1)
        got = lat.get_populations()
        G = lat.G
    ref = O.step(f0, 1, G=G, kind=c["stencil"], kBT=c["kBT"], seed=c["seed"], t0=1234)
    del f0
    assert_pop_close(got, ref, D, c["rho0"], c["precision"])


def test_full_size_two_step_launch_matches_oracle():
    # the 4096^2 E8 quench in the tiling the autotuner picks for it (the launch
    # bench.py times): one launch of the temporally blocked kernel advances two steps
    c = I.DEEP_QUENCH
    shape = (c["ny"], c["nx"])
    f0 = I.random_populations(9, shape, c["rho0"], 0.1, seed=22)
    p = _params(2, shape, c["stencil"], c["precision"], T_hat=c["T_hat"], rho0=c["rho0"],
                kBT=c["kBT"], seed=c["seed"])
    with fsc.Lattice(p) as lat:
        lat.set_populations(f0, 4321)
        lat.autotune()
        tiling = lat.tiling
        lat.step(2)
        got = lat.get_populations()
        G = lat.G
    print("tiling", tiling, flush=True)
    assert tiling["steps"] == 2
    # the same two steps as two single-step launches: bit for bit
    with fsc.Lattice(p) as lat:
        lat.set_populations(f0, 4321)
        lat.set_tiling(128, 1, 1, 1, 1024)
        lat.step(2)
        assert np.array_equal(lat.get_populations(), got)
    ref = O.step(f0, 2, G=G, kind=c["stencil"], kBT=c["kBT"], seed=c["seed"], t0=4321)
    del f0
    assert_pop_close(got, ref, 2, c["rho0"], c["precision"])


def test_bench_ensemble_launch_matches_oracle():
    # the 64-replica ensemble of bench.py (sides 128, 256 and 512) in its
    # autotuned launch configuration; replicas of every side start from random
    # states and are compared with the oracle after two steps (one launch of a
    # two-step tiling), the others from the flat state
    reps = I.ensemble_replicas(n=64, seed=0, kBT=1e-13)
    plist = [fsc.make_params(**{k: v for k, v in r.items() if k != "precision"}, precision="fp32")
             for r in reps]
    sample = []
    for side in (128, 256, 512):
        sample += [k for k, r in enumerate(reps) if r["nx"] == side][:2]
    ens = fsc.Ensemble(plist)
    ens.init_uniform()
    f0 = {}
    for k in sample:
        shape = (reps[k]["ny"], reps[k]["nx"])
        f0[k] = I.random_populations(9, shape, reps[k]["rho0"], 0.05, seed=40 + k)
        ens.set_populations(k, f0[k])
    ens.autotune()
    tiling = ens.tiling
    ens.run(2, 0)
    print("tiling", tiling, flush=True)
    for k in sample:
        got = ens.get_populations(k)
        G = O.coupling_from_reduced_temperature(reps[k]["T_hat"])
        ref = O.step(f0[k], 2, G=G, kind=4, kBT=reps[k]["kBT"], seed=0, replica=k, t0=0)
        assert_pop_close(got, ref, 2, reps[k]["rho0"], "fp32")
    # a replica left flat stays flat up to the noise
    flat = next(k for k in range(len(reps)) if k not in f0)
    got = ens.get_populations(flat)
    rf = reps[flat]
    ref = O.step(O.uniform_state(2, (rf["ny"], rf["nx"]), rf["rho0"]), 2,
                 G=O.coupling_from_reduced_temperature(rf["T_hat"]), kind=4, kBT=rf["kBT"], seed=0,
                 replica=flat, t0=0)
    assert_pop_close(got, ref, 2, rf["rho0"], "fp32")
    ens.close()


# ---------------------------------------------- statistics against theory ----
@pytest.mark.parametrize("precision,T_hat,rho0,kBT,stencil", [("fp32", 0.9, 0.5, 1e-6, 4),
                                                              ("fp32", 0.8, 0.62, 1e-13, 4),
                                                              ("fp64", 0.9, 2.0, 1e-6, 4),
                                                              ("fp32", 0.9, 0.5, 1e-6, 8)])
def test_gpu_structure_factor_matches_exact_theory(precision, T_hat, rho0, kBT, stencil):
    # stationary axis S(k) against Eq. 16 (E4) and its E8 form, whose sound
    # speed carries the E8 stencil's own h(k)
    L = 64
    p = _params(2, (L, L), stencil, precision, T_hat=T_hat, rho0=rho0, kBT=kBT, seed=17)
    nb = 40
    with fsc.Lattice(p) as lat:
        lat.init_uniform()
        lat.step(8000)  # burn-in: slowest mode relaxes in ~10^3 steps
        batches = []
        for _ in range(nb):
            lat.sk_reset()
            lat.run(5000, sk_every=10)
            s, _, c = lat.read_sk()
            batches.append(s.sum(axis=0) / np.maximum(c.sum(axis=0), 1))
        G = lat.G
    B = np.array(batches)
    z = []
    for m in range(1, L // 2 + 1):
        k = 2 * math.pi * m / L
        th = (T.sk_exact(k, rho0, G, kBT) if stencil == 4
              else float(T.sk_exact_axis(k, rho0, G, kBT, kind=8)[0]))
        mean = B[:, m].mean()
        err = B[:, m].std(ddof=1) / math.sqrt(nb)
        z.append((mean - th) / err)
        assert abs(mean / th - 1) < max(0.03, 4 * err / th)
    z = np.array(z)
    print("z-scores", np.round(z, 2))
    assert np.all(np.abs(z) < 4.0)
    assert np.mean(z ** 2) < 2.5


# --------------------------------------------------- S(k, t) and L(t) --------
@pytest.mark.parametrize("shape,precision", [((64, 64), "fp64"), ((64, 64), "fp32"),
                                             ((16, 16, 16), "fp32")])
def test_series_row_matches_oracle(shape, precision):
    D = len(shape)
    Q = 9 if D == 2 else 19
    f = I.smooth_density_populations(Q, shape, 1.0, 0.2, 6, seed=8)
    p = _params(D, shape, 4, precision, rho0=1.0)
    with fsc.Lattice(p) as lat:
        lat.series_enable(8)
        lat.set_populations(f, 77)
        lat.measure_sk()
        ser = lat.read_series()
    rho = O.density(f)
    assert list(ser["step"]) == [77]
    tol = 1e-10 if precision == "fp64" else 1e-4
    assert ser["L"][0] == pytest.approx(O.domain_length(rho), rel=tol)
    ref = O.shell_means(rho)
    assert np.allclose(ser["S"][0], ref, rtol=tol, atol=tol * ref.max())


def test_series_through_graph_replay_records_every_sample():
    p = _params(2, (128, 128), 8, "fp32", T_hat=0.7, rho0=1.0, kBT=1e-4, seed=2)
    with fsc.Lattice(p) as lat:
        lat.init_uniform()
        lat.series_enable(64)
        lat.run(1000, sk_every=50)
        ser = lat.read_series()
    assert list(ser["step"]) == list(range(50, 1001, 50))
    L = ser["L"]
    assert np.all(np.isfinite(L)) and np.all(L > 0)
    # spinodal decomposition: the domains coarsen once the unstable modes saturate
    assert L[-1] > L[4]
