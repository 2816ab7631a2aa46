"""Every compiled tiling and marching length gives bit-identical populations
(the per-node arithmetic does not depend on the tiling), on lattices with
ragged tiles in every direction; the two-step kernel equals two single steps
bit for bit, also across S(k) samples that split a pair, whole-row tiles,
narrow lattices and an odd number of steps."""
import numpy as np
import pytest

import fsc_inputs as I

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")

CASES = [
    # D, (nz, ny, nx) or (ny, nx), stencil, precision
    (2, (70, 301), 4, "fp32"),
    (2, (53, 200), 8, "fp32"),
    (2, (37, 128), 4, "fp32"),   # one whole-row tile of 128 (and of 256)
    (2, (13, 1100), 4, "fp32"),  # a last tile 76 wide: whole waves of it idle
    (2, (9, 6), 8, "fp32"),      # narrowest two-step width for E8 (2R + 2)
    (2, (41, 256), 8, "fp32"),
    (2, (11, 247), 8, "fp32"),   # 246-column in-tile-halo tiles: a last tile one column wide
    (2, (9, 251), 4, "fp32"),    # the same for E4's 250-column tiles
    (3, (23, 45, 37), 4, "fp32"),
    (3, (2, 3, 5), 4, "fp32"),   # thinner than the halo in every direction: all wraps
    (2, (40, 77), 8, "fp64"),
    (3, (12, 19, 21), 4, "fp64"),
    (3, (9, 17, 40), 4, "fp64"),  # ragged in x (32 + 8) and y (8 + 8 + 1)
]


def _params(D, shape, stencil, precision):
    nz, ny, nx = shape if D == 3 else (1,) + shape
    return fsc.make_params(D=D, nx=nx, ny=ny, nz=nz, stencil=stencil, precision=precision,
                           T_hat=0.8, rho0=0.9, kBT=1e-4, seed=13)


@pytest.mark.parametrize("D,shape,stencil,precision", CASES)
def test_all_tilings_are_bit_identical(D, shape, stencil, precision):
    p = _params(D, shape, stencil, precision)
    Q = 9 if D == 2 else 19
    f0 = I.smooth_density_populations(Q, shape, 0.9, 0.05, 3, seed=2)
    with fsc.Lattice(p) as ref:
        ref.set_populations(f0, 5)
        ref.step(9)
        want = ref.get_populations()
    shapes = fsc.tile_shapes(D, stencil, precision)
    assert len(shapes) >= 1
    for (tx, ty, pf, steps) in shapes:
        for target in (1, 37, 1 << 20):  # longest march, a ragged one, one plane per block
            with fsc.Lattice(p) as lat:
                lat.set_populations(f0, 5)
                lat.set_tiling(tx, ty, pf, steps, target)
                t = lat.tiling
                assert (t["tx"], t["ty"], t["pf"], t["steps"]) == (tx, ty, pf, steps)
                lat.step(9)
                got = lat.get_populations()
            print(tx, ty, pf, steps, target, t["blocks"], flush=True)
            assert np.array_equal(got, want), (tx, ty, pf, steps, target)


@pytest.mark.parametrize("stencil", [4, 8])
def test_two_step_runs_with_samples_equal_single_steps(stencil):
    # graph chunks with S(k) samples every 6 steps (pairs) and every 5 steps
    # (a single step before each sample), plus a remainder
    p = _params(2, (48, 300), stencil, "fp32")
    f0 = I.smooth_density_populations(9, (48, 300), 0.9, 0.05, 3, seed=4)
    two = [s for s in fsc.tile_shapes(2, stencil, "fp32") if s[3] == 2]
    assert two
    for every, n in ((6, 61), (5, 47)):
        with fsc.Lattice(p) as ref:
            ref.set_populations(f0, 3)
            ref.set_tiling(128, 1, 1, 1, 64)
            ref.run(n, every)
            want = ref.get_populations()
            s_want, q_want, c_want = ref.read_sk()
        for (tx, ty, pf, steps) in two:
            with fsc.Lattice(p) as lat:
                lat.set_populations(f0, 3)
                lat.set_tiling(tx, ty, pf, steps, 64)
                lat.run(n, every)
                assert np.array_equal(lat.get_populations(), want), (tx, every)
                s_got, q_got, c_got = lat.read_sk()
                assert np.array_equal(c_got, c_want)
                np.testing.assert_allclose(s_got, s_want, rtol=1e-12)
                np.testing.assert_allclose(q_got, q_want, rtol=1e-12)


def test_two_step_is_refused_on_narrow_lattices():
    p = _params(2, (16, 5), 8, "fp32")  # 5 < 2R + 2 = 6
    with fsc.Lattice(p) as lat:
        with pytest.raises(fsc.FscError):
            lat.set_tiling(128, 1, 0, 2, 100)


def test_uncompiled_tiling_is_refused():
    p = _params(2, (32, 32), 4, "fp32")
    with fsc.Lattice(p) as lat:
        with pytest.raises(fsc.FscError):
            lat.set_tiling(96, 1, 1, 1, 100)
        with pytest.raises(fsc.FscError):
            lat.set_tiling(128, 1, 1, 1, 0)
        with pytest.raises(fsc.FscError):
            lat.set_tiling(128, 1, 2, 2, 100)  # no two-step kernel with schedule 2


@pytest.mark.parametrize("stencil", [4, 8])
def test_two_step_in_a_mixed_ensemble_equals_single_steps(stencil):
    # whole-row tiles, several tiles per row, ragged widths and heights in one
    # launch, uneven parameters per replica, S(k) samples splitting pairs
    shapes = [(40, 128), (33, 300), (20, 256), (17, 77), (9, 6), (11, 1100)]
    plist = [fsc.make_params(D=2, nx=nx, ny=ny, stencil=stencil, precision="fp32",
                             T_hat=0.75 + 0.05 * k, rho0=0.6 + 0.2 * k, kBT=1e-4 * (k + 1),
                             seed=21, replica=k)
             for k, (ny, nx) in enumerate(shapes)]
    f0 = [I.smooth_density_populations(9, sh, p.rho0, 0.05, 3, seed=30 + k)
          for k, (sh, p) in enumerate(zip(shapes, plist))]

    def run(tiling):
        ens = fsc.Ensemble(plist)
        ens.init_uniform()
        for k in range(len(shapes)):
            ens.set_populations(k, f0[k])
        ens.set_tiling(*tiling)
        ens.run(37, 5)
        out = [ens.get_populations(k) for k in range(len(shapes))]
        ens.close()
        return out

    want = run((128, 1, 1, 1, 64))
    for (tx, ty, pf, steps) in fsc.tile_shapes(2, stencil, "fp32"):
        if steps != 2:
            continue
        for target in (1, 64, 1 << 20):
            got = run((tx, ty, pf, steps, target))
            for k in range(len(shapes)):
                assert np.array_equal(got[k], want[k]), (tx, pf, target, k)


@pytest.mark.parametrize("stencil", [4, 8])
def test_noise_free_two_step_equals_single_steps(stencil):
    p = fsc.make_params(D=2, nx=300, ny=41, stencil=stencil, precision="fp32", T_hat=0.8,
                        rho0=0.9, kBT=0.0, seed=13)
    f0 = I.smooth_density_populations(9, (41, 300), 0.9, 0.05, 3, seed=6)
    with fsc.Lattice(p) as ref:
        ref.set_populations(f0, 0)
        ref.set_tiling(128, 1, 1, 1, 64)
        ref.step(13)
        want = ref.get_populations()
    for (tx, ty, pf, steps) in fsc.tile_shapes(2, stencil, "fp32"):
        if steps == 2:
            with fsc.Lattice(p) as lat:
                lat.set_populations(f0, 0)
                lat.set_tiling(tx, ty, pf, steps, 64)
                lat.step(13)
                assert np.array_equal(lat.get_populations(), want), (tx, pf)


def test_two_step_checkpoint_resumes_bit_exactly(tmp_path):
    # the state sits in either buffer after an odd number of launches; a
    # checkpoint written there resumes into any tiling
    plist = [fsc.make_params(D=2, nx=nx, ny=ny, stencil=4, precision="fp32", T_hat=0.8,
                             rho0=0.7, kBT=1e-4, seed=3, replica=k)
             for k, (ny, nx) in enumerate([(30, 256), (25, 300)])]
    path = str(tmp_path / "two.ckpt")
    a = fsc.Ensemble(plist)
    a.init_uniform()
    a.set_tiling(256, 1, 0, 2, 64)
    a.run(61, 10)
    a.save(path)
    a.run(40, 10)
    b = fsc.Ensemble(plist)
    b.load(path)
    b.set_tiling(128, 1, 1, 1, 64)  # resume with single steps
    b.run(40, 10)
    c = fsc.Ensemble(plist)
    c.load(path)
    c.set_tiling(128, 1, 1, 2, 64)  # and with the other two-step schedule
    c.run(40, 10)
    for k in range(2):
        assert np.array_equal(a.get_populations(k), b.get_populations(k))
        assert np.array_equal(a.get_populations(k), c.get_populations(k))
    for e in (a, b, c):
        e.close()


@pytest.mark.parametrize("D,shape,stencil", [(2, (41, 300), 4), (2, (41, 300), 8), (3, (13, 20, 37), 4)])
def test_unequal_rates_give_identical_tilings(D, shape, stencil):
    # bulk, shear and ghost rates all different, so that each moment class
    # has its own rate and noise amplitude in every kernel (both levels of the
    # two-step kernel included)
    nz, ny, nx = shape if D == 3 else (1,) + shape
    p = fsc.make_params(D=D, nx=nx, ny=ny, nz=nz, stencil=stencil, precision="fp32", T_hat=0.8,
                        rho0=0.9, lam=(0.7, 1.3, 1.8), kBT=1e-4, seed=5)
    Q = 9 if D == 2 else 19
    f0 = I.smooth_density_populations(Q, shape, 0.9, 0.05, 3, seed=8)
    shapes = fsc.tile_shapes(D, stencil, "fp32")
    want = None
    for (tx, ty, pf, steps) in shapes:
        with fsc.Lattice(p) as lat:
            lat.set_populations(f0, 11)
            lat.set_tiling(tx, ty, pf, steps, 37)
            lat.step(6)
            got = lat.get_populations()
        if want is None:
            want = got
        assert np.array_equal(got, want), (tx, ty, pf, steps)
