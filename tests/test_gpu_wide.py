"""Lattices whose population buffers reach 4 GiB or more.  The step kernel then
addresses each population with a buffer resource of its own; results must
equal the FP64 oracle as for any other lattice (tolerance as in
test_gpu_parity: 1e-5 of max(|f|, w n0) in FP32, 1e-11 in FP64)."""
import numpy as np
import pytest

import fsc_inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")


def _max_rel(got, ref, D, rho0):
    _, w = O.lattice(D)
    scale = np.maximum(np.abs(ref), (w * rho0).reshape((-1,) + (1,) * (ref.ndim - 1)))
    return float(np.max(np.abs(got - ref) / scale))


@pytest.mark.parametrize("precision,n", [("fp32", 384), ("fp64", 306)])
def test_wide_3d_lattice_matches_oracle(precision, n):
    # 384^3 x 19 x 4 B = 4.30 GB and 306^3 x 19 x 8 B = 4.36 GB per buffer
    shape = (n, n, n)
    assert n ** 3 * 19 * (4 if precision == "fp32" else 8) >= 1 << 32
    p = fsc.make_params(D=3, nx=n, ny=n, nz=n, stencil=4, precision=precision, T_hat=0.8, rho0=0.62,
                        kBT=1e-6, seed=5)
    f0 = I.random_populations(19, shape, 0.62, 0.05, seed=8)
    with fsc.Lattice(p) as lat:
        lat.set_populations(f0, 77)
        lat.step(2)  # tunes over the single-step tilings first (a large lattice)
        tiling = lat.tiling
        got = lat.get_populations()
        G = lat.G
    print("tiling", tiling, flush=True)
    assert tiling["steps"] == 1
    ref = O.step(f0, 2, G=G, kind=4, kBT=1e-6, seed=5, t0=77)
    del f0
    assert np.isfinite(got).all()
    err = _max_rel(got, ref, 3, 0.62)
    tol = 1e-5 if precision == "fp32" else 1e-11
    assert err <= tol, f"max rel err {err:.3e}"


def test_wide_2d_lattice_runs_single_steps_only():
    n = 11008  # 11008^2 nodes x 9 x 4 B = 4.36 GB per buffer
    assert n * n * 9 * 4 >= 1 << 32
    p = fsc.make_params(D=2, nx=n, ny=n, stencil=4, precision="fp32", T_hat=0.8, rho0=0.62,
                        kBT=1e-6, seed=6)
    with fsc.Lattice(p) as lat:
        lat.init_uniform()
        with pytest.raises(fsc.FscError, match="4 GiB"):
            lat.set_tiling(256, 1, 1, 2, 741)
        lat.set_tiling(128, 1, 2, 1, 2048)
        lat.step(5)
        st = lat.stats()
    assert st["bad"] == 0 and st["nodes"] == n * n
    # the noise conserves mass: the total stays n0 N up to FP32 rounding
    assert abs(st["mass"] / (n * n * 0.62) - 1.0) < 1e-6
    assert 0.6 < st["rho_min"] <= st["rho_max"] < 0.64


def test_population_of_4gib_is_refused():
    # one population of 1100^3 FP32 values is 5.3 GB: refused before any allocation
    with pytest.raises(fsc.FscError, match="too large"):
        fsc.Lattice(fsc.make_params(D=3, nx=1100, ny=1100, nz=1100, stencil=4, precision="fp32",
                                    T_hat=0.8, rho0=0.62))
