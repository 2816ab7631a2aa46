"""GPU kernels of the learned surrogate against the FP64 reference.

BF16 operands with FP32 accumulation: outputs and gradients are compared
norm-wise with a few-percent tolerance (BF16 keeps 8 mantissa bits, so each
operand carries up to 2^-9 relative error; sums of hundreds of products with
mixed signs keep the relative error of a whole field near 1e-2).
"""
import numpy as np
import pytest

import fsc_inputs as I
import oracle as O
from oracle import surrogate as S

pytestmark = pytest.mark.gpu

fsc = pytest.importorskip("paper_2212_07848_amd")
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_mfma_layout_probe():
    rng = np.random.default_rng(0)
    A = rng.integers(-4, 5, size=(16, 32)).astype(np.float32)
    B = rng.integers(-4, 5, size=(32, 16)).astype(np.float32)
    Cm = fsc.mfma_probe(A, B)
    assert np.array_equal(Cm, A @ B)


def test_coarsen_matches_block_means():
    shape = (64, 96)
    f = I.smooth_density_populations(9, shape, 1.0, 0.2, 5, seed=3)
    p = fsc.make_params(D=2, nx=96, ny=64, rho0=1.0)
    out = torch.zeros((64 // 8, 96 // 8), dtype=torch.float32, device="cuda")
    with fsc.Lattice(p) as lat:
        lat.set_populations(f, 0)
        lat.coarsen(8, out)
        torch.cuda.synchronize()
    rho = O.density(f)
    ref = rho.reshape(8, 8, 12, 8).mean(axis=(1, 3))
    assert np.abs(out.cpu().numpy() - ref).max() < 2e-6


def test_field_structure_factor_and_length():
    rng = np.random.default_rng(5)
    fields = 1.0 + 0.1 * rng.normal(size=(3, 64, 64))
    shells, L = fsc.field_sk(_dev(fields), 3, 64)
    for b in range(3):
        f32 = fields[b].astype(np.float32).astype(np.float64)
        ref = O.shell_means(f32)
        assert np.allclose(shells[b], ref, rtol=1e-4, atol=1e-4 * ref.max())
        assert L[b] == pytest.approx(O.domain_length(f32), rel=1e-4)


def _net(seed, C=32, L=5):
    rng = np.random.default_rng(seed)
    p = S.init_params(C, L, seed)
    # non-zero biases so every term of the layers is exercised
    o = 0
    for co, ci in S.layer_shapes(C, L):
        o += co * ci * 9
        p[o:o + co] = 0.1 * rng.normal(size=co)
        o += co
    return p


@pytest.mark.parametrize("layers", [3, 5])
def test_forward_matches_reference(layers):
    rng = np.random.default_rng(1)
    B, H, W = 2, 32, 64
    p = _net(2, L=layers)
    rho = 1.0 + 0.3 * rng.normal(size=(B, H, W))
    sur = fsc.Surrogate(layers, H, W, B, seed=0)
    sur.set_params(p)
    sur.set_norm(1.0, 0.3, 0.05)
    x = _dev(rho)
    out = torch.zeros_like(x)
    sur.forward(x, out, B)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    ref = S.forward(p.astype(np.float32).astype(np.float64), rho.astype(np.float32), 32, layers,
                    1.0, 0.3, 0.05)
    inc_got = (got - rho.astype(np.float32)) / 0.05
    inc_ref = (ref - rho.astype(np.float32)) / 0.05
    err = np.linalg.norm(inc_got - inc_ref) / np.linalg.norm(inc_ref)
    print("relative increment error", err)
    assert err < 3e-2
    # each image's mean is conserved
    assert np.abs(got.mean(axis=(1, 2)) - rho.astype(np.float32).mean(axis=(1, 2))).max() < 1e-5
    sur.close()


def test_gradient_matches_reference():
    rng = np.random.default_rng(3)
    B, H, W, layers = 2, 32, 32, 5
    p = _net(4, L=layers).astype(np.float32)
    rho = (1.0 + 0.3 * rng.normal(size=(B, H, W))).astype(np.float32)
    tgt = (rho + 0.05 * rng.normal(size=rho.shape)).astype(np.float32)
    sur = fsc.Surrogate(layers, H, W, B, seed=0)
    sur.set_params(p)
    sur.set_norm(1.0, 0.3, 0.05)
    loss, g = sur.grad(_dev(rho), _dev(tgt), B)
    ref_loss, ref_g = S.loss_and_grad(p.astype(np.float64), rho, tgt, 32, layers, 1.0, 0.3, 0.05)
    assert loss == pytest.approx(ref_loss, rel=2e-2)
    o = 0
    scale = np.linalg.norm(ref_g)
    for l, (co, ci) in enumerate(S.layer_shapes(32, layers)):
        n = co * ci * 9
        for part, sl in (("W", slice(o, o + n)), ("b", slice(o + n, o + n + co))):
            gr, rr = g[sl].astype(np.float64), ref_g[sl]
            if l == layers - 1 and part == "b":
                # the mean-free output makes the loss independent of the last bias
                assert np.abs(rr).max() < 1e-12 * scale and np.abs(gr).max() < 1e-6 * scale
                continue
            err = np.linalg.norm(gr - rr) / max(np.linalg.norm(rr), 1e-30)
            print(f"layer {l} {part}: rel err {err:.3e}")
            assert err < 5e-2, (l, part, err)
        o += n + co
    sur.close()


def test_training_reduces_the_loss():
    # learn one explicit diffusion step rho' = rho + 0.1 lap(rho) on random fields
    rng = np.random.default_rng(7)
    B, H, W, layers = 8, 32, 32, 4

    def lap(r):
        return (np.roll(r, 1, 1) + np.roll(r, -1, 1) + np.roll(r, 1, 2) + np.roll(r, -1, 2)
                - 4 * r)

    sur = fsc.Surrogate(layers, H, W, B, seed=11)
    sur.set_norm(1.0, 0.3, 0.03)
    first = last = None
    for it in range(300):
        rho = 1.0 + 0.3 * rng.normal(size=(B, H, W))
        tgt = rho + 0.1 * lap(rho)
        loss = sur.train_step(_dev(rho), _dev(tgt), B, 2e-3)
        if it == 0:
            first = loss
        last = loss
    print("loss", first, "->", last)
    assert last < 0.1 * first
    sur.close()
