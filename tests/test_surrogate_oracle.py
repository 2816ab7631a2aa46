"""Pins of the FP64 surrogate reference (oracle/surrogate.py)."""
import os

import numpy as np
import pytest

from oracle import surrogate as S


def test_conv3x3_is_the_periodic_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 5, 6))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    out = S.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            for y in range(5):
                for xx in range(6):
                    v = b[o]
                    for c in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                v += W[o, c, ky, kx] * x[n, c, (y + ky - 1) % 5, (xx + kx - 1) % 6]
                    assert out[n, o, y, xx] == pytest.approx(v, abs=1e-12)


def test_conv_adjoint_identity():
    # <conv(x) - b, g> = <x, conv^T(g)>
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 7, 5))
    g = rng.normal(size=(2, 4, 7, 5))
    W = rng.normal(size=(4, 3, 3, 3))
    lhs = (S.conv3x3(x, W, np.zeros(4)) * g).sum()
    rhs = (x * S.conv3x3_input_grad(g, W)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    C, L = 3, 4
    p = S.init_params(C, L, seed=3) + 0.05 * rng.normal(size=S.n_params(C, L))
    rho = 1.0 + 0.3 * rng.normal(size=(2, 6, 6))
    tgt = rho + 0.05 * rng.normal(size=rho.shape)
    kw = dict(channels=C, layers=L, mean=1.0, in_scale=0.3, out_scale=0.05)
    loss, g = S.loss_and_grad(p, rho, tgt, **kw)
    h = 1e-6
    idx = rng.choice(p.size, size=40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = S.loss_and_grad(p + e, rho, tgt, **kw)
        lm, _ = S.loss_and_grad(p - e, rho, tgt, **kw)
        assert g[i] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9)


def test_prediction_conserves_the_image_mean():
    rng = np.random.default_rng(4)
    C, L = 4, 5
    p = S.init_params(C, L, seed=5)
    rho = 1.0 + 0.3 * rng.normal(size=(3, 8, 8))
    pred = S.forward(p, rho, C, L, 1.0, 0.3, 0.1)
    assert np.allclose(pred.mean(axis=(1, 2)), rho.mean(axis=(1, 2)), atol=1e-14)
    assert S.n_params(32, 5) == 288 + 32 + 3 * (9216 + 32) + 288 + 1


def test_two_channel_gradient_matches_central_differences():
    rng = np.random.default_rng(6)
    C, L = 3, 3
    p = S.init_params(C, L, seed=7, in_ch=2) + 0.05 * rng.normal(size=S.n_params(C, L, 2))
    rho = 1.0 + 0.3 * rng.normal(size=(2, 5, 6))
    prev = rho + 0.05 * rng.normal(size=rho.shape)
    tgt = rho + 0.05 * rng.normal(size=rho.shape)
    kw = dict(channels=C, layers=L, mean=1.0, in_scale=0.3, out_scale=0.05, prev=prev)
    loss, g = S.loss_and_grad(p, rho, tgt, **kw)
    h = 1e-6
    # every first-layer weight of the second channel, plus a random sample
    first = [(o * 2 + 1) * 9 + k for o in range(C) for k in range(9)]
    idx = np.concatenate([first, rng.choice(p.size, size=20, replace=False)])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = S.loss_and_grad(p + e, rho, tgt, **kw)
        lm, _ = S.loss_and_grad(p - e, rho, tgt, **kw)
        assert g[i] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9)


def test_two_channel_network_reduces_to_one_channel():
    # zero weights on the increment channel: the same map as the K = 1 network
    rng = np.random.default_rng(8)
    C, L = 4, 4
    p1 = S.init_params(C, L, seed=9, in_ch=1)
    p2 = np.zeros(S.n_params(C, L, 2))
    W1 = p1[:C * 9].reshape(C, 1, 9)
    W2 = np.zeros((C, 2, 9))
    W2[:, 0] = W1[:, 0]
    p2[:C * 18] = W2.ravel()
    p2[C * 18:] = p1[C * 9:]
    rho = 1.0 + 0.3 * rng.normal(size=(2, 6, 7))
    prev = rho + 0.1 * rng.normal(size=rho.shape)
    a = S.forward(p1, rho, C, L, 1.0, 0.3, 0.1)
    b = S.forward(p2, rho, C, L, 1.0, 0.3, 0.1, prev=prev)
    assert np.allclose(a, b, rtol=0, atol=1e-14)
    assert S.n_params(32, 5, 2) == S.n_params(32, 5) + 288


# ------------------------------------------------------- bfloat16 rounding --
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bf16_cases():
    rows = []
    with open(os.path.join(GOLDEN, "bf16_rne_cases.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                f, b = line.split()[:2]
                rows.append((int(f, 16), int(b, 16)))
    return rows


def test_bf16_rounding_matches_the_hand_written_table():
    rows = _bf16_cases()
    assert len(rows) >= 30
    f = np.array([r[0] for r in rows], dtype=np.uint32).view(np.float32)
    got = S.bf16_bits(f)
    for (fb, want), g in zip(rows, got):
        if want & 0x7F80 == 0x7F80 and want & 0x7F:
            # any NaN pattern with the quiet bit is a NaN; the table's is the canonical one
            assert g & 0x7F80 == 0x7F80 and g & 0x7F, hex(fb)
        else:
            assert int(g) == want, (hex(fb), hex(int(g)), hex(want))


def test_bf16_rounding_is_nearest_with_ties_to_even_on_random_floats():
    # properties of round-to-nearest-even against exact rational arithmetic in
    # float64 (every float32 and every bfloat16 is exact in float64)
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64).astype(np.uint32)
    f = bits.view(np.float32)
    f = f[np.isfinite(f) & (np.abs(f) < 3.3e38)]
    r = S.bf16_round(f)
    x = f.astype(np.float64)
    # the result is a bfloat16: its low 16 bits are zero
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    # the neighbours one bfloat16 step on either side are no closer
    rb = r.astype(np.float32).view(np.uint32)
    up = (rb + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    dn = (rb - np.uint32(0x10000)).view(np.float32).astype(np.float64)
    ok = np.isfinite(up) & np.isfinite(dn) & (np.sign(up) == np.sign(r)) & (np.sign(dn) == np.sign(r)) & (r != 0)
    d0 = np.abs(x - r)
    assert np.all(d0[ok] <= np.abs(x - up)[ok])
    assert np.all(d0[ok] <= np.abs(x - dn)[ok])
    # on an exact tie the kept pattern is even
    tie = ok & ((d0 == np.abs(x - up)) | (d0 == np.abs(x - dn)))
    assert tie.sum() == 0 or np.all(((rb[tie] >> 16) & 1) == 0)
    # idempotent on its own results
    assert np.array_equal(S.bf16_round(r), r)


def test_bf16_forward_is_the_fp64_forward_with_rounded_operands():
    # bf16=True differs from FP64 by the relative size of a bfloat16 rounding
    # (2^-9 per operand, a few parts in 1e3 in the output), and equals it when
    # every rounded operand is already a bfloat16: with the hidden layers cut
    # to 0 weights and biases on a bfloat16 grid the activations SiLU(b) are
    # rounded once and the C -> 1 layer sees exactly those values.
    rng = np.random.default_rng(6)
    C, L = 4, 4
    p = S.init_params(C, L, seed=2) + 0.05 * rng.normal(size=S.n_params(C, L))
    rho = 1.0 + 0.3 * rng.normal(size=(2, 8, 8))
    kw = dict(channels=C, layers=L, mean=1.0, in_scale=0.3, out_scale=0.05)
    a = S.forward(p, rho, **kw)
    b = S.forward(p, rho, bf16=True, **kw)
    rel = np.abs(b - a).max() / np.abs(a - rho).max()
    assert 1e-4 < rel < 3e-2
    # rounding placement: zero the C -> C layers' weights so that the last
    # hidden activation is SiLU(bias), rounded to bfloat16 before the C -> 1 layer
    q = p.copy()
    o = 0
    shapes = S.layer_shapes(C, L)
    for l, (co, ci) in enumerate(shapes):
        n = co * ci * 9
        if 0 < l < L - 1:
            q[o:o + n] = 0.0
        o += n + co
    _, c = S.forward(q, rho, bf16=True, keep=True, **kw)
    bias_last_hidden = S.unpack(q, C, L)[L - 2][1]
    assert np.array_equal(c["acts"][L - 1][0, :, 0, 0], S.bf16_round(S.silu(bias_last_hidden)))
