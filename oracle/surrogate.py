"""FP64 reference of the learned coarse-grained surrogate (test infrastructure).

The surrogate advances the block-averaged density of a phase-separating run
by a fixed number of lattice steps.  It is not part of the paper; its
definition (the library's own) is:

  x_0    = (rho - mean) / in_scale                          input normalisation
  x_1    = (rho - prev) / out_scale                         last increment (K = 2)
  a_0    = SiLU(conv(x; W_0, b_0))                          K -> C channels
  a_l    = SiLU(conv(a_{l-1}; W_l, b_l)),  l = 1 .. L-2     C -> C
  y      = conv(a_{L-2}; W_{L-1}, b_{L-1})                  C -> 1
  yhat   = y - <y>_image                                    mean-free increment
  rho'   = rho + out_scale * yhat                           conserves the mean

rho is the coarse field at time t, prev the one a stride earlier and rho' the
prediction a stride later; K = 1 networks see rho only.

conv is a 3x3 cross-correlation with circular padding (the lattice is
periodic); SiLU(z) = z / (1 + exp(-z)).  Training loss: mean over pixels and
batch of (yhat - (target - rho) / out_scale)^2.

Parameters are one flat float vector, per layer: weights [C_out][C_in][3][3]
then biases [C_out].

With bf16=True, forward and loss_and_grad round to bfloat16 (round to nearest,
ties to even, of the FP32 value) exactly the operands the library keeps in
that format, and nothing else: the weights of the C -> C layers; the hidden
activations a_l = SiLU(z_l); and, in the backward pass, the pre-activation
gradients of the hidden layers.  The first and last layers' weights, the
pre-activations z, the input channels and all sums stay in (here) FP64.  The
result differs from the library only by its FP32 sums and SiLU, and by the
rare BF16 rounding that those move across a rounding boundary.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(channels: int, layers: int, in_ch: int = 1):
    shapes = []
    for l in range(layers):
        ci = in_ch if l == 0 else channels
        co = 1 if l == layers - 1 else channels
        shapes.append((co, ci))
    return shapes


def n_params(channels: int, layers: int, in_ch: int = 1) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(channels, layers, in_ch))


def unpack(params: np.ndarray, channels: int, layers: int, in_ch: int = 1):
    out = []
    o = 0
    for co, ci in layer_shapes(channels, layers, in_ch):
        W = params[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = params[o:o + co]
        o += co
        out.append((W, b))
    return out


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[n, o, y, x] = b[o] + sum_{c, ky, kx} W[o, c, ky, kx] x[n, c, y+ky-1, x+kx-1] (periodic)."""
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:]) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(2, 3))
            out += np.einsum("oc,ncyx->noyx", W[:, :, ky, kx], xs)
    return out


def conv3x3_input_grad(g: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3 with respect to its input."""
    out = np.zeros((g.shape[0], W.shape[1]) + g.shape[2:])
    for ky in range(3):
        for kx in range(3):
            t = np.einsum("oc,noyx->ncyx", W[:, :, ky, kx], g)
            out += np.roll(t, shift=(ky - 1, kx - 1), axis=(2, 3))
    return out


def conv3x3_weight_grad(g: np.ndarray, x: np.ndarray):
    dW = np.zeros((g.shape[1], x.shape[1], 3, 3))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(2, 3))
            dW[:, :, ky, kx] = np.einsum("noyx,ncyx->oc", g, xs)
    return dW, g.sum(axis=(0, 2, 3))


def bf16_round(x):
    """bfloat16 value nearest to float32(x), ties to even, as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 mantissa bits
    of an IEEE float32.  Rounding adds 0x7FFF plus the lowest kept bit to the
    32-bit pattern and truncates to the top 16 bits: below half an ulp rounds
    down, above rounds up, an exact half rounds to the even pattern; a carry
    out of the mantissa moves to the next binade and past the largest finite
    value to infinity.  NaN stays NaN (quiet); infinities and zeros keep their
    sign; float32 subnormals round on the same bit grid."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) & np.uint64(0xFFFF)
    nan = np.isnan(f)
    r = np.where(nan, ((b >> np.uint64(16)) | np.uint64(0x0040)) & np.uint64(0xFFFF), r)
    return (r.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """16-bit pattern of bf16_round(x)."""
    return (bf16_round(x).astype(np.float32).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def network_input(rho, prev, mean, in_scale, out_scale):
    rho = np.asarray(rho, dtype=np.float64)
    chans = [(rho - mean) / in_scale]
    if prev is not None:
        chans.append((rho - np.asarray(prev, dtype=np.float64)) / out_scale)
    return np.stack(chans, axis=1)


def _layers(params, channels, layers, in_ch, bf16):
    P = unpack(np.asarray(params, dtype=np.float64), channels, layers, in_ch)
    if bf16:
        # the C -> C layers' weights feed the matrix cores in bfloat16
        P = [(bf16_round(W) if 0 < l < layers - 1 else W, b) for l, (W, b) in enumerate(P)]
    return P


def forward(params, rho, channels, layers, mean, in_scale, out_scale, keep=False, prev=None,
            bf16=False):
    """rho (and prev for two-channel networks): [B, H, W] -> prediction [B, H, W]
    (and the intermediates).  bf16: round as the library does (module text)."""
    in_ch = 1 if prev is None else 2
    P = _layers(params, channels, layers, in_ch, bf16)
    x = network_input(rho, prev, mean, in_scale, out_scale)
    zs, acts = [], [x]
    a = x
    for l, (W, b) in enumerate(P):
        z = conv3x3(a, W, b)
        if l < layers - 1:
            zs.append(z)
            a = silu(z)
            if bf16:
                a = bf16_round(a)
            acts.append(a)
        else:
            y = z[:, 0]
    yhat = y - y.mean(axis=(1, 2), keepdims=True)
    pred = rho + out_scale * yhat
    if keep:
        return pred, dict(zs=zs, acts=acts, yhat=yhat, P=P)
    return pred


def loss_and_grad(params, rho, target, channels, layers, mean, in_scale, out_scale, prev=None,
                  bf16=False):
    rho = np.asarray(rho, dtype=np.float64)
    _, c = forward(params, rho, channels, layers, mean, in_scale, out_scale, keep=True, prev=prev,
                   bf16=bf16)
    r = (np.asarray(target, dtype=np.float64) - rho) / out_scale
    e = c["yhat"] - r
    M = e.size
    loss = float((e * e).mean())
    g = 2.0 * e / M
    g = g - g.mean(axis=(1, 2), keepdims=True)  # through the mean-free projection
    grads = []
    delta = g[:, None]
    P = c["P"]
    for l in range(layers - 1, -1, -1):
        W, _ = P[l]
        dW, db = conv3x3_weight_grad(delta, c["acts"][l])
        grads.append((dW, db))
        if l > 0:
            delta = conv3x3_input_grad(delta, W) * dsilu(c["zs"][l - 1])
            if bf16:
                # hidden pre-activation gradients are kept in bfloat16
                delta = bf16_round(delta)
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def init_params(channels: int, layers: int, seed: int, in_ch: int = 1) -> np.ndarray:
    """He-style uniform initialisation (the library's own initialiser is
    separate; tests pass parameters explicitly)."""
    rng = np.random.default_rng(seed)
    out = []
    for co, ci in layer_shapes(channels, layers, in_ch):
        bound = np.sqrt(6.0 / (ci * 9))
        out.append(rng.uniform(-bound, bound, size=co * ci * 9))
        out.append(np.zeros(co))
    return np.concatenate(out)
