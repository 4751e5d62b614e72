"""CPU reference of the learned surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate is a small CNN: four 3x3 convolutions with zero padding,
33 -> 32 -> 32 -> 32 -> 1 channels, ReLU after the first three, whose output
is added to the plain short-window estimate (y = est + CNN).  Its input at
output time t is, per pixel, the 32 binary frames t-31 .. t (channels 0..31,
channel j = frame t-31+j) and the plain short-window estimate (channel 32).

Parameters are one flat float vector (``NPARAMS``), in this order:
W1 [32][9][33], b1 [32], W2 [32][9][32], b2 [32], W3 [32][9][32], b3 [32],
W4 [1][9][32], b4 [1]; tap k = 3*dy + dx reads the input at offset
(dy - 1, dx - 1).

With ``bf16=True`` the reference rounds to bfloat16 (round to nearest even)
at exactly the points where the GPU kernels store bfloat16: weights, the
input channels, the activations after each ReLU, the loss gradient dL/dy
and the backpropagated gradients after each ReLU mask.  Everything else is
float64.  With ``bf16=False`` it is the plain float64 network (used for the
finite-difference and library cross-checks).
"""
from __future__ import annotations

import numpy as np

C_IN = 33
C = 32
SHAPES = [("W1", (C, 9, C_IN)), ("b1", (C,)), ("W2", (C, 9, C)), ("b2", (C,)),
          ("W3", (C, 9, C)), ("b3", (C,)), ("W4", (1, 9, C)), ("b4", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(params):
    params = np.asarray(params, dtype=np.float64)
    assert params.shape == (NPARAMS,)
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = params[off:off + n].reshape(shape)
        off += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _id(x):
    return np.asarray(x, dtype=np.float64)


def conv3x3(x, w, b=None):
    """Cross-correlation with zero padding: x [B,H,W,Cin], w [Cout,9,Cin]."""
    B, H, W, Ci = x.shape
    Co = w.shape[0]
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((B, H, W, Co))
    for k in range(9):
        dy, dx = divmod(k, 3)
        y += xp[:, dy:dy + H, dx:dx + W, :] @ w[:, k, :].T
    if b is not None:
        y += b
    return y


def conv3x3_input_grad(g, w):
    """Gradient of conv3x3 with respect to its input: g [B,H,W,Cout]."""
    B, H, W, Co = g.shape
    gp = np.zeros((B, H + 2, W + 2, Co))
    gp[:, 1:-1, 1:-1, :] = g
    dx_ = np.zeros((B, H, W, w.shape[2]))
    for k in range(9):
        dy, dx = divmod(k, 3)
        # x[p + off(k)] contributed g[p] * w[k]: shift g back by off(k)
        dx_ += gp[:, 2 - dy:2 - dy + H, 2 - dx:2 - dx + W, :] @ w[:, k, :]
    return dx_


def conv3x3_weight_grad(g, x):
    """Gradient of conv3x3 with respect to its weights: [Cout, 9, Cin]."""
    B, H, W, Ci = x.shape
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, :] = x
    gw = np.zeros((g.shape[3], 9, Ci))
    g2 = g.reshape(-1, g.shape[3])
    for k in range(9):
        dy, dx = divmod(k, 3)
        gw[:, k, :] = g2.T @ xp[:, dy:dy + H, dx:dx + W, :].reshape(-1, Ci)
    return gw


def make_input(win_bits, est, bf=True):
    """win_bits: uint32 [B,H,W] (bit j = frame t-31+j); est float [B,H,W]."""
    win = np.asarray(win_bits, dtype=np.uint64)
    chans = [((win >> j) & 1).astype(np.float64) for j in range(32)]
    e = np.asarray(est, dtype=np.float64)
    chans.append(bf16(e) if bf else e)
    return np.stack(chans, axis=-1)


def forward(params, x0, bf=True, est=None):
    """Returns (y [B,H,W], activations (a0, a1, a2, a3)).  ``est`` (the
    unrounded estimate) is added to the output when given."""
    r = bf16 if bf else _id
    p = unflatten(params)
    a0 = x0
    a1 = r(np.maximum(conv3x3(a0, r(p["W1"]), p["b1"]), 0.0))
    a2 = r(np.maximum(conv3x3(a1, r(p["W2"]), p["b2"]), 0.0))
    a3 = r(np.maximum(conv3x3(a2, r(p["W3"]), p["b3"]), 0.0))
    y = conv3x3(a3, r(p["W4"]), p["b4"])[..., 0]
    if est is not None:
        y = y + np.asarray(est, dtype=np.float64)
    return y, (a0, a1, a2, a3)


def loss_and_grad(params, x0, target, bf=True, est=None):
    """Mean squared error over all pixels and its gradient (flat, float64)."""
    r = bf16 if bf else _id
    p = unflatten(params)
    y, (a0, a1, a2, a3) = forward(params, x0, bf, est)
    n = y.size
    loss = float(np.mean((y - target) ** 2))
    g4 = r(2.0 * (y - target) / n)[..., None]                    # dL/dy
    grads = {"W4": conv3x3_weight_grad(g4, a3), "b4": g4.sum(axis=(0, 1, 2))}
    g3 = r(conv3x3_input_grad(g4, r(p["W4"])) * (a3 > 0))
    grads["W3"] = conv3x3_weight_grad(g3, a2)
    grads["b3"] = g3.sum(axis=(0, 1, 2))
    g2 = r(conv3x3_input_grad(g3, r(p["W3"])) * (a2 > 0))
    grads["W2"] = conv3x3_weight_grad(g2, a1)
    grads["b2"] = g2.sum(axis=(0, 1, 2))
    g1 = r(conv3x3_input_grad(g2, r(p["W2"])) * (a1 > 0))
    grads["W1"] = conv3x3_weight_grad(g1, a0)
    grads["b1"] = g1.sum(axis=(0, 1, 2))
    return loss, flatten(grads), y


def adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015) with bias correction; float64."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def psnr(x, ref, peak=1.0):
    mse = float(np.mean((np.asarray(x, np.float64) - np.asarray(ref, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(peak * peak / mse)
