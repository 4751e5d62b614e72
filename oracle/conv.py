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


# ---------------------------------------------------------------------------
# Layer-by-layer checks of an implementation that rounds at the same points
#
# A device implementation stores the same kinds of bfloat16 values as the
# bf16=True reference (weights, input channels, activations, dL/dy and the
# masked backpropagated gradients) but accumulates its sums in float32.
# Given the values it stored, every stored value and every output can be
# checked element by element against the float64 reference computed from the
# device's own inputs to that layer:
#   - a float32 sum of k terms lies within GAMMA(k) times the sum of the
#     terms' magnitudes of the exact sum (the standard bound k*eps/(1 - k*eps);
#     products of two bfloat16 values are exact in float32);
#   - a stored bfloat16 value is the round-to-nearest-even of such a sum, so
#     it lies between the roundings of the interval's two ends (rounding is
#     monotone); ReLU before rounding likewise.
# A layer whose input the device does not keep (the gradient into the third
# activation is overwritten by the next layer's) is carried as the interval
# of bfloat16 values it can hold.

def GAMMA(k):
    # eps = 2^-23 rather than the round-to-nearest 2^-24: the bound then also
    # holds for an accumulator that rounds toward zero
    e = 2.0 ** -23
    return k * e / (1.0 - k * e)


def _in_rounded_interval(dev, lo, hi):
    """dev (bfloat16 values) between the roundings of [lo, hi]."""
    return (dev >= bf16(lo)) & (dev <= bf16(hi))


def layer_checks(params, win, est, target, dev):
    """Checks every value the device stored or returned for one forward and
    backward pass.  ``dev`` holds, as float64 arrays in this module's layouts:
    a1, a2, a3 (activations, [B,H,W,32]), y ([B,H,W]), dy (dL/dy, [B,H,W]),
    g1, g2 (gradients into a1 and a2, after the ReLU mask, [B,H,W,32]) and
    grad (the flat parameter gradient); without dy only the forward values
    are checked.  Returns {name: number of elements outside their bound}
    (all zero for a correct implementation)."""
    p = unflatten(params)
    W = {k: bf16(p[k]) for k in ("W1", "W2", "W3", "W4")}
    aW = {k: np.abs(v) for k, v in W.items()}
    x0 = make_input(win, est, bf=True)
    est = np.asarray(est, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    res = {}
    # forward: each layer from the device's own input activation
    ins = {"a1": x0, "a2": dev["a1"], "a3": dev["a2"]}
    for l, name in ((1, "a1"), (2, "a2"), (3, "a3")):
        a_in = ins[name]
        z = conv3x3(a_in, W["W%d" % l], p["b%d" % l])
        e = GAMMA(9 * a_in.shape[-1] + 1) * conv3x3(np.abs(a_in), aW["W%d" % l],
                                                    np.abs(p["b%d" % l]))
        ok = _in_rounded_interval(dev[name], np.maximum(z - e, 0.0), np.maximum(z + e, 0.0))
        res[name] = int((~ok).sum())
    a3 = dev["a3"]
    y = conv3x3(a3, W["W4"], p["b4"])[..., 0] + est
    ey = GAMMA(9 * 32 + 2) * (conv3x3(a3, aW["W4"], np.abs(p["b4"]))[..., 0] + np.abs(est))
    res["y"] = int((np.abs(dev["y"] - y) > ey).sum())
    if "dy" not in dev:
        return res   # a forward pass only
    # dL/dy from the device's output: (y - t) and the division by n round
    n = dev["y"].size
    h = 2.0 * (dev["y"] - target) / n
    e = GAMMA(2) * np.abs(h)
    res["dy"] = int((~_in_rounded_interval(dev["dy"], h - e, h + e)).sum())
    g4 = dev["dy"][..., None]
    # gradient into a3 (not kept by the device): the interval of its values
    hh = conv3x3_input_grad(g4, W["W4"])
    e = GAMMA(9) * conv3x3_input_grad(np.abs(g4), aW["W4"])
    on3 = a3 > 0
    g3_lo, g3_hi = bf16((hh - e) * on3), bf16((hh + e) * on3)
    g3_mid, g3_rad = 0.5 * (g3_lo + g3_hi), 0.5 * (g3_hi - g3_lo)
    # gradient into a2 and a1 (kept), each from the layer above
    hh = conv3x3_input_grad(g3_mid, W["W3"])
    e = (conv3x3_input_grad(g3_rad, aW["W3"]) +
         GAMMA(9 * 32) * conv3x3_input_grad(np.abs(g3_mid) + g3_rad, aW["W3"]))
    on2 = dev["a2"] > 0
    res["g2"] = int((~_in_rounded_interval(dev["g2"], (hh - e) * on2, (hh + e) * on2)).sum())
    hh = conv3x3_input_grad(dev["g2"], W["W2"])
    e = GAMMA(9 * 32) * conv3x3_input_grad(np.abs(dev["g2"]), aW["W2"])
    on1 = dev["a1"] > 0
    res["g1"] = int((~_in_rounded_interval(dev["g1"], (hh - e) * on1, (hh + e) * on1)).sum())
    # parameter gradients: sums over all n pixels of stored gradients times
    # stored activations
    ref, bnd = {}, {}
    for l, g, g_rad, a_in in ((4, g4, 0.0, a3), (3, g3_mid, g3_rad, dev["a2"]),
                              (2, dev["g2"], 0.0, dev["a1"]), (1, dev["g1"], 0.0, x0)):
        ga = np.abs(g) + g_rad
        ref["W%d" % l] = conv3x3_weight_grad(g, a_in)
        bnd["W%d" % l] = (conv3x3_weight_grad(g_rad + 0 * g, np.abs(a_in)) +
                          GAMMA(n) * conv3x3_weight_grad(ga, np.abs(a_in)))
        ref["b%d" % l] = g.sum(axis=(0, 1, 2))
        bnd["b%d" % l] = (g_rad + 0 * g).sum(axis=(0, 1, 2)) + GAMMA(n) * ga.sum(axis=(0, 1, 2))
    gref, gbnd = flatten(ref), flatten(bnd)
    bad = np.abs(np.asarray(dev["grad"], dtype=np.float64) - gref) > gbnd
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in SHAPES])
    for (name, _), a, b in zip(SHAPES, offs[:-1], offs[1:]):
        res["grad_" + name] = int(bad[a:b].sum())
    return res
