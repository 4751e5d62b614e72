"""Pins of the surrogate's CPU reference (oracle/conv.py) and of the
short-window estimate (oracle.window_estimate).

The convolution, its gradients and Adam are checked against library
routines (torch float64 conv2d, autograd, torch.optim.Adam) and against
central finite differences; bfloat16 rounding against torch's conversion;
the window estimate against the plain oracle run on the 32-frame window as a
stream of its own (its definition)."""
import numpy as np
import pytest
import torch

import oracle
import oracle.conv as oc
import spkgen


def rand_params(rng, scale=0.1):
    return rng.normal(0, scale, oc.NPARAMS)


def rand_input(rng, B=2, H=6, W=7):
    win = rng.integers(0, 1 << 32, size=(B, H, W), dtype=np.uint64).astype(np.uint32)
    est = rng.uniform(0, 1, size=(B, H, W))
    return win, est


def torch_forward(params, x0):
    p = {k: torch.tensor(v) for k, v in oc.unflatten(params).items()}
    for k in p:
        p[k].requires_grad_(True)
    x = torch.tensor(x0).permute(0, 3, 1, 2)

    def w(name):  # [Cout, 9, Cin] -> [Cout, Cin, 3, 3]
        t = p[name]
        return t.reshape(t.shape[0], 3, 3, t.shape[2]).permute(0, 3, 1, 2)

    a = torch.relu(torch.nn.functional.conv2d(x, w("W1"), p["b1"], padding=1))
    a = torch.relu(torch.nn.functional.conv2d(a, w("W2"), p["b2"], padding=1))
    a = torch.relu(torch.nn.functional.conv2d(a, w("W3"), p["b3"], padding=1))
    y = torch.nn.functional.conv2d(a, w("W4"), p["b4"], padding=1)[:, 0]
    return y, p


def test_nparams():
    assert oc.NPARAMS == 28224 + 97


def test_forward_matches_torch_conv2d():
    rng = np.random.default_rng(0)
    params = rand_params(rng)
    win, est = rand_input(rng)
    x0 = oc.make_input(win, est, bf=False)
    y, _ = oc.forward(params, x0, bf=False)
    yt, _ = torch_forward(params, x0)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_gradient_matches_autograd():
    rng = np.random.default_rng(1)
    params = rand_params(rng)
    win, est = rand_input(rng)
    x0 = oc.make_input(win, est, bf=False)
    target = rng.uniform(0, 1, size=win.shape)
    loss, g, _ = oc.loss_and_grad(params, x0, target, bf=False)
    yt, p = torch_forward(params, x0)
    lt = torch.mean((yt - torch.tensor(target)) ** 2)
    lt.backward()
    gt = np.concatenate([p[name].grad.numpy().reshape(-1) for name, _ in oc.SHAPES])
    assert abs(loss - lt.item()) < 1e-12
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-13)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    params = rand_params(rng, 0.2)
    win, est = rand_input(rng, B=1, H=5, W=6)
    x0 = oc.make_input(win, est, bf=False)
    target = rng.uniform(0, 1, size=win.shape)
    _, g, _ = oc.loss_and_grad(params, x0, target, bf=False)
    # probe every block: a few weights and biases of each layer
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in oc.SHAPES])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):
        idx += rng.integers(a, b, size=min(6, b - a)).tolist()
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oc.loss_and_grad(pp, x0, target, bf=False)[0]
              - oc.loss_and_grad(pm, x0, target, bf=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 10, 10000), rng.uniform(-1e-3, 1e-3, 1000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oc.bf16(x), ref)
    assert oc.bf16(1.0 + 2 ** -8) == 1.0          # tie to even
    assert oc.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=50)
    grads = rng.normal(size=(5, 50))
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for s in range(5):
        p, m, v = oc.adam(p, m, v, grads[s], s + 1, 1e-2)
        pt.grad = torch.tensor(grads[s])
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_window_estimate_is_the_plain_method_on_the_window():
    """O-S: the estimate at t is O-1..O-7 (FSR) on the stream of frames
    t-31..t alone at its last frame; fewer than two spikes gives theta*K/32."""
    H, W, T = 12, 40, 400
    s = spkgen.gratings(H, W, T, seed=31)
    for t in (31, 77, 250, 399):
        est, stable = oracle.window_estimate(s, H, W, T, 2.0, t)
        sub = s[t - 31:t + 1]
        ref, wf, wl, wn = oracle.reconstruct(sub, H, W, 32, 2.0, [31], windows=True)
        bits = spkgen.unpack(sub, H, W)
        K = bits.sum(axis=0)
        segs = oracle.segments(sub, H, W, 32, cap=32)[3].reshape(H, W)
        np.testing.assert_array_equal(est[K >= 2], ref[0][K >= 2])
        np.testing.assert_array_equal(est[K < 2], 2.0 * K[K < 2] / 32.0)
        np.testing.assert_array_equal(stable, (K >= 2) & (segs == 1))


def test_window_estimate_constant_rate():
    """A constant-rate window is one stable segment; when the interval
    divides 32 the estimate is exact."""
    H, W, T = 1, 4, 64
    bits = np.zeros((T, 4), dtype=np.uint8)
    bits[0::4, 0] = 1        # interval 4
    bits[1::8, 1] = 1        # interval 8
    bits[[40], 2] = 1        # one spike in the window
    s = spkgen.pack(bits)
    est, stable = oracle.window_estimate(s, H, W, T, 1.0, 63)
    assert est[0, 0] == 0.25 and stable[0, 0]
    assert est[0, 1] == 0.125 and stable[0, 1]
    assert est[0, 2] == 1.0 / 32 and not stable[0, 2]
    assert est[0, 3] == 0.0 and not stable[0, 3]


# ---------------------------------------------------------------------------
# The layer-by-layer checks of oracle.conv.layer_checks, pinned against an
# independent float32 implementation (torch CPU conv2d and its gradient
# routines) that rounds to bfloat16 at the same storage points: every value
# it stores must pass, and planted mistakes in it must fail.

def _f32_network(params, win, est, target, mistake=None):
    """float32 forward and backward with bfloat16 storage (torch CPU).
    Returns the stored values in layer_checks' layout."""
    F = torch.nn.functional
    bf = lambda t: t.to(torch.bfloat16).to(torch.float32)   # round to nearest even
    p = {k: torch.tensor(v, dtype=torch.float32) for k, v in oc.unflatten(params).items()}

    def w(name):  # [Cout, 9, Cin] -> [Cout, Cin, 3, 3], bfloat16 values
        t = bf(p[name])
        return t.reshape(t.shape[0], 3, 3, t.shape[2]).permute(0, 3, 1, 2).contiguous()

    x0 = torch.tensor(oc.make_input(win, est, bf=True), dtype=torch.float32)
    x0 = x0.permute(0, 3, 1, 2).contiguous()
    acts, cur = [x0], x0
    for l in (1, 2, 3):
        cur = bf(torch.relu(F.conv2d(cur, w("W%d" % l), p["b%d" % l], padding=1)))
        if mistake == "act" and l == 2:
            cur[0, 3, 2, 2] += 0.25
        acts.append(cur)
    y = F.conv2d(cur, w("W4"), p["b4"], padding=1)[:, 0] + torch.tensor(est, dtype=torch.float32)
    n = y.numel()
    dy = bf(2.0 * (y - torch.tensor(target, dtype=torch.float32)) / n)
    g = dy[:, None]
    grads, kept = {}, {}
    for l in (4, 3, 2, 1):
        a_in = acts[l - 1]
        gw = torch.nn.grad.conv2d_weight(a_in, (g.shape[1], a_in.shape[1], 3, 3), g, padding=1)
        grads["W%d" % l] = gw.permute(0, 2, 3, 1).reshape(g.shape[1], 9, a_in.shape[1])
        grads["b%d" % l] = g.sum(dim=(0, 2, 3))
        if l == 1:
            break
        h = torch.nn.grad.conv2d_input(a_in.shape, w("W%d" % l), g, padding=1)
        mask = (a_in > 0).to(torch.float32)
        if mistake == "no_mask" and l == 3:
            mask = torch.ones_like(mask)
        g = bf(h * mask)
        kept[l - 1] = g
    flat = oc.flatten({k: v.double().numpy() for k, v in grads.items()})
    if mistake == "sign":
        flat[oc.NPARAMS // 2] *= -1.0
    if mistake == "tap":
        # a transposed tap in the first layer's weight gradient
        w1 = flat[:32 * 9 * 33].reshape(32, 9, 33)
        w1[:, [0, 2]] = w1[:, [2, 0]]
    nhwc = lambda t: t.permute(0, 2, 3, 1).double().numpy()
    return {"a1": nhwc(acts[1]), "a2": nhwc(acts[2]), "a3": nhwc(acts[3]),
            "y": y.double().numpy(), "dy": dy.double().numpy(), "g2": nhwc(kept[2]),
            "g1": nhwc(kept[1]), "grad": flat}


def _case(seed, B=2, H=12, W=17):
    rng = np.random.default_rng(seed)
    params = rand_params(rng, 0.08)
    win = rng.integers(0, 1 << 32, size=(B, H, W), dtype=np.uint64).astype(np.uint32)
    win &= rng.integers(0, 1 << 32, size=(B, H, W), dtype=np.uint64).astype(np.uint32)
    est = rng.uniform(0, 1, size=(B, H, W)).astype(np.float32)
    target = rng.uniform(0, 1, size=(B, H, W)).astype(np.float32)
    return params, win, est, target


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_float32_implementation_passes_layer_checks(seed):
    params, win, est, target = _case(seed)
    dev = _f32_network(params, win, est, target)
    res = oc.layer_checks(params, win, est, target, dev)
    assert all(v == 0 for v in res.values()), res


@pytest.mark.parametrize("mistake,where", [("sign", "grad_W2"), ("no_mask", "g2"),
                                           ("tap", "grad_W1"), ("act", "a2")])
def test_layer_checks_catch_planted_mistakes(mistake, where):
    params, win, est, target = _case(5)
    dev = _f32_network(params, win, est, target, mistake=mistake)
    res = oc.layer_checks(params, win, est, target, dev)
    assert res[where] > 0, res


def test_layer_checks_pass_the_reference_itself():
    """The float64 reference's own stored values pass (its sums are exact up
    to float64 rounding, far inside every bound)."""
    params, win, est, target = _case(7)
    x0 = oc.make_input(win, est, bf=True)
    p = oc.unflatten(params)
    y, (a0, a1, a2, a3) = oc.forward(params, x0, bf=True, est=est.astype(np.float64))
    n = y.size
    dy = oc.bf16(2.0 * (y - target) / n)
    g3 = oc.bf16(oc.conv3x3_input_grad(dy[..., None], oc.bf16(p["W4"])) * (a3 > 0))
    g2 = oc.bf16(oc.conv3x3_input_grad(g3, oc.bf16(p["W3"])) * (a2 > 0))
    g1 = oc.bf16(oc.conv3x3_input_grad(g2, oc.bf16(p["W2"])) * (a1 > 0))
    _, grad, _ = oc.loss_and_grad(params, x0, target.astype(np.float64), bf=True,
                                  est=est.astype(np.float64))
    dev = {"a1": a1, "a2": a2, "a3": a3, "y": y, "dy": dy, "g2": g2, "g1": g1, "grad": grad}
    res = oc.layer_checks(params, win, est, target, dev)
    assert all(v == 0 for v in res.values()), res
