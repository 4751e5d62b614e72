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
