"""Surrogate kernels against the CPU reference (oracle/conv.py, oracle window
estimate).

Window bits, the short-window estimate (float32 rounding of the oracle's
double) and the stability flag must match exactly.  Network outputs and
gradients: both sides use the same bfloat16-rounded weights, inputs,
activations and gradients; they differ by float32 versus float64
accumulation and, rarely, by one bfloat16 step where a float32 sum lands on
the other side of a rounding boundary than its float64 value.  The bounds
below allow a few such steps (bfloat16 has 8 significant bits, 2^-8 = 0.4%).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import oracle.conv as oc
import spkgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sur():
    import paper_2412_11639_amd.surrogate as m
    assert torch.cuda.is_available(), "no GPU"
    return m


def _samples(streams, rng, B, Hc, Wc, T):
    out = []
    for b in range(B):
        s, H, W = streams[b % len(streams)]
        out.append(dict(stream=s, H=H, W=W, T=T, oy=int(rng.integers(0, H - Hc + 1)),
                        ox=int(rng.integers(0, W - Wc + 1)), t=int(rng.integers(31, T))))
    return out


# (13, 29): 13 row tiles per crop, an odd count, so the last pair of tiles
# is half empty; (130, 70): two tiles per row, the second ragged, and 4160
# pairs of tiles, more than the launch's waves, so waves walk several with
# the next one's loads in flight
@pytest.mark.parametrize("B,Hc,Wc,H,W", [(8, 13, 29, (40, 33), (100, 70)),
                                         (32, 130, 70, (140, 133), (160, 90))])
def test_input_matches_oracle(sur, B, Hc, Wc, H, W):
    rng = np.random.default_rng(0)
    T = 300
    g = spkgen.gratings(H[0], W[0], T, seed=51)
    k = spkgen.blocks(H[1], W[1], T, seed=52, vx=0.4)
    streams = [(torch.from_numpy(g).cuda(), H[0], W[0]), (torch.from_numpy(k).cuda(), H[1], W[1])]
    targets = [torch.from_numpy(rng.random((h, w), dtype=np.float32)).cuda()
               for h, w in zip(H, W)]
    hosts = [g, k]
    samples = _samples(streams, rng, B, Hc, Wc, T)
    for b, s in enumerate(samples):
        s["target"] = targets[b % 2]
    win, est, st, tg = sur.Surrogate.input(samples, Hc, Wc, theta=2.0, with_target=True)
    win, est, st = win.cpu().numpy().view(np.uint32), est.cpu().numpy(), st.cpu().numpy()
    tg = tg.cpu().numpy()
    for b, s in enumerate(samples):
        host = hosts[b % 2]
        Hs, Ws = s["H"], s["W"]
        bits = spkgen.unpack(host[s["t"] - 31:s["t"] + 1], Hs, Ws).astype(np.uint64)
        ref_win = sum(bits[j] << np.uint64(j) for j in range(32)).astype(np.uint32)
        crop = (slice(s["oy"], s["oy"] + Hc), slice(s["ox"], s["ox"] + Wc))
        np.testing.assert_array_equal(win[b], ref_win[crop])
        e, stab = oracle.window_estimate(host, Hs, Ws, T, 2.0, s["t"])
        np.testing.assert_array_equal(est[b], e[crop].astype(np.float32))
        np.testing.assert_array_equal(st[b].astype(bool), stab[crop])
        np.testing.assert_array_equal(tg[b], targets[b % 2].cpu().numpy()[crop])


def test_stream_step_matches_input(sur):
    H, W, T = 24, 50, 120
    s = spkgen.gratings(H, W, T, seed=53)
    ds = torch.from_numpy(s).cuda()
    fb = spkgen.frame_bytes(H, W)
    win = torch.zeros((H, W), dtype=torch.int32, device="cuda")
    est = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    st = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    for t in range(T):
        sur.Surrogate.stream_step(ds[t], H, W, 1.0, win, est, st)
        if t >= 31 and t % 17 == 0:
            w2, e2, s2 = sur.Surrogate.input([dict(stream=ds, H=H, W=W, T=T, oy=0, ox=0, t=t)],
                                             H, W, 1.0)
            assert torch.equal(win, w2[0]) and torch.equal(est, e2[0]) and torch.equal(st, s2[0])


def _rand_batch(rng, B, Hc, Wc):
    win = rng.integers(0, 1 << 32, size=(B, Hc, Wc), dtype=np.uint64).astype(np.uint32)
    # sparser windows, like real ones
    win &= rng.integers(0, 1 << 32, size=(B, Hc, Wc), dtype=np.uint64).astype(np.uint32)
    est = rng.uniform(0, 1, size=(B, Hc, Wc)).astype(np.float32)
    return win, est


def _to_dev(win, est):
    return (torch.from_numpy(win.view(np.int32).copy()).cuda(), torch.from_numpy(est).cuda())


# (4, 176, 200): 572 16x16 tiles, more than the weight-gradient kernels'
# workgroups, so some walk two tiles with the second one's loads in flight
@pytest.mark.parametrize("shape", [(2, 16, 16), (3, 19, 37), (1, 64, 80), (2, 21, 35),
                                   (4, 176, 200)])
def test_every_stored_value_and_gradient_matches_reference(sur, shape):
    """One forward and backward pass, checked element by element: every
    activation, the output, dL/dy, the kept input gradients and every
    parameter gradient against the float64 reference computed from the
    device's own inputs to each layer, within the float32-accumulation and
    bfloat16-rounding bounds of oracle.conv.layer_checks."""
    rng = np.random.default_rng(3)
    B, Hc, Wc = shape
    print("surrogate layers B=%d Hc=%d Wc=%d" % shape, flush=True)
    params = sur.init_params(4) + rng.normal(0, 0.05, sur.NPARAMS)
    model = sur.Surrogate(params)
    win, est = _rand_batch(rng, B, Hc, Wc)
    target = rng.uniform(0, 1, size=(B, Hc, Wc)).astype(np.float32)
    dwin, dest = _to_dev(win, est)
    y = model.forward(dwin, dest)
    lp = model.backward(dwin, dest, y, torch.from_numpy(target).cuda())
    dev = {k: v.cpu().numpy().astype(np.float64) for k, v in model.stored(B, Hc, Wc).items()}
    dev["y"] = y.cpu().numpy().astype(np.float64)
    dev["grad"] = model.grad.cpu().numpy().astype(np.float64)
    p64 = model.params.cpu().numpy().astype(np.float64)
    res = oc.layer_checks(p64, win, est, target, dev)
    assert all(v == 0 for v in res.values()), res
    # diagnostics: loss, and the relative L2 distance per block from the
    # reference run on its own (float64 sums, its own roundings)
    loss_ref, g_ref, _ = oc.loss_and_grad(p64, oc.make_input(win, est.astype(np.float64), bf=True),
                                          target.astype(np.float64), bf=True,
                                          est=est.astype(np.float64))
    loss = float(lp.sum().cpu()) / target.size
    assert abs(loss - loss_ref) <= 1e-3 * loss_ref
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in oc.SHAPES])
    for (name, _), a, b in zip(oc.SHAPES, offs[:-1], offs[1:]):
        d = np.linalg.norm(dev["grad"][a:b] - g_ref[a:b]) / max(np.linalg.norm(g_ref[a:b]), 1e-30)
        print("  %s: relative L2 from the reference's own pass %.2e" % (name, d))


def test_streaming_loop_matches_oracle(sur):
    """The per-frame serving loop on a moving scene, 300 frames: advance the
    32-frame window by one frame, run the pre-packed inference, apply the
    fallback mux.  Every frame from 31 on: the window bits, the short-window
    estimate and the stability flag equal the oracle's
    (oracle.window_estimate on the stream), the mux output equals the
    select of the device's network output and the oracle's estimate by the
    oracle's flag, element by element; every 30th frame the network's
    stored activations and output pass the forward layer checks."""
    H, W, T = 48, 80, 300
    s = spkgen.blocks(H, W, T, seed=61, vx=0.9, vy=-0.6)
    ds = torch.from_numpy(s).cuda()
    bits = spkgen.unpack(s, H, W).astype(np.uint64)
    rng = np.random.default_rng(14)
    model = sur.Surrogate(sur.init_params(8) + rng.normal(0, 0.05, sur.NPARAMS))
    p64 = model.params.cpu().numpy().astype(np.float64)
    win = torch.zeros((1, H, W), dtype=torch.int32, device="cuda")
    est = torch.zeros((1, H, W), dtype=torch.float32, device="cuda")
    st = torch.zeros((1, H, W), dtype=torch.uint8, device="cuda")
    y = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    mx = torch.empty((1, H, W), dtype=torch.float32, device="cuda")
    n_stable = 0
    for t in range(T):
        sur.Surrogate.stream_step(ds[t], H, W, 1.0, win, est, st)
        if t < 31:
            continue
        model.infer(win, est, out=y, prepacked=t > 31)
        sur.Surrogate.mux(y, est, st, out=mx)
        torch.cuda.synchronize()
        e_ref, st_ref = oracle.window_estimate(s, H, W, T, 1.0, t)
        w_ref = sum(bits[t - 31 + j] << np.uint64(j) for j in range(32)).astype(np.uint32)
        w_got = win[0].cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(w_got, w_ref, err_msg="window t=%d" % t)
        e32 = e_ref.astype(np.float32)
        np.testing.assert_array_equal(est[0].cpu().numpy(), e32, err_msg="estimate t=%d" % t)
        np.testing.assert_array_equal(st[0].cpu().numpy().astype(bool), st_ref,
                                      err_msg="flag t=%d" % t)
        y_got = y[0].cpu().numpy()
        np.testing.assert_array_equal(mx[0].cpu().numpy(), np.where(st_ref, y_got, e32),
                                      err_msg="mux t=%d" % t)
        n_stable += int(st_ref.sum())
        if t % 30 == 0:
            dev = {k: v.cpu().numpy().astype(np.float64)
                   for k, v in model.stored(1, H, W).items() if k in ("a1", "a2", "a3")}
            dev["y"] = y.cpu().numpy().astype(np.float64)
            res = oc.layer_checks(p64, w_ref[None], e32[None], None, dev)
            assert all(v == 0 for v in res.values()), (t, res)
    # both branches of the mux were taken
    assert 0 < n_stable < H * W * (T - 31)


def test_adam_matches_reference(sur):
    rng = np.random.default_rng(5)
    p0 = rng.normal(0, 0.1, sur.NPARAMS)
    model = sur.Surrogate(p0)
    p, m, v = model.params.cpu().numpy().astype(np.float64), np.zeros(sur.NPARAMS), np.zeros(sur.NPARAMS)
    for step in range(1, 4):
        gr = rng.normal(0, 1e-2, sur.NPARAMS).astype(np.float32)
        model.grad.copy_(torch.from_numpy(gr))
        model.adam(lr=1e-3)
        p, m, v = oc.adam(p, m, v, gr.astype(np.float64), step, 1e-3)
    np.testing.assert_allclose(model.params.cpu().numpy(), p, rtol=0, atol=1e-6)


def test_mux(sur):
    y = torch.rand(1000, device="cuda")
    e = torch.rand(1000, device="cuda")
    s = (torch.rand(1000, device="cuda") > 0.5).to(torch.uint8)
    out = sur.Surrogate.mux(y, e, s)
    assert torch.equal(out, torch.where(s.bool(), y, e))


def test_training_reduces_loss_and_beats_short_window(sur):
    """A short training run on block scenes lowers the loss, and on held-out
    scenes the network's output is closer to the long-window plain result
    than the plain short-window estimate is."""
    scenes = sur.SceneSet([10000 + i for i in range(6)], H=96, W=128, T=1024,
                          target_times=(31, 500, 1023))
    held = sur.SceneSet([20000, 20001], H=96, W=128, T=1024, target_times=(31, 500, 1023))
    model = sur.Surrogate(seed=0)
    losses = sur.train(model, scenes, steps=300, B=16, Hc=48, Wc=48, lr=2e-3, seed=1,
                       log_every=50)
    assert losses[-1] < losses[0], losses
    rng = np.random.default_rng(7)
    err_net, err_est = [], []
    for _ in range(4):
        smp = held.samples(rng, 8, 64, 64)
        win, est, st, tgt = sur.Surrogate.input(smp, 64, 64, 1.0, with_target=True)
        y = model.forward(win, est)
        err_net.append(((y - tgt) ** 2).mean().item())
        err_est.append(((est - tgt) ** 2).mean().item())
    print("held-out MSE net %.3g est %.3g" % (np.mean(err_net), np.mean(err_est)))
    assert np.mean(err_net) < np.mean(err_est)


@pytest.mark.parametrize("shape", [(2, 16, 16), (3, 19, 37), (1, 70, 45), (1, 1, 5)])
def test_infer_equals_forward(sur, shape):
    """Inference gives the training forward's output bit for bit."""
    rng = np.random.default_rng(9)
    B, Hc, Wc = shape
    model = sur.Surrogate(sur.init_params(6) + rng.normal(0, 0.05, sur.NPARAMS))
    win, est = _to_dev(*_rand_batch(rng, B, Hc, Wc))
    y = model.forward(win, est).clone()
    yi = model.infer(win, est).clone()
    torch.cuda.synchronize()
    assert torch.equal(y, yi)


def test_prepacked_inference_equals_infer(sur):
    """spk_sur_infer_prepacked on new inputs, with the weights an earlier
    inference packed into the workspace, equals a full inference bit for
    bit."""
    rng = np.random.default_rng(12)
    B, Hc, Wc = 2, 19, 37
    model = sur.Surrogate(sur.init_params(7) + rng.normal(0, 0.05, sur.NPARAMS))
    model.infer(*_to_dev(*_rand_batch(rng, B, Hc, Wc)))
    for _ in range(2):
        win, est = _to_dev(*_rand_batch(rng, B, Hc, Wc))
        got = model.infer(win, est, prepacked=True).clone()
        ref = model.infer(win, est).clone()
        torch.cuda.synchronize()
        assert torch.equal(got, ref)


@pytest.mark.parametrize("shape", [(1, 70, 45), (2, 40, 100)])
def test_conv_block_walk_is_bit_identical(sur, shape):
    """Each convolution workgroup walks a contiguous range of 16x16 blocks,
    loading the next block's halo while it computes the current one.
    Capping the workgroups (one walks every block; several walk ranges
    that cross image boundaries; some get no block) leaves the forward
    output, inference and the gradient bit-identical to one block per
    workgroup."""
    import paper_2412_11639_amd as spk
    rng = np.random.default_rng(10)
    B, Hc, Wc = shape
    model = sur.Surrogate(sur.init_params(7) + rng.normal(0, 0.05, sur.NPARAMS))
    win, est = _to_dev(*_rand_batch(rng, B, Hc, Wc))
    target = torch.rand((B, Hc, Wc), device="cuda")
    res = {}
    for cap in (0, 1, 3, 7):
        spk.set_surrogate_conv_workgroups(cap)
        try:
            y = model.forward(win, est)
            model.backward(win, est, y, target)
            res[cap] = (y.clone(), model.grad.clone(), model.infer(win, est).clone())
        finally:
            spk.set_surrogate_conv_workgroups(0)
    torch.cuda.synchronize()
    for cap in (1, 3, 7):
        for k in range(3):
            assert torch.equal(res[cap][k], res[0][k]), (cap, k)


def test_train_plan_equals_eager_training(sur):
    """The graph-replayed training plan gives the eager loop's parameters and
    Adam moments bit for bit (same crops, learning rates and step numbers),
    including when its steps are run in several batches, and records each
    step's loss."""
    scenes = sur.SceneSet([10000, 10001], H=128, W=160, T=512, target_times=(31, 255, 511))
    B, Hc, Wc, steps = 4, 32, 48, 9
    eager = sur.Surrogate(seed=3)
    losses_e = sur.train(eager, scenes, steps=steps, B=B, Hc=Hc, Wc=Wc, lr=2e-3, seed=5,
                         log_every=1)
    graph = sur.Surrogate(seed=3)
    rng = np.random.default_rng(5)
    lrs = [2e-3 * 0.5 * (1 + math.cos(math.pi * k / steps)) for k in range(steps)]
    plan = sur.TrainPlan(graph, [scenes.samples(rng, B, Hc, Wc) for _ in range(steps)], lrs,
                         Hc, Wc)
    plan.run(2)
    plan.run(0)
    plan.run(steps - 2)
    with pytest.raises(Exception):
        plan.run(1)  # no steps left
    torch.cuda.synchronize()
    losses_g = plan.losses()
    plan.close()
    assert graph.step_count == eager.step_count == steps
    assert torch.equal(graph.params, eager.params)
    assert torch.equal(graph.m, eager.m)
    assert torch.equal(graph.v, eager.v)
    np.testing.assert_allclose(losses_g, losses_e, rtol=1e-5)


def test_checkpoint_resume_is_bit_exact(sur, tmp_path):
    """Training 8 steps straight through equals training 3, writing a
    checkpoint (parameters, Adam moments, step count and the crop sampler's
    random state), loading it into a fresh model and training 5 more: the
    parameters, both moments and every step's loss agree bit for bit."""
    scenes = sur.SceneSet([10000, 10001], H=96, W=128, T=512, target_times=(31, 255, 511))
    kw = dict(B=4, Hc=32, Wc=48, lr=2e-3, log_every=1, schedule_steps=8)
    straight = sur.Surrogate(seed=2)
    losses_a = sur.train(straight, scenes, 8, rng=np.random.default_rng(9), **kw)
    first = sur.Surrogate(seed=2)
    rng = np.random.default_rng(9)
    losses_b = sur.train(first, scenes, 3, rng=rng, **kw)
    path = str(tmp_path / "ckpt.npz")
    first.save(path, extra={"rng": rng.bit_generator.state})
    resumed, extra = sur.Surrogate.load(path)
    assert resumed.step_count == 3
    rng2 = np.random.default_rng()
    rng2.bit_generator.state = extra["rng"]
    losses_b += sur.train(resumed, scenes, 5, rng=rng2, **kw)
    torch.cuda.synchronize()
    assert losses_b == losses_a
    assert torch.equal(resumed.params, straight.params)
    assert torch.equal(resumed.m, straight.m)
    assert torch.equal(resumed.v, straight.v)
    assert resumed.step_count == straight.step_count == 8
