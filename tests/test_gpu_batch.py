"""Batched plans (persistent kernel in a HIP graph) against the oracle and
against single-stream calls."""
import numpy as np
import pytest
import torch

import oracle
import spkgen
from regimes import regime_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spk():
    import paper_2412_11639_amd as m
    assert torch.cuda.is_available(), "no GPU"
    return m


def make_jobs(order_seed=0, unsorted=False):
    rng = np.random.default_rng(order_seed)
    shapes = [(37, 91, 1500), (64, 64, 777), (20, 250, 2049), (1, 7, 300), (50, 80, 1024)]
    jobs = []
    for i, (H, W, T) in enumerate(shapes):
        if i % 2:
            s = spkgen.gratings(H, W, T, seed=100 + i)
        else:
            s = spkgen.blocks(H, W, T, seed=100 + i, vx=0.2 * i, vy=-0.1 * i)
        t_out = sorted(set(rng.integers(0, T, 40).tolist()))
        if unsorted and i == 2:
            t_out = rng.integers(0, T, 60).tolist() + [0, 0, T - 1]
        jobs.append(dict(np_stream=s, stream=torch.from_numpy(s).cuda(), H=H, W=W, T=T,
                         t_out=t_out, theta=1.0 + 0.5 * i))
    return jobs


def check_against_oracle(jobs, outs, order):
    for j, out in zip(jobs, outs):
        print("job H=%d W=%d T=%d" % (j["H"], j["W"], j["T"]), flush=True)
        ref = oracle.reconstruct(j["np_stream"], j["H"], j["W"], j["T"], j["theta"], j["t_out"],
                                 order=order)
        np.testing.assert_array_equal(out.cpu().numpy(), ref.astype(np.float32))


@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("unsorted", [False, True])
def test_plan_matches_oracle(spk, order, unsorted):
    jobs = make_jobs(1, unsorted)
    plan = spk.Plan(jobs, order=order, autotune=True)
    # autotuning ran the kernel into the outputs: clear them, so that only
    # the graph replay below can produce the compared values
    for o in plan.outputs():
        o.fill_(-1.0)
    torch.cuda.synchronize()
    plan.execute()
    torch.cuda.synchronize()
    info = plan.info()
    assert info["items"] == sum((j["H"] * j["W"] + 63) // 64 for j in jobs)
    assert info["grid"] > 0 and info["grab"] > 0
    check_against_oracle(jobs, plan.outputs(), order)
    plan.close()


@pytest.mark.parametrize("order", [1, 2])
def test_graph_replays_match_eager(spk, order):
    """Replay the captured graph several times with unrelated eager work and
    synchronisations in between; every replay equals the single-stream
    result."""
    jobs = make_jobs(2)
    eager = [spk.reconstruct(j["stream"], j["H"], j["W"], j["T"], j["theta"], j["t_out"],
                             order=order) for j in jobs]
    plan = spk.Plan(jobs, order=order, autotune=False)
    for rep in range(4):
        for o in plan.outputs():
            o.fill_(-1.0)
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        plan.execute()
        torch.cuda.synchronize()
        for o, e in zip(plan.outputs(), eager):
            assert torch.equal(o, e), "replay %d differs" % rep
        del junk
    plan.close()


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_every_launch_shape_is_bit_identical(spk, order):
    """Every launch shape the autotuner can pick -- tiles per prefetch group
    4, 8, 16; one, two or four waves per workgroup; both register targets
    -- gives the single-stream results bit for bit (jobs with ragged strips,
    unsorted outputs with repeats)."""
    jobs = make_jobs(4, unsorted=True)
    eager = [spk.reconstruct(j["stream"], j["H"], j["W"], j["T"], j["theta"], j["t_out"],
                             order=order) for j in jobs]
    try:
        for kg in (4, 8, 16):
            for wpg in (1, 2, 4):
                for wpe in (0, 1):
                    spk.set_plan_shape(kg, wpg, wpe)
                    plan = spk.Plan(jobs, order=order, autotune=False)
                    assert plan.shape()["kgroup"] == kg
                    assert plan.shape()["waves_per_wg"] == wpg
                    for o in plan.outputs():
                        o.fill_(-1.0)
                    plan.execute()
                    torch.cuda.synchronize()
                    for o, e in zip(plan.outputs(), eager):
                        assert torch.equal(o, e), (kg, wpg, wpe)
                    plan.close()
    finally:
        spk.set_plan_shape(0, 0, 0)


def test_plan_without_graph_and_shapes_agree(spk):
    jobs = make_jobs(3)
    a = spk.Plan(jobs, order=1, autotune=False, graph=False)
    a.execute()
    torch.cuda.synchronize()
    first = [o.clone() for o in a.outputs()]
    a.close()
    b = spk.Plan(jobs, order=1, autotune=True)
    for o in b.outputs():
        o.zero_()
    b.execute()
    torch.cuda.synchronize()
    for x, y in zip(first, b.outputs()):
        assert torch.equal(x, y)
    b.close()


def test_full_batched_workload(spk):
    """The whole batched workload: 16 streams of 4096 frames with sizes from
    250x400 to 1000x1000 and 64 outputs each, in one autotuned plan (SSR).
    Every stream's output is compared with the oracle bit for bit, on every
    pixel of 8 of its 64 planes (the oracle segments every pixel's whole
    stream either way)."""
    import time
    jobs = spkgen.batch_workload()
    hosts, dev_jobs = [], []
    t0 = time.time()
    for j in jobs:
        s = spkgen.blocks(j["H"], j["W"], j["T"], j["seed"])
        hosts.append(s)
        dev_jobs.append(dict(j, stream=torch.from_numpy(s).cuda()))
    print("generated %d streams in %.1f s" % (len(jobs), time.time() - t0), flush=True)
    plan = spk.Plan(dev_jobs, order=spk.SSR, autotune=True)
    for o in plan.outputs():
        o.fill_(-1.0)
    torch.cuda.synchronize()
    plan.execute()
    torch.cuda.synchronize()
    print("plan executed: %s %s" % (plan.info(), plan.shape()), flush=True)
    planes = list(range(0, 64, 9))
    for j, s, out in zip(jobs, hosts, plan.outputs()):
        t_pick = [j["t_out"][k] for k in planes]
        ref = oracle.reconstruct(s, j["H"], j["W"], j["T"], 1.0, t_pick, order=spk.SSR)
        got = out[planes].cpu().numpy()
        print("stream %dx%d seed %d" % (j["H"], j["W"], j["seed"]), flush=True)
        np.testing.assert_array_equal(got, ref.astype(np.float32))
    plan.close()


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_plan_random_regimes(spk, order):
    """A plan over streams of random interval regimes (several strips each,
    ragged widths) against the oracle."""
    rng = np.random.default_rng(4000 + order)
    jobs = []
    for i in range(5):
        H, W, T = int(rng.integers(1, 4)), int(rng.integers(20, 150)), int(rng.integers(300, 2500))
        # H rows of W pixels, each pixel its own regime train
        bits = np.concatenate([spkgen.unpack(regime_stream(rng, T, W), 1, W) for _ in range(H)],
                              axis=1)
        s = spkgen.pack(bits)
        t_out = sorted(set(rng.integers(0, T, 50).tolist()))
        jobs.append(dict(np_stream=s, stream=torch.from_numpy(s).cuda(), H=H, W=W, T=T,
                         t_out=t_out, theta=1.0))
    plan = spk.Plan(jobs, order=order)
    plan.execute()
    torch.cuda.synchronize()
    check_against_oracle(jobs, plan.outputs(), order)
    plan.close()
