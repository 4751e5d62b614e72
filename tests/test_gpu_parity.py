"""Parity of the HIP reconstruction (through the C ABI) with the FP64 oracle.

Spike times, windows (first/last spike frame, interval count) and segment
lists must match bit for bit.  Intensities must agree within 1e-6 relative;
both sides evaluate theta*N/D in double precision and the library rounds it
once to float32, so they are in fact expected to be equal to the float32
rounding of the oracle's value.
"""
import numpy as np
import pytest
import torch

import oracle
import spkgen
from regimes import regime_stream
from test_oracle_pins import _read_golden, worked_example_stream

pytestmark = pytest.mark.gpu

REL_TOL = 1e-6


@pytest.fixture(scope="module")
def spk():
    import paper_2412_11639_amd as m
    assert torch.cuda.is_available(), "no GPU"
    return m


@pytest.fixture
def chunks(spk):
    yield spk.set_time_chunks
    spk.set_time_chunks(0)


@pytest.fixture
def warm(spk):
    yield spk.set_warm_tiles
    spk.set_warm_tiles(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_recon(spk, s, H, W, T, t_out, order, theta=1.0):
    print("recon H=%d W=%d T=%d n_out=%d order=%d" % (H, W, T, len(t_out), order), flush=True)
    ds = dev(s)
    out, wf, wl, wn = spk.reconstruct_windows(ds, H, W, T, theta, t_out, order=order)
    out2 = spk.reconstruct(ds, H, W, T, theta, t_out, order=order)
    torch.cuda.synchronize()
    ref, rf, rl, rn = oracle.reconstruct(s, H, W, T, theta, t_out, order=order, windows=True)
    np.testing.assert_array_equal(wf.cpu().numpy(), rf)
    np.testing.assert_array_equal(wl.cpu().numpy(), rl)
    np.testing.assert_array_equal(wn.cpu().numpy(), rn)
    o = out.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(o, ref, rtol=REL_TOL, atol=0)
    np.testing.assert_array_equal(out.cpu().numpy(), ref.astype(np.float32))
    np.testing.assert_array_equal(out2.cpu().numpy(), out.cpu().numpy())
    return out


def check_segments(spk, s, H, W, T, order, cap):
    print("segments H=%d W=%d T=%d order=%d" % (H, W, T, order), flush=True)
    sf, sl, sn, cnt = spk.segments(dev(s), H, W, T, order=order, cap=cap)
    torch.cuda.synchronize()
    rf, rl, rn, rc = oracle.segments(s, H, W, T, order=order, cap=cap)
    np.testing.assert_array_equal(cnt.cpu().numpy(), rc)
    np.testing.assert_array_equal(sf.cpu().numpy(), rf)
    np.testing.assert_array_equal(sl.cpu().numpy(), rl)
    np.testing.assert_array_equal(sn.cpu().numpy(), rn)
    # the same lists, each pixel's contiguous
    rec, cnt2 = spk.segments_packed(dev(s), H, W, T, order=order, cap=cap)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(cnt2.cpu().numpy(), rc)
    r = rec.cpu().numpy()
    np.testing.assert_array_equal(r[..., 0], rf.T)
    np.testing.assert_array_equal(r[..., 1], rl.T)
    np.testing.assert_array_equal(r[..., 2], rn.T)


def decode_both(spk, sf, sl, sn, cnt, H, W, T, t_out):
    """spk.decode on [cap][H*W] lists, checked equal (NaN where NaN) to
    spk.decode_packed on the same lists laid out per pixel."""
    got = spk.decode(sf, sl, sn, cnt, H, W, T, 1.0, t_out)
    rec = torch.stack((sf, sl, sn), dim=-1).transpose(0, 1).contiguous()
    got2 = spk.decode_packed(rec, cnt, H, W, T, 1.0, t_out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got2.cpu().numpy(), got.cpu().numpy())
    return got


@pytest.mark.parametrize("order", [1, 2])
def test_worked_example(spk, order):
    s, H, W, T = worked_example_stream()
    rows = [r for r in _read_golden() if r[0] == ("FSR" if order == 1 else "SSR")]
    t_out = [r[2] for r in rows]
    out = check_recon(spk, s, H, W, T, t_out, order).cpu().numpy()
    for k, (_, p, t, a, b, n, frac) in enumerate(rows):
        assert out[k, 0, p] == np.float32(float(frac))


@pytest.mark.parametrize("order", [1, 2])
def test_every_stream_of_12_frames(spk, order):
    T = 12
    n = 1 << T
    p = np.arange(n)
    bits = ((p[None, :] >> np.arange(T)[:, None]) & 1).astype(np.uint8)
    s = spkgen.pack(bits)
    check_segments(spk, s, 32, 128, T, order, cap=T)
    check_recon(spk, s, 32, 128, T, list(range(T)), order)


@pytest.mark.parametrize("order", [1, 2])
def test_blocks_250x400(spk, order):
    """Static 16x16 blocks, 250x400, 1024 frames, 8 outputs (+ first/last frame)."""
    H, W, T = 250, 400, 1024
    s = spkgen.blocks(H, W, T, seed=1)
    t_out = [64 + 128 * k for k in range(8)] + [0, T - 1]
    check_recon(spk, s, H, W, T, t_out, order)
    check_segments(spk, s, H, W, T, order, cap=4)


@pytest.mark.parametrize("order", [1, 2])
def test_gratings_ragged(spk, order):
    """Moving gratings + disk with Poisson noise; H*W and T not multiples of
    64; output times unsorted with duplicates."""
    H, W, T = 37, 91, 3001
    s = spkgen.gratings(H, W, T, seed=7)
    rng = np.random.default_rng(0)
    t_out = rng.integers(0, T, 300).tolist() + [0, 0, T - 1, 5, 5]
    check_recon(spk, s, H, W, T, t_out, order)
    check_segments(spk, s, H, W, T, order, cap=400)


@pytest.mark.parametrize("theta", [1e-44, 1.1754944e-38, 1e-30, 0.3, 255.0, 1e20, 3.4e38])
def test_intensity_extreme_theta(spk, theta):
    """Eq. 6 over the whole float range of theta (a subnormal, the smallest
    normal, the largest finite): the double quotient the kernels form,
    rounded once to float, is bit-identical to the oracle's division."""
    H, W, T = 19, 45, 1500
    s = spkgen.gratings(H, W, T, seed=17)
    th = float(np.float32(theta))
    for order, t_out in ((2, list(range(0, T, 23)) + [T - 1]), (1, list(range(5, T, 41)))):
        print("theta %g order %d" % (th, order), flush=True)
        out = spk.reconstruct(dev(s), H, W, T, th, t_out, order=order)
        torch.cuda.synchronize()
        ref = oracle.reconstruct(s, H, W, T, th, t_out, order=order)
        # bit for bit (results below the float normal range are subnormal,
        # so a relative bound does not apply to them)
        np.testing.assert_array_equal(out.cpu().numpy(), ref.astype(np.float32))


def _two_value_streams(rng, P, T, avals=tuple(range(1, 16)), group=15):
    """Per pixel an interval sequence over {a, a+1} (a from avals in turn):
    balanced (constant-rate) sequences, balanced ones with two neighbours
    swapped, i.i.d. ones and long runs, the kind changing every group
    pixels -- so the two values' S2 streams are stable over long stretches
    and then break at all kinds of places."""
    bits = np.zeros((T, P), dtype=np.uint8)
    for p in range(P):
        a = avals[p % len(avals)]
        kind = (p // group) % 4
        n = T // a + 2
        if kind == 0 or kind == 1:
            frac = rng.uniform(0.02, 0.98)
            ph = rng.uniform(0, 1)
            xs = a + (np.floor(frac * np.arange(1, n + 1) + ph)
                      - np.floor(frac * np.arange(n) + ph)).astype(int)
            if kind == 1:
                j = int(rng.integers(1, max(2, n - 2)))
                xs[j], xs[j + 1] = xs[j + 1], xs[j]
        elif kind == 2:
            xs = a + (rng.random(n) < rng.choice([0.1, 0.5, 0.9])).astype(int)
        else:
            xs = a + (np.arange(n) // int(rng.integers(1, 6)) % 2)
        tau = int(rng.integers(0, a + 1)) + np.concatenate([[0], np.cumsum(xs)])
        tau = tau[tau < T]
        bits[tau, p] = 1
    return bits


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_chunks", [0, 3, 24])
def test_two_value_words(spk, chunks, order, n_chunks):
    """Streams whose intervals take two adjacent values (the word-level SSR
    shortcut's domain), against the oracle, unchunked and chunked."""
    chunks(n_chunks)
    rng = np.random.default_rng(11)
    H, W, T = 6, 120, 1500
    bits = _two_value_streams(rng, H * W, T)
    s = spkgen.pack(bits)
    check_recon(spk, s, H, W, T, list(range(0, T, 7)) + [T - 1], order)
    check_segments(spk, s, H, W, T, order, cap=T)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_chunks", [0, 5])
def test_two_value_words_wide_gaps(spk, chunks, order, n_chunks):
    """As above with intervals up to 63 frames (the shortcut takes a <= 62)
    and one kind per 64-pixel strip, so whole waves take the word-level
    shortcut (balanced strips) or leave it (i.i.d. and run strips)."""
    chunks(n_chunks)
    rng = np.random.default_rng(12)
    H, W, T = 8, 128, 2500
    avals = tuple(range(1, 16)) + (16, 17, 21, 31, 32, 33, 40, 47, 60, 61, 62, 63)
    bits = _two_value_streams(rng, H * W, T, avals=avals, group=64)
    s = spkgen.pack(bits)
    check_recon(spk, s, H, W, T, list(range(0, T, 5)) + [T - 1], order)
    check_segments(spk, s, H, W, T, order, cap=T)


@pytest.mark.parametrize("order", [1, 2])
def test_moving_blocks(spk, order):
    H, W, T = 64, 80, 2048
    s = spkgen.blocks(H, W, T, seed=5, vx=0.7, vy=-0.4)
    check_recon(spk, s, H, W, T, list(range(0, T, 3)), order)
    check_segments(spk, s, H, W, T, order, cap=2048)


def test_edge_cases(spk):
    # one pixel, one frame
    s = spkgen.pack(np.ones((1, 1), dtype=np.uint8))
    check_recon(spk, s, 1, 1, 1, [0], 1)
    # pixels with 0, 1, 2 spikes; a pixel firing every frame; T = 65
    T = 65
    bits = np.zeros((T, 6), dtype=np.uint8)
    bits[40, 1] = 1
    bits[[3, 64], 2] = 1
    bits[:, 3] = 1
    bits[[0, 63, 64], 4] = 1
    bits[[63, 64], 5] = 1
    s = spkgen.pack(bits)
    for order in (1, 2, 3):
        check_recon(spk, s, 1, 6, T, list(range(T)), order)
        check_segments(spk, s, 1, 6, T, order, cap=T)
    # TFI with outputs on, between and before spikes, and words of one spike
    check_recon(spk, s, 1, 6, T, [0, 2, 3, 40, 41, 62, 63, 63, 64], 3)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_unsorted_duplicate_t_out_short_stream_and_no_outputs(spk, order):
    """t_out in any order with duplicates (plane k is always for t_out[k]),
    a stream shorter than one 64-frame tile, and n_out = 0."""
    H, W, T = 7, 45, 30
    s = spkgen.gratings(H, W, T, seed=71)
    check_recon(spk, s, H, W, T, [29, 0, 13, 13, 5, 29, 0], order)
    T = 700
    s = spkgen.blocks(H, W, T, seed=72, block=3, vx=0.3)
    check_recon(spk, s, H, W, T, [650, 3, 650, 64, 63, 0, 699, 128, 3], order)
    out = spk.reconstruct(dev(s), H, W, T, 1.0, [], order=order)
    torch.cuda.synchronize()
    assert tuple(out.shape) == (0, H, W)


def test_reconstruct_rejects_bad_t_out(spk):
    s = dev(np.zeros((4, 16), dtype=np.uint8))
    with pytest.raises(spk.SpkError):
        spk.reconstruct(s, 4, 4, 4, 1.0, [4])


@pytest.mark.parametrize("order", [1, 2])
def test_gratings_full_size_sampled(spk, order):
    """250x400, 20000 frames, every 10th frame out (the benchmark launch):
    the GPU computes all 2000 planes; 40 evenly spaced planes are checked
    against the oracle, element by element."""
    H, W, T = 250, 400, 20000
    s = _full_gratings()
    t_out = list(range(0, T, 10))
    print("full-size gratings order=%d" % order, flush=True)
    ds = dev(s)
    out = spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order)
    torch.cuda.synchronize()
    pick = list(range(0, len(t_out), 50))
    ref = oracle.reconstruct(s, H, W, T, 1.0, [t_out[k] for k in pick], order=order)
    got = out[pick].cpu().numpy()
    np.testing.assert_array_equal(got, ref.astype(np.float32))


_CACHE = {}


def _full_gratings():
    if "g" not in _CACHE:
        _CACHE["g"] = spkgen.gratings(250, 400, 20000, seed=2)
    return _CACHE["g"]


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_chunks", [2, 3, 7, 100])
def test_time_chunks_gratings(spk, chunks, order, n_chunks):
    """Time-chunked runs (speculative chunks + exact fixup) give the same
    result as the oracle for any chunk count, down to one tile per chunk."""
    chunks(n_chunks)
    H, W, T = 37, 91, 3001
    s = spkgen.gratings(H, W, T, seed=8)
    t_out = list(range(0, T, 7)) + [T - 1]
    check_recon(spk, s, H, W, T, t_out, order)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_warm", [1, 2])
@pytest.mark.parametrize("n_chunks", [3, 7])
def test_time_chunks_short_warmup(spk, chunks, warm, order, n_chunks, n_warm):
    """Chunks warmed up on one or two tiles start far from the true state;
    the fixup still makes the result exact."""
    chunks(n_chunks)
    warm(n_warm)
    H, W, T = 64, 128, 4096
    s = spkgen.gratings(H, W, T, seed=8)
    t_out = list(range(0, T, 9)) + [T - 1]
    check_recon(spk, s, H, W, T, t_out, order)


def _fsr_window_wider_than_warmup_stream(T=1024, W=64):
    """Every pixel: intervals 9 and 10 in turn (one FSR segment, window
    [9, 10]) up to frame 250, then only 10s, one 11 after frame 540, then
    10 and 11 in turn up to frame 800, then 13s.  Cut into 2 chunks of 8
    tiles, the second chunk's speculative state has seen only 10s in its 4
    warm-up tiles (window [10, 10]); the 11 cuts the true segment but not
    the speculative one, whose first cut (at the 13s) comes after the 4
    tiles in which the main pass records its window."""
    def train(off):
        t, s, k = off, [off], 0
        while t < 250:
            t += 9 if k % 2 == 0 else 10
            s.append(t)
            k += 1
        while t < 540:
            t += 10
            s.append(t)
        t += 11
        s.append(t)
        k = 0
        while t < 800:
            t += 10 if k % 2 == 0 else 11
            s.append(t)
            k += 1
        while t + 13 < T:
            t += 13
            s.append(t)
        return s
    bits = np.zeros((T, W), dtype=np.uint8)
    for p in range(W):
        bits[train(p % 5), p] = 1
    return spkgen.pack(bits)


@pytest.mark.parametrize("order", [1, 2])
def test_time_chunks_first_cut_after_capture_tiles(spk, chunks, order):
    """Default warm-up: the FSR fixup may not stop on the main pass's next
    cut when it has no record of the window up to that cut (regression: it
    stopped there and missed the true cut in between)."""
    T, W = 1024, 64
    s = _fsr_window_wider_than_warmup_stream(T, W)
    segs = oracle.segments(s, 1, W, T, order=1, cap=8)
    assert segs[0][1, 0] == 546 and segs[0][2, 0] == 809  # the true cuts
    chunks(2)
    check_recon(spk, s, 1, W, T, list(range(0, T, 4)) + [T - 1], order)


@pytest.mark.parametrize("case", range(48))
def test_time_chunks_random_regimes(spk, chunks, warm, case):
    """Random interval regimes, chunk counts, warm-up lengths and orders
    (TFI, FSR, SSR, third order) against the oracle."""
    rng = np.random.default_rng(1000 + case)
    T = int(rng.integers(700, 3500))
    W = 64 * int(rng.integers(1, 3)) - int(rng.integers(0, 9))
    order = [1, 2, 3, 4][case % 4]
    s = regime_stream(rng, T, W)
    chunks(int(rng.integers(2, 13)))
    warm(int(rng.integers(0, 6)))
    t_out = sorted(set(int(x) for x in rng.integers(0, T, 300))) + [T - 1]
    check_recon(spk, s, 1, W, T, t_out, order)


@pytest.mark.parametrize("case", range(12))
def test_segments_and_decode_random_regimes(spk, case):
    """Segment lists (both layouts) and their decode on random interval
    regimes, against the oracle."""
    rng = np.random.default_rng(2000 + case)
    T = int(rng.integers(300, 2500))
    W = int(rng.integers(30, 130))
    order = [1, 2, 4][case % 3]
    s = regime_stream(rng, T, W)
    cap = T
    check_segments(spk, s, 1, W, T, order, cap)
    sf, sl, sn, cnt = spk.segments(dev(s), 1, W, T, order=order, cap=cap)
    t_out = sorted(set(int(x) for x in rng.integers(0, T, 200))) + [T - 1]
    got = decode_both(spk, sf, sl, sn, cnt, 1, W, T, t_out).cpu().numpy()
    ref = oracle.reconstruct(s, 1, W, T, 1.0, t_out, order=order)
    np.testing.assert_array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_chunks", [4, 16])
def test_time_chunks_static_and_moving_blocks(spk, chunks, order, n_chunks):
    """Static blocks keep one segment across every chunk boundary (the fixup
    converges without a common cut); moving blocks cut often."""
    chunks(n_chunks)
    H, W, T = 48, 80, 2048
    check_recon(spk, spkgen.blocks(H, W, T, seed=21), H, W, T, list(range(0, T, 5)), order)
    check_recon(spk, spkgen.blocks(H, W, T, seed=22, vx=0.3, vy=0.2), H, W, T,
                list(range(3, T, 11)), order)


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("n_chunks", [2, 6, 16])
def test_time_chunks_constant_light_full_frame(spk, chunks, order, n_chunks):
    """The small static workload (250x400, 1024 frames, constant light per
    16x16 block) cut into chunks: the fixup takes words that cut neither
    the true nor the speculative machine whole, and its result equals the
    oracle and the unchunked run."""
    H, W, T = 250, 400, 1024
    s = spkgen.blocks(H, W, T, seed=1)
    t_out = [64 + 128 * k for k in range(8)] + [0, T - 1]
    chunks(0)
    ref = spk.reconstruct(dev(s), H, W, T, 1.0, t_out, order=order).cpu().numpy()
    chunks(n_chunks)
    out = check_recon(spk, s, H, W, T, t_out, order)
    np.testing.assert_array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("n_chunks", [5, 64])
def test_time_chunks_sparse_and_edge_pixels(spk, chunks, n_chunks):
    """Pixels whose first spike, or only spikes, fall in late chunks; chunks
    without any spike; unsorted output times with duplicates."""
    chunks(n_chunks)
    T = 64 * 64
    rng = np.random.default_rng(9)
    bits = np.zeros((T, 200), dtype=np.uint8)
    for p in range(200):
        kind = p % 5
        if kind == 0:
            continue                                   # no spike
        if kind == 1:
            bits[rng.integers(0, T), p] = 1            # one spike
        elif kind == 2:
            a, b = sorted(rng.integers(0, T, 2))
            bits[[a, b], p] = 1                        # two spikes far apart
        elif kind == 3:
            start = int(rng.integers(T // 2, T))       # spikes only late
            bits[start::int(rng.integers(1, 9)), p] = 1
        else:
            m = rng.random(T) < rng.uniform(0.01, 0.9)
            bits[m, p] = 1
    s = spkgen.pack(bits)
    t_out = rng.integers(0, T, 400).tolist() + [0, T - 1, T - 1]
    for order in (1, 2, 3):
        check_recon(spk, s, 1, 200, T, t_out, order)


# --------------------------------------------------------------------------
# the baselines (Sec. II): TFI as a third order, TFP windowed counts

@pytest.mark.parametrize("n_chunks", [0, 5])
def test_tfi_order(spk, chunks, n_chunks):
    chunks(n_chunks)
    H, W, T = 37, 91, 3001
    s = spkgen.gratings(H, W, T, seed=12)
    check_recon(spk, s, H, W, T, list(range(0, T, 5)) + [T - 1, 0], spk.TFI)
    check_segments(spk, s, H, W, T, spk.TFI, cap=T)
    s, H, W, T = worked_example_stream()
    check_recon(spk, s, H, W, T, list(range(T)), spk.TFI)


@pytest.mark.parametrize("window", [1, 7, 32, 64, 65, 300])
def test_tfp(spk, window):
    H, W, T = 33, 70, 700
    s = spkgen.gratings(H, W, T, seed=13)
    t_out = [0, 1, window - 1, window, T - 1, 350, 13] + list(range(2, T, 37))
    t_out = [t for t in t_out if 0 <= t < T]
    print("tfp window=%d n_out=%d" % (window, len(t_out)), flush=True)
    got = spk.tfp(dev(s), H, W, T, 1.5, window, t_out)
    torch.cuda.synchronize()
    ref = oracle.tfp(s, H, W, T, 1.5, window, t_out)
    np.testing.assert_array_equal(got.cpu().numpy(), ref.astype(np.float32))


# --------------------------------------------------------------------------
# segment encoding and its decoder

@pytest.mark.parametrize("order", [1, 2, 3])
def test_decode_of_segments_equals_reconstruct(spk, order):
    """Expanding the segment lists to frames gives exactly what the
    reconstruction writes from the stream (and so the oracle's values)."""
    H, W, T = 37, 91, 3001
    for s, h, w, T_ in ((spkgen.gratings(H, W, T, seed=14), H, W, T),
                        (spkgen.blocks(40, 64, 1500, seed=15, vx=0.6), 40, 64, 1500),
                        worked_example_stream()):
        ds = dev(s)
        t_out = list(range(0, T_, 3)) + [T_ - 1, 0, 0, 5]
        cnt = spk.segments(ds, h, w, T_, order=order, cap=0)[3]
        cap = max(1, int(cnt.max().item()))
        sf, sl, sn, cnt = spk.segments(ds, h, w, T_, order=order, cap=cap)
        got = decode_both(spk, sf, sl, sn, cnt, h, w, T_, t_out)
        ref = spk.reconstruct(ds, h, w, T_, 1.0, t_out, order=order)
        rec, cnt2 = spk.segments_packed(ds, h, w, T_, order=order, cap=cap)
        got2 = spk.decode_packed(rec, cnt2, h, w, T_, 1.0, t_out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
        np.testing.assert_array_equal(got2.cpu().numpy(), ref.cpu().numpy())
        np.testing.assert_array_equal(
            got.cpu().numpy(),
            oracle.reconstruct(s, h, w, T_, 1.0, t_out, order=order).astype(np.float32))


def test_decode_of_cut_lists_is_nan_past_cap(spk):
    """With lists cut at cap, outputs held by a stored segment decode to the
    oracle's value and later ones to NaN."""
    H, W, T = 20, 50, 2000
    s = spkgen.gratings(H, W, T, seed=16)
    t_out = list(range(0, T, 11))
    cap = 5
    sf, sl, sn, cnt = spk.segments(dev(s), H, W, T, order=2, cap=cap)
    got = decode_both(spk, sf, sl, sn, cnt, H, W, T, t_out).cpu().numpy().reshape(len(t_out), -1)
    ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=2).astype(np.float32)
    ref = ref.reshape(len(t_out), -1)
    rl = oracle.segments(s, H, W, T, order=2, cap=cap)[1]          # last spike of stored segments
    rc = oracle.segments(s, H, W, T, order=2, cap=cap)[3]
    for p in range(H * W):
        reach = rl[min(cap, rc[p]) - 1, p] if rc[p] > 0 else None
        for k, t in enumerate(t_out):
            if rc[p] <= cap or t <= reach:
                assert got[k, p] == ref[k, p], (p, t)
            else:
                assert np.isnan(got[k, p]), (p, t)


@pytest.mark.parametrize("order_name", ["FSR", "SSR", "TSR"])
def test_decode_every_frame_short_segments(spk, order_name):
    """Outputs at every frame over pixels whose segments last from one frame
    to hundreds (up to 16 segment boundaries inside one 32-frame tile of
    outputs); evenly spaced output times in both directions and at a stride,
    a single time, and shuffled times with repeats; a ragged last wave of
    pixels and a ragged last tile: decode equals reconstruct and the
    oracle."""
    order = getattr(spk, order_name)
    rng = np.random.default_rng(41)
    H, W, T = 3, 69, 701
    P = H * W
    # four kinds of pixel: i.i.d. spikes (probability from dense to sparse),
    # a fixed rate with occasional jumps, intervals alternating 1, 3 (a
    # segment boundary at every spike: 16 in a 32-frame tile) and intervals
    # i.i.d. over {a, a+1}, a = 2..4
    prob = rng.uniform(0.03, 0.95, size=P)
    bits = np.zeros((T, P), dtype=np.uint8)
    for p in range(P):
        if p % 4 == 0:
            bits[:, p] = rng.random(T) < prob[p]
            continue
        if p % 4 == 1:
            step = max(1, int(round(1 / prob[p])))
            gaps = step + np.where(rng.random(T) < 0.2, rng.integers(-1, 2, size=T), 0)
        else:
            if p % 4 == 2:
                gaps = 1 + 2 * ((np.arange(T) + p // 4) % 2)
            else:
                gaps = int(rng.integers(2, 5)) + (rng.random(T) < 0.5)
        t = int(rng.integers(0, 3))
        for g in gaps:
            if t >= T:
                break
            bits[t, p] = 1
            t += max(1, int(g))
    s = spkgen.pack(bits)
    ds = dev(s)
    cnt = spk.segments(ds, H, W, T, order=order, cap=0)[3]
    cap = max(1, int(cnt.max().item()))
    sf, sl, sn, cnt = spk.segments(ds, H, W, T, order=order, cap=cap)
    every = list(range(T))
    shuffled = [int(t) for t in rng.permutation(T)] + [0, T - 1, 17]
    ref_all = oracle.reconstruct(s, H, W, T, 1.0, every, order=order).astype(np.float32)
    # evenly spaced (ascending, descending, stride 7, one time) and not
    for t_out in (every, every[5:-3], every[::-1], every[2::7], [T // 2], shuffled):
        got = decode_both(spk, sf, sl, sn, cnt, H, W, T, t_out)
        ref = spk.reconstruct(ds, H, W, T, 1.0, t_out, order=order)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), ref.cpu().numpy())
        np.testing.assert_array_equal(got.cpu().numpy().reshape(len(t_out), -1),
                                      ref_all.reshape(T, -1)[t_out])


def test_decode_packed_window_edges(spk):
    """The per-pixel decoder holds 8 records of a list in registers and
    refills them in bursts: lists cut at every cap from 1 to 19 (shorter
    than, equal to and just past one or two windows) and pixels whose
    lists end at every length decode exactly as the [cap][H*W] decoder
    (NaN where NaN) and, where not cut, as the oracle."""
    rng = np.random.default_rng(77)
    H, W, T = 5, 41, 900
    P = H * W
    bits = np.zeros((T, P), dtype=np.uint8)
    for p in range(P):
        # segment counts from 0 to about 40: a fixed rate with a jump every
        # 20 + p frames (each jump can cut a segment)
        step = 2 + p % 5
        t, k = int(rng.integers(0, 3)), 0
        stop = int(rng.integers(0, T))
        while t < stop:
            bits[t, p] = 1
            k += 1
            t += step + (3 if k % (4 + p % 7) == 0 else 0)
    s = spkgen.pack(bits)
    ds = dev(s)
    t_out = list(range(0, T, 3))
    cnt = spk.segments(ds, H, W, T, order=spk.SSR, cap=0)[3]
    counts = cnt.cpu().numpy()
    assert counts.max() > 19 and (counts == 0).any()
    ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=2).astype(np.float32)
    ref = ref.reshape(len(t_out), -1)
    for cap in list(range(1, 20)) + [int(counts.max())]:
        print("decode window cap=%d" % cap, flush=True)
        rec, c2 = spk.segments_packed(ds, H, W, T, order=spk.SSR, cap=cap)
        got = spk.decode_packed(rec, c2, H, W, T, 1.0, t_out).cpu().numpy().reshape(len(t_out), -1)
        sf, sl, sn, c3 = spk.segments(ds, H, W, T, order=spk.SSR, cap=cap)
        want = spk.decode(sf, sl, sn, c3, H, W, T, 1.0, t_out).cpu().numpy().reshape(len(t_out), -1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got, want)
        whole = counts <= cap
        np.testing.assert_array_equal(got[:, whole], ref[:, whole])


def test_decode_with_no_stored_segments(spk):
    """Lists taken with cap 0 (no records at all): a pixel that has segments
    decodes to NaN at every requested frame, one with fewer than two spikes
    to 0, as the oracle gives for it."""
    H, W, T = 9, 37, 600
    bits = spkgen.unpack(spkgen.gratings(H, W, T, seed=21), H, W).reshape(T, H * W).copy()
    bits[:, :5] = 0                    # dark pixels
    bits[:, 5:8] = 0
    bits[T // 2, 5:8] = 1              # one spike each
    s = spkgen.pack(bits)
    ds = dev(s)
    t_out = list(range(0, T, 7)) + [T - 1, 3]
    for order in (spk.FSR, spk.SSR, spk.TSR):
        sf, sl, sn, cnt = spk.segments(ds, H, W, T, order=order, cap=0)
        got = decode_both(spk, sf, sl, sn, cnt, H, W, T, t_out).cpu().numpy().reshape(len(t_out), -1)
        c = cnt.cpu().numpy().reshape(-1)
        assert (c[:8] == 0).all() and (c[8:] > 0).all()
        assert (got[:, :8] == 0).all()
        assert np.isnan(got[:, 8:]).all()
        ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order).reshape(len(t_out), -1)
        assert (ref[:, :8] == 0).all()


# --------------------------------------------------------------------------
# the third order (n-order rule one step past SSR)

@pytest.mark.parametrize("n_chunks", [0, 3, 24])
def test_third_order(spk, chunks, n_chunks):
    chunks(n_chunks)
    H, W, T = 37, 91, 3001
    s = spkgen.gratings(H, W, T, seed=17)
    check_recon(spk, s, H, W, T, list(range(0, T, 5)) + [T - 1, 0], spk.TSR)
    check_segments(spk, s, H, W, T, spk.TSR, cap=T)
    rng = np.random.default_rng(18)
    bits = _two_value_streams(rng, 6 * 120, 1500)
    check_recon(spk, spkgen.pack(bits), 6, 120, 1500, list(range(0, 1500, 7)), spk.TSR)
    s = spkgen.blocks(48, 80, 2048, seed=19, vx=0.3, vy=0.2)
    check_recon(spk, s, 48, 80, 2048, list(range(3, 2048, 11)), spk.TSR)


def test_third_order_every_stream_of_12_frames(spk):
    T = 12
    n = 1 << T
    p = np.arange(n)
    bits = ((p[None, :] >> np.arange(T)[:, None]) & 1).astype(np.uint8)
    s = spkgen.pack(bits)
    check_segments(spk, s, 32, 128, T, spk.TSR, cap=T)
    check_recon(spk, s, 32, 128, T, list(range(T)), spk.TSR)


@pytest.mark.parametrize("n_chunks", [0, 7])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_motion_mask(spk, chunks, order, n_chunks):
    # the reconstruction pass writes the mask (chunked runs: the main pass
    # and the fixup pass both write it)
    chunks(n_chunks)
    for H, W, T in ((37, 91, 2500), (40, 96, 1500)):
        for s in (spkgen.blocks(H, W, T, seed=24, vx=0.4, vy=-0.2),
                  spkgen.gratings(H, W, T, seed=25)):
            t_out = list(range(0, T, 9)) + [T - 1, 3, 3]
            got = spk.motion(dev(s), H, W, T, 48, t_out, order=order)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got.cpu().numpy(),
                                          oracle.motion(s, H, W, T, 48, t_out, order=order))


@pytest.mark.parametrize("order", [1, 2])
def test_motion_mask_first_spike_edges(spk, order):
    # first spikes in every 64-frame chunk, in the ragged last chunk and at
    # the last frame, pixels that never fire or fire once, over a ragged
    # pixel count (the first-spike pass scans 64 frames per lane)
    H, W, T = 23, 57, 1000
    rng = np.random.default_rng(31)
    bits = spkgen.unpack(spkgen.blocks(H, W, T, seed=26, vx=0.3, vy=0.1), H, W).reshape(T, -1)
    bits = bits.copy()
    start = rng.integers(0, T, size=H * W)
    kind = rng.integers(0, 4, size=H * W)
    start[kind == 1] = T - 1 - rng.integers(0, 8, size=int((kind == 1).sum()))
    for p in range(H * W):
        bits[:start[p], p] = 0
        if kind[p] == 2:
            bits[:, p] = 0
        elif kind[p] == 3:
            bits[:, p] = 0
            bits[start[p], p] = 1
    s = spkgen.pack(bits)
    t_out = list(range(0, T, 7)) + [T - 1, 0]
    got = spk.motion(dev(s), H, W, T, 40, t_out, order=order)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(),
                                  oracle.motion(s, H, W, T, 40, t_out, order=order))
