"""Carry-state reconstruction on the GPU (spk_stream_*), through the C ABI:
frames fed in random pieces (single frames, empty pieces, pieces that end
inside a 64-frame tile and pieces longer than several tiles) must give,
after the finish, the single-pass spk_reconstruct output and the oracle's,
bit for bit, for every order, with windows; the oracle's own carry-state
form fed the same pieces agrees too."""
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


def _pieces(rng, T, kinds):
    cuts = [0]
    while cuts[-1] < T:
        k = kinds[len(cuts) % len(kinds)]
        step = {"one": 1, "empty": 0, "short": int(rng.integers(2, 64)),
                "long": int(rng.integers(64, 400))}[k]
        cuts.append(min(T, cuts[-1] + step))
    return cuts


@pytest.mark.parametrize("order_name", ["FSR", "SSR", "TFI", "TSR"])
@pytest.mark.parametrize("scene", ["gratings", "moving_blocks"])
def test_pieces_equal_single_pass_and_oracle(spk, order_name, scene):
    order = getattr(spk, order_name)
    rng = np.random.default_rng(hash((order_name, scene)) % 1000)
    H, W, T = 45, 131, 2500
    if scene == "gratings":
        s = spkgen.gratings(H, W, T, seed=91)
    else:
        s = spkgen.blocks(H, W, T, seed=92, vx=1.3, vy=0.4, block=8)
    ds = torch.from_numpy(s).cuda()
    t_out = [int(t) for t in rng.integers(0, T, 150)] + [0, T - 1, 7, 7]
    cuts = _pieces(rng, T, ["short", "one", "long", "empty", "short", "long"])
    print("stream %s %s: %d pieces" % (order_name, scene, len(cuts) - 1), flush=True)
    st = spk.Stream(H, W, 1.5, t_out, order=order, windows=True)
    for a, b in zip(cuts[:-1], cuts[1:]):
        st.feed(ds[a:b])
    assert st.frames() == T
    out, wf, wl, wn = st.finish()
    ref = spk.reconstruct_windows(ds, H, W, T, 1.5, t_out, order=order)
    torch.cuda.synchronize()
    for g, r in zip((out, wf, wl, wn), ref):
        assert torch.equal(g, r)
    o_out, o_wf, o_wl, o_wn = oracle.reconstruct(s, H, W, T, 1.5, t_out, order=order,
                                                 windows=True)
    np.testing.assert_array_equal(out.cpu().numpy(), o_out.astype(np.float32))
    np.testing.assert_array_equal(wf.cpu().numpy(), o_wf)
    np.testing.assert_array_equal(wl.cpu().numpy(), o_wl)
    np.testing.assert_array_equal(wn.cpu().numpy(), o_wn)
    st.close()


def test_live_camera_blocks_of_32(spk):
    """A 1000 x 1000 camera fed 32 frames at a time for 4096 frames, an
    output every 64th frame (SSR, no windows): equal to the single pass."""
    H, W, T = 1000, 1000, 4096
    s = spkgen.blocks(H, W, T, seed=5, vx=0.8, vy=-0.5)
    ds = torch.from_numpy(s).cuda()
    t_out = list(range(31, T, 64))
    st = spk.Stream(H, W, 1.0, t_out, order=spk.SSR)
    for a in range(0, T, 32):
        st.feed(ds[a:a + 32])
    out = st.finish()
    ref = spk.reconstruct(ds, H, W, T, 1.0, t_out, order=spk.SSR)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    st.close()


def test_silent_pixels_nothing_fed_and_late_outputs(spk):
    """No frames fed: every output 0 with window (-1, -1, 0).  Pixels that
    never fire or fire once: the same.  An output time past the frames fed
    takes the last segment, as the single pass with the stream extended by
    silent frames does."""
    H, W = 4, 70
    st = spk.Stream(H, W, 1.0, [0, 3], order=spk.SSR, windows=True)
    out, wf, wl, wn = st.finish()
    torch.cuda.synchronize()
    assert torch.all(out == 0) and torch.all(wf == -1) and torch.all(wl == -1)
    assert torch.all(wn == 0)
    st.close()
    T = 200
    bits = np.zeros((T, H, W), dtype=np.uint8)
    bits[::5, 0, :] = 1
    bits[17, 1, 3] = 1
    bits[[2, 9, 11, 40, 41], 2, 60:] = 1
    s = spkgen.pack(bits)
    ds = torch.from_numpy(s).cuda()
    st = spk.Stream(H, W, 1.0, [5, 150, 250], order=spk.FSR, windows=True)
    st.feed(ds[:100])
    st.feed(ds[100:])
    got = st.finish()
    longer = np.zeros((260, H, W), dtype=np.uint8)
    longer[:T] = bits
    dl = torch.from_numpy(spkgen.pack(longer)).cuda()
    ref = spk.reconstruct_windows(dl, H, W, 260, 1.0, [5, 150, 250], order=spk.FSR)
    torch.cuda.synchronize()
    for g, r in zip(got, ref):
        assert torch.equal(g, r)
    st.close()


@pytest.mark.parametrize("case", range(8))
def test_random_regimes_in_pieces(spk, case):
    """Random interval regimes (segments that outlast many pieces, windows
    that widen and narrow) fed in random pieces, every order, against the
    oracle."""
    rng = np.random.default_rng(3000 + case)
    T = int(rng.integers(500, 3000))
    W = int(rng.integers(20, 140))
    order = [spk.FSR, spk.SSR, spk.TFI, spk.TSR][case % 4]
    s = regime_stream(rng, T, W)
    ds = torch.from_numpy(s).cuda()
    t_out = [int(t) for t in rng.integers(0, T, 120)] + [0, T - 1]
    cuts = _pieces(rng, T, ["short", "long", "one", "short", "empty", "long"])
    print("regimes case %d: T=%d W=%d order=%d, %d pieces" % (case, T, W, order, len(cuts) - 1),
          flush=True)
    st = spk.Stream(1, W, 1.0, t_out, order=order, windows=True)
    for a, b in zip(cuts[:-1], cuts[1:]):
        st.feed(ds[a:b])
    out, wf, wl, wn = st.finish()
    torch.cuda.synchronize()
    o_out, o_wf, o_wl, o_wn = oracle.reconstruct(s, 1, W, T, 1.0, t_out, order=order,
                                                 windows=True)
    np.testing.assert_array_equal(out.cpu().numpy(), o_out.astype(np.float32))
    np.testing.assert_array_equal(wf.cpu().numpy(), o_wf)
    np.testing.assert_array_equal(wl.cpu().numpy(), o_wl)
    np.testing.assert_array_equal(wn.cpu().numpy(), o_wn)
