"""Pins of the oracle's carry-state form (O-5): the method run online, the
stream fed in pieces with a small per-pixel state carried between them.
Feeding any split of a stream and finishing must give exactly the
whole-stream oracle's outputs and windows (which the brute-force pins in
test_oracle_pins.py tie to the paper's definitions), for every order:
every stream of 12 frames split at every frame, and longer generated
scenes cut into random pieces (empty pieces included)."""
import numpy as np
import pytest

import oracle
import spkgen

ORDERS = [oracle.FSR, oracle.SSR, oracle.TFI, oracle.TSR]


def _all_streams(T):
    n = 1 << T
    p = np.arange(n)
    bits = ((p[None, :] >> np.arange(T)[:, None]) & 1).astype(np.uint8)
    return spkgen.pack(bits), n // 128, 128


def _fed(s, H, W, theta, t_out, order, cuts, lib=None):
    st = oracle.Stream(H, W, theta, t_out, order=order, windows=True, lib=lib)
    for a, b in zip(cuts[:-1], cuts[1:]):
        st.feed(s[a:b])
    return st.finish()


@pytest.mark.parametrize("order", ORDERS)
def test_every_12_frame_stream_split_at_every_frame(order):
    T = 12
    s, H, W = _all_streams(T)
    # every frame, plus repeats and an unsorted tail
    t_out = list(range(T)) + [5, 0, T - 1, 3]
    ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order, windows=True)
    for cut in range(T + 1):
        got = _fed(s, H, W, 1.0, t_out, order, [0, cut, T])
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r, err_msg="order %d cut %d" % (order, cut))


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("scene", ["gratings", "moving_blocks"])
def test_random_pieces_equal_single_pass(order, scene):
    rng = np.random.default_rng(order * 10 + len(scene))
    H, W, T = 14, 23, 900
    if scene == "gratings":
        s = spkgen.gratings(H, W, T, seed=81)
    else:
        s = spkgen.blocks(H, W, T, seed=82, vx=0.7, vy=-0.3, block=4)
    t_out = [int(t) for t in rng.integers(0, T, 60)] + [0, T - 1]
    ref = oracle.reconstruct(s, H, W, T, 2.5, t_out, order=order, windows=True)
    for trial in range(3):
        cuts = [0]
        while cuts[-1] < T:
            cuts.append(min(T, cuts[-1] + int(rng.integers(0, 90))))
        got = _fed(s, H, W, 2.5, t_out, order, cuts)
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)


def test_frame_by_frame_and_silent_pixels():
    """One frame per piece; pixels that never fire or fire once output 0 and
    the window (-1, -1, 0); no output times at all is allowed."""
    H, W, T = 3, 5, 80
    bits = np.zeros((T, H, W), dtype=np.uint8)
    bits[::7, 0, :] = 1          # regular
    bits[40, 1, 2] = 1           # a single spike
    bits[[3, 9, 10, 30, 31, 79], 2, 4] = 1
    s = spkgen.pack(bits)
    t_out = [0, 8, 40, 79, 79]
    for order in ORDERS:
        ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order, windows=True)
        got = _fed(s, H, W, 1.0, t_out, order, list(range(T + 1)))
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)
        assert np.all(got[0][:, 1, :] == 0.0) and np.all(got[1][:, 1, :] == -1)
    st = oracle.Stream(H, W, 1.0, [], order=oracle.SSR)
    st.feed(s)
    assert st.finish().shape == (0, H, W)


def test_stream_argument_errors():
    with pytest.raises(ValueError):
        oracle.Stream(0, 4, 1.0, [0])
    with pytest.raises(ValueError):
        oracle.Stream(4, 4, 1.0, [-1])
    with pytest.raises(ValueError):
        oracle.Stream(4, 4, 1.0, [0], order=7)
