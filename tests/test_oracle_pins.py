"""Pins of the reference oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
procedure: they check closed forms (Lemma 1, Lemma 2, Eq. 6 on constant
light), declarative definitions of the segmentations (brute force over every
stream of a few frames), special cases that reduce to the baseline methods
(TFI, TFP) and a hand-worked example.
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

import brute
import oracle
import spkgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# --------------------------------------------------------------------------
# the generator (sensor model, Eq. 2) against its closed form

def test_generator_constant_rate_closed_form():
    """Eq. 2 with constant increment Q <= theta and subtract reset: after
    frames 0..n the spike count is floor((V0 + (n+1) Q) / theta)."""
    rng = np.random.default_rng(0)
    H, W, T = 4, 50, 300
    theta = 997
    Q = rng.integers(1, theta + 1, size=H * W)
    v0 = rng.integers(0, theta, size=H * W)
    s = spkgen.from_increments(Q, v0, theta, H, W, T=T)
    bits = spkgen.unpack(s, H, W).reshape(T, -1).astype(np.int64)
    cum = np.cumsum(bits, axis=0)
    n = np.arange(T)[:, None]
    np.testing.assert_array_equal(cum, (v0[None, :] + (n + 1) * Q[None, :]) // theta)


# --------------------------------------------------------------------------
# Lemma 1 / Lemma 2 / Theorem 1 on generated constant-rate streams

def _spike_frames(bits_col):
    return np.flatnonzero(bits_col).tolist()


def _const_streams(theta_max=40, T=400):
    """One pixel per (Q, theta, V0) with theta <= theta_max, Q <= theta."""
    cases = [(q, th, v) for th in range(1, theta_max + 1) for q in range(1, th + 1)
             for v in range(0, th, max(1, th // 4))]
    Q = np.array([c[0] for c in cases], dtype=np.int64)
    TH = np.array([c[1] for c in cases], dtype=np.int64)
    V = np.array([c[2] for c in cases], dtype=np.int64)
    return cases, Q, TH, V, T


def _gen_multi_theta(Q, TH, V, T):
    """Streams with per-pixel thresholds: scale to a common threshold L =
    lcm-free form theta' = prod? -- use rational scaling by theta_i."""
    # integrate directly: per-pixel thresholds differ, so do it here in
    # integers (this is the sensor model only, not the method)
    n = len(Q)
    v = V.copy()
    bits = np.zeros((T, n), dtype=np.uint8)
    for t in range(T):
        v = v + Q
        f = v >= TH
        bits[t, f] = 1
        v = v - f * TH
    return bits


def test_lemma1_intervals_two_values():
    """Lemma 1 (Eq. 7-9): with fixed rate the intervals take only
    floor(theta/Q) and floor(theta/Q)+1 (one value when Q divides theta)."""
    cases, Q, TH, V, T = _const_streams()
    bits = _gen_multi_theta(Q, TH, V, T)
    for i, (q, th, v) in enumerate(cases):
        x = brute.intervals_of(_spike_frames(bits[:, i]))
        lo = th // q
        allowed = {lo} if th % q == 0 else {lo, lo + 1}
        assert set(x) <= allowed, (q, th, v, set(x))


def test_lemma2_s2_gaps_and_theorem1_third_order():
    """Lemma 2 (Eq. 13): S1 is itself spike-like with fixed rate, so its S2
    streams are zero-order stable, and (Theorem 1) so are the S3 streams."""
    cases, Q, TH, V, T = _const_streams(theta_max=64, T=1500)
    bits = _gen_multi_theta(Q, TH, V, T)
    for i, (q, th, v) in enumerate(cases):
        x = brute.intervals_of(_spike_frames(bits[:, i]))
        for val, gaps in brute.s2_streams(x).items():
            assert brute.zero_order_stable(gaps), (q, th, v, val)
            # third order: gap stream of each value of this S2
            for val2, gaps2 in brute.s2_streams(gaps).items():
                assert brute.zero_order_stable(gaps2), (q, th, v, val, val2)


@pytest.mark.parametrize("order", [oracle.FSR, oracle.SSR, oracle.TSR])
def test_constant_rate_single_segment_and_exact_intensity(order):
    """Theorem 1: a constant-rate pixel is absolutely stable, so FSR, SSR
    and the third order keep one segment; Eq. 6 over it is theta*(K-1)/(tau_K - tau_1).  When Q
    divides theta every interval is theta/Q and the estimate is exactly
    theta*Q/theta_int; otherwise its relative error is below
    1/(N*theta_int/Q - 1) (residuals at both ends are in [0, Q))."""
    rng = np.random.default_rng(1)
    H, W, T = 8, 64, 2048
    th_int = 4096
    divisors = [d for d in range(1, th_int + 1) if th_int % d == 0]
    Q = np.where(rng.random(H * W) < 0.5, rng.choice(divisors, H * W),
                 rng.integers(1, th_int + 1, H * W))
    v0 = rng.integers(0, th_int, H * W)
    s = spkgen.from_increments(Q, v0, th_int, H, W, T=T)
    theta = 255.0
    t_out = np.array([0, 5, 700, 2047], dtype=np.int32)
    out, wf, wl, wn = oracle.reconstruct(s, H, W, T, theta, t_out, order=order,
                                         windows=True)
    bits = spkgen.unpack(s, H, W).reshape(T, -1)
    out = out.reshape(len(t_out), -1)
    wf, wl, wn = (a.reshape(len(t_out), -1) for a in (wf, wl, wn))
    sf, sl, sn, cnt = oracle.segments(s, H, W, T, order=order, cap=4)
    for p in range(H * W):
        tau = _spike_frames(bits[:, p])
        K = len(tau)
        if K < 2:
            assert cnt[p] == 0
            continue
        assert cnt[p] == 1
        assert (sf[0, p], sl[0, p], sn[0, p]) == (tau[0], tau[-1], K - 1)
        for k in range(len(t_out)):
            assert (wf[k, p], wl[k, p], wn[k, p]) == (tau[0], tau[-1], K - 1)
            exact = theta * Q[p] / th_int
            if th_int % Q[p] == 0:
                assert out[k, p] == exact
            else:
                N = K - 1
                assert abs(out[k, p] - exact) / exact < 1.0 / (N * th_int / Q[p] - 1)


# --------------------------------------------------------------------------
# declarative definitions, brute force over every stream of a few frames

def _all_streams(T):
    """Every binary stream of T frames, one per pixel (pixel p = bits of p)."""
    n = 1 << T
    H, W = n // 128, 128
    p = np.arange(n)
    bits = ((p[None, :] >> np.arange(T)[:, None]) & 1).astype(np.uint8)
    return spkgen.pack(bits), bits, H, W


@pytest.mark.parametrize("T", [12, 14])
def test_fsr_ssr_all_streams_bruteforce(T):
    """Sec. III-B: on every stream of T frames the oracle's FSR partition is
    the unique stable + maximal one, and its SSR partition refines FSR and is
    the unique S2-stable + maximal one inside each FSR segment."""
    s, bits, H, W = _all_streams(T)
    cap = T
    f_first, f_last, f_n, f_cnt = oracle.segments(s, H, W, T, order=oracle.FSR, cap=cap)
    s_first, s_last, s_n, s_cnt = oracle.segments(s, H, W, T, order=oracle.SSR, cap=cap)
    for p in range(H * W):
        tau = _spike_frames(bits[:, p])
        x = brute.intervals_of(tau)
        # map windows back to interval-index starts
        idx = {t: i for i, t in enumerate(tau)}
        fs = [idx[f_first[k, p]] for k in range(f_cnt[p])]
        ss = [idx[s_first[k, p]] for k in range(s_cnt[p])]
        assert brute.is_fsr_partition(x, fs), (p, x, fs)
        assert brute.is_ssr_partition(x, ss, fs), (p, x, ss, fs)
        ts = oracle.segment_intervals(x, oracle.TSR)
        assert brute.is_tsr_partition(x, ts, ss), (p, x, ts, ss)
        # windows are consistent: last = first of the next, n counts intervals
        for k in range(f_cnt[p]):
            a = fs[k]
            b = (fs[k + 1] if k + 1 < f_cnt[p] else len(x)) - 1
            assert (f_last[k, p], f_n[k, p]) == (tau[b + 1], b - a + 1)
        for k in range(s_cnt[p]):
            a = ss[k]
            b = (ss[k + 1] if k + 1 < s_cnt[p] else len(x)) - 1
            assert (s_last[k, p], s_n[k, p]) == (tau[b + 1], b - a + 1)


def test_partition_uniqueness_by_enumeration():
    """The declarative FSR/SSR properties admit exactly one partition, and it
    is the oracle's (all partitions enumerated for short random S1)."""
    rng = np.random.default_rng(2)
    for _ in range(300):
        n = int(rng.integers(1, 11))
        base = int(rng.integers(1, 6))
        x = (base + rng.integers(-1, 3, n)).clip(1).tolist()
        fsr = brute.enumerate_partitions(x, lambda st: brute.is_fsr_partition(x, st))
        assert len(fsr) == 1
        assert oracle.segment_intervals(x, oracle.FSR) == fsr[0]
        ssr = brute.enumerate_partitions(x, lambda st: brute.is_ssr_partition(x, st, fsr[0]))
        assert len(ssr) == 1
        assert oracle.segment_intervals(x, oracle.SSR) == ssr[0]
        tsr = brute.enumerate_partitions(x, lambda st: brute.is_tsr_partition(x, st, ssr[0]))
        assert len(tsr) == 1
        assert oracle.segment_intervals(x, oracle.TSR) == tsr[0]


def test_random_long_interval_streams_declarative():
    """Longer random S1 with values drawn near a slowly drifting rate: both
    partitions satisfy their declarative definitions."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(20, 400))
        drift = np.cumsum(rng.normal(0, 0.1, n)) + rng.uniform(2, 12)
        x = np.maximum(1, np.round(drift + rng.integers(-1, 2, n))).astype(int).tolist()
        fs = oracle.segment_intervals(x, oracle.FSR)
        ss = oracle.segment_intervals(x, oracle.SSR)
        ts = oracle.segment_intervals(x, oracle.TSR)
        assert brute.is_fsr_partition(x, fs)
        assert brute.is_ssr_partition(x, ss, fs)
        assert brute.is_tsr_partition(x, ts, ss)


def test_break_function_monotone():
    """The FSR segment that starts earlier never ends later (a stable run
    stays stable when shortened from the left); SSR likewise inside one FSR
    segment.  Checked on the oracle's first segment from every start."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        n = int(rng.integers(5, 60))
        x = (4 + rng.integers(-1, 2, n) + (rng.random(n) < 0.1) * 3).tolist()
        for order in (oracle.FSR, oracle.SSR, oracle.TSR):
            ends = []
            for s in range(n):
                st = oracle.segment_intervals(x[s:], order)
                ends.append(s + (st[1] if len(st) > 1 else n - s))
            assert all(a <= b for a, b in zip(ends, ends[1:])), (order, x, ends)


# --------------------------------------------------------------------------
# special cases that reduce to the baseline methods (Sec. II)

def test_tfi_special_case():
    """When neighbouring intervals always differ by at least 2, every
    interval is its own segment and the estimate is TFI: theta / T0(m(t))."""
    rng = np.random.default_rng(5)
    H, W, T = 2, 32, 600
    bits = np.zeros((T, H * W), dtype=np.uint8)
    taus = []
    for p in range(H * W):
        t, prev, tau = int(rng.integers(0, 5)), None, []
        while t < T:
            tau.append(t)
            while True:
                x = int(rng.integers(1, 30))
                if prev is None or abs(x - prev) >= 2:
                    break
            prev = x
            t += x
        bits[tau, p] = 1
        taus.append(tau)
    s = spkgen.pack(bits)
    t_out = np.arange(0, T, 7, dtype=np.int32)
    for order in (oracle.FSR, oracle.SSR):
        out = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order).reshape(len(t_out), -1)
        for p in range(H * W):
            tau = taus[p]
            x = brute.intervals_of(tau)
            for k, t in enumerate(t_out):
                m = brute.interval_in_progress(tau, int(t))
                assert out[k, p] == 1.0 / x[m - 1]


def test_tfp_special_case():
    """A single stable segment from tau_1 to tau_K gives the TFP-style rate
    (spike count over the window's duration), for every output time."""
    H, W, T = 1, 3, 100
    bits = np.zeros((T, H * W), dtype=np.uint8)
    bits[[3, 6, 10, 13, 16, 20, 23], 0] = 1      # S1 = 3 4 3 3 4 3
    bits[[0, 1, 2, 3, 5, 6, 7, 9], 1] = 1        # S1 = 1 1 1 2 1 1 2
    bits[[50, 99], 2] = 1                        # one interval
    s = spkgen.pack(bits)
    t_out = np.arange(T, dtype=np.int32)
    for order in (oracle.FSR, oracle.SSR):
        out = oracle.reconstruct(s, H, W, T, 2.0, t_out, order=order).reshape(T, -1)
        np.testing.assert_array_equal(out[:, 0], 2.0 * 6 / 20)
        np.testing.assert_array_equal(out[:, 2], 2.0 * 1 / 49)
    # pixel 1 under FSR is one segment; under SSR the value-1 gaps are
    # 1 1 2 1 -> stable, the value-2 gaps are 3 -> stable: one segment too
    out = oracle.reconstruct(s, H, W, T, 2.0, t_out, order=oracle.SSR).reshape(T, -1)
    np.testing.assert_array_equal(out[:, 1], 2.0 * 7 / 9)


# --------------------------------------------------------------------------
# the hand-worked example

def _read_golden():
    rows = []
    with open(os.path.join(GOLDEN, "worked_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#") or line.startswith("order"):
                continue
            o, p, t, a, b, n, frac = line.split()
            rows.append((o, int(p), int(t), int(a), int(b), int(n), Fraction(frac)))
    return rows


def worked_example_stream():
    T = 70
    bits = np.zeros((T, 4), dtype=np.uint8)
    bits[[1, 5, 9, 13, 18, 22, 27, 32, 37, 42, 46, 50, 57, 64], 0] = 1
    bits[[10], 2] = 1
    bits[[0, 2, 7, 9, 18, 21], 3] = 1
    return spkgen.pack(bits), 1, 4, T


def test_worked_example_golden():
    s, H, W, T = worked_example_stream()
    rows = _read_golden()
    for order_name, order in (("FSR", oracle.FSR), ("SSR", oracle.SSR)):
        sel = [r for r in rows if r[0] == order_name]
        t_out = np.array([r[2] for r in sel], dtype=np.int32)
        out, wf, wl, wn = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order,
                                             windows=True)
        for k, (_, p, t, a, b, n, frac) in enumerate(sel):
            assert (wf[k, 0, p], wl[k, 0, p], wn[k, 0, p]) == (a, b, n), (order_name, p, t)
            assert out[k, 0, p] == float(frac), (order_name, p, t)


def test_ssr_refines_fsr_on_generated_scenes():
    """SSR never merges what FSR splits (Sec. III-B: SSR may break an FSR
    segment into shorter ones)."""
    H, W, T = 16, 32, 3000
    s = spkgen.gratings(H, W, T, seed=11)
    f = oracle.segments(s, H, W, T, order=oracle.FSR, cap=T)
    g = oracle.segments(s, H, W, T, order=oracle.SSR, cap=T)
    for p in range(H * W):
        fset = set(f[0][: f[3][p], p].tolist())
        sset = set(g[0][: g[3][p], p].tolist())
        assert fset <= sset
        assert g[3][p] >= f[3][p]


def test_argument_errors():
    s = np.zeros((4, 16), dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle.reconstruct(s, 1, 8, 4, 1.0, [4])          # t out of range
    with pytest.raises(ValueError):
        oracle.reconstruct(s, 1, 8, 4, 1.0, [0], order=5)  # unknown order
    with pytest.raises(ValueError):
        oracle.tfp(s, 1, 8, 4, 1.0, 0, [0])                # empty window


@pytest.mark.parametrize("order", [oracle.FSR, oracle.SSR])
def test_causal_reading_is_the_method_on_the_prefix(order):
    """Streaming reading: the causal output at t is, by definition, the
    method run on frames 0..t alone and valued at frame t.  Checked against
    exactly that (the oracle on each truncated stream), on moving noisy and
    moving block scenes, at every frame of a short stream."""
    H, W, T = 6, 21, 160
    for s in (spkgen.gratings(H, W, T, seed=61), spkgen.blocks(H, W, T, seed=62, block=4, vx=0.7)):
        t_out = list(range(T))
        got, gf, gl, gn = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order, windows=True,
                                             causal=True)
        for t in t_out:
            ref, rf, rl, rn = oracle.reconstruct(s[:t + 1], H, W, t + 1, 1.0, [t], order=order,
                                                 windows=True)
            np.testing.assert_array_equal(got[t], ref[0])
            np.testing.assert_array_equal(gf[t], rf[0])
            np.testing.assert_array_equal(gl[t], rl[0])
            np.testing.assert_array_equal(gn[t], rn[0])


def test_causal_reading_bruteforce():
    """On every stream of 12 frames and at every t: the causal output is
    theta*n/D of the last piece of the declarative FSR partition of the
    intervals that have ended by t (0 with fewer than two spikes)."""
    T = 12
    s, bits, H, W = _all_streams(T)
    got = oracle.reconstruct(s, H, W, T, 1.0, list(range(T)), order=oracle.FSR, causal=True)
    got = got.reshape(T, -1)
    for p in range(H * W):
        tau = _spike_frames(bits[:, p])
        for t in range(T):
            tt = [f for f in tau if f <= t]
            if len(tt) < 2:
                assert got[t, p] == 0.0
                continue
            x = brute.intervals_of(tt)
            parts = brute.enumerate_partitions(x, lambda st: brute.is_fsr_partition(x, st))
            a = parts[0][-1]
            assert got[t, p] == len(x[a:]) / (tt[-1] - tt[a]), (p, t, tt)


# --------------------------------------------------------------------------
# the baselines themselves (Sec. II): TFI as the order that keeps every
# interval on its own, TFP as a windowed spike count

def test_tfi_order_is_reciprocal_interval():
    """TFI: the estimate at t is theta / T0(m(t)) with window (tau_m,
    tau_m+1, 1), on streams whose intervals repeat and alternate (where FSR
    and SSR merge them) as well as on noisy ones; fewer than two spikes give
    0 and (-1, -1, 0)."""
    H, W, T = 3, 40, 300
    s = spkgen.gratings(H, W, T, seed=41)
    bits = spkgen.unpack(s, H, W).reshape(T, -1)
    bits[:, 0] = 0
    bits[:, 1] = 0
    bits[7, 1] = 1
    bits[:, 2] = 0
    bits[::3, 2] = 1
    s = spkgen.pack(bits)
    t_out = np.arange(T, dtype=np.int32)
    out, wf, wl, wn = oracle.reconstruct(s, H, W, T, 2.0, t_out, order=oracle.TFI, windows=True)
    out, wf, wl, wn = (a.reshape(T, -1) for a in (out, wf, wl, wn))
    for p in range(H * W):
        tau = _spike_frames(bits[:, p])
        for t in range(T):
            if len(tau) < 2:
                assert (out[t, p], wf[t, p], wl[t, p], wn[t, p]) == (0.0, -1, -1, 0)
                continue
            m = brute.interval_in_progress(tau, t)
            x = tau[m] - tau[m - 1]
            assert (wf[t, p], wl[t, p], wn[t, p]) == (tau[m - 1], tau[m], 1)
            assert out[t, p] == 2.0 / x


def test_tfi_equals_fsr_when_neighbours_differ_by_two():
    """Where no two neighbouring intervals are within 1 of each other, FSR
    and SSR keep every interval alone: all three orders agree exactly."""
    rng = np.random.default_rng(6)
    T = 800
    bits = np.zeros((T, 64), dtype=np.uint8)
    for p in range(64):
        t, prev = int(rng.integers(0, 5)), None
        while t < T:
            bits[t, p] = 1
            while True:
                x = int(rng.integers(1, 40))
                if prev is None or abs(x - prev) >= 2:
                    break
            prev = x
            t += x
    s = spkgen.pack(bits)
    t_out = np.arange(0, T, 3, dtype=np.int32)
    ref = oracle.reconstruct(s, 1, 64, T, 1.0, t_out, order=oracle.TFI)
    for order in (oracle.FSR, oracle.SSR):
        np.testing.assert_array_equal(oracle.reconstruct(s, 1, 64, T, 1.0, t_out, order=order), ref)


@pytest.mark.parametrize("window", [1, 7, 32, 64, 300])
def test_tfp_constant_rate_closed_form(window):
    """TFP on constant light (Eq. 2 with a constant increment): the window
    count is C(t) - C(t - L), C(n) = floor((V0 + (n+1) Q) / theta) spikes
    up to frame n, and the estimate is within theta / L of the rate."""
    rng = np.random.default_rng(window)
    H, W, T = 2, 64, 500
    th = 1009
    Q = rng.integers(1, th + 1, size=H * W)
    v0 = rng.integers(0, th, size=H * W)
    s = spkgen.from_increments(Q, v0, th, H, W, T=T)
    t_out = np.array(sorted(set(rng.integers(0, T, 60).tolist() + [0, window - 1, T - 1]) & set(range(T))),
                     dtype=np.int32)
    out = oracle.tfp(s, H, W, T, 3.0, window, t_out).reshape(len(t_out), -1)

    def C(n):
        return np.where(n < 0, 0, (v0 + (n + 1) * Q) // th)

    for k, t in enumerate(t_out):
        L = min(window, int(t) + 1)
        cnt = C(int(t)) - C(int(t) - L)
        np.testing.assert_array_equal(out[k], 3.0 * cnt / L)
        assert np.all(np.abs(out[k] - 3.0 * Q / th) < 3.0 / L + 1e-12)


def test_third_order_cuts_where_s3_breaks():
    """Worked by hand: S1 = 4 4 4 5 4 5 4 5 4 4.  FSR keeps {4, 5}; S2(4) =
    gaps of 4 at 0 1 2 4 6 8 9 = 1 1 2 2 2 1 and S2(5) = 2 2 are stable, so
    SSR keeps one piece.  S3(4, 1) = gaps between the positions 0 1 5 of the
    value 1 in S2(4) = 1 4: the S2 element that interval 9 adds breaks it,
    so the third order cuts before interval 9."""
    x = [4, 4, 4, 5, 4, 5, 4, 5, 4, 4]
    assert oracle.segment_intervals(x, oracle.FSR) == [0]
    assert oracle.segment_intervals(x, oracle.SSR) == [0]
    assert oracle.segment_intervals(x, oracle.TSR) == [0, 9]
    assert brute.is_tsr_partition(x, [0, 9], [0])


def test_third_order_refines_ssr_on_generated_scenes():
    """The third order never merges what SSR splits, and on noisy scenes it
    does cut inside SSR pieces (the order adds something)."""
    H, W, T = 8, 40, 3000
    s = spkgen.gratings(H, W, T, seed=23)
    _, sl, _, sc = oracle.segments(s, H, W, T, order=oracle.SSR, cap=T)
    _, tl, _, tc = oracle.segments(s, H, W, T, order=oracle.TSR, cap=T)
    assert np.all(tc >= sc)
    assert tc.sum() > sc.sum()
    for p in range(H * W):
        assert set(sl[:sc[p], p].tolist()) <= set(tl[:tc[p], p].tolist())


# --------------------------------------------------------------------------
# static / motion mask (the theorem's use named in the conclusion)

def test_motion_mask_constant_light_is_static():
    """Theorem 1: constant light keeps one segment, so no pixel is ever
    marked as moving, whatever the window."""
    rng = np.random.default_rng(8)
    H, W, T = 4, 64, 1500
    th = 4096
    s = spkgen.from_increments(rng.integers(1, th + 1, H * W), rng.integers(0, th, H * W), th,
                               H, W, T=T)
    for order in (oracle.FSR, oracle.SSR, oracle.TSR):
        m = oracle.motion(s, H, W, T, 64, list(range(0, T, 13)), order=order)
        assert m.sum() == 0


def test_motion_mask_after_a_step_in_light():
    """Intervals 4 up to frame ~200, then 9: FSR cuts at the first 9, whose
    segment starts at the last spike f of the 4-run.  With window L the mask
    is 1 exactly for t in (f, f + L) and 0 before."""
    T = 600
    tau = list(range(2, 203, 4))
    f = tau[-1]
    tau += list(range(f + 9, T, 9))
    bits = np.zeros((T, 1), dtype=np.uint8)
    bits[tau, 0] = 1
    s = spkgen.pack(bits)
    L = 50
    t_out = list(range(T))
    m = oracle.motion(s, 1, 1, T, L, t_out, order=oracle.FSR)[:, 0, 0]
    want = np.array([1 if f < t < f + L else 0 for t in t_out], dtype=np.uint8)
    np.testing.assert_array_equal(m, want)
