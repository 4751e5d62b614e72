"""Planted mistakes in the oracle must fail its pins.

Each case copies oracle.c, plants one plausible mistake (a dropped term, a
wrong comparison, an index off by one, a missing reset), builds the copy on
the CPU with gcc and runs a compact battery of the pins from
test_oracle_pins.py against it in a child process (a mutant may also crash
or abort, which counts as caught).  At least one pin must fail for every
mutant; the unmodified source must pass them all.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import brute
import oracle
import spkgen
from test_oracle_pins import _read_golden, worked_example_stream

MUTANTS = {
    "span_threshold": ("return hi - lo <= 1;", "return hi - lo <= 2;"),
    "no_reset_on_break": ("            start[nseg++] = m;\n            lo = hi = x[m];",
                          "            start[nseg++] = m;"),
    "count_off_by_one": ("I = (tk->theta * (double)cnt)", "I = (tk->theta * (double)(cnt + 1))"),
    "window_last_index": ("last = sc->tau[b + 1];", "last = sc->tau[b];"),
    "output_time_leq": ("if (tau[mid] < t) lo = mid + 1;", "if (tau[mid] <= t) lo = mid + 1;"),
    "clamp_high": ("if (m > K - 1) m = K - 1;", "if (m > K - 1) m = K - 2;"),
    "ssr_no_state_reset": ("                ntr = 0;\n                tr[ntr++] = (s2_track){v, m, 0, 0, 0};",
                           "                tr[j].last = m;"),
    "ssr_gap_not_recorded": ("            tr[j].has_gap = 1;\n", ""),
    "interval_sign": ("sc->x[i] = sc->tau[i + 1] - sc->tau[i];",
                      "sc->x[i] = sc->tau[i] - sc->tau[i + 1] + 2 * (sc->tau[i + 1] - sc->tau[i]) - (i == 0);"),
    "causal_excludes_spike_at_t": ("spikes_before(sc->tau, K, tk->t_out[k] + 1)",
                                   "spikes_before(sc->tau, K, tk->t_out[k])"),
    "causal_untruncated": ("                last = sc->tau[i + 1];",
                           "                last = sc->tau[i + 1 < K - 1 ? i + 2 : i + 1];"),
    "tfi_merges_pairs": ("for (int32_t i = 0; i < n; i++) start[i] = i;\n        return n;",
                         "for (int32_t i = 0; i < n; i++) start[i / 2] = i & ~1;\n        return (n + 1) / 2;"),
    "tfp_window_off_by_one": ("int32_t f0 = t - window + 1 < 0 ? 0 : t - window + 1;",
                              "int32_t f0 = t - window < 0 ? 0 : t - window;"),
    "tsr_no_reset_at_cut": ("                start[nseg++] = m;\n                ntr = 0;\n                tr[ntr].value = v;",
                            "                start[nseg++] = m;\n                tr[ntr].value = v;"),
    "tsr_last_not_updated": ("            u->has_gap = 1;\n            u->last = t->n2;\n        } else {\n            /* S2(v)",
                             "            u->has_gap = 1;\n        } else {\n            /* S2(v)"),
    "stream_tsr_last_not_updated": ("            u->has_gap = 1;\n            u->last = t->n2;\n        } else {\n            if (t->nt3",
                                    "            u->has_gap = 1;\n        } else {\n            if (t->nt3"),
    "stream_ssr_cut_keeps_tracks": ("                    cut = 1;\n                    tracks_fresh(q, x, m, 1);\n                } else if",
                                    "                    cut = 1;\n                    tracks_fresh(q, x, m, 0);\n                } else if"),
    "stream_close_before_last_spike": ("int32_t kc = outputs_upto(s, q->lastspk);",
                                       "int32_t kc = outputs_upto(s, q->lastspk - 1);"),
    "stream_forgets_frames_fed": ("online_spike(s, p, s->fed + j);", "online_spike(s, p, j);"),
    "first_segment_start": ("    start[nseg++] = 0;\n    int32_t lo = x[0], hi = x[0];",
                            "    start[nseg++] = 0;\n    int32_t lo = x[0], hi = x[0] + 1;"),
}


def _battery(lib):
    """Returns the list of pin names that fail for the oracle library lib."""
    failed = []
    # hand-worked example
    s, H, W, T = worked_example_stream()
    rows = _read_golden()
    ok = True
    for order_name, order in (("FSR", oracle.FSR), ("SSR", oracle.SSR)):
        sel = [r for r in rows if r[0] == order_name]
        t_out = np.array([r[2] for r in sel], dtype=np.int32)
        out, wf, wl, wn = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order,
                                             windows=True, lib=lib)
        for k, (_, p, t, a, b, n, frac) in enumerate(sel):
            if (wf[k, 0, p], wl[k, 0, p], wn[k, 0, p]) != (a, b, n) or out[k, 0, p] != float(frac):
                ok = False
    if not ok:
        failed.append("golden")
    # declarative partitions on every stream of 11 frames
    T = 11
    n = 1 << T
    p = np.arange(n)
    bits = ((p[None, :] >> np.arange(T)[:, None]) & 1).astype(np.uint8)
    s = spkgen.pack(bits)
    f = oracle.segments(s, 16, 128, T, order=oracle.FSR, cap=T, lib=lib)
    g = oracle.segments(s, 16, 128, T, order=oracle.SSR, cap=T, lib=lib)
    h = oracle.segments(s, 16, 128, T, order=oracle.TSR, cap=T, lib=lib)
    ok = True
    for q in range(n):
        tau = np.flatnonzero(bits[:, q]).tolist()
        x = brute.intervals_of(tau)
        idx = {t: i for i, t in enumerate(tau)}
        try:
            fs = [idx[f[0][k, q]] for k in range(f[3][q])]
            ss = [idx[g[0][k, q]] for k in range(g[3][q])]
            ts = [idx[h[0][k, q]] for k in range(h[3][q])]
        except KeyError:
            ok = False
            break
        if not (brute.is_fsr_partition(x, fs) and brute.is_ssr_partition(x, ss, fs)
                and brute.is_tsr_partition(x, ts, ss)):
            ok = False
            break
    if not ok:
        failed.append("bruteforce")
    # constant rate, Q divides theta: exact intensity
    th = 64
    Q = np.array([1, 2, 4, 8, 16, 32, 64, 8], dtype=np.int64)
    v0 = np.array([0, 1, 3, 7, 15, 31, 63, 5], dtype=np.int64)
    s = spkgen.from_increments(Q, v0, th, 1, 8, T=300)
    out = oracle.reconstruct(s, 1, 8, 300, 1.0, [0, 150, 299], lib=lib)
    if not np.all(out[:, 0, :] == (Q / th)[None, :]):
        failed.append("exact_intensity")
    # TFI = reciprocal of the interval in progress; TFP = windowed count
    Qv = np.array([3, 5, 7, 11, 13, 17, 19, 23], dtype=np.int64)
    s = spkgen.from_increments(Qv, v0, th, 1, 8, T=300)
    t_chk = list(range(100, 160))
    tfi = oracle.reconstruct(s, 1, 8, 300, 1.0, t_chk, order=oracle.TFI, lib=lib)
    bits = spkgen.unpack(s, 1, 8).reshape(300, -1)
    ok = True
    for q in range(8):
        tau = np.flatnonzero(bits[:, q]).tolist()
        for k, t in enumerate(t_chk):
            m = brute.interval_in_progress(tau, t)
            ok = ok and tfi[k, 0, q] == 1.0 / (tau[m] - tau[m - 1])
    if not ok:
        failed.append("tfi")
    tp = oracle.tfp(s, 1, 8, 300, 1.0, 10, [100], lib=lib)
    cnt = bits[91:101].sum(axis=0)
    if not np.array_equal(tp[0, 0], cnt / 10.0):
        failed.append("tfp")
    # carry-state form: any split of a stream == the whole stream
    H, W, T = 4, 9, 300
    s = spkgen.gratings(H, W, T, seed=63)
    t_out = list(range(0, T, 3))
    for order in (oracle.FSR, oracle.SSR, oracle.TSR):
        ref = oracle.reconstruct(s, H, W, T, 1.0, t_out, order=order, windows=True, lib=lib)
        st = oracle.Stream(H, W, 1.0, t_out, order=order, windows=True, lib=lib)
        for a in range(0, T, 37):
            st.feed(s[a:a + 37])
        got = st.finish()
        if not all(np.array_equal(g, r) for g, r in zip(got, ref)):
            failed.append("stream_resume")
            break
    # causal reading == the method on each prefix
    H, W, T = 4, 9, 60
    s = spkgen.blocks(H, W, T, seed=62, block=3, vx=0.7)
    got = oracle.reconstruct(s, H, W, T, 1.0, list(range(T)), causal=True, lib=lib)
    for t in range(T):
        ref = oracle.reconstruct(s[:t + 1], H, W, t + 1, 1.0, [t], lib=lib)
        if not np.array_equal(got[t], ref[0]):
            failed.append("causal_prefix")
            break
    return failed


@pytest.fixture(scope="module")
def src_text():
    with open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")) as f:
        return f.read()


def _run_battery(tmp_path, text):
    """Build ``text`` as an oracle library and run the battery in a child
    process; returns (exit code, output).  Exit 0 means every pin passed."""
    path = tmp_path / "o.c"
    path.write_text(text)
    lib = oracle.build(src=str(path), out=str(tmp_path / "lib.so"))
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys, oracle, test_oracle_mutants as m\n"
            "f = m._battery(oracle.load(sys.argv[1]))\n"
            "print(f)\n"
            "sys.exit(1 if f else 0)\n")
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([here, os.path.dirname(here)]))
    r = subprocess.run([sys.executable, "-c", code, lib], cwd=here, env=env,
                       capture_output=True, text=True, timeout=300)
    return r.returncode, r.stdout + r.stderr[-2000:]


def test_unmodified_oracle_passes_battery(tmp_path, src_text):
    rc, out = _run_battery(tmp_path, src_text)
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, src_text, name):
    old, new = MUTANTS[name]
    assert src_text.count(old) == 1, name
    rc, out = _run_battery(tmp_path, src_text.replace(old, new))
    assert rc != 0, "mutant %s passed every pin" % name
