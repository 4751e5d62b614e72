"""The C-ABI library on the CPU: it loads, exports every declared entry point,
and rejects bad arguments on the host before touching any device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(spk_\w+)\s*\(", text, re.M):
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2412_11639_amd import _lib
    return _lib.load()


def test_headers_declare_entry_points():
    names = declared_functions()
    for n in ["spk_frame_bytes", "spk_strerror", "spk_version", "spk_reconstruct",
              "spk_reconstruct_windows", "spk_segments"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(os.path.join(ROOT, "paper_2412_11639_amd", "libspk.so"))
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert missing == []


def test_frame_bytes(lib):
    assert lib.spk_frame_bytes(250, 400) == 12512
    assert lib.spk_frame_bytes(1000, 1000) == 125008
    assert lib.spk_frame_bytes(1, 1) == 16
    assert lib.spk_frame_bytes(0, 5) == 0
    for H, W in [(1, 128), (1, 129), (3, 43), (720, 1280)]:
        fb = lib.spk_frame_bytes(H, W)
        assert fb % 16 == 0 and fb * 8 >= H * W and (fb - 16) * 8 < H * W


def test_strerror(lib):
    assert lib.spk_strerror(0) == b"ok"
    assert b"invalid" in lib.spk_strerror(-1)


FAKE = 4096  # a non-null pointer value; validation must fail before any use


@pytest.mark.parametrize("args", [
    dict(stream=0), dict(stream=FAKE + 8),  # null, not 16-byte aligned
    dict(H=0), dict(W=-1), dict(T=0),
    dict(theta=0.0), dict(theta=-1.0), dict(theta=float("nan")), dict(theta=float("inf")),
    dict(n_out=-1),
    dict(t_out=[5, 10]),          # 10 >= T
    dict(t_out=[-1]),
    dict(order=0), dict(order=5),
    dict(out=0),
    dict(H=65536, W=65536),       # H*W overflows int32
])
def test_reconstruct_rejects_bad_arguments(lib, args):
    a = dict(stream=FAKE, H=4, W=4, T=10, theta=1.0, t_out=[0, 5], n_out=None, out=FAKE,
             order=1)
    a.update(args)
    t = (ctypes.c_int32 * max(1, len(a["t_out"])))(*a["t_out"])
    n_out = len(a["t_out"]) if a["n_out"] is None else a["n_out"]
    rc = lib.spk_reconstruct(a["stream"], a["H"], a["W"], a["T"], a["theta"],
                             ctypes.addressof(t), n_out, a["out"], a["order"], None)
    assert rc == -1


def test_segments_rejects_bad_arguments(lib):
    assert lib.spk_segments(FAKE, 4, 4, 10, 1, -1, FAKE, FAKE, FAKE, FAKE, None) == -1
    assert lib.spk_segments(FAKE, 4, 4, 10, 1, 4, 0, FAKE, FAKE, FAKE, None) == -1
    assert lib.spk_segments(FAKE, 4, 4, 10, 1, 4, FAKE, FAKE, FAKE, 0, None) == -1
    assert lib.spk_segments(FAKE, 4, 4, 10, 5, 4, FAKE, FAKE, FAKE, FAKE, None) == -1
    assert lib.spk_segments(FAKE + 8, 4, 4, 10, 1, 4, FAKE, FAKE, FAKE, FAKE, None) == -1


@pytest.mark.parametrize("args", [
    dict(stream=0), dict(stream=FAKE + 8), dict(H=0), dict(T=-1), dict(theta=0.0),
    dict(theta=float("nan")), dict(window=0), dict(window=-3), dict(n_out=-1),
    dict(t_out=[10]), dict(t_out=[-1]), dict(out=0),
])
def test_tfp_rejects_bad_arguments(lib, args):
    a = dict(stream=FAKE, H=4, W=4, T=10, theta=1.0, window=5, t_out=[0, 5], n_out=None,
             out=FAKE)
    a.update(args)
    t = (ctypes.c_int32 * max(1, len(a["t_out"])))(*a["t_out"])
    n_out = len(a["t_out"]) if a["n_out"] is None else a["n_out"]
    rc = lib.spk_tfp(a["stream"], a["H"], a["W"], a["T"], a["theta"], a["window"],
                     ctypes.addressof(t), n_out, a["out"], None)
    assert rc == -1


@pytest.mark.parametrize("args", [
    dict(count=0), dict(cap=-1), dict(sf=0), dict(H=0), dict(T=0), dict(theta=-2.0),
    dict(n_out=-1), dict(t_out=[10]), dict(t_out=[-1]), dict(out=0),
])
def test_decode_rejects_bad_arguments(lib, args):
    a = dict(sf=FAKE, sl=FAKE, sn=FAKE, count=FAKE, cap=4, H=4, W=4, T=10, theta=1.0,
             t_out=[0, 5], n_out=None, out=FAKE)
    a.update(args)
    t = (ctypes.c_int32 * max(1, len(a["t_out"])))(*a["t_out"])
    n_out = len(a["t_out"]) if a["n_out"] is None else a["n_out"]
    rc = lib.spk_decode(a["sf"], a["sl"], a["sn"], a["count"], a["cap"], a["H"], a["W"], a["T"],
                        a["theta"], ctypes.addressof(t), n_out, a["out"], None)
    assert rc == -1


def test_segments_packed_rejects_bad_arguments(lib):
    assert lib.spk_segments_packed(FAKE, 4, 4, 10, 1, -1, FAKE, FAKE, None) == -1
    assert lib.spk_segments_packed(FAKE, 4, 4, 10, 1, 4, 0, FAKE, None) == -1
    assert lib.spk_segments_packed(FAKE, 4, 4, 10, 1, 4, FAKE, 0, None) == -1
    assert lib.spk_segments_packed(FAKE, 4, 4, 10, 5, 4, FAKE, FAKE, None) == -1
    assert lib.spk_segments_packed(FAKE + 8, 4, 4, 10, 1, 4, FAKE, FAKE, None) == -1
    assert lib.spk_segments_packed(FAKE, 0, 4, 10, 1, 4, FAKE, FAKE, None) == -1


@pytest.mark.parametrize("args", [
    dict(count=0), dict(cap=-1), dict(rec=0), dict(H=0), dict(W=0), dict(T=0), dict(theta=-2.0),
    dict(theta=float("nan")), dict(n_out=-1), dict(t_out=[10]), dict(t_out=[-1]), dict(out=0),
])
def test_decode_packed_rejects_bad_arguments(lib, args):
    a = dict(rec=FAKE, count=FAKE, cap=4, H=4, W=4, T=10, theta=1.0, t_out=[0, 5], n_out=None,
             out=FAKE)
    a.update(args)
    t = (ctypes.c_int32 * max(1, len(a["t_out"])))(*a["t_out"])
    n_out = len(a["t_out"]) if a["n_out"] is None else a["n_out"]
    rc = lib.spk_decode_packed(a["rec"], a["count"], a["cap"], a["H"], a["W"], a["T"],
                               a["theta"], ctypes.addressof(t), n_out, a["out"], None)
    assert rc == -1


@pytest.mark.parametrize("args", [
    dict(stream=0), dict(stream=FAKE + 8), dict(H=0), dict(order=0), dict(window=0),
    dict(n_out=-1),
    dict(t_out=[10]), dict(mask=0),
])
def test_motion_rejects_bad_arguments(lib, args):
    a = dict(stream=FAKE, H=4, W=4, T=10, order=2, window=5, t_out=[0, 5], n_out=None,
             mask=FAKE)
    a.update(args)
    t = (ctypes.c_int32 * max(1, len(a["t_out"])))(*a["t_out"])
    n_out = len(a["t_out"]) if a["n_out"] is None else a["n_out"]
    rc = lib.spk_motion(a["stream"], a["H"], a["W"], a["T"], a["order"], a["window"],
                        ctypes.addressof(t), n_out, a["mask"], None)
    assert rc == -1


def test_zero_outputs_is_noop(lib):
    # n_out == 0 returns before any device work
    assert lib.spk_reconstruct(FAKE, 4, 4, 10, 1.0, None, 0, None, 1, None) == 0


def _job(lib, **kw):
    from paper_2412_11639_amd._lib import SpkJob
    t = (ctypes.c_int32 * 4)(*kw.pop("t_out", [0, 1, 2, 3]))
    a = dict(stream=FAKE, H=4, W=4, T=10, theta=1.0, n_out=4, out=FAKE)
    a.update(kw)
    j = SpkJob(a["stream"], a["H"], a["W"], a["T"], a["theta"], ctypes.addressof(t), a["n_out"],
               a["out"])
    return j, t


@pytest.mark.parametrize("bad", [
    dict(stream=0), dict(stream=FAKE + 8), dict(out=0), dict(H=0), dict(T=-1), dict(theta=0.0),
    dict(theta=float("nan")), dict(n_out=0), dict(t_out=[0, 1, 2, 10]),
    dict(H=65536, W=65536)])
def test_plan_create_rejects_bad_jobs(lib, bad):
    from paper_2412_11639_amd._lib import SpkJob
    good, tg = _job(lib)
    badj, tb = _job(lib, **bad)
    arr = (SpkJob * 2)(good, badj)
    h = ctypes.c_void_p()
    assert lib.spk_plan_create(ctypes.byref(h), arr, 2, 1, 0) == -1
    assert not h.value


def test_plan_create_rejects_bad_arguments(lib):
    from paper_2412_11639_amd._lib import SpkJob
    good, tg = _job(lib)
    arr = (SpkJob * 1)(good)
    h = ctypes.c_void_p()
    assert lib.spk_plan_create(None, arr, 1, 1, 0) == -1
    assert lib.spk_plan_create(ctypes.byref(h), arr, 0, 1, 0) == -1
    assert lib.spk_plan_create(ctypes.byref(h), arr, 1, 5, 0) == -1
    assert lib.spk_plan_create(ctypes.byref(h), arr, 1, 1, 8) == -1
    assert lib.spk_plan_execute(None, None) == -1
    assert lib.spk_plan_destroy(None) == 0


def test_options(lib):
    assert lib.spk_set_option(99, 1) == -1
    assert lib.spk_set_option(1, -1) == -1
    assert lib.spk_get_option(99) == -1
    # option 2 (a former two-layer surrogate kernel switch) no longer exists;
    # surrogate convolution workgroup cap
    assert lib.spk_set_option(2, 0) == -1 and lib.spk_get_option(2) == -1
    assert lib.spk_set_option(3, -1) == -1
    assert lib.spk_set_option(3, 5) == 0 and lib.spk_get_option(3) == 5
    assert lib.spk_set_option(3, 0) == 0 and lib.spk_get_option(3) == 0
    # warm-up tiles of speculative chunks: 0 = automatic
    assert lib.spk_set_option(7, -1) == -1
    assert lib.spk_set_option(7, 2) == 0 and lib.spk_get_option(7) == 2
    assert lib.spk_set_option(7, 0) == 0 and lib.spk_get_option(7) == 0
    # batched plan shape: group size, waves per workgroup, register target
    for opt, good, bad in ((4, (4, 8, 16, 0), (3, 32, -1)), (5, (1, 2, 4, 0), (3, 8, -1)),
                           (6, (1, 0), (2, -1))):
        for v in good:
            assert lib.spk_set_option(opt, v) == 0 and lib.spk_get_option(opt) == v
        for v in bad:
            assert lib.spk_set_option(opt, v) == -1
        assert lib.spk_get_option(opt) == 0


def test_sur_train_plan_rejects_bad_arguments():
    """The graph-replayed training plan validates everything on the host."""
    import paper_2412_11639_amd.surrogate as sur
    lib = sur._lib_sur()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: rejected before use
    good = sur.SurSample(0x2000, 250, 400, 4096, 0, 0, 100, 0x3000)
    lr = (ctypes.c_float * 2)(1e-3, 1e-3)

    def create(samples, steps=2, B=1, Hc=64, Wc=64, theta=1.0, b1=0.9, b2=0.999, eps=1e-8,
               step0=1, lrs=lr, plan=True):
        h = ctypes.c_void_p()
        arr = (sur.SurSample * len(samples))(*samples)
        return lib.spk_sur_train_create(ctypes.byref(h) if plan else None, fake, fake, fake, arr,
                                        ctypes.cast(lrs, ctypes.c_void_p), steps, B, Hc, Wc, theta,
                                        b1, b2, eps, step0, None)

    assert create([good, good], plan=False) == -1
    assert create([good, good], steps=0) == -1
    assert create([good] * 65, steps=1, B=65) == -1
    assert create([good, good], step0=0) == -1
    assert create([good, good], theta=0.0) == -1
    assert create([good, good], b1=1.0) == -1
    assert create([good, good], eps=0.0) == -1
    assert create([good, good], lrs=(ctypes.c_float * 2)(1e-3, 0.0)) == -1
    assert create([good, sur.SurSample(None, 250, 400, 4096, 0, 0, 100, 0x3000)]) == -1
    assert create([good, sur.SurSample(0x2000, 250, 400, 4096, 0, 0, 100, None)]) == -1
    assert create([good, sur.SurSample(0x2000, 250, 400, 4096, 200, 0, 100, 0x3000)]) == -1
    assert create([good, sur.SurSample(0x2000, 250, 400, 4096, 0, 0, 30, 0x3000)]) == -1
    # stream not 16-byte aligned (frames are read as 8-byte words of 16-byte rows)
    assert create([good, sur.SurSample(0x2008, 250, 400, 4096, 0, 0, 100, 0x3000)]) == -1
    assert lib.spk_sur_train_run(None, 1, None) == -1
    assert lib.spk_sur_train_destroy(None) == 0


def test_sur_infer_prepacked_rejects_bad_arguments():
    """The pre-packed inference validates its arguments on the host like
    spk_sur_infer (no device access before that)."""
    import paper_2412_11639_amd.surrogate as sur
    lib = sur._lib_sur()
    p = ctypes.c_void_p(0x1000)   # never dereferenced: rejected before use
    for f in (lib.spk_sur_infer, lib.spk_sur_infer_prepacked):
        assert f(None, p, p, 1, 8, 8, p, p, None) == -1
        assert f(p, None, p, 1, 8, 8, p, p, None) == -1
        assert f(p, p, p, 1, 8, 8, p, None, None) == -1
        assert f(p, p, p, 0, 8, 8, p, p, None) == -1
        assert f(p, p, p, 1, 0, 8, p, p, None) == -1


def test_sur_input_rejects_unaligned_stream():
    """spk_sur_input checks every crop record like the rest of the ABI: a
    stream pointer that is not 16-byte aligned is rejected before any
    launch."""
    import paper_2412_11639_amd.surrogate as sur
    lib = sur._lib_sur()
    p = ctypes.c_void_p(0x1000)   # never dereferenced: rejected before use
    for base, rc in ((0x2008, -1), (0x2004, -1), (0x2001, -1)):
        arr = (sur.SurSample * 1)(sur.SurSample(base, 250, 400, 4096, 0, 0, 100, None))
        assert lib.spk_sur_input(arr, 1, 8, 8, 1.0, p, p, p, None, None) == rc


def test_noalloc_rejects_what_does_not_fit(lib):
    """spk_reconstruct_noalloc checks its fixed scratch limits on the host,
    before any device access: output-time tables past the array are
    SPK_ERANGE, bad arguments SPK_EINVAL as for spk_reconstruct."""
    fake = FAKE   # never dereferenced
    t = (ctypes.c_int32 * 2)(0, 1)
    f = lib.spk_reconstruct_noalloc
    assert f(fake, 8, 8, 1 << 24, 1.0, t, 2, fake, 1, None) == -5
    assert f(fake, 8, 8, 100, 1.0, t, 2, 0, 1, None) == -1        # no out
    assert f(fake + 8, 8, 8, 100, 1.0, t, 2, fake, 1, None) == -1  # unaligned stream
    assert f(fake, 8, 8, 100, 0.0, t, 2, fake, 1, None) == -1      # theta
    assert f(fake, 8, 8, 1, 1.0, t, 2, fake, 1, None) == -1        # t_out >= T
    assert f(fake, 8, 8, 100, 1.0, t, 0, fake, 1, None) == 0       # nothing to do
    assert lib.spk_strerror(-5)


def test_stream_rejects_bad_arguments(lib):
    """spk_stream_create / feed / finish validate on the host; nothing is
    allocated or enqueued for a bad argument."""
    h = ctypes.c_void_p()
    t = (ctypes.c_int32 * 2)(0, 5)
    bad_t = (ctypes.c_int32 * 2)(0, -1)
    create = lib.spk_stream_create
    assert create(None, 4, 4, 1.0, 1, t, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 0, 4, 1.0, 1, t, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 4, 4, 0.0, 1, t, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 4, 4, float("inf"), 1, t, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 4, 4, 1.0, 5, t, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 4, 4, 1.0, 1, None, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 4, 4, 1.0, 1, bad_t, 2, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 4, 4, 1.0, 1, t, -1, FAKE, None, None, None) == -1
    assert create(ctypes.byref(h), 65536, 65536, 1.0, 1, t, 2, FAKE, None, None, None) == -1
    assert not h.value
    assert lib.spk_stream_feed(None, FAKE, 4, None) == -1
    assert lib.spk_stream_finish(None, None) == -1
    assert lib.spk_stream_frames(None) == -1
    assert lib.spk_stream_destroy(None) == 0


def test_surrogate_checkpoint_round_trip(tmp_path):
    """A checkpoint is a plain .npz (no pickles) that restores parameters,
    both Adam moments, the step count and the extra state exactly (CPU
    tensors; the device path is the same code)."""
    import numpy as np
    import torch
    import paper_2412_11639_amd.surrogate as sur
    rng = np.random.default_rng(0)
    m = sur.Surrogate(sur.init_params(1) + rng.normal(0, 0.01, sur.NPARAMS), device="cpu")
    m.m.copy_(torch.from_numpy(rng.normal(0, 1, sur.NPARAMS).astype(np.float32)))
    m.v.copy_(torch.from_numpy(rng.uniform(0, 1, sur.NPARAMS).astype(np.float32)))
    m.step_count = 123
    p = str(tmp_path / "c.npz")
    m.save(p, extra={"rng": rng.bit_generator.state, "note": "x"})
    with np.load(p, allow_pickle=False) as z:
        assert set(z.files) == {"version", "params", "m", "v", "step", "extra"}
    r, extra = sur.Surrogate.load(p, device="cpu")
    assert torch.equal(r.params, m.params) and torch.equal(r.m, m.m) and torch.equal(r.v, m.v)
    assert r.step_count == 123 and extra["note"] == "x"
    assert extra["rng"] == rng.bit_generator.state
