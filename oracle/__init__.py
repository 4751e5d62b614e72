"""Reference oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, double-precision CPU reconstruction (``oracle.c``, built with
gcc) plus the CPU reference of the surrogate network (``conv.py``).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2412_11639_amd``) and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

FSR = 1
SSR = 2
TFI = 3
TSR = 4

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

P_u8 = ctypes.POINTER(ctypes.c_uint8)
P_i32 = ctypes.POINTER(ctypes.c_int32)
P_f64 = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True, src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compile oracle.c with gcc into a shared library."""
    if not force and os.path.exists(out):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", src,
                           "-o", tmp])
    os.replace(tmp, out)
    return out


def _bind(lib):
    lib.spk_oracle_segment_intervals.restype = ctypes.c_int32
    lib.spk_oracle_segment_intervals.argtypes = [P_i32, ctypes.c_int32, ctypes.c_int32, P_i32]
    lib.spk_oracle_reconstruct.restype = ctypes.c_int32
    lib.spk_oracle_reconstruct.argtypes = [
        P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, P_i32,
        ctypes.c_int32, ctypes.c_int32, P_f64, P_i32, P_i32, P_i32, ctypes.c_int32]
    lib.spk_oracle_reconstruct_causal.restype = ctypes.c_int32
    lib.spk_oracle_reconstruct_causal.argtypes = lib.spk_oracle_reconstruct.argtypes
    lib.spk_oracle_tfp.restype = ctypes.c_int32
    lib.spk_oracle_tfp.argtypes = [P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_int32, P_i32, ctypes.c_int32, P_f64]
    lib.spk_oracle_window.restype = ctypes.c_int32
    lib.spk_oracle_window.argtypes = [P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_double, ctypes.c_int32, P_f64,
                                      ctypes.POINTER(ctypes.c_uint8)]
    lib.spk_oracle_stream_create.restype = ctypes.c_void_p
    lib.spk_oracle_stream_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_int32, P_i32, ctypes.c_int32, P_f64, P_i32,
                                             P_i32, P_i32]
    lib.spk_oracle_stream_feed.restype = ctypes.c_int32
    lib.spk_oracle_stream_feed.argtypes = [ctypes.c_void_p, P_u8, ctypes.c_int32]
    lib.spk_oracle_stream_finish.restype = ctypes.c_int32
    lib.spk_oracle_stream_finish.argtypes = [ctypes.c_void_p]
    lib.spk_oracle_stream_destroy.restype = None
    lib.spk_oracle_stream_destroy.argtypes = [ctypes.c_void_p]
    lib.spk_oracle_segments.restype = ctypes.c_int32
    lib.spk_oracle_segments.argtypes = [
        P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
        P_i32, P_i32, P_i32, P_i32, ctypes.c_int32]
    return lib


def load(path: str | None = None):
    """Load the oracle library (building it if absent); ``path`` loads another
    build of the same source, e.g. a deliberately broken copy in a test."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _nthreads(n):
    # at most 16 threads: one GPU's share of the host's cores
    return int(n if n is not None else min(16, len(os.sched_getaffinity(0))))


def segment_intervals(x, order: int = FSR, lib=None) -> list:
    """Segment an interval stream S1 directly; returns the list of segment
    start indices (0-based interval indices)."""
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.int32)
    start = np.zeros(max(1, len(x)), dtype=np.int32)
    n = lib.spk_oracle_segment_intervals(_ptr(x, P_i32), len(x), order, _ptr(start, P_i32))
    if n < 0:
        raise ValueError("bad arguments")
    return start[:n].tolist()


def reconstruct(stream, H, W, T, theta, t_out, order=FSR, windows=False, nthreads=None,
                lib=None, causal=False):
    """Intensity per output time and pixel, [n_out, H, W] float64.  With
    ``windows`` also returns (first, last, n) int32 arrays of the same shape.
    With ``causal`` the output at t is the method's result on frames 0..t
    alone (streaming reading)."""
    lib = lib or load()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    t_out = np.ascontiguousarray(t_out, dtype=np.int32)
    n_out = len(t_out)
    out = np.zeros((n_out, H, W), dtype=np.float64)
    wf = wl = wn = None
    if windows:
        wf = np.zeros((n_out, H, W), dtype=np.int32)
        wl = np.zeros((n_out, H, W), dtype=np.int32)
        wn = np.zeros((n_out, H, W), dtype=np.int32)
    fn = lib.spk_oracle_reconstruct_causal if causal else lib.spk_oracle_reconstruct
    rc = fn(_ptr(stream, P_u8), H, W, T, float(theta), _ptr(t_out, P_i32), n_out, order,
            _ptr(out, P_f64), _ptr(wf, P_i32), _ptr(wl, P_i32), _ptr(wn, P_i32),
            _nthreads(nthreads))
    if rc != 0:
        raise ValueError("spk_oracle_reconstruct: bad arguments")
    return (out, wf, wl, wn) if windows else out


def tfp(stream, H, W, T, theta, window, t_out, lib=None):
    """TFP: theta * (spikes in the window of ``window`` frames ending at t)
    / window length, [n_out, H, W] float64."""
    lib = lib or load()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    t_out = np.ascontiguousarray(t_out, dtype=np.int32)
    out = np.zeros((len(t_out), H, W), dtype=np.float64)
    rc = lib.spk_oracle_tfp(_ptr(stream, P_u8), H, W, T, float(theta), int(window),
                            _ptr(t_out, P_i32), len(t_out), _ptr(out, P_f64))
    if rc != 0:
        raise ValueError("spk_oracle_tfp: bad arguments")
    return out


def motion(stream, H, W, T, window, t_out, order=SSR, lib=None):
    """Static / motion mask (uint8 [n_out, H, W]): 1 where the segment that
    holds the interval in progress at t began at a cut less than ``window``
    frames back -- its first spike f > t - window and it is not the pixel's
    first segment (whose start is the first spike, no cut)."""
    _, wf, _, _ = reconstruct(stream, H, W, T, 1.0, t_out, order=order, windows=True, lib=lib)
    first = segments(stream, H, W, T, order=order, cap=1, lib=lib)[0][0].reshape(H, W)
    t = np.asarray(t_out, dtype=np.int64).reshape(-1, 1, 1)
    return ((wf >= 0) & (wf != first[None]) & (wf > t - window)).astype(np.uint8)


def segments(stream, H, W, T, order=FSR, cap=64, nthreads=None, lib=None):
    """All segments per pixel: (first, last, n) each [cap, H*W] int32, and
    the total count per pixel [H*W]."""
    lib = lib or load()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    hw = H * W
    sf = np.full((cap, hw), -1, dtype=np.int32)
    sl = np.full((cap, hw), -1, dtype=np.int32)
    sn = np.zeros((cap, hw), dtype=np.int32)
    cnt = np.zeros(hw, dtype=np.int32)
    rc = lib.spk_oracle_segments(_ptr(stream, P_u8), H, W, T, order, cap, _ptr(sf, P_i32),
                                 _ptr(sl, P_i32), _ptr(sn, P_i32), _ptr(cnt, P_i32),
                                 _nthreads(nthreads))
    if rc != 0:
        raise ValueError("spk_oracle_segments: bad arguments")
    return sf, sl, sn, cnt


def window_estimate(stream, H, W, T, theta, t, lib=None):
    """Short-window estimate and stability flag at output time t (>= 31):
    (est float64 [H, W], stable bool [H, W])."""
    lib = lib or load()
    stream = np.ascontiguousarray(stream, dtype=np.uint8)
    est = np.zeros((H, W), dtype=np.float64)
    st = np.zeros((H, W), dtype=np.uint8)
    rc = lib.spk_oracle_window(_ptr(stream, P_u8), H, W, T, float(theta), int(t),
                               _ptr(est, P_f64), st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise ValueError("spk_oracle_window: bad arguments")
    return est, st.astype(bool)


class Stream:
    """The method online (O-5): frames fed in pieces, a small per-pixel
    state carried between pieces; ``finish`` writes every output still
    waiting.  After finish, ``out`` (and with ``windows`` the first/last/n
    arrays) hold what ``reconstruct`` gives on the whole stream."""

    def __init__(self, H, W, theta, t_out, order=FSR, windows=False, lib=None):
        self.lib = lib or load()
        self.H, self.W = H, W
        self.t_out = np.ascontiguousarray(t_out, dtype=np.int32)
        n_out = len(self.t_out)
        self.out = np.zeros((n_out, H, W), dtype=np.float64)
        self.wf = self.wl = self.wn = None
        if windows:
            self.wf = np.zeros((n_out, H, W), dtype=np.int32)
            self.wl = np.zeros((n_out, H, W), dtype=np.int32)
            self.wn = np.zeros((n_out, H, W), dtype=np.int32)
        self._h = self.lib.spk_oracle_stream_create(
            H, W, float(theta), order, _ptr(self.t_out, P_i32), n_out, _ptr(self.out, P_f64),
            _ptr(self.wf, P_i32), _ptr(self.wl, P_i32), _ptr(self.wn, P_i32))
        if not self._h:
            raise ValueError("spk_oracle_stream_create: bad arguments")

    def feed(self, frames):
        frames = np.ascontiguousarray(frames, dtype=np.uint8)
        if self.lib.spk_oracle_stream_feed(self._h, _ptr(frames, P_u8), frames.shape[0]) != 0:
            raise ValueError("spk_oracle_stream_feed: bad arguments")

    def finish(self):
        self.lib.spk_oracle_stream_finish(self._h)
        return (self.out, self.wf, self.wl, self.wn) if self.wf is not None else self.out

    def __del__(self):
        if getattr(self, "_h", None):
            self.lib.spk_oracle_stream_destroy(self._h)
            self._h = None
