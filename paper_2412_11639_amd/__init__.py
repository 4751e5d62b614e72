"""Spike-camera reconstruction on MI355X (gfx950): Python binding of libspk.

Thin argument marshalling over the C ABI in ``include/spk.h``: every step of
the reconstruction runs in the library's HIP kernels.  PyTorch supplies
device memory and the current HIP stream only.

Method: arXiv 2412.11639 -- inter-spike intervals cut into zero-order stable
segments at first (FSR) or second (SSR) order, intensity theta*N/duration
per segment (Eq. 6).  The baselines it is compared with (Sec. II): TFI as a
third order (every interval alone) and TFP (``tfp``, windowed spike counts).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import SpkError

FSR = 1
SSR = 2
TFI = 3
TSR = 4

__all__ = ["FSR", "SSR", "TFI", "TSR", "SpkError", "tfp", "decode", "motion", "frame_bytes", "reconstruct", "reconstruct_windows",
           "segments", "segments_packed", "decode_packed", "version", "set_time_chunks", "get_time_chunks",
           "set_warm_tiles", "get_warm_tiles", "Plan",
           "PLAN_AUTOTUNE", "PLAN_NO_GRAPH"]

PLAN_AUTOTUNE = 1
PLAN_NO_GRAPH = 2


def frame_bytes(H: int, W: int) -> int:
    """Bytes per packed frame: ceil(H*W/128)*16."""
    return int(_lib.load().spk_frame_bytes(H, W))


OPT_TIME_CHUNKS = 1
OPT_WARM_TILES = 7


def version() -> int:
    return int(_lib.load().spk_version())


def set_time_chunks(n: int) -> None:
    """Number of time chunks for long streams (0 = automatic).  Results are
    identical for every setting; only the degree of parallelism changes."""
    _lib.check("spk_set_option", _lib.load().spk_set_option(OPT_TIME_CHUNKS, int(n)))


def get_time_chunks() -> int:
    return int(_lib.load().spk_get_option(OPT_TIME_CHUNKS))


def set_warm_tiles(n: int) -> None:
    """64-frame tiles each speculative time chunk warms up on (0 =
    automatic).  Results are identical for every setting."""
    _lib.check("spk_set_option", _lib.load().spk_set_option(OPT_WARM_TILES, int(n)))


def get_warm_tiles() -> int:
    return int(_lib.load().spk_get_option(OPT_WARM_TILES))


OPT_PLAN_KGROUP, OPT_PLAN_WAVES_PER_WG, OPT_PLAN_WPE = 4, 5, 6


def set_plan_shape(kgroup: int = 0, waves_per_wg: int = 0, wpe_variant: int = 0) -> None:
    """Launch shape of plans created without autotuning (0 = default).
    Results are identical for every shape."""
    lib = _lib.load()
    for opt, v in ((OPT_PLAN_KGROUP, kgroup), (OPT_PLAN_WAVES_PER_WG, waves_per_wg),
                   (OPT_PLAN_WPE, wpe_variant)):
        _lib.check("spk_set_option", lib.spk_set_option(opt, int(v)))


OPT_SUR_CONV_WG = 3


def set_surrogate_conv_workgroups(n: int) -> None:
    """Cap the workgroups of each layer-by-layer surrogate convolution (0:
    as many as fit on the device).  Results are identical."""
    _lib.check("spk_set_option", _lib.load().spk_set_option(OPT_SUR_CONV_WG, int(n)))


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check_stream_tensor(stream_t, H, W, T):
    if not isinstance(stream_t, torch.Tensor) or not stream_t.is_cuda:
        raise TypeError("stream must be a device tensor")
    if stream_t.dtype != torch.uint8 or not stream_t.is_contiguous():
        raise TypeError("stream must be contiguous uint8")
    if stream_t.numel() < T * frame_bytes(H, W):
        raise ValueError("stream holds fewer than T frames")


def _host_times(t_out):
    t = np.ascontiguousarray(np.asarray(t_out, dtype=np.int32).reshape(-1))
    return t, t.ctypes.data


def reconstruct(stream_t: torch.Tensor, H: int, W: int, T: int, theta: float, t_out,
                order: int = FSR, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Intensity at each output frame: float32 [n_out, H, W] on the device.

    ``stream_t``: device uint8 tensor of T packed frames; ``t_out``: host
    sequence of frame indices (any order, duplicates allowed)."""
    _check_stream_tensor(stream_t, H, W, T)
    t, tp = _host_times(t_out)
    n_out = len(t)
    if out is None:
        out = torch.empty((n_out, H, W), dtype=torch.float32, device=stream_t.device)
    assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n_out * H * W
    rc = _lib.load().spk_reconstruct(stream_t.data_ptr(), H, W, T, float(theta), tp, n_out,
                                     out.data_ptr(), order, _stream_handle(stream))
    _lib.check("spk_reconstruct", rc)
    return out


def reconstruct_noalloc(stream_t: torch.Tensor, H: int, W: int, T: int, theta: float, t_out,
                        out: torch.Tensor, order: int = FSR, stream=None) -> torch.Tensor:
    """``reconstruct`` through the allocation-free entry point
    (``spk_reconstruct_noalloc``): the caller passes ``out``; the library
    allocates nothing and uses its fixed per-GPU scratch array."""
    _check_stream_tensor(stream_t, H, W, T)
    t, tp = _host_times(t_out)
    n_out = len(t)
    assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n_out * H * W
    rc = _lib.load().spk_reconstruct_noalloc(stream_t.data_ptr(), H, W, T, float(theta), tp,
                                             n_out, out.data_ptr(), order, _stream_handle(stream))
    _lib.check("spk_reconstruct_noalloc", rc)
    return out


def tfp(stream_t, H, W, T, theta, window, t_out, out=None, stream=None):
    """TFP baseline: theta * (spikes in the ``window`` frames ending at t) /
    window length (clipped at frame 0), float32 [n_out, H, W]."""
    _check_stream_tensor(stream_t, H, W, T)
    t, tp = _host_times(t_out)
    n_out = len(t)
    if out is None:
        out = torch.empty((n_out, H, W), dtype=torch.float32, device=stream_t.device)
    assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n_out * H * W
    rc = _lib.load().spk_tfp(stream_t.data_ptr(), H, W, T, float(theta), int(window), tp, n_out,
                             out.data_ptr(), _stream_handle(stream))
    _lib.check("spk_tfp", rc)
    return out


def decode(seg_first, seg_last, seg_n, count, H, W, T, theta, t_out, out=None, stream=None):
    """Intensity at the requested frames from segment lists (as returned by
    ``segments``), float32 [n_out, H, W]; NaN where a list was cut at cap."""
    cap = seg_first.shape[0]
    for a in (seg_first, seg_last, seg_n):
        assert a.dtype == torch.int32 and a.is_contiguous() and a.shape == (cap, H * W)
    assert count.dtype == torch.int32 and count.numel() == H * W
    t, tp = _host_times(t_out)
    n_out = len(t)
    if out is None:
        out = torch.empty((n_out, H, W), dtype=torch.float32, device=count.device)
    assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n_out * H * W
    rc = _lib.load().spk_decode(seg_first.data_ptr(), seg_last.data_ptr(), seg_n.data_ptr(),
                                count.data_ptr(), cap, H, W, T, float(theta), tp, n_out,
                                out.data_ptr(), _stream_handle(stream))
    _lib.check("spk_decode", rc)
    return out


def segments_packed(stream_t, H, W, T, order=FSR, cap=64, stream=None):
    """Every segment of every pixel, each pixel's list contiguous: records
    int32 [H*W, cap, 3] (first, last, n) and the per-pixel total count
    int32 [H*W]."""
    _check_stream_tensor(stream_t, H, W, T)
    dev = stream_t.device
    hw = H * W
    rec = torch.empty((hw, cap, 3), dtype=torch.int32, device=dev)
    if cap:
        rec[..., :2].fill_(-1)
        rec[..., 2].zero_()
    cnt = torch.zeros(hw, dtype=torch.int32, device=dev)
    rc = _lib.load().spk_segments_packed(stream_t.data_ptr(), H, W, T, order, cap,
                                         rec.data_ptr(), cnt.data_ptr(), _stream_handle(stream))
    _lib.check("spk_segments_packed", rc)
    return rec, cnt


def decode_packed(rec, count, H, W, T, theta, t_out, out=None, stream=None):
    """``decode`` from per-pixel contiguous lists (as ``segments_packed``
    returns them)."""
    cap = rec.shape[1]
    assert rec.dtype == torch.int32 and rec.is_contiguous() and rec.shape == (H * W, cap, 3)
    assert count.dtype == torch.int32 and count.numel() == H * W
    t, tp = _host_times(t_out)
    n_out = len(t)
    if out is None:
        out = torch.empty((n_out, H, W), dtype=torch.float32, device=count.device)
    assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n_out * H * W
    rc = _lib.load().spk_decode_packed(rec.data_ptr(), count.data_ptr(), cap, H, W, T,
                                       float(theta), tp, n_out, out.data_ptr(),
                                       _stream_handle(stream))
    _lib.check("spk_decode_packed", rc)
    return out


def motion(stream_t, H, W, T, window, t_out, order=SSR, stream=None):
    """Static / motion mask, uint8 [n_out, H, W]: 1 where the segment holding
    t begins at a cut less than ``window`` frames back."""
    _check_stream_tensor(stream_t, H, W, T)
    t, tp = _host_times(t_out)
    n_out = len(t)
    mask = torch.empty((n_out, H, W), dtype=torch.uint8, device=stream_t.device)
    rc = _lib.load().spk_motion(stream_t.data_ptr(), H, W, T, order, int(window), tp, n_out,
                                mask.data_ptr(), _stream_handle(stream))
    _lib.check("spk_motion", rc)
    return mask


def reconstruct_windows(stream_t, H, W, T, theta, t_out, order=FSR, stream=None):
    """Intensity plus the window of the segment used for each output:
    (out float32, first int32, last int32, n int32), each [n_out, H, W]."""
    _check_stream_tensor(stream_t, H, W, T)
    t, tp = _host_times(t_out)
    n_out = len(t)
    dev = stream_t.device
    out = torch.empty((n_out, H, W), dtype=torch.float32, device=dev)
    wf, wl, wn = (torch.empty((n_out, H, W), dtype=torch.int32, device=dev) for _ in range(3))
    rc = _lib.load().spk_reconstruct_windows(stream_t.data_ptr(), H, W, T, float(theta), tp,
                                             n_out, out.data_ptr(), wf.data_ptr(),
                                             wl.data_ptr(), wn.data_ptr(), order,
                                             _stream_handle(stream))
    _lib.check("spk_reconstruct_windows", rc)
    return out, wf, wl, wn


def segments(stream_t, H, W, T, order=FSR, cap=64, stream=None):
    """Every segment of every pixel: (first, last, n) int32 [cap, H*W] and
    the per-pixel total count int32 [H*W]."""
    _check_stream_tensor(stream_t, H, W, T)
    dev = stream_t.device
    hw = H * W
    sf = torch.full((cap, hw), -1, dtype=torch.int32, device=dev)
    sl = torch.full((cap, hw), -1, dtype=torch.int32, device=dev)
    sn = torch.zeros((cap, hw), dtype=torch.int32, device=dev)
    cnt = torch.zeros(hw, dtype=torch.int32, device=dev)
    rc = _lib.load().spk_segments(stream_t.data_ptr(), H, W, T, order, cap, sf.data_ptr(),
                                  sl.data_ptr(), sn.data_ptr(), cnt.data_ptr(),
                                  _stream_handle(stream))
    _lib.check("spk_segments", rc)
    return sf, sl, sn, cnt


class Stream:
    """Carry-state reconstruction of a live stream (``spk_stream_*``):
    ``feed`` device frames in pieces of any length, then ``finish``; the
    outputs (float32 [n_out, H, W], and with ``windows`` the first / last /
    n int32 arrays) then equal ``reconstruct`` on the whole stream.  All
    calls go on one HIP stream (the current one unless given)."""

    def __init__(self, H: int, W: int, theta: float, t_out, order: int = FSR,
                 windows: bool = False, device="cuda", out: torch.Tensor | None = None):
        import ctypes
        self.H, self.W = int(H), int(W)
        self._t, tp = _host_times(t_out)
        n_out = len(self._t)
        if out is None:
            out = torch.empty((n_out, H, W), dtype=torch.float32, device=device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() >= n_out * H * W
        self.out = out
        self.windows = None
        if windows:
            self.windows = tuple(torch.empty((n_out, H, W), dtype=torch.int32, device=device)
                                 for _ in range(3))
        wp = [w.data_ptr() for w in self.windows] if windows else [None, None, None]
        h = ctypes.c_void_p()
        _lib.check("spk_stream_create", _lib.load().spk_stream_create(
            ctypes.byref(h), self.H, self.W, float(theta), order, tp, n_out,
            self.out.data_ptr(), *wp))
        self._h = h
        self._frames = []   # pieces stay alive until finish

    def feed(self, frames: torch.Tensor, stream=None):
        if not isinstance(frames, torch.Tensor) or not frames.is_cuda:
            raise TypeError("frames must be a device tensor")
        fb = frame_bytes(self.H, self.W)
        n = frames.shape[0] if frames.numel() else 0
        if frames.dtype != torch.uint8 or not frames.is_contiguous() or frames.numel() != n * fb:
            raise ValueError("frames must be contiguous uint8 [n, %d]" % fb)
        self._frames.append(frames)
        _lib.check("spk_stream_feed", _lib.load().spk_stream_feed(
            self._h, frames.data_ptr() if n else None, n, _stream_handle(stream)))

    def frames(self) -> int:
        return int(_lib.load().spk_stream_frames(self._h))

    def finish(self, stream=None):
        _lib.check("spk_stream_finish", _lib.load().spk_stream_finish(self._h,
                                                                      _stream_handle(stream)))
        return (self.out,) + self.windows if self.windows else self.out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check("spk_stream_destroy", _lib.load().spk_stream_destroy(self._h))
            self._h = None
            self._frames = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A batched reconstruction of several streams (``spk_plan_*``).

    ``jobs`` is a sequence of dicts with keys ``stream`` (device uint8
    tensor), ``H``, ``W``, ``T``, ``t_out`` (host sequence), ``theta``
    (default 1.0) and optionally ``out`` (device float32 tensor
    [n_out, H, W]; allocated if absent).  The tensors must stay alive and in
    place for the plan's life; ``execute`` re-runs the captured graph."""

    def __init__(self, jobs, order: int = FSR, autotune: bool = True, graph: bool = True):
        import ctypes
        lib = _lib.load()
        self.jobs = []
        arr = (_lib.SpkJob * len(jobs))()
        self._keep = []
        for i, j in enumerate(jobs):
            H, W, T = int(j["H"]), int(j["W"]), int(j["T"])
            _check_stream_tensor(j["stream"], H, W, T)
            t, tp = _host_times(j["t_out"])
            out = j.get("out")
            if out is None:
                out = torch.empty((len(t), H, W), dtype=torch.float32, device=j["stream"].device)
            assert out.dtype == torch.float32 and out.is_contiguous()
            assert out.numel() >= len(t) * H * W
            self._keep.append((j["stream"], t, out))
            self.jobs.append(dict(j, out=out))
            arr[i] = _lib.SpkJob(j["stream"].data_ptr(), H, W, T, float(j.get("theta", 1.0)), tp,
                                 len(t), out.data_ptr())
        flags = (PLAN_AUTOTUNE if autotune else 0) | (0 if graph else PLAN_NO_GRAPH)
        handle = ctypes.c_void_p()
        rc = lib.spk_plan_create(ctypes.byref(handle), arr, len(jobs), order, flags)
        _lib.check("spk_plan_create", rc)
        self._h = handle

    def execute(self, stream=None):
        _lib.check("spk_plan_execute", _lib.load().spk_plan_execute(self._h,
                                                                    _stream_handle(stream)))

    def info(self):
        import ctypes
        g, b, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check("spk_plan_info", _lib.load().spk_plan_info(self._h, ctypes.byref(g),
                                                              ctypes.byref(b), ctypes.byref(n)))
        return {"grid": g.value, "grab": b.value, "items": n.value}

    def shape(self):
        """Tiles per prefetch group, waves per workgroup, waves per SIMD."""
        import ctypes
        k, w, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check("spk_plan_shape", _lib.load().spk_plan_shape(
            self._h, ctypes.byref(k), ctypes.byref(w), ctypes.byref(e)))
        return {"kgroup": k.value, "waves_per_wg": w.value, "waves_per_simd": e.value}

    def outputs(self):
        return [j["out"] for j in self.jobs]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check("spk_plan_destroy", _lib.load().spk_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
