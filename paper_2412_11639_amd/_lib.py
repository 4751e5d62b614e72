"""ctypes loader for the in-tree ``libspk.so`` (gfx950).

There is no fallback: if the library is missing or cannot be loaded the
import of anything that computes raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libspk.so")

P_u8 = ctypes.c_void_p
P_i32 = ctypes.c_void_p
P_f32 = ctypes.c_void_p
c_i32 = ctypes.c_int32

_lib = None


class SpkError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__("%s failed: %s (%d)" % (fn, msg, code))
        self.code = code


def _declare(lib):
    lib.spk_frame_bytes.restype = ctypes.c_size_t
    lib.spk_frame_bytes.argtypes = [c_i32, c_i32]
    lib.spk_strerror.restype = ctypes.c_char_p
    lib.spk_strerror.argtypes = [ctypes.c_int]
    lib.spk_version.restype = ctypes.c_int
    lib.spk_version.argtypes = []
    lib.spk_set_option.restype = ctypes.c_int
    lib.spk_set_option.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.spk_get_option.restype = ctypes.c_int
    lib.spk_get_option.argtypes = [ctypes.c_int]
    lib.spk_reconstruct.restype = ctypes.c_int
    lib.spk_reconstruct.argtypes = [P_u8, c_i32, c_i32, c_i32, ctypes.c_float, P_i32, c_i32,
                                    P_f32, c_i32, ctypes.c_void_p]
    lib.spk_reconstruct_windows.restype = ctypes.c_int
    lib.spk_reconstruct_windows.argtypes = [P_u8, c_i32, c_i32, c_i32, ctypes.c_float, P_i32,
                                            c_i32, P_f32, P_i32, P_i32, P_i32, c_i32,
                                            ctypes.c_void_p]
    lib.spk_tfp.restype = ctypes.c_int
    lib.spk_tfp.argtypes = [P_u8, c_i32, c_i32, c_i32, ctypes.c_float, c_i32, P_i32, c_i32, P_f32,
                            ctypes.c_void_p]
    lib.spk_decode.restype = ctypes.c_int
    lib.spk_decode.argtypes = [P_i32, P_i32, P_i32, P_i32, c_i32, c_i32, c_i32, c_i32,
                               ctypes.c_float, P_i32, c_i32, P_f32, ctypes.c_void_p]
    lib.spk_motion.restype = ctypes.c_int
    lib.spk_motion.argtypes = [P_u8, c_i32, c_i32, c_i32, c_i32, c_i32, P_i32, c_i32,
                               ctypes.c_void_p, ctypes.c_void_p]
    lib.spk_segments.restype = ctypes.c_int
    lib.spk_segments.argtypes = [P_u8, c_i32, c_i32, c_i32, c_i32, c_i32, P_i32, P_i32, P_i32,
                                 P_i32, ctypes.c_void_p]
    lib.spk_segments_packed.restype = ctypes.c_int
    lib.spk_segments_packed.argtypes = [P_u8, c_i32, c_i32, c_i32, c_i32, c_i32, P_i32, P_i32,
                                        ctypes.c_void_p]
    lib.spk_decode_packed.restype = ctypes.c_int
    lib.spk_decode_packed.argtypes = [P_i32, P_i32, c_i32, c_i32, c_i32, c_i32, ctypes.c_float,
                                      P_i32, c_i32, P_f32, ctypes.c_void_p]
    for name, argtypes in EXTRA_DECLS.items():
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = argtypes
    return lib


class SpkJob(ctypes.Structure):
    """Mirror of ``spk_job`` in include/spk.h."""
    _fields_ = [("stream", ctypes.c_void_p), ("H", c_i32), ("W", c_i32), ("T", c_i32),
                ("theta", ctypes.c_float), ("t_out", ctypes.c_void_p), ("n_out", c_i32),
                ("out", ctypes.c_void_p)]


EXTRA_DECLS: dict = {
    "spk_reconstruct_noalloc": [P_u8, c_i32, c_i32, c_i32, ctypes.c_float, P_i32, c_i32, P_f32,
                                c_i32, ctypes.c_void_p],
    "spk_stream_create": [ctypes.POINTER(ctypes.c_void_p), c_i32, c_i32, ctypes.c_float, c_i32,
                          P_i32, c_i32, P_f32, P_i32, P_i32, P_i32],
    "spk_stream_feed": [ctypes.c_void_p, P_u8, c_i32, ctypes.c_void_p],
    "spk_stream_finish": [ctypes.c_void_p, ctypes.c_void_p],
    "spk_stream_frames": [ctypes.c_void_p],
    "spk_stream_destroy": [ctypes.c_void_p],
    "spk_plan_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(SpkJob), c_i32, c_i32,
                        c_i32],
    "spk_plan_execute": [ctypes.c_void_p, ctypes.c_void_p],
    "spk_plan_shape": [ctypes.c_void_p, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                       ctypes.POINTER(c_i32)],
    "spk_plan_info": [ctypes.c_void_p, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                      ctypes.POINTER(c_i32)],
    "spk_plan_destroy": [ctypes.c_void_p],
}


def load():
    """Load libspk.so (building it first only if no build exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _build
            _build.build()
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def check(fn: str, code: int):
    if code != 0:
        msg = load().spk_strerror(code).decode()
        raise SpkError(fn, code, msg)
