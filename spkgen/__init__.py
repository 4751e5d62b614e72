"""Seeded synthetic spike streams (input generation only).

The C source ``gen.c`` models the sensor (discrete integrate-and-fire with a
subtract-threshold reset, Eq. 2) and packs binary frames in the layout the
reconstruction library reads: frame-major, ``fb = ceil(H*W/128)*16`` bytes
per frame, pixel ``p = y*W + x`` at bit ``p & 7`` of byte ``p >> 3``.

Nothing here reconstructs anything: the reference oracle and the GPU library
both consume these streams, and neither shares code with the other.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libspkgen.so")
_lib = None

P_u8 = ctypes.POINTER(ctypes.c_uint8)
P_i64 = ctypes.POINTER(ctypes.c_int64)
P_i32 = ctypes.POINTER(ctypes.c_int32)
P_f32 = ctypes.POINTER(ctypes.c_float)


def build(force: bool = True) -> str:
    """Compile gen.c with gcc into spkgen/_build/libspkgen.so."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-pthread",
         _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.spkgen_frame_bytes.restype = ctypes.c_size_t
        lib.spkgen_frame_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.spkgen_rng_u64.restype = ctypes.c_uint64
        lib.spkgen_rng_u64.argtypes = [ctypes.c_uint64] * 3
        lib.spkgen_from_increments.argtypes = [
            P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P_i64, ctypes.c_int32,
            P_i64, ctypes.c_int64, ctypes.c_int32]
        lib.spkgen_blocks.argtypes = [
            P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int32]
        lib.spkgen_blocks_truth.argtypes = [
            P_f32, ctypes.c_int32, ctypes.c_int32, P_i32, ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double]
        lib.spkgen_gratings.argtypes = [
            P_u8, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_double, ctypes.c_int32]
        lib.spkgen_gratings_truth.argtypes = [
            P_f32, ctypes.c_int32, ctypes.c_int32, P_i32, ctypes.c_int32, ctypes.c_uint64,
            ctypes.c_double]
        _lib = lib
    return _lib


def _threads(n):
    if n is None:
        n = min(16, os.cpu_count() or 1)
    return int(n)


def frame_bytes(H: int, W: int) -> int:
    """Bytes per packed frame: ceil(H*W/128)*16 (every frame 16-byte aligned)."""
    return ((H * W + 127) // 128) * 16


def rng_u64(seed: int, tag: int, i: int) -> int:
    return int(_load().spkgen_rng_u64(seed, tag, i))


def pack(bits: np.ndarray) -> np.ndarray:
    """Pack a [T, H, W] (or [T, H*W]) 0/1 array into [T, fb] uint8 frames."""
    bits = np.asarray(bits)
    T = bits.shape[0]
    flat = bits.reshape(T, -1).astype(np.uint8)
    hw = flat.shape[1]
    fb = ((hw + 127) // 128) * 16
    padded = np.zeros((T, fb * 8), dtype=np.uint8)
    padded[:, :hw] = flat
    return np.packbits(padded, axis=1, bitorder="little")


def unpack(stream: np.ndarray, H: int, W: int) -> np.ndarray:
    """Inverse of pack: [T, fb] uint8 -> [T, H, W] uint8 of 0/1."""
    stream = np.asarray(stream, dtype=np.uint8)
    T = stream.shape[0]
    bits = np.unpackbits(stream.reshape(T, -1), axis=1, bitorder="little")
    return bits[:, : H * W].reshape(T, H, W)


def from_increments(inc: np.ndarray, v0: np.ndarray, theta: int, H: int, W: int,
                    T: int | None = None, nthreads=None) -> np.ndarray:
    """Integrate-and-fire (Eq. 2) of integer increments.

    ``inc`` is [H*W] (a constant rate per pixel, needs ``T``) or [T, H*W];
    ``v0`` is the initial accumulator per pixel.  Returns [T, fb] uint8.
    """
    inc = np.ascontiguousarray(inc, dtype=np.int64)
    v0 = np.ascontiguousarray(np.broadcast_to(np.asarray(v0, dtype=np.int64), (H * W,)))
    per_frame = 1 if inc.ndim == 2 else 0
    if per_frame:
        T = inc.shape[0]
    assert T is not None and T > 0
    assert inc.reshape(-1).shape[0] == (T * H * W if per_frame else H * W)
    out = np.zeros((T, frame_bytes(H, W)), dtype=np.uint8)
    rc = _load().spkgen_from_increments(
        out.ctypes.data_as(P_u8), H, W, T, inc.ctypes.data_as(P_i64), per_frame,
        v0.ctypes.data_as(P_i64), int(theta), _threads(nthreads))
    if rc != 0:
        raise ValueError("spkgen_from_increments failed (%d)" % rc)
    return out


def blocks(H: int, W: int, T: int, seed: int, block: int = 16, qmin: float = 0.02,
           qmax: float = 1.0, vx: float = 0.0, vy: float = 0.0, nthreads=None) -> np.ndarray:
    """Piecewise-constant blocks (threshold 65536, increment round(q*65536))."""
    out = np.zeros((T, frame_bytes(H, W)), dtype=np.uint8)
    rc = _load().spkgen_blocks(out.ctypes.data_as(P_u8), H, W, T, seed, block, qmin, qmax,
                               vx, vy, _threads(nthreads))
    if rc != 0:
        raise ValueError("spkgen_blocks failed (%d)" % rc)
    return out


def blocks_truth(H, W, frames, seed, block=16, qmin=0.02, qmax=1.0, vx=0.0, vy=0.0):
    frames = np.ascontiguousarray(frames, dtype=np.int32)
    out = np.zeros((len(frames), H, W), dtype=np.float32)
    rc = _load().spkgen_blocks_truth(out.ctypes.data_as(P_f32), H, W,
                                     frames.ctypes.data_as(P_i32), len(frames), seed, block,
                                     qmin, qmax, vx, vy)
    if rc != 0:
        raise ValueError("spkgen_blocks_truth failed (%d)" % rc)
    return out


def gratings(H: int, W: int, T: int, seed: int, phi: float = 1000.0, nthreads=None):
    """Moving gratings + rotating disk with Poisson photon noise."""
    out = np.zeros((T, frame_bytes(H, W)), dtype=np.uint8)
    rc = _load().spkgen_gratings(out.ctypes.data_as(P_u8), H, W, T, seed, phi,
                                 _threads(nthreads))
    if rc != 0:
        raise ValueError("spkgen_gratings failed (%d)" % rc)
    return out


def gratings_truth(H, W, frames, seed, phi=1000.0):
    frames = np.ascontiguousarray(frames, dtype=np.int32)
    out = np.zeros((len(frames), H, W), dtype=np.float32)
    rc = _load().spkgen_gratings_truth(out.ctypes.data_as(P_f32), H, W,
                                       frames.ctypes.data_as(P_i32), len(frames), seed, phi)
    if rc != 0:
        raise ValueError("spkgen_gratings_truth failed (%d)" % rc)
    return out


# ---------------------------------------------------------------------------
# Named workloads (shapes and seeds of the measured configurations)

@dataclass(frozen=True)
class Workload:
    name: str
    H: int
    W: int
    T: int
    seed: int
    kind: str          # "blocks" | "gratings"
    out_every: int = 0  # 0: explicit times below
    t_out: tuple = ()

    def times(self) -> np.ndarray:
        if self.out_every:
            return np.arange(0, self.T, self.out_every, dtype=np.int32)
        return np.asarray(self.t_out, dtype=np.int32)

    def generate(self, T: int | None = None, nthreads=None) -> np.ndarray:
        T = self.T if T is None else T
        if self.kind == "blocks":
            return blocks(self.H, self.W, T, self.seed, nthreads=nthreads)
        return gratings(self.H, self.W, T, self.seed, nthreads=nthreads)


# 250x400 static blocks, 1024 frames, 8 outputs at 64 + 128 k
BLOCKS_250x400 = Workload("blocks_250x400_T1024", 250, 400, 1024, 1, "blocks",
                          t_out=tuple(64 + 128 * k for k in range(8)))
# 250x400 moving gratings + disk with Poisson noise, 20000 frames, every 10th out
GRATINGS_250x400 = Workload("gratings_250x400_T20000_every10", 250, 400, 20000, 2,
                            "gratings", out_every=10)


# 16 streams of 4096 frames, sizes drawn uniformly from four resolutions
# (seed 3), static blocks per stream (seed 3000 + i), 64 outputs at 32 + 64 k
BATCH_SIZES = ((250, 400), (500, 800), (720, 1280), (1000, 1000))


def batch_workload(n_streams: int = 16, T: int = 4096, seed: int = 3):
    """Shapes, seeds and output times of the batched workload."""
    rng_sizes = [BATCH_SIZES[rng_u64(seed, 6, i) % len(BATCH_SIZES)] for i in range(n_streams)]
    t_out = [32 + 64 * k for k in range(64) if 32 + 64 * k < T]
    return [dict(H=H, W=W, T=T, seed=3000 + i, t_out=t_out) for i, (H, W) in enumerate(rng_sizes)]
