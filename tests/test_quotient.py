"""The Eq. 6 quotient of the reconstruction kernels, replayed on the CPU.

The kernels form theta * N / D in double precision from the hardware
reciprocal, two Newton-Raphson refinements and one Markstein correction,
without the exponent scaling and special-case steps of a general IEEE
division (those only act near the exponent limits; here 2^-149 <=
theta * N < 2^160 and 1 <= D < 2^31).  tests/quotient_replay.c replays that
fma sequence from a reciprocal perturbed far beyond any hardware error in
both directions and requires the correctly rounded double quotient: for
every D below 2^20 against a grid of numerators over the whole range, and
on random (numerator, D) pairs up to 2^31.  A replay with a refinement
taken out must fail (the check is not vacuous).
"""
import ctypes
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

# relative errors of the starting reciprocal, both directions
DELTAS = [0.0] + [s * 2.0 ** -k for k in (52, 40, 23, 14) for s in (1, -1)]


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp(prefix="quot_")
    so = os.path.join(d, "quotient_replay.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-shared",
                    "-fPIC", os.path.join(HERE, "quotient_replay.c"), "-o", so, "-lm"],
                   check=True)
    lib = ctypes.CDLL(so)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.check_range.restype = ctypes.c_int64
    lib.check_range.argtypes = [ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_int32, dp,
                                ctypes.c_int32, ctypes.c_int32, dp]
    lib.check_pairs.restype = ctypes.c_int64
    lib.check_pairs.argtypes = [dp, dp, ctypes.c_int64, dp, ctypes.c_int32, ctypes.c_int32, dp]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _numerators(rng):
    """theta * N rounded to double, theta a float from the smallest
    subnormal to the largest finite one, N from 1 to 2^31 - 1."""
    thetas = [np.float32(2.0 ** -149), np.float32(2.0 ** -126), np.float32(1.0),
              np.float32(255.0), np.finfo(np.float32).max]
    thetas += [np.float32(rng.uniform(1, 2) * 2.0 ** e) for e in (-140, -60, -3, 30, 126)]
    ns = [1, 3, 7, 1000, (1 << 20) - 1, (1 << 31) - 1]
    xs = sorted({float(np.float64(t) * n) for t in thetas for n in ns})
    return np.array(xs, dtype=np.float64)


def test_every_small_denominator(lib):
    rng = np.random.default_rng(0)
    xs = _numerators(rng)
    deltas = np.array(DELTAS)
    # d ranges in parallel threads (ctypes releases the interpreter lock)
    cuts = np.linspace(1, 1 << 20, 9).astype(np.int64)
    bads = [np.zeros(3) for _ in range(8)]

    def part(i):
        return lib.check_range(int(cuts[i]), int(cuts[i + 1]), _ptr(xs), len(xs), _ptr(deltas),
                               len(deltas), 2, _ptr(bads[i]))

    with ThreadPoolExecutor(8) as ex:
        fails = list(ex.map(part, range(8)))
    for f, bad in zip(fails, bads):
        assert f == 0, ("x=%r d=%r delta=%r" % tuple(bad), f)


def test_random_pairs_whole_range(lib):
    rng = np.random.default_rng(1)
    n = 200_000
    theta = (rng.uniform(1, 2, n) * 2.0 ** rng.integers(-149, 128, n)).astype(np.float32)
    N = rng.integers(1, 1 << 31, n)
    xs = theta.astype(np.float64) * N.astype(np.float64)
    ds = rng.integers(1, 1 << 31, n).astype(np.float64)
    deltas = np.array(DELTAS)
    bad = np.zeros(3)
    fails = lib.check_pairs(_ptr(xs), _ptr(ds), n, _ptr(deltas), len(deltas), 2, _ptr(bad))
    assert fails == 0, ("x=%r d=%r delta=%r" % tuple(bad), fails)


def test_one_refinement_is_caught(lib):
    """With one refinement a reciprocal off by 2^-14 is not accurate
    enough; the check must see it."""
    rng = np.random.default_rng(2)
    xs = _numerators(rng)
    deltas = np.array([2.0 ** -14, -2.0 ** -14])
    bad = np.zeros(3)
    assert lib.check_range(1, 1 << 12, _ptr(xs), len(xs), _ptr(deltas), len(deltas), 1,
                           _ptr(bad)) > 0
