"""Synthetic spike trains for the parity tests: per pixel, random regimes of
inter-spike intervals (input generation only, no reconstruction arithmetic)."""
import numpy as np

import spkgen


def regime_stream(rng, T, W):
    """Pixels whose intervals follow random regimes: a base interval a (1 to
    40) held for a random stretch, drawn from {a}, {a, a + 1}, {a - 1, a,
    a + 1} or a few far values.  Windows widen and narrow across chunk
    boundaries, and some segments outlast several tiles."""
    bits = np.zeros((T, W), dtype=np.uint8)
    for p in range(W):
        t = int(rng.integers(0, 40))
        while t < T:
            a = int(rng.integers(1, 41))
            kind = int(rng.integers(0, 4))
            end = t + int(rng.integers(40, 900))
            while t < min(end, T):
                bits[t, p] = 1
                if kind == 0:
                    d = a
                elif kind == 1:
                    d = a + int(rng.integers(0, 2))
                elif kind == 2:
                    d = max(1, a + int(rng.integers(-1, 2)))
                else:
                    d = int(rng.choice([a, a + 3, max(1, a - 2), 2 * a]))
                t += d
    return spkgen.pack(bits)
