"""Declarative definitions used to pin the oracle (pure Python, no shared code).

These restate what the paper's segmentation must produce as properties of
the result rather than as the greedy procedure the oracle runs:

* zero-order stability (Def. 2): a sequence holds one value, or two values
  that differ by exactly 1 -- equivalently max - min <= 1;
* FSR (Sec. III-B): a contiguous partition of S1 whose parts are zero-order
  stable and where no part (but the last) stays stable when the next interval
  is appended (the stability module of Sec. III-C closes a segment exactly
  when the new element violates);
* SSR (Sec. III-B, Fig. 1 caption): inside each FSR segment, a contiguous
  partition whose parts have a zero-order stable S2 for every interval value
  (S2 of a value = gaps between its consecutive occurrences, Eq. 5), again
  maximal;
* third order (the n-order rule of Sec. III-A once more): inside each SSR
  piece, parts whose S3 streams (gaps between consecutive positions of each
  S2 value inside S2) are zero-order stable, again maximal.

Both properties are prefix-closed, so at most one partition satisfies them;
``enumerate_partitions`` checks that claim by brute force on small inputs.
"""
from __future__ import annotations

import itertools


def zero_order_stable(seq) -> bool:
    seq = list(seq)
    return len(seq) == 0 or max(seq) - min(seq) <= 1


def s2_streams(part) -> dict:
    """S2 per interval value of a piece of S1: value -> list of gaps between
    consecutive occurrences (index differences)."""
    pos = {}
    for i, v in enumerate(part):
        pos.setdefault(v, []).append(i)
    return {v: [b - a for a, b in zip(p, p[1:])] for v, p in pos.items()}


def s2_stable(part) -> bool:
    return all(zero_order_stable(g) for g in s2_streams(part).values())


def parts_of(x, starts):
    bounds = list(starts) + [len(x)]
    return [x[bounds[i]:bounds[i + 1]] for i in range(len(starts))]


def is_fsr_partition(x, starts) -> bool:
    """True iff ``starts`` (segment starts) is the FSR partition of ``x``."""
    if len(x) == 0:
        return list(starts) == []
    if not starts or starts[0] != 0 or list(starts) != sorted(set(starts)):
        return False
    if starts[-1] >= len(x):
        return False
    bounds = list(starts) + [len(x)]
    for a, b in zip(bounds, bounds[1:]):
        if not zero_order_stable(x[a:b]):
            return False
        if b < len(x) and zero_order_stable(x[a:b + 1]):
            return False
    return True


def is_ssr_partition(x, starts, fsr_starts) -> bool:
    """True iff ``starts`` refines the FSR partition and, inside each FSR
    segment, is the maximal S2-stable partition."""
    if len(x) == 0:
        return list(starts) == []
    if not set(fsr_starts) <= set(starts):
        return False
    if not starts or starts[0] != 0 or list(starts) != sorted(set(starts)):
        return False
    fb = list(fsr_starts) + [len(x)]
    sb = list(starts) + [len(x)]
    for a, b in zip(sb, sb[1:]):
        # the FSR segment holding this piece
        seg_end = min(e for e in fb if e > a)
        if b > seg_end:
            return False
        if not (zero_order_stable(x[a:b]) and s2_stable(x[a:b])):
            return False
        if b < seg_end and s2_stable(x[a:b + 1]):
            return False
    return True


def s3_stable(part) -> bool:
    """Third order (the n-order rule of Sec. III-A applied to S2): for every
    interval value v and every value g of S2(v), the gaps between
    consecutive positions of g in S2(v) are zero-order stable."""
    for gaps in s2_streams(part).values():
        for s3 in s2_streams(gaps).values():
            if not zero_order_stable(s3):
                return False
    return True


def is_tsr_partition(x, starts, ssr_starts) -> bool:
    """True iff ``starts`` refines the SSR partition and, inside each SSR
    piece, is the maximal partition into third-order stable parts."""
    if len(x) == 0:
        return list(starts) == []
    if not set(ssr_starts) <= set(starts):
        return False
    if not starts or starts[0] != 0 or list(starts) != sorted(set(starts)):
        return False
    pb = list(ssr_starts) + [len(x)]
    sb = list(starts) + [len(x)]
    for a, b in zip(sb, sb[1:]):
        piece_end = min(e for e in pb if e > a)
        if b > piece_end:
            return False
        part = x[a:b]
        if not (zero_order_stable(part) and s2_stable(part) and s3_stable(part)):
            return False
        if b < piece_end and s3_stable(x[a:b + 1]):
            return False
    return True


def enumerate_partitions(x, pred):
    """All segment-start lists of ``x`` accepted by ``pred`` (brute force)."""
    n = len(x)
    if n == 0:
        return [[]] if pred([]) else []
    found = []
    for cuts in itertools.product((0, 1), repeat=n - 1):
        starts = [0] + [i + 1 for i, c in enumerate(cuts) if c]
        if pred(starts):
            found.append(starts)
    return found


def intervals_of(spike_frames):
    return [b - a for a, b in zip(spike_frames, spike_frames[1:])]


def interval_in_progress(spike_frames, t):
    """1-based index m(t) of the interval covering frame t (clamped)."""
    K = len(spike_frames)
    c = sum(1 for s in spike_frames if s < t)
    return min(max(c, 1), K - 1)
