"""Peak counts on S/N planes (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper names peak counting on the S/N of the aperture mass as a
cosmological probe (Sec. 2.2; Sec. 4.3) without defining a peak.  Reading
used here: pixel x of a plane is a peak when

    value(x) > t   and   value(x) > value(y) for all 8 neighbours y,

neighbours taken periodically, comparisons strict, made in float64 on the
plane's exact values (a float32 plane is widened exactly).  Any comparison
with a NaN is false, so a NaN is never a peak and a pixel next to a NaN is
not one either.  Plateaus give no peak.

Pins (tests/test_oracle_peaks.py): hand-made planes (single delta, plateau,
a peak across the periodic wrap, NaN, a value exactly at t) and a pure-Python
loop count on random planes.
"""

import numpy as np


def count_peaks(plane, t):
    """Number of strict 8-neighbour local maxima above t on one plane."""
    p = np.asarray(plane).astype(np.float64)
    mask = p > float(t)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            mask &= p > np.roll(p, (dy, dx), axis=(0, 1))
    return int(np.count_nonzero(mask))


def count_peaks_planes(planes, t):
    """count_peaks for every plane of a stack; returns a list of ints."""
    return [count_peaks(pl, t) for pl in planes]
