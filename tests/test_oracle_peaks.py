"""Pins of the oracle's peak counts (Sec. 2.2, Sec. 4.3)."""
import numpy as np
import pytest

import oracle as O


def _brute(plane, t):
    n0, n1 = plane.shape
    c = 0
    for y in range(n0):
        for x in range(n1):
            v = float(plane[y, x])
            if not v > t:
                continue
            ok = True
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dy or dx) and not v > float(plane[(y + dy) % n0, (x + dx) % n1]):
                        ok = False
            c += ok
    return c


def test_single_delta_and_threshold():
    p = np.zeros((16, 16))
    p[5, 7] = 4.0
    assert O.count_peaks(p, 3.0) == 1
    assert O.count_peaks(p, 4.0) == 0  # strictly above t
    p[5, 7] = 3.0
    assert O.count_peaks(p, 3.0) == 0


def test_plateau_is_not_a_peak():
    p = np.zeros((16, 16))
    p[4, 4] = p[4, 5] = 5.0
    assert O.count_peaks(p, 3.0) == 0


def test_peak_across_periodic_wrap():
    p = np.zeros((16, 16))
    p[0, 0] = 5.0
    p[15, 15] = 4.0  # diagonal neighbour across both edges
    assert O.count_peaks(p, 3.0) == 1
    p[15, 15] = 6.0
    assert O.count_peaks(p, 3.0) == 1
    p[0, 0] = 6.0
    assert O.count_peaks(p, 3.0) == 0


def test_nan_is_never_a_peak():
    p = np.zeros((16, 16), dtype=np.float32)
    p[3, 3] = np.nan
    p[8, 8] = 5.0
    p[8, 9] = np.nan  # neighbour of a candidate
    p[12, 2] = 7.0
    assert O.count_peaks(p, 3.0) == 1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_planes_match_bruteforce(seed):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal((48, 48)) * 2.0).astype(np.float32)
    p[rng.random((48, 48)) < 0.05] = 3.5  # ties at a value above t
    assert O.count_peaks(p, 3.0) == _brute(p, 3.0)
    assert O.count_peaks(p, 1.0) == _brute(p, 1.0)
