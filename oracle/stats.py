"""Statistics of aperture-mass maps beyond the maps themselves (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2.2 of the paper names the statistics drawn from M_ap maps for
cosmology: the variance <M_ap^2>(theta) (eq:varmap relates it to the power
spectrum through the filter's power spectrum), the third moment (skewness)
and the kurtosis, and peak counts.  With the starlet, plane w_j is the M_ap
map at theta = 2^j, so these are moments and peak statistics of the planes.

* ``plane_moments``: mean and the central moments m2, m3, m4 of a plane,
  m_k = (1/N^2) sum_x (x - mean)^k (population moments, float64); the
  variance is m2, the normalised skewness m3 / m2^1.5 and the excess
  kurtosis m4 / m2^2 - 3.
* ``peak_histogram``: heights of the strict 8-neighbour local maxima of
  s * value (s = +1 peaks, s = -1 troughs; periodic neighbours, strict
  comparisons in float64, NaN never a peak), binned into ``nbins`` equal bins
  over [lo, hi): bin = floor((s * value - lo) / ((hi - lo) / nbins)) in
  float64, counted when 0 <= bin < nbins.  Counts above several thresholds
  follow by summing bins.

Pins (tests/test_oracle_stats.py): the variance of each starlet plane equals
the sum over wavenumbers of |kappa_hat|^2 times the squared transfer
function of that plane, built from the B3 taps in Fourier space (the
discrete form of eq:varmap; an independent route through the FFT);
moments of a checkerboard, a single delta and a constant plane in closed
form; agreement with scipy.stats for random planes; the histogram against a
pure-Python loop on random planes, its sum against count_peaks, troughs as
peaks of the negated plane, and hand-made planes.
"""

import numpy as np


def plane_moments(plane):
    """[mean, m2, m3, m4] of one plane (float64 population moments)."""
    p = np.asarray(plane, dtype=np.float64)
    mu = float(p.mean())
    d = p - mu
    return [mu, float(np.mean(d ** 2)), float(np.mean(d ** 3)), float(np.mean(d ** 4))]


def plane_moments_stack(planes):
    """plane_moments of every plane of a stack, as an (nplanes, 4) array."""
    return np.array([plane_moments(pl) for pl in planes])


def _local_max(p):
    mask = np.ones(p.shape, dtype=bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            mask &= p > np.roll(p, (dy, dx), axis=(0, 1))
    return mask


def peak_histogram(plane, lo, hi, nbins, sign=1):
    """Binned heights of the strict local maxima of sign * plane."""
    if nbins < 1 or not hi > lo or sign not in (1, -1):
        raise ValueError("need nbins >= 1, hi > lo and sign = +-1")
    p = float(sign) * np.asarray(plane).astype(np.float64)
    h = p[_local_max(p)]
    width = (float(hi) - float(lo)) / float(nbins)
    b = np.floor((h - float(lo)) / width)
    b = b[(b >= 0) & (b < nbins)].astype(np.int64)
    return np.bincount(b, minlength=nbins).astype(np.int64)


def peak_histogram_planes(planes, lo, hi, nbins, sign=1):
    """peak_histogram of every plane, as an (nplanes, nbins) int64 array."""
    return np.array([peak_histogram(pl, lo, hi, nbins, sign) for pl in planes], dtype=np.int64)
