"""Pins of the oracle's M_ap-map statistics (moments, peak histograms)."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle as O
import synth as S


def transfer(n, j):
    """Fourier transfer function of starlet smoothing to level j (product of
    the dilated B3 responses (6 + 8 cos w + 2 cos 2w)/16 along x and y)."""
    w = 2.0 * np.pi * np.fft.fftfreq(n)
    wy, wx = np.meshgrid(w, w, indexing="ij")
    h = np.ones((n, n))
    for i in range(j):
        s = float(1 << i)
        h *= ((6 + 8 * np.cos(s * wx) + 2 * np.cos(2 * s * wx)) / 16.0) * \
             ((6 + 8 * np.cos(s * wy) + 2 * np.cos(2 * s * wy)) / 16.0)
    return h


@pytest.mark.parametrize("n,J", [(32, 4), (64, 5), (128, 6)])
def test_plane_variance_equals_filtered_power(n, J):
    # discrete eq:varmap: the variance of w_j is the power of kappa through
    # the plane's transfer function (Parseval), computed here in Fourier space
    kappa = S.grf_kappa(n, 5 + J)
    planes = O.starlet_forward(kappa, J)
    kh = np.fft.fft2(kappa)
    for j in range(1, J):
        t = transfer(n, j - 1) - transfer(n, j)
        m2_fourier = float(np.sum(np.abs(kh * t) ** 2)) / n ** 4
        mu, m2, _, _ = O.plane_moments(planes[j - 1])
        assert abs(mu) < 1e-16
        assert m2 == pytest.approx(m2_fourier, rel=1e-11)
    # the smooth plane keeps the mean
    t = transfer(n, J - 1)
    mu, m2, _, _ = O.plane_moments(planes[J - 1])
    assert mu == pytest.approx(kappa.mean(), abs=1e-17)
    power = float(np.sum(np.abs(kh * t) ** 2) - abs(kh[0, 0]) ** 2) / n ** 4
    assert m2 == pytest.approx(power, rel=1e-11)


def test_moments_closed_forms():
    n, a = 16, 0.7
    iy, ix = np.indices((n, n))
    board = a * (-1.0) ** (ix + iy)
    assert O.plane_moments(board) == pytest.approx([0.0, a * a, 0.0, a ** 4], abs=1e-15)
    delta = np.zeros((n, n))
    delta[3, 5] = 1.0
    mu = 1.0 / (n * n)
    want = [mu, mu * (1 - mu), mu * (1 - mu) * (1 - 2 * mu), mu * (1 - mu) * (1 - 3 * mu + 3 * mu * mu)]
    assert O.plane_moments(delta) == pytest.approx(want, rel=1e-12)
    assert O.plane_moments(np.full((n, n), 2.5)) == pytest.approx([2.5, 0, 0, 0], abs=1e-15)


def test_moments_match_scipy():
    rng = np.random.default_rng(4)
    x = rng.gamma(2.0, 1.5, size=(48, 48))    # skewed, heavy-tailed
    mu, m2, m3, m4 = O.plane_moments(x)
    f = x.ravel()
    assert m2 == pytest.approx(scipy.stats.moment(f, 2), rel=1e-12)
    assert m3 == pytest.approx(scipy.stats.moment(f, 3), rel=1e-12)
    assert m4 == pytest.approx(scipy.stats.moment(f, 4), rel=1e-12)
    assert m3 / m2 ** 1.5 == pytest.approx(scipy.stats.skew(f), rel=1e-12)
    assert m4 / m2 ** 2 - 3 == pytest.approx(scipy.stats.kurtosis(f), rel=1e-12)


def brute_histogram(plane, lo, hi, nbins, sign):
    n0, n1 = plane.shape
    out = [0] * nbins
    width = (hi - lo) / nbins
    for y in range(n0):
        for x in range(n1):
            v = sign * float(plane[y, x])
            ok = True
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dy or dx:
                        if not v > sign * float(plane[(y + dy) % n0, (x + dx) % n1]):
                            ok = False
            if ok:
                b = math.floor((v - lo) / width)
                if 0 <= b < nbins:
                    out[b] += 1
    return out


@pytest.mark.parametrize("sign", [1, -1])
def test_histogram_matches_bruteforce(sign):
    rng = np.random.default_rng(8 + sign)
    plane = rng.integers(-6, 7, size=(14, 14)).astype(np.float64) * 0.5   # ties and plateaus
    plane += rng.standard_normal((14, 14)) * (rng.random((14, 14)) < 0.5)
    got = O.peak_histogram(plane, -2.0, 3.0, 7, sign)
    assert list(got) == brute_histogram(plane, -2.0, 3.0, 7, sign)


def test_histogram_sums_to_peak_counts_and_troughs_are_negated_peaks():
    rng = np.random.default_rng(12)
    plane = rng.standard_normal((40, 40))
    for t in (-0.5, 0.0, 1.3):
        assert int(O.peak_histogram(plane, t, 1e30, 1).sum()) == O.count_peaks(plane, t)
    a = O.peak_histogram(plane, -1.0, 2.0, 12, -1)
    b = O.peak_histogram(-plane, -1.0, 2.0, 12, 1)
    assert np.array_equal(a, b)


def test_histogram_hand_made():
    p = np.zeros((10, 10))
    p[4, 4] = 5.0            # the only strict maximum; the zero plateau gives none
    p[7, 1] = -5.0           # the only strict minimum
    p[0, 9] = np.nan         # never a peak, and blocks its neighbours
    h = O.peak_histogram(p, 0.0, 10.0, 10, 1)
    assert list(h) == [0, 0, 0, 0, 0, 1, 0, 0, 0, 0]
    h = O.peak_histogram(p, 0.0, 10.0, 10, -1)
    assert list(h) == [0, 0, 0, 0, 0, 1, 0, 0, 0, 0]
    # heights exactly on a bin edge fall in the upper bin; hi is excluded
    assert list(O.peak_histogram(p, 4.0, 6.0, 2, 1)) == [0, 1]
    assert list(O.peak_histogram(p, 3.0, 5.0, 2, 1)) == [0, 0]
