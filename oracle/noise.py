"""Noise maps from randomised shears, and S/N planes (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Sec. 1: the noise of an aperture-mass reconstruction is assessed by
randomising the input data many times and taking the variance of the
resulting reconstructions, sigma^2_Map; the signal-to-noise is S = M_ap /
sigma_Map.  Sec. 4.3 adds that the noise map is made in the same manner as
the signal.  Readings used here:

  * randomisation: every pixel's shear is rotated by an independent uniform
    angle, gamma' = gamma * exp(i beta), beta = 2 pi u, with u from
    ``oracle.rng`` (seed, realisation r);
  * each realisation goes through the same KS inversion and starlet transform
    as the signal; only the detail planes w_1 .. w_{J-1} are used;
  * sigma_j(x) is the unbiased sample standard deviation over the R
    realisations (divisor R - 1), per pixel and per scale, accumulated here
    with Welford's update; statistics of disjoint runs of realisations
    combine by the pairwise update of Chan, Golub & LeVeque (1979);
  * snr_j = w_j / sigma_j, and 0 where sigma_j = 0.

Pins (tests/test_oracle_noise.py): the expected variance has a closed form by
linearity, E[sigma_j^2(x)] = 1/2 sum_y |K_j(x - y)|^2 |gamma(y)|^2 with K_j
the complex impulse response of KS followed by scale j, checked on the mean
over pixels within its chi-square scatter; degenerate angle streams
(beta = 0 gives sigma = 0; beta alternating 0, pi gives sigma^2 = R/(R-1) w^2).
The pairwise merge is pinned against numpy's variance of the pooled samples.
"""

import numpy as np

from .ks import ks_invert
from .starlet import starlet_forward
from .rng import phase_uniforms


def rotate_shear(g1, g2, u):
    """gamma * exp(2 pi i u), per pixel."""
    beta = 2.0 * np.pi * np.asarray(u, dtype=np.float64)
    c, s = np.cos(beta), np.sin(beta)
    return g1 * c - g2 * s, g1 * s + g2 * c


def noise_moments(g1, g2, J, seed, r_begin, r_end, uniforms=None):
    """Running statistics of the detail planes over realisations
    r_begin .. r_end - 1: ``(count, mean, m2)``, with mean and m2 of shape
    (J-1, N, N) and m2 the sum of squared deviations from the mean, built by
    Welford's update one realisation at a time.

    ``uniforms(n, seed, r)`` overrides the angle source (tests only).
    """
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    n = g1.shape[0]
    draw = phase_uniforms if uniforms is None else uniforms
    mean = np.zeros((J - 1, n, n))
    m2 = np.zeros((J - 1, n, n))
    count = 0
    for r in range(r_begin, r_end):
        a1, a2 = rotate_shear(g1, g2, draw(n, seed, r))
        kE, _ = ks_invert(a1, a2)
        w = starlet_forward(kE, J)[:J - 1]
        count += 1
        delta = w - mean
        mean += delta / count
        m2 += delta * (w - mean)
    return count, mean, m2


def merge_moments(a, b):
    """Statistics of the union of two disjoint sample sets from those of the
    parts (the pairwise update of Chan, Golub & LeVeque, 1979):
    n = na + nb, mean = ma + d nb / n, m2 = m2a + m2b + d^2 na nb / n with
    d = mb - ma.  Each argument is ``(count, mean, m2)``."""
    na, ma, qa = a
    nb, mb, qb = b
    if nb == 0:
        return a
    if na == 0:
        return b
    n = na + nb
    d = mb - ma
    return n, ma + d * (nb / n), qa + qb + d * d * (na * nb / n)


def noise_sigma(g1, g2, J, n_real, seed, uniforms=None):
    """Per-pixel, per-scale noise sigma_j (shape (J-1, N, N)).

    ``uniforms(n, seed, r)`` overrides the angle source (tests only).
    """
    if n_real < 2:
        raise ValueError("need at least two realisations")
    count, _, m2 = noise_moments(g1, g2, J, seed, 0, n_real, uniforms)
    return sigma_from_moments(count, m2)


def sigma_from_moments(count, m2):
    """Unbiased sample standard deviation sqrt(m2 / (count - 1))."""
    if count < 2:
        raise ValueError("need at least two realisations")
    return np.sqrt(m2 / (count - 1))


def snr_planes(planes_signal, sigma):
    """S = w_j / sigma_j per pixel for the J-1 detail planes (0 where sigma = 0)."""
    w = np.asarray(planes_signal, dtype=np.float64)[: sigma.shape[0]]
    out = np.zeros_like(w)
    nz = sigma > 0
    out[nz] = w[nz] / sigma[nz]
    return out
