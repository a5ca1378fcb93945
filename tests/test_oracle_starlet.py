"""Pins of the oracle's starlet transform (Sec. 3, Sec. 4.2)."""
import numpy as np
import pytest

import oracle as O
import synth as S


def _rms(a):
    return float(np.sqrt(np.mean(np.asarray(a) ** 2)))


def _smooth_141(a):
    s = np.array([1.0, 4.0, 1.0]) / 6.0
    return sum(s[dy + 1] * s[dx + 1] * np.roll(a, (dy, dx), axis=(0, 1))
               for dy in (-1, 0, 1) for dx in (-1, 0, 1))


@pytest.mark.parametrize("j", [1, 2, 3, 4])
def test_cascade_identity_samples_of_phi(j):
    # c_j of a delta, smoothed by [1,4,1]/6 per axis, equals the samples
    # phi(mx/2^j) phi(my/2^j) / 4^j (two-scale relation of the B3 spline)
    n, J = 64, 5
    planes = O.starlet_impulse_response(n, J)
    c = np.zeros((n, n))
    c[0, 0] = 1.0
    for i in range(j):
        c -= planes[i]
    got = _smooth_141(c)
    i = np.arange(n)
    m = np.where(i < n // 2, i, i - n).astype(float)
    p = O.phi_b3(m / 2 ** j) / 2 ** j
    assert np.max(np.abs(got - np.outer(p, p))) < 1e-15


@pytest.mark.parametrize("j", [1, 2, 3])
def test_kappa_form_separable_identity(j):
    # sum_d psi_theta(d) kappa(x + d) == ([1,4,1]/6 (x) [1,4,1]/6 * w_j)(x), theta = 2^j
    kappa = S.grf_kappa(64, 4)
    planes = O.starlet_forward(kappa, 4)
    theta = 2 ** j
    offs, w = O.separable_psi_taps(theta)
    M = np.zeros_like(kappa)
    for a, dy in enumerate(offs):
        for b, dx in enumerate(offs):
            if w[a, b] != 0.0:
                M += w[a, b] * np.roll(kappa, (-dy, -dx), axis=(0, 1))
    ref = _smooth_141(planes[j - 1])
    assert np.max(np.abs(M - ref)) < 1e-14 * _rms(kappa) * 1e2


@pytest.mark.parametrize("n,J", [(16, 3), (32, 4)])
def test_matches_bruteforce_convolution(n, J):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((n, n))
    planes = O.starlet_forward(a, J)
    imp = O.starlet_impulse_response(n, J)
    for p in range(J):
        ref = O.convolve_periodic(a, imp[p])
        assert np.max(np.abs(planes[p] - ref)) < 1e-13 * _rms(a)


@pytest.mark.parametrize("n,J", [(16, 2), (64, 6), (256, 5), (256, 8)])
def test_exact_reconstruction_and_zero_mean(n, J):
    kappa = S.grf_kappa(n, 21)
    planes = O.starlet_forward(kappa, J)
    assert planes.shape == (J, n, n)
    rec = O.starlet_reconstruct(planes)
    assert np.max(np.abs(rec - kappa)) < 1e-13 * _rms(kappa)
    for p in range(J - 1):
        assert abs(planes[p].mean()) < 1e-15 * _rms(kappa) * 10


def test_scale_limit():
    with pytest.raises(ValueError):
        O.starlet_forward(np.zeros((16, 16)), 5)
    with pytest.raises(ValueError):
        O.starlet_forward(np.zeros((16, 16)), 1)
