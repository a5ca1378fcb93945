"""Pins of the oracle's noise maps and S/N (Sec. 1, Sec. 5.1)."""
import numpy as np
import pytest

import oracle as O
import synth as S


def test_zero_angles_give_zero_sigma():
    _, g1, g2 = S.shear_map(32, 5, 6)
    sig = O.noise_sigma(g1, g2, 4, 5, 0, uniforms=lambda n, seed, r: np.zeros((n, n)))
    assert np.all(sig == 0.0)
    snr = O.snr_planes(O.starlet_forward(O.ks_invert(g1, g2)[0], 4), sig)
    assert np.all(snr == 0.0)


def test_alternating_sign_gives_closed_form_variance():
    # beta = 0, pi, 0, pi, ... : w_r = +-w, sample mean 0 (R even), so
    # sigma^2 = R w^2 / (R - 1)
    _, g1, g2 = S.shear_map(32, 5, 6)
    R, J = 6, 4
    sig = O.noise_sigma(g1, g2, J, R, 0,
                        uniforms=lambda n, seed, r: np.full((n, n), 0.5 * (r % 2)))
    w = O.starlet_forward(O.ks_invert(g1, g2)[0], J)[:J - 1]
    ref = np.sqrt(R / (R - 1.0)) * np.abs(w)
    assert np.max(np.abs(sig - ref)) < 1e-12 * np.max(np.abs(w))


def test_expected_variance_closed_form():
    # By linearity w_j(x) = sum_y A_j(x-y) g1'(y) + B_j(x-y) g2'(y); a uniform
    # phase gives Var = 1/2 sum_y (A_j^2 + B_j^2)(x-y) |gamma(y)|^2.
    n, J, R = 32, 4, 400
    rng = np.random.default_rng(12)
    g1 = rng.standard_normal((n, n)) * np.linspace(0.2, 1.5, n)[None, :]
    g2 = rng.standard_normal((n, n))
    d = np.zeros((n, n))
    d[0, 0] = 1.0
    A = O.starlet_forward(O.ks_invert(d, 0 * d)[0], J)[:J - 1]
    B = O.starlet_forward(O.ks_invert(0 * d, d)[0], J)[:J - 1]
    mod2 = g1 ** 2 + g2 ** 2
    sig = O.noise_sigma(g1, g2, J, R, 77)
    for j in range(J - 1):
        kern = 0.5 * (A[j] ** 2 + B[j] ** 2)
        expect = np.fft.ifft2(np.fft.fft2(kern) * np.fft.fft2(mod2)).real
        ratio = sig[j] ** 2 / expect
        # pixel-mean of a chi-square(R-1)/(R-1) ratio; pixels are correlated,
        # so allow 4x the independent-pixel scatter plus a small floor
        assert abs(ratio.mean() - 1.0) < 4 * np.sqrt(2.0 / (R - 1)) / 4 + 0.01, (j, ratio.mean())
        assert ratio.std() == pytest.approx(np.sqrt(2.0 / (R - 1)), rel=0.35)


def test_snr_definition():
    w = np.array([[[1.0, -2.0], [3.0, 0.5]]])
    s = np.array([[[2.0, 0.0], [1.5, 0.25]]])
    assert np.array_equal(O.snr_planes(w, s), np.array([[[0.5, 0.0], [2.0, 2.0]]]))


def test_rotation_is_a_phase():
    rng = np.random.default_rng(1)
    g1, g2 = rng.standard_normal((2, 8, 8))
    u = rng.random((8, 8))
    a1, a2 = O.rotate_shear(g1, g2, u)
    z = (g1 + 1j * g2) * np.exp(2j * np.pi * u)
    assert np.max(np.abs(a1 - z.real)) < 1e-15 and np.max(np.abs(a2 - z.imag)) < 1e-15


def test_merge_moments_matches_pooled_variance():
    # Chan-Golub-LeVeque pairwise update vs numpy's mean and variance of the
    # pooled samples; unequal parts with far-apart means exercise the
    # between-part term d^2 na nb / n
    rng = np.random.default_rng(5)
    parts = [rng.standard_normal((k, 3, 4)) * s + m
             for k, s, m in ((3, 1.0, 0.0), (1, 0.5, 40.0), (7, 2.0, -3.0), (2, 0.1, 9.0))]
    acc = (0, 0.0, 0.0)
    for p in parts:
        acc = O.merge_moments(acc, (p.shape[0], p.mean(axis=0), ((p - p.mean(axis=0)) ** 2).sum(axis=0)))
    pooled = np.concatenate(parts)
    assert acc[0] == pooled.shape[0]
    assert np.allclose(acc[1], pooled.mean(axis=0), rtol=0, atol=1e-13 * np.abs(pooled).max())
    ref = np.var(pooled, axis=0) * pooled.shape[0]
    assert np.allclose(acc[2], ref, rtol=1e-12, atol=0)
    # merging with an empty part is the identity
    assert O.merge_moments(acc, (0, 0.0, 0.0)) is acc


def test_noise_moments_split_runs_merge_to_the_single_run():
    _, g1, g2 = S.shear_map(32, 7, 8)
    J, R, seed = 4, 9, 31
    whole = O.noise_moments(g1, g2, J, seed, 0, R)
    acc = (0, 0.0, 0.0)
    for a, b in ((0, 2), (2, 3), (3, 9)):
        acc = O.merge_moments(acc, O.noise_moments(g1, g2, J, seed, a, b))
    assert acc[0] == whole[0] == R
    scale = np.abs(whole[1]).max()
    assert np.max(np.abs(acc[1] - whole[1])) <= 1e-14 * scale
    assert np.max(np.abs(acc[2] - whole[2])) <= 1e-13 * np.abs(whole[2]).max()
    sig = O.noise_sigma(g1, g2, J, R, seed)
    assert np.array_equal(O.sigma_from_moments(*whole[::2]), sig)


def test_pooled_oracle_helper_equals_noise_sigma():
    # the process-pool helper the large GPU parity tests use
    import oracle_pool
    _, g1, g2 = S.shear_map(32, 9, 10)
    J, R, seed = 4, 7, 12
    ref = O.noise_sigma(g1, g2, J, R, seed)
    got = oracle_pool.noise_sigma_pool(g1, g2, J, R, seed, workers=3)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(ref)
