"""Pins of the oracle's Kaiser-Squires inversion (Sec. 1, Sec. 4.5)."""
import numpy as np
import pytest

import oracle as O
import synth as S


def _rms(a):
    return float(np.sqrt(np.mean(np.asarray(a) ** 2)))


@pytest.mark.parametrize("n", [8, 16])
def test_ks_matches_bruteforce_dft(n):
    rng = np.random.default_rng(100 + n)
    g1, g2 = rng.standard_normal((2, n, n))
    G = O.dft2_brute(g1 + 1j * g2)
    k = O.dft2_brute(np.conj(O.ks_kernel(n)) * G, inverse=True)
    kE, kB = O.ks_invert(g1, g2)
    assert np.max(np.abs(kE - k.real)) < 1e-12
    assert np.max(np.abs(kB - k.imag)) < 1e-12


@pytest.mark.parametrize("n,seed", [(32, 3), (256, 1)])
def test_ks_recovers_emode_kappa(n, seed):
    kappa, g1, g2 = S.shear_map(n, seed, None)
    kE, kB = O.ks_invert(g1, g2)
    assert np.max(np.abs(kE - kappa)) < 1e-12 * _rms(kappa)
    assert np.max(np.abs(kB)) < 1e-12 * _rms(kappa)


def test_pure_bmode_gives_zero_kappa_e():
    kb = S.grf_kappa(64, 9)
    g1, g2 = S.bmode_shear(kb)
    kE, kB = O.ks_invert(g1, g2)
    assert np.max(np.abs(kE)) < 1e-12 * _rms(kb)
    assert np.max(np.abs(kB - kb)) < 1e-12 * _rms(kb)


def test_nyquist_rule_makes_real_form_real_and_equal():
    # kappa_E = F^-1[D1 F(g1) + D2 F(g2)] with D1 = (k1^2-k2^2)/k^2 and
    # D2 = 2 k1 k2/k^2 must be a real field for real shears; on a Nyquist line
    # the mirror of a wavenumber aliases onto itself while D2 changes sign, so
    # D2 has to vanish there.  With that, the complex form agrees.
    n = 64
    rng = np.random.default_rng(5)
    g1, g2 = rng.standard_normal((2, n, n))
    i = np.arange(n)
    m = np.where(i < n // 2, i, i - n)
    my, mx = np.meshgrid(m, m, indexing="ij")
    ky, kx = 2 * np.pi * my / n, 2 * np.pi * mx / n
    ksq = kx ** 2 + ky ** 2
    ksq[0, 0] = 1.0
    D1 = (kx ** 2 - ky ** 2) / ksq
    D2 = 2 * kx * ky / ksq
    D1[0, 0] = D2[0, 0] = 0.0
    raw = np.fft.ifft2(D1 * np.fft.fft2(g1) + D2 * np.fft.fft2(g2))
    assert np.max(np.abs(raw.imag)) > 0.05  # without the rule: not real
    D2[(mx == -n // 2) | (my == -n // 2)] = 0.0
    fixed = np.fft.ifft2(D1 * np.fft.fft2(g1) + D2 * np.fft.fft2(g2))
    assert np.max(np.abs(fixed.imag)) < 1e-13
    kE, _ = O.ks_invert(g1, g2)
    assert np.max(np.abs(kE - fixed.real)) < 1e-13


def test_diagonal_reflection_symmetry():
    # reflecting across the diagonal x <-> y maps (g1, g2) -> (-g1^T, g2^T);
    # kappa_E is a scalar (transposes), kappa_B a pseudo-scalar (changes sign)
    rng = np.random.default_rng(7)
    g1, g2 = rng.standard_normal((2, 32, 32))
    kE, kB = O.ks_invert(g1, g2)
    rE, rB = O.ks_invert(-g1.T, g2.T)
    assert np.max(np.abs(rE - kE.T)) < 1e-13
    assert np.max(np.abs(rB + kB.T)) < 1e-13


def test_kappa_e_has_zero_mean():
    rng = np.random.default_rng(8)
    g1, g2 = rng.standard_normal((2, 32, 32)) + 0.3
    kE, kB = O.ks_invert(g1, g2)
    assert abs(kE.mean()) < 1e-15 and abs(kB.mean()) < 1e-15
