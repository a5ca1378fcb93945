"""Kaiser-Squires inversion: shear map -> convergence map (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper converts the pixelised shear map into a convergence map "in Fourier
space" (Sec. 1; Sec. 4.5) without printing the formula.  This module states
the standard Kaiser-Squires relation on a periodic N x N grid:

  * wavenumbers: m(i) = i for i < N/2, else i - N (so the Nyquist index maps
    to -N/2); k = 2 pi m / N; k1 along x (columns), k2 along y (rows);
  * forward DFT with exp(-2 pi i m.x/N), inverse with exp(+...) and 1/N^2;
  * D(k) = [(k1^2 - k2^2) + 2 i nu k1 k2] / (k1^2 + k2^2), D(0) = 0, where
    nu = 0 on the Nyquist row and column (m1 = -N/2 or m2 = -N/2) and 1
    elsewhere.  The cross term is odd in each wavenumber, so it has no
    well-defined value on a Nyquist line; zeroing it there makes the complex
    single-transform form agree with the two-real-transform form;
  * kappa = F^-1[ conj(D) F(gamma1 + i gamma2) ], kappa_E = Re, kappa_B = Im.

Pins (tests/test_oracle_ks.py): an O(N^4) brute-force DFT on 8^2/16^2 maps;
recovery of kappa from E-mode shears synthesised through the lensing
potential (independent arithmetic, ``synth``); a pure B-mode input gives
kappa_E = 0; the two-real-transform form agrees with the complex form; the
diagonal-reflection symmetry gamma1 -> -gamma1 transposes kappa.
"""

import numpy as np


def wavenumbers(n):
    """Signed integer frequency index m(i) (Nyquist -> -n/2) as float64."""
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n).astype(np.float64)


def ks_kernel(n):
    """The complex KS kernel D(k) on the n x n frequency grid, indexed [m2, m1]."""
    m = wavenumbers(n)
    k = 2.0 * np.pi * m / n
    k2, k1 = np.meshgrid(k, k, indexing="ij")  # axis 0 = y (k2), axis 1 = x (k1)
    nyq = -(n // 2)
    m2, m1 = np.meshgrid(m, m, indexing="ij")
    nu = np.where((m1 == nyq) | (m2 == nyq), 0.0, 1.0)
    ksq = k1 * k1 + k2 * k2
    D = np.zeros((n, n), dtype=np.complex128)
    nz = ksq > 0
    D[nz] = ((k1 * k1 - k2 * k2) + 2j * nu * k1 * k2)[nz] / ksq[nz]
    return D


def ks_invert(g1, g2):
    """Kaiser-Squires inversion of a periodic shear map; returns (kappa_E, kappa_B)."""
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    n = g1.shape[0]
    assert g1.shape == (n, n) and g2.shape == (n, n)
    G = np.fft.fft2(g1 + 1j * g2)
    K = np.conj(ks_kernel(n)) * G
    kappa = np.fft.ifft2(K)
    return kappa.real.copy(), kappa.imag.copy()


def dft2_brute(a, inverse=False):
    """O(N^4) two-dimensional DFT written out as a double sum (tiny maps only).

    forward: A[m2, m1] = sum_{y,x} a[y, x] exp(-2 pi i (m1 x + m2 y)/N)
    inverse: same with +i and a 1/N^2 factor.
    """
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[0]
    sgn = 1.0 if inverse else -1.0
    out = np.zeros((n, n), dtype=np.complex128)
    for m2 in range(n):
        for m1 in range(n):
            s = 0.0 + 0.0j
            for y in range(n):
                for x in range(n):
                    s += a[y, x] * np.exp(sgn * 2j * np.pi * (m1 * x + m2 * y) / n)
            out[m2, m1] = s
    if inverse:
        out /= n * n
    return out
