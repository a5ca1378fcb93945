"""Seeded synthetic inputs for the aperture-mass path.

Used by the tests (on both the oracle and the HIP side), by ``bench.py`` and
by the smoke check.  It holds none of the path's own arithmetic (no KS
inversion, no starlet, no noise maps, no peak finding): it only produces the
shear maps and workload descriptions the path is run on.

Recipe (what the paper's inputs look like; the paper's own maps are not
available, so seeded Gaussian random fields stand in for them):

  * convergence kappa: a periodic Gaussian random field with power spectrum
    P(k) ~ k^-2 (Fourier amplitude |k|^-1 applied to white noise), the k = 0
    mode and the Nyquist row and column set to zero, rescaled so that its
    root-mean-square is exactly ``rms`` (0.02 by default);
  * shear from kappa through the lensing potential psi (kappa = lap(psi)/2):
    gamma1 = (psi_11 - psi_22)/2, gamma2 = psi_12, evaluated spectrally on
    the periodic grid -- each component is a real field built separately;
  * shape noise: independent N(0, 0.3/sqrt(20)) on each of gamma1, gamma2;
  * survey masks (missing data, end of Sec. 5): discs cut out around bright
    stars, radii log-uniform in [1.5, 12] pixels at uniform positions until
    about ``frac`` of the field is covered, plus one bad column and one bad
    row of pixels at seeded positions.

White noise comes from numpy's PCG64 seeded with the given integer seed.
"""

import math

import numpy as np

SHAPE_NOISE_SIGMA = 0.3 / math.sqrt(20.0)


def _signed_freq(n):
    i = np.arange(n)
    return np.where(i < n // 2, i, i - n)


def _spectral_grid(n):
    m = _signed_freq(n)
    my, mx = np.meshgrid(m, m, indexing="ij")
    ky = 2.0 * np.pi * my / n
    kx = 2.0 * np.pi * mx / n
    nyq = (mx == -(n // 2)) | (my == -(n // 2))
    return kx, ky, nyq


def grf_kappa(n, seed, rms=0.02):
    """Periodic Gaussian random field with P(k) ~ k^-2 and exact rms."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n))
    kx, ky, nyq = _spectral_grid(n)
    kk = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros((n, n))
    keep = (kk > 0) & ~nyq
    amp[keep] = 1.0 / kk[keep]
    field = np.fft.ifft2(np.fft.fft2(white) * amp).real
    return field * (rms / np.sqrt(np.mean(field * field)))


def emode_shear(kappa):
    """Shear (gamma1, gamma2) of a convergence map, via the lensing potential.

    In Fourier space psi = -2 kappa/|k|^2 (k != 0), second derivatives bring
    down -k_a k_b, so gamma1 = -(kx^2 - ky^2) psi / 2 and gamma2 = -kx ky psi.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    n = kappa.shape[0]
    kx, ky, _ = _spectral_grid(n)
    ksq = kx * kx + ky * ky
    kap = np.fft.fft2(kappa)
    psi = np.zeros_like(kap)
    nz = ksq > 0
    psi[nz] = -2.0 * kap[nz] / ksq[nz]
    g1 = np.fft.ifft2(-0.5 * (kx * kx - ky * ky) * psi).real
    g2 = np.fft.ifft2(-(kx * ky) * psi).real
    return g1, g2


def bmode_shear(kappa_b):
    """A pure B-mode shear field: the E-mode shear of ``kappa_b`` turned by 45
    degrees (gamma -> i gamma), i.e. (gamma1, gamma2) = (-e2, e1)."""
    e1, e2 = emode_shear(kappa_b)
    return -e2, e1


def shape_noise(n, seed, sigma=SHAPE_NOISE_SIGMA):
    """Independent Gaussian shape noise on the two shear components."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal((n, n)), sigma * rng.standard_normal((n, n))


def shear_map(n, grf_seed, noise_seed=None, rms=0.02):
    """Return (kappa_true, gamma1, gamma2) for one synthetic map.

    With ``noise_seed`` None the shears are noise-free.
    """
    kappa = grf_kappa(n, grf_seed, rms)
    g1, g2 = emode_shear(kappa)
    if noise_seed is not None:
        n1, n2 = shape_noise(n, noise_seed)
        g1 = g1 + n1
        g2 = g2 + n2
    return kappa, g1, g2


# Workload descriptions -----------------------------------------------------

#: single-map configurations: (name, N, grf seed, shape-noise seed, J)
SMALL_FP64 = ("256x256 fp64 map, J=5", 256, 1, 2, 5)
MAP_1024 = ("1024x1024 fp32 map, J=7", 1024, 11, 12, 7)
#: noise-map configuration on MAP_1024: realisations and phase seed
NOISE_1024 = {"n_real": 256, "seed": 23, "threshold": 3.0}


def uneven_batch_sides(count=512, seed=31):
    """Sides of an uneven batch: i.i.d. from {128, 256, 512, 1024, 2048}
    with weights 4:4:3:2:1."""
    rng = np.random.default_rng(seed)
    sides = np.array([128, 256, 512, 1024, 2048])
    w = np.array([4, 4, 3, 2, 1], dtype=np.float64)
    return [int(s) for s in rng.choice(sides, size=count, p=w / w.sum())]


def served_stream(count, qps, seed_arrivals=41, seed_sides=42):
    """Poisson arrival times (seconds) and log-uniform power-of-two sides in
    256..4096 for a served request stream."""
    ra = np.random.default_rng(seed_arrivals)
    rs = np.random.default_rng(seed_sides)
    gaps = ra.exponential(1.0 / qps, size=count)
    times = np.cumsum(gaps) - gaps[0]
    sides = [int(1 << int(e)) for e in rs.integers(8, 13, size=count)]
    return times, sides


def survey_mask(ny, nx, seed, frac=0.1):
    """Seeded observed/missing mask (uint8, 1 = observed) of an ny x nx field:
    star discs covering about ``frac`` of the area, one bad column, one bad row."""
    rng = np.random.default_rng(seed)
    m = np.ones((ny, nx), dtype=np.uint8)
    missing, target = 0, frac * ny * nx
    while missing < target:
        r = math.exp(rng.uniform(math.log(1.5), math.log(12.0)))
        cy, cx = rng.uniform(0, ny), rng.uniform(0, nx)
        y0, y1 = max(0, int(cy - r)), min(ny, int(cy + r) + 2)
        x0, x1 = max(0, int(cx - r)), min(nx, int(cx + r) + 2)
        yy, xx = np.mgrid[y0:y1, x0:x1]
        hit = ((yy - cy) ** 2 + (xx - cx) ** 2 <= r * r) & (m[y0:y1, x0:x1] != 0)
        m[y0:y1, x0:x1][hit] = 0
        missing += int(np.count_nonzero(hit))
    m[:, int(rng.integers(0, nx))] = 0
    m[int(rng.integers(0, ny)), :] = 0
    return m
