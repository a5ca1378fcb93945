"""Starlet (isotropic undecimated, a trous) wavelet transform (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows Sec. 3 (the decomposition kappa = c_J + sum_j w_j into J = j_max + 1
sub-arrays, with w_j the map filtered at scale 2^j) and Sec. 4.2 (eq:splinewl
and the B3 spline phi).  Reading of the paper used here:

  * c_0 = kappa.  For j = 1 .. J-1, with dilation s = 2^(j-1) and the B3
    taps h = (1,4,6,4,1)/16:
        r(x, y)   = sum_t h_t c_{j-1}(x + t s, y)        (row pass, along x)
        c_j(x, y) = sum_t h_t r(x, y + t s)              (column pass, along y)
        w_j       = c_{j-1} - c_j
    indices taken modulo N (periodic boundary);
  * output planes, in order: w_1 .. w_{J-1}, c_{J-1};
  * the transform needs 2^J <= N (Sec. 5.1).

Pins (tests/test_oracle_starlet.py): the cascade identity (impulse response of
c_j convolved with [1,4,1]/6 equals samples of phi(m/2^j)/2^j, exact
rationals); the kappa-form identity sum_d psi_theta(d) kappa(x + d) =
([1,4,1]/6 (x) [1,4,1]/6 * w_j)(x) for theta = 2^j; brute-force periodic
convolution with the transform's own impulse response; exact reconstruction
(Sec. 3 decomposition); zero mean of every w_j (wavelets are compensated,
Sec. 3).
"""

import numpy as np

from .filters import b3_taps, phi_b3


def smooth_step(c, s):
    """One a trous smoothing step at dilation s: row pass then column pass."""
    h = b3_taps()
    r = np.zeros_like(c)
    for t in range(-2, 3):
        # np.roll(c, -t*s, axis=1)[y, x] == c[y, (x + t*s) mod N]
        r += h[t + 2] * np.roll(c, -t * s, axis=1)
    out = np.zeros_like(c)
    for t in range(-2, 3):
        out += h[t + 2] * np.roll(r, -t * s, axis=0)
    return out


def starlet_forward(kappa, J):
    """Starlet decomposition into J planes [w_1, ..., w_{J-1}, c_{J-1}]."""
    c = np.asarray(kappa, dtype=np.float64)
    n = c.shape[0]
    if J < 2 or (1 << J) > n:
        raise ValueError("need 2 <= J and 2^J <= N (J=%d, N=%d)" % (J, n))
    planes = np.empty((J, n, n), dtype=np.float64)
    for j in range(1, J):
        c_next = smooth_step(c, 1 << (j - 1))
        planes[j - 1] = c - c_next
        c = c_next
    planes[J - 1] = c
    return planes


def starlet_reconstruct(planes):
    """Inverse of the decomposition of Sec. 3: kappa = c_{J-1} + sum_j w_j."""
    planes = np.asarray(planes, dtype=np.float64)
    out = planes[-1].copy()
    for j in range(planes.shape[0] - 1):
        out += planes[j]
    return out


def starlet_impulse_response(n, J):
    """Planes of the transform applied to a unit delta at the origin (n x n)."""
    d = np.zeros((n, n))
    d[0, 0] = 1.0
    return starlet_forward(d, J)


def convolve_periodic(a, kern):
    """Brute-force periodic convolution (a * kern)(x) = sum_y kern(y) a(x - y).

    ``kern`` is an n x n array indexed by offset modulo n.  O(N^4); tiny maps.
    """
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    out = np.zeros_like(a)
    for oy in range(n):
        for ox in range(n):
            k = kern[oy, ox]
            if k != 0.0:
                out += k * np.roll(a, (oy, ox), axis=(0, 1))
    return out


def separable_psi_taps(theta):
    """Samples of psi_theta(dx, dy) = theta^-2 [4 phi(2dx/theta) phi(2dy/theta)
    - phi(dx/theta) phi(dy/theta)] at integer offsets |d|_inf <= 2 theta
    (eq:splinewl scaled to aperture radius theta, pixel area 1).

    Returns (offsets, weights): offsets is the 1-D range -2theta..2theta and
    weights is the 2-D array indexed [dy, dx] over that range.
    """
    R = int(2 * theta)
    d = np.arange(-R, R + 1, dtype=np.float64)
    a = phi_b3(2.0 * d / theta)
    b = phi_b3(d / theta)
    w = (4.0 * np.outer(a, a) - np.outer(b, b)) / theta ** 2
    return d.astype(int), w
