"""Brute-force aperture mass from the tangential shear (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows eq:shearmap (M_ap as the integral of Q times the tangential shear
about the aperture centre), on a periodic pixel grid with pixel area 1, the
filters of Sec. 4 (``oracle.filters``), and the truncation of Sec. 5.1
(filters cut at a radius vartheta_cut; the cut is inclusive, as the Heaviside
step of eq:sch):

    M(x) = sum over integer offsets d with 0 < |d|^2 <= cut^2 of
           Q_theta(|d|) * gamma_t(x + d; x),
    gamma_t = -[gamma1(x+d) cos 2phi + gamma2(x+d) sin 2phi],
    cos 2phi = (dx^2 - dy^2)/|d|^2,  sin 2phi = 2 dx dy/|d|^2,

indices modulo N.  The inclusion test |d|^2 <= cut^2 is made in float64.
The cost is O(N^2 cut^2), the complexity quoted in Sec. 5.1.

Pins (tests/test_oracle_direct.py): a pure tangential shear pattern about a
pixel returns gamma0 * sum_d Q (sign and angle conventions); translation
equivariance and linearity; the tangential form agrees with the convergence
form sum_d U_theta(|d|) kappa(x + d) for an E-mode field (eq:mapdef vs
eq:shearmap, to the discretisation tolerance); the starlet filter's map
agrees with the smoothed starlet plane (the paper's claim that w_j is the
aperture mass at theta = 2^j, to the anisotropy tolerance).
"""

import numpy as np

from .filters import filter_Q_theta, natural_cut, FILTER_STARLET, starlet_U


def _offsets(cut):
    """Integer offsets (dy, dx) with 0 < dx^2 + dy^2 <= cut^2 (float64 test)."""
    R = int(np.floor(cut))
    c2 = float(cut) * float(cut)
    out = []
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            r2 = float(dx * dx + dy * dy)
            if r2 == 0.0 or r2 > c2:
                continue
            out.append((dy, dx))
    return out


def _resolve_cut(filt, theta, cut):
    return natural_cut(filt, theta) if cut is None or cut <= 0 else float(cut)


def map_direct(g1, g2, theta, filt=FILTER_STARLET, fparam=0.0, cut=None):
    """Aperture-mass map by direct summation of the tangential shear."""
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    cut = _resolve_cut(filt, theta, cut)
    Q = filter_Q_theta(filt, theta, fparam)
    M = np.zeros_like(g1)
    for dy, dx in _offsets(cut):
        r2 = float(dx * dx + dy * dy)
        q = float(Q(np.sqrt(r2)))
        if q == 0.0:
            continue
        c2 = (dx * dx - dy * dy) / r2
        s2 = 2.0 * dx * dy / r2
        # np.roll(a, (-dy, -dx))[y, x] == a[(y + dy) mod N, (x + dx) mod N]
        s1 = np.roll(g1, (-dy, -dx), axis=(0, 1))
        s2g = np.roll(g2, (-dy, -dx), axis=(0, 1))
        M += q * (-(s1 * c2 + s2g * s2))
    return M


def map_direct_at(g1, g2, theta, points, filt=FILTER_STARLET, fparam=0.0, cut=None):
    """The same sum evaluated only at the given pixels ``points`` = [(y, x), ...]."""
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    n = g1.shape[0]
    cut = _resolve_cut(filt, theta, cut)
    Q = filter_Q_theta(filt, theta, fparam)
    offs = _offsets(cut)
    out = np.zeros(len(points))
    for i, (y, x) in enumerate(points):
        s = 0.0
        for dy, dx in offs:
            r2 = float(dx * dx + dy * dy)
            q = float(Q(np.sqrt(r2)))
            if q == 0.0:
                continue
            yy = (y + dy) % n
            xx = (x + dx) % n
            gt = -(g1[yy, xx] * (dx * dx - dy * dy) + g2[yy, xx] * 2.0 * dx * dy) / r2
            s += q * gt
        out[i] = s
    return out


def map_kappa_form_radial(kappa, theta, cut=None):
    """eq:mapdef with the radial starlet U of Sec. 4.2:
    M(x) = sum_{|d| <= cut} U(|d|/theta)/theta^2 kappa(x + d)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    cut = 2.0 * theta if cut is None or cut <= 0 else float(cut)
    R = int(np.floor(cut))
    M = np.zeros_like(kappa)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            r2 = float(dx * dx + dy * dy)
            if r2 > cut * cut:
                continue
            u = float(starlet_U(np.sqrt(r2) / theta)) / theta ** 2
            if u == 0.0:
                continue
            M += u * np.roll(kappa, (-dy, -dx), axis=(0, 1))
    return M
