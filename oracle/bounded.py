"""Starlet and Kaiser-Squires on fields of any size with stated boundaries (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's fields are periodic squares of side 2^k only where it says so;
real survey fields have edges and arbitrary sizes, which the paper raises at
the end of Sec. 5 without fixing a rule.  Readings used here:

  * a field is ny x nx (any sizes >= 2), row-major [y][x];
  * the starlet cascade is that of ``oracle.starlet`` (B3 taps (1,4,6,4,1)/16
    at dilation 2^(j-1) for smoothing step j, row pass along x then column
    pass along y, planes w_1 .. w_{J-1}, c_{J-1}), with every index that
    falls outside [0, n) taken through one of three boundary rules, applied
    to c_{j-1} at every step and on each axis separately:
      - periodic: i mod n;
      - mirror (whole-sample symmetric): reflection about the first and last
        samples, c(-i) = c(i) and c(n-1+i) = c(n-1-i), i.e. the index taken
        modulo 2(n-1) and folded back; the edge samples are not repeated;
      - zero: c = 0 outside the field;
  * noise maps of a bounded field follow Sec. 1 and Sec. 5.1 as in
    ``oracle.noise``: realisation r rotates every pixel's shear by
    2 pi u, u the Philox uniform of flat pixel index y * nx + x (the
    definition of ``oracle.rng``), and the rotated field goes through the
    same padded KS and bounded starlet as the signal; sigma_j is the
    unbiased per-pixel sample standard deviation (Welford's update);
  * a peak of a bounded plane is a strict 8-neighbour maximum above t (as in
    ``oracle.peaks``) with each neighbour's row and column index taken
    through the plane's edge rule (under the zero rule a neighbour outside
    the field has value 0; under the mirror rule an edge pixel meets its
    inner neighbour twice);
  * KS of a bounded field: the shear is zero outside its ny x nx rectangle,
    which is placed at the origin of a P x P periodic grid (P a power of two,
    P >= max(ny, nx)); the periodic KS of ``oracle.ks`` is applied there and
    the ny x nx rectangle is read back.  P = n for an n x n field (n a power
    of two) is the periodic inversion itself.

Pins (tests/test_oracle_bounded.py): the mirror transform equals the periodic
transform of the field's even extension (2(ny-1) x 2(nx-1)), restricted to
the field; the periodic transform of a non-power-of-two, non-square field
equals Fourier multiplication by the B3 transfer functions; the zero rule
equals a brute-force two-dimensional sum with zeros outside, on a small
field; exact reconstruction under every rule; a constant field has zero
detail planes under the mirror rule; the padded KS with P = n reproduces the
periodic inversion, and on a small field equals the inversion carried out
with the O(N^4) brute-force DFT; the bounded noise sigma under the periodic
rule with P = n equals ``oracle.noise.noise_sigma``, and its variance tracks
the closed form 1/2 sum_y |gamma(y)|^2 (A1(x, y)^2 + A2(x, y)^2), A1 and A2
the responses of w_j(x) to unit gamma1 and gamma2 at y, within chi-square
scatter; bounded peak counts under the periodic rule equal
``oracle.peaks.count_peaks``, and under every rule equal a pure-Python loop
over pixels and neighbours.
"""

import numpy as np

from .filters import b3_taps
from .ks import ks_invert
from .noise import rotate_shear
from .rng import phase_uniforms_u32

BC_PERIODIC = 0
BC_MIRROR = 1
BC_ZERO = 2


def boundary_index(i, n, mode):
    """Index array i mapped into [0, n) by the boundary rule; -1 marks a
    sample outside the field under the zero rule."""
    i = np.asarray(i, dtype=np.int64)
    if mode == BC_PERIODIC:
        return np.mod(i, n)
    if mode == BC_MIRROR:
        if n < 2:
            raise ValueError("the mirror rule needs n >= 2")
        p = 2 * (n - 1)
        k = np.mod(i, p)
        return np.where(k < n, k, p - k)
    if mode == BC_ZERO:
        return np.where((i >= 0) & (i < n), i, -1)
    raise ValueError("unknown boundary rule %r" % (mode,))


def _take(c, idx, axis):
    """c sampled at boundary-mapped indices idx along axis (0 where idx < 0)."""
    safe = np.where(idx < 0, 0, idx)
    out = np.take(c, safe, axis=axis)
    if np.any(idx < 0):
        shape = [1, 1]
        shape[axis] = -1
        out = np.where(idx.reshape(shape) < 0, 0.0, out)
    return out


def smooth_step_bc(c, s, mode):
    """One a trous smoothing step at dilation s under a boundary rule."""
    h = b3_taps()
    ny, nx = c.shape
    r = np.zeros_like(c)
    for t in range(-2, 3):
        r += h[t + 2] * _take(c, boundary_index(np.arange(nx) + t * s, nx, mode), axis=1)
    out = np.zeros_like(c)
    for t in range(-2, 3):
        out += h[t + 2] * _take(r, boundary_index(np.arange(ny) + t * s, ny, mode), axis=0)
    return out


def starlet_forward_bc(image, J, mode):
    """Starlet planes [w_1, ..., w_{J-1}, c_{J-1}] of an ny x nx field."""
    c = np.asarray(image, dtype=np.float64)
    if c.ndim != 2 or min(c.shape) < 2:
        raise ValueError("need a 2-D field of at least 2 x 2")
    if J < 2:
        raise ValueError("need J >= 2")
    planes = np.empty((J,) + c.shape, dtype=np.float64)
    for j in range(1, J):
        c_next = smooth_step_bc(c, 1 << (j - 1), mode)
        planes[j - 1] = c - c_next
        c = c_next
    planes[J - 1] = c
    return planes


def even_extension(a):
    """Whole-sample symmetric extension of an ny x nx field to 2(ny-1) x 2(nx-1)."""
    a = np.asarray(a, dtype=np.float64)
    ny, nx = a.shape
    iy = boundary_index(np.arange(2 * (ny - 1)), ny, BC_MIRROR)
    ix = boundary_index(np.arange(2 * (nx - 1)), nx, BC_MIRROR)
    return a[np.ix_(iy, ix)]


def ks_invert_padded(g1, g2, P):
    """KS of an ny x nx shear field zero-extended into a P x P periodic grid;
    returns (kappa_E, kappa_B) on the field's rectangle."""
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    ny, nx = g1.shape
    assert g2.shape == (ny, nx)
    if P < max(ny, nx) or P & (P - 1):
        raise ValueError("P must be a power of two >= max(ny, nx)")
    a1 = np.zeros((P, P))
    a2 = np.zeros((P, P))
    a1[:ny, :nx] = g1
    a2[:ny, :nx] = g2
    kE, kB = ks_invert(a1, a2)
    return kE[:ny, :nx].copy(), kB[:ny, :nx].copy()


def noise_sigma_bc(g1, g2, P, J, mode, n_real, seed):
    """Per-pixel, per-scale noise sigma_j of an ny x nx field (shape (J-1, ny, nx))."""
    if n_real < 2:
        raise ValueError("need at least two realisations")
    g1 = np.asarray(g1, dtype=np.float64)
    g2 = np.asarray(g2, dtype=np.float64)
    ny, nx = g1.shape
    mean = np.zeros((J - 1, ny, nx))
    m2 = np.zeros((J - 1, ny, nx))
    for r in range(n_real):
        v = phase_uniforms_u32(ny * nx, seed, r)
        u = ((v >> np.uint32(8)).astype(np.float64) * 2.0 ** -24).reshape(ny, nx)
        a1, a2 = rotate_shear(g1, g2, u)
        kE, _ = ks_invert_padded(a1, a2, P)
        w = starlet_forward_bc(kE, J, mode)[:J - 1]
        delta = w - mean
        mean += delta / (r + 1)
        m2 += delta * (w - mean)
    return np.sqrt(m2 / (n_real - 1))


def count_peaks_bc(plane, t, mode):
    """Strict 8-neighbour maxima above t of an ny x nx plane under an edge rule."""
    p = np.asarray(plane).astype(np.float64)
    ny, nx = p.shape
    mask = p > float(t)
    for dy in (-1, 0, 1):
        iy = boundary_index(np.arange(ny) + dy, ny, mode)
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            ix = boundary_index(np.arange(nx) + dx, nx, mode)
            q = _take(_take(p, iy, axis=0), ix, axis=1)
            mask &= p > q
    return int(np.count_nonzero(mask))
