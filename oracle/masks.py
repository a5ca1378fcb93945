"""Masked fields: missing data inside the field (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The end of Sec. 5 names missing data (stars and bad pixels cut out of the
image) as a source of bias that the reconstruction does not undo, and leaves
its handling to other work.  Readings used here:

  * a mask is an ny x nx array of bytes, non-zero where the pixel is observed
    and zero where it is missing;
  * a missing pixel carries no shear: the shear field that enters the
    Kaiser-Squires inversion is the mask times the measured shear (nothing is
    recovered inside the holes, as the paper says of plain reconstruction);
    the noise realisations rotate that same field, so missing pixels stay
    empty in every realisation;
  * a peak of a masked plane is a peak of ``oracle.bounded.count_peaks_bc``
    (strict 8-neighbour maximum above t, neighbours through the edge rule)
    whose own pixel and all eight neighbours are observed: a maximum that
    touches missing data is not counted.  A neighbour that the edge rule
    takes outside the field (the zero rule) has no mask value and does not
    veto the peak; under the periodic and mirror rules the neighbour's mask
    value is read at the same mapped index as its plane value.

Pins (tests/test_oracle_masks.py): with every pixel observed the masked count
equals ``count_peaks_bc`` under every rule; a pure-Python loop over pixels
and neighbours (its own edge arithmetic) gives the same counts on small
random planes and masks; a single missing pixel removes exactly the unmasked
peaks within one pixel of it (Chebyshev distance through the edge rule); a
fully missing field has no peaks and a zero shear; the masked shear and the
shear of the complementary mask add up to the full shear, so by linearity of
the inversion their convergences add up to that of the full field.
"""

import numpy as np

from .bounded import boundary_index


def mask_shear(g1, g2, mask):
    """Shear of a masked field: zero where the mask is zero (float64 copies)."""
    m = np.asarray(mask) != 0
    a1 = np.where(m, np.asarray(g1, dtype=np.float64), 0.0)
    a2 = np.where(m, np.asarray(g2, dtype=np.float64), 0.0)
    return a1, a2


def count_peaks_masked(plane, t, mode, mask):
    """Peaks above t of an ny x nx plane whose pixel and 8 neighbours are observed."""
    p = np.asarray(plane).astype(np.float64)
    obs = np.asarray(mask) != 0
    ny, nx = p.shape
    if obs.shape != p.shape:
        raise ValueError("mask and plane shapes differ")
    keep = (p > float(t)) & obs
    for dy in (-1, 0, 1):
        iy = boundary_index(np.arange(ny) + dy, ny, mode)
        for dx in (-1, 0, 1):
            if dy == 0 and dx == 0:
                continue
            ix = boundary_index(np.arange(nx) + dx, nx, mode)
            inside = (iy[:, None] >= 0) & (ix[None, :] >= 0)
            yy = np.where(iy < 0, 0, iy)
            xx = np.where(ix < 0, 0, ix)
            q = np.where(inside, p[np.ix_(yy, xx)], 0.0)
            qm = np.where(inside, obs[np.ix_(yy, xx)], True)
            keep &= (p > q) & qm
    return int(np.count_nonzero(keep))


def count_peaks_masked_planes(planes, t, mode, mask):
    """count_peaks_masked over a stack of planes (one mask for all)."""
    return [count_peaks_masked(pl, t, mode, mask) for pl in planes]
