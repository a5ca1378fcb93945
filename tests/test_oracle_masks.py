"""Pins of the oracle's masked-field routines (missing data inside the field):
the masked shear and the masked peak count."""
import numpy as np
import pytest

import oracle as O
import synth as S

RULES = [O.BC_PERIODIC, O.BC_MIRROR, O.BC_ZERO]


def edge(i, n, mode):
    """Index i through an edge rule, by walking (no modular formula);
    None outside the field under the zero rule."""
    if mode == O.BC_PERIODIC:
        while i < 0:
            i += n
        while i >= n:
            i -= n
        return i
    if mode == O.BC_MIRROR:
        while i < 0 or i >= n:
            i = -i if i < 0 else 2 * (n - 1) - i
        return i
    return i if 0 <= i < n else None


def brute_masked(plane, t, mode, mask):
    ny, nx = plane.shape
    count = 0
    for y in range(ny):
        for x in range(nx):
            v = float(plane[y, x])
            ok = v > t and mask[y, x] != 0
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dy, dx) == (0, 0):
                        continue
                    yy, xx = edge(y + dy, ny, mode), edge(x + dx, nx, mode)
                    if yy is None or xx is None:
                        ok = ok and v > 0.0
                    else:
                        ok = ok and v > float(plane[yy, xx]) and mask[yy, xx] != 0
            count += ok
    return count


def peak_positions(plane, t, mode):
    """Unmasked peaks, found pixel by pixel with the walking edge rule."""
    ny, nx = plane.shape
    out = []
    for y in range(ny):
        for x in range(nx):
            v = float(plane[y, x])
            ok = v > t
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dy, dx) == (0, 0):
                        continue
                    yy, xx = edge(y + dy, ny, mode), edge(x + dx, nx, mode)
                    q = 0.0 if (yy is None or xx is None) else float(plane[yy, xx])
                    ok = ok and v > q
            if ok:
                out.append((y, x))
    return out


def test_edge_walk_agrees_with_the_rules_on_small_cases():
    # the walking rule against hand-written sequences
    assert [edge(i, 4, O.BC_PERIODIC) for i in range(-5, 9)] == [3, 0, 1, 2, 3, 0, 1, 2, 3, 0, 1, 2, 3, 0]
    assert [edge(i, 4, O.BC_MIRROR) for i in range(-5, 9)] == [1, 2, 3, 2, 1, 0, 1, 2, 3, 2, 1, 0, 1, 2]
    assert [edge(i, 4, O.BC_ZERO) for i in (-1, 0, 3, 4)] == [None, 0, 3, None]


@pytest.mark.parametrize("mode", RULES)
def test_all_observed_equals_the_bounded_count(mode):
    rng = np.random.default_rng(70 + mode)
    plane = rng.standard_normal((23, 31))
    ones = np.ones(plane.shape, dtype=np.uint8)
    for t in (-2.0, 0.0, 1.0):
        assert O.count_peaks_masked(plane, t, mode, ones) == O.count_peaks_bc(plane, t, mode)


@pytest.mark.parametrize("mode", RULES)
def test_masked_count_matches_brute_force(mode):
    rng = np.random.default_rng(80 + mode)
    ny, nx = 13, 17
    plane = rng.integers(-3, 4, size=(ny, nx)).astype(np.float64) * 0.5   # ties and plateaus
    plane += rng.standard_normal((ny, nx)) * (rng.random((ny, nx)) < 0.7)
    plane[0, 0], plane[12, 9], plane[6, 16] = 9.0, 8.0, 7.0          # corner and edge peaks
    for trial in range(4):
        mask = (rng.random((ny, nx)) > 0.15 * trial).astype(np.uint8)
        mask[0, 1] = 0 if trial % 2 else 1      # a hole beside the corner peak
        for t in (-10.0, 0.0, 1.0):
            assert O.count_peaks_masked(plane, t, mode, mask) == brute_masked(plane, t, mode, mask)


@pytest.mark.parametrize("mode", RULES)
def test_single_hole_removes_the_peaks_around_it(mode):
    rng = np.random.default_rng(90 + mode)
    ny, nx = 20, 24
    plane = rng.standard_normal((ny, nx))
    t = 0.5
    peaks = peak_positions(plane, t, mode)
    assert len(peaks) >= 5
    for (hy, hx) in [peaks[0], peaks[len(peaks) // 2], (0, 0), (ny - 1, nx - 1), (7, 0)]:
        mask = np.ones((ny, nx), dtype=np.uint8)
        mask[hy, hx] = 0
        near = 0
        for (y, x) in peaks:
            touched = (y, x) == (hy, hx)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (edge(y + dy, ny, mode), edge(x + dx, nx, mode)) == (hy, hx):
                        touched = True
            near += touched
        assert O.count_peaks_masked(plane, t, mode, mask) == len(peaks) - near


def test_fully_missing_field():
    rng = np.random.default_rng(3)
    g1, g2 = rng.standard_normal((2, 16, 24))
    none = np.zeros((16, 24), dtype=np.uint8)
    a1, a2 = O.mask_shear(g1, g2, none)
    assert not np.any(a1) and not np.any(a2)
    kE, kB = O.ks_invert_padded(a1, a2, 32)
    assert not np.any(kE) and not np.any(kB)
    for mode in RULES:
        assert O.count_peaks_masked(rng.standard_normal((16, 24)), -5.0, mode, none) == 0


def test_mask_shear_keeps_observed_pixels_exactly():
    _, g1, g2 = S.shear_map(64, 5, 6)
    m = S.survey_mask(64, 64, 7)
    a1, a2 = O.mask_shear(g1, g2, m)
    assert np.array_equal(a1[m != 0], g1[m != 0]) and np.array_equal(a2[m != 0], g2[m != 0])
    assert not np.any(a1[m == 0]) and not np.any(a2[m == 0])


@pytest.mark.parametrize("ny,nx,P", [(40, 56, 64), (64, 64, 64), (30, 50, 128)])
def test_masked_and_complementary_convergence_add_up(ny, nx, P):
    # the inversion is linear: KS(m g) + KS((1-m) g) = KS(g)
    rng = np.random.default_rng(ny * nx)
    g1, g2 = rng.standard_normal((2, ny, nx)) * 0.05
    m = S.survey_mask(ny, nx, 11, frac=0.2)
    a = O.ks_invert_padded(*O.mask_shear(g1, g2, m), P)
    b = O.ks_invert_padded(*O.mask_shear(g1, g2, 1 - m), P)
    full = O.ks_invert_padded(g1, g2, P)
    for k in range(2):
        assert np.max(np.abs(a[k] + b[k] - full[k])) < 1e-14
        assert np.max(np.abs(a[k] - full[k])) > 1e-3      # the mask matters


def test_survey_mask_recipe():
    m = S.survey_mask(256, 192, 5, frac=0.1)
    assert m.dtype == np.uint8 and m.shape == (256, 192)
    f = np.mean(m == 0)
    assert 0.1 <= f < 0.2
    assert np.array_equal(m, S.survey_mask(256, 192, 5, frac=0.1))
    assert (np.all(m == 0, axis=0)).sum() >= 1 and (np.all(m == 0, axis=1)).sum() >= 1


def test_bad_mask_shape():
    with pytest.raises(ValueError):
        O.count_peaks_masked(np.zeros((4, 5)), 0.0, O.BC_ZERO, np.ones((5, 4), dtype=np.uint8))
