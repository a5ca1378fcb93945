"""Pins of the oracle's bounded-field starlet and padded KS (any sizes; periodic,
mirror and zero boundary rules)."""
import numpy as np
import pytest

import oracle as O
import synth as S


def transfer_1d(n, j):
    """Fourier response along one axis of starlet smoothing to level j."""
    w = 2.0 * np.pi * np.fft.fftfreq(n)
    h = np.ones(n)
    for i in range(j):
        s = float(1 << i)
        h *= (6 + 8 * np.cos(s * w) + 2 * np.cos(2 * s * w)) / 16.0
    return h


def test_boundary_index_rules():
    i = np.arange(-7, 12)
    assert list(O.boundary_index(i, 5, O.BC_PERIODIC)) == [int(v) % 5 for v in i]
    # whole-sample symmetric: ... 2 1 | 0 1 2 3 4 | 3 2 1 0 1 ...
    want = [1, 2, 3, 4, 3, 2, 1, 0, 1, 2, 3, 4, 3, 2, 1, 0, 1, 2, 3]
    assert list(O.boundary_index(i, 5, O.BC_MIRROR)) == want
    assert list(O.boundary_index(i, 5, O.BC_ZERO)) == [v if 0 <= v < 5 else -1 for v in i]
    assert list(O.boundary_index(np.arange(-3, 5), 2, O.BC_MIRROR)) == [1, 0, 1, 0, 1, 0, 1, 0]


@pytest.mark.parametrize("ny,nx,J", [(9, 17, 4), (33, 17, 5), (5, 9, 4), (17, 17, 6)])
def test_mirror_equals_periodic_on_the_even_extension(ny, nx, J):
    # the mirror rule is the periodic transform of the whole-sample symmetric
    # extension (period 2(n-1)), read back on the field; dilations reaching
    # past the field (J = 6 on 17 pixels) fold more than once
    rng = np.random.default_rng(ny * 100 + nx)
    a = rng.standard_normal((ny, nx))
    got = O.starlet_forward_bc(a, J, O.BC_MIRROR)
    ext = O.even_extension(a)
    assert ext.shape == (2 * (ny - 1), 2 * (nx - 1))
    c = ext
    for j in range(1, J):
        c_next = O.smooth_step(c, 1 << (j - 1))
        assert np.max(np.abs(got[j - 1] - (c - c_next)[:ny, :nx])) < 1e-13
        c = c_next
    assert np.max(np.abs(got[J - 1] - c[:ny, :nx])) < 1e-13


@pytest.mark.parametrize("ny,nx,J", [(24, 40, 4), (48, 20, 5), (30, 30, 3)])
def test_periodic_any_size_equals_fourier_transfer(ny, nx, J):
    # non-power-of-two, non-square periodic fields: every plane is the field
    # filtered by products of the 1-D B3 transfer functions
    rng = np.random.default_rng(ny + 7 * nx)
    a = rng.standard_normal((ny, nx))
    planes = O.starlet_forward_bc(a, J, O.BC_PERIODIC)
    A = np.fft.fft2(a)
    for j in range(1, J):
        t = np.outer(transfer_1d(ny, j - 1), transfer_1d(nx, j - 1)) - \
            np.outer(transfer_1d(ny, j), transfer_1d(nx, j))
        assert np.max(np.abs(planes[j - 1] - np.fft.ifft2(A * t).real)) < 1e-13
    t = np.outer(transfer_1d(ny, J - 1), transfer_1d(nx, J - 1))
    assert np.max(np.abs(planes[J - 1] - np.fft.ifft2(A * t).real)) < 1e-13


def test_periodic_rule_matches_the_square_transform():
    kappa = S.grf_kappa(64, 3)
    assert np.max(np.abs(O.starlet_forward_bc(kappa, 5, O.BC_PERIODIC) -
                         O.starlet_forward(kappa, 5))) < 1e-15


def brute_zero_cascade(a, J):
    """Plain loops: each smoothing step as a 2-D sum with zeros outside."""
    h = [1 / 16, 4 / 16, 6 / 16, 4 / 16, 1 / 16]
    ny, nx = a.shape
    c = [[float(a[y][x]) for x in range(nx)] for y in range(ny)]
    out = []
    for j in range(1, J):
        s = 1 << (j - 1)
        nxt = [[0.0] * nx for _ in range(ny)]
        for y in range(ny):
            for x in range(nx):
                acc = 0.0
                for ta in range(5):
                    for tb in range(5):
                        yy, xx = y + (ta - 2) * s, x + (tb - 2) * s
                        if 0 <= yy < ny and 0 <= xx < nx:
                            acc += h[ta] * h[tb] * c[yy][xx]
                nxt[y][x] = acc
        out.append([[c[y][x] - nxt[y][x] for x in range(nx)] for y in range(ny)])
        c = nxt
    out.append(c)
    return np.array(out)


def test_zero_rule_equals_brute_force_sum():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((7, 9))
    got = O.starlet_forward_bc(a, 4, O.BC_ZERO)
    assert np.max(np.abs(got - brute_zero_cascade(a, 4))) < 1e-14


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_reconstruction_under_every_rule(mode):
    rng = np.random.default_rng(10 + mode)
    a = rng.standard_normal((21, 34))
    planes = O.starlet_forward_bc(a, 5, mode)
    assert np.max(np.abs(planes.sum(axis=0) - a)) < 1e-13


def test_constant_field_has_no_details_under_mirror():
    planes = O.starlet_forward_bc(np.full((13, 6), 2.5), 5, O.BC_MIRROR)
    assert np.max(np.abs(planes[:-1])) < 1e-15
    assert np.max(np.abs(planes[-1] - 2.5)) < 1e-15
    # the zero rule leaks at the edges: the details are not zero there
    z = O.starlet_forward_bc(np.full((13, 6), 2.5), 3, O.BC_ZERO)
    assert np.max(np.abs(z[0])) > 0.1


def test_padded_ks_with_p_equal_n_is_the_periodic_inversion():
    _, g1, g2 = S.shear_map(32, 5, 6)
    kE, kB = O.ks_invert_padded(g1, g2, 32)
    rE, rB = O.ks_invert(g1, g2)
    assert np.array_equal(kE, rE) and np.array_equal(kB, rB)


def test_padded_ks_equals_brute_force_dft_route():
    # zero-extended 5 x 6 field in an 8 x 8 grid, inverted with the O(N^4)
    # DFT and the KS kernel written out here, read back on the rectangle
    rng = np.random.default_rng(8)
    g1, g2 = rng.standard_normal((5, 6)), rng.standard_normal((5, 6))
    P = 8
    a = np.zeros((P, P), dtype=np.complex128)
    a[:5, :6] = g1 + 1j * g2
    G = O.dft2_brute(a)
    K = np.zeros_like(G)
    for y in range(P):
        for x in range(P):
            m1 = x if x < P // 2 else x - P
            m2 = y if y < P // 2 else y - P
            den = m1 * m1 + m2 * m2
            if den == 0:
                continue
            nu = 0.0 if (m1 == -P // 2 or m2 == -P // 2) else 1.0
            D = ((m1 * m1 - m2 * m2) + 2j * nu * m1 * m2) / den
            K[y, x] = np.conj(D) * G[y, x]
    k = O.dft2_brute(K, inverse=True)
    kE, kB = O.ks_invert_padded(g1, g2, P)
    assert np.max(np.abs(kE - k.real[:5, :6])) < 1e-12
    assert np.max(np.abs(kB - k.imag[:5, :6])) < 1e-12


def test_bad_arguments():
    with pytest.raises(ValueError):
        O.starlet_forward_bc(np.zeros((1, 8)), 3, O.BC_MIRROR)
    with pytest.raises(ValueError):
        O.starlet_forward_bc(np.zeros((8, 8)), 3, 7)
    with pytest.raises(ValueError):
        O.ks_invert_padded(np.zeros((5, 6)), np.zeros((5, 6)), 4)
    with pytest.raises(ValueError):
        O.ks_invert_padded(np.zeros((5, 6)), np.zeros((5, 6)), 12)


def test_bounded_noise_reduces_to_the_periodic_noise():
    _, g1, g2 = S.shear_map(32, 11, 12)
    a = O.noise_sigma_bc(g1, g2, 32, 4, O.BC_PERIODIC, 5, 77)
    b = O.noise_sigma(g1, g2, 4, 5, 77)
    assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("mode", [O.BC_MIRROR, O.BC_ZERO])
def test_bounded_noise_variance_tracks_its_expectation(mode):
    # var w_j(x) = 1/2 sum_y |gamma(y)|^2 (A1(x,y)^2 + A2(x,y)^2) for uniform
    # rotation angles; A1, A2 probed with unit shears at every pixel
    ny, nx, P, J, R = 10, 12, 32, 3, 1200
    rng = np.random.default_rng(20 + mode)
    g1, g2 = 0.3 * rng.standard_normal((ny, nx)), 0.3 * rng.standard_normal((ny, nx))
    expect = np.zeros((J - 1, ny, nx))
    for y in range(ny):
        for x in range(nx):
            d = np.zeros((ny, nx))
            d[y, x] = 1.0
            A1 = O.starlet_forward_bc(O.ks_invert_padded(d, 0 * d, P)[0], J, mode)[:J - 1]
            A2 = O.starlet_forward_bc(O.ks_invert_padded(0 * d, d, P)[0], J, mode)[:J - 1]
            expect += 0.5 * (g1[y, x] ** 2 + g2[y, x] ** 2) * (A1 ** 2 + A2 ** 2)
    got = O.noise_sigma_bc(g1, g2, P, J, mode, R, 5) ** 2
    ratio = got / expect
    # chi-square scatter of a sample variance over R draws: sqrt(2/(R-1)) ~ 4%;
    # the pixel mean of the ratio is far tighter
    assert abs(float(ratio.mean()) - 1.0) < 0.02
    assert float(np.max(np.abs(ratio - 1.0))) < 6 * np.sqrt(2.0 / (R - 1)) * 1.5


def brute_peaks_bc(plane, t, mode):
    ny, nx = plane.shape
    rows = O.boundary_index(np.arange(-1, ny + 1), ny, mode)   # rows[y + 1] is row y
    cols = O.boundary_index(np.arange(-1, nx + 1), nx, mode)
    count = 0
    for y in range(ny):
        for x in range(nx):
            v = float(plane[y, x])
            ok = v > t
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if dy == 0 and dx == 0:
                        continue
                    yy, xx = int(rows[y + dy + 1]), int(cols[x + dx + 1])
                    q = 0.0 if (yy < 0 or xx < 0) else float(plane[yy, xx])
                    ok = ok and v > q
            count += ok
    return count


@pytest.mark.parametrize("mode", [O.BC_PERIODIC, O.BC_MIRROR, O.BC_ZERO])
def test_bounded_peaks_match_brute_force(mode):
    rng = np.random.default_rng(50 + mode)
    plane = rng.integers(-4, 5, size=(11, 14)).astype(np.float64) * 0.5   # ties and plateaus
    plane += rng.standard_normal((11, 14)) * (rng.random((11, 14)) < 0.6)
    plane[0, 0] = 9.0          # corner peak under every rule
    plane[10, 7] = 8.0         # bottom-edge peak
    for t in (-10.0, 0.0, 1.0):
        assert O.count_peaks_bc(plane, t, mode) == brute_peaks_bc(plane, t, mode)


def test_bounded_peaks_reduce_to_the_periodic_count():
    rng = np.random.default_rng(4)
    plane = rng.standard_normal((32, 32))
    for t in (-1.0, 0.5, 2.0):
        assert O.count_peaks_bc(plane, t, O.BC_PERIODIC) == O.count_peaks(plane, t)


def test_bounded_peaks_edge_rules_differ_as_stated():
    # a bright edge pixel is a peak under every rule; a raised edge pixel in
    # a negative plane is one under the mirror rule but not under the zero
    # rule, whose outside zeros are higher
    p = np.zeros((5, 6))
    p[2, 5] = 1.0
    assert O.count_peaks_bc(p, 0.5, O.BC_MIRROR) == 1
    assert O.count_peaks_bc(p, 0.5, O.BC_ZERO) == 1
    assert O.count_peaks_bc(p, 0.5, O.BC_PERIODIC) == 1
    q = np.full((5, 6), -1.0)
    q[2, 5] = -0.5
    assert O.count_peaks_bc(q, -0.9, O.BC_MIRROR) == 1
    assert O.count_peaks_bc(q, -0.9, O.BC_ZERO) == 0     # the zeros outside are higher
