"""Plane statistics through the C ABI against the oracle: central moments
(float64 accumulation; within 1e-10 relative of the oracle on the same
planes) and peak-height histograms (integer counts, bit-exact on identical
planes, both signs)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = amap.Context(0)
    yield c
    c.close()


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("n,J", [(16, 3), (64, 5), (256, 6), (1024, 7)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_moments_of_starlet_planes(ctx, n, J, dtype):
    print("moments n=%d J=%d %s" % (n, J, dtype), flush=True)
    kappa = S.grf_kappa(n, 80 + J)
    planes = ctx.starlet_forward(dev(kappa, dtype), J)
    got = ctx.plane_moments(planes).cpu().numpy()
    ref = O.plane_moments_stack(planes.double().cpu().numpy())   # the same values
    for p in range(J):
        scale = max(abs(ref[p, 1]), 1e-300)
        assert abs(got[p, 0] - ref[p, 0]) <= 1e-10 * np.sqrt(scale)
        assert abs(got[p, 1] - ref[p, 1]) <= 1e-10 * scale
        assert abs(got[p, 2] - ref[p, 2]) <= 1e-10 * scale ** 1.5
        assert abs(got[p, 3] - ref[p, 3]) <= 1e-10 * scale ** 2


def test_moments_special_planes(ctx):
    n = 64
    iy, ix = np.indices((n, n))
    board = 0.7 * (-1.0) ** (ix + iy)
    delta = np.zeros((n, n))
    delta[3, 5] = 1.0
    const = np.full((n, n), 2.5)
    rng = np.random.default_rng(6)
    skewed = rng.gamma(2.0, 1.5, size=(n, n))
    stack = np.stack([board, delta, const, skewed])
    got = ctx.plane_moments(dev(stack, torch.float64)).cpu().numpy()
    ref = O.plane_moments_stack(stack)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-15)
    # reproducible bit for bit
    again = ctx.plane_moments(dev(stack, torch.float64)).cpu().numpy()
    assert np.array_equal(got, again)


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_histogram_bit_exact(ctx, sign, dtype):
    rng = np.random.default_rng(10 + sign)
    planes = rng.standard_normal((4, 128, 128)) * 2.0
    planes[0, 0, 0] = 11.0           # across the wrap
    planes[1, 5, 5:7] = 4.0          # plateau
    planes[2, 9, 9] = np.nan
    planes[3] = np.round(planes[3] * 2) / 2   # many ties
    t = dev(planes, dtype)
    same = t.double().cpu().numpy()
    for lo, hi, nb in ((-1.0, 5.0, 12), (0.0, 1e6, 1), (2.5, 3.5, 1000)):
        got = ctx.peak_histogram(t, lo, hi, nb, sign).cpu().numpy()
        ref = O.peak_histogram_planes(same, lo, hi, nb, sign)
        assert np.array_equal(got, ref), (lo, hi, nb)


def test_histogram_on_the_noise_path_planes(ctx):
    # the full 1024^2 path's S/N planes: histogram of peaks and troughs
    # bit-exact against the oracle on the same planes; the sum above t
    # equals the path's own peak counts
    _, g1, g2 = S.shear_map(1024, 11, 12)
    t1, t2 = dev(g1, torch.float32), dev(g2, torch.float32)
    out = ctx.run_path(t1, t2, 7, 16, 23, 3.0)
    snr = out["snr"]
    same = snr.double().cpu().numpy()
    for sign in (1, -1):
        got = ctx.peak_histogram(snr, -2.0, 8.0, 40, sign).cpu().numpy()
        assert np.array_equal(got, O.peak_histogram_planes(same, -2.0, 8.0, 40, sign))
    # h > 3 exactly: no float lies between 3 and the next double above it
    above = ctx.peak_histogram(snr, float(np.nextafter(3.0, 4.0)), 1e30, 1, 1).cpu().numpy()[:, 0]
    assert [int(v) for v in above] == [int(v) for v in out["peaks"].cpu()]


def test_statistics_reject_bad_arguments(ctx):
    t = torch.zeros((2, 64, 64), device="cuda")
    with pytest.raises(amap.AmapError):
        ctx.peak_histogram(t, 1.0, 1.0, 4)
    with pytest.raises(amap.AmapError):
        ctx.peak_histogram(t, 0.0, 1.0, 0)
    with pytest.raises(amap.AmapError):
        ctx.peak_histogram(t, 0.0, 1.0, 4, sign=2)
