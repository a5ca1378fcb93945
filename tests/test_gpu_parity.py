"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: float32 outputs within max-abs 1e-5 * rms(kappa) of the oracle;
float64 outputs within 1e-10 * rms(kappa); S/N within 1e-5 * rms(kappa) /
sigma pointwise; integer outputs (Philox bits, peak counts on identical
planes) bit-exact.  rms(kappa) is the population rms of the oracle's kappa_E
for the map under test.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-10}


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = amap.Context(0)
    yield c
    c.close()


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.double().cpu().numpy()


def rms(a):
    return float(np.sqrt(np.mean(np.asarray(a, dtype=np.float64) ** 2)))


def maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))))


# ---- Kaiser-Squires ---------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_ks_invert(ctx, n, dtype):
    print("ks_invert n=%d %s" % (n, dtype), flush=True)
    _, g1, g2 = S.shear_map(n, 7 + n, 8 + n)
    kE, kB = O.ks_invert(g1, g2)
    e, b = ctx.ks_invert(dev(g1, dtype), dev(g2, dtype), want_b=True)
    torch.cuda.synchronize()
    tol = TOL[dtype] * rms(kE)
    assert maxerr(host(e), kE) <= tol
    assert maxerr(host(b), kB) <= tol


def test_ks_white_noise_and_nyquist(ctx):
    # white input excites every wavenumber, including the Nyquist lines
    rng = np.random.default_rng(3)
    g1, g2 = rng.standard_normal((2, 64, 64))
    kE, kB = O.ks_invert(g1, g2)
    e, b = ctx.ks_invert(dev(g1, torch.float64), dev(g2, torch.float64), want_b=True)
    torch.cuda.synchronize()
    assert maxerr(host(e), kE) <= 1e-10 * rms(kE)
    assert maxerr(host(b), kB) <= 1e-10 * rms(kE)


def test_ks_recovers_emode_kappa_on_gpu(ctx):
    kappa, g1, g2 = S.shear_map(1024, 11, None)
    e, b = ctx.ks_invert(dev(g1, torch.float32), dev(g2, torch.float32), want_b=True)
    torch.cuda.synchronize()
    assert maxerr(host(e), kappa) <= 1e-5 * rms(kappa)
    assert float(host(b).__abs__().max()) <= 1e-5 * rms(kappa)


# ---- starlet ------------------------------------------------------------------

@pytest.mark.parametrize("n,J", [(16, 2), (16, 4), (32, 5), (64, 6), (128, 7), (256, 5), (256, 8),
                                 (1024, 7), (1024, 10), (2048, 9), (4096, 9), (4096, 12)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_starlet_forward(ctx, n, J, dtype):
    if dtype == torch.float64 and n * n * J > 4096 * 4096 * 9:
        pytest.skip("float64 checked up to 4096^2 with J = 9 to keep the suite short")
    print("starlet n=%d J=%d %s" % (n, J, dtype), flush=True)
    kappa = S.grf_kappa(n, 30 + J)
    ref = O.starlet_forward(kappa, J)
    got = ctx.starlet_forward(dev(kappa, dtype), J)
    torch.cuda.synchronize()
    assert got.shape == (J, n, n)
    assert maxerr(host(got), ref) <= TOL[dtype] * rms(kappa)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_reconstruct_and_zero_mean_on_gpu(ctx, dtype):
    n, J = 1024, 7
    kappa = S.grf_kappa(n, 12)
    k = dev(kappa, dtype)
    planes = ctx.starlet_forward(k, J)
    rec = ctx.starlet_reconstruct(planes)
    torch.cuda.synchronize()
    r = rms(kappa)
    assert maxerr(host(rec), kappa) <= TOL[dtype] * r
    assert maxerr(host(rec), O.starlet_reconstruct(host(planes))) <= TOL[dtype] * r
    means = host(planes[: J - 1]).mean(axis=(1, 2))
    assert np.all(np.abs(means) <= (1e-6 if dtype == torch.float32 else 1e-12) * r)


# ---- noise phases -----------------------------------------------------------------

@pytest.mark.parametrize("n,seed,r", [(16, 0, 0), (64, 23, 5), (1024, 23, 255),
                                      (256, 2 ** 63 + 7, 1 << 33)])
def test_phase_uniforms_bit_exact(ctx, n, seed, r):
    got = ctx.phase_uniforms(n, seed, r)
    torch.cuda.synchronize()
    ref = O.phase_uniforms_u32(n * n, seed, r).reshape(n, n)
    assert np.array_equal(got.cpu().numpy().view(np.uint32), ref)


# ---- noise maps, S/N, peaks ---------------------------------------------------------

@pytest.mark.parametrize("n,J,R,dtype", [(64, 4, 8, torch.float32), (128, 5, 20, torch.float32),
                                         (256, 5, 5, torch.float32), (64, 3, 3, torch.float64),
                                         (256, 8, 4, torch.float32), (256, 5, 3, torch.float64),
                                         (1024, 7, 18, torch.float32), (1024, 10, 3, torch.float32)])
def test_noise_maps_and_snr(ctx, n, J, R, dtype):
    print("noise n=%d J=%d R=%d %s" % (n, J, R, dtype), flush=True)
    seed = 40 + n
    _, g1, g2 = S.shear_map(n, 5 + n, 6 + n)
    kE, _ = O.ks_invert(g1, g2)
    planes_ref = O.starlet_forward(kE, J)
    sig_ref = O.noise_sigma(g1, g2, J, R, seed)
    snr_ref = O.snr_planes(planes_ref, sig_ref)
    t1, t2 = dev(g1, dtype), dev(g2, dtype)
    planes = ctx.starlet_forward(ctx.ks_invert(t1, t2)[0], J)
    sigma, snr = ctx.noise_maps(t1, t2, J, R, seed, planes_signal=planes)
    torch.cuda.synchronize()
    r = rms(kE)
    tol = TOL[dtype] * r
    sg, sn = host(sigma), host(snr)
    assert maxerr(sg, sig_ref) <= tol
    # S = w / sigma: errors of w and sigma (each within tol) propagate as
    # sigma |dS| <= |dw| + |S| |dsigma| <= tol (1 + |S|)
    assert np.all(np.abs(sn - snr_ref) * sig_ref <= tol * (1.0 + np.abs(snr_ref)) * (1 + 1e-6))
    # and the stored quotient reproduces the signal plane wherever sigma > 0
    w = planes_ref[: J - 1]
    nz = sg > 0
    assert np.max(np.abs(sn * sg - w)[nz]) <= 2 * tol
    assert np.all(sn[~nz] == 0.0)


def test_noise_expected_variance_full_size(ctx):
    # 1024^2, J = 7, R = 256: the sample variance tracks its closed-form
    # expectation 1/2 sum_y (A_j^2 + B_j^2)(x - y) |gamma(y)|^2 (pixel mean).
    n, J, R = 1024, 7, 256
    _, g1, g2 = S.shear_map(n, 11, 12)
    sigma, _ = ctx.noise_maps(dev(g1, torch.float32), dev(g2, torch.float32), J, R, 23,
                              want_snr=False)
    torch.cuda.synchronize()
    d = np.zeros((n, n))
    d[0, 0] = 1.0
    A = O.starlet_forward(O.ks_invert(d, 0 * d)[0], J)[: J - 1]
    B = O.starlet_forward(O.ks_invert(0 * d, d)[0], J)[: J - 1]
    mod2 = np.fft.fft2(g1 ** 2 + g2 ** 2)
    s2 = host(sigma) ** 2
    for j in range(J - 1):
        expect = np.fft.ifft2(np.fft.fft2(0.5 * (A[j] ** 2 + B[j] ** 2)) * mod2).real
        ratio = s2[j].mean() / expect.mean()
        assert abs(ratio - 1.0) < 0.03, (j, ratio)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_count_peaks_bit_exact_on_identical_planes(ctx, dtype):
    rng = np.random.default_rng(9)
    planes = (rng.standard_normal((5, 256, 256)) * 2.0)
    planes[0, 0, 0] = 9.0           # peak across the wrap
    planes[0, 255, 255] = 8.0
    planes[1, 10, 10:12] = 7.0      # plateau
    planes[2, 5, 5] = np.nan
    planes[2, 5, 6] = 6.0           # next to a NaN
    planes[3, 7, 7] = 3.0           # exactly at t
    planes[3, 7, 8] = np.float32(3.0000002)
    t = dev(planes, dtype)
    counts = ctx.count_peaks(t, 3.0)
    torch.cuda.synchronize()
    same = host(t)  # the exact values the GPU saw
    assert [int(v) for v in counts.cpu()] == O.count_peaks_planes(same, 3.0)


def test_peaks_both_directions_on_path_planes(ctx):
    n, J, R = 256, 5, 16
    _, g1, g2 = S.shear_map(n, 21, 22)
    out = ctx.run_path(dev(g1, torch.float32), dev(g2, torch.float32), J, R, 77, threshold=2.0)
    torch.cuda.synchronize()
    # GPU planes -> oracle count
    snr_gpu = out["snr"].cpu().numpy()
    assert [int(v) for v in out["peaks"].cpu()] == O.count_peaks_planes(snr_gpu, 2.0)
    # oracle planes (rounded to float32) -> GPU count
    ref = O.run_path(g1, g2, J, R, 77, threshold=2.0)
    snr32 = ref["snr"].astype(np.float32)
    got = ctx.count_peaks(dev(snr32, torch.float32), 2.0)
    torch.cuda.synchronize()
    assert [int(v) for v in got.cpu()] == O.count_peaks_planes(snr32, 2.0)


def test_run_path_matches_oracle_and_separate_calls(ctx):
    n, J, R, seed = 128, 5, 12, 3
    _, g1, g2 = S.shear_map(n, 31, 32)
    t1, t2 = dev(g1, torch.float32), dev(g2, torch.float32)
    out = ctx.run_path(t1, t2, J, R, seed, threshold=2.5)
    planes = ctx.starlet_forward(ctx.ks_invert(t1, t2)[0], J)
    sigma, snr = ctx.noise_maps(t1, t2, J, R, seed, planes_signal=planes)
    torch.cuda.synchronize()
    assert torch.equal(out["planes"], planes)
    assert torch.equal(out["sigma"], sigma)
    assert torch.equal(out["snr"], snr)
    ref = O.run_path(g1, g2, J, R, seed, threshold=2.5)
    r = rms(ref["kappa_e"])
    for key in ("kappa_e", "planes", "sigma"):
        assert maxerr(host(out[key]), ref[key]) <= 1e-5 * r, key


def test_determinism(ctx):
    n, J, R = 256, 6, 10
    _, g1, g2 = S.shear_map(n, 41, 42)
    t1, t2 = dev(g1, torch.float32), dev(g2, torch.float32)
    a = ctx.run_path(t1, t2, J, R, 9)
    b = ctx.run_path(t1, t2, J, R, 9)
    torch.cuda.synchronize()
    for key in ("kappa_e", "planes", "sigma", "snr", "peaks"):
        assert torch.equal(a[key], b[key]), key


# ---- direct aperture mass ---------------------------------------------------------------

@pytest.mark.parametrize("filt,fparam,theta,cut", [
    (O.FILTER_STARLET, 0.0, 2.0, 4.0), (O.FILTER_STARLET, 0.0, 4.0, 0.0),
    (O.FILTER_STARLET, 0.0, 3.0, 3.5), (O.FILTER_S98, 3.0, 4.0, 0.0),
    (O.FILTER_S98, 1.0, 5.0, 5.0), (O.FILTER_JBJ04, 0.5, 2.0, 0.0), (O.FILTER_JBJ04, 4.0, 4.0, 4.0)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_map_direct(ctx, filt, fparam, theta, cut, dtype):
    n = 128
    kappa, g1, g2 = S.shear_map(n, 51, 52)
    kE, _ = O.ks_invert(g1, g2)
    ref = O.map_direct(g1, g2, theta, filt, fparam, cut)
    got = ctx.map_direct(dev(g1, dtype), dev(g2, dtype), theta, filt, fparam, cut)
    torch.cuda.synchronize()
    assert maxerr(host(got), ref) <= TOL[dtype] * rms(kE)


@pytest.mark.parametrize("filt,fparam,theta,cut", [
    (O.FILTER_STARLET, 0.0, 4.0, 0.0), (O.FILTER_STARLET, 0.0, 3.5, 7.3), (O.FILTER_S98, 2.0, 6.0, 6.0),
    (O.FILTER_JBJ04, 1.0, 3.0, 0.0), (O.FILTER_STARLET, 0.0, 1.0, 1.0)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_map_direct_row_kernel(ctx, filt, fparam, theta, cut, dtype):
    # maps from 512 px wide run the LDS row kernel (taps in groups of four
    # dx, zero-padded outside the disc): whole-map parity at 512^2
    n = 512
    print("map_direct rows n=%d theta=%g cut=%g %s" % (n, theta, cut, dtype), flush=True)
    _, g1, g2 = S.shear_map(n, 53, 54)
    kE, _ = O.ks_invert(g1, g2)
    ref = O.map_direct(g1, g2, theta, filt, fparam, cut)
    got = ctx.map_direct(dev(g1, dtype), dev(g2, dtype), theta, filt, fparam, cut)
    torch.cuda.synchronize()
    assert maxerr(host(got), ref) <= TOL[dtype] * rms(kE)


@pytest.mark.parametrize("theta", [2, 16, 64])
def test_map_direct_full_size_sampled(ctx, theta):
    n = 1024
    _, g1, g2 = S.shear_map(n, 11, 12)
    kE, _ = O.ks_invert(g1, g2)
    got = host(ctx.map_direct(dev(g1, torch.float32), dev(g2, torch.float32), float(theta),
                              O.FILTER_STARLET, 0.0, float(theta)))
    rng = np.random.default_rng(theta)
    pts = [(0, 0), (n - 1, n - 1), (0, n - 1)] + [tuple(p) for p in rng.integers(0, n, (13, 2))]
    ref = O.map_direct_at(g1, g2, float(theta), pts, O.FILTER_STARLET, 0.0, float(theta))
    assert maxerr([got[p] for p in pts], ref) <= 1e-5 * rms(kE)


def test_map_direct_agrees_with_starlet_plane_on_gpu(ctx):
    # Sec. 3: w_j is the aperture mass at theta = 2^j (anisotropy tolerance)
    n, J = 256, 5
    _, g1, g2 = S.shear_map(n, 1, None)
    t1, t2 = dev(g1, torch.float64), dev(g2, torch.float64)
    planes = host(ctx.starlet_forward(ctx.ks_invert(t1, t2)[0], J))
    s = np.array([1.0, 4.0, 1.0]) / 6.0
    for j in (2, 3):
        theta = 2 ** j
        w = planes[j - 1]
        sw = sum(s[a + 1] * s[b + 1] * np.roll(w, (a, b), axis=(0, 1))
                 for a in (-1, 0, 1) for b in (-1, 0, 1))
        M = host(ctx.map_direct(t1, t2, float(theta), O.FILTER_STARLET, 0.0, 2.0 * theta))
        torch.cuda.synchronize()
        assert np.linalg.norm(M - sw) / np.linalg.norm(sw) < 0.05


# ---- validation on a live context ------------------------------------------------------

def test_invalid_arguments_raise(ctx):
    t = torch.zeros((48, 48), device="cuda")
    with pytest.raises(amap.AmapError):
        ctx.ks_invert(t, t)
    t = torch.zeros((64, 64), device="cuda")
    with pytest.raises(amap.AmapError):
        ctx.starlet_forward(t, 7)
    with pytest.raises(amap.AmapError):
        ctx.noise_maps(t, t, 3, 1, 0)
    with pytest.raises(amap.AmapError):
        ctx.map_direct(t, t, 20.0, O.FILTER_STARLET, 0.0, 0.0)  # cut 40 > n/2
    with pytest.raises(amap.AmapError):
        ctx.ks_invert(t, t, kappa_e=t)  # output aliases input
