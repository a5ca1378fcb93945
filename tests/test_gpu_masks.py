"""Masked fields (missing data inside the field, end of Sec. 5) through the C
ABI against the FP64 oracle: the masked shear, the masked peak count, and a
masked field through the bounded and the periodic paths.

The masked shear is bit-exact (a copy or a zero); peak counts are bit-exact
on identical planes in both directions; planes, sigma and S/N follow the
bounds of the unmasked paths (1e-5 * rms for FP32, the propagated bound for
S/N).  Masks come from ``synth.survey_mask``: star discs covering about a
tenth of the field, one bad column and one bad row.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-10}
RULES = [amap.BC_PERIODIC, amap.BC_MIRROR, amap.BC_ZERO]


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    c = amap.Context(0)
    yield c
    c.close()


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rms(a):
    return float(np.sqrt(np.mean(np.asarray(a, dtype=np.float64) ** 2)))


@pytest.mark.parametrize("ny,nx", [(96, 80), (37, 51), (1, 3), (1000, 1000)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_mask_shear_bit_exact(ctx, ny, nx, dtype):
    print("mask shear %dx%d %s" % (ny, nx, dtype), flush=True)
    rng = np.random.default_rng(ny + nx)
    g1, g2 = rng.standard_normal((2, ny, nx))
    m = S.survey_mask(ny, nx, 5) if min(ny, nx) > 8 else (rng.random((ny, nx)) > 0.5).astype(np.uint8)
    t1, t2, tm = dev(g1, dtype), dev(g2, dtype), torch.tensor(m, device="cuda")
    a1, a2 = ctx.mask_shear(t1, t2, tm)
    torch.cuda.synchronize()
    r1, r2 = O.mask_shear(t1.double().cpu().numpy(), t2.double().cpu().numpy(), m)
    assert np.array_equal(a1.double().cpu().numpy(), r1) and np.array_equal(a2.double().cpu().numpy(), r2)
    # in place
    ctx.mask_shear(t1, t2, tm, out1=t1, out2=t2)
    torch.cuda.synchronize()
    assert torch.equal(t1, a1) and torch.equal(t2, a2)


@pytest.mark.parametrize("rule", RULES)
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_masked_peaks_bit_exact(ctx, rule, dtype):
    rng = np.random.default_rng(100 + rule)
    ny, nx = 77, 131
    planes = rng.integers(-4, 5, size=(4, ny, nx)).astype(np.float64) * 0.5    # ties and plateaus
    planes += rng.standard_normal(planes.shape) * (rng.random(planes.shape) < 0.6)
    planes[0, 0, 0] = 9.0          # corner
    planes[1, 76, 40] = 8.0        # bottom edge
    planes[2, 10, 10] = np.nan
    planes[3] = -np.abs(planes[3])
    m = S.survey_mask(ny, nx, 9 + rule, frac=0.15)
    m[0, 1] = 0                    # a hole beside the corner peak
    t, tm = dev(planes, dtype), torch.tensor(m, device="cuda")
    same = t.double().cpu().numpy()
    for thr in (-10.0, -0.25, 0.0, 1.0, 3.0):
        got = ctx.count_peaks_masked(t, tm, thr, rule).cpu().numpy()
        ref = O.count_peaks_masked_planes(same, thr, rule, m)
        assert [int(v) for v in got] == ref, (thr, rule)
    # every pixel observed: the bounded count
    ones = torch.ones((ny, nx), dtype=torch.uint8, device="cuda")
    a = ctx.count_peaks_masked(t, ones, 0.0, rule)
    b = ctx.count_peaks_bc(t, 0.0, rule)
    assert torch.equal(a, b)


@pytest.mark.parametrize("ny,nx,P,J,R,rule", [(200, 168, 256, 5, 8, amap.BC_MIRROR),
                                              (120, 90, 256, 4, 5, amap.BC_ZERO)])
def test_masked_bounded_field_end_to_end(ctx, ny, nx, P, J, R, rule):
    print("masked bounded %dx%d P=%d J=%d R=%d rule=%d" % (ny, nx, P, J, R, rule), flush=True)
    _, g1, g2 = S.shear_map(256, 130 + ny, 131 + nx)
    g1, g2 = np.ascontiguousarray(g1[:ny, :nx]), np.ascontiguousarray(g2[:ny, :nx])
    m = S.survey_mask(ny, nx, 17)
    seed, thr = 500 + ny, 2.0
    a1, a2 = O.mask_shear(g1, g2, m)
    kE_ref, _ = O.ks_invert_padded(a1, a2, P)
    planes_ref = O.starlet_forward_bc(kE_ref, J, rule)
    sig_ref = O.noise_sigma_bc(a1, a2, P, J, rule, R, seed)
    snr_ref = O.snr_planes(planes_ref, sig_ref)

    tm = torch.tensor(m, device="cuda")
    t1, t2 = ctx.mask_shear(dev(g1, torch.float32), dev(g2, torch.float32), tm)
    planes = ctx.starlet_forward_bc(ctx.ks_invert_padded(t1, t2, P)[0], J, rule)
    sigma, snr = ctx.noise_maps_bc(t1, t2, P, J, rule, R, seed, planes_signal=planes)
    counts = ctx.count_peaks_masked(snr, tm, thr, rule)
    torch.cuda.synchronize()
    tol = TOL[torch.float32] * rms(kE_ref)
    assert float(np.max(np.abs(planes.double().cpu().numpy() - planes_ref))) <= tol
    sg, sn = sigma.double().cpu().numpy(), snr.double().cpu().numpy()
    assert float(np.max(np.abs(sg - sig_ref))) <= tol
    assert np.all(np.abs(sn - snr_ref) * sig_ref <= tol * (1.0 + np.abs(snr_ref)) * (1 + 1e-6))
    # peaks: GPU planes counted by the oracle, oracle planes (in float32) by the GPU
    assert [int(v) for v in counts.cpu()] == O.count_peaks_masked_planes(snr.cpu().numpy(), thr, rule, m)
    snr32 = snr_ref.astype(np.float32)
    c2 = ctx.count_peaks_masked(dev(snr32, torch.float32), tm, thr, rule)
    assert [int(v) for v in c2.cpu()] == O.count_peaks_masked_planes(snr32, thr, rule, m)
    # the mask removes peaks that the unmasked count keeps
    assert sum(int(v) for v in ctx.count_peaks_bc(snr, thr, rule).cpu()) > sum(int(v) for v in counts.cpu())


def test_masked_periodic_map_through_the_path(ctx):
    # a power-of-two square: the masked shear goes through run_path, whose
    # S/N planes are counted with the mask under the periodic rule
    n, J, R, seed, thr = 256, 6, 6, 77, 2.0
    _, g1, g2 = S.shear_map(n, 31, 32)
    m = S.survey_mask(n, n, 33)
    a1, a2 = O.mask_shear(g1, g2, m)
    tm = torch.tensor(m, device="cuda")
    t1, t2 = ctx.mask_shear(dev(g1, torch.float32), dev(g2, torch.float32), tm)
    out = ctx.run_path(t1, t2, J, R, seed, thr)
    counts = ctx.count_peaks_masked(out["snr"], tm, thr, amap.BC_PERIODIC)
    torch.cuda.synchronize()
    kE, _ = O.ks_invert(a1, a2)
    tol = TOL[torch.float32] * rms(kE)
    assert float(np.max(np.abs(out["planes"].double().cpu().numpy() - O.starlet_forward(kE, J)))) <= tol
    assert float(np.max(np.abs(out["sigma"].double().cpu().numpy() - O.noise_sigma(a1, a2, J, R, seed)))) <= tol
    snr = out["snr"].cpu().numpy()
    assert [int(v) for v in counts.cpu()] == O.count_peaks_masked_planes(snr, thr, O.BC_PERIODIC, m)


def test_mask_calls_reject_bad_arguments(ctx):
    lib = amap.load()
    g = torch.zeros((2, 20, 32), device="cuda")
    o = torch.zeros((2, 20, 32), device="cuda")
    m = torch.ones((2, 20, 32), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    a, b, oa, ob = g[0].data_ptr(), g[1].data_ptr(), o[0].data_ptr(), o[1].data_ptr()

    def call(fn, *args):
        with pytest.raises(amap.AmapError):
            amap._check(fn(ctx._h, *args))

    # masked peaks: no mask, a misaligned mask
    call(lib.amap_count_peaks_masked, amap.F32, 20, 32, 1, 0, a, None, 0.0, cnt.data_ptr(), None)
    call(lib.amap_count_peaks_masked, amap.F32, 20, 32, 1, 0, a, m.data_ptr() + 1, 0.0,
         cnt.data_ptr(), None)
    # masked shear: both outputs in one buffer, an output on the other input,
    # a misaligned output, an empty field
    call(lib.amap_mask_shear, amap.F32, 20, 32, m.data_ptr(), a, b, oa, oa, None)
    call(lib.amap_mask_shear, amap.F32, 20, 32, m.data_ptr(), a, b, b, ob, None)
    call(lib.amap_mask_shear, amap.F32, 20, 32, m.data_ptr(), a, b, oa + 4, ob, None)
    call(lib.amap_mask_shear, amap.F32, 0, 32, m.data_ptr(), a, b, oa, ob, None)
    # valid: separate outputs, and in place
    amap._check(lib.amap_mask_shear(ctx._h, amap.F32, 20, 32, m.data_ptr(), a, b, oa, ob, None))
    amap._check(lib.amap_mask_shear(ctx._h, amap.F32, 20, 32, m.data_ptr(), a, b, a, b, None))
    torch.cuda.synchronize()
