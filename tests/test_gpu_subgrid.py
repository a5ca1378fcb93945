"""The final noise stage on whole sub-grids (scales from j0 on, run on the
periodic m x m sub-grids of pixels congruent mod 2^(j0-1), m <= 64).

The schedule is forced with autotune mode 2 (the analytic planner ending in
a sub-grid stage) and checked against the FP64 oracle at 1e-5 * rms(kappa)
(float32) or 1e-10 (float64), and against the tile-only analytic schedule:
both run the same B3 cascade on the same coarse planes, so sigma differs
only in how per-group partial statistics are merged.
"""
import numpy as np
import pytest
import torch

import oracle as O
import oracle_pool
import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-10}


@pytest.fixture(scope="module")
def ctxs():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    sub, tile = amap.Context(0), amap.Context(0)
    sub.set_autotune(2)
    tile.set_autotune(False)
    yield sub, tile
    sub.close()
    tile.close()


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def rms(a):
    return float(np.sqrt(np.mean(np.asarray(a, dtype=np.float64) ** 2)))


# (n, J, R, dtype, first scale of the sub-grid stage)
CASES = [(1024, 7, 18, torch.float32, 5), (1024, 10, 3, torch.float32, 6),
         (512, 7, 5, torch.float32, 4), (256, 6, 6, torch.float32, 3),
         (64, 4, 8, torch.float32, 1), (128, 5, 4, torch.float64, 3),
         (64, 5, 3, torch.float64, 2), (2048, 9, 3, torch.float32, 6)]


@pytest.mark.parametrize("n,J,R,dtype,j0", CASES)
def test_subgrid_stage_against_oracle_and_tiles(ctxs, n, J, R, dtype, j0):
    sub, tile = ctxs
    print("sub-grid stage n=%d J=%d R=%d %s" % (n, J, R, dtype), flush=True)
    seed = 90 + n + J
    _, g1, g2 = S.shear_map(n, 7 + n, 8 + n)
    t1, t2 = dev(g1, dtype), dev(g2, dtype)
    sa, _ = sub.noise_maps(t1, t2, J, R, seed, want_snr=False)
    sb, _ = tile.noise_maps(t1, t2, J, R, seed, want_snr=False)
    torch.cuda.synchronize()
    stages = [p["stages"] for p in sub.plans() if p["mode"] == 2 and p["noise"] and p["logn"] == n.bit_length() - 1
              and p["J"] == J]
    assert stages and stages[0][-1][5] == 1 and stages[0][-1][0] == j0, stages
    a, b = sa.double().cpu().numpy(), sb.double().cpu().numpy()
    scale = float(np.abs(b).max())
    assert float(np.abs(a - b).max()) <= (1e-6 if dtype == torch.float32 else 1e-12) * scale
    kE, _ = O.ks_invert(g1, g2)
    ref = oracle_pool.noise_sigma_pool(g1, g2, J, R, seed)
    assert float(np.abs(a - ref).max()) <= TOL[dtype] * rms(kE)


def test_subgrid_path_snr_and_peaks_match_oracle(ctxs):
    # the whole path through the sub-grid schedule: S/N from the oracle's
    # sigma within the propagated tolerance, peaks bit-exact on the same planes
    sub, _ = ctxs
    n, J, R, seed = 256, 6, 7, 31
    _, g1, g2 = S.shear_map(n, 41, 42)
    out = sub.run_path(dev(g1, torch.float32), dev(g2, torch.float32), J, R, seed, 2.0)
    torch.cuda.synchronize()
    kE, _ = O.ks_invert(g1, g2)
    planes_ref = O.starlet_forward(kE, J)
    sig_ref = O.noise_sigma(g1, g2, J, R, seed)
    snr_ref = O.snr_planes(planes_ref, sig_ref)
    tol = 1e-5 * rms(kE)
    sn = out["snr"].double().cpu().numpy()
    assert np.all(np.abs(sn - snr_ref) * sig_ref <= tol * (1.0 + np.abs(snr_ref)) * (1 + 1e-6))
    got = [int(v) for v in out["peaks"].cpu()]
    assert got == O.count_peaks_planes(out["snr"].cpu().numpy(), 2.0)


def test_autotune_mode_is_validated(ctxs):
    sub, _ = ctxs
    with pytest.raises(amap.AmapError):
        sub.set_autotune(3)
    sub.set_autotune(2)
