"""The entry point that allocates nothing (amap_ks_invert_noalloc): its
spectrum lives in the library's static scratch array, so it must give
exactly what amap_ks_invert gives (same kernels) and match the FP64 oracle
within 1e-5 * rms(kappa) (float32) / 1e-10 (float64), on consecutive calls
with a smaller map second, without the context growing any workspace."""
import numpy as np
import pytest
import torch

import oracle as O
import synth as S
import paper_1204_4293_amd as amap

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-10}


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_ks_invert_on_consecutive_calls(dtype):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ref_ctx, ctx = amap.Context(0), amap.Context(0)
    try:
        for n in (2048, 128):  # the second call smaller than the first
            print("ks_invert_noalloc n=%d %s" % (n, dtype), flush=True)
            _, g1, g2 = S.shear_map(n, 60 + n, 61 + n)
            t1, t2 = dev(g1, dtype), dev(g2, dtype)
            e = torch.full((n, n), float("nan"), dtype=dtype, device="cuda")
            b = torch.full((n, n), float("nan"), dtype=dtype, device="cuda")
            ctx.ks_invert_noalloc(t1, t2, e, b)
            er, br = ref_ctx.ks_invert(t1, t2, want_b=True)
            torch.cuda.synchronize()
            assert torch.equal(e, er) and torch.equal(b, br)
            kE, kB = O.ks_invert(g1, g2)
            tol = TOL[dtype] * float(np.sqrt(np.mean(kE ** 2)))
            assert np.max(np.abs(e.double().cpu().numpy() - kE)) <= tol
            assert np.max(np.abs(b.double().cpu().numpy() - kB)) <= tol
        assert ctx.workspace_bytes() == 0  # nothing was allocated for it
    finally:
        ctx.close()
        ref_ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    ctx = amap.Context(0)
    try:
        t = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda")
        out = torch.empty_like(t)
        with pytest.raises(amap.AmapError) as err:
            ctx.ks_invert_noalloc(t, t.clone(), out)
        assert err.value.status == 1 and "scratch" in str(err.value)
        assert ctx.workspace_bytes() == 0
    finally:
        ctx.close()
