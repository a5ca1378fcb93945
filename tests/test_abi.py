"""The C-ABI library loads and exports every symbol include/amap.h declares,
and the host-side validation rejects bad arguments before touching a device.
No compute call is made here (no GPU needed)."""
import ctypes
import os

import pytest

import paper_1204_4293_amd as amap


def test_library_is_built():
    assert os.path.exists(amap.LIB_PATH), "run __graft_entry__.build() first"


def test_every_header_symbol_is_exported():
    lib = ctypes.CDLL(amap.LIB_PATH)
    names = amap.header_symbols()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    lib = amap.load()
    for name in amap.header_symbols():
        fn = getattr(lib, name)
        assert fn.restype is not None or name == "amap_last_error"


def test_null_context_is_rejected_without_device():
    lib = amap.load()
    P = ctypes.c_void_p
    st = lib.amap_ks_invert(None, 0, 64, P(256), P(512), P(768), None, None)
    assert st == 1
    assert b"ctx" in lib.amap_last_error()
    st = lib.amap_starlet_forward(None, 0, 64, 3, P(256), P(512), None)
    assert st == 1
    st = lib.amap_batch_run(None, None)
    assert st == 1
    assert lib.amap_plan_destroy(None) == 0
    assert lib.amap_destroy(None) == 0


@pytest.mark.parametrize("n,J,ok", [(64, 4, True), (16, 4, True), (16, 5, False), (4096, 12, True),
                                    (8192, 7, False), (48, 3, False), (64, 1, False)])
def test_footprint_validates_sizes(n, J, ok):
    b = amap.job_footprint_bytes(amap.F32, n, J, 0)
    assert (b > 0) == ok
    if ok:
        # spectrum + kappa + scratch for the signal at least
        assert b >= 4 * n * n * 4
        assert amap.job_footprint_bytes(amap.F32, n, J, 32) > b
        assert amap.job_footprint_bytes(amap.F64, n, J, 0) > b


def test_create_without_device_reports_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = amap.load()
    h = ctypes.c_void_p()
    st = lib.amap_create(0, ctypes.byref(h))
    assert st != 0 and not h.value


def test_noise_batch_bounds():
    assert amap.noise_batch(1024, 256) == 128
    assert amap.noise_batch(1024, 40) == 40
    assert amap.noise_batch(4096, 32) == 8
    assert amap.noise_batch(64, 2) == 2
    assert amap.noise_batch(8192, 32) == 0
    assert amap.noise_batch(48, 32) == 0
    assert amap.noise_batch(64, 1) == 0
