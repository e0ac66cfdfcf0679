"""The device-rate microbenchmarks (include/clmap_calib.h) through the C-ABI:
the copy reproduces its source byte for byte (including a size that is not a
multiple of the grid's stride), the reported work is what the header states,
and the rates are finite and below the device's published peaks."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def clm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2202_06427_amd as clm
    return clm


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, 64 << 20])
def test_copy_is_exact(clm, nbytes):
    from paper_2202_06427_amd import _lib as L
    g = np.random.default_rng(nbytes)
    src = torch.from_numpy(g.integers(0, 256, size=nbytes, dtype=np.uint8)).to("cuda:0")
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda:0")
    ms, work = ctypes.c_double(0.0), ctypes.c_double(0.0)
    ctx = clm._context(torch.device("cuda:0"))
    L.check(L.lib().clm_calibrate(ctx, 2, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  nbytes, 2, ctypes.byref(ms), ctypes.byref(work)))
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert work.value == 2.0 * nbytes and ms.value > 0.0


def test_rates_are_plausible(clm):
    _, w32, r32 = clm.calibrate("fma_f32", reps=2)
    _, w64, r64 = clm.calibrate("fma_f64", reps=2)
    _, wc, rc = clm.calibrate("copy", nbytes=256 << 20, reps=2)
    assert w32 == w64 == 2.0 * 8 * 8192 * 4096 * 256
    assert wc == 2.0 * (256 << 20)
    assert 1.0 < r32 < 157.3 and 1.0 < r64 < 78.6 * 1.05   # TFLOP/s
    assert 100.0 < rc < 8000.0                              # GB/s


def test_rejects_bad_arguments(clm):
    from paper_2202_06427_amd import _lib as L
    ctx = clm._context(torch.device("cuda:0"))
    buf = torch.empty(64, dtype=torch.uint8, device="cuda:0")
    ms, work = ctypes.c_double(0.0), ctypes.c_double(0.0)
    p = ctypes.c_void_p(buf.data_ptr())
    # copy size not a multiple of 16, overlapping buffers, FMA scratch too small
    assert L.lib().clm_calibrate(ctx, 2, p, ctypes.c_void_p(buf.data_ptr() + 32), 24, 1,
                                 ctypes.byref(ms), ctypes.byref(work)) == L.STATUS_CODES["CLM_E_INVALID_ARG"]
    assert L.lib().clm_calibrate(ctx, 2, p, ctypes.c_void_p(buf.data_ptr() + 16), 32, 1,
                                 ctypes.byref(ms), ctypes.byref(work)) == L.STATUS_CODES["CLM_E_INVALID_ARG"]
    assert L.lib().clm_calibrate(ctx, 0, None, p, 64, 1,
                                 ctypes.byref(ms), ctypes.byref(work)) == L.STATUS_CODES["CLM_E_WORKSPACE"]
