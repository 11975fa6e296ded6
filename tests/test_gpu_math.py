"""Accuracy of the flux kernel's Newton-refined divide and rsqrt and of its
erf and exp (lskum_math.h) on the GPU, against numpy / scipy double
precision."""
import ctypes
import numpy as np
import pytest
import torch

from paper_2403_13287_amd import _build

pytestmark = pytest.mark.gpu

ULP = 2.0 ** -52


@pytest.fixture(scope="module")
def calib():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    lib = ctypes.CDLL(_build.CALIB_LIB)
    lib.lskum_calib_elementary.restype = ctypes.c_int
    lib.lskum_calib_elementary.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]

    def run(fn, x, y=None):
        xd = torch.from_numpy(np.ascontiguousarray(x, np.float64)).cuda()
        yd = torch.from_numpy(np.ascontiguousarray(y if y is not None else x, np.float64)).cuda()
        out = torch.empty_like(xd)
        rc = lib.lskum_calib_elementary(fn, xd.numel(), xd.data_ptr(), yd.data_ptr(),
                                        out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert rc == 0
        torch.cuda.synchronize()
        return out.cpu().numpy()

    return run


def test_div_and_rsqrt(calib):
    rng = np.random.Generator(np.random.PCG64(3))
    b = np.exp(rng.uniform(-30, 30, 200000))
    a = rng.normal(size=b.size) * np.exp(rng.uniform(-30, 30, b.size))
    got = calib(9, b, a)
    rel = np.abs(got - a / b) / np.abs(a / b)
    assert rel.max() <= 2 * ULP, rel.max()
    # one Newton step on the hardware reciprocal, no correction (the
    # limiter's quotient): the estimate's relative error e0 leaves e0^2
    # plus the rounding of three operations
    got = calib(13, b, a)
    rel = np.abs(got - a / b) / np.abs(a / b)
    assert rel.max() <= 16 * ULP, rel.max()
    x = np.exp(rng.uniform(-40, 40, 200000))
    got = calib(10, x)
    ref = 1.0 / np.sqrt(x)
    rel = np.abs(got - ref) / ref
    assert rel.max() <= 3 * ULP, rel.max()


def test_erf(calib):
    """lk_erf: its own polynomial for |x| < 1, the device library beyond;
    within 2 ulp of 1 (absolute) of scipy's erf everywhere, and within 3 ulp
    relative for |x| < 1, where erf(x) ~ 2x/sqrt(pi) may be tiny; odd."""
    from scipy.special import erf
    rng = np.random.Generator(np.random.PCG64(5))
    x = np.concatenate([rng.uniform(-1, 1, 200000), rng.uniform(-7, 7, 200000),
                        np.sign(rng.normal(size=20000)) * np.exp(rng.uniform(-700, 0, 20000)),
                        [0.0, -0.0, 1.0, -1.0, np.nextafter(1.0, 0.0), 6.0, 30.0, -30.0]])
    got = calib(11, x)
    ref = erf(x)
    assert np.max(np.abs(got - ref)) <= 2 * ULP
    small = np.abs(x) < 1
    nz = small & (ref != 0)
    rel = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
    assert rel.max() <= 3 * ULP, rel.max()
    assert np.array_equal(calib(11, -x), -got)
    assert np.all(np.isnan(calib(11, np.array([np.nan]))))


def test_exp(calib):
    """lk_exp within 2 ulp (relative) of numpy's exp over the whole finite
    range, 0 below the underflow threshold, +inf above the overflow one,
    NaN for NaN; exact at 0."""
    rng = np.random.Generator(np.random.PCG64(6))
    x = np.concatenate([rng.uniform(-1, 1, 100000), rng.uniform(-50, 5, 200000),
                        rng.uniform(-708, 709, 100000), [0.0, -0.0, 1.0, -1.0, 0.5, 700.0]])
    got = calib(12, x)
    ref = np.exp(x)
    rel = np.abs(got - ref) / ref
    assert rel.max() <= 2 * ULP, rel.max()
    assert calib(12, np.array([0.0]))[0] == 1.0
    edge = calib(12, np.array([-800.0, -1e10, 720.0, 1e10, np.nan]))
    assert edge[0] == 0.0 and edge[1] == 0.0
    assert np.isinf(edge[2]) and np.isinf(edge[3]) and edge[2] > 0
    assert np.isnan(edge[4])
