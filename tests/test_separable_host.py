"""Separable-kernel detection (tc_conv_kernel_rank1) on the host: outer
products are recognised with factors that reproduce the kernel, anything else
is refused.  No GPU needed."""
import ctypes as C

import numpy as np
import pytest

from paper_1612_08825_amd import _lib as L

TOL = 2.0 ** -20


@pytest.fixture(scope="module")
def api():
    L.load()
    from paper_1612_08825_amd import api

    return api


def gaussian(K, sigma):
    t = np.arange(K) - (K - 1) / 2
    g = np.exp(-t * t / (2 * sigma * sigma))
    return g / g.sum()


@pytest.mark.parametrize("k", [
    np.outer(gaussian(15, 2.5), gaussian(15, 2.5)),
    np.outer(gaussian(7, 1.0), gaussian(7, 3.0)),
    np.full((5, 5), 1.0 / 25),
    np.outer([1.0, 2.0, 1.0], [-1.0, 0.0, 1.0]),       # a Sobel derivative
    np.outer([-0.5, 0.5], [0.5, 0.5]),                   # the 2x2 first difference
    np.outer(np.arange(1.0, 10.0), -np.arange(9.0, 0.0, -1.0)),
])
def test_outer_products_are_detected(api, k):
    kf = k.astype(np.float32)
    ok, u, v = api.conv_kernel_rank1(kf, TOL)
    assert ok
    rec = np.outer(u.astype(np.float64), v.astype(np.float64))
    assert np.max(np.abs(rec - kf)) <= TOL * np.max(np.abs(kf))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_general_kernels_are_refused(api, seed):
    rng = np.random.default_rng(seed)
    k = rng.standard_normal((7, 7)).astype(np.float32)
    assert not api.conv_kernel_rank1(k, TOL)[0]
    # rank one plus a perturbation well above the tolerance
    g = np.outer(gaussian(9, 2.0), gaussian(9, 2.0))
    g[4, 5] += 1e-3 * g.max()
    assert not api.conv_kernel_rank1(g.astype(np.float32), TOL)[0]


def test_zero_and_nonfinite(api):
    ok, u, v = api.conv_kernel_rank1(np.zeros((3, 3), np.float32))
    assert ok and not u.any() and not v.any()
    k = np.ones((3, 3), np.float32)
    k[1, 1] = np.nan
    assert not api.conv_kernel_rank1(k)[0]
    k[1, 1] = np.inf
    assert not api.conv_kernel_rank1(k)[0]


def test_bad_arguments(api):
    lib = L.load()
    fp = C.POINTER(C.c_float)
    buf = (C.c_float * 9)()
    assert lib.tc_conv_kernel_rank1(None, 3, 3, TOL, buf, buf) == L.TC_EINVAL
    assert lib.tc_conv_kernel_rank1(buf, 0, 3, TOL, buf, buf) == L.TC_EINVAL
    assert lib.tc_conv_kernel_rank1(buf, 3, 3, -1.0, buf, buf) == L.TC_EINVAL
    assert lib.tc_conv_kernel_rank1(C.cast(buf, fp), 3, 3, TOL, None, buf) == L.TC_EINVAL
