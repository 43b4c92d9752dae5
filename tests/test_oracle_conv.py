"""Pins of the convolution oracle against things other than itself:
brute force, numpy/scipy library routines, hand-worked values, and identities
of the convolution (delta, commutativity, sum, ramp derivative, separability,
flip = correlation)."""
import json
import os

import numpy as np
import pytest
import scipy.signal

import oracle as O
from paper_1612_08825_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_1d_example():
    g = json.load(open(os.path.join(GOLDEN, "conv_1d_worked.json")))
    x = np.array(g["x"], dtype=np.float64)
    k = np.array(g["k"], dtype=np.float64)
    np.testing.assert_array_equal(O.conv(x, k, "full"), g["expected_full"])
    np.testing.assert_array_equal(O.conv(x, k, "same"), g["expected_same"])
    np.testing.assert_array_equal(O.conv(x, k, "valid"), g["expected_valid"])


@pytest.mark.parametrize("xs,ks", [((7,), (3,)), ((6, 7), (3, 2)), ((4, 5, 3), (2, 2, 2)), ((2, 3), (4, 5)),
                                   ((5,), (5,)), ((1, 1), (3, 3))])
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_bruteforce_int_exact(xs, ks, mode):
    rng = np.random.default_rng(0)
    x = rng.integers(0, 256, xs).astype(np.uint8)
    k = rng.integers(-8, 9, ks).astype(np.int32)
    if mode == "valid":
        try:
            O.conv_out_shape(xs, ks, mode)
        except ValueError:
            pytest.skip("mixed extents are rejected in valid mode")
    y = O.conv(x, k, mode)
    b = O.conv_bruteforce(x, k, mode)
    assert y.shape == b.shape
    assert all(int(a) == int(c) for a, c in zip(y.ravel(), b.ravel()))


@pytest.mark.parametrize("xs,ks", [((6, 7), (3, 2)), ((4, 5, 3), (2, 2, 2)), ((9,), (4,))])
def test_bruteforce_float(xs, ks):
    rng = np.random.default_rng(1)
    x = rng.random(xs).astype(np.float32)
    k = rng.standard_normal(ks).astype(np.float32)
    for mode in ("full", "same", "valid"):
        y = O.conv(x, k, mode)
        b = O.conv_bruteforce(x, k, mode).astype(np.float64)
        np.testing.assert_allclose(y, b, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n,m", [(10, 3), (3, 10), (17, 17), (1, 5), (64, 15)])
def test_numpy_convolve_1d(n, m):
    rng = np.random.default_rng(2)
    x = rng.random(n)
    k = rng.standard_normal(m)
    for mode in ("full", "same", "valid"):
        ref = np.convolve(x, k, mode)
        if mode == "same" and m > n:
            # numpy's 'same' has the length of the longer input; ours keeps x's extent
            ref = scipy.signal.convolve(x, k, mode="same", method="direct")
        np.testing.assert_allclose(O.conv(x, k, mode), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("xs,ks", [((33, 40), (3, 3)), ((21, 19), (7, 7)), ((30, 31), (15, 15)),
                                   ((6, 9, 8), (3, 3, 3)), ((5, 4, 3, 6), (2, 3, 2, 2)), ((3, 4), (7, 9))])
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_scipy_direct_nd(xs, ks, mode):
    rng = np.random.default_rng(3)
    x = rng.random(xs)
    k = rng.standard_normal(ks)
    ref = scipy.signal.convolve(x, k, mode=mode, method="direct")
    np.testing.assert_allclose(O.conv(x, k, mode), ref, rtol=1e-11, atol=1e-11)


def test_delta_kernel():
    x = synth.conv_image((13, 17), case=5)
    d = np.zeros((1, 1), np.float32)
    d[0, 0] = 1
    np.testing.assert_array_equal(O.conv(x, d, "full"), x.astype(np.float64))
    # a delta at (2, 3) shifts x by (2, 3) in full mode
    d = np.zeros((4, 5), np.float32)
    d[2, 3] = 1
    y = O.conv(x, d, "full")
    assert y.shape == (16, 21)
    np.testing.assert_array_equal(y[2:15, 3:20], x.astype(np.float64))
    assert np.count_nonzero(y) == np.count_nonzero(x)


def test_commutative_full_int():
    x = synth.conv_image((9, 11), dtype="u8")
    k = synth.conv_kernel((4, 3), dtype="i32")
    a = O.conv(x, k, "full")
    b = O.conv(k, x, "full")
    assert a.dtype == np.int64
    np.testing.assert_array_equal(a, b)


def test_sum_identity_int():
    x = synth.conv_image((23, 19), dtype="u8", case=2)
    k = synth.conv_kernel((5, 5), dtype="i32", case=2)
    y = O.conv(x, k, "full")
    assert int(y.sum()) == int(x.astype(np.int64).sum()) * int(k.astype(np.int64).sum())


def test_ramp_derivative():
    a, b = 3.0, -2.0
    i, j = np.meshgrid(np.arange(12), np.arange(14), indexing="ij")
    x = a * i + b * j + 7.0
    kx = 0.5 * np.array([[-1.0, 1.0], [-1.0, 1.0]])  # the paper's E_x kernel (a correlation mask)
    ky = kx.T
    gx = O.conv(x, kx[::-1, ::-1], "valid")  # convolution with the flipped mask = the mask's correlation
    gy = O.conv(x, ky[::-1, ::-1], "valid")
    np.testing.assert_array_equal(gx, np.full((11, 13), b))
    np.testing.assert_array_equal(gy, np.full((11, 13), a))


def test_separable_equals_two_passes():
    rng = np.random.default_rng(4)
    x = rng.random((20, 25))
    u = rng.standard_normal(5)
    v = rng.standard_normal(3)
    k = np.outer(u, v)
    two = O.conv(O.conv(x, u[:, None], "full"), v[None, :], "full")
    np.testing.assert_allclose(O.conv(x, k, "full"), two, rtol=1e-12, atol=1e-12)


def test_flip_is_correlation():
    rng = np.random.default_rng(5)
    x = rng.random((15, 16, 4))
    k = rng.standard_normal((3, 4, 2))
    ref = scipy.signal.correlate(x, k, mode="full", method="direct")
    np.testing.assert_allclose(O.conv(x, k[::-1, ::-1, ::-1], "full"), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv_at_matches_conv(mode):
    x = synth.conv_image((31, 29), case=7)
    k = synth.conv_kernel((7, 5), case=7)
    y = O.conv(x, k, mode)
    rng = np.random.default_rng(6)
    idx = [tuple(int(rng.integers(e)) for e in y.shape) for _ in range(40)]
    idx += [(0, 0), tuple(e - 1 for e in y.shape)]
    at = O.conv_at(x, k, mode, idx)
    np.testing.assert_allclose(at, [y[t] for t in idx], rtol=1e-13, atol=1e-13)
    xi = synth.conv_image((31, 29), dtype="u8")
    ki = synth.conv_kernel((7, 5), dtype="i32")
    yi = O.conv(xi, ki, mode)
    np.testing.assert_array_equal(O.conv_at(xi, ki, mode, idx), [yi[t] for t in idx])


def test_empty_and_mixed_valid():
    assert O.conv(np.zeros((0, 4)), np.ones((2, 2)), "full").shape == (1, 5)
    with pytest.raises(ValueError):
        O.conv_out_shape((5, 3), (3, 5), "valid")
    assert O.conv_out_shape((3, 4), (5, 6), "valid") == (3, 3)
