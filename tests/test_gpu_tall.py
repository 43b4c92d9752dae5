"""Images taller than the grid's y extent (65535): the kernels that take one
grid row per image row (or per tile of rows) loop over the rest; the results
are checked against the oracle on every row or on sampled outputs."""
import numpy as np
import pytest
import torch

import oracle as O
from test_gpu_variant import check_variant

pytestmark = pytest.mark.gpu

TALL = 70001


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def test_tall_pyramid_and_derivatives(api):
    rng = np.random.default_rng(1)
    a = rng.integers(0, 256, (2 * TALL, 6), dtype=np.uint8)
    b = rng.integers(0, 256, (2 * TALL, 6), dtype=np.uint8)
    lv = api.image_pyramid(torch.from_numpy(a).cuda(), 2)
    ex, ey, et = api.horn_derivs(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), exact_int=True)
    torch.cuda.synchronize()
    assert np.array_equal(lv[0].cpu().numpy(), O.reduce2(a))
    nx, ny, nt = O.horn_numerators(a, b)
    assert np.array_equal(ex.cpu().numpy(), nx) and np.array_equal(ey.cpu().numpy(), ny)
    assert np.array_equal(et.cpu().numpy(), nt)


@pytest.mark.parametrize("W", [8, 7])  # the vector and the any-stride gradient kernels
def test_tall_gradient(api, W):
    rng = np.random.default_rng(W)
    img = rng.integers(0, 256, (4 * TALL, W), dtype=np.uint8)
    g = api.gradient(torch.from_numpy(img).cuda(), "sobel3")
    torch.cuda.synchronize()
    ref = O.gradient(img.astype(np.float64), "sobel3")
    assert np.array_equal(g["ex"].cpu().numpy(), ref["ex"]) and np.array_equal(g["ey"].cpu().numpy(), ref["ey"])


def test_tall_lowpass_variant(api):
    # level 1 of a 2 x 65537-row image has 65537 rows: the low-pass kernel loops
    rng = np.random.default_rng(3)
    f = rng.integers(0, 256, (2, 2 * 65537, 8), dtype=np.uint8)
    fr = torch.from_numpy(f).cuda()
    lv, pk = api.ttc_solve_variant(fr[0], fr[1], 2, "sobel3", "binomial3")
    torch.cuda.synchronize()
    check_variant(api.decode_levels(lv), api.decode_picks(pk)[0], f[0], f[1], 2, "sobel3", "binomial3", "tall")


def test_tall_tiled_convolution(api):
    # 65535 row tiles of 64 rows end at row 4,194,240: sample outputs past it
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (4_200_000, 12)).astype(np.float32)
    k = rng.normal(0, 1, (3, 17)).astype(np.float32)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "full")
    torch.cuda.synchronize()
    idx = [(0, 0), (1000, 10), (4_194_239, 5), (4_194_240, 20), (4_199_999, 27), (4_200_001, 3), (4_196_000, 16)]
    got = y.cpu().numpy()
    want = O.conv_at(x, k, "full", idx)
    bnd = O.conv_at(np.abs(x), np.abs(k), "full", idx)
    for (i, j), w, b in zip(idx, want, bnd):
        assert abs(float(got[i, j]) - float(w)) <= 1e-5 * float(b), (i, j)
