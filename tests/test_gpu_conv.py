"""GPU parity of tc_conv_nd against the FP64 / exact-integer oracle.

Integer convolutions must match exactly; float ones within
|y - y64| <= 1e-5 * (|x| (*) |k|) element-wise and 1e-5 norm-wise.  Shapes span
several 64x64 output tiles with ragged tails, kernels larger than the image,
strided views, every mode, ranks 1-4, and the full benchmark sizes (checked on
sampled outputs the oracle computes one at a time)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_08825_amd import synth
from tolerance import TAU_CONV, conv_bound

pytestmark = pytest.mark.gpu

MAXERR = {}


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def _check_float(y, x, k, mode, tag):
    ref = O.conv(x, k, mode)
    bound = conv_bound(x, k, mode)
    err = np.abs(y.astype(np.float64) - ref)
    rel = float((err / np.maximum(bound / TAU_CONV, 1e-300)).max()) if err.size else 0.0
    MAXERR[tag] = rel
    print(f"[conv {tag}] max |err| / sum|x||k| = {rel:.3e}", flush=True)
    assert np.all(err <= bound + 1e-30)
    if ref.size:
        assert err.max() <= TAU_CONV * max(np.abs(ref).max(), 1e-30)


SHAPES_2D = [((70, 130), (3, 3)), ((129, 65), (7, 7)), ((100, 77), (15, 15)), ((5, 6), (9, 11)),
             ((64, 64), (1, 1)), ((1, 200), (1, 5)), ((67, 67), (2, 5)), ((40, 33), (16, 16)), ((33, 19), (20, 3)),
             # several bands and 256-column waves with ragged tails (interior items take the unchecked path)
             ((61, 777), (3, 3)), ((45, 600), (2, 2)), ((37, 530), (5, 5)), ((29, 1100), (7, 7)), ((3, 5), (5, 5)),
             ((70, 560), (15, 15)), ((9, 300), (15, 15)),
             # the 32-wide tiled kernel (kernel rows of 17..32 taps)
             ((150, 140), (23, 23)), ((80, 200), (17, 31)), ((70, 66), (64, 32)), ((20, 25), (31, 31)),
             # the 48- and 64-wide tiled kernels (rows of 33..64 taps, up to 64 rows)
             ((90, 150), (47, 47)), ((40, 300), (48, 64)), ((66, 70), (33, 40)), ((100, 90), (64, 48)),
             ((100, 90), (64, 64)), ((70, 80), (63, 57))]


@pytest.mark.parametrize("xs,ks", SHAPES_2D)
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv2d_f32(api, xs, ks, mode):
    try:
        O.conv_out_shape(xs, ks, mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    x = synth.conv_image(xs, case=1)
    k = synth.conv_kernel(ks, case=1)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
    _check_float(y, x, k, mode, f"f32 {xs}*{ks} {mode}")


@pytest.mark.parametrize("xs,ks", SHAPES_2D[:5] + SHAPES_2D[-8:-6] + SHAPES_2D[-4:-3])
@pytest.mark.parametrize("mode", ["full", "valid"])
def test_conv2d_u8_exact(api, xs, ks, mode):
    try:
        O.conv_out_shape(xs, ks, mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    x = synth.conv_image(xs, case=2, dtype="u8")
    k = synth.conv_kernel(ks, case=2, dtype="i32")
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
    assert y.dtype == np.int32
    np.testing.assert_array_equal(y.astype(np.int64), O.conv(x, k, mode))


@pytest.mark.parametrize("xs,ks", [((130, 140), (95, 80)), ((40, 50), (65, 70)), ((70, 300), (20, 129)),
                                   ((4, 80, 90), (2, 66, 70)), ((10, 12), (3, 260))])
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv_kernel_blocks(api, xs, ks, mode):
    """Kernels over 64 taps along a row or column run as 64 x 64 blocks of the
    tiled kernel, the first writing the output and the rest adding to it (a
    kernel over 256 taps takes the generic kernel): FP32 within the bound, u8 *
    i32 bit for bit."""
    try:
        O.conv_out_shape(xs, ks, mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    x = synth.conv_image(xs, case=6)
    k = synth.conv_kernel(ks, case=6)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
    _check_float(y, x, k, mode, f"blocks {xs}*{ks} {mode}")
    xu = synth.conv_image(xs, case=6, dtype="u8")
    ku = synth.conv_kernel(ks, case=6, dtype="i32")
    yu = api.conv_nd(torch.from_numpy(xu).cuda(), torch.from_numpy(ku).cuda(), mode).cpu().numpy()
    np.testing.assert_array_equal(yu.astype(np.int64), O.conv(xu, ku, mode))


def test_conv2d_f16_input(api):
    x = synth.conv_image((90, 75), case=3, dtype="f16")
    k = synth.conv_kernel((5, 5), case=3)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "same").cpu().numpy()
    _check_float(y, x, k, "same", "f16 90x75*5x5")


def test_conv_strided_views(api):
    base = synth.conv_image((150, 140), case=4)
    xg = torch.from_numpy(base).cuda()[3::2, 5:128]  # row stride 280, column slice
    x = base[3::2, 5:128]
    k = synth.conv_kernel((3, 4), case=4)
    kg = torch.from_numpy(k).cuda()
    big = torch.full((200, 200), -7.0, device="cuda")
    out = big[10:10 + x.shape[0] + 2, 20:20 + x.shape[1] + 3]
    api.conv_nd(xg, kg, "full", out=out)
    _check_float(out.cpu().numpy(), x, k, "full", "strided")
    assert float(big[0, 0]) == -7.0 and float(big[199, 199]) == -7.0  # nothing written outside the view


@pytest.mark.parametrize("xs,ks", [((9, 70, 66), (3, 3, 3)), ((3, 5, 4), (4, 6, 5)), ((6, 31, 29), (2, 7, 1)),
                                   ((5, 21, 600), (3, 3, 3)), ((4, 19, 300), (2, 5, 5))])
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv3d(api, xs, ks, mode):
    try:
        O.conv_out_shape(xs, ks, mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    x = synth.conv_image(xs, case=5)
    k = synth.conv_kernel(ks, case=5)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
    _check_float(y, x, k, mode, f"3d {xs}*{ks} {mode}")
    xu = synth.conv_image(xs, case=5, dtype="u8")
    ku = synth.conv_kernel(ks, case=5, dtype="i32")
    yu = api.conv_nd(torch.from_numpy(xu).cuda(), torch.from_numpy(ku).cuda(), mode).cpu().numpy()
    np.testing.assert_array_equal(yu.astype(np.int64), O.conv(xu, ku, mode))


@pytest.mark.parametrize("xs,ks", [((1000,), (7,)), ((5,), (9,)), ((4, 5, 6, 7), (2, 3, 2, 3)), ((3, 2, 2, 2, 3), (2, 2, 1, 2, 2))])
def test_conv_other_ranks(api, xs, ks):
    for mode in ("full", "same"):
        x = synth.conv_image(xs, case=6)
        k = synth.conv_kernel(ks, case=6)
        y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
        _check_float(y, x, k, mode, f"rank{len(xs)} {xs} {mode}")
        xu = synth.conv_image(xs, case=6, dtype="u8")
        ku = synth.conv_kernel(ks, case=6, dtype="i32")
        yu = api.conv_nd(torch.from_numpy(xu).cuda(), torch.from_numpy(ku).cuda(), mode).cpu().numpy()
        np.testing.assert_array_equal(yu.astype(np.int64), O.conv(xu, ku, mode))


def test_conv_int_bounds(api):
    from paper_1612_08825_amd import _lib as L

    x = torch.from_numpy(synth.conv_image((20, 20), dtype="u8")).cuda()
    k = torch.zeros((3, 3), dtype=torch.int32)
    k[1, 1] = 8421504  # 255 * 8421504 = 2147483520 <= 2^31 - 1, beyond the 24-bit multiply
    y = api.conv_nd(x, k.cuda(), "same").cpu().numpy()
    np.testing.assert_array_equal(y.astype(np.int64), O.conv(x.cpu().numpy(), k.numpy(), "same"))
    k[0, 0] = 1
    with pytest.raises(L.TTCError) as e:
        api.conv_nd(x, k.cuda(), "same")
    assert e.value.code == L.TC_EOVERFLOW


def _sample_index(shape, n, rng):
    idx = [tuple(int(rng.integers(e)) for e in shape) for _ in range(n)]
    corners = [tuple(c) for c in np.ndindex(*(2,) * len(shape))]
    idx += [tuple(0 if b == 0 else e - 1 for b, e in zip(c, shape)) for c in corners]
    idx += [tuple(min(7, e - 1) if d == 0 else e // 2 for d, e in enumerate(shape))]
    return idx


@pytest.mark.parametrize("N", [1024, 2048, 4096])
@pytest.mark.parametrize("K", [3, 7, 15])
def test_conv_benchmark_sizes_sampled(api, N, K):
    x = synth.conv_image((N, N), case=100 + N)
    k = synth.conv_kernel((K, K), case=100 + K)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "full")
    assert tuple(y.shape) == (N + K - 1, N + K - 1)
    rng = np.random.default_rng(N * K)
    idx = _sample_index(tuple(y.shape), 400, rng)
    got = y.cpu().numpy()[tuple(np.array(idx).T)]
    ref = O.conv_at(x, k, "full", idx)
    bound = TAU_CONV * O.conv_at(np.abs(x.astype(np.float64)), np.abs(k.astype(np.float64)), "full", idx)
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16"])
def test_conv3d_rolling_runs(api, dtype):
    """3 x 3 x 3 kernels over enough planes that a wave walks a run of several
    output planes (each input plane loaded once and added into the three
    output planes it feeds); the last run of each mode is shorter than the
    others.  Every output element against the oracle."""
    xs, ks = (100, 130, 300), (3, 3, 3)
    x = synth.conv_image(xs, case=36, dtype=dtype)
    for mode in ("full", "same", "valid"):
        if dtype == "u8":
            k = synth.conv_kernel(ks, case=36, dtype="i32")
            y = api.conv_nd_ex(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode, k_host=k).cpu().numpy()
            np.testing.assert_array_equal(y.astype(np.int64), O.conv(x, k, mode))
        else:
            k = synth.conv_kernel(ks, case=36)
            y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
            _check_float(y, x, k, mode, f"{dtype} 3d runs {mode}")


def test_conv3d_benchmark_size_sampled(api):
    x = synth.conv_image((64, 256, 256), case=300)
    k = synth.conv_kernel((3, 3, 3), case=300)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "full")
    assert tuple(y.shape) == (66, 258, 258)
    rng = np.random.default_rng(3)
    idx = _sample_index(tuple(y.shape), 400, rng)
    got = y.cpu().numpy()[tuple(np.array(idx).T)]
    ref = O.conv_at(x, k, "full", idx)
    bound = TAU_CONV * O.conv_at(np.abs(x.astype(np.float64)), np.abs(k.astype(np.float64)), "full", idx)
    assert np.all(np.abs(got - ref) <= bound)


def test_conv_u8_benchmark_size_sampled(api):
    x = synth.conv_image((2048, 2048), case=400, dtype="u8")
    k = synth.conv_kernel((7, 7), case=400, dtype="i32")
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "full").cpu().numpy()
    rng = np.random.default_rng(4)
    idx = _sample_index(y.shape, 1000, rng)
    np.testing.assert_array_equal(y[tuple(np.array(idx).T)].astype(np.int64), O.conv_at(x, k, "full", idx))


# ----------------------------------------------------------------------------- separable kernels
def _gauss(K, sigma):
    t = np.arange(K) - (K - 1) / 2
    g = np.exp(-t * t / (2 * sigma * sigma))
    return (g / g.sum()).astype(np.float32)


@pytest.mark.parametrize("K", [3, 5, 7, 9, 11, 15])
@pytest.mark.parametrize("xs", [(70, 600), (37, 261), (9, 40)])
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv2d_separable(api, K, xs, mode):
    """The fused two-pass kernel against the oracle's direct convolution with
    the outer product of the two FP32 factors (formed in FP64)."""
    try:
        O.conv_out_shape(xs, (K, K), mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    rng = np.random.default_rng([K, xs[0], xs[1]])
    u = rng.standard_normal(K).astype(np.float32)
    v = rng.standard_normal(K).astype(np.float32)
    x = synth.conv_image(xs, case=3)
    y = api.conv_nd_separable(torch.from_numpy(x).cuda(), torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(),
                              mode).cpu().numpy()
    k64 = np.outer(u.astype(np.float64), v.astype(np.float64))
    _check_float(y, x, k64, mode, f"sep K{K} {xs} {mode}")


def test_conv_auto_detects_separable(api):
    x = synth.conv_image((200, 530), case=4)
    g = np.outer(_gauss(15, 2.5), _gauss(15, 2.5)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y_auto = api.conv_nd_auto(xt, torch.from_numpy(g).cuda(), "same").cpu().numpy()
    _check_float(y_auto, x, g.astype(np.float64), "same", "auto gaussian 15")
    # a general kernel falls back to the direct path: bitwise what conv_nd gives
    k = synth.conv_kernel((7, 7), case=4)
    kt = torch.from_numpy(k).cuda()
    assert torch.equal(api.conv_nd_auto(xt, kt, "full"), api.conv_nd(xt, kt, "full"))


def test_conv_separable_rejects(api):
    from paper_1612_08825_amd import _lib as L

    x = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    u = torch.zeros(4, dtype=torch.float32, device="cuda")
    with pytest.raises(L.TTCError):
        api.conv_nd_separable(x, u, u, "full")           # K = 4 is not built
    u5 = torch.zeros(5, dtype=torch.float32, device="cuda")
    with pytest.raises(L.TTCError):
        api.conv_nd_separable(x.t(), u5, u5, "full")      # rows not contiguous


# ----------------------------------------------------------------------------- row kernels for u8 and f16 images
ROW_SHAPES = [((70, 130), (3, 3)), ((61, 777), (3, 3)), ((45, 601), (2, 2)), ((37, 530), (5, 5)), ((29, 1101), (7, 7)),
              ((9, 300), (7, 7)), ((3, 5), (5, 5)), ((130, 255), (3, 3))]


@pytest.mark.parametrize("xs,ks", ROW_SHAPES)
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv2d_rows_u8_exact(api, xs, ks, mode):
    """u8 (*) int32 through the row-streaming kernel: bit-exact."""
    try:
        O.conv_out_shape(xs, ks, mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    x = synth.conv_image(xs, case=31, dtype="u8")
    k = synth.conv_kernel(ks, case=31, dtype="i32", int_range=100)
    y = api.conv_nd_ex(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode, method="direct",
                       k_host=k).cpu().numpy()
    np.testing.assert_array_equal(y.astype(np.int64), O.conv(x, k, mode))


@pytest.mark.parametrize("xs,ks", ROW_SHAPES)
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_conv2d_rows_f16(api, xs, ks, mode):
    try:
        O.conv_out_shape(xs, ks, mode)
    except ValueError:
        pytest.skip("mixed extents are rejected in valid mode")
    x = synth.conv_image(xs, case=32, dtype="f16")
    k = synth.conv_kernel(ks, case=32)
    y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
    _check_float(y, x, k, mode, f"f16 rows {xs}*{ks} {mode}")


def test_conv_rows_unaligned_views(api):
    """u8 and f16 views whose rows do not start on 4-byte boundaries take the
    tiled kernels; results are the same definition."""
    xu = synth.conv_image((40, 203), case=33, dtype="u8")
    ku = synth.conv_kernel((3, 3), case=33, dtype="i32")
    base = torch.from_numpy(xu).cuda()
    v = base[:, 1:]  # row starts at an odd byte
    y = api.conv_nd_ex(v, torch.from_numpy(ku).cuda(), "full", k_host=ku).cpu().numpy()
    np.testing.assert_array_equal(y.astype(np.int64), O.conv(xu[:, 1:], ku, "full"))
    xh = synth.conv_image((40, 203), case=34, dtype="f16")
    kh = synth.conv_kernel((5, 5), case=34)
    vh = torch.from_numpy(xh).cuda()[:, 1:]
    yh = api.conv_nd(vh, torch.from_numpy(kh).cuda(), "same").cpu().numpy()
    _check_float(yh, xh[:, 1:], kh, "same", "f16 unaligned")


@pytest.mark.parametrize("dtype,K", [("u8", 3), ("u8", 7), ("f16", 3), ("f16", 7)])
def test_conv_rows_benchmark_sizes_sampled(api, dtype, K):
    x = synth.conv_image((4096, 4096), case=500 + K, dtype=dtype)
    if dtype == "u8":
        k = synth.conv_kernel((K, K), case=500 + K, dtype="i32")
        y = api.conv_nd_ex(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "full", k_host=k)
    else:
        k = synth.conv_kernel((K, K), case=500 + K)
        y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), "full")
    rng = np.random.default_rng(K)
    idx = _sample_index(tuple(y.shape), 600, rng)
    got = y.cpu().numpy()[tuple(np.array(idx).T)]
    ref = O.conv_at(x, k, "full", idx)
    if dtype == "u8":
        np.testing.assert_array_equal(got.astype(np.int64), ref)
    else:
        bound = TAU_CONV * O.conv_at(np.abs(x.astype(np.float64)), np.abs(k.astype(np.float64)), "full", idx)
        assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("dtype", ["u8", "f16"])
def test_conv3d_rows_u8_f16(api, dtype):
    xs, ks = (6, 40, 260), (3, 3, 3)
    x = synth.conv_image(xs, case=35, dtype=dtype)
    for mode in ("full", "same", "valid"):
        if dtype == "u8":
            k = synth.conv_kernel(ks, case=35, dtype="i32")
            y = api.conv_nd_ex(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode, k_host=k).cpu().numpy()
            np.testing.assert_array_equal(y.astype(np.int64), O.conv(x, k, mode))
        else:
            k = synth.conv_kernel(ks, case=35)
            y = api.conv_nd(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode).cpu().numpy()
            _check_float(y, x, k, mode, f"f16 3d {mode}")


@pytest.mark.parametrize("dtype", ["f32", "f16", "u8"])
@pytest.mark.parametrize("xs,K", [((61, 777), 3), ((37, 530), 5), ((29, 1100), 7), ((45, 600), 2), ((6, 19, 300), 5)])
def test_band_rows_bitwise(api, dtype, xs, K):
    """Every band height of the row-streaming kernels (2, 4, 8 output rows
    per wave, and the default) gives the same output bit for bit, within the
    oracle's bound (exact for u8)."""
    ks = (K,) * len(xs)
    x = synth.conv_image(xs, case=40 + K, dtype=dtype)
    xg = torch.from_numpy(x).cuda()
    if dtype == "u8":
        k = synth.conv_kernel(ks, case=40 + K, dtype="i32")
        kabs = int(np.abs(k.astype(np.int64)).sum())
    else:
        k = synth.conv_kernel(ks, case=40 + K)
        kabs = None
    kg = torch.from_numpy(k).cuda()
    outs = [api.conv_nd_ex(xg, kg, "full", method="direct", k_abs_sum=kabs, band_rows=br) for br in (0, 2, 4, 8)]
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    y = outs[0].cpu().numpy()
    if dtype == "u8":
        np.testing.assert_array_equal(y.astype(np.int64), O.conv(x, k, "full"))
    else:
        _check_float(y, x, k, "full", f"band rows {dtype} {xs}*{K}")
