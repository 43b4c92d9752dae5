"""GPU parity of tc_gradient (E_x, E_y, magnitude, direction under the 2x2 and
3x3 masks) against the FP64 oracle.

Tolerances, from the FP32 arithmetic of the kernel (u = 2^-24): each of E_x,
E_y is a sum of at most six masked pixel differences and one scale, so its
error is at most TAU_E = 8u times the same sum taken over absolute values
(the oracle's mask applied to |E| with |mask|).  The magnitude moves by at most
the error vector's length plus 4u of itself (squares, sum, correctly rounded
square root).  The direction moves by at most twice the error vector's length
over the magnitude plus the inverse tangent's own error (taken as 8 ulp of pi);
it is compared on the circle and only where the magnitude exceeds four times
that error length (elsewhere it is not determined by the data).  U8 images
under the 2x2 mask and the Sobel mask are exact (integer numerators, a
power-of-two scale), and so is the direction wherever the gradient is zero."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_08825_amd import synth

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
TAU_E = 8 * U
ATAN_ABS = 8 * U * math.pi


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def image(H, W, dtype, seed):
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        # flat patches, edges and noise: zero gradients occur, as in video
        a = rng.integers(0, 256, (H, W)).astype(np.uint8)
        a[: H // 3, : W // 3] = 77
        return a
    if dtype == "f16":
        return rng.uniform(0, 1, (H, W)).astype(np.float16)
    return rng.normal(0, 3, (H, W)).astype(np.float32)


def check(api, img_np, stencil, got, ctx):
    g = O.gradient(img_np.astype(np.float64), stencil)
    mx, my = O.masks(stencil)
    a = np.abs(img_np.astype(np.float64))
    tx = TAU_E * O.apply_mask(a, np.abs(mx)) + 1e-30
    ty = TAU_E * O.apply_mask(a, np.abs(my)) + 1e-30
    ex, ey = got["ex"].double().cpu().numpy(), got["ey"].double().cpu().numpy()
    mag, dr = got["mag"].double().cpu().numpy(), got["dir"].double().cpu().numpy()
    assert ex.shape == g["ex"].shape, ctx
    assert np.all(np.abs(ex - g["ex"]) <= tx), (ctx, np.max(np.abs(ex - g["ex"]) / tx))
    assert np.all(np.abs(ey - g["ey"]) <= ty), (ctx, np.max(np.abs(ey - g["ey"]) / ty))
    te = np.hypot(tx, ty)
    assert np.all(np.abs(mag - g["mag"]) <= te + 4 * U * g["mag"]), ctx
    det = g["mag"] > 4 * te
    d = np.abs(np.angle(np.exp(1j * (dr - g["dir"]))))
    bound = 2 * te / np.maximum(g["mag"], 1e-300) + ATAN_ABS
    assert np.all(d[det] <= bound[det]), (ctx, np.max((d - bound)[det]))
    assert np.all(np.abs(dr) <= math.pi + 1e-6), ctx
    zero = g["mag"] == 0
    assert np.all(dr[zero] == 0.0) and np.all(mag[zero] == 0.0), ctx
    if img_np.dtype == np.uint8 and stencil in ("fd2", "sobel3"):
        assert np.array_equal(ex, g["ex"]) and np.array_equal(ey, g["ey"]), ctx
    return det.mean() if det.size else 1.0


@pytest.mark.parametrize("stencil", ["fd2", "roberts", "prewitt3", "sobel3"])
@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
# W a multiple of 4 takes the vector kernel (aligned input rows; output rows of
# any alignment), other widths the any-stride kernel
@pytest.mark.parametrize("H,W", [(37, 300), (64, 257), (5, 1031), (3, 3), (45, 1028), (9, 8), (2, 4), (70, 2052)])
def test_gradient_matches_oracle(api, stencil, dtype, H, W):
    img = image(H, W, dtype, seed=H * 1000 + W)
    got = api.gradient(torch.from_numpy(img).cuda(), stencil)
    torch.cuda.synchronize()
    check(api, img, stencil, got, (stencil, dtype, H, W))


@pytest.mark.parametrize("stencil", ["fd2", "sobel3"])
def test_gradient_of_video_frame(api, stencil):
    """A frame of the synthetic time-to-contact video at full 480 x 640."""
    v = synth.multiscale_video(H=480, W=640, F=2, foe=(40, -30), ttc_start=40, ttc_end=39, dtype="u8")
    got = api.gradient(torch.from_numpy(v.frames[0]).cuda(), stencil)
    torch.cuda.synchronize()
    frac = check(api, v.frames[0], stencil, got, ("video", stencil))
    assert frac > 0.5  # the direction is checked over most of the frame


def test_strided_input_and_outputs(api):
    img = image(50, 90, "f32", seed=3)
    big = torch.from_numpy(img).cuda()
    view = big.t()  # column-major view: stride (1, 90)
    H, W = view.shape
    outs = {n: torch.full((H + 3, 2 * (W - 2)), -7.0, device="cuda") for n in ("ex", "ey", "mag", "dir")}
    views = {n: t[1:H - 1, ::2] for n, t in outs.items()}
    from paper_1612_08825_amd import _lib as L
    import ctypes as C

    L.check("tc_gradient", api._lib().tc_gradient(C.byref(api._desc(view)), L.TC_STENCIL_SOBEL3,
                                                  *[C.byref(api._desc(views[n])) for n in ("ex", "ey", "mag", "dir")],
                                                  api._stream()))
    torch.cuda.synchronize()
    check(api, np.ascontiguousarray(img.T), "sobel3", views, "strided")
    for t in outs.values():  # nothing outside the views was written
        assert bool((t[0] == -7).all()) and bool((t[H - 1:] == -7).all()) and bool((t[:, 1::2] == -7).all())


def test_optional_outputs_and_empty(api):
    img = torch.from_numpy(image(20, 30, "u8", seed=9)).cuda()
    full = api.gradient(img, "prewitt3")
    part = api.gradient(img, "prewitt3", want=("dir",))
    torch.cuda.synchronize()
    assert set(part) == {"dir"} and torch.equal(part["dir"], full["dir"])
    for H, W, st in [(1, 40, "fd2"), (2, 2, "prewitt3"), (40, 1, "roberts")]:
        e = api.gradient(torch.zeros((H, W), dtype=torch.uint8, device="cuda"), st)
        assert all(t.numel() == 0 for t in e.values())


def test_rejections(api):
    from paper_1612_08825_amd import _lib as L
    import ctypes as C

    img = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    bad_shape = torch.zeros((7, 6), device="cuda")
    bad_dtype = torch.zeros((7, 7), dtype=torch.float16, device="cuda")
    lib = api._lib()
    d = C.byref(api._desc(img))
    assert lib.tc_gradient(d, 4, None, None, None, None, None) == L.TC_EINVAL
    assert lib.tc_gradient(d, 0, C.byref(api._desc(bad_shape)), None, None, None, None) == L.TC_ESHAPE
    assert lib.tc_gradient(d, 0, C.byref(api._desc(bad_dtype)), None, None, None, None) == L.TC_EDTYPE
    i32 = torch.zeros((8, 8), dtype=torch.int32, device="cuda")
    assert lib.tc_gradient(C.byref(api._desc(i32)), 0, None, None, None, None, None) == L.TC_EDTYPE


@pytest.mark.parametrize("stencil", ["fd2", "sobel3"])
@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
def test_vector_kernel_equals_any_stride_kernel(api, stencil, dtype):
    """The same image through both kernels (an odd row stride forces the
    any-stride one): equal results; outputs whose rows start at every 4-byte
    offset of a 16-byte line."""
    H, W = 23, 1540
    img = image(H, W, dtype, seed=77)
    k = 3 if stencil == "sobel3" else 2
    Ho, Wo = H - k + 1, W - k + 1
    dense = torch.from_numpy(img).cuda()
    odd = torch.empty((H, W + 1), dtype=dense.dtype, device="cuda")[:, :W]
    odd.copy_(dense)
    assert odd.stride(0) % 4 != 0
    names = ("ex", "ey", "mag", "dir")
    a = api.gradient(dense, stencil)
    b = api.gradient(odd, stencil)
    # outputs offset by 1..3 floats inside rows of stride Wo + 5
    par = {n: torch.full((Ho, Wo + 5), -9.0, device="cuda") for n in names}
    c = api.gradient(dense, stencil, out={n: par[n][:, 1 + i % 3:1 + i % 3 + Wo] for i, n in enumerate(names)})
    torch.cuda.synchronize()
    for i, n in enumerate(names):
        assert torch.equal(a[n], b[n]), n
        assert torch.equal(a[n], c[n]), n
        off = 1 + i % 3
        assert bool((par[n][:, :off] == -9).all()) and bool((par[n][:, off + Wo:] == -9).all()), n
    check(api, img, stencil, a, ("vec", stencil, dtype))
