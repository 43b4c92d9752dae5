"""GPU parity of the FFT branch of 2-D and 3-D convolution (tc_conv_fft,
tc_conv2d_fft) against the FP64 oracle's direct convolution, and of the hybrid
dispatchers.

Tolerance.  The FFT result carries a norm-wise error (every output mixes every
input).  For a radix-2 transform with accurate twiddles the relative 2-norm
error of one N-point transform is at most log2(N) * eta with eta <= 8u
(u = 2^-24; Higham, Accuracy and Stability of Numerical Algorithms, the FFT
chapter).  The mixed-radix transform here runs stages of radix R in {2, 3, 4,
5}; a radix-R stage is charged as log2(R) radix-2 levels, eta_R =
8u log2(R), plus 2(R - 1)u for the twiddle powers w^2 .. w^(R-1) formed by
repeated multiplication from one table value (itself rounded from FP64).  The
path transforms x and k forward (the stages of every axis), takes one complex
product per point and transforms back; with ||x (*) k||_2 <= ||x||_2 ||k||_1

    ||y - y64||_2 <= TAU_FFT ||x||_2 ||k||_1,
    TAU_FFT = 3 * sum over the axes' stages of (8 log2(R) + 2 (R - 1)) u + 4u,

which the tests check, together with the element-wise consequence
max |y - y64| <= ||y - y64||_2.  That bound is a worst case and sits two to
three orders of magnitude above the measured errors, so on its own it would
let through a transform with a wrong twiddle in a late stage; the tests also
hold the measured error to RATIO_MAX of the bound and to REL2_MAX relative to
||y64||_2 (rounding errors of an FFT grow like sqrt(log2 N) u on random data).

Padded extents: each axis but the last is padded to the smallest 2^a 3^b 5^c
holding the full output; its stages are radix 4 while two factors of 2 remain,
one radix 2 for an odd one, then the 3s and the 5s (`fft_axis` below restates
that rule).  The last axis is real: it is padded to twice such a number
holding half the full output and transformed as half as many complex points
(`axis_plan`).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
RATIO_MAX = 0.05
TAU_CONV_ABS = 1e-5
REL2_MAX = 1e-5


def fft_axis(n):
    """(padded extent, stage radices) of one axis of extent n."""
    m = max(1, n)
    while True:
        r, e = m, {2: 0, 3: 0, 5: 0}
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
                e[p] += 1
        if r == 1:
            return m, [4] * (e[2] // 2) + [2] * (e[2] % 2) + [3] * e[3] + [5] * e[5]
        m += 1


def axis_plan(xs, ks):
    """(padded extent, stages) per axis: the last (real) axis is transformed as
    half as many complex points, padded to twice a 2^a 3^b 5^c, plus the real
    post-/pre-step, charged as one more radix-2 stage."""
    out = []
    for i, (a, b) in enumerate(zip(xs, ks)):
        full = a + b - 1
        if i == len(xs) - 1:
            m, st = fft_axis((full + 1) // 2)
            out.append((2 * m, st + [2]))
        else:
            out.append(fft_axis(full))
    return out


def tau_fft(xs, ks):
    stages = sum((st for _, st in axis_plan(xs, ks)), [])
    return 3 * U * sum(8 * math.log2(R) + 2 * (R - 1) for R in stages) + 4 * U


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def check(x, k, y, ref):
    err = np.asarray(y, dtype=np.float64) - ref
    bound = tau_fft(x.shape, k.shape) * np.linalg.norm(x) * np.abs(k).sum()
    e2 = float(np.linalg.norm(err))
    assert e2 <= bound, (e2, bound)
    # the worst case sits far above typical errors only once there are a few
    # stages (a 1 x 1 transform is one rounded product, at the bound's scale)
    n_stages = sum(len(st) for _, st in axis_plan(x.shape, k.shape))
    if n_stages >= 4:
        assert e2 <= RATIO_MAX * bound, (e2, bound)
    n2 = float(np.linalg.norm(ref))
    if n2 > 0:
        assert e2 <= REL2_MAX * n2, (e2, n2)
    return e2 / bound


@pytest.mark.parametrize("xs,ks", [((37, 50), (5, 7)), ((20, 33), (15, 15)), ((3, 4), (6, 9)), ((64, 64), (64, 64)),
                                   ((100, 300), (31, 31)), ((1, 1), (1, 1)), ((257, 129), (2, 40))])
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_fft_matches_oracle(api, xs, ks, mode):
    ge = all(a >= b for a, b in zip(xs, ks))
    le = all(a <= b for a, b in zip(xs, ks))
    if mode == "valid" and not (ge or le):
        pytest.skip("valid mode needs x >= k or x <= k in every dimension")
    rng = np.random.default_rng(sum(xs) + 7 * sum(ks))
    x = rng.normal(0, 1, xs).astype(np.float32)
    k = rng.normal(0, 1, ks).astype(np.float32)
    y = api.conv2d_fft(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode)
    torch.cuda.synchronize()
    ref = O.conv(x.astype(np.float64), k.astype(np.float64), mode)
    assert tuple(y.shape) == ref.shape
    r = check(x, k, y.cpu().numpy(), ref)
    print(f"[fft] {xs}*{ks} {mode}: error / bound {r:.3f}")


def test_fft_large_against_direct_and_sampled_oracle(api):
    """2048 x 2048 image, 31 x 31 kernel (near the size where the hybrid
    switches): against the direct kernels (pinned element-wise elsewhere) and
    sampled oracle outputs."""
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (2048, 2048)).astype(np.float32)
    k = rng.normal(0, 1, (31, 31)).astype(np.float32)
    xd, kd = torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda()
    yf = api.conv2d_fft(xd, kd, "full")
    yd = api.conv_nd(xd, kd, "full")
    torch.cuda.synchronize()
    bound = tau_fft(x.shape, k.shape) * np.linalg.norm(x) * np.abs(k).sum()
    diff = (yf.double() - yd.double()).cpu().numpy()
    assert float(np.linalg.norm(diff)) <= RATIO_MAX * bound
    assert float(np.linalg.norm(diff)) <= REL2_MAX * float(torch.linalg.vector_norm(yd.double()))
    idx = [(0, 0), (15, 15), (1000, 1234), (2077, 2077), (2060, 5), (30, 2070)]
    want = O.conv_at(x, k, "full", idx)
    got = yf.cpu().numpy()
    # per element: an FFT output carries about the rms error of the whole
    # result, i.e. ||err||_2 / sqrt(#outputs); allow 8 times that estimate
    # (taken from the measured norm-wise error against the direct kernels)
    rms = float(np.linalg.norm(diff)) / np.sqrt(diff.size)
    for (i, j), w in zip(idx, want):
        assert abs(float(got[i, j]) - float(w)) <= max(8 * rms, TAU_CONV_ABS * abs(float(w))), (i, j)


def test_hybrid_dispatch(api):
    x = torch.randn(200, 300, device="cuda")
    small = torch.randn(api.FFT_THRESHOLD - 2, 5, device="cuda")
    big = torch.randn(api.FFT_THRESHOLD, 3, device="cuda")
    a = api.conv2d_hybrid(x, small, "same")
    b = api.conv_nd(x, small, "same")
    c = api.conv2d_hybrid(x, big, "same")
    d = api.conv2d_fft(x, big, "same")
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, d)


def test_strided_input_output(api):
    rng = np.random.default_rng(8)
    x = rng.normal(0, 1, (60, 90)).astype(np.float32)
    k = rng.normal(0, 1, (9, 5)).astype(np.float32)
    xt = torch.from_numpy(np.ascontiguousarray(x.T)).cuda().t()  # column-major view
    yb = torch.full((68 + 4, 2 * 94), -5.0, device="cuda")
    yv = yb[2:70, ::2]
    api.conv2d_fft(xt, torch.from_numpy(k).cuda(), "full", out=yv)
    torch.cuda.synchronize()
    check(x, k, yv.cpu().numpy(), O.conv(x.astype(np.float64), k.astype(np.float64), "full"))
    assert bool((yb[:2] == -5).all()) and bool((yb[70:] == -5).all()) and bool((yb[:, 1::2] == -5).all())


def test_rejections(api):
    from paper_1612_08825_amd import _lib as L
    import ctypes as C

    lib = api._lib()
    n = C.c_size_t(0)
    big = torch.zeros((4000, 10), device="cuda")
    k = torch.zeros((200, 3), device="cuda")
    assert lib.tc_conv2d_fft_workspace_size(C.byref(api._desc(big)), C.byref(api._desc(k)), L.MODES["full"],
                                            C.byref(n)) == L.TC_ESHAPE
    h = torch.zeros((10, 10), dtype=torch.float16, device="cuda")
    assert lib.tc_conv2d_fft_workspace_size(C.byref(api._desc(h)), C.byref(api._desc(k)), L.MODES["full"],
                                            C.byref(n)) == L.TC_EDTYPE
    x = torch.zeros((10, 10), device="cuda")
    kk = torch.zeros((3, 3), device="cuda")
    y = torch.zeros((12, 12), device="cuda")
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    assert lib.tc_conv2d_fft(C.byref(api._desc(x)), C.byref(api._desc(kk)), L.MODES["full"], C.byref(api._desc(y)),
                             C.c_void_p(ws.data_ptr()), 64, None) == L.TC_ENOMEM


# ----------------------------------------------------------------------------- mixed radix and rank 3
@pytest.mark.parametrize("xs,ks", [((41, 52), (5, 9)), ((27, 22), (19, 3)), ((60, 7), (16, 24)), ((125, 2), (1, 1))])
def test_fft_mixed_radix_2d(api, xs, ks):
    """Padded extents with factors 3 and 5 (every radix the row pass has)."""
    radices = {R for _, st in axis_plan(xs, ks) for R in st}
    assert radices & {3, 5}
    rng = np.random.default_rng(11 + sum(xs))
    x = rng.normal(0, 1, xs).astype(np.float32)
    k = rng.normal(0, 1, ks).astype(np.float32)
    for mode in ("full", "same"):
        y = api.conv_fft(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode)
        ref = O.conv(x.astype(np.float64), k.astype(np.float64), mode)
        r = check(x, k, y.cpu().numpy(), ref)
        print(f"[fft] {xs}*{ks} {mode} (padded {[n for n, _ in axis_plan(xs, ks)]}): {r:.4f}")


SHAPES_3D = [((9, 20, 17), (3, 5, 4)), ((16, 16, 16), (9, 9, 9)), ((5, 31, 40), (5, 2, 7)), ((1, 1, 1), (1, 1, 1)),
             ((7, 3, 50), (2, 9, 11)), ((12, 14, 6), (12, 14, 6)), ((3, 4, 5), (6, 7, 8))]


@pytest.mark.parametrize("xs,ks", SHAPES_3D)
@pytest.mark.parametrize("mode", ["full", "same", "valid"])
def test_fft3d_matches_oracle(api, xs, ks, mode):
    ge = all(a >= b for a, b in zip(xs, ks))
    le = all(a <= b for a, b in zip(xs, ks))
    if mode == "valid" and not (ge or le):
        pytest.skip("valid mode needs x >= k or x <= k in every dimension")
    rng = np.random.default_rng(3 * sum(xs) + sum(ks))
    x = rng.normal(0, 1, xs).astype(np.float32)
    k = rng.normal(0, 1, ks).astype(np.float32)
    y = api.conv_fft(torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda(), mode)
    ref = O.conv(x.astype(np.float64), k.astype(np.float64), mode)
    assert tuple(y.shape) == ref.shape
    r = check(x, k, y.cpu().numpy(), ref)
    print(f"[fft3d] {xs}*{ks} {mode}: error / bound {r:.4f}")


def test_fft3d_strided_input_and_output(api):
    rng = np.random.default_rng(5)
    big = torch.from_numpy(rng.normal(0, 1, (12, 30, 41)).astype(np.float32)).cuda()
    x = big[2:10, 3:25:2, 1:40]  # strided in every dimension
    k = torch.from_numpy(rng.normal(0, 1, (3, 4, 6)).astype(np.float32)).cuda()
    ref = O.conv(x.cpu().numpy().astype(np.float64), k.cpu().numpy().astype(np.float64), "full")
    out_big = torch.full((ref.shape[0], ref.shape[1], ref.shape[2] + 7), -3.0, device="cuda")
    out = out_big[:, :, 2:2 + ref.shape[2]]
    api.conv_fft(x, k, "full", out=out)
    check(x.cpu().numpy(), k.cpu().numpy(), out.cpu().numpy(), ref)
    assert float(out_big[:, :, :2].abs().max()) == 3.0 and float(out_big[:, :, 2 + ref.shape[2]:].abs().max()) == 3.0


def test_fft3d_volume_against_direct_and_sampled_oracle(api):
    """A 64 x 256 x 256 volume and a 15^3 kernel (padded 80 x 270 x 270):
    against the direct kernels and sampled oracle outputs."""
    rng = np.random.default_rng(9)
    x = rng.uniform(0, 1, (64, 256, 256)).astype(np.float32)
    k = rng.normal(0, 1, (15, 15, 15)).astype(np.float32)
    xd, kd = torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda()
    yf = api.conv_fft(xd, kd, "full")
    yd = api.conv_nd(xd, kd, "full")
    torch.cuda.synchronize()
    bound = tau_fft(x.shape, k.shape) * np.linalg.norm(x) * np.abs(k).sum()
    diff = (yf.double() - yd.double()).cpu().numpy()
    e2 = float(np.linalg.norm(diff))
    assert e2 <= RATIO_MAX * bound, (e2, bound)
    assert e2 <= REL2_MAX * float(torch.linalg.vector_norm(yd.double())), e2
    idx = [(0, 0, 0), (7, 100, 200), (77, 269, 269), (40, 3, 260), (70, 135, 7)]
    want = O.conv_at(x, k, "full", idx)
    got = yf.cpu().numpy()
    rms = e2 / np.sqrt(diff.size)
    for (a, b, c), w in zip(idx, want):
        assert abs(float(got[a, b, c]) - float(w)) <= max(8 * rms, TAU_CONV_ABS * abs(float(w))), (a, b, c)


def test_dispatcher_rank3(api):
    """tc_conv_nd_ex picks the FFT branch for 3-D kernels from the measured
    3-D crossover on (given a workspace), the direct kernels below it."""
    x = torch.randn(20, 40, 36, device="cuda")
    big = torch.randn(api.FFT_THRESHOLD_3D, 3, 4, device="cuda")
    small = torch.randn(api.FFT_THRESHOLD_3D - 2, 3, 3, device="cuda")
    ws = torch.empty(api.conv_workspace_size(x, big, "same"), dtype=torch.uint8, device="cuda")
    a = api.conv_nd_ex(x, big, "same", ws=ws)
    b = api.conv_fft(x, big, "same")
    c = api.conv_nd_ex(x, small, "same", ws=ws)
    d = api.conv_nd(x, small, "same")
    e = api.conv_hybrid(x, big, "same")
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(c, d) and torch.equal(e, b)


def test_fft_rejections(api):
    from paper_1612_08825_amd import _lib as L

    x3 = torch.zeros((4, 5, 6), device="cuda")
    k2 = torch.zeros((3, 3), device="cuda")
    with pytest.raises(L.TTCError) as e:
        api.conv_fft_workspace_size(x3, k2)  # rank mismatch
    assert e.value.code == L.TC_ESHAPE
    with pytest.raises(L.TTCError) as e:
        api.conv2d_fft_workspace_size(x3, torch.zeros((3, 3, 3), device="cuda"))  # the 2-D entry, rank 3
    assert e.value.code == L.TC_ESHAPE
    with pytest.raises(L.TTCError) as e:
        api.conv_fft_workspace_size(torch.zeros((1, 4090), device="cuda"), torch.zeros((1, 8), device="cuda"))
    assert e.value.code == L.TC_ESHAPE  # 4097 > 4096
    x4 = torch.zeros((2, 2, 2, 2), device="cuda")
    with pytest.raises(L.TTCError) as e:
        api.conv_fft_workspace_size(x4, x4)
    assert e.value.code == L.TC_ESHAPE
    # a workspace smaller than tc_conv_fft_workspace_size: refused, nothing launched
    x = torch.ones((30, 30, 30), device="cuda")
    k = torch.ones((5, 5, 5), device="cuda")
    y = torch.full((34, 34, 34), 7.0, device="cuda")
    ws = torch.zeros(64, dtype=torch.uint8, device="cuda")
    lib = api._lib()
    rc = lib.tc_conv_fft(api.C.byref(api._desc(x)), api.C.byref(api._desc(k)), L.MODES["full"],
                         api.C.byref(api._desc(y)), api.C.c_void_p(ws.data_ptr()), 64, None)
    torch.cuda.synchronize()
    assert rc == L.TC_ENOMEM and float(y.min()) == 7.0 and float(y.max()) == 7.0
