"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its struct layouts match the binding, and argument
validation rejects bad input before anything is launched (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

from paper_1612_08825_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttcconv.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libttcconv.so is not built (python -m paper_1612_08825_amd.build)")
    return L.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(tc_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_function(lib):
    names = header_functions()
    assert len(names) >= 16
    assert set(names) == set(L.SIGNATURES), "binding signatures and header disagree"
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (tc_[a-z0-9_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_struct_layouts_match_header():
    src = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "ttcconv.h"
    int main(void) {
      printf("%zu %zu %zu %zu\n", sizeof(tc_tensor), sizeof(tc_seq), sizeof(tc_ttc_level), sizeof(tc_ttc_pick));
      printf("%zu %zu %zu %zu\n", offsetof(tc_ttc_level, A), offsetof(tc_ttc_level, n), offsetof(tc_ttc_level, status),
             offsetof(tc_ttc_pick, level));
      printf("%zu %zu\n", offsetof(tc_tensor, shape), offsetof(tc_seq, H));
      printf("%zu %zu %zu\n", sizeof(tc_conv_opts), offsetof(tc_conv_opts, workspace_bytes),
             offsetof(tc_conv_opts, band_rows));
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == C.sizeof(L.TcTensor)
    assert vals[1] == C.sizeof(L.TcSeq)
    assert vals[2] == L.LEVEL_DTYPE.itemsize
    assert vals[3] == L.PICK_DTYPE.itemsize
    assert vals[4] == L.LEVEL_DTYPE.fields["A"][1]
    assert vals[5] == L.LEVEL_DTYPE.fields["n"][1]
    assert vals[6] == L.LEVEL_DTYPE.fields["status"][1]
    assert vals[7] == L.PICK_DTYPE.fields["level"][1]
    assert vals[8] == L.TcTensor.shape.offset
    assert vals[9] == L.TcSeq.H.offset
    assert vals[10] == C.sizeof(L.TcConvOpts)
    assert vals[11] == L.TcConvOpts.workspace_bytes.offset
    assert vals[12] == L.TcConvOpts.band_rows.offset


def test_status_strings(lib):
    for code in (0, 1, 2, 3, -1, -2, -3, -4, -5, -6, 99):
        assert lib.tc_status_str(code)
    assert lib.tc_version() == 100


def _desc(shape, dt, data=None):
    d = L.TcTensor()
    d.data = data
    d.dtype = dt
    d.ndim = len(shape)
    s = 1
    for i in range(len(shape) - 1, -1, -1):
        d.shape[i] = shape[i]
        d.stride[i] = s
        s *= shape[i]
    return d


def test_conv_out_shape_queries(lib):
    out = (C.c_int64 * 8)()
    x, k = _desc((10, 7), L.TC_F32), _desc((3, 4), L.TC_F32)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(k), L.TC_FULL, out) == 0
    assert (out[0], out[1]) == (12, 10)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(k), L.TC_SAME, out) == 0
    assert (out[0], out[1]) == (10, 7)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(k), L.TC_VALID, out) == 0
    assert (out[0], out[1]) == (8, 4)
    big = _desc((12, 9), L.TC_F32)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(big), L.TC_VALID, out) == 0
    assert (out[0], out[1]) == (3, 3)
    mixed = _desc((12, 3), L.TC_F32)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(mixed), L.TC_VALID, out) == L.TC_ESHAPE
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(k), 7, out) == L.TC_EINVAL
    kr = _desc((3,), L.TC_F32)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(kr), L.TC_FULL, out) == L.TC_ESHAPE
    ki = _desc((3, 4), L.TC_I32)
    assert lib.tc_conv_out_shape(C.byref(x), C.byref(ki), L.TC_FULL, out) == L.TC_EDTYPE
    xu = _desc((10, 7), L.TC_U8)
    assert lib.tc_conv_out_shape(C.byref(xu), C.byref(ki), L.TC_FULL, out) == 0
    assert lib.tc_conv_out_shape(C.byref(xu), C.byref(k), L.TC_FULL, out) == L.TC_EDTYPE


def test_conv_nd_rejects_before_launch(lib):
    x = _desc((10, 7), L.TC_F32, data=16)
    k = _desc((3, 3), L.TC_F32, data=16)
    y_bad = _desc((11, 9), L.TC_F32, data=16)
    assert lib.tc_conv_nd(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y_bad), None) == L.TC_ESHAPE
    y_dt = _desc((12, 9), L.TC_I32, data=16)
    assert lib.tc_conv_nd(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y_dt), None) == L.TC_EDTYPE
    x_null = _desc((10, 7), L.TC_F32, data=None)
    y = _desc((12, 9), L.TC_F32, data=16)
    assert lib.tc_conv_nd(C.byref(x_null), C.byref(k), L.TC_FULL, C.byref(y), None) == L.TC_EINVAL
    k_strided = _desc((3, 3), L.TC_F32, data=16)
    k_strided.stride[1] = 2
    assert lib.tc_conv_nd(C.byref(x), C.byref(k_strided), L.TC_FULL, C.byref(y), None) == L.TC_ESHAPE
    x0 = _desc((10, 7), L.TC_F32, data=16)
    x0.stride[0] = 0
    assert lib.tc_conv_nd(C.byref(x0), C.byref(k), L.TC_FULL, C.byref(y), None) == L.TC_ESHAPE


def test_conv_nd_ex_rejects_before_launch(lib):
    """Integer kernels: the exactness bound comes from the caller (a stated
    sum |k| or a host copy of k), never from a device read; every rejection
    happens before anything is launched."""
    import numpy as np

    xu = _desc((10, 7), L.TC_U8, data=16)
    ki = _desc((3, 3), L.TC_I32, data=16)
    yi = _desc((12, 9), L.TC_I32, data=16)
    # the plain entry point refuses integer kernels outright
    assert lib.tc_conv_nd(C.byref(xu), C.byref(ki), L.TC_FULL, C.byref(yi), None) == L.TC_EINVAL
    # no bound given
    assert lib.tc_conv_nd_ex(C.byref(xu), C.byref(ki), L.TC_FULL, C.byref(yi), None, None) == L.TC_EINVAL
    o = L.TcConvOpts()
    o.method = L.TC_CONV_DIRECT
    o.k_abs_sum = -1
    assert lib.tc_conv_nd_ex(C.byref(xu), C.byref(ki), L.TC_FULL, C.byref(yi), C.byref(o), None) == L.TC_EINVAL
    # a stated bound past 2^31 / 255
    o.k_abs_sum = 2147483647 // 255 + 1
    assert lib.tc_conv_nd_ex(C.byref(xu), C.byref(ki), L.TC_FULL, C.byref(yi), C.byref(o), None) == L.TC_EOVERFLOW
    # a host copy whose taps break the bound (255 * 8421505 > 2^31 - 1)
    kh = np.zeros((3, 3), np.int32)
    kh[0, 0] = 8421504
    kh[2, 2] = -1
    o.k_abs_sum = -1
    o.k_host = kh.ctypes.data
    assert lib.tc_conv_nd_ex(C.byref(xu), C.byref(ki), L.TC_FULL, C.byref(yi), C.byref(o), None) == L.TC_EOVERFLOW
    # bad method, bad threshold
    o2 = L.TcConvOpts()
    o2.method = 9
    x = _desc((10, 7), L.TC_F32, data=16)
    k = _desc((3, 3), L.TC_F32, data=16)
    y = _desc((12, 9), L.TC_F32, data=16)
    assert lib.tc_conv_nd_ex(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y), C.byref(o2), None) == L.TC_EINVAL
    o2.method = L.TC_CONV_AUTO
    o2.fft_threshold = -3
    assert lib.tc_conv_nd_ex(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y), C.byref(o2), None) == L.TC_EINVAL
    # band heights other than 0, 2, 4, 8, and a non-zero reserved field
    for br in (1, 3, 16, -2):
        o2 = L.TcConvOpts()
        o2.band_rows = br
        assert lib.tc_conv_nd_ex(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y), C.byref(o2), None) == L.TC_EINVAL
    o2 = L.TcConvOpts()
    o2.reserved = 1
    assert lib.tc_conv_nd_ex(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y), C.byref(o2), None) == L.TC_EINVAL
    # FFT forced on shapes it does not take, or without a workspace
    o3 = L.TcConvOpts()
    o3.method = L.TC_CONV_FFT
    xh = _desc((10, 7), L.TC_F16, data=16)
    assert lib.tc_conv_nd_ex(C.byref(xh), C.byref(k), L.TC_FULL, C.byref(y), C.byref(o3), None) == L.TC_EDTYPE
    assert lib.tc_conv_nd_ex(C.byref(x), C.byref(k), L.TC_FULL, C.byref(y), C.byref(o3), None) == L.TC_EINVAL
    n = C.c_size_t(123)
    assert lib.tc_conv_workspace_size(C.byref(x), C.byref(k), L.TC_FULL, L.TC_CONV_DIRECT, C.byref(n)) == 0
    assert n.value == 0
    assert lib.tc_conv_workspace_size(C.byref(x), C.byref(k), L.TC_FULL, L.TC_CONV_FFT, C.byref(n)) == 0
    assert n.value > 0
    assert lib.tc_conv_workspace_size(C.byref(xh), C.byref(k), L.TC_FULL, L.TC_CONV_AUTO, C.byref(n)) == 0
    assert n.value == 0
    assert lib.tc_conv_workspace_size(C.byref(xh), C.byref(k), L.TC_FULL, L.TC_CONV_FFT, C.byref(n)) == L.TC_EDTYPE


def test_pyramid_and_horn_validation(lib):
    Hl, Wl = C.c_int64(), C.c_int64()
    assert lib.tc_pyramid_shape(481, 641, 3, C.byref(Hl), C.byref(Wl)) == 0
    assert (Hl.value, Wl.value) == (60, 80)
    f = _desc((16, 16), L.TC_U8, data=16)
    assert lib.tc_image_pyramid(C.byref(f), 0, None, None) == L.TC_EINVAL
    assert lib.tc_image_pyramid(C.byref(f), 6, None, None) == L.TC_ESHAPE  # 16 >> 5 == 0
    outs = (L.TcTensor * 1)(_desc((8, 8), L.TC_F16, data=16))
    assert lib.tc_image_pyramid(C.byref(f), 2, outs, None) == L.TC_EDTYPE
    outs = (L.TcTensor * 1)(_desc((8, 7), L.TC_F32, data=16))
    assert lib.tc_image_pyramid(C.byref(f), 2, outs, None) == L.TC_ESHAPE
    g = _desc((16, 16), L.TC_F16, data=16)
    e = _desc((15, 15), L.TC_F32, data=16)
    assert lib.tc_horn_derivs(C.byref(f), C.byref(g), C.byref(e), C.byref(e), C.byref(e), None) == L.TC_EDTYPE
    ei = _desc((15, 15), L.TC_I32, data=16)
    assert lib.tc_horn_derivs(C.byref(g), C.byref(g), C.byref(ei), C.byref(ei), C.byref(ei), None) == L.TC_EDTYPE
    e_bad = _desc((15, 16), L.TC_F32, data=16)
    assert lib.tc_horn_derivs(C.byref(f), C.byref(f), C.byref(e_bad), C.byref(e), C.byref(e), None) == L.TC_ESHAPE


def _seq(H, W, F=2, levels=1, ptr=4096, row_stride=None):
    q = L.TcSeq()
    q.frame0 = ptr
    q.frame_stride = H * (row_stride or W)
    q.row_stride = row_stride or W
    q.H, q.W, q.n_frames, q.levels = H, W, F, levels
    return q


def test_ttc_plan_validation(lib):
    h = C.c_void_p()
    bad = [
        (_seq(64, 64, levels=5), L.TC_U8, L.TC_EINVAL),
        (_seq(64, 64, F=1), L.TC_U8, L.TC_EINVAL),
        (_seq(12, 64, levels=4), L.TC_U8, L.TC_ESHAPE),  # level 3 would be 1 row
        (_seq(64, 64), L.TC_F32, L.TC_EDTYPE),
        (_seq(64, 64, ptr=4097), L.TC_F16, L.TC_EINVAL),  # frame not aligned to its element size
        (_seq(64, 64, row_stride=32), L.TC_U8, L.TC_ESHAPE),
    ]
    for q, dt, code in bad:
        arr = (L.TcSeq * 1)(q)
        assert lib.tc_ttc_plan_create(arr, 1, dt, C.byref(h)) == code
    mixed = (L.TcSeq * 2)(_seq(64, 64, levels=2), _seq(64, 64, levels=3))
    assert lib.tc_ttc_plan_create(mixed, 2, L.TC_U8, C.byref(h)) == L.TC_EINVAL
    n = C.c_size_t()
    assert lib.tc_ttc_workspace_size(480, 640, 4, C.byref(n)) == 0 and n.value > 0
    assert lib.tc_ttc_workspace_size(480, 640, 5, C.byref(n)) == L.TC_EINVAL


def test_ttc_tuning_defaults_and_rejections(lib):
    t = L.TcTuning()
    # the sweep's choices, per frame type and level count
    want = {(L.TC_F16, 4): (128, 128), (L.TC_F16, 2): (128, 128), (L.TC_F16, 1): (128, 128), (L.TC_U8, 3): (128, 128),
            (L.TC_U8, 4): (128, 128)}
    for (dt, lv), shape in want.items():
        assert lib.tc_ttc_tuning_default(dt, lv, C.byref(t)) == 0
        assert (t.band_rows, t.groups_per_cu) == shape, (dt, lv)
    assert lib.tc_ttc_tuning_default(L.TC_F32, 3, C.byref(t)) == L.TC_EDTYPE
    h = C.c_void_p()
    arr = (L.TcSeq * 1)(_seq(64, 64, levels=3))
    for rows, gpc in [(12, 32), (8, 32), (24, 32), (272, 32), (16, 0), (16, 257), (0, 8)]:
        t.band_rows, t.groups_per_cu = rows, gpc
        assert lib.tc_ttc_plan_create_ex(arr, 1, L.TC_U8, C.byref(t), C.byref(h)) == L.TC_EINVAL, (rows, gpc)
        assert not h.value
    # re-planning needs a plan and a valid batch
    assert lib.tc_ttc_plan_reset(None, arr, 1) == L.TC_EINVAL


def _fft_axis_extent(n):
    m = max(1, n)
    while True:
        r = m
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def test_fft_workspace_follows_the_padding_rule(lib):
    """tc_conv_fft_workspace_size: one twiddle table per axis and three complex
    volumes of the stored spectrum, every axis but the last padded to the
    smallest 2^a 3^b 5^c holding the full output, the last (real) one to twice
    that of half of it and stored as half plus one frequencies (at most 4096
    points per axis), 256-byte aligned pieces."""
    al = lambda v: (v + 255) // 256 * 256
    cases = [((2048, 2048), (37, 37)), ((37, 50), (5, 7)), ((64, 256, 256), (15, 15, 15)), ((1, 1), (1, 1)),
             ((9, 20, 17), (3, 5, 4)), ((4000, 7), (97, 1))]
    for xs, ks in cases:
        n = [_fft_axis_extent(a + b - 1) for a, b in zip(xs[:-1], ks[:-1])]
        m = _fft_axis_extent((xs[-1] + ks[-1]) // 2)  # the real last axis: half its full extent, rounded up
        vol = m + 1  # its stored frequencies
        for v in n:
            vol *= v
        want = sum(al(v * 8) for v in n) + al(2 * m * 8) + 3 * al(vol * 8)
        got = C.c_size_t(0)
        x, k = _desc(xs, L.TC_F32), _desc(ks, L.TC_F32)
        assert lib.tc_conv_fft_workspace_size(C.byref(x), C.byref(k), L.TC_FULL, C.byref(got)) == L.TC_OK
        assert got.value == want, (xs, ks, n, got.value, want)
        if len(xs) == 2:
            g2 = C.c_size_t(0)
            assert lib.tc_conv2d_fft_workspace_size(C.byref(x), C.byref(k), L.TC_FULL, C.byref(g2)) == L.TC_OK
            assert g2.value == want
        else:
            assert lib.tc_conv2d_fft_workspace_size(C.byref(x), C.byref(k), L.TC_FULL, C.byref(got)) == L.TC_ESHAPE
    assert _fft_axis_extent(2084) == 2160 and _fft_axis_extent(4097) == 4320
    bad = [((1, 4090), (1, 8), L.TC_F32), ((2, 2, 2, 2), (1, 1, 1, 1), L.TC_F32), ((4, 5, 6), (3, 3), L.TC_F32)]
    for xs, ks, dt in bad:
        assert lib.tc_conv_fft_workspace_size(C.byref(_desc(xs, dt)), C.byref(_desc(ks, dt)), L.TC_FULL,
                                              C.byref(C.c_size_t(0))) == L.TC_ESHAPE, (xs, ks)
    assert lib.tc_conv_fft_workspace_size(C.byref(_desc((8, 8), L.TC_F16)), C.byref(_desc((3, 3), L.TC_F32)),
                                          L.TC_FULL, C.byref(C.c_size_t(0))) == L.TC_EDTYPE
