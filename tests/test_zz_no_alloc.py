"""tc_ttc_solve_noalloc (the entry point for callers that cannot allocate)
through the C ABI: bitwise the same records as tc_ttc_solve with a caller
workspace, on two calls in a row (the second on a smaller frame pair, so the
scratch array still holds the first call's larger partials), and within the
oracle bounds; too large a pair is refused before any launch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1612_08825_amd import synth
from ttc_check import check_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def _noalloc(api, prev, nxt, levels):
    from paper_1612_08825_amd import _lib as L

    lv = torch.full((levels * L.LEVEL_DTYPE.itemsize,), 0xA5, dtype=torch.uint8, device="cuda")
    pk = torch.full((L.PICK_DTYPE.itemsize,), 0x5A, dtype=torch.uint8, device="cuda")
    rc = api._lib().tc_ttc_solve_noalloc(C.byref(api._desc(prev)), C.byref(api._desc(nxt)), levels,
                                         C.c_void_p(lv.data_ptr()), C.c_void_p(pk.data_ptr()), api._stream())
    assert rc == L.TC_OK, rc
    return lv, pk


@pytest.mark.parametrize("dtype", ["u8", "f16"])
def test_noalloc_equals_workspace_entry_point(api, dtype):
    cases = [(480, 640, 4), (97, 131, 3)]  # the second call is smaller
    for case, (H, W, levels) in enumerate(cases):
        v = synth.multiscale_video(case=60 + case, H=H, W=W, F=2, foe=(W / 8, -H / 10), ttc_start=45, ttc_end=44,
                                   dtype=dtype)
        fr = torch.from_numpy(v.frames).cuda()
        lv_n, pk_n = _noalloc(api, fr[0], fr[1], levels)
        lv_w, pk_w = api.ttc_solve(fr[0], fr[1], levels)
        torch.cuda.synchronize()
        assert lv_n.cpu().numpy().tobytes() == lv_w.cpu().numpy().tobytes(), (dtype, H, W)
        assert pk_n.cpu().numpy().tobytes() == pk_w.cpu().numpy().tobytes(), (dtype, H, W)
        check_pair(api.decode_levels(lv_n), api.decode_picks(pk_n)[0], v.frames[0], v.frames[1], levels,
                   f"noalloc {dtype} {H}x{W}")


def test_noalloc_rejects_beyond_scratch(api):
    from paper_1612_08825_amd import _lib as L

    lib = api._lib()
    side, levels = 60000, 4
    # the descriptors below claim a frame far larger than the buffer behind
    # them; that is safe only because the entry point refuses the pair on the
    # host, before any launch.  Make sure of that first, on the host: the
    # pair's workspace must exceed the scratch array.
    n = C.c_size_t(0)
    assert lib.tc_ttc_workspace_size(side, side, levels, C.byref(n)) == L.TC_OK
    assert n.value > 4 * L.TC_NOALLOC_SCRATCH_BYTES, n.value
    buf = torch.zeros((2, 64, 64), dtype=torch.uint8, device="cuda")
    d0, d1 = api._desc(buf[0]), api._desc(buf[1])
    for d in (d0, d1):
        d.shape[0] = d.shape[1] = side
        d.stride[0] = side
    lv = torch.zeros(levels * L.LEVEL_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    pk = torch.zeros(L.PICK_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    rc = lib.tc_ttc_solve_noalloc(C.byref(d0), C.byref(d1), levels, C.c_void_p(lv.data_ptr()),
                                  C.c_void_p(pk.data_ptr()), api._stream())
    assert rc == L.TC_ENOMEM
    torch.cuda.synchronize()
    assert int(lv.sum()) == 0 and int(pk.sum()) == 0
