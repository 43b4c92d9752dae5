"""Graph-captured forms of the hot path, and the convolution dispatcher behind
the C ABI.

* The batched TTC plan (one persistent fused launch + the finishing launch)
  recorded into a HIP graph and replayed several times, with eager work and
  synchronisations between the replays: every replay is bitwise the eager run
  and matches the FP64 oracle (the bounds of tests/tolerance.py).
* u8 (*) int32 convolution through tc_conv_nd_ex with the caller's sum |k|:
  launch-only, so it records into a graph; every replay is bit-exact against
  the exact-integer oracle.
* tc_conv_nd_ex's method choice (direct, separable, FFT) against the oracle,
  and its rejections."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_08825_amd import synth
from tolerance import TAU_CONV, conv_bound
from ttc_check import check_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def _videos(dtype, levels):
    # uneven sizes, including a width that is not a multiple of 8 (element-wise
    # loads) and one taller than several bands
    sizes = [(120, 160), (75, 203), (240, 320), (64, 1000)] + ([(150, 90)] if dtype == "f16" else [])
    vids = []
    for i, (H, W) in enumerate(sizes):
        F = 3 + (i % 3)
        vids.append(synth.multiscale_video(case=40 + i, H=H, W=W, F=F, foe=(W / 7, -H / 9), ttc_start=50,
                                           ttc_end=40, dtype=dtype))
    return vids


@pytest.mark.parametrize("dtype,levels", [("u8", 3), ("f16", 4)])
def test_plan_graph_replay(api, dtype, levels):
    vids = _videos(dtype, levels)
    gpu = [torch.from_numpy(v.frames).cuda() for v in vids]
    tdt = torch.uint8 if dtype == "u8" else torch.float16
    plan = api.TTCPlan([api.seq_from_frames(g, levels) for g in gpu], tdt, keep=gpu)
    plan.upload()
    plan.run()
    torch.cuda.synchronize()
    eager_l, eager_p = plan.results()
    eager_l, eager_p = eager_l.copy(), eager_p.copy()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            plan.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        plan.levels_buf.fill_(0xA5)
        plan.picks_buf.fill_(0x5A)
        junk = torch.randn(1 << 20, device="cuda") * 3.0  # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        del junk
        lv, pk = plan.results()
        assert lv.tobytes() == eager_l.tobytes(), rep
        assert pk.tobytes() == eager_p.tobytes(), rep
    # the replayed records against the oracle, pair by pair
    lv, pk = plan.results()
    off = 0
    for v in vids:
        n = v.n_frames - 1
        for t in range(n):
            check_pair(lv[(off + t) * levels:(off + t + 1) * levels], pk[off + t], v.frames[t], v.frames[t + 1],
                       levels, f"graph {dtype} {v.frames.shape} t{t}")
        off += n
    del graph
    plan.close()


def test_conv_int_graph_replay(api):
    x = synth.conv_image((300, 517), case=21, dtype="u8")
    k = synth.conv_kernel((7, 7), case=21, dtype="i32")
    ref = O.conv(x, k, "full")
    xg, kg = torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda()
    out = torch.empty(ref.shape, dtype=torch.int32, device="cuda")
    kabs = int(np.abs(k.astype(np.int64)).sum())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            api.conv_nd_ex(xg, kg, "full", method="direct", k_abs_sum=kabs, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy().astype(np.int64), ref)
    del graph


def test_conv_ex_int_bound_sources(api):
    """The bound from k_abs_sum, from a host copy of k, or neither (rejected)."""
    from paper_1612_08825_amd import _lib as L

    x = synth.conv_image((64, 70), case=22, dtype="u8")
    k = synth.conv_kernel((5, 3), case=22, dtype="i32")
    ref = O.conv(x, k, "same")
    xg, kg = torch.from_numpy(x).cuda(), torch.from_numpy(k).cuda()
    y1 = api.conv_nd_ex(xg, kg, "same", k_host=k).cpu().numpy()
    y2 = api.conv_nd_ex(xg, kg, "same", k_abs_sum=int(np.abs(k).sum())).cpu().numpy()
    np.testing.assert_array_equal(y1.astype(np.int64), ref)
    np.testing.assert_array_equal(y2.astype(np.int64), ref)
    with pytest.raises(L.TTCError) as e:
        api.conv_nd_ex(xg, kg, "same")
    assert e.value.code == L.TC_EINVAL
    with pytest.raises(L.TTCError) as e:
        api.conv_nd_ex(xg, kg, "same", k_abs_sum=2147483647 // 255 + 1)
    assert e.value.code == L.TC_EOVERFLOW
    # a single tap beyond the 24-bit multiply range, still within the bound
    kb = np.zeros((3, 3), np.int32)
    kb[1, 1] = 8421504
    yb = api.conv_nd_ex(xg, torch.from_numpy(kb).cuda(), "same", k_host=kb).cpu().numpy()
    np.testing.assert_array_equal(yb.astype(np.int64), O.conv(x, kb, "same"))
    # the plain entry point never reads taps back: integer kernels are refused
    lib = api._lib()
    yy = torch.empty_like(torch.from_numpy(y1)).cuda()
    assert lib.tc_conv_nd(api.C.byref(api._desc(xg)), api.C.byref(api._desc(kg)), L.TC_SAME,
                          api.C.byref(api._desc(yy)), None) == L.TC_EINVAL


def _gauss(K, sigma):
    t = np.arange(K) - (K - 1) / 2
    g = np.exp(-t * t / (2 * sigma * sigma))
    return (g / g.sum()).astype(np.float32)


def test_conv_ex_methods(api):
    x = synth.conv_image((150, 260), case=23)
    xg = torch.from_numpy(x).cuda()
    # a general small kernel: AUTO is the direct path, bit for bit
    k = synth.conv_kernel((7, 7), case=23)
    kg = torch.from_numpy(k).cuda()
    assert torch.equal(api.conv_nd_ex(xg, kg, "full", k_host=k), api.conv_nd(xg, kg, "full"))
    # a Gaussian with a host copy: AUTO takes the separable kernel (factors by value)
    g = np.outer(_gauss(11, 2.0), _gauss(11, 2.0)).astype(np.float32)
    gg = torch.from_numpy(g).cuda()
    ya = api.conv_nd_ex(xg, gg, "same", k_host=g).cpu().numpy()
    ok, u, v = api.conv_kernel_rank1(g)
    assert ok
    ys = api.conv_nd_separable(xg, torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(), "same").cpu().numpy()
    np.testing.assert_array_equal(ya, ys)
    k64 = np.outer(u.astype(np.float64), v.astype(np.float64))
    err = np.abs(ya.astype(np.float64) - O.conv(x, k64, "same"))
    assert np.all(err <= conv_bound(x, k64, "same") + 1e-30)
    # a large kernel with a workspace: AUTO takes the FFT branch, bitwise the
    # FFT entry point, within the FFT error of the oracle
    kb = synth.conv_kernel((41, 39), case=23)
    kbg = torch.from_numpy(kb).cuda()
    yf = api.conv_nd_ex(xg, kbg, "full")
    yfft = api.conv2d_fft(xg, kbg, "full")
    assert torch.equal(yf, yfft)
    # forced direct for the same kernel agrees with the oracle element-wise
    yd = api.conv_nd_ex(xg, kbg, "full", method="direct").cpu().numpy()
    err = np.abs(yd.astype(np.float64) - O.conv(x, kb, "full"))
    assert np.all(err <= conv_bound(x, kb, "full") + 1e-30)
    # a threshold above the kernel keeps AUTO on the direct path
    yt = api.conv_nd_ex(xg, kbg, "full", fft_threshold=64)
    assert torch.equal(yt, torch.from_numpy(yd).cuda())


def test_conv_ex_fft_rejections(api):
    from paper_1612_08825_amd import _lib as L

    x16 = torch.zeros((40, 40), dtype=torch.float16, device="cuda")
    k = torch.zeros((5, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(L.TTCError) as e:
        api.conv_nd_ex(x16, k, "full", method="fft")
    assert e.value.code == L.TC_EDTYPE
    x = torch.zeros((40, 40), device="cuda")
    with pytest.raises(L.TTCError) as e:
        api.conv_nd_ex(x, k, "full", method="fft", ws=torch.zeros(16, dtype=torch.uint8, device="cuda"))
    assert e.value.code == L.TC_ENOMEM
