"""GPU parity of the fused time-to-contact path (tc_ttc_solve, the batched
plan) against the FP64 oracle.

Per level: every sum within TAU_SUM * sum|terms| of the oracle's; A, B, C,
TTC, FOE within the first-order propagation of those bounds through the 3x3
solve (tests/tolerance.py); statuses equal; the multi-scale choice equal
wherever neighbouring levels are not within tolerance of a tie."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1612_08825_amd import synth
from tolerance import TAU_SUM, abs_sums, solution_bounds
from ttc_check import WORST, _frames_np, check_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api(gpu_lib):
    from paper_1612_08825_amd import api

    return api


def test_plain_video_single_pairs(api):
    """The 8-frame 128x128 u8 video, one tc_ttc_solve call per pair, 1 level."""
    v = synth.plain_ttc_video()
    fr = torch.from_numpy(v.frames).cuda()
    for t in range(v.n_frames - 1):
        lv, pk = api.ttc_solve(fr[t], fr[t + 1], 1)
        rec = api.decode_levels(lv)
        pick = api.decode_picks(pk)[0]
        check_pair(rec, pick, v.frames[t], v.frames[t + 1], 1, f"pair{t}")
        assert abs(rec[0]["ttc"] - 40.0) < 2.0  # the analytic ground truth is 40 frames
    print(f"[ttc plain] worst sum err/sum|t| {WORST['sum']:.2e} rel C {WORST['C']:.2e} foe {WORST['foe']:.2e}")


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_plain_video_batched_levels(api, levels):
    v = synth.plain_ttc_video(F=8)
    fr = torch.from_numpy(v.frames).cuda()
    recs, picks = api.ttc_solve_batched([fr], levels)
    assert recs.shape == (7 * levels,) and picks.shape == (7,)
    for t in range(7):
        check_pair(recs[t * levels:(t + 1) * levels], picks[t], v.frames[t], v.frames[t + 1], levels, f"t{t}")


@pytest.mark.parametrize("H,W,levels,dtype", [(97, 131, 3, "u8"), (130, 250, 4, "f16"), (67, 700, 2, "u8"),
                                              (200, 489, 4, "u8"), (16, 16, 4, "f16"), (171, 1000, 1, "f16"),
                                              (9, 9, 1, "u8")])
def test_ragged_sizes(api, H, W, levels, dtype):
    v = synth.multiscale_video(H=H, W=W, F=3, foe=(W / 10, -H / 12), ttc_start=40, ttc_end=35, dtype=dtype)
    fr = torch.from_numpy(v.frames).cuda()
    recs, picks = api.ttc_solve_batched([fr], levels)
    for t in range(2):
        check_pair(recs[t * levels:(t + 1) * levels], picks[t], v.frames[t], v.frames[t + 1], levels, f"{H}x{W}")


@pytest.mark.parametrize("W", [64, 65, 71, 72, 505, 511, 512, 513, 519, 1008, 1009, 1016, 1023])
@pytest.mark.parametrize("dtype", ["u8", "f16"])
def test_edge_columns_every_residue(api, W, dtype):
    """Widths around lane and column-wave boundaries, every residue mod 8: the
    lane at the right edge lacks only its last cube column at each level when
    W is a multiple of 8 (that column alone is masked) and other sets
    otherwise (every column checked)."""
    H = 40
    v = synth.multiscale_video(H=H, W=W, F=3, foe=(W / 7, -H / 9), ttc_start=45, ttc_end=40, dtype=dtype)
    fr = torch.from_numpy(v.frames).cuda()
    recs, picks = api.ttc_solve_batched([fr], 4)
    for t in range(2):
        check_pair(recs[t * 4:(t + 1) * 4], picks[t], v.frames[t], v.frames[t + 1], 4, f"{H}x{W}")


def test_batch_mix_equals_alone(api):
    """Streams of uneven sizes in one plan: each pair equals the oracle, and the
    records are bit-identical to running each stream alone."""
    sizes = [(60, 80), (240, 320), (123, 517), (48, 1000), (480, 640)]
    vids = []
    for i, (H, W) in enumerate(sizes):
        v = synth.multiscale_video(case=i, H=H, W=W, F=4, foe=(W / 9, H / 11), ttc_start=60, ttc_end=50)
        vids.append(v)
    gpu = [torch.from_numpy(v.frames).cuda() for v in vids]
    recs, picks = api.ttc_solve_batched(gpu, 3)
    off = 0
    for v, g in zip(vids, gpu):
        n = v.n_frames - 1
        alone, alone_p = api.ttc_solve_batched([g], 3)
        assert alone.tobytes() == recs[off * 3:(off + n) * 3].tobytes()
        assert alone_p.tobytes() == picks[off:off + n].tobytes()
        for t in range(n):
            check_pair(recs[(off + t) * 3:(off + t + 1) * 3], picks[off + t], v.frames[t], v.frames[t + 1], 3)
        off += n


def test_pairs_as_two_frame_streams(api):
    """Unrelated prev/next buffers described by frame_stride = next - prev."""
    v = synth.multiscale_video(H=100, W=150, F=2, foe=(5, 5), ttc_start=50, ttc_end=49)
    a = torch.from_numpy(v.frames[0]).cuda()
    junk = torch.empty(12345, dtype=torch.uint8, device="cuda")
    b = torch.from_numpy(v.frames[1]).cuda()
    del junk
    plan = api.TTCPlan([api.seq_from_pair(a, b, 2)], torch.uint8, keep=[a, b])
    plan.run()
    torch.cuda.synchronize()
    recs, picks = plan.results()
    plan.close()
    check_pair(recs, picks[0], v.frames[0], v.frames[1], 2, "pair-stream")


def test_symmetric_video(api):
    v = synth.plain_ttc_video(H=64, W=80, F=2, symmetric=True)
    fr = torch.from_numpy(v.frames).cuda()
    recs, _ = api.ttc_solve_batched([fr], 3)
    for l in range(3):
        r = recs[l]
        ref = O.ttc_pair(v.frames[0], v.frames[1], 3)[l]
        assert ref["A"] == 0.0 and ref["B"] == 0.0
        p0 = O.pyramid(v.frames[0], 3)[l]
        p1 = O.pyramid(v.frames[1], 3)[l]
        b = solution_bounds(ref["sums"], abs_sums(p0, p1, l, 64, 80))
        assert abs(r["A"]) <= b["A"] and abs(r["B"]) <= b["B"]


def test_ramp_is_singular_and_nan_is_nonfinite(api):
    i, j = np.meshgrid(np.arange(32), np.arange(48), indexing="ij")
    ramp = np.stack([(2 * j + i + 20 + 3 * t).astype(np.uint8) for t in range(2)])
    recs, picks = api.ttc_solve_batched([torch.from_numpy(ramp).cuda()], 2)
    assert all(r["status"] == O.STATUS_SINGULAR for r in recs)
    assert math.isnan(picks[0]["ttc"])
    v = synth.plain_ttc_video(H=32, W=32, F=2, dtype="f16")
    f = v.frames.copy()
    f[1, 5, 7] = np.float16(np.nan)
    recs, picks = api.ttc_solve_batched([torch.from_numpy(f).cuda()], 1)
    assert recs[0]["status"] == O.STATUS_NONFINITE


def test_multiscale_video_sampled(api):
    """The 300-frame 640x480 u8 multi-scale video (4 levels): every pair on the
    GPU in one pass, a sample of pairs against the oracle."""
    v = synth.multiscale_video(device="cuda")
    fr = v.frames
    recs, picks = api.ttc_solve_batched([fr], 4)
    assert recs.shape == (299 * 4,)
    host = fr.cpu().numpy()
    for t in (0, 57, 150, 298):
        check_pair(recs[t * 4:(t + 1) * 4], picks[t], host[t], host[t + 1], 4, f"ms{t}")
    print(f"[ttc multiscale] worst sum err/sum|t| {WORST['sum']:.2e} rel C {WORST['C']:.2e} foe {WORST['foe']:.2e}")


def test_batched_workload_sampled(api):
    """64 streams of uneven sizes, 16 f16 frames each, 4 levels, in one plan;
    sampled pairs against the oracle."""
    specs = synth.batched_specs()
    vids = [s.render(device="cuda") for s in specs]
    recs, picks = api.ttc_solve_batched(vids, 4)
    assert picks.shape == (64 * 15,)
    big = max(range(64), key=lambda i: specs[i].H * specs[i].W)
    small = min(range(64), key=lambda i: specs[i].H * specs[i].W)
    # one stream of every size: each size gets its own column-strip shape
    # (1920 and 320 wide one 504-column strip per wave, 640 two of 248, 1280 three of 160)
    first = {}
    for i, s in enumerate(specs):
        first.setdefault((s.W, s.H), i)
    assert len(first) == 4
    samples = [(big, 7), (small, 0), (5, 14)] + [(i, 3) for i in first.values() if i not in (big, small)]
    for s_i, t in samples:
        host = vids[s_i].cpu().numpy()
        g = s_i * 15 + t
        check_pair(recs[g * 4:(g + 1) * 4], picks[g], host[t], host[t + 1], 4, f"stream{s_i}")
    print(f"[ttc batched] worst sum err/sum|t| {WORST['sum']:.2e} rel C {WORST['C']:.2e} foe {WORST['foe']:.2e}")


def _small_batch(dtype, case):
    specs = synth.stream_specs(4, 3, 4, dtype, sizes=[(160, 120), (200, 96), (136, 80)], case=case)
    return specs, [torch.from_numpy(np.ascontiguousarray(s.render())).cuda() for s in specs]


@pytest.mark.parametrize("dtype,levels", [("u8", 3), ("f16", 4)])
def test_every_tuning_candidate(api, dtype, levels):
    """Work-groups per CU never change a result (bitwise); every band height
    stays within the oracle tolerance."""
    specs, vids = _small_batch(dtype, 9)
    # and one stream tall enough for several full bands at every height (the
    # unchecked walk with its inner loop) besides the bottom band
    tall = synth.stream_specs(4, 1, 3, dtype, sizes=[(700, 300)], case=10)
    specs = list(specs) + tall
    vids = list(vids) + [torch.from_numpy(np.ascontiguousarray(tall[0].render())).cuda()]
    for rows in (16, 32, 64, 128):
        ref = None
        for gpc in (1, 8, 64, 256):
            recs, picks = api.ttc_solve_batched(vids, levels, tuning=(rows, gpc))
            if ref is None:
                ref = (recs.tobytes(), picks.tobytes())
                q = 0
                for s, v in zip(specs, vids):
                    fr = _frames_np(v)
                    for t in range(fr.shape[0] - 1):
                        check_pair(recs[q * levels:(q + 1) * levels], picks[q], fr[t], fr[t + 1], levels,
                                   f"rows{rows} {s.W}x{s.H} pair{t}")
                        q += 1
            else:
                assert (recs.tobytes(), picks.tobytes()) == ref, (rows, gpc)


def test_plan_reset_matches_fresh_plan(api):
    _, a = _small_batch("u8", 21)
    specsb, b = _small_batch("u8", 22)
    b = b[:2]
    plan = api.TTCPlan([api.seq_from_frames(v, 3) for v in a], torch.uint8, keep=a)
    plan.run()
    torch.cuda.synchronize()
    ra = [x.tobytes() for x in plan.results()]
    plan.reset([api.seq_from_frames(v, 3) for v in b], keep=b)
    plan.run()
    torch.cuda.synchronize()
    rb = [x.tobytes() for x in plan.results()]
    fresh = [x.tobytes() for x in api.ttc_solve_batched(b, 3)]
    assert rb == fresh
    plan.reset([api.seq_from_frames(v, 3) for v in a], keep=a)
    plan.run()
    torch.cuda.synchronize()
    assert [x.tobytes() for x in plan.results()] == ra
    plan.close()


def _resid_tol(r, a):
    """The residual bound of check_pair, per cube."""
    return (1e-3 * abs(r["resid"]) + 1e-6 * a[9]) / r["n"]


@pytest.mark.parametrize("dtype,case", [("u8", 31), ("f16", 32)])
def test_reselect_rules(api, dtype, case):
    """tc_ttc_reselect on a plan's device records: the decreasing-TTC rule
    reproduces the plan's own picks bitwise; the residual rule equals the
    oracle's rule applied to the same device records (exact decisions on the
    same numbers), and the oracle's rule on its own records wherever no two
    valid levels are within tolerance of a tie."""
    levels = 4
    specs, vids = _small_batch(dtype, case)
    plan = api.TTCPlan([api.seq_from_frames(v, levels) for v in vids], vids[0].dtype, keep=vids)
    plan.run()
    n = plan.n_pairs
    p0 = api.ttc_reselect(plan.levels_buf, n, levels, "decreasing_ttc")
    p1 = api.ttc_reselect(plan.levels_buf, n, levels, "min_residual")
    torch.cuda.synchronize()
    recs, picks = plan.results()
    assert api.decode_picks(p0[: n * 56]).tobytes() == picks.tobytes()
    got = api.decode_picks(p1[: n * 56])
    q = 0
    differs = 0
    for s, v in zip(specs, vids):
        fr = _frames_np(v)
        for t in range(fr.shape[0] - 1):
            rec = recs[q * levels:(q + 1) * levels]
            dev = [{k: rec[l][k] for k in ("ttc", "status", "resid", "n")} for l in range(levels)]
            l1 = O.select_level_residual(dev)
            assert got[q]["level"] == l1
            for k in ("ttc", "x0", "y0", "A", "B", "C", "status"):
                assert got[q][k].tobytes() == rec[l1][k].tobytes(), (q, k)
            differs += int(l1 != picks[q]["level"])
            ref = O.ttc_pair(fr[t], fr[t + 1], levels)
            pa, pb = O.pyramid(fr[t], levels), O.pyramid(fr[t + 1], levels)
            valid = [l for l in range(levels) if ref[l]["status"] == 0 and ref[l]["ttc"] > 0]
            per = {l: (ref[l]["resid"] / ref[l]["n"], _resid_tol(ref[l], abs_sums(pa[l], pb[l], l, *fr[t].shape)))
                   for l in valid}
            tie = any(abs(per[i][0] - per[j][0]) <= per[i][1] + per[j][1] for i in valid for j in valid if i < j)
            if not tie:
                assert l1 == O.select_level_residual(ref), (q, per)
            q += 1
    assert q == n
    print(f"[reselect {dtype}] {n} pairs, the residual rule picks another level on {differs}")


def test_reselect_rejections(api):
    from paper_1612_08825_amd import _lib as L

    lib = api._lib()
    buf = torch.zeros(4 * 152, dtype=torch.uint8, device="cuda")
    out = torch.zeros(56, dtype=torch.uint8, device="cuda")
    ptr = buf.data_ptr()
    assert lib.tc_ttc_reselect(ptr, 1, 4, 2, out.data_ptr(), None) == L.TC_EINVAL
    assert lib.tc_ttc_reselect(ptr, 1, 0, 0, out.data_ptr(), None) == L.TC_EINVAL
    assert lib.tc_ttc_reselect(ptr, -1, 4, 0, out.data_ptr(), None) == L.TC_EINVAL
    assert lib.tc_ttc_reselect(None, 1, 4, 0, out.data_ptr(), None) == L.TC_EINVAL
    assert lib.tc_ttc_reselect(None, 0, 4, 0, None, None) == L.TC_OK
