"""The serving loop on the GPU: every answered pair matches the FP64 oracle,
each stream's answers are bitwise the same served alone and in the mix, and a
device-memory budget below the working set still answers everything (with
re-priming after evictions)."""
import math

import numpy as np
import pytest
import torch

from paper_1612_08825_amd import serving as S
from paper_1612_08825_amd import synth
from ttc_check import check_pair

pytestmark = pytest.mark.gpu

LEVELS = 3
SIZES = [(64, 48), (80, 60), (128, 96), (160, 120), (72, 64), (100, 52)]  # (W, H)
N_FRAMES = 6


@pytest.fixture(scope="module")
def streams(gpu_lib):
    specs = synth.serving_specs(case=2, n_streams=len(SIZES), n_frames=N_FRAMES, sizes=SIZES)
    host = []
    for sp in specs:
        t = torch.from_numpy(np.ascontiguousarray(sp.render())).pin_memory()
        host.append(t)
    return specs, host


def serve(host, sizes, times, ids, budget=1 << 30, max_inflight=2):
    sched = S.Scheduler(sizes, budget)
    ex = S.GpuExecutor(host, levels=LEVELS, max_inflight=max_inflight)
    st = S.run_open_loop(sched, ex, times, ids, max_inflight=max_inflight)
    torch.cuda.synchronize()
    return sched, st


def interleaved(n_streams, per_stream, gap=2e-5):
    ids = np.tile(np.arange(n_streams), per_stream)
    return np.arange(ids.size) * gap, ids


def test_served_pairs_match_oracle(streams):
    specs, host = streams
    sizes = [tuple(h.shape[1:]) for h in host]
    # one more request than frames: the last pair wraps to frame 0
    times, ids = interleaved(len(host), N_FRAMES + 1)
    sched, st = serve(host, sizes, times, ids)
    n_pairs = 0
    for r in st.requests:
        assert not math.isnan(r.t_done)
        if r.kind == S.PRIME:
            assert r.status == S.TC_NEED_PREV and r.k == 0
            continue
        fr = host[r.stream].numpy()
        P0, P1 = fr[(r.k - 1) % N_FRAMES], fr[r.k % N_FRAMES]
        check_pair(r.levels, r.pick, P0, P1, LEVELS, f"stream{r.stream} k{r.k}")
        n_pairs += 1
    assert n_pairs == len(host) * N_FRAMES
    print(f"[serve] {n_pairs} pairs in {st.batches} batches, sizes {st.batch_sizes[:12]}")


def test_alone_equals_mix(streams):
    specs, host = streams
    sizes = [tuple(h.shape[1:]) for h in host]
    times, ids = interleaved(len(host), N_FRAMES)
    _, mix = serve(host, sizes, times, ids)
    assert max(mix.batch_sizes) > 1
    for sid in range(len(host)):
        m = [r for r in mix.requests if r.stream == sid and r.kind == S.PAIR]
        t1 = np.arange(N_FRAMES) * 1e-4
        _, alone = serve([host[sid]], [sizes[sid]], t1, np.zeros(N_FRAMES, dtype=np.int64))
        a = [r for r in alone.requests if r.kind == S.PAIR]
        assert [r.k for r in a] == [r.k for r in m]
        for ra, rm in zip(a, m):
            assert ra.pick.tobytes() == rm.pick.tobytes(), (sid, ra.k)
            assert ra.levels.tobytes() == rm.levels.tobytes(), (sid, ra.k)


def test_budget_below_working_set(streams):
    specs, host = streams
    sizes = [tuple(h.shape[1:]) for h in host]
    one = max(S.slot_bytes(H, W, 3) for H, W in sizes)
    times, ids = interleaved(len(host), N_FRAMES, gap=5e-5)
    sched, st = serve(host, sizes, times, ids, budget=2 * one)
    assert sched.evictions > 0 and sched.peak_bytes <= 2 * one
    for r in st.requests:
        assert not math.isnan(r.t_done)
        if r.kind == S.PAIR:
            fr = host[r.stream].numpy()
            check_pair(r.levels, r.pick, fr[(r.k - 1) % N_FRAMES], fr[r.k % N_FRAMES], LEVELS,
                       f"budget stream{r.stream} k{r.k}")


def test_served_pairs_at_camera_sizes(gpu_lib):
    """u8 frames, 3 levels, the library's u8 launch shape (what the serving
    workload runs) at the two largest camera sizes: every served pair against
    the FP64 oracle, and the streams served together equal to served alone."""
    sizes = [(1280, 720), (1920, 1080)]  # (W, H)
    nf = 3
    specs = [synth.serving_specs(case=7 + i, n_streams=1, n_frames=nf, sizes=[sz])[0] for i, sz in enumerate(sizes)]
    host = [torch.from_numpy(np.ascontiguousarray(sp.render())).pin_memory() for sp in specs]
    hw = [tuple(h.shape[1:]) for h in host]
    assert sorted(hw) == [(720, 1280), (1080, 1920)]
    times, ids = interleaved(len(host), nf)
    _, st = serve(host, hw, times, ids)
    n_pairs = 0
    for r in st.requests:
        assert not math.isnan(r.t_done)
        if r.kind != S.PAIR:
            continue
        fr = host[r.stream].numpy()
        check_pair(r.levels, r.pick, fr[(r.k - 1) % nf], fr[r.k % nf], LEVELS, f"{hw[r.stream]} k{r.k}")
        n_pairs += 1
    assert n_pairs == len(host) * (nf - 1)
    for sid in range(len(host)):
        _, alone = serve([host[sid]], [hw[sid]], np.arange(nf) * 1e-4, np.zeros(nf, dtype=np.int64))
        a = [r for r in alone.requests if r.kind == S.PAIR]
        m = [r for r in st.requests if r.stream == sid and r.kind == S.PAIR]
        for ra, rm in zip(a, m):
            assert ra.levels.tobytes() == rm.levels.tobytes() and ra.pick.tobytes() == rm.pick.tobytes()
