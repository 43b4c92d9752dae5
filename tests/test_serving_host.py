"""Serving scheduler on the CPU with a fake executor and a fake clock:
admission against the device-memory budget, back-pressure, eviction and
re-priming, per-stream ordering, the ring-buffer reuse rule, cancellation, and
the statistics of the Poisson arrival generator."""
import math

import numpy as np
import pytest

from paper_1612_08825_amd import serving as S
from paper_1612_08825_amd import synth


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a batch ``base + per_px * pixels`` seconds after its launch,
    one batch at a time in launch order, and checks the ring-buffer rule: no
    frame buffer is written while an unfinished request still reads it."""

    def __init__(self, clock, sched, base=50e-6, per_px=1e-12):
        self.clock, self.sched, self.base, self.per_px = clock, sched, base, per_px
        self.busy_until = 0.0
        self.queue = []
        self.reading = {}     # (stream, slot id, buffer) -> count of unfinished readers
        self.alloc_ids = 0
        self.live = set()
        self.launched = []

    def allocate(self, s):
        self.alloc_ids += 1
        self.live.add(self.alloc_ids)
        return self.alloc_ids

    def release(self, s):
        assert s.inflight == 0
        self.live.discard(s.slot)

    def _bufs(self, r, s):
        ring = self.sched.ring
        reads = [(s.sid, s.slot, r.k % ring)]
        if r.kind == S.PAIR:
            reads.append((s.sid, s.slot, (r.k - 1) % ring))
        return reads

    def launch(self, batch, sched):
        assert len({r.stream for r in batch}) == len(batch), "two requests of one stream in a batch"
        px = 0
        for r in batch:
            s = sched.streams[r.stream]
            assert s.slot in self.live
            write = (s.sid, s.slot, r.k % sched.ring)
            assert self.reading.get(write, 0) == 0, "ring buffer overwritten while read"
            for b in self._bufs(r, s):
                self.reading[b] = self.reading.get(b, 0) + 1
            if r.kind == S.PAIR:
                px += s.H * s.W
        start = max(self.clock(), self.busy_until)
        self.busy_until = start + self.base + self.per_px * px
        h = (self.busy_until, [(r, sched.streams[r.stream].slot) for r in batch])
        self.launched.append(batch)
        return h

    def done(self, h):
        return self.clock() >= h[0]

    def collect(self, h, batch):
        for r, slot in h[1]:
            s = self.sched.streams[r.stream]
            ring = self.sched.ring
            for b in [(s.sid, slot, r.k % ring)] + ([(s.sid, slot, (r.k - 1) % ring)] if r.kind == S.PAIR else []):
                self.reading[b] -= 1
            r.status = S.TC_NEED_PREV if r.kind == S.PRIME else 0

    def next_done(self):
        return self.busy_until


def run(sizes, budget, times, ids, max_inflight=2, **kw):
    clock = FakeClock()
    sched = S.Scheduler(sizes, budget, **kw)
    ex = FakeExecutor(clock, sched)

    def idle(nxt):
        cand = [nxt]
        if ex.busy_until > clock.t:
            cand.append(ex.busy_until)
        t = min(cand)
        assert math.isfinite(t), "idle with nothing to wait for"
        clock.t = max(clock.t, t)

    stats = S.run_open_loop(sched, ex, times, ids, clock=clock, idle=idle, max_inflight=max_inflight)
    return sched, ex, stats


def check_order(reqs, sched):
    by = {}
    for r in reqs:
        by.setdefault(r.stream, []).append(r)
    for sid, rs in by.items():
        rs.sort(key=lambda r: r.rid)
        launches = [r.t_launch for r in rs]
        assert launches == sorted(launches), "stream served out of order"
        dones = [r.t_done for r in rs]
        assert dones == sorted(dones)
        # frame numbers count up from each (re-)priming
        for a, b in zip(rs, rs[1:]):
            assert b.k == a.k + 1 or b.k == 0
        assert rs[0].k == 0 and rs[0].kind == S.PRIME


def test_poisson_statistics():
    rate, dur, n = 20000.0, 2.0, 256
    t, ids = synth.poisson_arrivals(rate, dur, n, case=3)
    assert abs(t.size - rate * dur) < 5 * math.sqrt(rate * dur)
    gaps = np.diff(t)
    assert abs(gaps.mean() * rate - 1) < 0.02
    # exponential gaps: coefficient of variation 1, P(gap > mean) = e^-1
    assert abs(gaps.std() / gaps.mean() - 1) < 0.03
    assert abs((gaps > 1 / rate).mean() - math.exp(-1)) < 0.01
    # streams uniform: chi-square with 255 degrees of freedom, far tail cut
    counts = np.bincount(ids, minlength=n)
    chi2 = ((counts - t.size / n) ** 2 / (t.size / n)).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)
    assert np.all(np.diff(t) >= 0) and t[-1] < dur


def test_all_admitted_every_request_answered_in_order():
    sizes = [(240, 320), (480, 640), (720, 1280), (1080, 1920)] * 4
    t, ids = synth.poisson_arrivals(4000.0, 0.5, len(sizes), case=7)
    sched, ex, st = run(sizes, 1 << 31, t, ids)
    reqs = st.requests
    assert all(not math.isnan(r.t_done) for r in reqs)
    assert sched.evictions == 0 and sched.admissions == len(set(ids.tolist()))
    check_order(reqs, sched)
    assert sum(r.kind == S.PRIME for r in reqs) == len(set(ids.tolist()))
    assert sched.peak_bytes <= sched.budget
    assert max(st.batch_sizes) > 1, "no batching happened"
    lat = S.latency_summary(reqs)
    assert lat["n"] == sum(r.kind == S.PAIR for r in reqs) and lat["p50_ms"] > 0


def test_budget_below_working_set_queues_and_evicts():
    sizes = [(480, 640)] * 8
    one = S.slot_bytes(480, 640, 3)
    t, ids = synth.poisson_arrivals(3000.0, 0.3, 8, case=11)
    sched, ex, st = run(sizes, 2 * one + 100, t, ids)
    reqs = st.requests
    assert all(not math.isnan(r.t_done) for r in reqs), "a request was never answered"
    assert sched.peak_bytes <= sched.budget
    assert sched.evictions > 0
    check_order(reqs, sched)
    # each eviction costs a re-priming request
    primes = sum(r.kind == S.PRIME for r in reqs)
    assert primes == sched.admissions
    # under a budget that holds every stream nothing is re-primed
    big, _, st_big = run(sizes, 1 << 30, t, ids)
    assert big.evictions == 0
    assert sum(r.kind == S.PAIR for r in st_big.requests) > sum(r.kind == S.PAIR for r in reqs)


def test_ring_rule_limits_requests_in_flight_per_stream():
    # one stream, a burst of requests: never more than ring - 1 on the device
    t = np.zeros(40)
    ids = np.zeros(40, dtype=np.int64)
    for ring in (3, 4):
        sched, ex, st = run([(64, 64)], 1 << 20, t, ids, max_inflight=4, ring=ring)
        for b in ex.launched:
            assert len(b) == 1
        # at any launch, requests of the stream still unfinished
        for r in st.requests:
            overlapping = [q for q in st.requests if q.t_launch <= r.t_launch < q.t_done and q is not r]
            assert len(overlapping) <= ring - 2
        check_order(st.requests, sched)


def test_rejected_stream_larger_than_budget():
    sizes = [(1080, 1920), (240, 320)]
    budget = S.slot_bytes(240, 320, 3) * 2
    t = np.array([0.0, 0.0, 1e-3, 2e-3])
    ids = np.array([0, 1, 0, 1])
    sched, ex, st = run(sizes, budget, t, ids)
    assert [r.status for r in st.requests if r.stream == 0] == [S.REJECTED, S.REJECTED]
    assert [r.kind for r in st.requests if r.stream == 1] == [S.PRIME, S.PAIR]


def test_cancel_drops_queued_and_releases_after_inflight():
    clock = FakeClock()
    sched = S.Scheduler([(64, 64), (64, 64)], 1 << 20)
    ex = FakeExecutor(clock, sched, base=1e-3)
    reqs = [S.Request(i, 0, 0.0) for i in range(5)] + [S.Request(5, 1, 0.0)]
    for r in reqs:
        sched.submit(r, 0.0)
    b = sched.form_batch(0.0, ex)
    assert {r.stream for r in b} == {0, 1}
    h = ex.launch(b, sched)
    dropped = sched.cancel(0, 0.0, ex)
    assert len(dropped) == 4 and all(r.status == S.CANCELLED for r in dropped)
    assert sched.streams[0].admitted and sched.streams[0].cancel_pending
    clock.t = 1.0
    assert ex.done(h)
    ex.collect(h, b)
    sched.finish(b, 1.0, ex)
    assert not sched.streams[0].admitted
    assert sched.bytes_used == sched.streams[1].nbytes
    # cancel of an idle admitted stream releases at once
    sched.cancel(1, 1.0, ex)
    assert sched.bytes_used == 0 and sched.pending() == 0


def test_starving_stream_preempts_busy_streams():
    # two streams fit; a third waits, and under steady load on the first two
    # it still gets in after the preemption delay
    sizes = [(64, 64)] * 3
    one = S.slot_bytes(64, 64, 3)
    n = 600
    t = np.arange(n) * 1e-4
    ids = np.array([0, 1] * (n // 2))
    ids[5] = 2
    sched, ex, st = run(sizes, 2 * one, t, ids, preempt_after=2e-3)
    r2 = [r for r in st.requests if r.stream == 2]
    assert r2[0].t_done - r2[0].t_arrival < 0.01
    assert sched.evictions >= 1
    check_order(st.requests, sched)
