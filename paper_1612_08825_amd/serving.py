"""Continuous-batching TTC server for many camera streams (frame-pair form).

A request carries one new frame of one stream.  Its answer is the multi-scale
time to contact and focus of expansion of the pair (the stream's previous
frame, the new frame): the least-squares fit of the Formulation under Time to
Contact, at every pyramid level, with the level chosen by the multi-scale
search of the Results section.  The first frame of a stream (or the first after
its state was evicted) only primes it and is answered TC_NEED_PREV.

Three parts:

* ``Scheduler`` -- host logic only (no torch): per-stream FIFO queues,
  admission of streams against a device-memory budget (each admitted stream
  holds a ring of ``ring`` frame buffers on the device), eviction of idle
  streams in least-recently-used order when others wait, per-stream ordering,
  and batch formation (at most one request per stream per batch).
* ``GpuExecutor`` -- one batch = host-to-device copies of the new frames on a
  copy stream, then on a compute stream one re-planned persistent fused launch
  plus the finishing launch over every pair in the batch, then a
  device-to-host copy of the results; completion is an event the loop polls.
* ``run_open_loop`` -- the request loop: arrivals are admitted as they come
  (open loop, timestamps fixed in advance), a new batch is launched whenever
  fewer than ``max_inflight`` batches are on the device, so requests that
  arrive while others are being computed go into the next batch and overlap
  with it.  Latency = result in host memory - arrival time.

Frame ``k`` of a stream lives in ring buffer ``k % ring``.  Request ``k``
writes buffer ``k % ring`` and reads ``(k-1) % ring``; the buffer it writes
was last read by request ``k - ring + 1``, so a stream may have at most
``ring - 2`` requests on the device when another is launched.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np

TC_NEED_PREV = 2  # library status: first frame of a stream, no pair yet
CANCELLED = -100  # request dropped by cancel() before it was launched
REJECTED = -101   # stream state larger than the whole budget

PRIME = 0
PAIR = 1


@dataclass
class Request:
    rid: int
    stream: int
    t_arrival: float
    k: int = -1                 # frame number within the stream, set at launch
    kind: int = -1              # PRIME or PAIR
    t_launch: float = math.nan
    t_done: float = math.nan
    status: int = -1            # library status of the pick, or CANCELLED / REJECTED
    pick: Optional[np.void] = None
    levels: Optional[np.ndarray] = None


@dataclass
class StreamState:
    sid: int
    H: int
    W: int
    nbytes: int
    queue: Deque[Request] = field(default_factory=collections.deque)
    admitted: bool = False
    waiting: bool = False       # in the admission queue
    last_k: int = -1            # frame number of the last launched frame (-1: none resident)
    inflight: int = 0
    last_used: float = 0.0
    cancel_pending: bool = False
    slot: object = None         # executor's device buffers


def slot_bytes(H: int, W: int, ring: int, elem: int = 1, align: int = 256) -> int:
    """Device bytes one admitted stream holds: ``ring`` frames of H x W."""
    one = (H * W * elem + align - 1) // align * align
    return ring * one


class Scheduler:
    """Admission, ordering and batch formation; knows nothing of the device."""

    def __init__(self, sizes: Sequence[Tuple[int, int]], budget_bytes: int, ring: int = 3,
                 max_batch: int = 512, elem: int = 1, preempt_after: float = 0.05):
        if ring < 3:
            raise ValueError("ring must hold at least 3 frames")
        self.ring = ring
        self.preempt_after = preempt_after
        self.max_batch = max_batch
        self.budget = int(budget_bytes)
        self.streams = [StreamState(i, H, W, slot_bytes(H, W, ring, elem)) for i, (H, W) in enumerate(sizes)]
        self.bytes_used = 0
        self.admit_queue: Deque[int] = collections.deque()
        self.evictions = 0
        self.admissions = 0
        self.rejected = 0
        self.peak_bytes = 0
        self._queued = 0
        self._ready: Dict[int, None] = {}   # admitted streams with queued requests (insertion-ordered)

    # ---- arrivals -----------------------------------------------------------
    def submit(self, req: Request, now: float) -> None:
        s = self.streams[req.stream]
        if s.nbytes > self.budget:
            req.status = REJECTED
            req.t_done = now
            self.rejected += 1
            return
        s.queue.append(req)
        self._queued += 1
        if s.admitted:
            self._ready[s.sid] = None
        elif not s.waiting:
            s.waiting = True
            self.admit_queue.append(s.sid)

    def cancel(self, sid: int, now: float, executor) -> List[Request]:
        """Drops the stream's queued requests; its device state is released once
        nothing of it is on the device.  Returns the dropped requests."""
        s = self.streams[sid]
        dropped = list(s.queue)
        for r in dropped:
            r.status = CANCELLED
            r.t_done = now
        self._queued -= len(dropped)
        s.queue.clear()
        self._ready.pop(sid, None)
        if s.waiting:
            self.admit_queue.remove(sid)
            s.waiting = False
        if s.admitted:
            if s.inflight == 0:
                self._release(s, executor)
            else:
                s.cancel_pending = True
        return dropped

    def pending(self) -> int:
        return self._queued

    def next_deadline(self) -> float:
        """When the stream at the head of the admission queue may preempt others."""
        if not self.admit_queue:
            return math.inf
        return self.streams[self.admit_queue[0]].queue[0].t_arrival + self.preempt_after

    # ---- admission ------------------------------------------------------------
    def _release(self, s: StreamState, executor) -> None:
        executor.release(s)
        s.slot = None
        s.admitted = False
        s.last_k = -1
        s.cancel_pending = False
        self.bytes_used -= s.nbytes

    def _evictable(self, busy_too: bool = False) -> List[StreamState]:
        """Admitted streams with nothing on the device, least recently used
        first; idle ones (empty queue) before busy ones when ``busy_too``."""
        idle = sorted((s for s in self.streams if s.admitted and s.inflight == 0 and not s.queue),
                      key=lambda s: s.last_used)
        if not busy_too:
            return idle
        busy = sorted((s for s in self.streams if s.admitted and s.inflight == 0 and s.queue),
                      key=lambda s: s.last_used)
        return idle + busy

    def _admit(self, now: float, executor) -> None:
        while self.admit_queue:
            s = self.streams[self.admit_queue[0]]
            if self.bytes_used + s.nbytes > self.budget:
                need = self.bytes_used + s.nbytes - self.budget
                # a stream that has waited too long may push out streams that
                # still have requests queued (they go back to the admission queue)
                starving = now - s.queue[0].t_arrival > self.preempt_after
                victims, freed = [], 0
                for v in self._evictable(busy_too=starving):
                    if freed >= need:
                        break
                    victims.append(v)
                    freed += v.nbytes
                if freed < need:
                    return          # head of line waits: no starvation of large streams
                for v in victims:
                    self._release(v, executor)
                    self.evictions += 1
                    if v.queue:
                        self._ready.pop(v.sid, None)
                        v.waiting = True
                        self.admit_queue.append(v.sid)
            self.admit_queue.popleft()
            s.waiting = False
            s.slot = executor.allocate(s)
            s.admitted = True
            s.last_k = -1
            self.bytes_used += s.nbytes
            self.peak_bytes = max(self.peak_bytes, self.bytes_used)
            self.admissions += 1
            if s.queue:
                self._ready[s.sid] = None

    # ---- batches --------------------------------------------------------------
    def form_batch(self, now: float, executor) -> List[Request]:
        self._admit(now, executor)
        batch: List[Request] = []
        done_ids = []
        for sid in self._ready:
            if len(batch) >= self.max_batch:
                break
            s = self.streams[sid]
            if s.inflight > self.ring - 2:
                continue
            r = s.queue.popleft()
            self._queued -= 1
            r.k = s.last_k + 1
            r.kind = PRIME if r.k == 0 else PAIR
            r.t_launch = now
            s.last_k = r.k
            s.inflight += 1
            s.last_used = now
            batch.append(r)
            if not s.queue:
                done_ids.append(sid)
        for sid in done_ids:
            del self._ready[sid]
        # serve the oldest waiting streams first next time
        for r in batch:
            if r.stream in self._ready:
                self._ready.pop(r.stream)
                self._ready[r.stream] = None
        return batch

    def finish(self, batch: Sequence[Request], now: float, executor) -> None:
        for r in batch:
            s = self.streams[r.stream]
            s.inflight -= 1
            s.last_used = now
            if s.cancel_pending and s.inflight == 0 and s.admitted:
                self._release(s, executor)

    def in_use(self) -> int:
        return self.bytes_used


# ---------------------------------------------------------------------------
# Request loop
# ---------------------------------------------------------------------------
@dataclass
class LoopStats:
    requests: List[Request]
    wall_s: float
    batches: int
    batch_sizes: List[int]


def run_open_loop(sched: Scheduler, executor, times: np.ndarray, stream_ids: np.ndarray,
                  clock: Callable[[], float] = time.perf_counter, idle: Optional[Callable[[float], None]] = None,
                  max_inflight: int = 2, drain: bool = True) -> LoopStats:
    """Serves arrivals at ``times`` (seconds from the start) for ``stream_ids``.

    ``idle(next_event_time)`` is called when there is nothing to do; by default
    it spins.  With a fake clock it advances time."""
    n = len(times)
    reqs = [Request(i, int(stream_ids[i]), float(times[i])) for i in range(n)]
    inflight: Deque[Tuple[object, List[Request]]] = collections.deque()
    t0 = clock()
    i = 0
    nb = 0
    sizes = []
    while i < n or (drain and (sched.pending() or inflight)):
        now = clock() - t0
        while i < n and reqs[i].t_arrival <= now:
            sched.submit(reqs[i], now)
            i += 1
        progressed = False
        while inflight and executor.done(inflight[0][0]):
            h, batch = inflight.popleft()
            t = clock() - t0
            executor.collect(h, batch)
            for r in batch:
                r.t_done = t
            sched.finish(batch, t, executor)
            progressed = True
        if len(inflight) < max_inflight and sched.pending():
            batch = sched.form_batch(now, executor)
            if batch:
                inflight.append((executor.launch(batch, sched), batch))
                nb += 1
                sizes.append(len(batch))
                progressed = True
        if not progressed:
            if not inflight and not sched.pending() and i >= n:
                break
            if idle is not None:
                nxt = reqs[i].t_arrival if i < n else math.inf
                idle(min(nxt, sched.next_deadline()))
    return LoopStats(reqs, clock() - t0, nb, sizes)


def latency_summary(reqs: Sequence[Request], t_from: float = 0.0) -> Dict[str, float]:
    """p50/p99/max latency (ms) of answered pair requests that arrived at or after ``t_from``."""
    lat = np.array([r.t_done - r.t_arrival for r in reqs
                    if r.kind == PAIR and r.t_arrival >= t_from and not math.isnan(r.t_done)])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


# ---------------------------------------------------------------------------
# Device executor
# ---------------------------------------------------------------------------
class GpuExecutor:
    """Runs batches on the GPU through the C ABI (re-planned persistent launch).

    ``host_frames[sid]`` is a pinned [F, H, W] u8 tensor; request ``k`` of
    stream ``sid`` carries frame ``k % F`` of it."""

    # A tick carries few pairs: short bands spread each pair over many waves
    # (the library's built-in launch shape is chosen for large batches).
    LATENCY_TUNING = (16, 32)

    def __init__(self, host_frames: Sequence, levels: int = 3, ring: int = 3, max_inflight: int = 2,
                 tuning=LATENCY_TUNING, device=None):
        import torch

        from . import api
        from . import _lib as L

        self.torch, self.api, self.L = torch, api, L
        self.host_frames = host_frames
        self.levels = levels
        self.ring = ring
        self.tuning = tuning
        self.dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.copy_stream = torch.cuda.Stream(device=self.dev)
        self.compute_stream = torch.cuda.Stream(device=self.dev)
        self.n_slots = max_inflight + 1
        self.plans: List[Optional[object]] = [None] * self.n_slots
        self.host_levels = [None] * self.n_slots
        self.host_picks = [None] * self.n_slots
        self.slot_busy = [False] * self.n_slots
        self.allocated = 0

    # stream state ------------------------------------------------------------
    def allocate(self, s: StreamState):
        self.allocated += 1
        return self.torch.empty((self.ring, s.H, s.W), dtype=self.torch.uint8, device=self.dev)

    def release(self, s: StreamState) -> None:
        s.slot = None

    # batches -----------------------------------------------------------------
    def _pinned(self, cur, nbytes):
        if cur is None or cur.numel() < nbytes:
            return self.torch.empty(max(nbytes, 4096), dtype=self.torch.uint8, pin_memory=True)
        return cur

    def launch(self, batch: Sequence[Request], sched: Scheduler):
        torch, api, L = self.torch, self.api, self.L
        j = self.slot_busy.index(False)
        self.slot_busy[j] = True
        with torch.cuda.stream(self.copy_stream):
            for r in batch:
                s = sched.streams[r.stream]
                frames = self.host_frames[r.stream]
                s.slot[r.k % self.ring].copy_(frames[r.k % frames.shape[0]], non_blocking=True)
        ev_copy = torch.cuda.Event()
        ev_copy.record(self.copy_stream)
        self.compute_stream.wait_event(ev_copy)
        pairs = [r for r in batch if r.kind == PAIR]
        n_pairs = 0
        if pairs:
            seqs = []
            for r in pairs:
                buf = sched.streams[r.stream].slot
                seqs.append(api.seq_from_pair(buf[(r.k - 1) % self.ring], buf[r.k % self.ring], self.levels))
            plan = self.plans[j]
            if plan is None:
                plan = api.TTCPlan(seqs, torch.uint8, self.dev, tuning=self.tuning)
                self.plans[j] = plan
            else:
                plan.reset(seqs)
            plan.upload(self.compute_stream)
            plan.run(self.compute_stream)
            n_pairs = plan.n_pairs
            lv_bytes = plan.n_records * L.LEVEL_DTYPE.itemsize
            pk_bytes = plan.n_pairs * L.PICK_DTYPE.itemsize
            self.host_levels[j] = self._pinned(self.host_levels[j], lv_bytes)
            self.host_picks[j] = self._pinned(self.host_picks[j], pk_bytes)
            with torch.cuda.stream(self.compute_stream):
                self.host_levels[j][:lv_bytes].copy_(plan.levels_buf[:lv_bytes], non_blocking=True)
                self.host_picks[j][:pk_bytes].copy_(plan.picks_buf[:pk_bytes], non_blocking=True)
        ev_done = torch.cuda.Event()
        ev_done.record(self.compute_stream)
        # the copy stream must not overwrite a ring buffer before the compute
        # work that reads it: the scheduler's in-flight limit guarantees the
        # reader finished on the host's clock, which implies it on the device.
        return (j, ev_done, n_pairs)

    def done(self, h) -> bool:
        return h[1].query()

    def collect(self, h, batch: Sequence[Request]) -> None:
        j, _, n_pairs = h
        L = self.L
        if n_pairs:
            picks = self.host_picks[j][: n_pairs * L.PICK_DTYPE.itemsize].numpy().view(L.PICK_DTYPE).copy()
            levels = self.host_levels[j][: n_pairs * self.levels * L.LEVEL_DTYPE.itemsize].numpy() \
                .view(L.LEVEL_DTYPE).copy()
        q = 0
        for r in batch:
            if r.kind == PRIME:
                r.status = TC_NEED_PREV
                continue
            r.pick = picks[q]
            r.levels = levels[q * self.levels:(q + 1) * self.levels]
            r.status = int(picks[q]["status"])
            q += 1
        self.slot_busy[j] = False
