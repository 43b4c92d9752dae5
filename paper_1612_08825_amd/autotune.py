"""Tuning sweeps: the fused TTC pass and the row-streaming direct convolution.

For a (dtype, levels) class the sweep times the fused kernel over a
representative batch for every candidate launch shape -- band height (rows a
wave walks for one pair: 16, 32, 64, 128) and persistent work-groups per compute unit -- with HIP
events on the launch stream, and keeps the fastest.  Candidates that fail to
create a plan are skipped.  The table it prints is what the library's built-in
default (``tc_ttc_tuning_default``) is set from; callers can also pass a tuning
to ``TTCPlan(..., tuning=(band_rows, groups_per_cu))``.

Direct convolution (``--conv``): for every (input type, taps per side, size
class) the sweep times the row-streaming kernels at every band height (output
rows per wave: 2, 4, 8) through ``tc_conv_nd_ex``'s ``band_rows``, as a replayed
graph over buffers rotated past the last-level cache, and keeps the fastest;
a candidate is accepted only if its output equals the others' bit for bit
(the band height must not change a result).  The library's default table
(``default_band_rows`` in the row kernels) is set from it.

    python -m paper_1612_08825_amd.autotune [--out table.json] [--conv]
"""
from __future__ import annotations

import argparse
import json
import sys
from typing import Dict, List, Sequence, Tuple

BAND_ROWS = (16, 32, 64, 128)
GROUPS_PER_CU = (8, 16, 32, 64, 128)


def time_plan(api, torch, videos, levels: int, tuning: Tuple[int, int], reps: int, warmup: int) -> float:
    """Average fused-pass milliseconds for one launch shape."""
    plan = api.TTCPlan([api.seq_from_frames(v, levels) for v in videos], videos[0].dtype, keep=videos, tuning=tuning)
    try:
        plan.upload()
        for _ in range(warmup):
            plan.run_phase(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.run_phase(1)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        plan.close()


def sweep(videos, levels: int, band_rows: Sequence[int] = BAND_ROWS, groups: Sequence[int] = GROUPS_PER_CU,
          reps: int = 10, warmup: int = 2) -> List[Dict]:
    import torch

    from . import api

    rows = []
    for rh in band_rows:
        for gpc in groups:
            try:
                ms = time_plan(api, torch, videos, levels, (rh, gpc), reps, warmup)
            except Exception as exc:  # a shape this build does not provide
                rows.append({"band_rows": rh, "groups_per_cu": gpc, "ms": None, "error": str(exc)})
                continue
            rows.append({"band_rows": rh, "groups_per_cu": gpc, "ms": round(ms, 4)})
            print(f"[tune] rows={rh:2d} groups/CU={gpc:2d}: {ms:.4f} ms", file=sys.stderr, flush=True)
    return rows


def best(rows: List[Dict]) -> Dict:
    ok = [r for r in rows if r.get("ms") is not None]
    return min(ok, key=lambda r: r["ms"])


def workloads(torch):
    """Representative batches: the batched f16 workload and a u8 mix like the
    serving streams, each swept at every level count (1..4)."""
    from . import synth

    f16 = []
    for s in synth.batched_specs():
        f16.append(s.render(device="cuda"))
        torch.cuda.synchronize()  # keep the queue shallow while rendering
    u8 = []
    for s in synth.serving_specs(n_streams=64):
        u8.append(s.render(device="cuda"))
        torch.cuda.synchronize()
    return {("f16", lv): f16 for lv in (4, 3, 2, 1)} | {("u8", lv): u8 for lv in (3, 4, 2, 1)}


CONV_BAND_ROWS = (2, 4, 8)
CONV_TAPS = (2, 3, 5, 7)
CONV_SIZES = (("small", 1024), ("medium", 2048), ("large", 4096))  # square images, full mode
CONV_DTYPES = ("f32", "f16", "u8")


def conv_sweep(reps: int = 20) -> Dict:
    """Band height of the row-streaming convolution per (input type, K, size
    class), gated on bitwise-equal outputs across heights."""
    import math

    import numpy as np
    import torch

    from . import api, synth

    table = {}
    for dt in CONV_DTYPES:
        for cls, n in CONV_SIZES:
            x0 = torch.from_numpy(synth.conv_image((n, n), case=17, dtype=dt)).cuda()
            for K in CONV_TAPS:
                if dt == "u8":
                    kh = synth.conv_kernel((K, K), case=17, dtype="i32")
                    kabs = int(np.abs(kh.astype(np.int64)).sum())
                else:
                    kh = synth.conv_kernel((K, K), case=17)
                    kabs = None
                k = torch.from_numpy(kh).cuda()
                ys = (n + K - 1, n + K - 1)
                ydt = torch.int32 if dt == "u8" else torch.float32
                nbytes = x0.element_size() * n * n + 4 * ys[0] * ys[1]
                nbuf = max(2, min(64, int(math.ceil(1.1 * 2 ** 30 / nbytes))))
                xb = [x0.clone() for _ in range(nbuf)]
                yb = [torch.empty(ys, dtype=ydt, device="cuda") for _ in range(nbuf)]
                res, outs = {}, {}
                for br in CONV_BAND_ROWS:
                    def launch(i):
                        api.conv_nd_ex(xb[i % nbuf], k, "full", method="direct", k_abs_sum=kabs, out=yb[i % nbuf],
                                       band_rows=br)
                    n_l = max(reps, 2 * nbuf)
                    for i in range(3):
                        launch(i)
                    torch.cuda.synchronize()
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g):
                        for i in range(n_l):
                            launch(i)
                    g.replay()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    g.replay()
                    e1.record()
                    torch.cuda.synchronize()
                    res[br] = round(e0.elapsed_time(e1) / n_l, 5)
                    outs[br] = yb[0].clone()
                    del g
                equal = all(torch.equal(outs[br], outs[CONV_BAND_ROWS[-1]]) for br in CONV_BAND_ROWS)
                ok = {br: ms for br, ms in res.items() if equal}
                bestb = min(ok, key=ok.get) if ok else None
                table[f"{dt}/K{K}/{cls}"] = {"best_band_rows": bestb, "ms": res, "bitwise_equal": equal}
                print(f"[tune] conv {dt} K={K} {cls}: {res} best {bestb} equal {equal}", file=sys.stderr, flush=True)
                del xb, yb, outs
                torch.cuda.empty_cache()
    return table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--conv", action="store_true", help="the convolution sweep instead of the fused TTC pass")
    args = ap.parse_args()
    import torch

    if args.conv:
        text = json.dumps(conv_sweep(), indent=1)
        print(text)
        if args.out:
            with open(args.out, "w") as f:
                f.write(text)
        return

    table = {}
    for (dt, levels), vids in workloads(torch).items():
        print(f"[tune] {dt} {levels} levels", file=sys.stderr, flush=True)
        rows = sweep(vids, levels, reps=args.reps)
        b = best(rows)
        table[f"{dt}/L{levels}"] = {"best": {"band_rows": b["band_rows"], "groups_per_cu": b["groups_per_cu"],
                                             "ms": b["ms"]}, "sweep": rows}
    torch.cuda.empty_cache()
    text = json.dumps(table, indent=1)
    print(text)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()
