"""Tuning sweep of the fused TTC pass.

For a (dtype, levels) class the sweep times the fused kernel over a
representative batch for every candidate launch shape -- band height (rows a
wave walks for one pair: 16, 32, 64, 128) and persistent work-groups per compute unit -- with HIP
events on the launch stream, and keeps the fastest.  Candidates that fail to
create a plan are skipped.  The table it prints is what the library's built-in
default (``tc_ttc_tuning_default``) is set from; callers can also pass a tuning
to ``TTCPlan(..., tuning=(band_rows, groups_per_cu))``.

    python -m paper_1612_08825_amd.autotune [--out table.json]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    import torch

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
