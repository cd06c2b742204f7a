"""Autotuner for the batched form: per size bucket, pick rows per thread,
workgroup size, LDS-or-device-memory group tables and rows per work item by
measuring candidates on the bucket's own instances (successive halving), then
LDS-or-device-memory join tables for the winner (every option measured).

The search logic takes a `measure(bucket, candidate) -> seconds` callable, so
it runs unchanged against the GPU (`gpu_measure`) or against fake timings.
"""
from __future__ import annotations

import itertools
import json
import math
import os
from dataclasses import dataclass, replace

# Size buckets: instances with n < 2^b go to the first bucket whose bound exceeds n.
BUCKETS = (12, 15, 18, 31)
IPT = (1, 2, 4, 8)
BLOCK = (128, 256, 512)
LDS_GROUPS = (0, 128, 512)
ROWS_PER_ITEM = (4096, 16384, 65536)
LDS_JOIN = (0, 1024)  # dim keys up to which a work item builds its join table in LDS

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "batch_mi355x.json")


@dataclass(frozen=True)
class Candidate:
    items_per_thread: int
    block: int
    lds_groups_max: int
    rows_per_item: int
    lds_join_max: int = 0

    def entry(self, log2_rows_below: int) -> dict:
        return dict(log2_rows_below=log2_rows_below, items_per_thread=self.items_per_thread, block=self.block,
                    lds_groups_max=self.lds_groups_max, rows_per_item=self.rows_per_item,
                    lds_join_max=self.lds_join_max)

    def name(self) -> str:
        return f"{self.items_per_thread}/{self.block}/{self.lds_groups_max}/{self.rows_per_item}/{self.lds_join_max}"


def candidates() -> list[Candidate]:
    out = []
    for ipt, blk, lds, rpi in itertools.product(IPT, BLOCK, LDS_GROUPS, ROWS_PER_ITEM):
        if rpi % (ipt * blk) == 0:
            out.append(Candidate(ipt, blk, lds, rpi))
    return out


def bucket_of(n: int) -> int:
    for i, b in enumerate(BUCKETS):
        if n < (1 << b):
            return i
    return len(BUCKETS) - 1


def successive_halving(cands: list[Candidate], measure, rounds: int = 3, keep: float = 1 / 3,
                       progress=None) -> tuple[Candidate, dict]:
    """Measure every candidate, keep the fastest third, measure again (times
    accumulate as a running minimum), until one is left or rounds run out."""
    best_time: dict[Candidate, float] = {}
    alive = list(cands)
    for r in range(rounds):
        for c in alive:
            t = float(measure(c))
            best_time[c] = min(best_time.get(c, math.inf), t)
        if progress:
            progress(f"round {r}: {len(alive)} candidates, best {min(best_time[c] for c in alive) * 1e3:.3f} ms")
        alive.sort(key=lambda c: (best_time[c], c.items_per_thread, c.block, c.lds_groups_max, c.rows_per_item,
                                  c.lds_join_max))
        if len(alive) == 1:
            break
        alive = alive[:max(1, int(math.ceil(len(alive) * keep)))]
    return alive[0], {c.name(): t for c, t in best_time.items()}


def tune(bucket_measure, buckets=BUCKETS, rounds: int = 3, progress=None) -> tuple[list[dict], dict]:
    """bucket_measure(bucket_index) -> measure(candidate) or None (empty bucket).
    Returns the tuning table (one entry per non-empty bucket, ascending, the
    last one extended to 31 bits) and the measured times."""
    table, report = [], {}
    for i, b in enumerate(buckets):
        meas = bucket_measure(i)
        if meas is None:
            continue
        prog = (lambda msg, b=b: progress(f"bucket n < 2^{b}: {msg}")) if progress else None
        best, times = successive_halving(candidates(), meas, rounds=rounds, progress=prog)
        # the join table's placement for the winner: every option, measured alike
        best, jtimes = successive_halving([replace(best, lds_join_max=j) for j in LDS_JOIN], meas, rounds=rounds,
                                          keep=1.0, progress=prog)
        table.append(best.entry(b))
        report[str(b)] = {**times, **{f"join {k}": t for k, t in jtimes.items()}}
    if table:
        table[-1]["log2_rows_below"] = 31
    return table, report


def save(table: list[dict], path: str = DEFAULT_TABLE, report: dict | None = None):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"tuning": table, "report": report or {}}, f, indent=1)


def load(path: str = DEFAULT_TABLE) -> list[dict] | None:
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["tuning"]


def gpu_measure(ctx, instances, reps: int = 3):
    """measure(candidate) for a list of device instances: median time of
    `reps` graph launches of a batch built with that candidate for all of them."""
    import torch

    from . import rel

    def measure(c: Candidate) -> float:
        b = rel.Batch(ctx, instances, tuning=[c.entry(31)])
        b.run()  # warm-up
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.run()
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        b.close()
        times.sort()
        return times[len(times) // 2]

    return measure
