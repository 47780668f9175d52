"""Exhaustive schedule search for SpMV and SpMM.

A schedule is a partition kind plus its tile parameters (spl_schedule).  The
autotuner times every candidate on the operand it is given (the same calls a
user makes; each timing brackets the whole call, tile bounds and carry
fix-up included) and returns the fastest.  The candidate grids are bounded so
that tuning stays cheap relative to the work it tunes.
"""
from __future__ import annotations

from typing import Callable, Dict, List, Tuple

import torch

from . import schedule

SPMV_CANDIDATES: List[Dict] = (
    [dict(kind="row", lanes_per_row=L) for L in (1, 2, 4, 8, 16, 32, 64)] +
    [dict(kind="nnz", tile=T, items_per_lane=8) for T in (1024, 2048, 4096)] +
    [dict(kind="merge", tile=256 * it, items_per_lane=it) for it in (4, 8)]
)

SPMM_CANDIDATES: List[Dict] = (
    [dict(kind="row", col_tile=32)] +
    [dict(kind="nnz", tile=T, col_tile=32, items_per_lane=16) for T in (256, 1024)] +
    [dict(kind="merge", tile=8 * it * k, col_tile=32, items_per_lane=it)
     for it in (8, 16, 32) for k in (1, 4)]
)

# BF16 values and dense rows: 16-byte lanes (8 columns, 4 lanes per 32-column
# group) by default, 8-byte lanes (variant 2) as the alternative
SPMM_BF16_CANDIDATES: List[Dict] = (
    [dict(kind="row", col_tile=32)] +
    [dict(kind="nnz", tile=T, col_tile=32, items_per_lane=16) for T in (256, 1024)] +
    [dict(kind="merge", tile=64 * it * k, col_tile=32, items_per_lane=it)
     for it in (8, 16) for k in (1, 4)] +
    [dict(kind="merge", tile=32 * it, col_tile=32, items_per_lane=it, variant=2)
     for it in (8, 16)]
)


MTTKRP_CANDIDATES: List[Dict] = [
    # items per lane group left to the library (5 with 4-column FP32 lanes, 3
    # with 8-column BF16 lanes), at two tile sizes
    dict(kind="merge", tile=512, col_tile=32),
    dict(kind="merge", tile=768, col_tile=32),
    # 4 items per lane group: the vector-lane leaves only (R and every ld
    # multiples of 4); more waves per SIMD than with 8
    dict(kind="merge", tile=512, col_tile=32, items_per_lane=4),
    dict(kind="merge", tile=1024, col_tile=32, items_per_lane=4),
    dict(kind="merge", tile=512, col_tile=32, items_per_lane=16),
    dict(kind="merge", tile=256, col_tile=32, items_per_lane=8),
    dict(kind="merge", tile=1024, col_tile=32, items_per_lane=8),
    dict(kind="merge", tile=4096, col_tile=32, items_per_lane=8),
    dict(kind="merge", tile=512, col_tile=64, items_per_lane=8),
    dict(kind="nnz", tile=2048, col_tile=32, items_per_lane=16),
    dict(kind="nnz", tile=512, col_tile=32, items_per_lane=8),
]


def time_call(fn: Callable[[], object], reps: int = 5, warmup: int = 2) -> float:
    """Median milliseconds of fn() over `reps` runs on the current stream."""
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def search(make_call: Callable[[object], Callable[[], object]], candidates: List[Dict],
           reps: int = 5) -> Tuple[Dict, List[Tuple[Dict, float]]]:
    """Time every candidate; return (best candidate, [(candidate, ms), ...])."""
    results = []
    for cand in candidates:
        ms = time_call(make_call(schedule(**cand)), reps=reps)
        results.append((cand, ms))
    best = min(results, key=lambda r: r[1])[0]
    return best, results
