"""Autotuner for the batched forward + backward of many cameras.

The search space is the tile edge (8, 16, 32 pixels), the render scheduling
(one workgroup per tile, or a persistent grid of n workgroups taking the
next tile of the heaviest-first order from one global counter) and the batch
size (cameras per launch: every camera
of a group goes through one launch per stage and one hipGraph).  A
coordinate search tries the tile edges first, then the scheduling for the
best edge, then the batch sizes; every candidate is timed as replays of its
captured graphs with HIP events on the replay stream.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Optional, Sequence

import torch

from .render import BatchRenderer, DeviceScene


def time_batch(br: BatchRenderer, reps: int = 3) -> float:
    """Milliseconds per replay of all of br's graphs."""
    br.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(br.stream)
    for _ in range(reps):
        br.replay()
    e1.record(br.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _candidate(ds, cams, K, grad, group, tile, persistent, reps, activation):
    br = BatchRenderer(ds, cams, K, group=group, tile=tile, persistent=persistent,
                       activation=activation)
    br.capture(grad)
    ms = time_batch(br, reps)
    ok = br.check_overflow()
    nbytes = br.workspace_bytes()
    del br
    torch.cuda.empty_cache()
    return ms, ok, nbytes


def tune(ds: DeviceScene, cams: Sequence, K: int, grad_rgba: torch.Tensor,
         tiles=(8, 16, 32), persistent: Optional[Sequence[int]] = None,
         groups: Optional[Sequence[int]] = None, reps: int = 3, activation: int = 0,
         log: Optional[Callable[[str], None]] = None) -> Dict:
    n = len(cams)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if groups is None:
        cand = {n, math.ceil(n / 2), math.ceil(n / 3), math.ceil(n / 4), math.ceil(n / 8)}
        groups = sorted(g for g in cand if 1 <= g <= 32)
    table: List[Dict] = []

    def run(group, tile, pers):
        ms, ok, nbytes = _candidate(ds, cams, K, grad_rgba, group, tile, pers, reps, activation)
        row = {"group": group, "tile": tile, "persistent": pers, "ms": ms, "overflow": not ok,
               "workspace_bytes": nbytes}
        table.append(row)
        if log:
            log("autotune: cameras/launch=%d tile=%d persistent=%d -> %.3f ms" % (
                group, tile, pers, ms))
        return ms if ok else float("inf")

    g0 = max(groups)
    best_tile = min(tiles, key=lambda t: run(g0, t, 0))
    if persistent is None:
        # persistent grids sized in resident waves per SIMD (4 SIMDs per CU)
        waves_per_wg = max(1, best_tile * best_tile // 64)
        persistent = [0] + [cus * 4 * w // waves_per_wg for w in (4, 8)]
    best_pers = min(persistent, key=lambda p: (run(g0, best_tile, p) if p else
                                               next(r["ms"] for r in table
                                                    if r["tile"] == best_tile and
                                                    r["persistent"] == 0 and r["group"] == g0)))
    rest = [g for g in groups if g != g0]
    scores = {g0: next(r["ms"] for r in table if r["tile"] == best_tile and
                       r["persistent"] == best_pers and r["group"] == g0)}
    for g in rest:
        scores[g] = run(g, best_tile, best_pers)
    best_group = min(scores, key=scores.get)
    return {"tile": best_tile, "persistent": best_pers, "group": best_group,
            "ms": scores[best_group], "table": table}
