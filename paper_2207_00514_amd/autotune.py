"""Autotuner for the traversal shape.

Every traversal variant computes the same tree; they differ only in speed,
and the fastest depends on the cloud's size, dimension and on whether it
runs alone or in a batch.  ``autotune`` times the candidate variants on
synthetic clouds of the workload recipes (or on the caller's own batch),
keeps the fastest per size bucket and installs the result as the context's
traversal-shape table (``emst_set_autotune``); calls left on the automatic
choice (``set_traversal(-1)``, the default) then look their variant up by
mode, dimension and size.  The table is JSON, so it can be saved and passed
to a later ``Context(device, autotune_json=...)``.
"""
from __future__ import annotations

import json
import math
import time
from typing import Dict, Iterable, List, Optional, Sequence

import numpy as np

from . import workloads as W

SINGLE_CANDIDATES = (5, 7, 8, 10, 11, 13)
BATCHED_CANDIDATES = (0, 5, 7, 8, 13)


def _median_seconds(fn, repeats: int) -> float:
    import torch
    fn()  # warm-up (kernels, workspace)
    torch.cuda.synchronize()
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return float(np.median(times))


def _bucket_starts(sizes: Sequence[int]) -> List[int]:
    """Bucket of sizes[i] = [geometric midpoint to sizes[i-1], midpoint to
    sizes[i+1]); the first bucket starts at 0."""
    starts = [0]
    for a, b in zip(sizes, sizes[1:]):
        starts.append(int(math.sqrt(a * b)))
    return starts


def tune_single(ctx, sizes: Sequence[int] = (10_000, 100_000, 1_000_000, 4_000_000),
                dims: Iterable[int] = (2, 3), candidates: Sequence[int] = SINGLE_CANDIDATES,
                repeats: int = 3) -> List[Dict]:
    """One entry per (dim, size bucket): the fastest candidate on a cloud of
    that size (3D: the clustered recipe; 2D: the uniform one)."""
    import torch
    sizes = sorted(int(s) for s in sizes)
    entries = []
    for dim in dims:
        for n, n_min in zip(sizes, _bucket_starts(sizes)):
            pts_np = W.clustered3d(n) if dim == 3 else W.uniform2d(n)
            pts = torch.from_numpy(pts_np).cuda(ctx.device)
            out = [None]

            def run():
                out[0] = ctx.build(pts, out=out[0])

            ms = {}
            for v in candidates:
                ctx.set_traversal(v)
                ms[v] = 1e3 * _median_seconds(run, repeats)
            best = min(ms, key=ms.get)
            entries.append({"mode": "single", "dim": int(dim), "n_min": int(n_min), "variant": int(best),
                            "tuned_on": int(n), "ms": {str(k): round(t, 4) for k, t in ms.items()}})
    ctx.set_traversal(-1)
    return entries


def tune_batched(ctx, clouds, candidates: Sequence[int] = BATCHED_CANDIDATES, repeats: int = 3) -> List[Dict]:
    """One entry for batches: the fastest candidate on the caller's clouds
    (a list of device tensors, as ``Context.build_batched`` takes them)."""
    ms = {}
    for v in candidates:
        ctx.set_traversal(v)
        ms[v] = 1e3 * _median_seconds(lambda: ctx.build_batched(clouds), repeats)
    ctx.set_traversal(-1)
    best = min(ms, key=ms.get)
    total = int(sum(int(c.shape[0]) for c in clouds))
    return [{"mode": "batched", "dim": 3, "n_min": 0, "variant": int(best), "tuned_on": total,
             "ms": {str(k): round(t, 4) for k, t in ms.items()}}]


def table_json(entries: List[Dict]) -> str:
    return json.dumps({"entries": entries})


def autotune(ctx, single_sizes: Optional[Sequence[int]] = (10_000, 100_000, 1_000_000, 4_000_000),
             dims: Iterable[int] = (2, 3), batched_clouds=None, repeats: int = 3) -> str:
    """Tune, install the table on ``ctx`` and return it as JSON."""
    entries: List[Dict] = []
    if single_sizes:
        entries += tune_single(ctx, single_sizes, dims, repeats=repeats)
    if batched_clouds is not None:
        entries += tune_batched(ctx, batched_clouds, repeats=repeats)
    text = table_json(entries)
    ctx.set_autotune(text)
    ctx.set_traversal(-1)
    return text
