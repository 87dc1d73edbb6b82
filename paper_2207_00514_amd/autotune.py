"""Autotuner for the traversal shape.

Every traversal shape -- the variant and, for the default variant 13, the
depth of its LDS stack ring -- computes the same tree; they differ only in
speed, and the fastest depends on the cloud's size, dimension and on whether
it runs alone or in a batch.  ``autotune`` times the candidate shapes on
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

# (traversal variant, LDS stack ring depth of variant 13): the two axes of
# the traversal shape (the fixed-depth variants 5, 7, 8 have rings of 16, 8
# and 4 entries of their own)
SINGLE_CANDIDATES = ((5, 8), (7, 8), (8, 8), (10, 8), (11, 8), (13, 4), (13, 8), (13, 16))
BATCHED_CANDIDATES = ((0, 8), (5, 8), (7, 8), (8, 8), (13, 4), (13, 8), (13, 16))


def _label(shape) -> str:
    v, d = shape
    return f"{v}" if v != 13 else f"{v}/{d}"


def _set_shape(ctx, shape) -> None:
    v, d = shape
    ctx.set_traversal(v)
    ctx.set_lds_depth(d)


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
                dims: Iterable[int] = (2, 3), candidates: Sequence[tuple] = SINGLE_CANDIDATES,
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
            for shape in candidates:
                _set_shape(ctx, shape)
                ms[shape] = 1e3 * _median_seconds(run, repeats)
            best = min(ms, key=ms.get)
            entries.append({"mode": "single", "dim": int(dim), "n_min": int(n_min), "variant": int(best[0]),
                            "lds_depth": int(best[1]), "tuned_on": int(n),
                            "ms": {_label(k): round(t, 4) for k, t in ms.items()}})
    _set_shape(ctx, (-1, 0))
    return entries


def tune_batched(ctx, clouds, candidates: Sequence[tuple] = BATCHED_CANDIDATES, repeats: int = 3) -> List[Dict]:
    """One entry for batches: the fastest candidate on the caller's clouds
    (a list of device tensors, as ``Context.build_batched`` takes them)."""
    ms = {}
    for shape in candidates:
        _set_shape(ctx, shape)
        ms[shape] = 1e3 * _median_seconds(lambda: ctx.build_batched(clouds), repeats)
    _set_shape(ctx, (-1, 0))
    best = min(ms, key=ms.get)
    total = int(sum(int(c.shape[0]) for c in clouds))
    return [{"mode": "batched", "dim": 3, "n_min": 0, "variant": int(best[0]), "lds_depth": int(best[1]),
             "tuned_on": total, "ms": {_label(k): round(t, 4) for k, t in ms.items()}}]


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
    _set_shape(ctx, (-1, 0))
    return text
