"""Schedule autotuner for batched cross-validation (pichol_cv_batch).

The kernels' tile shape is fixed by the tile-packed layout (128 x 128
tiles), so what is left to choose for a batch of uneven problems is its
schedule: how many library streams run the independent buckets
concurrently, and whether buckets are dealt out by decreasing work or in
input order.  ``tune`` times every candidate on the caller's batch (a few
replays of a captured HIP graph each, so host launch cost does not blur the
comparison) and keeps the fastest.  Results are cached in a JSON file keyed
by the batch's signature (the multiset of problem shapes, the method and the
device name), so a batch of the same shapes reuses the choice without
timing again.
"""
from __future__ import annotations

import json
import os

from . import binding as B

CANDIDATES = [
    {"streams": s, "order": o} for s in (1, 2, 4) for o in (0, 1)
]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pichol_autotune.json")


def signature(batch: B.Batch, method: int) -> str:
    shapes = []
    for i in range(batch.n):
        p = batch.items[i].p
        shapes.append((p.d, p.c, p.k, p.g, p.r, p.q, p.precision))
    shapes.sort()
    import torch
    devname = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return json.dumps({"method": method, "device": devname, "shapes": shapes})


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass  # a cache that cannot be written only costs a re-tune


def time_schedule(batch, method, tune, ws, nbytes, reps=3):
    """Mean milliseconds of one graph replay of the batch with `tune`."""
    import torch
    g = B.pichol_cv_batch_graph(batch, method, tune, ws, nbytes)
    try:
        B.pichol_graph_launch(g)  # warm-up
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            B.pichol_graph_launch(g)
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps
    finally:
        B.pichol_graph_destroy(g)


def tune(batch: B.Batch, method: int, ws, nbytes, cache: str | None = DEFAULT_CACHE,
         reps: int = 3, force: bool = False):
    """Returns (best tuning dict, {candidate: ms} timings or None when the
    cached choice was used)."""
    key = signature(batch, method)
    table = _load(cache) if cache else {}
    if not force and key in table:
        return table[key]["tune"], None
    times = {}
    for cand in CANDIDATES:
        times[json.dumps(cand, sort_keys=True)] = time_schedule(batch, method, cand, ws,
                                                               nbytes, reps)
    best = min(times, key=times.get)
    choice = json.loads(best)
    if cache:
        table[key] = {"tune": choice, "ms": times[best]}
        _store(cache, table)
    return choice, times
