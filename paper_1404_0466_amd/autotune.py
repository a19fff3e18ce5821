"""Autotuner for batched cross-validation (pichol_cv_batch).

The kernels' tile edge is fixed at 128 by the tile-packed layout; what is
tuned is which kernels run on the tiles and how they are scheduled:
  1. per d bucket, the number of 128-wide panels taken per delayed
     trailing update of the factorizations (the panel group: a larger group
     reads and writes the trailing tiles fewer times but lengthens the
     per-column updates inside the group) -- each bucket's problems are
     timed alone for every candidate group size;
  2. per d bucket (interpolated method), the form of the solves: the
     stacked product over the r+1 coefficient planes, or the per-lambda
     kernel that evaluates each lambda's tile in registers and pads its c
     columns to 16 (the better one depends on c and q);
  3. for the whole batch, how many library streams run the independent
     buckets concurrently and whether buckets are dealt out by decreasing
     work or in input order.
Every candidate is timed as a few replays of a captured HIP graph on the
caller's own batch, so host launch cost does not blur the comparison.
Choices are cached in a JSON file keyed by the batch's signature (the
multiset of problem shapes, the method and the device name).
"""
from __future__ import annotations

import json
import os

from . import binding as B

CANDIDATES = [
    {"streams": s, "order": o} for s in (1, 2, 4) for o in (0, 1)
]
GROUPS = (2, 4, 6)


class _Subset:
    """The items of a batch whose indices are given (same host arrays)."""

    def __init__(self, batch, idx):
        self.n = len(idx)
        self.items = (B.BatchItem * self.n)(*[batch.items[i] for i in idx])
        self._parent = batch


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


def tune_groups(batch, method, ws, nbytes, reps=3, groups=GROUPS):
    """Best panel group per d bucket: {nt: group}, and the timings
    {nt: {group: ms}}."""
    by_nt = {}
    for i in range(batch.n):
        nt = (batch.items[i].p.d + 127) // 128
        by_nt.setdefault(nt, []).append(i)
    best, times = {}, {}
    for nt, idx in sorted(by_nt.items()):
        if nt > 32:
            continue
        sub = _Subset(batch, idx)
        times[nt] = {}
        for gsz in groups:
            tune_ = {"streams": 1, "order": 0, "panel_group": {nt: gsz}}
            times[nt][gsz] = time_schedule(sub, method, tune_, ws, nbytes, reps)
        best[nt] = min(times[nt], key=times[nt].get)
    return best, times


FORMS = (1, 2)


def tune_forms(batch, method, ws, nbytes, groups, reps=3, forms=FORMS):
    """Best solve form per d bucket for the interpolated method: {nt: form},
    and the timings {nt: {form: ms}} (each bucket alone, with its chosen
    panel group)."""
    if method != B.PICHOL_METHOD_INTERP:
        return {}, {}
    by_nt = {}
    for i in range(batch.n):
        nt = (batch.items[i].p.d + 127) // 128
        by_nt.setdefault(nt, []).append(i)
    best, times = {}, {}
    for nt, idx in sorted(by_nt.items()):
        if nt > 32:
            continue
        sub = _Subset(batch, idx)
        times[nt] = {}
        for form in forms:
            tune_ = {"streams": 1, "order": 0, "panel_group": {nt: groups.get(nt, 0)},
                     "solve_form": {nt: form}}
            times[nt][form] = time_schedule(sub, method, tune_, ws, nbytes, reps)
        best[nt] = min(times[nt], key=times[nt].get)
    return best, times


def tune(batch: B.Batch, method: int, ws, nbytes, cache: str | None = DEFAULT_CACHE,
         reps: int = 3, force: bool = False, groups=GROUPS):
    """Returns (best tuning dict, timings or None when the cached choice was
    used).  The tuning dict has streams, order, panel_group ({nt: group})
    and solve_form ({nt: form})."""
    key = signature(batch, method)
    table = _load(cache) if cache else {}
    if not force and key in table:
        choice = table[key]["tune"]
        for field in ("panel_group", "solve_form"):
            choice[field] = {int(k): v for k, v in choice.get(field, {}).items()}
        return choice, None
    best_groups, group_times = tune_groups(batch, method, ws, nbytes, reps, groups)
    best_forms, form_times = tune_forms(batch, method, ws, nbytes, best_groups, reps)
    times = {}
    for cand in CANDIDATES:
        c = dict(cand, panel_group=best_groups, solve_form=best_forms)
        times[json.dumps(cand, sort_keys=True)] = time_schedule(batch, method, c, ws,
                                                               nbytes, reps)
    best = min(times, key=times.get)
    choice = dict(json.loads(best), panel_group=best_groups, solve_form=best_forms)
    if cache:
        table[key] = {"tune": choice, "ms": times[best]}
        _store(cache, table)
    return choice, {"schedule": times, "panel_group": group_times,
                    "solve_form": form_times}
