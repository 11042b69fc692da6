"""Schedule autotuner for the H product (lanes per row).

The lanes-per-row choice (8, 16, 32 or 64 lanes of a wave per CSR row) is
picked per (register size, dtype, mapping, device) by timing the batched H
product phase of a real plan over the candidates, and cached.  The choice is
a function of that key alone, so a state gets the same schedule (and the same
floating-point summation order) whether it runs alone or inside any batch.

Cache: ``tuned_schedules.json`` next to this file (committed results), plus
the file named by ADAPTVQE_TUNE_CACHE when set (written after tuning).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import binding as B

CANDIDATES = (8, 16, 32, 64)
_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "tuned_schedules.json")
_memo: dict = {}


def _key(ctx, ds) -> str:
    _, name = ctx.info()
    return f"{name}|n{ds.n_qubits}|{ds.dtype}|{ds.key[2]}"


def _load() -> dict:
    out = {}
    for path in (DEFAULT_CACHE, os.environ.get("ADAPTVQE_TUNE_CACHE")):
        if path and os.path.exists(path):
            with open(path) as f:
                out.update(json.load(f))
    return out


def _store(key: str, rec: dict):
    path = os.environ.get("ADAPTVQE_TUNE_CACHE")
    if not path:
        return
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = rec
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def time_batch_spmv(ctx, systems, lanes: int, reps: int = 10) -> float:
    """Average milliseconds of the batched H-product phase with the given lanes."""
    import torch
    from .batch import make_batch
    plan = make_batch(ctx, systems, lanes=[lanes] * len(systems))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    for _ in range(3):
        plan.step(update=False)
    times = []
    for _ in range(reps):
        plan.step_timed(ev, update=False)
        ctx.stream.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    plan.close()
    return float(np.median(times))


def tune_lanes(ctx, systems, candidates=CANDIDATES) -> dict:
    """Time every candidate on the given (same-size) systems; return the record."""
    res = {int(L): time_batch_spmv(ctx, systems, L) for L in candidates}
    best = min(res, key=res.get)
    return {"lanes": best, "ms": res}


def lanes_for(ctx, ds, systems=None, retune: bool = False) -> int:
    """Tuned lanes for systems shaped like ``ds`` (tuning on ``systems`` or
    [ds] when no cached entry exists)."""
    key = _key(ctx, ds)
    if not retune:
        if key in _memo:
            return _memo[key]
        cache = _load()
        if key in cache:
            _memo[key] = int(cache[key]["lanes"])
            return _memo[key]
    rec = tune_lanes(ctx, systems or [ds])
    _memo[key] = rec["lanes"]
    _store(key, rec)
    return rec["lanes"]


def default_lanes(ds) -> int:
    return B.default_lanes(ds.H)
