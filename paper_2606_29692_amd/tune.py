"""Schedule autotuner for the H product.

A schedule is the number of wave lanes per CSR row (8, 16, 32, 64) with the
VQE_SPMV_* options: wide loads (VEC4), the state staged in LDS (LDS, DEEP),
the pipelined loads (PREFETCH), 16-bit column codes (X16), the complex
values in the row-padded layout (PAD), for a real H the real values in
that layout (REAL), and the sliced layout with one row per lane (SLICED,
with 2, 4 or 8 entries per lane and load in place of the lanes, or 3 or 6
with the flip masks' 10-bit indices in place of the columns, XIDX; an
operator with too many masks for it times as infinite).  It is picked
per (register size, dtype, mapping, value form, device) by timing the batched
H product phase of a real plan over the candidates, and cached.  The value
form "complex" keeps the interleaved complex values of the CSR (candidates
without REAL); "any" also admits REAL, which applies to Hamiltonians whose
entries are all real.  The choice is a function of that key alone, so a state
gets the same schedule (and the same floating-point summation order) whether
it runs alone or inside any batch.

A batch of several register sizes runs one H-product launch per schedule in
use; schedules_for_batch may instead give every state one shared schedule,
when one launch for the whole batch is faster (the smaller states' workgroups
then fill the CUs that a few large states leave idle).  That choice depends on
the batch, so it gives up the alone-or-in-any-batch property above.

Cache: ``tuned_schedules.json`` next to this file (committed results), plus
the file named by ADAPTVQE_TUNE_CACHE when set (written after tuning).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import binding as B

_L, _V, _D, _P = B.VQE_SPMV_LDS, B.VQE_SPMV_VEC4, B.VQE_SPMV_DEEP, B.VQE_SPMV_PREFETCH
_X, _R, _Q, _S = B.VQE_SPMV_X16, B.VQE_SPMV_REAL, B.VQE_SPMV_PAD, B.VQE_SPMV_SLICED
_I = B.VQE_SPMV_XIDX
CANDIDATES = (8, 16, 32, 64, 16 | _V, 32 | _V, 64 | _V,
              8 | _L, 16 | _L, 32 | _L, 64 | _L, 8 | _L | _D, 16 | _L | _D, 32 | _L | _D, 64 | _L | _D,
              32 | _L | _P, 64 | _L | _P, 32 | _L | _P | _D, 64 | _L | _P | _D,
              8 | _L | _P, 16 | _L | _P, 16 | _L | _P | _D,
              32 | _L | _P | _X, 64 | _L | _P | _X, 32 | _L | _P | _D | _X, 64 | _L | _P | _D | _X,
              16 | _L | _P | _X | _R, 32 | _L | _P | _X | _R, 64 | _L | _P | _X | _R,
              32 | _L | _P | _D | _X | _R,
              64 | _L | _P | _D | _X | _R,
              16 | _L | _P | _X | _Q, 32 | _L | _P | _X | _Q, 64 | _L | _P | _X | _Q,
              32 | _L | _P | _D | _X | _Q,
              # narrow sub-groups (the blocked product of states larger than LDS)
              8 | _L | _P | _D, 8 | _L | _P | _X, 8 | _L | _P | _D | _X, 16 | _L | _P | _X,
              16 | _L | _P | _D | _X, 4 | _L | _P, 4 | _L | _P | _D, 4 | _L | _P | _X,
              # one row per lane, rows sorted by length into slices of 64
              2 | _L | _S, 4 | _L | _S, 8 | _L | _S, 2 | _L | _S | _D, 4 | _L | _S | _D,
              2 | _L | _S | _R, 4 | _L | _S | _R, 8 | _L | _S | _R,
              # and with the flip masks' 10-bit indices in place of the columns
              3 | _L | _S | _I, 6 | _L | _S | _I, 3 | _L | _S | _I | _R, 6 | _L | _S | _I | _R)
_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "tuned_schedules.json")
_memo: dict = {}
_last_timings: dict = {}


VALUE_FORMS = ("any", "complex")


def _device_tag(ctx) -> str:
    """The device part of a cache key: the architecture name and the CU count
    (the marketing name the runtime reports can differ between processes of
    the same machine, for instance under a profiler)."""
    n_cu, name = ctx.info()
    arch = name[name.rfind("(") + 1:name.rfind(")")] if "(" in name and ")" in name else name
    return f"{arch}|{n_cu}cu"


def _key(ctx, ds, value_form: str = "any") -> str:
    if value_form not in VALUE_FORMS:
        raise ValueError(f"value form {value_form!r}: expected one of {VALUE_FORMS}")
    key = f"{_device_tag(ctx)}|n{ds.n_qubits}|{ds.dtype}|{ds.key[2]}"
    return key if value_form == "any" else key + "|complex"


def candidates_for(value_form: str = "any") -> tuple:
    return CANDIDATES if value_form == "any" else tuple(c for c in CANDIDATES if not c & _R)


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


def time_batch_spmv(ctx, systems, schedule, reps: int = 10) -> float:
    """Milliseconds per launch of the batched H products with the given
    schedule (one for every system, or a list with one per system): the
    median of three runs of `reps` back-to-back launches (infinite for a
    schedule the operators do not support)."""
    from .batch import make_batch
    scheds = [int(x) for x in schedule] if isinstance(schedule, (list, tuple)) else \
        [int(schedule)] * len(systems)
    try:
        plan = make_batch(ctx, systems, schedules=scheds)
    except B.VqeError as e:
        if e.status != B.VQE_ENOTSUP:
            raise
        return float("inf")
    for _ in range(3):
        plan.step(update=False)
    times = [plan.time_products(reps) for _ in range(3)]
    plan.close()
    return float(np.median(times))


def tune_schedule(ctx, systems, candidates=CANDIDATES) -> dict:
    """Time every candidate on the given (same-size) systems; return the record."""
    res = {int(c): time_batch_spmv(ctx, systems, c) for c in candidates}
    _last_timings.clear()
    _last_timings.update(res)
    best = min(res, key=res.get)
    return {"schedule": best, "ms": {str(k): v for k, v in res.items()}}


def schedule_for(ctx, ds, systems=None, retune: bool = False, value_form: str = "any") -> int:
    """Tuned schedule for systems shaped like ``ds`` (tuning on ``systems`` or
    [ds] when no cached entry exists); value_form "complex" restricts the
    candidates to schedules that stream the complex values."""
    key = _key(ctx, ds, value_form)
    if not retune:
        if key in _memo:
            return _memo[key]
        cache = _load()
        if key in cache:
            _memo[key] = int(cache[key]["schedule"])
            return _memo[key]
    rec = tune_schedule(ctx, systems or [ds], candidates_for(value_form))
    _memo[key] = rec["schedule"]
    _store(key, rec)
    return rec["schedule"]


def _batch_key(ctx, ds: list, value_form: str) -> str:
    counts: dict = {}
    for d in ds:
        k = f"n{d.n_qubits}|{d.dtype}|{d.key[2]}"
        counts[k] = counts.get(k, 0) + 1
    comp = ",".join(f"{k}x{counts[k]}" for k in sorted(counts))
    return f"{_device_tag(ctx)}|batch|{comp}" + ("" if value_form == "any" else "|complex")


def schedules_for_batch(ctx, ds: list, retune: bool = False, value_form: str = "any") -> list:
    """One schedule per state of a batch of several register sizes: each
    size's own (schedule_for, tuned on that size's states of the batch), or,
    when it is faster for the batch as a whole, one schedule shared by every
    state (candidates: the sizes' own schedules that every state supports).
    The batch's H products are timed with each choice; the record is cached
    under the batch's composition (sizes and counts)."""
    sizes = sorted({d.n_qubits for d in ds})
    own = {}
    for n in sizes:
        same = [d for d in ds if d.n_qubits == n]
        own[n] = schedule_for(ctx, same[0], systems=same, value_form=value_form)
    if len(sizes) == 1:
        return [own[sizes[0]]] * len(ds)
    key = _batch_key(ctx, ds, value_form)
    rec = None
    if not retune:
        rec = _memo.get(key) or _load().get(key)
    if rec is None:
        per_size = [own[d.n_qubits] for d in ds]
        ms = {"per-size": time_batch_spmv(ctx, ds, per_size)}
        for c in sorted(set(own.values())):
            try:
                ms[str(c)] = time_batch_spmv(ctx, ds, c)
            except B.VqeError as e:      # a size's schedule that another size refuses
                if e.status != B.VQE_EINVAL:
                    raise
                ms[str(c)] = float("inf")
        best = min(ms, key=ms.get)
        rec = {"shared": None if best == "per-size" else int(best),
               "own": {str(n): own[n] for n in sizes}, "ms": ms}
        _store(key, rec)
    _memo[key] = rec
    if rec["shared"] is not None:
        return [int(rec["shared"])] * len(ds)
    return [own[d.n_qubits] for d in ds]


def last_batch_record(ctx, ds: list, value_form: str = "any") -> dict | None:
    key = _batch_key(ctx, ds, value_form)
    return _memo.get(key) or _load().get(key)


def last_record(ctx, ds, value_form: str = "any") -> dict | None:
    return _load().get(_key(ctx, ds, value_form))


def default_schedule(ds) -> int:
    return B.default_schedule(ds.H)
