"""Autotuner for fused executions.

A fused launch has three knobs that trade load balance against per-item
overhead and LDS residency (paper Section 3.2 leaves the thread-block and
queue granularity to the implementation; Section 4.1 places small hash
tables in shared memory):

* ``rows_per_item``: rows per work item claimed from the device queue;
* ``wg_per_cu``: resident workgroups per compute unit;
* ``lds_hash_bytes``: LDS budget per workgroup for dimension-table copies
  (0 keeps every table in HBM).

``tune`` times every point of the grid on the caller's plans (device events,
median of ``reps`` runs after one warm-up), skips points the library rejects
(an LDS budget that does not fit, for instance), and caches the table and
the winner in a JSON file keyed by the device and the shapes of the plans.

``tune_chunks`` adds the encode-time axis, the chunk size (the paper's page
size, which Section 5.3 varies): the caller re-encodes its tables at each
size in ``CHUNK_ROWS`` and each encoding is tuned over the launch grid.
"""
from __future__ import annotations

import itertools
import json
import os
import time

from . import dpf

GRID = {
    "rows_per_item": [16384, 32768, 65536, 131072],
    "wg_per_cu": [1, 2, 4, 6],
    "lds_hash_bytes": [0, 32768, 65536, 131072],
}
CHUNK_ROWS = [16384, 32768, 65536, 131072]
MAX_LDS_PER_CU = 160 * 1024


def default_cache_path() -> str:
    base = os.environ.get("DPF_TUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2605_10511_amd", "tune.json")


def signature(plans: list, device_name: str) -> str:
    """Cache key: device plus each plan's row count, column count and
    footprint (plans of the same template and table size share a key)."""
    parts = [device_name]
    for p in plans:
        parts.append(f"{p.nrows}:{p.ncols}:{p.footprint()}")
    return "|".join(parts)


def _points(grid: dict):
    for rpi, wg, lds in itertools.product(grid["rows_per_item"], grid["wg_per_cu"], grid["lds_hash_bytes"]):
        if wg * lds > MAX_LDS_PER_CU:
            continue  # the budget of all resident workgroups must fit the CU's LDS
        yield {"rows_per_item": rpi, "wg_per_cu": wg, "lds_hash_bytes": lds}


def time_point(ctx, plans: list, knobs: dict, reps: int = 3, stream=None) -> float:
    """Median device milliseconds of one fused execution of ``plans``."""
    import torch
    s = stream or torch.cuda.current_stream()
    dpf.execute(ctx, plans, stream=s, **knobs).release()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        r = dpf.execute(ctx, plans, stream=s, **knobs)
        e1.record(s)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
        r.release()
    ts.sort()
    return ts[len(ts) // 2]


def tune(ctx, plans: list, grid: dict | None = None, reps: int = 3, cache: str | None = None,
         refresh: bool = False, stream=None, log=None, tag: str = "") -> dict:
    """Return {"best": knobs, "ms": t, "table": [...], "key": ...}, from the
    cache when it holds this key (unless ``refresh``); ``tag`` extends the
    key (the chunk size, for ``tune_chunks``)."""
    import torch
    grid = grid or GRID
    path = cache or default_cache_path()
    key = signature(plans, torch.cuda.get_device_name(ctx.device)) + (f"|{tag}" if tag else "")
    db = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if not refresh and key in db:
        return db[key]
    table = []
    t0 = time.time()
    for knobs in _points(grid):
        try:
            ms = time_point(ctx, plans, knobs, reps, stream)
        except dpf.DpfError as e:
            table.append({**knobs, "ms": None, "error": str(e)})
            continue
        table.append({**knobs, "ms": ms})
        if log:
            log(f"[tune] {knobs} -> {ms:.3f} ms")
    ok = [t for t in table if t["ms"] is not None]
    if not ok:
        raise RuntimeError("no point of the tuning grid ran")
    best = min(ok, key=lambda t: t["ms"])
    entry = {"key": key, "best": {k: best[k] for k in ("rows_per_item", "wg_per_cu", "lds_hash_bytes")},
             "ms": best["ms"], "table": table, "seconds": time.time() - t0}
    db[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1)
        os.replace(tmp, path)
    except OSError:
        pass  # an unwritable cache only costs a re-tune
    return entry


def tune_chunks(ctx, make_plans, chunk_rows: list | None = None, grid: dict | None = None, reps: int = 3,
                cache: str | None = None, refresh: bool = False, stream=None, log=None) -> dict:
    """Tune the chunk size with the launch knobs.  ``make_plans(rows)``
    encodes the caller's tables with chunks of ``rows`` rows and returns
    (plans, release), release() freeing them.  Returns {"best": {"chunk_rows":
    ..., knobs...}, "ms": t, "per_chunk": [{"chunk_rows", "best", "ms",
    "seconds"}]}."""
    per = []
    for rows in chunk_rows or CHUNK_ROWS:
        t0 = time.time()
        plans, release = make_plans(rows)
        try:
            e = tune(ctx, plans, grid, reps, cache, refresh, stream, log, tag=f"chunk_rows={rows}")
        finally:
            release()
        per.append({"chunk_rows": rows, "best": e["best"], "ms": e["ms"], "seconds": time.time() - t0})
        if log:
            log(f"[tune] chunk_rows {rows}: best {e['best']} -> {e['ms']:.3f} ms")
    win = min(per, key=lambda p: p["ms"])
    return {"best": {"chunk_rows": win["chunk_rows"], **win["best"]}, "ms": win["ms"], "per_chunk": per}
