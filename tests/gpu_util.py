"""Helpers for GPU parity tests: encode tables, prepare a query description
through the library, run it fused or fragmented, and compare with the oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2605_10511_amd import dpf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_db(ctx, tables: dict, encodings: dict | None = None, chunk_rows: int = 65536,
            placement: str = "HBM") -> dpf.Database:
    db = dpf.Database(ctx)
    enc = encodings or {}
    for name, cols in tables.items():
        db.add_table(name, cols, enc.get(name), chunk_rows=chunk_rows, placement=placement)
    return db


def run_gpu(db: dpf.Database, spec: dict, mode: str = "FUSED", placements=None, **kw) -> np.ndarray:
    import torch
    plan = db.plan(spec, placements=placements)
    res = dpf.execute(db.ctx, [plan], mode=mode, **kw)
    torch.cuda.synchronize()
    out = res.get(0)
    res.release()
    plan.release()
    for h in plan.hashes:
        h.release()
    return out


def assert_same(got: np.ndarray, want: np.ndarray, what: str = ""):
    got = np.asarray(got, dtype=np.int64)
    want = np.asarray(want, dtype=np.int64).reshape(-1, got.shape[1] if got.size else want.shape[1] if want.ndim > 1 else 0)
    assert got.shape == want.shape, f"{what}: shape {got.shape} vs {want.shape}"
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)[:5]
        raise AssertionError(f"{what}: mismatch at {bad.tolist()}\n got  {got[bad[:, 0]].tolist()}\n want {want[bad[:, 0]].tolist()}")
