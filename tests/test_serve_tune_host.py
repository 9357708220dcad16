"""Host logic of the serving loop and the knob tuner (no GPU)."""
from __future__ import annotations

import math

import numpy as np

from datagen import workloads as W
from paper_2605_10511_amd import serve, tune


def test_requests_are_seeded_and_poisson():
    a = W.serve_requests(5, 200.0, 20.0, "res")
    b = W.serve_requests(5, 200.0, 20.0, "res")
    assert [(t, k) for t, k, _ in a] == [(t, k) for t, k, _ in b]
    ts = np.array([t for t, _, _ in a])
    assert np.all(np.diff(ts) > 0) and ts[-1] < 20.0
    # count over 20 s at 200/s: mean 4000, sd ~63
    assert abs(len(a) - 4000) < 5 * math.sqrt(4000)
    gaps = np.diff(ts)
    assert abs(gaps.mean() - 1 / 200.0) < 0.1 / 200.0
    # exponential gaps: the coefficient of variation is 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.1
    fa = sum(1 for _, k, _ in a if k == "FA")
    assert abs(fa - len(a) / 2) < 5 * math.sqrt(len(a) / 4)
    c = W.serve_requests(6, 200.0, 20.0, "res")
    assert [t for t, _, _ in c][:5] != [t for t, _, _ in a][:5]


def test_request_constants_in_domain():
    for t, k, spec in W.serve_requests(7, 100.0, 10.0, "res"):
        assert spec["fact"] == "res"
        if k == "FA":
            f = {p["col"]: p for p in spec["filters"]}
            assert 0 <= f["date"]["value"] < W.NDATES
            assert 0 <= f["discount"]["lo"] <= 8 and f["discount"]["hi"] == f["discount"]["lo"] + 2
            assert 2 <= f["quantity"]["value"] <= 51
        else:
            assert [p["dim"] for p in spec["probes"]] == ["part", "supplier", "date", "customer"]


def test_latency_stats():
    rs = []
    for i in range(200):
        r = serve.Request(i * 0.01, "FA" if i % 2 else "SJ", {}, "res")
        r.issued = r.t + 0.0005
        r.done = r.t + 0.001 * (1 + (i % 100))
        rs.append(r)
    st = serve.latency_stats(rs, 2.0)
    assert st["completed"] == 200 and st["qps"] == 100.0
    lat = np.array([(r.done - r.t) * 1e3 for r in rs])
    assert st["p50_ms"] == np.percentile(lat, 50) and st["p99_ms"] == np.percentile(lat, 99)
    assert st["FA"]["n"] == 100 and st["SJ"]["n"] == 100
    assert abs(st["queue_wait_p50_ms"] - 0.5) < 1e-9
    assert abs(st["service_p50_ms"] + st["queue_wait_p50_ms"] - st["p50_ms"]) < 1e-6
    assert serve.latency_stats([], 1.0)["completed"] == 0


def test_tune_grid_respects_lds():
    pts = list(tune._points(tune.GRID))
    assert all(p["wg_per_cu"] * p["lds_hash_bytes"] <= tune.MAX_LDS_PER_CU for p in pts)
    full = len(tune.GRID["rows_per_item"]) * len(tune.GRID["wg_per_cu"]) * len(tune.GRID["lds_hash_bytes"])
    assert 0 < len(pts) < full
    assert {"rows_per_item": 131072, "wg_per_cu": 4, "lds_hash_bytes": 65536} not in pts


def test_tune_chunks_picks_the_fastest_encoding(monkeypatch):
    """The chunk-size axis: every size in CHUNK_ROWS is encoded, tuned under
    its own cache tag and released; the winner carries its chunk size and
    launch knobs."""
    made, released, tags = [], [], []
    fake_ms = {16384: 3.0, 32768: 2.0, 65536: 2.5, 131072: 4.0}

    def fake_tune(ctx, plans, grid, reps, cache, refresh, stream, log, tag=""):
        tags.append(tag)
        rows = plans[0]
        return {"best": {"rows_per_item": rows * 2, "wg_per_cu": 2, "lds_hash_bytes": 0}, "ms": fake_ms[rows]}

    def make(rows):
        made.append(rows)
        return [rows], lambda: released.append(rows)

    monkeypatch.setattr(tune, "tune", fake_tune)
    out = tune.tune_chunks(None, make)
    assert made == tune.CHUNK_ROWS == released
    assert tags == [f"chunk_rows={r}" for r in tune.CHUNK_ROWS]
    assert out["best"] == {"chunk_rows": 32768, "rows_per_item": 65536, "wg_per_cu": 2, "lds_hash_bytes": 0}
    assert out["ms"] == 2.0 and len(out["per_chunk"]) == 4


def test_union_table_has_both_templates():
    t = W.union_table(5000, seed=5)
    for c in ("date", "quantity", "price", "discount", "flagA", "flagB",
              "lo_datekey", "lo_custkey", "lo_suppkey", "lo_partkey", "lo_revenue"):
        assert len(t[c]) == 5000
    assert np.all(np.diff(t["date"]) >= 0)
