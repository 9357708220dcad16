"""GPU: the launch-knob tuner and the serving loop.  Served results must equal
the oracle's and a lone execution's, whatever batch they shared."""
import numpy as np
import pytest

import oracle
from datagen import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2605_10511_amd import dpf
    assert torch.cuda.is_available()
    ctx = dpf.Context(0)
    dims = W.sj_dims(seed=3, scale=0.01)
    res = W.union_table(300_000, seed=5, dims=dims)
    tables = {"res": res, **dims}
    db = G.make_db(ctx, tables, {"res": W.FA_ENCODINGS})
    return ctx, db, tables


def test_tuner_picks_a_measured_point(env, tmp_path):
    from paper_2605_10511_amd import dpf, tune
    ctx, db, tables = env
    specs = [W.fa_query("res"), W.sj_query("res", part_attr=3)]
    plans = [db.plan(s) for s in specs]
    grid = {"rows_per_item": [16384, 65536], "wg_per_cu": [1, 2], "lds_hash_bytes": [0, 32768]}
    cache = str(tmp_path / "tune.json")
    G.say("tuner: 8 points")
    e = tune.tune(ctx, plans, grid=grid, reps=2, cache=cache)
    ok = [t for t in e["table"] if t["ms"] is not None]
    assert ok and e["ms"] == min(t["ms"] for t in ok)
    again = tune.tune(ctx, plans, grid=grid, cache=cache)
    assert again["best"] == e["best"] and again["key"] == e["key"]
    import torch
    # a plan's executions share its result buffer: read each before the next
    r1 = dpf.execute(ctx, plans, **e["best"])
    torch.cuda.synchronize()
    tuned = [r1.get(i) for i in range(len(specs))]
    r1.release()
    r2 = dpf.execute(ctx, plans)
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        G.assert_same(tuned[i], oracle.run(s, tables), f"tuned plan {i}")
        G.assert_same(r2.get(i), tuned[i], f"default plan {i}")
    r2.release()
    for p in plans:
        p.release()


def _alone(ctx, db, srv, r):
    import torch
    from paper_2605_10511_amd import dpf
    p = db.plan(r.spec, hashes=[srv._hash(pr) for pr in r.spec.get("probes", [])])
    out = dpf.execute(ctx, [p])
    torch.cuda.synchronize()
    rows = out.get(0)
    out.release()
    p.release()
    return rows


def test_served_results_equal_oracle_and_alone(env):
    from paper_2605_10511_amd import serve
    ctx, db, tables = env
    gen = W.serve_requests(11, 400.0, 0.1, "res")
    reqs = [serve.Request(t, k, s, "res") for t, k, s in gen]
    G.say(f"serving {len(reqs)} requests")
    srv = serve.Server(ctx, db, nstreams=4, slots=8, state_budget=1 << 30)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert all(r.done >= r.t for r in done)
    for r in done:
        G.assert_same(r.rows, oracle.run(r.spec, tables), f"served {r.template} at {r.t:.4f}")
        G.assert_same(_alone(ctx, db, srv, r), r.rows, "alone vs served")
    srv.close()


def test_burst_mixes_requests(env):
    """A burst of 40 requests at time 0 with 4 plans per launch: the loop
    must put several requests into one launch and have several launches on
    the device at once (continuous batching, not a queue), and every result
    must equal the oracle's and a lone execution's."""
    from paper_2605_10511_amd import serve
    ctx, db, tables = env
    gen = W.serve_requests(21, 1000.0, 0.06, "res")[:40]
    reqs = [serve.Request(0.0, k, s, "res") for _, k, s in gen]
    assert len(reqs) == 40
    srv = serve.Server(ctx, db, nstreams=4, slots=16, state_budget=1 << 30, max_batch=4)
    srv.warm(reqs)
    G.say(f"burst of {len(reqs)} requests")
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert max(srv.batch_sizes) > 1, srv.batch_sizes
    assert srv.max_inflight > 1, srv.max_inflight
    G.say(f"batches {srv.batch_sizes}, at most {srv.max_inflight} in flight")
    for r in done:
        G.assert_same(r.rows, oracle.run(r.spec, tables), f"burst {r.template}")
        G.assert_same(_alone(ctx, db, srv, r), r.rows, "alone vs burst")
    srv.close()


def test_state_budget_serialises_batches(env):
    from paper_2605_10511_amd import serve
    ctx, db, tables = env
    gen = W.serve_requests(12, 1000.0, 0.02, "res")
    reqs = [serve.Request(t, k, s, "res") for t, k, s in gen]
    srv = serve.Server(ctx, db, nstreams=2, slots=8, state_budget=1)  # one request at a time
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    for r in done:
        G.assert_same(r.rows, oracle.run(r.spec, tables), "budget-limited")
    srv.close()


def test_host_table_requests_run_apart(env):
    """Requests on a host-mapped table run on their own stream, never in a
    resident batch; every result still equals the oracle's."""
    from paper_2605_10511_amd import serve
    ctx, db, tables = env
    host = W.union_table(120_000, seed=55, dims={k: tables[k] for k in ("date", "customer", "supplier", "part")})
    db.add_table("host", host, W.FA_ENCODINGS, placement="HOST_MAPPED")
    tabs = {**tables, "host": host}
    reqs = [serve.Request(t, k, s, "res") for t, k, s in W.serve_requests(13, 300.0, 0.05, "res")]
    reqs += [serve.Request(t, k, s, "host") for t, k, s in W.serve_requests(14, 100.0, 0.05, "host", stream="h")]
    G.say(f"serving {len(reqs)} requests, some on a host-mapped table")
    srv = serve.Server(ctx, db, nstreams=3, slots=8, state_budget=1 << 30, host_tables=("host",))
    srv.warm(reqs)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    for r in done:
        G.assert_same(r.rows, oracle.run(r.spec, tabs), f"served {r.table}/{r.template}")
    srv.close()
