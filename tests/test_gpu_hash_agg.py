"""GPU parity for hash aggregation (paper Section 3.1, Kernel #3's hash
aggregation table): group-key domains above the 2^22 slots of a direct
table take an open-addressing table in HBM, fused and fragmented, against
the oracle -- nearly every row its own group, a huge domain holding a few
groups, a batch beside a direct-table plan with a HIP graph replayed three
times, and the allocation-free entry point twice in a row."""
import numpy as np
import pytest

import oracle
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_10511_amd import dpf
    assert torch.cuda.is_available()
    return dpf.Context(0)


def _table(n, seed, a_hi=99_999, b_hi=999):
    rng = np.random.default_rng(seed)
    return {"a": rng.integers(0, a_hi + 1, n).astype(np.int32),
            "b": rng.integers(0, b_hi + 1, n).astype(np.int32),
            "x": rng.integers(-1000, 100_000, n).astype(np.int64),
            "d": rng.integers(0, 200, n).astype(np.int32)}


def _spec(table="t", keys=("a", "b"), d_lt=150):
    return {"fact": table, "filters": [{"col": "d", "op": "LT", "value": d_lt}], "probes": [],
            "group_by": [{"col": k} for k in keys],
            "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "x"}}]},
                     {"op": "SUM", "terms": [{"ref": {"col": "x"}}, {"ref": {"col": "b"}, "add": 1}]}]}


@pytest.mark.parametrize("n,chunk_rows", [(1, 65536), (5_000, 65536), (200_003, 65536), (200_003, 4096)])
def test_distinct_groups(ctx, n, chunk_rows):
    """A 10^8-value domain: almost every qualifying row is its own group."""
    G.say(f"hash agg distinct n={n} chunk_rows={chunk_rows}")
    t = _table(n, seed=n)
    db = G.make_db(ctx, {"t": t}, chunk_rows=chunk_rows)
    spec = _spec()
    want = oracle.run(spec, {"t": t})
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"n={n} {mode}")


def test_few_groups_in_a_huge_domain(ctx):
    """Three keys spanning ~2^40 values, but only a dozen groups: every
    row lands on a slot that is already taken."""
    G.say("hash agg few groups")
    n = 300_000
    rng = np.random.default_rng(5)
    t = _table(n, seed=6)
    t["a"] = (rng.integers(0, 3, n) * 40_000_000).astype(np.int32)
    t["b"] = (rng.integers(0, 2, n) * 1_000_000).astype(np.int32)
    t["c"] = rng.choice(np.array([0, 9_999], np.int32), n)
    db = G.make_db(ctx, {"t": t})
    spec = _spec(keys=("a", "b", "c"))
    want = oracle.run(spec, {"t": t})
    assert 1 < len(want) <= 12
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, mode)


def test_batch_and_graph_replay(ctx):
    """A hash-table plan and a direct-table plan in one launch, eagerly and
    replayed from a HIP graph three times (the table's keys are cleared by
    every execution)."""
    import torch
    from paper_2605_10511_amd import dpf
    G.say("hash agg batch + graph")
    t = _table(120_001, seed=11)
    db = G.make_db(ctx, {"t": t})
    specs = [_spec(), _spec(keys=("d",)), _spec(d_lt=40)]
    wants = [oracle.run(s, {"t": t}) for s in specs]
    plans = [db.plan(s) for s in specs]
    res = dpf.execute(ctx, plans)
    torch.cuda.synchronize()
    for i, w in enumerate(wants):
        G.assert_same(res.get(i), w, f"eager plan {i}")
    res.release()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            r = dpf.execute(ctx, plans, stream=s)
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        for i, w in enumerate(wants):
            G.assert_same(r.get(i), w, f"replay {k} plan {i}")
        e = dpf.execute(ctx, plans[:1], mode="FRAGMENTED")
        torch.cuda.synchronize()
        G.assert_same(e.get(0), wants[0], f"fragmented after replay {k}")
        e.release()
    r.release()
    del g
    for p in plans:
        p.release()


def test_noalloc_twice(ctx):
    """The allocation-free entry point on a hash-table plan, then on a
    smaller one: its static table keeps the last call's contents, so the
    keys must start cleared."""
    import torch
    from paper_2605_10511_amd import dpf
    G.say("hash agg noalloc")
    for n in (20_000, 7_001):
        t = _table(n, seed=n)
        db = G.make_db(ctx, {"t": t})
        spec = _spec()
        p = db.plan(spec)
        r = dpf.execute_noalloc(ctx, [p])
        torch.cuda.synchronize()
        G.assert_same(r.get(0), oracle.run(spec, {"t": t}), f"noalloc n={n}")
        r.release()
        p.release()


def test_domain_limits(ctx):
    """A domain above 2^62 (three 32-bit keys) is refused; one of 2^32 over
    1,000 rows takes a 2,048-slot table; a hash table above 2^22 slots is
    refused, and the same table still groups by a small key."""
    from paper_2605_10511_amd import dpf
    n = 1000
    rng = np.random.default_rng(3)
    t = {k: rng.integers(-2**31, 2**31 - 1, n).astype(np.int64) for k in ("p", "q", "r")}
    t["d"] = np.zeros(n, np.int32)
    t["x"] = np.ones(n, np.int64)
    t["b"] = np.zeros(n, np.int32)
    db = G.make_db(ctx, {"t": t})
    with pytest.raises(dpf.DpfError):
        db.plan(_spec(keys=("p", "q", "r")))
    spec = _spec(keys=("p", "b"), d_lt=1)
    G.assert_same(G.run_gpu(db, spec), oracle.run(spec, {"t": t}), "2^32 domain over 1000 rows")
    # 2^21 + 1 rows under a 10^8 range would need 2^23 slots: refused
    big = _table(2**21 + 1, seed=4)
    dbb = G.make_db(ctx, {"t": big})
    with pytest.raises(dpf.DpfError):
        dbb.plan(_spec())
    G.assert_same(G.run_gpu(dbb, _spec(keys=("b",))), oracle.run(_spec(keys=("b",)), {"t": big}), "direct table")
