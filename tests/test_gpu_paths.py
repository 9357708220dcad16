"""GPU parity for kernel paths the workload configs do not reach on their own:
group tables too large for a workgroup's LDS (rows aggregate straight into
device memory), dimension tables whose keys span too wide a range for a
membership bitmap (hash chains walked in lockstep, with long forced chains),
variable-length heaps read from pinned host memory, and a 64-plan batch run
eagerly and replayed from a HIP graph.  Every result is compared with the
CPU oracle element by element, for the fused and the fragmented execution."""
import numpy as np
import pytest

import oracle
from datagen import uniform
from datagen import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_10511_amd import dpf
    assert torch.cuda.is_available()
    return dpf.Context(0)


def _wide_groups_table(n: int, seed: int) -> dict:
    return {
        "g": uniform(seed, "g", n, 0, 2999, dtype=np.int32),      # 3,000 group values
        "h": uniform(seed, "h", n, 0, 6, dtype=np.int32),
        "v": uniform(seed, "v", n, 1, 1000, dtype=np.int64),
        "w": uniform(seed, "w", n, -500, 500, dtype=np.int64),
        "x": uniform(seed, "x", n, 0, 99, dtype=np.int32),
        "fk": uniform(seed, "fk", n, 0, 399, dtype=np.int32),
    }


def test_group_table_in_device_memory(ctx):
    """3,000 (or 21,000) groups x 4 accumulators: 96 KB and more of int64,
    beyond the 16 KB a workgroup keeps in LDS, so stage B adds every row into
    the plan's device table and the workgroup publishes through a release
    fence.  Covers a filtered plan, an unfiltered unjoined one (every row
    through stage B) and a plan grouped by a probe payload; then all three in
    one launch beside a plan whose table does fit LDS."""
    import torch
    from paper_2605_10511_amd import dpf
    n = 150_001
    fact = _wide_groups_table(n, seed=61)
    dim = {"k": np.arange(400, dtype=np.int32), "cat": (np.arange(400) * 7 % 1000).astype(np.int32)}
    tables = {"f": fact, "d": dim}
    aggs = [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "v"}}]},
            {"op": "SUM", "terms": [{"ref": {"col": "v"}}, {"ref": {"col": "x"}, "mul": -1, "add": 100}]},
            {"op": "AVG", "terms": [{"ref": {"col": "w"}}]}]
    specs = {
        "filtered": {"fact": "f", "filters": [{"col": "x", "op": "LT", "value": 60}], "probes": [],
                     "group_by": [{"col": "g"}], "aggs": aggs},
        "two keys, no filter": {"fact": "f", "filters": [], "probes": [],
                                "group_by": [{"col": "g"}, {"col": "h"}], "aggs": aggs},
        "payload key": {"fact": "f", "filters": [{"col": "h", "op": "NE", "value": 3}],
                        "probes": [{"fk": "fk", "dim": "d", "key": "k",
                                    "filters": [{"col": "k", "op": "GE", "value": 50}], "payloads": ["cat"]}],
                        "group_by": [{"probe": 0, "payload": 0}, {"col": "h"}], "aggs": aggs},
        "small table": {"fact": "f", "filters": [{"col": "x", "op": "GE", "value": 90}], "probes": [],
                        "group_by": [{"col": "h"}], "aggs": aggs},
    }
    db = G.make_db(ctx, tables, chunk_rows=16384)
    wants = {}
    for name, spec in specs.items():
        wants[name] = oracle.run(spec, tables)
        assert len(wants[name]) > 0
        for mode in ("FUSED", "FRAGMENTED"):
            G.say(f"device group table: {name} {mode}")
            G.assert_same(G.run_gpu(db, spec, mode=mode), wants[name], f"{name} {mode}")
    plans = [db.plan(s) for s in specs.values()]
    for kw in ({}, {"rows_per_item": 1024, "wg_per_cu": 1}):
        G.say(f"device group tables in one launch {kw}")
        res = dpf.execute(ctx, plans, **kw)
        torch.cuda.synchronize()
        for i, name in enumerate(specs):
            G.assert_same(res.get(i), wants[name], f"batch {name} {kw}")
        res.release()
    for p in plans:
        p.release()
        for h in p.hashes:
            h.release()


def _colliding_keys(count: int, log2cap: int, slots: int, n: int, lo: int, avoid: set) -> list:
    """n int32 keys >= lo whose multiplicative hash (the table's slot
    function: key * 0x9E3779B1 mod 2^32, top log2cap bits) lands in the first
    ``slots`` slots of a table of 2^log2cap slots: they form one long
    linear-probing chain."""
    out = []
    k = lo
    while len(out) < n:
        cand = np.arange(k, k + 1_000_000, dtype=np.uint64)
        h = ((cand * np.uint64(0x9E3779B1)) & np.uint64(0xFFFFFFFF)) >> np.uint64(32 - log2cap)
        for c in cand[h < slots].tolist():
            if c not in avoid:
                out.append(int(c))
                if len(out) == n:
                    break
        k += 1_000_000
    return out


def test_probe_without_bitmap(ctx):
    """Dimension keys spread over more than 2^25 values get no membership
    bitmap, so the semi-join of the first probe walks the hash chains in
    lockstep (from LDS, or from device memory behind the LDS bit filter) and
    stage B finds payloads by chain walks.  A quarter of the keys share the
    first four slots of the table: their chain is hundreds of slots long, and
    fact keys that miss are drawn both inside and outside it."""
    from paper_2605_10511_amd import dpf
    spread = [7 + 40_000 * i for i in range(1500)]                    # span 6.0e7 > 2^25
    count = 2000
    log2cap = 12                                                       # capacity 4096 >= 2 * 2000
    chain = _colliding_keys(count, log2cap, 4, count - len(spread), 70_000_000, set(spread))
    keys = np.array(spread + chain, dtype=np.int32)
    perm = np.random.default_rng(5).permutation(len(keys))
    nk = len(keys)
    dim = {"k": keys[perm], "a": (np.arange(nk) % 5).astype(np.int32)[perm],
           "b": (np.arange(nk) % 13).astype(np.int32)[perm]}
    misses = _colliding_keys(count, log2cap, 4, 300, 90_000_000, set(chain)) + [3 + 40_000 * i for i in range(300)]
    n = 120_003
    rng = np.random.default_rng(17)
    pick = rng.integers(0, nk, n)
    miss = rng.random(n) < 0.4
    fk = np.where(miss, np.array(misses, dtype=np.int64)[rng.integers(0, len(misses), n)], keys[pick].astype(np.int64))
    second = {"k2": np.array([11 + 50_000 * i for i in range(900)], dtype=np.int32),
              "c": (np.arange(900) % 6).astype(np.int32)}
    fact = {"fk": fk.astype(np.int32), "fk2": second["k2"][rng.integers(0, 900, n)],
            "v": rng.integers(1, 1000, n).astype(np.int64)}
    tables = {"f": fact, "d": dim, "e": second}
    spec = {"fact": "f", "filters": [],
            "probes": [{"fk": "fk", "dim": "d", "key": "k", "filters": [{"col": "a", "op": "NE", "value": 9}],
                        "payloads": ["b"]},
                       {"fk": "fk2", "dim": "e", "key": "k2", "filters": [{"col": "c", "op": "LE", "value": 3}],
                        "payloads": ["c"]}],
            "group_by": [{"probe": 0, "payload": 0}, {"probe": 1, "payload": 0}],
            "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "v"}}]}]}
    want = oracle.run(spec, tables)
    assert len(want) > 0 and 0 < int(want[:, 2].sum()) < n
    db = G.make_db(ctx, tables, chunk_rows=8192)
    hs = db.build_hashes(spec)
    for h in hs:
        s = h.info()
        assert s.key_max - s.key_min >= (1 << 25), "the dimension must be too wide for a bitmap"
        h.release()
    for placements in (None, ["LDS", "LDS"], ["HBM", "HBM"], ["HBM", "LDS"]):
        for mode in ("FUSED", "FRAGMENTED"):
            G.say(f"no bitmap {placements} {mode}")
            G.assert_same(G.run_gpu(db, spec, mode=mode, placements=placements), want, f"{placements} {mode}")
    # the same probes behind a fact predicate: both probes in stage B
    spec2 = dict(spec, filters=[{"col": "v", "op": "LT", "value": 700}])
    want2 = oracle.run(spec2, tables)
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec2, mode=mode, placements=["HBM", "HBM"]), want2, f"filtered {mode}")
    with pytest.raises(dpf.DpfError):  # a duplicate among the colliding keys is still found
        dup = {"k": np.array(chain[:50] + chain[:1], dtype=np.int32)}
        dpf.Hash(ctx, {"k": dpf.Column(ctx, dup["k"])}, "k", [], [])


def test_strings_from_host_memory(ctx):
    """The wide table with every column, the string heap included, in pinned
    host memory that the kernels read over the host link: every scan mode of
    the string test, fused and fragmented."""
    t = W.wide_table(120_000, seed=2)
    w1, w2, vocab = W.wide_words(2)
    db = G.make_db(ctx, {"fact": t}, {"fact": W.WIDE_ENCODINGS}, chunk_rows=16384, placement="HOST_MAPPED")
    for (a, b) in ((w1, w2), (vocab[5][:2], vocab[9][:1]), (vocab[3][:5], vocab[7][:4])):
        spec = W.wide_query(a, b)
        want = oracle.run(spec, {"fact": t})
        for mode in ("FUSED", "FRAGMENTED"):
            G.say(f"host-mapped strings {a}/{b} {mode}")
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{a}/{b} {mode}")


def test_batch_of_64_and_graph_replay(ctx):
    """The batched mix at reduced sizes: 64 filter-aggregate and star-join
    plans over 8 tables in ONE launch with the automatic knobs (more than 8
    plans: no LDS dimension tables), against the oracle; then the same launch
    captured in a HIP graph and replayed three times, with eager launches and
    synchronisations between the replays, every replay checked."""
    import torch
    from paper_2605_10511_amd import dpf
    M = W.mix_plan(seed=4, min_rows=20_000, max_rows=400_000)
    dims = W.sj_dims(seed=3, scale=0.01)
    tables = dict(dims)
    for t, n in enumerate(M["fa_sizes"]):
        tables[f"fa{t}"] = W.fa_table(n, seed=400 + t)
    for t, n in enumerate(M["sj_sizes"]):
        tables[f"sj{t}"] = W.sj_fact(n, seed=440 + t, dims=dims, name=f"sj{t}")
    encs = {f"fa{t}": W.FA_ENCODINGS for t in range(len(M["fa_sizes"]))}
    db = G.make_db(ctx, tables, encs, chunk_rows=16384)
    specs = [q[2] for q in M["queries"]]
    # denser star joins at this scale: a part category (1/25) instead of one attribute value (1/1000)
    for k, (tmpl, _, sp) in enumerate(M["queries"]):
        if tmpl == "SJ" and k % 2:
            sp["probes"][0]["filters"] = [{"col": "p_category", "op": "EQ", "value": k % 25}]
    assert len(specs) == 64
    wants = [oracle.run(s, tables) for s in specs]
    assert sum(len(w) > 0 for w in wants) > 16
    plans = [db.plan(s) for s in specs]
    G.say("64 plans, eager")
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
        G.say(f"64 plans, graph replay {k}")
        g.replay()
        torch.cuda.synchronize()
        for i, w in enumerate(wants):
            G.assert_same(r.get(i), w, f"replay {k} plan {i}")
        e = dpf.execute(ctx, plans[k::7])  # eager work between replays
        torch.cuda.synchronize()
        for j, i in enumerate(range(k, 64, 7)):
            G.assert_same(e.get(j), wants[i], f"eager after replay {k}, plan {i}")
        e.release()
    r.release()
    del g
    for p in plans:
        p.release()
        for h in p.hashes:
            h.release()
