"""GPU parity: the library's fused and fragmented executions against the CPU
oracle, bit-exactly, on seeded inputs spanning several mini blocks, chunks
and a ragged tail; plus hand-computed cases, batching, host-mapped placement,
graph replay and device-reported errors."""
import numpy as np
import pytest

import oracle
from datagen import workloads as W
from tests import gpu_util as G
from tests.test_oracle_pins import _random_instance, _random_query

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_10511_amd import dpf
    assert torch.cuda.is_available()
    return dpf.Context(0)


def test_hand_cases(ctx, hand_cases):
    from paper_2605_10511_amd import dpf
    tables, cases = hand_cases
    db = G.make_db(ctx, tables, chunk_rows=256)
    for case in cases:
        G.say("hand case", case["name"])
        if "error" in case:
            want = {"duplicate": dpf.DPF_ERR_DUPLICATE_KEY, "overflow": dpf.DPF_ERR_OVERFLOW}[case["error"]]
            with pytest.raises(dpf.DpfError) as e:
                G.run_gpu(db, case["query"])
            assert e.value.code == want, case["name"]
            continue
        for mode in ("FUSED", "FRAGMENTED"):
            got = G.run_gpu(db, case["query"], mode=mode)
            assert got.tolist() == case["expect"], (case["name"], mode)


def test_filter_aggregate_1m(ctx):
    G.say("filter-aggregate 1,000,000 rows")
    t = W.fa_table(1_000_000, seed=1)
    spec = W.fa_query()
    want = oracle.run(spec, {"fact": t})
    db = G.make_db(ctx, {"fact": t}, {"fact": W.FA_ENCODINGS})
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, mode)
    for rpi, wg in ((256, 1), (16384, 2), (131072, 4)):
        G.assert_same(G.run_gpu(db, spec, rows_per_item=rpi, wg_per_cu=wg), want, f"items {rpi} wg {wg}")


@pytest.mark.parametrize("chunk_rows", [256, 65536])
def test_filter_aggregate_ragged(ctx, chunk_rows):
    G.say("filter-aggregate ragged, chunk", chunk_rows)
    t = W.fa_table(70_001, seed=5)
    for spec in (W.fa_query(), W.fa_query(date_lt=100, disc_lo=0, disc_hi=10, qty_lt=51),
                 W.fa_query(date_lt=0)):
        want = oracle.run(spec, {"fact": t})
        db = G.make_db(ctx, {"fact": t}, {"fact": W.FA_ENCODINGS}, chunk_rows=chunk_rows)
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, mode)


def test_wide_strings(ctx):
    G.say("wide table with strings, 300,000 rows")
    t = W.wide_table(300_000, seed=2)
    w1, w2, vocab = W.wide_words(2)
    db = G.make_db(ctx, {"fact": t}, {"fact": W.WIDE_ENCODINGS})
    for (a, b) in ((w1, w2), (w2, w1), (vocab[5][:2], vocab[9][:1]), (b"a", b"e"), (b" ", b" ")):
        spec = W.wide_query(a, b)
        want = oracle.run(spec, {"fact": t})
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{a}/{b} {mode}")


def test_long_strings(ctx):
    """Strings of up to 300 bytes: a mini block's heap spans up to ~38 of the
    string scan's 2 KB segments, so both segment buffers alternate many times
    and hit records carry across segment boundaries."""
    G.say("long strings")
    from tests.conftest import to_strings
    rng = np.random.default_rng(4)
    n = 2000
    items = []
    for i in range(n):
        L = int(rng.integers(0, 300))
        s = bytes(rng.choice(np.frombuffer(b"ab c", np.uint8), L))
        items.append(s)
    t = {"s": to_strings(items), "g": (np.arange(n) % 3).astype(np.int32)}
    db = G.make_db(ctx, {"t": t})
    for a, b in ((b"ab", b"c"), (b"abc", b"ba"), (b"a", b"a"), (b"c c", b"b")):
        spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": a, "s2": b}],
                "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
        want = oracle.run(spec, {"t": t})
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{a}/{b} {mode}")


@pytest.mark.parametrize("n1,n2", [(1, 1), (3, 5), (4, 4), (5, 6), (6, 7), (7, 7), (7, 9), (8, 8),
                                   (9, 12), (12, 7), (16, 3), (32, 8)])
def test_string_scan_modes(ctx, n1, n2):
    """Every scan mode of the string test (some word under 4 bytes, under 7,
    or both at least 7) on a five-letter alphabet, so that prefix hits are
    dense and queue overflows happen, with rows long enough that a mini
    block's heap spans several segments; words are planted at every byte
    alignment, in order, reversed and overlapping."""
    G.say("string scan modes", n1, n2)
    from tests.conftest import to_strings
    rng = np.random.default_rng(700 + 37 * n1 + n2)
    alpha = np.frombuffer(b"abcd ", np.uint8)
    s1 = bytes(rng.choice(alpha[:4], n1))
    s2 = bytes(rng.choice(alpha[:4], n2))
    n = 6000
    items = []
    for i in range(n):
        s = bytearray(rng.choice(alpha, int(rng.integers(0, 90))).tobytes())
        r = rng.random()
        if r < 0.15:
            a = int(rng.integers(0, len(s) + 1))
            s[a:a] = s1
            b = int(rng.integers(a + n1, len(s) + 1))
            s[b:b] = s2
        elif r < 0.25:
            a = int(rng.integers(0, len(s) + 1))
            s[a:a] = s2 + s1  # wrong order (unless they overlap into a match)
        elif r < 0.3:
            s = bytearray((s1 + s2)[: max(0, n1 + n2 - 1)])  # one byte short
        items.append(bytes(s))
    t = {"s": to_strings(items), "g": (np.arange(n) % 5).astype(np.int32)}
    db = G.make_db(ctx, {"t": t}, chunk_rows=2048)
    spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": s1, "s2": s2}],
            "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
    want = oracle.run(spec, {"t": t})
    assert sum(r[-1] for r in want) > 0
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{s1}/{s2} {mode}")


def test_string_table_fallback(ctx):
    """Words whose first 4-byte shifts are bitwise complements collide in
    every rotation's slot (x ^ rotr(x, r) is the same for x and ~x), so the
    plan gets no lookup table and the kernel compares byte windows."""
    G.say("string table fallback")
    from tests.conftest import to_strings
    s1 = b"abcdefg"
    s2 = bytes(255 - c for c in s1[:4]) + b"xyz"
    rng = np.random.default_rng(11)
    alpha = np.frombuffer(b"abcdefgxyz ", np.uint8)
    n = 5000
    items = []
    for i in range(n):
        s = bytearray(rng.choice(alpha, int(rng.integers(0, 60))).tobytes())
        r = rng.random()
        if r < 0.2:
            a = int(rng.integers(0, len(s) + 1))
            s[a:a] = s1
            b = int(rng.integers(a + len(s1), len(s) + 1))
            s[b:b] = s2
        elif r < 0.3:
            s[0:0] = s2 + s1
        items.append(bytes(s))
    t = {"s": to_strings(items), "g": (np.arange(n) % 4).astype(np.int32)}
    db = G.make_db(ctx, {"t": t}, chunk_rows=2048)
    spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": s1, "s2": s2}],
            "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
    want = oracle.run(spec, {"t": t})
    assert sum(r[-1] for r in want) > 0
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, mode)


def test_chunk_pruning(ctx):
    """Zone-map pruning of whole chunks: date-clustered and key-clustered
    columns in 2,048-row chunks, predicates that rule out most chunks (a
    range, NE on a per-chunk constant, IN, a string too long for the short
    rows, a probe whose qualifying keys cover few chunks' foreign keys) and
    one that rules out every chunk.  Fused (pruned) and fragmented (full)
    executions agree with the oracle, and the plan reports the blocks it
    skips."""
    G.say("chunk pruning")
    from paper_2605_10511_amd import dpf
    from tests.conftest import to_strings
    rng = np.random.default_rng(21)
    n = 200_000 + 77
    date = np.sort(rng.integers(0, 2556, n)).astype(np.int32)
    seg = (np.arange(n) // 2048).astype(np.int32)  # constant per chunk
    fk = (np.arange(n) // 40).astype(np.int32)     # clustered foreign key
    val = rng.integers(1, 1000, n).astype(np.int64)
    g = (rng.integers(0, 3, n)).astype(np.int32)
    items = [bytes(rng.choice(np.frombuffer(b"ab ", np.uint8), int(rng.integers(0, 12) if i < n // 2 else rng.integers(20, 40))))
             for i in range(n)]
    for i in range(n // 2, n, 7):
        items[i] = b"aab" + items[i][3:] + b"bba" * 5
    fact = {"date": date, "seg": seg, "fk": fk, "val": val, "g": g, "s": to_strings(items)}
    nd = n // 40 + 1
    dim = {"k": np.arange(nd, dtype=np.int32), "cat": (np.arange(nd) % 5).astype(np.int32),
           "zone": (np.arange(nd) // 500).astype(np.int32)}
    tables = {"f": fact, "d": dim}
    db = G.make_db(ctx, tables, {"f": {"date": "DELTA"}}, chunk_rows=2048)
    aggs = [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "val"}}]}]
    base = {"fact": "f", "probes": [], "group_by": [{"col": "g"}], "aggs": aggs}
    cases = [
        ("range", {**base, "filters": [{"col": "date", "op": "BETWEEN", "lo": 600, "hi": 700}]}, True),
        ("ne", {**base, "filters": [{"col": "seg", "op": "NE", "value": 3},
                                    {"col": "date", "op": "LT", "value": 300}]}, True),
        ("in", {**base, "filters": [{"col": "seg", "op": "IN", "values": [5, 9, 40]}]}, True),
        ("string", {**base, "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": b"aab", "s2": b"bba" * 5}]}, True),
        ("string-short", {**base, "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": b"aab", "s2": b"bba"}]}, False),
        ("probe", {**base, "filters": [],
                   "probes": [{"fk": "fk", "dim": "d", "key": "k", "filters": [{"col": "zone", "op": "EQ", "value": 3}],
                               "payloads": ["cat"]}],
                   "group_by": [{"probe": 0, "payload": 0}]}, True),
        ("none", {**base, "filters": [{"col": "date", "op": "GT", "value": 9999}]}, True),
        ("unpruned", {**base, "filters": [{"col": "val", "op": "LT", "value": 500}]}, False),
    ]
    wants = []
    for name, spec, prunes in cases:
        want = oracle.run(spec, tables)
        wants.append(want)
        plan = db.plan(spec)
        scanned, total = plan.blocks()
        plan.release()
        for h in plan.hashes:
            h.release()
        assert total == (n + 2047) // 2048, name
        assert (scanned < total) == prunes, (name, scanned, total)
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{name} {mode}")
    # every case in one fused launch: pruned, unpruned and empty plans share
    # the work queue, with the default and a caller's item size
    import torch
    plans = [db.plan(spec) for _, spec, _ in cases]
    for kw in ({}, {"rows_per_item": 1024}):
        res = dpf.execute(ctx, plans, **kw)
        torch.cuda.synchronize()
        for k, (name, _, _) in enumerate(cases):
            G.assert_same(res.get(k), wants[k], f"batch {name} {kw}")
        res.release()
    for p in plans:
        p.release()
        for h in p.hashes:
            h.release()


def test_plain_columns(ctx):
    """Every integer column PLAIN (full width, the uncompressed reference):
    the wide query with strings and a small star join, fused and fragmented,
    against the oracle."""
    G.say("plain columns")
    t = W.wide_table(120_000, seed=2)
    w1, w2, _ = W.wide_words(2)
    enc = {c: ("VARLEN" if c == "comment" else "PLAIN") for c in t}
    db = G.make_db(ctx, {"fact": t}, {"fact": enc})
    spec = W.wide_query(w1, w2)
    want = oracle.run(spec, {"fact": t})
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"wide {mode}")
    dims = W.sj_dims(seed=3, scale=0.01)
    fact = W.sj_fact(300_000, seed=3, dims=dims)
    tables = {"lo": fact, **dims}
    spec = W.sj_query(part_category=4, date_dow=None)
    want = oracle.run(spec, tables)
    db = G.make_db(ctx, tables, {"lo": {c: "PLAIN" for c in fact}})
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"sj {mode}")


@pytest.mark.parametrize("variant", ["3a", "3b"])
def test_star_join_small(ctx, variant):
    G.say("star join small", variant)
    # at 1/100 of the dimension sizes the 1/1000 part filter leaves almost
    # no fact rows, so the small test filters part by category (1/25)
    dims = W.sj_dims(seed=3, scale=0.01)
    fact = W.sj_fact(1_000_000, seed=3, dims=dims)
    spec = (W.sj_query(part_category=4, date_dow=2) if variant == "3a"
            else W.sj_query(date_dow=None, part_category=4))
    tables = {"lo": fact, **dims}
    want = oracle.run(spec, tables)
    assert len(want) > 0
    db = G.make_db(ctx, tables)
    for placements in (None, ["HBM", "LDS", "LDS", "HBM"], ["HBM"] * 4, ["LDS"] * 4):
        for mode in ("FUSED", "FRAGMENTED"):
            got = G.run_gpu(db, spec, mode=mode, placements=placements)
            G.assert_same(got, want, f"{placements} {mode}")


@pytest.mark.parametrize("seed", range(12))
def test_random_queries(ctx, seed):
    G.say("random queries seed", seed)
    from paper_2605_10511_amd import dpf
    rng = np.random.default_rng(5000 + seed)
    tables = _random_instance(rng, n=3000 + 97 * seed)
    db = G.make_db(ctx, tables, chunk_rows=512)
    for _ in range(4):
        spec = _random_query(rng)
        try:
            want = oracle.run(spec, tables)
        except oracle.OracleError as e:
            if e.code == oracle.ERR_DUPLICATE:
                continue
            raise
        for mode in ("FUSED", "FRAGMENTED"):
            try:
                got = G.run_gpu(db, spec, mode=mode)
            except dpf.DpfError as e:
                # the static int64 bound may refuse a plan the data never overflows
                assert e.code == dpf.DPF_ERR_OVERFLOW, e
                continue
            G.assert_same(got, want, f"{spec} {mode}")


def test_batch_equals_solo(ctx):
    G.say("batched plans in one launch")
    import torch
    from paper_2605_10511_amd import dpf
    fa = W.fa_table(200_000, seed=8)
    fa2 = W.fa_table(35_000, seed=9)
    dims = W.sj_dims(seed=3, scale=0.01)
    lo = W.sj_fact(150_000, seed=10, dims=dims)
    tables = {"fa": fa, "fa2": fa2, "lo": lo, **dims}
    db = G.make_db(ctx, tables, {"fa": W.FA_ENCODINGS, "fa2": W.FA_ENCODINGS})
    specs = [W.fa_query("fa"), W.fa_query("fa2", date_lt=900, disc_lo=2, disc_hi=4, qty_lt=40),
             W.sj_query(part_category=3, date_dow=None), W.sj_query(part_attr=5),
             W.fa_query("fa", date_lt=2555, disc_lo=0, disc_hi=10, qty_lt=51)]
    wants = [oracle.run(s, tables) for s in specs]
    plans = [db.plan(s) for s in specs]
    for rpi in (0, 16384):
        res = dpf.execute(ctx, plans, rows_per_item=rpi)
        torch.cuda.synchronize()
        for i, w in enumerate(wants):
            G.assert_same(res.get(i), w, f"batch plan {i}")
        res.release()
    for i, p in enumerate(plans):
        res = dpf.execute(ctx, [p])
        torch.cuda.synchronize()
        G.assert_same(res.get(0), wants[i], f"solo plan {i}")
        res.release()


def test_host_mapped_equals_hbm(ctx):
    G.say("host-mapped placement")
    t = W.fa_table(300_000, seed=11)
    spec = W.fa_query()
    want = oracle.run(spec, {"fact": t})
    for place in ("HBM", "HOST_MAPPED"):
        db = G.make_db(ctx, {"fact": t}, {"fact": W.FA_ENCODINGS}, placement=place)
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{place} {mode}")


def test_corrupt_header_reported(ctx):
    G.say("corrupt mini-block header")
    from paper_2605_10511_amd import dpf
    t = W.fa_table(20_000, seed=12)
    spec = W.fa_query()
    db = G.make_db(ctx, {"fact": t}, {"fact": W.FA_ENCODINGS}, placement="HOST_MAPPED")
    offs = db.tables["fact"]["quantity"].debug_offsets()
    saved = offs[5]
    offs[5] = saved + 3  # no longer a whole number of 8-word groups
    with pytest.raises(dpf.DpfError) as e:
        G.run_gpu(db, spec)
    assert e.value.code == dpf.DPF_ERR_CORRUPT
    offs[5] = saved
    G.assert_same(G.run_gpu(db, spec), oracle.run(spec, {"fact": t}), "after repair")


def test_hash_stats_and_duplicates(ctx):
    G.say("hash build stats")
    from paper_2605_10511_amd import dpf
    dims = W.sj_dims(seed=3, scale=0.01)
    cols = {c: dpf.Column(ctx, v) for c, v in dims["part"].items()}
    h = dpf.Hash(ctx, cols, "p_partkey", [{"col": "p_category", "op": "EQ", "value": 7}], ["p_brand"])
    s = h.info()
    m = dims["part"]["p_category"] == 7
    assert s.entries == int(m.sum())
    assert s.capacity >= 2 * s.entries and s.capacity & (s.capacity - 1) == 0
    assert s.payload_min[0] == dims["part"]["p_brand"][m].min()
    assert s.payload_max[0] == dims["part"]["p_brand"][m].max()
    dup = {"k": dpf.Column(ctx, np.array([1, 2, 3, 2], np.int32))}
    with pytest.raises(dpf.DpfError) as e:
        dpf.Hash(ctx, dup, "k", [], [])
    assert e.value.code == dpf.DPF_ERR_DUPLICATE_KEY


def test_graph_replay(ctx):
    G.say("graph capture and replay")
    import torch
    from paper_2605_10511_amd import dpf
    t = W.fa_table(500_000, seed=13)
    spec = W.fa_query()
    want = oracle.run(spec, {"fact": t})
    db = G.make_db(ctx, {"fact": t}, {"fact": W.FA_ENCODINGS})
    plan = db.plan(spec)
    res = dpf.execute(ctx, [plan])  # warm (sets the LDS layout once)
    torch.cuda.synchronize()
    G.assert_same(res.get(0), want, "eager")
    res.release()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            r = dpf.execute(ctx, [plan], stream=s)
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        G.assert_same(r.get(0), want, f"replay {k}")
        res = dpf.execute(ctx, [plan])
        torch.cuda.synchronize()
        G.assert_same(res.get(0), want, f"eager after replay {k}")
        res.release()
    r.release()


@pytest.mark.parametrize("cut", [0, 255, 256, 1000, 2555, 2556, 9999])
def test_zone_decided_atoms(ctx, cut):
    """Atoms that a mini block's header settles (all rows pass / none) must
    give the same rows as decoding: ascending and descending DELTA columns
    (negative minimum difference), a constant column (width 0), and range,
    NE and EQ atoms with cut points inside, between and outside blocks."""
    n = 70_000
    asc = W.fa_table(n, seed=9)["date"]
    desc_ = asc[::-1].copy()
    const = np.full(n, 7, dtype=np.int32)
    qty = W.fa_table(n, seed=9)["quantity"]
    t = {"z": {"asc": asc, "desc": desc_, "const": const, "qty": qty}}
    enc = {"z": {"asc": "DELTA", "desc": "DELTA", "const": "FOR", "qty": "FOR"}}
    db = G.make_db(ctx, t, enc, chunk_rows=65536)
    cases = [
        [{"col": "asc", "op": "LT", "value": cut}],
        [{"col": "asc", "op": "GE", "value": cut}, {"col": "qty", "op": "LT", "value": 30}],
        [{"col": "desc", "op": "BETWEEN", "lo": cut - 300, "hi": cut}],
        [{"col": "const", "op": "NE", "value": 7 if cut % 2 else cut}],
        [{"col": "const", "op": "EQ", "value": 7}, {"col": "desc", "op": "GT", "value": cut}],
        [{"col": "asc", "op": "NE", "value": cut}],
    ]
    for f in cases:
        spec = {"fact": "z", "filters": f, "probes": [], "group_by": [],
                "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "qty"}}]}]}
        G.say(f"zone cut {cut}: {f}")
        G.assert_same(G.run_gpu(db, spec), oracle.run(spec, t), f"zone {f}")


@pytest.mark.parametrize("cap", [1, 3, 64])
def test_grid_cap(ctx, cap):
    """A capped grid (max_workgroups) drains the same work queue: same rows."""
    t = {"fact": W.fa_table(300_000, seed=5)}
    db = G.make_db(ctx, t, {"fact": W.FA_ENCODINGS})
    spec = W.fa_query()
    G.say(f"grid cap {cap}")
    G.assert_same(G.run_gpu(db, spec, max_workgroups=cap), oracle.run(spec, t), f"cap {cap}")


@pytest.mark.parametrize("mode", ["FUSED", "FRAGMENTED"])
def test_delta_cuts_every_path(ctx, mode):
    """A sorted DELTA column cut at many points, by every execution path: the
    fragmented kernels decode every mini block (no header shortcut), the
    fused one decodes the blocks the header does not settle."""
    t = {"fact": W.fa_table(1_300_000, seed=400)}
    db = G.make_db(ctx, t, {"fact": W.FA_ENCODINGS})
    for c in (100, 1500, 1882, 2203, 2555):
        spec = {"fact": "fact", "filters": [{"col": "date", "op": "LT", "value": c}], "probes": [],
                "group_by": [{"col": "flagA"}],
                "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "date"}}]}]}
        G.say(f"{mode} date < {c}")
        G.assert_same(G.run_gpu(db, spec, mode=mode), oracle.run(spec, t), f"{mode} date < {c}")
