"""GPU parity for FSST string columns (paper Sections 3.4.2 and 4.1) against
the unchanged oracle, which evaluates the string predicate on the raw
strings: the fused kernel's code-level automaton and the fragmented path's
two-pass record decode, on the string workload's comments (ragged sizes,
small chunks so that work items cross chunk boundaries, host-mapped
placement), on dense small alphabets with words planted at every position
(word completions inside symbols, the switch to the second word inside a
symbol, words up to 32 bytes), on arbitrary bytes (escape codes), and in a
batch beside a VARLEN plan."""
import numpy as np
import pytest

import oracle
from datagen import workloads as W
from tests import gpu_util as G
from tests.conftest import to_strings

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_10511_amd import dpf
    assert torch.cuda.is_available()
    return dpf.Context(0)


def _enc(fsst_col="comment"):
    e = dict(W.WIDE_ENCODINGS)
    e[fsst_col] = "FSST"
    return e


@pytest.mark.parametrize("n,chunk_rows,placement", [(1, 65536, "HBM"), (257, 65536, "HBM"),
                                                    (70_001, 65536, "HBM"), (70_001, 512, "HBM"),
                                                    (300_000, 65536, "HBM"), (100_003, 4096, "HOST_MAPPED")])
def test_comment_queries(ctx, n, chunk_rows, placement):
    G.say(f"fsst comments n={n} chunk_rows={chunk_rows} {placement}")
    t = W.wide_table(n, seed=2)
    w1, w2, vocab = W.wide_words(2)
    db = G.make_db(ctx, {"fact": t}, {"fact": _enc()}, chunk_rows=chunk_rows, placement=placement)
    assert db.tables["fact"]["comment"].info().encoding == 6
    for (a, b) in ((w1, w2), (w2, w1), (vocab[5][:2], vocab[9][:1]), (b"a", b"e"), (b" ", b" "),
                   (vocab[3], vocab[3]), (vocab[7] + b" " + vocab[8], b"q")):
        spec = W.wide_query(a, b)
        want = oracle.run(spec, {"fact": t})
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{a}/{b} {mode}")


@pytest.mark.parametrize("n1,n2", [(1, 1), (2, 3), (4, 4), (5, 9), (8, 8), (9, 12), (16, 3), (16, 16)])
def test_planted_words(ctx, n1, n2):
    """A four-letter alphabet, so that the chunk's symbols are long runs of
    the same letters as the words: words complete inside symbols, and the
    second word starts inside the symbol that ends the first."""
    G.say("fsst planted words", n1, n2)
    rng = np.random.default_rng(900 + 37 * n1 + n2)
    alpha = np.frombuffer(b"abcd ", np.uint8)
    s1 = bytes(rng.choice(alpha[:4], n1))
    s2 = bytes(rng.choice(alpha[:4], n2))
    n = 20_000
    items = []
    for i in range(n):
        s = bytearray(rng.choice(alpha, int(rng.integers(0, 90))).tobytes())
        r = rng.random()
        if r < 0.2:
            a = int(rng.integers(0, len(s) + 1))
            s[a:a] = s1
            b = int(rng.integers(a + n1, len(s) + 1))
            s[b:b] = s2
        elif r < 0.3:
            a = int(rng.integers(0, len(s) + 1))
            s[a:a] = s2 + s1
        elif r < 0.35:
            s = bytearray(s1 + s2)
        items.append(bytes(s))
    t = {"s": to_strings(items), "g": (np.arange(n) % 5).astype(np.int32)}
    db = G.make_db(ctx, {"t": t}, {"t": {"s": "FSST"}}, chunk_rows=2048)
    spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": s1, "s2": s2}],
            "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
    want = oracle.run(spec, {"t": t})
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{s1}/{s2} {mode}")


def test_escapes_and_arbitrary_bytes(ctx):
    """Random bytes: most codes are escapes or short symbols; the words hold
    bytes that no symbol starts with."""
    G.say("fsst arbitrary bytes")
    rng = np.random.default_rng(31)
    n = 30_000
    items = []
    for i in range(n):
        s = bytearray(rng.integers(0, 256, int(rng.integers(0, 40))).astype(np.uint8).tobytes())
        if i % 7 == 0:
            s[len(s) // 2:len(s) // 2] = b"\xfe\x00\x01" + bytes(rng.integers(0, 256, 3).astype(np.uint8)) + b"\xff\x80"
        items.append(bytes(s))
    t = {"s": to_strings(items), "g": (np.arange(n) % 3).astype(np.int32)}
    db = G.make_db(ctx, {"t": t}, {"t": {"s": "FSST"}}, chunk_rows=4096)
    for a, b in ((b"\xfe\x00\x01", b"\xff\x80"), (b"\xfe", b"\xfe"), (b"\x00", b"\x01")):
        spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": a, "s2": b}],
                "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
        want = oracle.run(spec, {"t": t})
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{a}/{b} {mode}")


def test_batch_with_varlen_plan(ctx):
    """An FSST plan and a VARLEN plan of the same comments in one launch."""
    import torch
    from paper_2605_10511_amd import dpf
    G.say("fsst batch beside varlen")
    t = W.wide_table(90_001, seed=2)
    w1, w2, _ = W.wide_words(2)
    dbf = G.make_db(ctx, {"fact": t}, {"fact": _enc()})
    dbv = G.make_db(ctx, {"fact": t}, {"fact": W.WIDE_ENCODINGS})
    specs = [W.wide_query(w1, w2), W.wide_query(w2, w1)]
    plans = [dbf.plan(specs[0]), dbv.plan(specs[0]), dbf.plan(specs[1]), dbv.plan(specs[1])]
    res = dpf.execute(ctx, plans)
    torch.cuda.synchronize()
    for i, p in enumerate(plans):
        G.assert_same(res.get(i), oracle.run(specs[i // 2], {"fact": t}), f"plan {i}")
    res.release()
    for p in plans:
        p.release()


def test_fsst_word_limits(ctx):
    """Words of up to 32 bytes on an FSST column (the longest give the
    largest code table, 131 rows); a longer word, and a second FSST
    predicate in one plan, are refused."""
    from paper_2605_10511_amd import dpf
    t = {"s": to_strings([b"abc"] * 300), "u": to_strings([b"abd"] * 300), "g": np.zeros(300, np.int32)}
    db = G.make_db(ctx, {"t": t}, {"t": {"s": "FSST", "u": "FSST"}})
    base = {"fact": "t", "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
    with pytest.raises(dpf.DpfError):
        db.plan(dict(base, filters=[{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": b"a" * 33, "s2": b"b"}]))
    with pytest.raises(dpf.DpfError):
        db.plan(dict(base, filters=[{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": b"a", "s2": b"b"},
                                    {"col": "u", "op": "STR_CONTAINS_SEQ", "s1": b"a", "s2": b"d"}]))
    spec = dict(base, filters=[{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": b"a", "s2": b"c"}])
    G.assert_same(G.run_gpu(db, spec), oracle.run(spec, {"t": t}), "abc")


@pytest.mark.parametrize("n1,n2", [(17, 5), (24, 24), (32, 32), (31, 1)])
def test_long_words(ctx, n1, n2):
    """Words of 17..32 bytes planted in text of the same alphabet."""
    G.say("fsst long words", n1, n2)
    rng = np.random.default_rng(1300 + n1 * 33 + n2)
    alpha = np.frombuffer(b"abc ", np.uint8)
    s1 = bytes(rng.choice(alpha[:3], n1))
    s2 = bytes(rng.choice(alpha[:3], n2))
    n = 8000
    items = []
    for i in range(n):
        s = bytearray(rng.choice(alpha, int(rng.integers(0, 120))).tobytes())
        r = rng.random()
        if r < 0.3:
            a = int(rng.integers(0, len(s) + 1))
            s[a:a] = s1
            b = int(rng.integers(a + n1, len(s) + 1))
            s[b:b] = s2
        elif r < 0.4:
            s = bytearray(s1[:-1] + s2 + s1)  # s1 only after s2, and a near miss
        items.append(bytes(s))
    t = {"s": to_strings(items), "g": (np.arange(n) % 4).astype(np.int32)}
    db = G.make_db(ctx, {"t": t}, {"t": {"s": "FSST"}}, chunk_rows=1024)
    spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": s1, "s2": s2}],
            "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
    want = oracle.run(spec, {"t": t})
    for mode in ("FUSED", "FRAGMENTED"):
        G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{n1}/{n2} {mode}")


def test_pruned_chunks_and_graph_replay(ctx):
    """FSST plans whose date cutoff prunes most chunks (work items then map
    onto the surviving blocks, each crossing the code-table rebuild at its
    chunk), in one launch beside VARLEN and filter-aggregate plans, eagerly
    and replayed from a HIP graph three times with eager work in between;
    every result against the oracle."""
    import torch
    from paper_2605_10511_amd import dpf
    G.say("fsst pruned chunks, graph replay")
    t = W.wide_table(300_000, seed=2)
    w1, w2, vocab = W.wide_words(2)
    dbf = G.make_db(ctx, {"fact": t}, {"fact": _enc()}, chunk_rows=4096)
    dbv = G.make_db(ctx, {"fact": t}, {"fact": W.WIDE_ENCODINGS}, chunk_rows=4096)
    specs = [W.wide_query(w1, w2, date_lt=300), W.wide_query(vocab[4][:3], vocab[6][:2], date_lt=1200),
             W.wide_query(b"e", b"a", date_lt=2556), W.wide_query(w1, w2, date_lt=300)]
    plans = [dbf.plan(specs[0]), dbf.plan(specs[1]), dbf.plan(specs[2]), dbv.plan(specs[3])]
    assert plans[0].blocks()[0] < plans[0].blocks()[1]  # chunks were pruned
    wants = [oracle.run(sp, {"fact": t}) for sp in specs]
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
        e = dpf.execute(ctx, plans[k:k + 2])
        torch.cuda.synchronize()
        for j in range(2):
            G.assert_same(e.get(j), wants[k + j], f"eager after replay {k}, plan {k + j}")
        e.release()
    r.release()
    del g
    for p in plans:
        p.release()


def test_tiny_records(ctx):
    """Runs of empty and 1-3 byte strings between longer ones, so that a
    lane's four rows hold fewer bytes than one symbol write spans and the
    record decode's spill reaches past the next lane; a three-letter
    alphabet makes the predicate depend on nearly every decoded byte."""
    G.say("fsst tiny records")
    rng = np.random.default_rng(77)
    alpha = np.frombuffer(b"xyz", np.uint8)
    n = 50_000
    lens = rng.choice(np.array([0, 0, 1, 2, 3, 1, 0, 30]), n)
    items = [bytes(rng.choice(alpha, int(k))) for k in lens]
    t = {"s": to_strings(items), "g": (np.arange(n) % 7).astype(np.int32)}
    db = G.make_db(ctx, {"t": t}, {"t": {"s": "FSST"}}, chunk_rows=4096)
    for a, b in ((b"x", b"y"), (b"z", b"z"), (b"xy", b"x"), (b"y", b"xz")):
        spec = {"fact": "t", "filters": [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": a, "s2": b}],
                "probes": [], "group_by": [{"col": "g"}], "aggs": [{"op": "COUNT"}]}
        want = oracle.run(spec, {"t": t})
        for mode in ("FUSED", "FRAGMENTED"):
            G.assert_same(G.run_gpu(db, spec, mode=mode), want, f"{a}/{b} {mode}")
