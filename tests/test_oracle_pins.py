"""Pins for the CPU oracle against things other than itself: hand-computed
results, a brute-force evaluator, closed forms, library routines and
invariants; plus deliberately broken copies of the oracle that must fail at
least one pin.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from datagen import workloads as W
from datagen import vocabulary, comments
from tests import bruteforce as BF
from tests.conftest import to_strings


# --------------------------------------------------------------------------
# P2: hand-computed results
# --------------------------------------------------------------------------
def _run_case(tables, case):
    if "error" in case:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.run(case["query"], tables)
        want = {"duplicate": oracle.ERR_DUPLICATE, "overflow": oracle.ERR_OVERFLOW}[case["error"]]
        assert ei.value.code == want, case["name"]
    else:
        got = oracle.run(case["query"], tables)
        assert got.tolist() == case["expect"], case["name"]


def test_hand_cases(hand_cases):
    tables, cases = hand_cases
    for case in cases:
        _run_case(tables, case)


def test_bruteforce_agrees_with_hand_cases(hand_cases):
    """The brute-force evaluator is itself checked against the hand results."""
    tables, cases = hand_cases
    for case in cases:
        if "error" in case:
            exc = {"duplicate": BF.Duplicate, "overflow": BF.Overflow}[case["error"]]
            with pytest.raises(exc):
                BF.evaluate(case["query"], tables)
        else:
            assert BF.evaluate(case["query"], tables) == case["expect"], case["name"]


# --------------------------------------------------------------------------
# P1: brute force on small random inputs
# --------------------------------------------------------------------------
def _random_instance(rng, n=300):
    alphabet = np.frombuffer(b"ab ", dtype=np.uint8)
    strs = [bytes(alphabet[rng.integers(0, 3, rng.integers(0, 9))]) for _ in range(n)]
    fact = {
        "a": rng.integers(0, 20, n).astype(np.int64),
        "b": rng.integers(-5, 6, n).astype(np.int64),
        "c": rng.integers(0, 4, n).astype(np.int64),
        "fk1": rng.integers(0, 31, n).astype(np.int64),
        "fk2": rng.integers(0, 16, n).astype(np.int64),
        "p": rng.integers(0, 100000, n).astype(np.int64),
        "s": to_strings(strs),
    }
    d1 = {"k": rng.permutation(25).astype(np.int64),
          "x": rng.integers(0, 5, 25).astype(np.int64),
          "y": rng.integers(-3, 4, 25).astype(np.int64)}
    d2 = {"k": rng.permutation(15).astype(np.int64),
          "x": rng.integers(0, 3, 15).astype(np.int64),
          "y": rng.integers(10, 13, 15).astype(np.int64)}
    # D1's rows join D3 through f3 when a query chains the build side
    d1["f3"] = rng.integers(0, 14, 25).astype(np.int64)
    d3 = {"k": rng.permutation(11).astype(np.int64),
          "z": rng.integers(0, 4, 11).astype(np.int64)}
    return {"F": fact, "D1": d1, "D2": d2, "D3": d3}


def _random_pred(rng, cols):
    col = cols[rng.integers(0, len(cols))]
    op = ["LT", "LE", "GT", "GE", "EQ", "NE", "BETWEEN", "IN"][rng.integers(0, 8)]
    v = int(rng.integers(-6, 22))
    if op == "BETWEEN":
        return {"col": col, "op": op, "lo": v, "hi": v + int(rng.integers(0, 10))}
    if op == "IN":
        return {"col": col, "op": op, "values": [int(x) for x in rng.integers(-5, 20, rng.integers(1, 5))]}
    return {"col": col, "op": op, "value": v}


def _random_query(rng):
    words = [b"a", b"b", b"ab", b"ba", b"a b", b"aa", b"b a"]
    filters = [_random_pred(rng, ["a", "b", "c", "p"]) for _ in range(rng.integers(0, 3))]
    if rng.random() < 0.4:
        filters.append({"col": "s", "op": "STR_CONTAINS_SEQ",
                        "s1": words[rng.integers(0, len(words))], "s2": words[rng.integers(0, len(words))]})
    probes = []
    for j, (dim, fk) in enumerate([("D1", "fk1"), ("D2", "fk2")]):
        if rng.random() < 0.6:
            pf = [_random_pred(rng, ["x", "y"]) for _ in range(rng.integers(0, 2))]
            pr = {"fk": fk, "dim": dim, "key": "k", "filters": pf,
                  "payloads": ["x", "y"][:int(rng.integers(0, 3))]}
            if dim == "D1" and rng.random() < 0.4:
                # a joined build side: D1 rows qualify only with a D3 match
                zf = [_random_pred(rng, ["z"]) for _ in range(rng.integers(0, 2))]
                pr["probes"] = [{"fk": "f3", "dim": "D3", "key": "k", "filters": zf, "payloads": ["z"]}]
                if rng.random() < 0.6:
                    pr["payloads"] = pr["payloads"][:1] + [{"probe": 0, "payload": 0}]
            probes.append(pr)
    refs = [{"col": "a"}, {"col": "b"}, {"col": "c"}, {"col": "p"}]
    for j, pr in enumerate(probes):
        refs += [{"probe": j, "payload": k} for k in range(len(pr["payloads"]))]
    keys = [refs[i] for i in rng.choice(len(refs), size=rng.integers(0, 3), replace=False)
            if "col" not in refs[i] or refs[i]["col"] != "p"]
    aggs = []
    for _ in range(rng.integers(1, 4)):
        op = ["COUNT", "SUM", "AVG"][rng.integers(0, 3)]
        if op == "COUNT":
            aggs.append({"op": op})
            continue
        terms = []
        for _ in range(rng.integers(1, 4)):
            if rng.random() < 0.15:
                terms.append({"const": int(rng.integers(-4, 5))})
            else:
                terms.append({"ref": refs[rng.integers(0, len(refs))],
                              "mul": int([1, -1, 2][rng.integers(0, 3)]), "add": int(rng.integers(-3, 4))})
        aggs.append({"op": op, "terms": terms})
    return {"fact": "F", "filters": filters, "probes": probes, "group_by": keys, "aggs": aggs}


def _bf_or_error(spec, tables):
    try:
        return BF.evaluate(spec, tables)
    except BF.Duplicate:
        return "duplicate"
    except BF.Overflow:
        return "overflow"


def _oracle_or_error(spec, tables):
    try:
        return oracle.run(spec, tables).tolist()
    except oracle.OracleError as e:
        return {oracle.ERR_DUPLICATE: "duplicate", oracle.ERR_OVERFLOW: "overflow"}.get(e.code, e.code)


RANDOM_SEEDS = list(range(40))


@pytest.mark.parametrize("seed", RANDOM_SEEDS)
def test_bruteforce_random(seed):
    rng = np.random.default_rng(1000 + seed)
    tables = _random_instance(rng)
    for _ in range(3):
        spec = _random_query(rng)
        assert _oracle_or_error(spec, tables) == _bf_or_error(spec, tables), spec


# --------------------------------------------------------------------------
# P3: closed forms at full scale (10^6 rows)
# --------------------------------------------------------------------------
def test_closed_form_filter_aggregate():
    """Structured columns qty = 1 + i mod 50, disc = i mod 11,
    date = floor(i * 2556 / n), price = 90000 + i mod 1000, flag = i mod 3.
    For date < 2400 AND disc in [5, 7] AND qty < 24 grouped by flag, the rows
    are i < N with N = ceil(2400 n / 2556); residues mod 11, mod 1000 (which
    fixes i mod 50) and mod 3 are independent over a period of 33000, so
    per period and flag: count = 3 * 460, sum(qty) = 3 * 20 * sum_{b<23}(1+b),
    sum(price) = 3 * S, sum(price * (100 - disc)) = (95 + 94 + 93) * S with
    S = 460 * 90000 + sum of the 460 valid residues mod 1000."""
    n = 1_000_000
    i = np.arange(n, dtype=np.int64)
    table = {"date": (i * 2556) // n, "quantity": 1 + i % 50, "price": 90000 + i % 1000,
             "discount": i % 11, "flag": i % 3}
    spec = {"fact": "t",
            "filters": [{"col": "date", "op": "LT", "value": 2400},
                        {"col": "discount", "op": "BETWEEN", "lo": 5, "hi": 7},
                        {"col": "quantity", "op": "LT", "value": 24}],
            "probes": [], "group_by": [{"col": "flag"}],
            "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "quantity"}}]},
                     {"op": "SUM", "terms": [{"ref": {"col": "price"}}]},
                     {"op": "SUM", "terms": [{"ref": {"col": "price"}},
                                             {"ref": {"col": "discount"}, "mul": -1, "add": 100}]}]}
    got = oracle.run(spec, {"t": table})

    N = -(-2400 * n // 2556)
    period = 33000
    valid_r1000 = [r for r in range(1000) if r % 50 <= 22]
    assert len(valid_r1000) == 460
    S = 460 * 90000 + (23 * 50 * sum(range(20)) + 20 * sum(range(23)))
    per = {"count": 3 * 460, "qty": 3 * 20 * sum(1 + b for b in range(23)), "price": 3 * S,
           "disc": (95 + 94 + 93) * S}
    full = N // period
    expect = {f: [full * per["count"], full * per["qty"], full * per["price"], full * per["disc"]]
              for f in range(3)}
    # The partial period [full * period, N): every residue class appears at
    # most once, counted directly.
    for k in range(full * period, N):
        if k % 11 in (5, 6, 7) and k % 50 <= 22:
            e = expect[k % 3]
            e[0] += 1
            e[1] += 1 + k % 50
            e[2] += 90000 + k % 1000
            e[3] += (90000 + k % 1000) * (100 - k % 11)
    want = [[f] + expect[f] for f in range(3)]
    assert got.tolist() == want


def test_closed_form_no_filter_sum():
    """No predicate: count = n and sum(x) = n (n - 1) / 2 for x = i."""
    n = 777_777
    t = {"x": np.arange(n, dtype=np.int64)}
    spec = {"fact": "t", "filters": [], "probes": [], "group_by": [],
            "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "x"}}]},
                     {"op": "SUM", "terms": [{"ref": {"col": "x"}, "mul": -1, "add": n - 1}]}]}
    got = oracle.run(spec, {"t": t}).tolist()
    assert got == [[n, n * (n - 1) // 2, n * (n - 1) // 2]]


# --------------------------------------------------------------------------
# P4: library routines
# --------------------------------------------------------------------------
def test_string_predicate_vs_bytes_find():
    """contains-in-order == (p = s.find(w1)) >= 0 and s.find(w2, p + len(w1)) >= 0,
    over generated comments and word pairs taken from the vocabulary and from
    substrings of the comments themselves."""
    vocab = vocabulary(7, 200, 2, 5)
    strs = comments(7, "c", 4000, vocab, 0, 40, plant=vocab[3] + b" " + vocab[4], plant_pct=5)
    rng = np.random.default_rng(5)
    pairs = [(vocab[3], vocab[4]), (vocab[4], vocab[3]), (b"a", b"a"), (b" ", b" ")]
    for _ in range(12):
        s = strs.get(int(rng.integers(0, len(strs))))
        if len(s) >= 4:
            a = int(rng.integers(0, len(s) - 2))
            pairs.append((s[a:a + 2], vocab[int(rng.integers(0, len(vocab)))][:2]))
    for w1, w2 in pairs:
        want = 0
        for i in range(len(strs)):
            s = strs.get(i)
            p = s.find(w1)
            want += p >= 0 and s.find(w2, p + len(w1)) >= 0
        got = oracle.count_filter({"s": strs}, [{"col": "s", "op": "STR_CONTAINS_SEQ", "s1": w1, "s2": w2}])
        assert got == want, (w1, w2)


def test_star_join_vs_sort_merge():
    """The star-join query against an independent join: dimension keys sorted
    and located with numpy.searchsorted, groups by numpy.unique, sums by
    numpy.add.at."""
    dims = W.sj_dims(seed=11, scale=0.002)
    fact = W.sj_fact(200_000, seed=11, dims=dims)
    spec = W.sj_query(part_attr=3, supp_nation=2, date_dow=None, cust_region=1, part_category=4)
    tables = {"lo": fact, **dims}
    got = oracle.run(spec, tables)

    keep = np.ones(len(fact["lo_revenue"]), dtype=bool)
    pays = {}
    for j, pr in enumerate(spec["probes"]):
        d = dims[pr["dim"]]
        m = np.ones(len(d[pr["key"]]), dtype=bool)
        for p in pr["filters"]:
            m &= d[p["col"]] == p["value"]
        keys = d[pr["key"]][m]
        order = np.argsort(keys, kind="stable")
        sk = keys[order]
        fk = fact[pr["fk"]]
        pos = np.clip(np.searchsorted(sk, fk), 0, max(len(sk) - 1, 0))
        hit = (len(sk) > 0) & (sk[pos] == fk) if len(sk) else np.zeros(len(fk), bool)
        keep &= hit
        pays[j] = [d[c][m][order][pos] for c in pr["payloads"]]
    year = pays[2][0][keep].astype(np.int64)
    brand = pays[0][0][keep].astype(np.int64)
    rev = fact["lo_revenue"][keep].astype(np.int64)
    gk = year * 1000 + brand
    uk, inv = np.unique(gk, return_inverse=True)
    sums = np.zeros(len(uk), dtype=np.int64)
    cnts = np.zeros(len(uk), dtype=np.int64)
    np.add.at(sums, inv, rev)
    np.add.at(cnts, inv, 1)
    want = [[int(k // 1000), int(k % 1000), int(s), int(c)] for k, s, c in zip(uk, sums, cnts)]
    assert len(want) > 20
    assert got.tolist() == want


def test_filter_count_vs_numpy():
    t = W.fa_table(300_000, seed=9)
    preds = W.fa_query()["filters"]
    want = int(np.count_nonzero((t["date"] < 2400) & (t["discount"] >= 5) & (t["discount"] <= 7)
                                & (t["quantity"] < 24)))
    assert oracle.count_filter(t, preds) == want


# --------------------------------------------------------------------------
# P5: invariants
# --------------------------------------------------------------------------
def test_invariants_filter_aggregate():
    t = W.fa_table(500_000, seed=12)
    spec = W.fa_query()
    got = oracle.run(spec, {"fact": t})
    assert (got[:, 2] >= 1).all()
    assert int(got[:, 2].sum()) == oracle.count_filter(t, spec["filters"])
    # no predicate: counts add up to n and sums to the column totals
    spec2 = dict(spec, filters=[])
    got2 = oracle.run(spec2, {"fact": t})
    assert int(got2[:, 2].sum()) == len(t["date"])
    assert int(got2[:, 3].sum()) == int(t["quantity"].astype(np.int64).sum())
    assert int(got2[:, 4].sum()) == int(t["price"].sum())
    assert got2.shape[0] == 6


# --------------------------------------------------------------------------
# Broken copies of the oracle must fail the pins
# --------------------------------------------------------------------------
MUTANTS = [
    ("case ORC_LT: return x < p->a;", "case ORC_LT: return x <= p->a;"),
    ("case ORC_GE: return x >= p->a;", "case ORC_GE: return x > p->a;"),
    ("case ORC_BETWEEN: return x >= p->a && x <= p->b;", "case ORC_BETWEEN: return x >= p->a && x < p->b;"),
    ("const uint8_t* rest = p + n1;", "const uint8_t* rest = p + 1;"),
    ("__builtin_mul_overflow(tm->mul, x, &mx)", "__builtin_mul_overflow((int64_t)1, x, &mx)"),
    ("__builtin_add_overflow(mx, tm->add, &v)", "__builtin_add_overflow(mx, (int64_t)0, &v)"),
    ("if (kind == ORC_AGG_AVG) o[c++] = acc[0];", "if (kind == ORC_AGG_AVG) o[c++] = acc[1];"),
    ("if (e[i].key == e[i - 1].key) {", "if (0) {"),
    ("if (a[i] < b[i]) return -1;", "if (a[i] < b[i]) return 1;"),
    ("cols[pr->pay_col[k]].ival[r] : 0;", "cols[pr->pay_col[0]].ival[r] : 0;"),
    ("if (!rc && __builtin_mul_overflow(prod, v, &prod)) rc = ORC_ERR_OVERFLOW;", "if (!rc) prod *= v;"),
    # joined build sides
    ("hit[j] = probe_dim(&sub[j], cols[pr->sub[j].fact_fk_col].ival[r]);",
     "hit[j] = probe_dim(&sub[j], cols[pr->sub[j].fact_fk_col].ival[r]); if (!hit[j]) hit[j] = sub[j].e;"),
    ("e[n].pay[k] = hit[pr->pay_src[k]]->pay[pr->pay_col[k]];", "e[n].pay[k] = cols[pr->pay_col[k]].ival[r];"),
    ("for (int32_t i = 0; i < pr->npreds && ok; ++i) ok = eval_pred(&pr->preds[i], cols, r);",
     "for (int32_t i = 0; i < pr->npreds && ok && depth == 0; ++i) ok = eval_pred(&pr->preds[i], cols, r);"),
]


@pytest.mark.parametrize("idx", range(len(MUTANTS)))
def test_broken_oracle_fails_a_pin(idx, hand_cases, tmp_path):
    old, new = MUTANTS[idx]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert src.count(old) == 1, old
    d = tmp_path / "mut"
    d.mkdir()
    (d / "oracle.c").write_text(src.replace(old, new))
    shutil.copy(os.path.join(os.path.dirname(oracle.__file__), "oracle.h"), d / "oracle.h")
    so = str(d / "liboracle_mut.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", so, str(d / "oracle.c")])
    tables, cases = hand_cases
    failed = False
    oracle.use_library(so)
    try:
        for case in cases:
            try:
                _run_case(tables, case)
            except (AssertionError, oracle.OracleError, pytest.fail.Exception):
                failed = True
                break
        if not failed:
            for seed in RANDOM_SEEDS[:10]:
                rng = np.random.default_rng(1000 + seed)
                t = _random_instance(rng)
                for _ in range(3):
                    spec = _random_query(rng)
                    if _oracle_or_error(spec, t) != _bf_or_error(spec, t):
                        failed = True
                        break
                if failed:
                    break
    finally:
        oracle.use_library(None)
    assert failed, f"mutant {idx} passed every pin: {new}"


# --------------------------------------------------------------------------
# The timing-only threaded oracle returns the single-thread records
# --------------------------------------------------------------------------
@pytest.mark.parametrize("threads", [2, 3, 8, 64])
def test_threaded_oracle_equals_single_thread(threads):
    t = W.fa_table(400_003, seed=31)
    for spec in (W.fa_query(), dict(W.fa_query(), filters=[])):
        assert np.array_equal(oracle.run(spec, {"fact": t}, threads=threads), oracle.run(spec, {"fact": t}))
    wide = W.wide_table(60_000, seed=2)
    w1, w2, _ = W.wide_words(2)
    spec = W.wide_query(w1, w2)
    assert np.array_equal(oracle.run(spec, {"fact": wide}, threads=threads), oracle.run(spec, {"fact": wide}))
    dims = W.sj_dims(seed=3, scale=0.01)
    fact = W.sj_fact(200_000, seed=3, dims=dims)
    tables = {"lo": fact, **dims}
    spec = W.sj_query(part_category=4, date_dow=None)
    assert np.array_equal(oracle.run(spec, tables, threads=threads), oracle.run(spec, tables))
    rng = np.random.default_rng(77 + threads)
    for _ in range(6):
        inst = _random_instance(rng, n=int(rng.integers(0, 50)))  # also fewer rows than threads
        spec = _random_query(rng)
        try:
            want = oracle.run(spec, inst)
        except oracle.OracleError as e:
            with pytest.raises(oracle.OracleError) as e2:
                oracle.run(spec, inst, threads=threads)
            assert e2.value.code == e.code
            continue
        assert np.array_equal(oracle.run(spec, inst, threads=threads), want)
