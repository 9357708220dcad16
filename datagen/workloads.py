"""Synthetic star-schema tables and query descriptions.

The paper evaluates on TPC-H and SSB at scale factor 100 (Section 5.1); those
datasets and their query texts are not used here.  Seeded synthetic tables of
the same shape stand in for them: a date-clustered fact table with
low-cardinality flags, quantities, discounts and scaled-integer prices
(filter-aggregate), a wide variant with a variable-length comment string, and
a fact table with four foreign keys into date/customer/supplier/part
dimensions (star join).  Values are drawn by :mod:`datagen`.

Query description format (plain data; the oracle and the library binding each
translate it on their own)::

    {"fact": table,
     "filters": [pred, ...],                  # conjunction over fact columns
     "probes": [{"fk": col, "dim": table, "key": col,
                 "filters": [pred, ...], "payloads": [col, ...]}, ...],
     "group_by": [ref, ...],
     "aggs": [agg, ...]}

    pred = {"col": c, "op": "LT"|"LE"|"GT"|"GE"|"EQ"|"NE", "value": v}
         | {"col": c, "op": "BETWEEN", "lo": a, "hi": b}          # inclusive
         | {"col": c, "op": "IN", "values": [v, ...]}
         | {"col": c, "op": "STR_CONTAINS_SEQ", "s1": b"..", "s2": b".."}
    ref  = {"col": c} | {"probe": j, "payload": k}
    term = {"ref": ref, "mul": m, "add": a}   # value m * x + a (mul 1, add 0 default)
         | {"const": c}
    agg  = {"op": "COUNT"} | {"op": "SUM", "terms": [term, ...]}
         | {"op": "AVG", "terms": [term, ...]}   # reported as (sum, count)

Result: one int64 record per non-empty group, the group key values first,
then COUNT -> count, SUM -> sum, AVG -> sum, count; ascending by group key.
"""
from __future__ import annotations

import math

import numpy as np

from . import Strings, comments, sorted_uniform, uniform, vocabulary, raw

FLAG_A_VALUES = (ord("X"), ord("Y"), ord("Z"))
FLAG_B_VALUES = (ord("P"), ord("Q"))
NDATES = 2556

# Encoding each column is given to the library (the oracle ignores this).
FA_ENCODINGS = {"date": "DELTA", "quantity": "FOR", "price": "FOR", "discount": "FOR",
                "flagA": "DICT", "flagB": "DICT"}


def _pick(values, idx):
    return np.asarray(values, dtype=np.int32)[idx]


# ----------------------------------------------------------------------------
# Filter-aggregate schema (6 columns)
# ----------------------------------------------------------------------------
def fa_table(n: int = 1_000_000, seed: int = 1) -> dict:
    """Date-clustered fact table: date sorted uniform in [0, 2556), quantity
    1..50, price 90000..10500000 (int64 cents), discount 0..10, flagA one of 3
    values and flagB one of 2, independent and uniform."""
    return {
        "date": sorted_uniform(seed, "date", n, 0, NDATES - 1, dtype=np.int32),
        "quantity": uniform(seed, "quantity", n, 1, 50, dtype=np.int32),
        "price": uniform(seed, "price", n, 90000, 10500000, dtype=np.int64),
        "discount": uniform(seed, "discount", n, 0, 10, dtype=np.int32),
        "flagA": _pick(FLAG_A_VALUES, uniform(seed, "flagA", n, 0, 2, dtype=np.int32)),
        "flagB": _pick(FLAG_B_VALUES, uniform(seed, "flagB", n, 0, 1, dtype=np.int32)),
    }


def fa_query(table: str = "fact", date_lt: int = 2400, disc_lo: int = 5, disc_hi: int = 7,
             qty_lt: int = 24) -> dict:
    """date < date_lt AND discount BETWEEN disc_lo AND disc_hi AND
    quantity < qty_lt, grouped by (flagA, flagB): count, sum(quantity),
    sum(price), sum(price * (100 - discount))."""
    return {
        "fact": table,
        "filters": [
            {"col": "date", "op": "LT", "value": date_lt},
            {"col": "discount", "op": "BETWEEN", "lo": disc_lo, "hi": disc_hi},
            {"col": "quantity", "op": "LT", "value": qty_lt},
        ],
        "probes": [],
        "group_by": [{"col": "flagA"}, {"col": "flagB"}],
        "aggs": [
            {"op": "COUNT"},
            {"op": "SUM", "terms": [{"ref": {"col": "quantity"}}]},
            {"op": "SUM", "terms": [{"ref": {"col": "price"}}]},
            {"op": "SUM", "terms": [{"ref": {"col": "price"}},
                                    {"ref": {"col": "discount"}, "mul": -1, "add": 100}]},
        ],
    }


# ----------------------------------------------------------------------------
# Wide filter-aggregate schema with a comment string (16 columns)
# ----------------------------------------------------------------------------
WIDE_FLAGB_CUTOFF = 1278

WIDE_ENCODINGS = {"k1": "DELTA", "date": "DELTA", "flagA": "DICT", "flagB": "DICT",
                  "comment": "VARLEN"}


def wide_words(seed: int = 2) -> tuple[bytes, bytes, list[bytes]]:
    """The 2,000-word vocabulary and the two words of the string predicate."""
    vocab = vocabulary(seed, 2000, 3, 10)
    return vocab[0], vocab[1], vocab


def wide_table(n: int = 60_000_000, seed: int = 2, plant_pct: int = 1) -> dict:
    """16 columns: k1 = row // 4 (sorted), k2..k8 uniform int32 keys and
    measures, d1..d4 uniform int64 decimals (cents), a sorted date, flags
    correlated with the date (flagB = date >= cutoff; flagA uniform over 3
    values when flagB is the first value, fixed otherwise) and a comment of
    10..43 bytes built from the vocabulary; plant_pct percent of comments start
    with "w1 w2 "."""
    w1, w2, vocab = wide_words(seed)
    date = sorted_uniform(seed, "date", n, 0, NDATES - 1, dtype=np.int32)
    late = date >= WIDE_FLAGB_CUTOFF
    fa = _pick(FLAG_A_VALUES, uniform(seed, "flagA", n, 0, 2, dtype=np.int32))
    fa = np.where(late, np.int32(FLAG_A_VALUES[1]), fa).astype(np.int32)
    fb = np.where(late, np.int32(FLAG_B_VALUES[1]), np.int32(FLAG_B_VALUES[0])).astype(np.int32)
    return {
        "k1": (np.arange(n, dtype=np.int64) // 4).astype(np.int32),
        "k2": uniform(seed, "k2", n, 1, 3_000_000, dtype=np.int32),
        "k3": uniform(seed, "k3", n, 1, 200_000, dtype=np.int32),
        "k4": uniform(seed, "k4", n, 1, 1_400_000, dtype=np.int32),
        "k5": uniform(seed, "k5", n, 1, 50, dtype=np.int32),
        "k6": uniform(seed, "k6", n, 0, 10, dtype=np.int32),
        "k7": uniform(seed, "k7", n, 0, 8, dtype=np.int32),
        "k8": uniform(seed, "k8", n, 1, 7, dtype=np.int32),
        "d1": uniform(seed, "d1", n, 90000, 10500000, dtype=np.int64),
        "d2": uniform(seed, "d2", n, 100, 100000, dtype=np.int64),
        "d3": uniform(seed, "d3", n, 0, 10_000_000, dtype=np.int64),
        "d4": uniform(seed, "d4", n, 0, 1_000_000, dtype=np.int64),
        "flagA": fa,
        "flagB": fb,
        "date": date,
        "comment": comments(seed, "comment", n, vocab, 10, 43,
                            plant=w1 + b" " + w2 + b" ", plant_pct=plant_pct),
    }


def wide_query(w1: bytes, w2: bytes, table: str = "fact", date_lt: int = 2505) -> dict:
    """date < date_lt AND comment contains w1 then w2, grouped by (flagA,
    flagB): sum(k5), sum(d1), sum(d1*(100-k6)), sum(d1*(100-k6)*(100+k7)),
    avg(k5), avg(d1), avg(k6) (each as sum and count) and count."""
    d1 = {"ref": {"col": "d1"}}
    disc = {"ref": {"col": "k6"}, "mul": -1, "add": 100}
    tax = {"ref": {"col": "k7"}, "add": 100}
    return {
        "fact": table,
        "filters": [
            {"col": "date", "op": "LT", "value": date_lt},
            {"col": "comment", "op": "STR_CONTAINS_SEQ", "s1": w1, "s2": w2},
        ],
        "probes": [],
        "group_by": [{"col": "flagA"}, {"col": "flagB"}],
        "aggs": [
            {"op": "SUM", "terms": [{"ref": {"col": "k5"}}]},
            {"op": "SUM", "terms": [d1]},
            {"op": "SUM", "terms": [d1, disc]},
            {"op": "SUM", "terms": [d1, disc, tax]},
            {"op": "AVG", "terms": [{"ref": {"col": "k5"}}]},
            {"op": "AVG", "terms": [d1]},
            {"op": "AVG", "terms": [{"ref": {"col": "k6"}}]},
            {"op": "COUNT"},
        ],
    }


# ----------------------------------------------------------------------------
# Star-join schema: fact with 4 foreign keys, 4 dimensions
# ----------------------------------------------------------------------------
SJ_DIM_ROWS = {"date": NDATES, "customer": 3_000_000, "supplier": 200_000, "part": 1_400_000}
SJ_ENCODINGS = {}


def sj_dims(seed: int = 3, scale: float = 1.0) -> dict:
    """Dimension tables keyed densely (date 0..2555, others 1..N): date(year =
    7*key // 2556, dow = key mod 7), customer(region 0..4), supplier(nation
    0..24), part(attr 0..999, category 0..24, brand 0..39).  ``scale`` shrinks
    customer/supplier/part for small tests."""
    nc = max(1, int(SJ_DIM_ROWS["customer"] * scale))
    ns = max(1, int(SJ_DIM_ROWS["supplier"] * scale))
    npart = max(1, int(SJ_DIM_ROWS["part"] * scale))
    dk = np.arange(NDATES, dtype=np.int32)
    return {
        "date": {"d_datekey": dk, "d_year": (7 * dk // NDATES).astype(np.int32),
                 "d_dow": (dk % 7).astype(np.int32)},
        "customer": {"c_custkey": np.arange(1, nc + 1, dtype=np.int32),
                     "c_region": uniform(seed, "c_region", nc, 0, 4, dtype=np.int32)},
        "supplier": {"s_suppkey": np.arange(1, ns + 1, dtype=np.int32),
                     "s_nation": uniform(seed, "s_nation", ns, 0, 24, dtype=np.int32)},
        "part": {"p_partkey": np.arange(1, npart + 1, dtype=np.int32),
                 "p_attr": uniform(seed, "p_attr", npart, 0, 999, dtype=np.int32),
                 "p_category": uniform(seed, "p_category", npart, 0, 24, dtype=np.int32),
                 "p_brand": uniform(seed, "p_brand", npart, 0, 39, dtype=np.int32)},
    }


def sj_fact(n: int = 120_000_000, seed: int = 3, dims: dict | None = None, name: str = "lo") -> dict:
    """Fact rows with uniform foreign keys into the dimensions and a revenue
    uniform in 90000..10500000 (int64 cents)."""
    nc = len(dims["customer"]["c_custkey"]) if dims else SJ_DIM_ROWS["customer"]
    ns = len(dims["supplier"]["s_suppkey"]) if dims else SJ_DIM_ROWS["supplier"]
    npart = len(dims["part"]["p_partkey"]) if dims else SJ_DIM_ROWS["part"]
    return {
        "lo_datekey": uniform(seed, name + "_datekey", n, 0, NDATES - 1, dtype=np.int32),
        "lo_custkey": uniform(seed, name + "_custkey", n, 1, nc, dtype=np.int32),
        "lo_suppkey": uniform(seed, name + "_suppkey", n, 1, ns, dtype=np.int32),
        "lo_partkey": uniform(seed, name + "_partkey", n, 1, npart, dtype=np.int32),
        "lo_revenue": uniform(seed, name + "_revenue", n, 90000, 10500000, dtype=np.int64),
    }


def sj_query(table: str = "lo", part_attr: int = 17, supp_nation: int = 3, date_dow: int | None = 2,
             cust_region: int = 1, part_category: int | None = None) -> dict:
    """Probe part (attr = c, or category = c), supplier (nation = c), date
    (dow = c, or unfiltered) and customer (region = c) in that order; group by
    (date.year, part.brand); sum(revenue) and count."""
    pf = ([{"col": "p_category", "op": "EQ", "value": part_category}] if part_category is not None
          else [{"col": "p_attr", "op": "EQ", "value": part_attr}])
    df = [] if date_dow is None else [{"col": "d_dow", "op": "EQ", "value": date_dow}]
    return {
        "fact": table,
        "filters": [],
        "probes": [
            {"fk": "lo_partkey", "dim": "part", "key": "p_partkey", "filters": pf,
             "payloads": ["p_brand"]},
            {"fk": "lo_suppkey", "dim": "supplier", "key": "s_suppkey",
             "filters": [{"col": "s_nation", "op": "EQ", "value": supp_nation}], "payloads": []},
            {"fk": "lo_datekey", "dim": "date", "key": "d_datekey", "filters": df,
             "payloads": ["d_year"]},
            {"fk": "lo_custkey", "dim": "customer", "key": "c_custkey",
             "filters": [{"col": "c_region", "op": "EQ", "value": cust_region}], "payloads": []},
        ],
        "group_by": [{"probe": 2, "payload": 0}, {"probe": 0, "payload": 0}],
        "aggs": [{"op": "SUM", "terms": [{"ref": {"col": "lo_revenue"}}]}, {"op": "COUNT"}],
    }


# ----------------------------------------------------------------------------
# Join chain: a 3-table pipeline (customer -> orders -> lineitem)
# ----------------------------------------------------------------------------
def chain_tables(n_line: int = 120_000_000, seed: int = 6, n_orders: int | None = None,
                 n_cust: int | None = None) -> dict:
    """customer(custkey 1..C, region 0..4, segment 0..9); orders(orderkey
    1..O, custkey uniform, priority 1..5, odate in [0, 2556)); lineitem
    (orderkey uniform, quantity 1..50, extprice 90000..10500000 cents).  By
    default O = n_line / 4 and C = O / 10 (the order-to-line and
    customer-to-order ratios of a star schema's snowflake arm)."""
    n_orders = n_orders or max(1, n_line // 4)
    n_cust = n_cust or max(1, n_orders // 10)
    return {
        "customer": {"c_custkey": np.arange(1, n_cust + 1, dtype=np.int32),
                     "c_region": uniform(seed, "c_region", n_cust, 0, 4, dtype=np.int32),
                     "c_segment": uniform(seed, "c_segment", n_cust, 0, 9, dtype=np.int32)},
        "orders": {"o_orderkey": np.arange(1, n_orders + 1, dtype=np.int32),
                   "o_custkey": uniform(seed, "o_custkey", n_orders, 1, n_cust, dtype=np.int32),
                   "o_priority": uniform(seed, "o_priority", n_orders, 1, 5, dtype=np.int32),
                   "o_date": uniform(seed, "o_date", n_orders, 0, NDATES - 1, dtype=np.int32)},
        "lineitem": {"l_orderkey": uniform(seed, "l_orderkey", n_line, 1, n_orders, dtype=np.int32),
                     "l_quantity": uniform(seed, "l_quantity", n_line, 1, 50, dtype=np.int32),
                     "l_extprice": uniform(seed, "l_extprice", n_line, 90000, 10500000, dtype=np.int64)},
    }


def chain_query(segment: int = 3, date_lo: int = 700, date_hi: int = 1600, qty_lt: int = 30) -> dict:
    """Section 3.1's running example in shape: customers of one market
    segment build table #1; orders in a date window probe it and build table
    #2 keyed by order, carrying the customer's region and the order
    priority; line items (quantity below a cutoff) probe table #2 and
    aggregate count, sum(quantity) and sum(extprice * priority) by (region,
    priority)."""
    return {
        "fact": "lineitem",
        "filters": [{"col": "l_quantity", "op": "LT", "value": qty_lt}],
        "probes": [{"fk": "l_orderkey", "dim": "orders", "key": "o_orderkey",
                    "filters": [{"col": "o_date", "op": "BETWEEN", "lo": date_lo, "hi": date_hi}],
                    "payloads": [{"probe": 0, "payload": 0}, "o_priority"],
                    "probes": [{"fk": "o_custkey", "dim": "customer", "key": "c_custkey",
                                "filters": [{"col": "c_segment", "op": "EQ", "value": segment}],
                                "payloads": ["c_region"]}]}],
        "group_by": [{"probe": 0, "payload": 0}, {"probe": 0, "payload": 1}],
        "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "l_quantity"}}]},
                 {"op": "SUM", "terms": [{"ref": {"col": "l_extprice"}}, {"ref": {"probe": 0, "payload": 1}}]}],
    }


# ----------------------------------------------------------------------------
# Batched mix: 64 queries over a pool of tables of log-uniform size
# ----------------------------------------------------------------------------
def mix_plan(seed: int = 4, nq: int = 64, min_rows: int = 1_000_000, max_rows: int = 120_000_000,
             pool: int = 4) -> dict:
    """Describe a query mix: a pool of ``pool`` filter-aggregate tables and
    ``pool`` star-join fact tables with sizes log-uniform in [min_rows,
    max_rows]; each of ``nq`` queries picks a template (50/50), a table of
    that template from the pool and its predicate constants uniformly."""
    u = raw(seed, "mix", 16 * (nq + 2 * pool)).astype(np.float64) / 2.0**64
    k = 0

    def nxt():
        nonlocal k
        k += 1
        return float(u[k - 1])

    lo, hi = math.log(min_rows), math.log(max_rows)
    fa_sizes = [int(math.exp(lo + (hi - lo) * nxt())) for _ in range(pool)]
    sj_sizes = [int(math.exp(lo + (hi - lo) * nxt())) for _ in range(pool)]
    queries = []
    for q in range(nq):
        if nxt() < 0.5:
            t = min(int(nxt() * pool), pool - 1)
            c = min(int(nxt() * 9), 8)
            queries.append(("FA", t, fa_query(f"fa{t}", date_lt=min(int(nxt() * NDATES), NDATES - 1),
                                              disc_lo=c, disc_hi=c + 2,
                                              qty_lt=2 + min(int(nxt() * 50), 49))))
        else:
            t = min(int(nxt() * pool), pool - 1)
            queries.append(("SJ", t, sj_query(f"sj{t}", part_attr=min(int(nxt() * 1000), 999),
                                              supp_nation=min(int(nxt() * 25), 24),
                                              date_dow=min(int(nxt() * 7), 6),
                                              cust_region=min(int(nxt() * 5), 4))))
    return {"fa_sizes": fa_sizes, "sj_sizes": sj_sizes, "queries": queries}


# ----------------------------------------------------------------------------
# Serving: a union-schema fact table and Poisson request streams
# ----------------------------------------------------------------------------
def union_table(n: int, seed: int = 5, dims: dict | None = None) -> dict:
    """The filter-aggregate columns and the star-join foreign keys and revenue
    in one fact table of n rows (both query templates run on it)."""
    t = fa_table(n, seed=seed)
    t.update(sj_fact(n, seed=seed, dims=dims, name="u"))
    return t


def serve_requests(seed: int, qps: float, seconds: float, table: str, stream: str = "req") -> list:
    """Poisson arrivals at ``qps`` for ``seconds``: [(arrival_s, template,
    spec)], exponential gaps and template constants from one seeded stream
    (template FA or SJ with probability 1/2, constants uniform over each
    attribute's domain)."""
    n = max(16, int(qps * seconds * 1.5) + 64)
    u = (raw(seed, f"{stream}@{qps:g}", 8 * n).astype(np.float64) + 0.5) / 2.0**64
    k = 0

    def nxt():
        nonlocal k
        k += 1
        return float(u[k - 1])

    out = []
    t = 0.0
    while True:
        t += -math.log(nxt()) / qps
        if t >= seconds:
            break
        if nxt() < 0.5:
            c = min(int(nxt() * 9), 8)
            spec = fa_query(table, date_lt=min(int(nxt() * NDATES), NDATES - 1), disc_lo=c, disc_hi=c + 2,
                            qty_lt=2 + min(int(nxt() * 50), 49))
            out.append((t, "FA", spec))
        else:
            spec = sj_query(table, part_attr=min(int(nxt() * 1000), 999), supp_nation=min(int(nxt() * 25), 24),
                            date_dow=min(int(nxt() * 7), 6), cust_region=min(int(nxt() * 5), 4))
            out.append((t, "SJ", spec))
        if k + 8 > len(u):
            break
    return out


__all__ = ["Strings", "chain_tables", "chain_query", "union_table", "serve_requests", "fa_table", "fa_query", "wide_table", "wide_query", "wide_words",
           "sj_dims", "sj_fact", "sj_query", "mix_plan", "FA_ENCODINGS", "WIDE_ENCODINGS",
           "FLAG_A_VALUES", "FLAG_B_VALUES", "NDATES"]
