"""GPU: the allocation-free fused execution (dpf_execute_noalloc, its scratch
state in the library's static device array) returns exactly what
dpf_execute returns, through the C ABI, on two calls in a row -- the second
over a smaller input -- and refuses a batch whose scratch would not fit."""
import numpy as np
import pytest

import oracle
from datagen import workloads as W
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2605_10511_amd import dpf
    assert torch.cuda.is_available()
    return dpf.Context(0)


def _both(ctx, plans):
    """(rows of dpf_execute, rows of dpf_execute_noalloc) for every plan."""
    import torch
    from paper_2605_10511_amd import dpf
    r = dpf.execute(ctx, plans)
    torch.cuda.synchronize()
    want = [r.get(i) for i in range(len(plans))]
    r.release()
    r = dpf.execute_noalloc(ctx, plans)
    torch.cuda.synchronize()
    got = [r.get(i) for i in range(len(plans))]
    r.release()
    return want, got


def test_noalloc_equals_execute_twice(ctx):
    # first call: a filter-aggregate, the wide query with strings, a star
    # join and a plan whose group table is too large for LDS, in one launch
    fa = W.fa_table(300_000, seed=81)
    wide = W.wide_table(150_000, seed=2)
    dims = W.sj_dims(seed=3, scale=0.01)
    lo = W.sj_fact(400_000, seed=82, dims=dims)
    tables = {"fa": fa, "wide": wide, "lo": lo, **dims}
    db = G.make_db(ctx, tables, {"fa": W.FA_ENCODINGS, "wide": W.WIDE_ENCODINGS}, chunk_rows=16384)
    w1, w2, _ = W.wide_words(2)
    specs = [W.fa_query("fa"), W.wide_query(w1, w2, table="wide"), W.sj_query(part_category=4, date_dow=None),
             {"fact": "lo", "filters": [{"col": "lo_revenue", "op": "LT", "value": 3_000_000}], "probes": [],
              "group_by": [{"col": "lo_suppkey"}], "aggs": [{"op": "COUNT"},
                                                              {"op": "SUM", "terms": [{"ref": {"col": "lo_revenue"}}]}]}]
    plans = [db.plan(s) for s in specs]
    G.say("noalloc: first call, 4 plans")
    want, got = _both(ctx, plans)
    for i, s in enumerate(specs):
        G.assert_same(got[i], want[i], f"first call plan {i}")
        G.assert_same(got[i], oracle.run(s, tables), f"first call plan {i} vs oracle")
    # second call: a smaller input (fewer rows, one plan, a smaller group table)
    small = W.fa_table(5_003, seed=83)
    db2 = G.make_db(ctx, {"fact": small}, {"fact": W.FA_ENCODINGS}, chunk_rows=2048)
    spec2 = W.fa_query(date_lt=1800, disc_lo=1, disc_hi=9, qty_lt=45)
    p2 = db2.plan(spec2)
    G.say("noalloc: second call, smaller input")
    want2, got2 = _both(ctx, [p2])
    G.assert_same(got2[0], want2[0], "second call")
    G.assert_same(got2[0], oracle.run(spec2, {"fact": small}), "second call vs oracle")
    # and the first batch once more: nothing left over from the smaller call
    want3, got3 = _both(ctx, plans)
    for i in range(len(specs)):
        G.assert_same(got3[i], want[i], f"third call plan {i}")
    for p in plans + [p2]:
        p.release()
        for h in p.hashes:
            h.release()


def test_noalloc_refuses_oversized_scratch(ctx):
    from paper_2605_10511_amd import dpf
    n = 70_000
    t = {"a": np.arange(n, dtype=np.int32) * 7, "v": np.ones(n, dtype=np.int64)}
    db = G.make_db(ctx, {"t": t})
    # 490,000 key values x 3 accumulators x 8 B = 11.8 MB > 8 MiB
    spec = {"fact": "t", "filters": [], "probes": [], "group_by": [{"col": "a"}],
            "aggs": [{"op": "COUNT"}, {"op": "SUM", "terms": [{"ref": {"col": "v"}}]},
                     {"op": "SUM", "terms": [{"ref": {"col": "a"}}]}]}
    p = db.plan(spec)
    with pytest.raises(dpf.DpfError) as e:
        dpf.execute_noalloc(ctx, [p])
    assert e.value.code == dpf.DPF_ERR_UNSUPPORTED
    # the fragmented mode is not offered without allocation
    import ctypes as C
    arr = (C.c_void_p * 1)(p.h.value)
    o = dpf.dpf_exec_opts(dpf.DPF_MODE_FRAGMENTED, 0, 0, -1, 0, 0)
    h = C.c_void_p()
    st = dpf.load().dpf_execute_noalloc(ctx.h, 1, C.cast(arr, C.c_void_p), C.byref(o), None, C.byref(h))
    assert st == dpf.DPF_ERR_UNSUPPORTED and not h.value
    # the ordinary execution of the same plan still works
    G.assert_same(G.run_gpu(db, spec), oracle.run(spec, {"t": t}), "dpf_execute of the oversized plan")
    p.release()
