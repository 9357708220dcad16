"""GPU parity for join chains (paper Section 3.1's running example: a scan
that probes one hash table and builds the next, whose table a later
pipeline probes): a 3-table pipeline customer -> orders -> lineitem against
the CPU oracle, fused and fragmented, with the chained table in LDS or
device memory, and chained tables reused across a batch."""
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


@pytest.fixture(scope="module")
def chain(ctx):
    tables = W.chain_tables(1_000_003, seed=6)
    db = G.make_db(ctx, tables, chunk_rows=16384)
    return db, tables


@pytest.mark.parametrize("segment,lo,hi,qty", [(3, 700, 1600, 30), (0, 0, 2555, 51), (9, 2000, 2100, 5)])
def test_three_table_pipeline(chain, segment, lo, hi, qty):
    db, tables = chain
    spec = W.chain_query(segment, lo, hi, qty)
    want = oracle.run(spec, tables)
    assert len(want) > 0
    for placements in (None, ["HBM"], ["LDS"]):
        for mode in ("FUSED", "FRAGMENTED"):
            G.say(f"chain {segment} {lo}-{hi} {qty} {placements} {mode}")
            G.assert_same(G.run_gpu(db, spec, mode=mode, placements=placements), want, f"{placements} {mode}")


def test_chained_table_stats(ctx, chain):
    """The chained table holds exactly the orders that pass their filter and
    find a customer of the segment, with payloads from both sides."""
    db, tables = chain
    spec = W.chain_query(3, 700, 1600, 30)
    h = db.build_hash(spec["probes"][0])
    s = h.info()
    o, c = tables["orders"], tables["customer"]
    seg = c["c_segment"][o["o_custkey"] - 1]
    keep = (o["o_date"] >= 700) & (o["o_date"] <= 1600) & (seg == 3)
    assert s.entries == int(keep.sum())
    assert s.key_min == int(o["o_orderkey"][keep].min()) and s.key_max == int(o["o_orderkey"][keep].max())
    region = c["c_region"][o["o_custkey"][keep] - 1]
    assert s.payload_min[0] == int(region.min()) and s.payload_max[0] == int(region.max())
    assert s.payload_min[1] == int(o["o_priority"][keep].min())
    h.release()


def test_chain_in_a_batch(ctx, chain):
    """Several chain queries and a plain probe of the same orders table in one
    fused launch."""
    import torch
    from paper_2605_10511_amd import dpf
    db, tables = chain
    specs = [W.chain_query(s, 300 * s, 300 * s + 900, 10 + 5 * s) for s in range(5)]
    plain = W.chain_query(4)
    del plain["probes"][0]["probes"]
    plain["probes"][0]["payloads"] = ["o_priority", "o_priority"]
    specs.append(plain)
    wants = [oracle.run(s, tables) for s in specs]
    plans = [db.plan(s) for s in specs]
    res = dpf.execute(ctx, plans)
    torch.cuda.synchronize()
    for i, w in enumerate(wants):
        G.assert_same(res.get(i), w, f"batch plan {i}")
    res.release()
    for p in plans:
        p.release()
        for h in p.hashes:
            h.release()
