import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from datagen import Strings  # noqa: E402


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def to_strings(items) -> Strings:
    bs = [s.encode() if isinstance(s, str) else bytes(s) for s in items]
    off = np.zeros(len(bs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(b) for b in bs])
    data = np.frombuffer(b"".join(bs), dtype=np.uint8).copy()
    return Strings(off, data)


def _decode_query(q):
    """JSON strings -> bytes for the string predicate words."""
    q = json.loads(json.dumps(q))
    for p in q.get("filters", []):
        if p["op"] == "STR_CONTAINS_SEQ":
            p["s1"], p["s2"] = p["s1"].encode(), p["s2"].encode()
    return q


def load_hand_cases():
    path = os.path.join(ROOT, "tests", "golden", "hand_cases.json")
    with open(path) as f:
        doc = json.load(f)
    tables = {}
    for tname, cols in doc["tables"].items():
        t = {}
        for cname, vals in cols.items():
            if vals and isinstance(vals[0], str):
                t[cname] = to_strings(vals)
            else:
                t[cname] = np.asarray(vals, dtype=np.int64)
        tables[tname] = t
    cases = []
    for c in doc["cases"]:
        c = dict(c)
        c["query"] = _decode_query(c["query"])
        cases.append(c)
    return tables, cases


@pytest.fixture(scope="session")
def hand_cases():
    return load_hand_cases()
