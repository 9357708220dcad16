"""A second, deliberately naive evaluator of the query description, used only
to pin the oracle on tiny inputs: nested loops over dimension rows (no hash,
no sort), an all-pairs scan for the in-order string predicate, a dict of
groups, Python integers with explicit int64 range checks."""
from __future__ import annotations

INT64_MIN, INT64_MAX = -(2**63), 2**63 - 1


class Overflow(Exception):
    pass


class Duplicate(Exception):
    pass


def _chk(v: int) -> int:
    if v < INT64_MIN or v > INT64_MAX:
        raise Overflow()
    return v


def _cell(col, r):
    if hasattr(col, "offsets"):
        return col.data[col.offsets[r]:col.offsets[r + 1]].tobytes()
    return int(col[r])


def contains_in_order_allpairs(s: bytes, w1: bytes, w2: bytes) -> bool:
    n, n1, n2 = len(s), len(w1), len(w2)
    for i in range(n - n1 + 1):
        if s[i:i + n1] != w1:
            continue
        for j in range(i + n1, n - n2 + 1):
            if s[j:j + n2] == w2:
                return True
    return False


def pred_holds(p: dict, table: dict, r: int) -> bool:
    x = _cell(table[p["col"]], r)
    op = p["op"]
    if op == "STR_CONTAINS_SEQ":
        return contains_in_order_allpairs(x, p["s1"], p["s2"])
    if op == "LT":
        return x < p["value"]
    if op == "LE":
        return x <= p["value"]
    if op == "GT":
        return x > p["value"]
    if op == "GE":
        return x >= p["value"]
    if op == "EQ":
        return x == p["value"]
    if op == "NE":
        return x != p["value"]
    if op == "BETWEEN":
        return p["lo"] <= x <= p["hi"]
    if op == "IN":
        return any(x == v for v in p["values"])
    raise ValueError(op)


def _nrows(table):
    c = next(iter(table.values()))
    return len(c.offsets) - 1 if hasattr(c, "offsets") else len(c)


def qualifying(pr: dict, tables: dict) -> list:
    """[(key, [payload values])] of the dimension rows a probe joins with: the
    rows passing its filters that also find a match in each of its own
    probes (a joined build side), found by nested loops."""
    dim = tables[pr["dim"]]
    subs = [qualifying(sp, tables) for sp in pr.get("probes", [])]
    out = []
    for d in range(_nrows(dim)):
        if not all(pred_holds(p, dim, d) for p in pr.get("filters", [])):
            continue
        sub_hits = []
        for sp, rows in zip(pr.get("probes", []), subs):
            fk = _cell(dim[sp["fk"]], d)
            m = [pay for key, pay in rows if key == fk]
            if not m:
                break
            sub_hits.append(m[0])
        if len(sub_hits) != len(subs):
            continue
        pays = []
        for c in pr.get("payloads", []):
            pays.append(sub_hits[c["probe"]][c["payload"]] if isinstance(c, dict) else _cell(dim[c], d))
        out.append((_cell(dim[pr["key"]], d), pays))
    keys = [k for k, _ in out]
    if len(keys) != len(set(keys)):
        raise Duplicate()
    return out


def evaluate(spec: dict, tables: dict) -> list:
    fact = tables[spec["fact"]]
    probes = spec.get("probes", [])
    groups = {}
    quals = [qualifying(pr, tables) for pr in probes]  # raises Duplicate up front
    for r in range(_nrows(fact)):
        if not all(pred_holds(p, fact, r) for p in spec.get("filters", [])):
            continue
        hits = []
        for pr, rows in zip(probes, quals):
            fk = _cell(fact[pr["fk"]], r)
            found = [pay for key, pay in rows if key == fk]
            if not found:
                break
            hits.append(found[0])
        if len(hits) != len(probes):
            continue

        def val(ref):
            if "col" in ref:
                return _cell(fact[ref["col"]], r)
            return hits[ref["probe"]][ref["payload"]]

        key = tuple(val(k) for k in spec.get("group_by", []))
        acc = groups.setdefault(key, [0] * (1 + len(spec["aggs"])))
        acc[0] = _chk(acc[0] + 1)
        for a, ag in enumerate(spec["aggs"]):
            if ag["op"] == "COUNT":
                continue
            prod = 1
            for t in ag["terms"]:
                if "const" in t:
                    v = t["const"]
                else:
                    v = _chk(_chk(t.get("mul", 1) * val(t["ref"])) + t.get("add", 0))
                prod = _chk(prod * v)
            acc[1 + a] = _chk(acc[1 + a] + prod)
    out = []
    for key in sorted(groups):
        acc = groups[key]
        row = list(key)
        for a, ag in enumerate(spec["aggs"]):
            if ag["op"] == "COUNT":
                row.append(acc[0])
            elif ag["op"] == "SUM":
                row.append(acc[1 + a])
            else:
                row += [acc[1 + a], acc[0]]
        out.append(row)
    return out
