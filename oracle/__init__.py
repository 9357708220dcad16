"""Python entry to the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the GPU path; it translates the plain query description of
:mod:`datagen.workloads` into the oracle's own structures and evaluates it
row at a time over the uncompressed columns.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

OK, ERR_INVALID, ERR_OVERFLOW, ERR_DUPLICATE, ERR_OOM = 0, 1, 2, 3, 4
_OPS = {"LT": 1, "LE": 2, "GT": 3, "GE": 4, "EQ": 5, "NE": 6, "BETWEEN": 7, "IN": 8,
        "STR_CONTAINS_SEQ": 9}
_AGGS = {"COUNT": 0, "SUM": 1, "AVG": 2}
MAX_PROBES, MAX_KEYS, MAX_AGGS, MAX_TERMS, MAX_PAYLOADS = 8, 8, 16, 3, 2


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({1: "invalid query", 2: "int64 overflow", 3: "duplicate build key",
                          4: "out of memory"}.get(code, f"error {code}"))
        self.code = code


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-pthread", "-o", tmp, _SRC])
    os.replace(tmp, _SO)
    return _SO


class _Col(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ival", C.c_void_p), ("str_off", C.c_void_p),
                ("str_bytes", C.c_void_p)]


class _Pred(C.Structure):
    _fields_ = [("col", C.c_int32), ("op", C.c_int32), ("a", C.c_int64), ("b", C.c_int64),
                ("nin", C.c_int32), ("in_", C.c_void_p), ("s1", C.c_void_p), ("n1", C.c_int32),
                ("s2", C.c_void_p), ("n2", C.c_int32)]


class _Probe(C.Structure):
    pass


_Probe._fields_ = [("cols", C.c_void_p), ("ncols", C.c_int32), ("key_col", C.c_int32),
                   ("preds", C.c_void_p), ("npreds", C.c_int32), ("npay", C.c_int32),
                   ("pay_col", C.c_int32 * MAX_PAYLOADS), ("fact_fk_col", C.c_int32),
                   ("pay_src", C.c_int32 * MAX_PAYLOADS), ("sub", C.c_void_p), ("nsub", C.c_int32)]


class _Ref(C.Structure):
    _fields_ = [("src", C.c_int32), ("idx", C.c_int32)]


class _Term(C.Structure):
    _fields_ = [("has_ref", C.c_int32), ("ref", _Ref), ("mul", C.c_int64), ("add", C.c_int64)]


class _Agg(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nterms", C.c_int32), ("terms", _Term * MAX_TERMS)]


class _Query(C.Structure):
    _fields_ = [("fact", C.c_void_p), ("nfact", C.c_int32), ("preds", C.c_void_p),
                ("npreds", C.c_int32), ("probes", C.c_void_p), ("nprobes", C.c_int32),
                ("keys", C.c_void_p), ("nkeys", C.c_int32), ("aggs", C.c_void_p),
                ("naggs", C.c_int32)]


_lib = None


def use_library(path: str | None) -> None:
    """Point the wrapper at another build of ``oracle.c`` (the tests use this
    to check that deliberately broken copies fail the pins); None restores
    the default build."""
    global _lib, _SO
    _SO = path or os.path.join(_HERE, "liboracle.so")
    _lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = C.CDLL(_SO)
        lib.orc_run.argtypes = [C.POINTER(_Query), C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int32)]
        lib.orc_run.restype = C.c_int
        lib.orc_run_threads.argtypes = [C.POINTER(_Query), C.c_int32, C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        lib.orc_run_threads.restype = C.c_int
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_free.restype = None
        lib.orc_count_filter.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32]
        lib.orc_count_filter.restype = C.c_int64
        _lib = lib
    return _lib


class _Keep:
    """Holds every buffer the C structures point to until the call returns."""

    def __init__(self):
        self.objs = []

    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.objs.append(a)
        return a.ctypes.data_as(C.c_void_p)

    def raw(self, b: bytes):
        a = np.frombuffer(b, dtype=np.uint8).copy() if b else np.zeros(1, np.uint8)
        self.objs.append(a)
        return a.ctypes.data_as(C.c_void_p)


def _is_str(col) -> bool:
    return hasattr(col, "offsets") and hasattr(col, "data")


def _columns(table: dict, keep: _Keep):
    names = list(table.keys())
    cols = (_Col * max(1, len(names)))()
    for i, nm in enumerate(names):
        c = table[nm]
        if _is_str(c):
            cols[i].nrows = len(c.offsets) - 1
            cols[i].str_off = keep.arr(c.offsets, np.int64)
            cols[i].str_bytes = keep.arr(c.data if len(c.data) else np.zeros(1, np.uint8), np.uint8)
        else:
            cols[i].nrows = len(c)
            cols[i].ival = keep.arr(c, np.int64)
    keep.objs.append(cols)
    return cols, {nm: i for i, nm in enumerate(names)}


def _preds(preds: list, index: dict, keep: _Keep):
    arr = (_Pred * max(1, len(preds)))()
    for i, p in enumerate(preds):
        arr[i].col = index[p["col"]]
        arr[i].op = _OPS[p["op"]]
        if p["op"] == "BETWEEN":
            arr[i].a, arr[i].b = int(p["lo"]), int(p["hi"])
        elif p["op"] == "IN":
            vals = [int(v) for v in p["values"]]
            arr[i].nin = len(vals)
            arr[i].in_ = keep.arr(np.array(vals if vals else [0], dtype=np.int64), np.int64)
        elif p["op"] == "STR_CONTAINS_SEQ":
            arr[i].s1, arr[i].n1 = keep.raw(p["s1"]), len(p["s1"])
            arr[i].s2, arr[i].n2 = keep.raw(p["s2"]), len(p["s2"])
        else:
            arr[i].a = int(p["value"])
    keep.objs.append(arr)
    return arr


def _ref(r: dict, index: dict) -> _Ref:
    if "col" in r:
        return _Ref(-1, index[r["col"]])
    return _Ref(int(r["probe"]), int(r["payload"]))


def _probe_array(probes: list, parent_index: dict, tables: dict, keep: _Keep):
    """The probes of one table (the fact table, or a joined dimension) as an
    array of _Probe; a probe's own "probes" describe its joined build side,
    and a payload {"probe": j, "payload": k} takes payload k of that side's
    probe j."""
    if len(probes) > MAX_PROBES:
        raise OracleError(ERR_INVALID)
    parr = (_Probe * max(1, len(probes)))()
    for j, pr in enumerate(probes):
        dcols, dindex = _columns(tables[pr["dim"]], keep)
        parr[j].cols = C.cast(dcols, C.c_void_p)
        parr[j].ncols = len(dindex)
        parr[j].key_col = dindex[pr["key"]]
        dp = _preds(pr.get("filters", []), dindex, keep)
        parr[j].preds = C.cast(dp, C.c_void_p)
        parr[j].npreds = len(pr.get("filters", []))
        pays = pr.get("payloads", [])
        if len(pays) > MAX_PAYLOADS:
            raise OracleError(ERR_INVALID)
        parr[j].npay = len(pays)
        for k, pc in enumerate(pays):
            if isinstance(pc, dict):
                parr[j].pay_src[k] = int(pc["probe"])
                parr[j].pay_col[k] = int(pc["payload"])
            else:
                parr[j].pay_src[k] = -1
                parr[j].pay_col[k] = dindex[pc]
        parr[j].fact_fk_col = parent_index[pr["fk"]]
        subs = pr.get("probes", [])
        if subs:
            sarr = _probe_array(subs, dindex, tables, keep)
            parr[j].sub = C.cast(sarr, C.c_void_p)
            parr[j].nsub = len(subs)
    keep.objs.append(parr)
    return parr


def run(spec: dict, tables: dict, threads: int = 1) -> np.ndarray:
    """Evaluate a query description over uncompressed tables; returns the
    (ngroups, ncols) int64 result, ascending by group key.  threads > 1 runs
    the timing-only variant that splits the fact rows over that many host
    threads (same records)."""
    lib = _load()
    keep = _Keep()
    fact = tables[spec["fact"]]
    fcols, findex = _columns(fact, keep)
    probes = spec.get("probes", [])
    parr = _probe_array(probes, findex, tables, keep)
    keys = spec.get("group_by", [])
    karr = (_Ref * max(1, len(keys)))(*[_ref(r, findex) for r in keys])
    aggs = spec.get("aggs", [])
    aarr = (_Agg * max(1, len(aggs)))()
    for a, ag in enumerate(aggs):
        aarr[a].kind = _AGGS[ag["op"]]
        terms = ag.get("terms", [])
        if len(terms) > MAX_TERMS:
            raise OracleError(ERR_INVALID)
        aarr[a].nterms = len(terms)
        for t, tm in enumerate(terms):
            if "const" in tm:
                aarr[a].terms[t] = _Term(0, _Ref(0, 0), 1, int(tm["const"]))
            else:
                aarr[a].terms[t] = _Term(1, _ref(tm["ref"], findex), int(tm.get("mul", 1)),
                                         int(tm.get("add", 0)))
    fp = _preds(spec.get("filters", []), findex, keep)
    q = _Query(C.cast(fcols, C.c_void_p), len(findex), C.cast(fp, C.c_void_p),
               len(spec.get("filters", [])), C.cast(parr, C.c_void_p), len(probes),
               C.cast(karr, C.c_void_p), len(keys), C.cast(aarr, C.c_void_p), len(aggs))
    out = C.c_void_p()
    ng = C.c_int64()
    nc = C.c_int32()
    if threads > 1:
        rc = lib.orc_run_threads(C.byref(q), int(threads), C.byref(out), C.byref(ng), C.byref(nc))
    else:
        rc = lib.orc_run(C.byref(q), C.byref(out), C.byref(ng), C.byref(nc))
    if rc != OK:
        raise OracleError(rc)
    try:
        n = ng.value * nc.value
        res = np.ctypeslib.as_array((C.c_int64 * max(1, n)).from_address(out.value))[:n].copy()
    finally:
        lib.orc_free(out)
    return res.reshape(ng.value, nc.value)


def count_filter(table: dict, preds: list) -> int:
    """Number of rows of ``table`` that pass the conjunction ``preds``."""
    lib = _load()
    keep = _Keep()
    cols, index = _columns(table, keep)
    p = _preds(preds, index, keep)
    n = lib.orc_count_filter(C.cast(cols, C.c_void_p), len(index), C.cast(p, C.c_void_p), len(preds))
    if n < 0:
        raise OracleError(ERR_INVALID)
    return int(n)
