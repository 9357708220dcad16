"""ctypes binding of libdpf (include/dpf.h).

The ``dpf_*`` functions here have the names and arguments of the C ABI and
only marshal arguments; every step of a query runs in the library's HIP
kernels.  The small classes below wrap handles and translate the plain query
description of :mod:`datagen.workloads` into ``dpf_plan_desc`` structures.
PyTorch is used for device memory (its caching allocator can back the
library's HBM allocations) and for streams.

The library must be built (``python -m paper_2605_10511_amd.build``); there is
no fallback path: loading fails loudly when ``libdpf.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdpf.so")

# status codes
DPF_OK = 0
DPF_ERR_INVALID_ARG, DPF_ERR_OOM, DPF_ERR_HIP, DPF_ERR_UNSUPPORTED = -1, -2, -3, -4
DPF_ERR_OVERFLOW, DPF_ERR_CAPACITY, DPF_ERR_DUPLICATE_KEY, DPF_ERR_CORRUPT, DPF_ERR_NOT_READY = -5, -6, -7, -8, -9
DPF_MEM_HBM, DPF_MEM_HOST_MAPPED = 0, 1
DPF_TYPE_I32, DPF_TYPE_I64, DPF_TYPE_STR = 1, 2, 3
DPF_ENC_AUTO, DPF_ENC_FOR, DPF_ENC_DELTA, DPF_ENC_DICT, DPF_ENC_VARLEN, DPF_ENC_PLAIN, DPF_ENC_FSST = 0, 1, 2, 3, 4, 5, 6
DPF_PLACE_HBM, DPF_PLACE_HOST_MAPPED, DPF_PLACE_HOST = 0, 1, 2
DPF_OP = {"LT": 1, "LE": 2, "GT": 3, "GE": 4, "EQ": 5, "NE": 6, "BETWEEN": 7, "IN": 8, "STR_CONTAINS_SEQ": 9}
DPF_HASH_AUTO, DPF_HASH_LDS, DPF_HASH_HBM = 0, 1, 2
DPF_REF_COL, DPF_REF_PAYLOAD = 0, 1
DPF_AGG = {"COUNT": 0, "SUM": 1, "AVG": 2}
DPF_MODE_FUSED, DPF_MODE_FRAGMENTED = 0, 1
ENCODINGS = {"AUTO": 0, "FOR": 1, "DELTA": 2, "DICT": 3, "VARLEN": 4, "PLAIN": 5, "FSST": 6}
PLACEMENTS = {"HBM": 0, "HOST_MAPPED": 1, "HOST": 2}
HASH_PLACEMENTS = {"AUTO": 0, "LDS": 1, "HBM": 2}


class dpf_allocator(C.Structure):
    _fields_ = [("user", C.c_void_p),
                ("alloc", C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_int32))]


class dpf_ctx_info(C.Structure):
    _fields_ = [("device", C.c_int32), ("num_cus", C.c_int32), ("lds_per_block", C.c_int64),
                ("hbm_bytes", C.c_int64), ("launches", C.c_int64)]


class dpf_column_src(C.Structure):
    _fields_ = [("type", C.c_int32), ("nrows", C.c_int64), ("values", C.c_void_p),
                ("str_offsets", C.c_void_p), ("str_bytes", C.c_void_p)]


class dpf_encode_opts(C.Structure):
    _fields_ = [("encoding", C.c_int32), ("chunk_rows", C.c_int32), ("placement", C.c_int32),
                ("threads", C.c_int32)]


class dpf_column_stats(C.Structure):
    _fields_ = [("type", C.c_int32), ("encoding", C.c_int32), ("placement", C.c_int32),
                ("chunk_rows", C.c_int32), ("nrows", C.c_int64), ("nchunks", C.c_int64),
                ("nminiblocks", C.c_int64), ("compressed_bytes", C.c_int64), ("min", C.c_int64),
                ("max", C.c_int64), ("ndict", C.c_int64), ("str_bytes", C.c_int64)]


class dpf_chunk_info(C.Structure):
    _fields_ = [("row_start", C.c_int64), ("nrows", C.c_int64), ("byte_offset", C.c_int64),
                ("byte_length", C.c_int64), ("min", C.c_int64), ("max", C.c_int64)]


class dpf_pred(C.Structure):
    _fields_ = [("col", C.c_int32), ("op", C.c_int32), ("a", C.c_int64), ("b", C.c_int64),
                ("n_in", C.c_int32), ("in_values", C.c_void_p), ("s1", C.c_void_p), ("n1", C.c_int32),
                ("s2", C.c_void_p), ("n2", C.c_int32)]


class dpf_hash_desc(C.Structure):
    _fields_ = [("ncols", C.c_int32), ("cols", C.c_void_p), ("key_col", C.c_int32),
                ("npreds", C.c_int32), ("preds", C.c_void_p), ("npayloads", C.c_int32),
                ("payload_cols", C.c_int32 * 2), ("placement", C.c_int32),
                ("nprobes", C.c_int32), ("probes", C.c_void_p), ("payload_probe", C.c_int32 * 2)]


class dpf_hash_stats(C.Structure):
    _fields_ = [("entries", C.c_int64), ("capacity", C.c_int64), ("bytes", C.c_int64),
                ("lds_eligible", C.c_int32), ("placement", C.c_int32), ("npayloads", C.c_int32),
                ("key_min", C.c_int64), ("key_max", C.c_int64),
                ("payload_min", C.c_int64 * 2), ("payload_max", C.c_int64 * 2),
                ("device_bytes", C.c_int64)]


class dpf_ref(C.Structure):
    _fields_ = [("kind", C.c_int32), ("idx", C.c_int32), ("probe", C.c_int32)]


class dpf_term(C.Structure):
    _fields_ = [("has_ref", C.c_int32), ("ref", dpf_ref), ("mul", C.c_int64), ("add", C.c_int64)]


class dpf_agg(C.Structure):
    _fields_ = [("op", C.c_int32), ("nterms", C.c_int32), ("terms", dpf_term * 3)]


class dpf_probe(C.Structure):
    _fields_ = [("fk_col", C.c_int32), ("hash", C.c_void_p)]


class dpf_plan_desc(C.Structure):
    _fields_ = [("ncols", C.c_int32), ("cols", C.c_void_p), ("npreds", C.c_int32), ("preds", C.c_void_p),
                ("nprobes", C.c_int32), ("probes", C.c_void_p), ("nkeys", C.c_int32), ("keys", C.c_void_p),
                ("naggs", C.c_int32), ("aggs", C.c_void_p)]


class dpf_exec_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("wg_per_cu", C.c_int32), ("rows_per_item", C.c_int32),
                ("lds_hash_bytes", C.c_int32), ("waves_per_wg", C.c_int32), ("max_workgroups", C.c_int32)]


# Function table: name -> (restype, argtypes)
_P = C.c_void_p
_FUNCS = {
    "dpf_last_error": (C.c_char_p, []),
    "dpf_ctx_create": (C.c_int32, [C.c_int32, _P, C.POINTER(_P)]),
    "dpf_ctx_destroy": (None, [_P]),
    "dpf_ctx_get_info": (C.c_int32, [_P, C.POINTER(dpf_ctx_info)]),
    "dpf_column_encode": (C.c_int32, [_P, C.POINTER(dpf_column_src), C.POINTER(dpf_encode_opts), C.POINTER(_P)]),
    "dpf_column_info": (C.c_int32, [_P, C.POINTER(dpf_column_stats)]),
    "dpf_column_chunk": (C.c_int32, [_P, C.c_int64, C.POINTER(dpf_chunk_info)]),
    "dpf_column_decode": (C.c_int32, [_P, _P, _P, _P, C.c_size_t]),
    "dpf_column_debug_offsets": (C.c_int32, [_P, C.POINTER(_P)]),
    "dpf_column_release": (None, [_P]),
    "dpf_hash_build": (C.c_int32, [_P, C.POINTER(dpf_hash_desc), _P, C.POINTER(_P)]),
    "dpf_hash_info": (C.c_int32, [_P, C.POINTER(dpf_hash_stats)]),
    "dpf_hash_release": (None, [_P]),
    "dpf_plan_build": (C.c_int32, [_P, C.POINTER(dpf_plan_desc), C.POINTER(_P)]),
    "dpf_plan_footprint": (C.c_int32, [_P, C.POINTER(C.c_size_t)]),
    "dpf_plan_blocks": (C.c_int32, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "dpf_plan_release": (None, [_P]),
    "dpf_execute": (C.c_int32, [_P, C.c_int32, _P, C.POINTER(dpf_exec_opts), _P, C.POINTER(_P)]),
    "dpf_execute_noalloc": (C.c_int32, [_P, C.c_int32, _P, C.POINTER(dpf_exec_opts), _P, C.POINTER(_P)]),
    "dpf_result_get": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                   C.POINTER(C.POINTER(C.c_int64))]),
    "dpf_result_release": (None, [_P]),
    "dpf_measure_read": (C.c_int32, [_P, C.c_int32, C.c_size_t, C.c_int32, C.c_int32, _P, C.POINTER(C.c_float)]),
}

_lib = None


def load() -> C.CDLL:
    """Load libdpf.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_10511_amd.build`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _FUNCS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def exported_names() -> list[str]:
    return list(_FUNCS)


class DpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpf error {code}: {msg}")
        self.code = code


def _check(st: int):
    if st != DPF_OK:
        raise DpfError(st, load().dpf_last_error().decode(errors="replace"))


def __getattr__(name):
    # dpf_* names resolve to the C functions themselves
    if name.startswith("dpf_") and name in _FUNCS:
        return getattr(load(), name)
    raise AttributeError(name)


# ---------------------------------------------------------------------------
# Memory: torch's caching allocator for HBM, pinned torch tensors for
# host-mapped memory
# ---------------------------------------------------------------------------
class TorchAllocator:
    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device
        self.host = {}
        self.c = dpf_allocator(None, dpf_allocator._fields_[1][1](self._alloc),
                               dpf_allocator._fields_[2][1](self._free))

    def _alloc(self, user, nbytes, kind):
        try:
            if kind == DPF_MEM_HBM:
                return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, pin_memory=True)
            self.host[t.data_ptr()] = t
            return t.data_ptr()
        except Exception:
            return None

    def _free(self, user, p, kind):
        try:
            if kind == DPF_MEM_HBM:
                self.torch.cuda.caching_allocator_delete(p)
            else:
                self.host.pop(p, None)
        except Exception:
            pass


class Context:
    """A library context on one GPU (device=-1: host-only encoding).  By
    default its device memory comes from torch's caching allocator and its
    pinned host memory from torch's pinned-memory allocator."""

    def __init__(self, device: int = 0, torch_allocator: bool = True):
        lib = load()
        self._alloc = TorchAllocator(device) if (torch_allocator and device >= 0) else None
        h = C.c_void_p()
        _check(lib.dpf_ctx_create(device, C.byref(self._alloc.c) if self._alloc else None, C.byref(h)))
        self.h = h
        self.device = device

    def info(self) -> dpf_ctx_info:
        out = dpf_ctx_info()
        _check(load().dpf_ctx_get_info(self.h, C.byref(out)))
        return out

    def close(self):
        if self.h:
            load().dpf_ctx_destroy(self.h)
            self.h = None


def _is_str(a) -> bool:
    return hasattr(a, "offsets") and hasattr(a, "data")


class Column:
    """An encoded column (paper Section 3.4)."""

    def __init__(self, ctx: Context, values, encoding: str = "AUTO", chunk_rows: int = 65536,
                 placement: str = "HBM", threads: int = 0):
        lib = load()
        src = dpf_column_src()
        keep = []
        if _is_str(values):
            off = np.ascontiguousarray(values.offsets, dtype=np.int64)
            data = np.ascontiguousarray(values.data, dtype=np.uint8)
            if data.size == 0:
                data = np.zeros(1, np.uint8)
            keep += [off, data]
            src.type, src.nrows = DPF_TYPE_STR, len(off) - 1
            src.str_offsets, src.str_bytes = off.ctypes.data, data.ctypes.data
        else:
            arr = np.asarray(values)
            if arr.dtype == np.int32:
                src.type = DPF_TYPE_I32
            else:
                arr = arr.astype(np.int64, copy=False)
                src.type = DPF_TYPE_I64
            arr = np.ascontiguousarray(arr)
            keep.append(arr)
            src.nrows = len(arr)
            src.values = arr.ctypes.data if len(arr) else None
        opts = dpf_encode_opts(ENCODINGS[encoding], chunk_rows, PLACEMENTS[placement], threads)
        h = C.c_void_p()
        _check(lib.dpf_column_encode(ctx.h, C.byref(src), C.byref(opts), C.byref(h)))
        self.h = h
        self.ctx = ctx
        self.is_str = _is_str(values)

    def info(self) -> dpf_column_stats:
        s = dpf_column_stats()
        _check(load().dpf_column_info(self.h, C.byref(s)))
        return s

    def chunk(self, k: int) -> dpf_chunk_info:
        c = dpf_chunk_info()
        _check(load().dpf_column_chunk(self.h, k, C.byref(c)))
        return c

    def decode(self):
        s = self.info()
        if s.type == DPF_TYPE_STR:
            off = np.zeros(s.nrows + 1, dtype=np.int64)
            data = np.zeros(max(1, s.str_bytes), dtype=np.uint8)
            _check(load().dpf_column_decode(self.h, None, off.ctypes.data, data.ctypes.data, data.size))
            return off, data[:s.str_bytes]
        out = np.zeros(s.nrows, dtype=np.int32 if s.type == DPF_TYPE_I32 else np.int64)
        _check(load().dpf_column_decode(self.h, out.ctypes.data if s.nrows else None, None, None, 0))
        return out

    def debug_offsets(self) -> np.ndarray:
        p = C.c_void_p()
        _check(load().dpf_column_debug_offsets(self.h, C.byref(p)))
        n = self.info().nminiblocks + 1
        return np.ctypeslib.as_array((C.c_uint32 * n).from_address(p.value))

    def release(self):
        if self.h:
            load().dpf_column_release(self.h)
            self.h = None


def _stream_handle(stream) -> int | None:
    if stream is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream or None
        except Exception:
            return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class _Keep(list):
    def arr(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.append(a)
        return a.ctypes.data

    def raw(self, b: bytes):
        a = np.frombuffer(b, dtype=np.uint8).copy() if b else np.zeros(1, np.uint8)
        self.append(a)
        return a.ctypes.data


def _preds(preds: list, index: dict, keep: _Keep):
    arr = (dpf_pred * max(1, len(preds)))()
    for i, p in enumerate(preds):
        arr[i].col = index[p["col"]]
        arr[i].op = DPF_OP[p["op"]]
        if p["op"] == "BETWEEN":
            arr[i].a, arr[i].b = int(p["lo"]), int(p["hi"])
        elif p["op"] == "IN":
            vals = [int(v) for v in p["values"]]
            arr[i].n_in = len(vals)
            arr[i].in_values = keep.arr(vals or [0], np.int64)
        elif p["op"] == "STR_CONTAINS_SEQ":
            arr[i].s1, arr[i].n1 = keep.raw(p["s1"]), len(p["s1"])
            arr[i].s2, arr[i].n2 = keep.raw(p["s2"]), len(p["s2"])
        else:
            arr[i].a = int(p["value"])
    keep.append(arr)
    return arr


class Hash:
    """A dimension hash table (paper Section 3.1, Kernel #1; with ``probes``,
    a joined build side as in Kernel #2: ``probes`` is a list of (foreign-key
    column of ``cols``, Hash), and a payload {"probe": j, "payload": k} takes
    payload k of probe j)."""

    def __init__(self, ctx: Context, cols: dict, key: str, filters: list, payloads: list,
                 placement: str = "AUTO", stream=None, probes: list | None = None):
        lib = load()
        names = list(cols)
        index = {n: i for i, n in enumerate(names)}
        keep = _Keep()
        handles = (C.c_void_p * len(names))(*[cols[n].h.value for n in names])
        keep.append(handles)
        preds = _preds(filters, index, keep)
        d = dpf_hash_desc()
        d.ncols, d.cols = len(names), C.cast(handles, C.c_void_p)
        d.key_col = index[key]
        d.npreds, d.preds = len(filters), C.cast(preds, C.c_void_p)
        d.npayloads = len(payloads)
        for k, pc in enumerate(payloads):
            if isinstance(pc, dict):
                d.payload_cols[k], d.payload_probe[k] = int(pc["payload"]), int(pc["probe"])
            else:
                d.payload_cols[k], d.payload_probe[k] = index[pc], -1
        d.placement = HASH_PLACEMENTS[placement]
        probes = probes or []
        parr = (dpf_probe * max(1, len(probes)))()
        for j, (fk, h) in enumerate(probes):
            parr[j].fk_col = index[fk]
            parr[j].hash = h.h.value
        keep.append(parr)
        d.nprobes, d.probes = len(probes), C.cast(parr, C.c_void_p)
        h = C.c_void_p()
        _check(lib.dpf_hash_build(ctx.h, C.byref(d), _stream_handle(stream), C.byref(h)))
        self.h = h

    def info(self) -> dpf_hash_stats:
        s = dpf_hash_stats()
        _check(load().dpf_hash_info(self.h, C.byref(s)))
        return s

    def release(self):
        if self.h:
            load().dpf_hash_release(self.h)
            self.h = None


class Plan:
    """A compiled scan -> filter -> probe -> aggregate plan over fact columns."""

    def __init__(self, ctx: Context, fact: dict, spec: dict, hashes: list):
        lib = load()
        names = list(fact)
        index = {n: i for i, n in enumerate(names)}
        keep = _Keep()
        handles = (C.c_void_p * len(names))(*[fact[n].h.value for n in names])
        keep.append(handles)
        filters = spec.get("filters", [])
        preds = _preds(filters, index, keep)
        probes = spec.get("probes", [])
        parr = (dpf_probe * max(1, len(probes)))()
        for j, pr in enumerate(probes):
            parr[j].fk_col = index[pr["fk"]]
            parr[j].hash = hashes[j].h.value
        keys = spec.get("group_by", [])
        karr = (dpf_ref * max(1, len(keys)))(*[self._ref(r, index) for r in keys])
        aggs = spec["aggs"]
        aarr = (dpf_agg * max(1, len(aggs)))()
        for a, ag in enumerate(aggs):
            aarr[a].op = DPF_AGG[ag["op"]]
            terms = ag.get("terms", [])
            aarr[a].nterms = len(terms)
            for t, tm in enumerate(terms):
                if "const" in tm:
                    aarr[a].terms[t] = dpf_term(0, dpf_ref(0, 0, 0), 1, int(tm["const"]))
                else:
                    aarr[a].terms[t] = dpf_term(1, self._ref(tm["ref"], index), int(tm.get("mul", 1)),
                                                int(tm.get("add", 0)))
        d = dpf_plan_desc(len(names), C.cast(handles, C.c_void_p), len(filters), C.cast(preds, C.c_void_p),
                          len(probes), C.cast(parr, C.c_void_p), len(keys), C.cast(karr, C.c_void_p),
                          len(aggs), C.cast(aarr, C.c_void_p))
        h = C.c_void_p()
        _check(lib.dpf_plan_build(ctx.h, C.byref(d), C.byref(h)))
        self.h = h
        self.ctx = ctx
        self.ncols = len(names)
        self.nrows = fact[names[0]].info().nrows

    @staticmethod
    def _ref(r: dict, index: dict) -> dpf_ref:
        if "col" in r:
            return dpf_ref(DPF_REF_COL, index[r["col"]], 0)
        return dpf_ref(DPF_REF_PAYLOAD, int(r["payload"]), int(r["probe"]))

    def footprint(self) -> int:
        n = C.c_size_t()
        _check(load().dpf_plan_footprint(self.h, C.byref(n)))
        return n.value

    def blocks(self) -> tuple[int, int]:
        """(scanned, total) blocks of the fused scan after chunk pruning."""
        a, b = C.c_int64(), C.c_int64()
        _check(load().dpf_plan_blocks(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def release(self):
        if self.h:
            load().dpf_plan_release(self.h)
            self.h = None


class Result:
    def __init__(self, h, n: int):
        self.h = h
        self.n = n

    def get(self, i: int = 0) -> np.ndarray:
        ng, nc = C.c_int64(), C.c_int32()
        rows = C.POINTER(C.c_int64)()
        _check(load().dpf_result_get(self.h, i, C.byref(ng), C.byref(nc), C.byref(rows)))
        n = ng.value * nc.value
        if n == 0:
            return np.zeros((ng.value, nc.value), dtype=np.int64)
        return np.ctypeslib.as_array(rows, shape=(n,)).copy().reshape(ng.value, nc.value)

    def release(self):
        if self.h:
            load().dpf_result_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def execute(ctx: Context, plans: list, mode: str = "FUSED", wg_per_cu: int = 0, rows_per_item: int = 0,
            lds_hash_bytes: int = -1, waves_per_wg: int = 0, max_workgroups: int = 0,
            stream=None) -> Result:
    """Enqueue plans (one fused launch, or the fragmented kernel sequence)."""
    lib = load()
    arr = (C.c_void_p * len(plans))(*[p.h.value for p in plans])
    o = dpf_exec_opts(DPF_MODE_FUSED if mode == "FUSED" else DPF_MODE_FRAGMENTED, wg_per_cu, rows_per_item,
                      lds_hash_bytes, waves_per_wg, max_workgroups)
    h = C.c_void_p()
    _check(lib.dpf_execute(ctx.h, len(plans), C.cast(arr, C.c_void_p), C.byref(o), _stream_handle(stream),
                           C.byref(h)))
    return Result(h, len(plans))


def execute_noalloc(ctx: Context, plans: list, wg_per_cu: int = 0, rows_per_item: int = 0,
                    lds_hash_bytes: int = -1, waves_per_wg: int = 0, max_workgroups: int = 0,
                    stream=None) -> Result:
    """Fused execution whose scratch state lives in the library's static
    device array (dpf_execute_noalloc); read the result after synchronising."""
    lib = load()
    arr = (C.c_void_p * len(plans))(*[p.h.value for p in plans])
    o = dpf_exec_opts(DPF_MODE_FUSED, wg_per_cu, rows_per_item, lds_hash_bytes, waves_per_wg, max_workgroups)
    h = C.c_void_p()
    _check(lib.dpf_execute_noalloc(ctx.h, len(plans), C.cast(arr, C.c_void_p), C.byref(o), _stream_handle(stream),
                                   C.byref(h)))
    return Result(h, len(plans))


def measure_read(ctx: Context, kind: str, nbytes: int, reps: int = 10, grid: int = 0, stream=None) -> list:
    """Per-launch milliseconds of a streaming read of nbytes from "HBM" or
    "HOST_MAPPED" memory (dpf_measure_read)."""
    ms = (C.c_float * reps)()
    k = DPF_MEM_HBM if kind == "HBM" else DPF_MEM_HOST_MAPPED
    _check(load().dpf_measure_read(ctx.h, k, int(nbytes), int(grid), int(reps), _stream_handle(stream), ms))
    return [float(x) for x in ms]


# ---------------------------------------------------------------------------
# Tables and prepared queries
# ---------------------------------------------------------------------------
class Database:
    """Encoded tables (name -> {column -> Column}) and query preparation."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.tables: dict[str, dict[str, Column]] = {}

    def add_table(self, name: str, columns: dict, encodings: dict | None = None, chunk_rows: int = 65536,
                  placement: str = "HBM", threads: int = 0):
        enc = encodings or {}
        self.tables[name] = {c: Column(self.ctx, v, enc.get(c, "AUTO"), chunk_rows, placement, threads)
                             for c, v in columns.items()}
        return self.tables[name]

    def build_hash(self, pr: dict, placement: str = "AUTO", stream=None) -> Hash:
        """The hash table a probe description joins with; a probe that has
        its own "probes" (a joined build side) has those built first, used
        during the build and released."""
        cols = self.tables[pr["dim"]]
        subs = [self.build_hash(sp, "AUTO", stream) for sp in pr.get("probes", [])]
        try:
            used = [pr["key"]] + [p["col"] for p in pr.get("filters", [])]
            used += [c for c in pr.get("payloads", []) if not isinstance(c, dict)]
            used += [sp["fk"] for sp in pr.get("probes", [])]
            sub = {c: cols[c] for c in dict.fromkeys(used)}
            return Hash(self.ctx, sub, pr["key"], pr.get("filters", []), pr.get("payloads", []), placement, stream,
                        probes=[(sp["fk"], h) for sp, h in zip(pr.get("probes", []), subs)])
        finally:
            for h in subs:
                h.release()

    def build_hashes(self, spec: dict, placements: list | None = None, stream=None) -> list:
        return [self.build_hash(pr, placements[j] if placements else "AUTO", stream)
                for j, pr in enumerate(spec.get("probes", []))]

    def plan(self, spec: dict, hashes: list | None = None, placements: list | None = None) -> Plan:
        if hashes is None:
            hashes = self.build_hashes(spec, placements)
        fact = self.tables[spec["fact"]]
        used = [p["col"] for p in spec.get("filters", [])] + [pr["fk"] for pr in spec.get("probes", [])]
        for r in spec.get("group_by", []):
            if "col" in r:
                used.append(r["col"])
        for ag in spec["aggs"]:
            for t in ag.get("terms", []):
                if "ref" in t and "col" in t["ref"]:
                    used.append(t["ref"]["col"])
        sub = {c: fact[c] for c in dict.fromkeys(used)} if used else {next(iter(fact)): next(iter(fact.values()))}
        p = Plan(self.ctx, sub, spec, hashes)
        p.hashes = hashes
        return p

    def release(self):
        for t in self.tables.values():
            for c in t.values():
                c.release()
        self.tables.clear()
