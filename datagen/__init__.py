"""Seeded, counter-based synthetic inputs shared by the oracle tests, the GPU
tests and the benchmark.

This package holds input generation only: value streams, tables shaped like
the star-schema workloads of the paper's evaluation (Section 5.1), and plain
query descriptions.  It contains none of the query method's arithmetic (no
encoding, filtering, joining or aggregation), so the oracle and the GPU path
can both consume it without sharing any of the computation they check.

Random source: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), counter based:
``x_i = mix(stream + (i + 1) * GAMMA)`` with ``stream = mix(seed ^ fnv1a(name))``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdatagen.so")
_SRC = os.path.join(_HERE, "datagen.c")


def build() -> str:
    """Compile the generator library with gcc (always recompiles)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        u64, i64, i32, p = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.dg_fnv1a.argtypes, lib.dg_fnv1a.restype = [ctypes.c_char_p], u64
        lib.dg_stream.argtypes, lib.dg_stream.restype = [u64, ctypes.c_char_p], u64
        lib.dg_raw.argtypes = [u64, i64, i64, p]
        lib.dg_uniform_i64.argtypes = [u64, i64, i64, i64, i64, p]
        lib.dg_uniform_i32.argtypes = [u64, i64, i64, i64, i64, p]
        lib.dg_hist.argtypes = [u64, i64, i64, i64, p]
        lib.dg_sorted_from_hist.argtypes = [p, i64, i64, i64, i64, p]
        lib.dg_vocab.argtypes, lib.dg_vocab.restype = [u64, i32, i32, i32, p, p], i32
        lib.dg_comment_offsets.argtypes = [u64, i64, i64, i32, i32, p]
        lib.dg_comment_bytes.argtypes = [u64, p, p, i32, i32, i64, i64, i32, i32, p, i32, i32, p, p]
        for f in ("dg_raw", "dg_uniform_i64", "dg_uniform_i32", "dg_hist", "dg_sorted_from_hist",
                  "dg_comment_offsets", "dg_comment_bytes"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Strings(NamedTuple):
    """A variable-length string column: ``offsets`` (int64, n + 1 entries,
    offsets[0] == 0) into the concatenated ``data`` bytes (uint8)."""

    offsets: np.ndarray
    data: np.ndarray

    def __len__(self) -> int:
        return len(self.offsets) - 1

    def get(self, i: int) -> bytes:
        return self.data[self.offsets[i]:self.offsets[i + 1]].tobytes()


def stream(seed: int, name: str) -> int:
    return int(_load().dg_stream(seed & (2**64 - 1), name.encode()))


def raw(seed: int, name: str, n: int, row0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().dg_raw(stream(seed, name), row0, n, _ptr(out))
    return out


def uniform(seed: int, name: str, n: int, lo: int, hi: int, row0: int = 0,
            dtype=np.int64) -> np.ndarray:
    """Rows row0..row0+n-1 of a column uniform on [lo, hi] (inclusive)."""
    lib = _load()
    st = stream(seed, name)
    if np.dtype(dtype) == np.int32:
        out = np.empty(n, dtype=np.int32)
        lib.dg_uniform_i32(st, row0, n, lo, hi, _ptr(out))
    else:
        out = np.empty(n, dtype=np.int64)
        lib.dg_uniform_i64(st, row0, n, lo, hi, _ptr(out))
    return out


def sorted_uniform(seed: int, name: str, n: int, lo: int, hi: int, dtype=np.int64) -> np.ndarray:
    """The n draws of ``uniform(seed, name, n, lo, hi)`` in ascending order
    (one histogram pass, then a fill from the prefix counts)."""
    lib = _load()
    nb = hi - lo + 1
    counts = np.empty(nb, dtype=np.int64)
    lib.dg_hist(stream(seed, name), n, lo, hi, _ptr(counts))
    out = np.empty(n, dtype=np.int64)
    if n:
        lib.dg_sorted_from_hist(_ptr(counts), nb, lo, 0, n, _ptr(out))
    return out.astype(dtype, copy=False)


def vocabulary(seed: int, nwords: int = 2000, minlen: int = 3, maxlen: int = 10) -> list[bytes]:
    """nwords distinct lowercase words with lengths uniform in [minlen, maxlen]."""
    buf = np.zeros(nwords * maxlen, dtype=np.uint8)
    lens = np.zeros(nwords, dtype=np.int32)
    rc = _load().dg_vocab(seed, nwords, minlen, maxlen, _ptr(buf), _ptr(lens))
    if rc != 0:
        raise ValueError("vocabulary space too small")
    return [buf[k * maxlen:k * maxlen + lens[k]].tobytes() for k in range(nwords)]


def comments(seed: int, name: str, n: int, vocab: list[bytes], minlen: int = 10, maxlen: int = 43,
             plant: bytes = b"", plant_pct: int = 0, row0: int = 0) -> Strings:
    """Comment strings of rows row0..row0+n-1: vocabulary words joined by
    single spaces and truncated to a length uniform in [minlen, maxlen];
    plant_pct percent of rows start with ``plant``."""
    lib = _load()
    st = stream(seed, name)
    maxw = max(len(w) for w in vocab)
    vbuf = np.zeros(len(vocab) * maxw, dtype=np.uint8)
    vlens = np.zeros(len(vocab), dtype=np.int32)
    for k, w in enumerate(vocab):
        vbuf[k * maxw:k * maxw + len(w)] = np.frombuffer(w, dtype=np.uint8)
        vlens[k] = len(w)
    offsets = np.empty(n + 1, dtype=np.int64)
    lib.dg_comment_offsets(st, row0, n, minlen, maxlen, _ptr(offsets))
    data = np.empty(int(offsets[-1]) + 1, dtype=np.uint8)  # +1 keeps the pointer valid at n == 0
    pl = np.frombuffer(plant, dtype=np.uint8).copy() if plant else np.zeros(1, dtype=np.uint8)
    lib.dg_comment_bytes(st, _ptr(vbuf), _ptr(vlens), len(vocab), maxw, row0, n, minlen, maxlen,
                         _ptr(pl), len(plant), plant_pct, _ptr(offsets), _ptr(data))
    return Strings(offsets, data[:int(offsets[-1])])
