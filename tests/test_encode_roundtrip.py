"""Encoder/decoder round trips and format invariants, on the host (no GPU):
decode(encode(x)) == x bit-exactly for every encoding and bit width 0..64,
negative values, int64 extremes, constant blocks, chunk tails, empty and long
strings; compressed size = sum over mini blocks of header + 256 * width / 8;
the chunk directory's row starts are the prefix sum of its row counts (the
row-id index of paper Section 3.4.2) and its zone maps bound the values."""
import numpy as np
import pytest

from paper_2605_10511_amd import dpf
from tests.conftest import to_strings


@pytest.fixture(scope="module")
def hctx():
    return dpf.Context(-1)


def _roundtrip(ctx, x, enc, chunk_rows=65536):
    c = dpf.Column(ctx, x, enc, chunk_rows=chunk_rows, placement="HOST", threads=4)
    y = c.decode()
    return c, y


def _check_dir(c, x):
    s = c.info()
    start = 0
    for k in range(s.nchunks):
        ch = c.chunk(k)
        assert ch.row_start == start
        seg = x[ch.row_start:ch.row_start + ch.nrows]
        assert ch.nrows == len(seg)
        if len(seg):
            assert ch.min == int(seg.min()) and ch.max == int(seg.max())
        start += ch.nrows
    assert start == s.nrows


@pytest.mark.parametrize("enc", ["FOR", "DELTA", "DICT", "AUTO"])
@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 65536 * 2 + 17])
def test_roundtrip_sizes(hctx, enc, n):
    rng = np.random.default_rng(n)
    x = rng.integers(-50, 50, n).astype(np.int32)
    c, y = _roundtrip(hctx, x, enc)
    assert y.dtype == np.int32 and (y == x).all()
    _check_dir(c, x)


@pytest.mark.parametrize("width", list(range(0, 65)))
def test_every_width_for(hctx, width):
    rng = np.random.default_rng(width)
    n = 1000
    if width == 0:
        x = np.full(n, -7, dtype=np.int64)
    elif width == 64:
        x = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64)
        x[0], x[1] = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    else:
        hi = (1 << width) - 1
        x = (rng.integers(0, hi, n, dtype=np.uint64, endpoint=True).astype(np.int64)) - (1 << (width - 1))
        x[::256] = -(1 << (width - 1))   # pin the block minimum ...
        x[1::256] = hi - (1 << (width - 1))  # ... and maximum, so the width is exact
    c, y = _roundtrip(hctx, x, "FOR")
    assert (y == x).all()
    s = c.info()
    nmb = s.nminiblocks
    # full-range blocks use exactly `width` bits: size = headers + packed words
    assert s.compressed_bytes == nmb * 8 + (nmb + 1) * 4 + nmb * 8 * width * 4


@pytest.mark.parametrize("width", [0, 1, 7, 31, 33, 63, 64])
def test_delta_widths_and_extremes(hctx, width):
    rng = np.random.default_rng(100 + width)
    n = 3000
    if width == 64:
        x = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64)
    else:
        step = rng.integers(0, 1 << width, n, dtype=np.uint64) if width else np.zeros(n, np.uint64)
        x = (np.cumsum(step.astype(object)) % (1 << 63)).astype(np.int64) - (1 << 62)
    c, y = _roundtrip(hctx, x, "DELTA")
    assert (y == x).all()


def test_int64_extremes_all_encodings(hctx):
    mn, mx = np.iinfo(np.int64).min, np.iinfo(np.int64).max
    x = np.array([mn, mx, 0, -1, 1, mn, mx, mx, mn] * 100, dtype=np.int64)
    for enc in ("FOR", "DELTA", "DICT"):
        _, y = _roundtrip(hctx, x, enc)
        assert (y == x).all(), enc


def test_constant_blocks_cost_headers_only(hctx):
    x = np.repeat(np.arange(10, dtype=np.int64) * 1000, 256)
    c, y = _roundtrip(hctx, x, "FOR")
    assert (y == x).all()
    s = c.info()
    assert s.compressed_bytes == 10 * 8 + 11 * 4


def test_sorted_date_delta_is_small(hctx):
    from datagen import sorted_uniform
    x = sorted_uniform(1, "date", 1_000_000, 0, 2555, dtype=np.int32)
    c, y = _roundtrip(hctx, x, "AUTO")
    assert c.info().encoding == dpf.DPF_ENC_DELTA
    assert (y == x).all()
    # a sorted 2,556-value column needs at most 1 bit per row plus headers
    assert c.info().compressed_bytes < 1_000_000 / 8 + 3907 * 24


def test_dict_codes_and_values(hctx):
    vals = np.array([ord("Z"), ord("X"), ord("Y")], dtype=np.int32)
    x = vals[np.random.default_rng(3).integers(0, 3, 5000)]
    c, y = _roundtrip(hctx, x, "DICT")
    assert (y == x).all()
    s = c.info()
    assert s.ndict == 3


@pytest.mark.parametrize("chunk_rows", [256, 512, 16384, 65536, 131072])
def test_chunk_sizes(hctx, chunk_rows):
    x = np.random.default_rng(chunk_rows).integers(0, 1 << 20, 300_001).astype(np.int64)
    c, y = _roundtrip(hctx, x, "FOR", chunk_rows)
    assert (y == x).all()
    _check_dir(c, x)
    assert c.info().nchunks == -(-len(x) // chunk_rows)


def test_bad_chunk_rows(hctx):
    with pytest.raises(dpf.DpfError) as e:
        dpf.Column(hctx, np.arange(10, dtype=np.int64), "FOR", chunk_rows=1000, placement="HOST")
    assert e.value.code == dpf.DPF_ERR_INVALID_ARG


def test_strings_roundtrip(hctx):
    rng = np.random.default_rng(9)
    items = [b""] * 5 + [bytes(rng.integers(0, 256, rng.integers(0, 50)).astype(np.uint8)) for _ in range(3000)]
    items += [b"x" * 100_000, b"", b"tail"]
    s = to_strings(items)
    c = dpf.Column(hctx, s, "VARLEN", chunk_rows=512, placement="HOST")
    off, data = c.decode()
    assert (off == s.offsets).all() and (data == s.data).all()
    info = c.info()
    assert info.str_bytes == len(s.data)
    _check_dir(c, np.diff(s.offsets))


def test_empty_strings_column(hctx):
    s = to_strings([])
    c = dpf.Column(hctx, s, "VARLEN", placement="HOST")
    off, data = c.decode()
    assert list(off) == [0] and len(data) == 0


def test_generated_tables_roundtrip(hctx):
    from datagen import workloads as W
    t = W.wide_table(70_000)
    for name, col in t.items():
        enc = W.WIDE_ENCODINGS.get(name, "AUTO")
        c = dpf.Column(hctx, col, enc, placement="HOST")
        if hasattr(col, "offsets"):
            off, data = c.decode()
            assert (off == col.offsets).all() and (data == col.data).all()
        else:
            assert (c.decode() == col).all(), name


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("n", [0, 1, 256, 65536 + 999])
def test_plain_roundtrip_and_size(hctx, dtype, n):
    """PLAIN keeps every value at full width (32 or 64 bits) whatever the
    block holds: size = headers + n * width / 8, rounded up to whole mini
    blocks; values round-trip bit-exactly, extremes and constants included."""
    rng = np.random.default_rng(n + (7 if dtype == np.int64 else 0))
    info = np.iinfo(dtype)
    x = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
    if n >= 2:
        x[0], x[1] = info.min, info.max
    if n >= 256:
        x[100:200] = 5  # a constant run does not narrow the width
    c, y = _roundtrip(hctx, x, "PLAIN")
    assert y.dtype == dtype and (y == x).all()
    _check_dir(c, x)
    nmb = (n + 255) // 256
    width = 32 if dtype == np.int32 else 64
    assert c.info().compressed_bytes == nmb * 8 + (nmb + 1) * 4 + nmb * 256 * width // 8


def test_plain_rejects_strings(hctx):
    with pytest.raises(dpf.DpfError):
        dpf.Column(hctx, to_strings([b"a", b"bc"]), "PLAIN", placement="HOST")
