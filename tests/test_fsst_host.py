"""FSST string columns on the host (no GPU): decode(encode(x)) == x bit-exactly
(paper Sections 3.4.2 and 4.1: a static table of at most 255 symbols per
chunk, every record decodable on its own), for text, arbitrary bytes (escape
codes), empty strings, an empty column, strings longer than the sample cut
and chunk tails; the code heap never exceeds twice the raw bytes (one escape
pair per byte is the worst case) and stays below the raw bytes for the text
of the string workloads; zone maps hold the decoded lengths."""
import numpy as np
import pytest

from paper_2605_10511_amd import dpf
from tests.conftest import to_strings


@pytest.fixture(scope="module")
def hctx():
    return dpf.Context(-1)


def _col(ctx, s, chunk_rows=65536, enc="FSST"):
    return dpf.Column(ctx, s, enc, chunk_rows=chunk_rows, placement="HOST", threads=4)


def _check(c, s):
    off, data = c.decode()
    assert (off == s.offsets).all() and (data == s.data).all()
    info = c.info()
    assert info.encoding == dpf.DPF_ENC_FSST
    assert info.str_bytes == len(s.data)
    lens = np.diff(s.offsets)
    start = 0
    for k in range(info.nchunks):
        ch = c.chunk(k)
        assert ch.row_start == start
        seg = lens[ch.row_start:ch.row_start + ch.nrows]
        if len(seg):
            assert ch.min == int(seg.min()) and ch.max == int(seg.max())
        start += ch.nrows
    assert start == info.nrows


def _code_bytes(c):
    """Code heap bytes: compressed size less the headers and tables."""
    info = c.info()
    nmb, nchunks = info.nminiblocks, info.nchunks
    return c, info.compressed_bytes - nmb * 8 - (nmb + 1) * 4 - (nmb + 1) * 8 - nchunks * 2304


def test_mixed_bytes_roundtrip(hctx):
    rng = np.random.default_rng(9)
    items = [b""] * 5 + [bytes(rng.integers(0, 256, rng.integers(0, 50)).astype(np.uint8)) for _ in range(3000)]
    items += [b"x" * 100_000, b"", b"tail", bytes(range(256)) * 3]
    s = to_strings(items)
    _check(_col(hctx, s, chunk_rows=512), s)


def test_empty_column_and_all_empty_strings(hctx):
    s = to_strings([])
    c = _col(hctx, s)
    off, data = c.decode()
    assert list(off) == [0] and len(data) == 0
    s = to_strings([b""] * 1000)
    _check(_col(hctx, s, chunk_rows=256), s)


@pytest.mark.parametrize("n", [1, 255, 256, 257, 70_001])
def test_comment_text_compresses(hctx, n):
    from datagen import workloads as W
    t = W.wide_table(n, seed=2)
    s = t["comment"]
    c = _col(hctx, s)
    _check(c, s)
    v = dpf.Column(hctx, s, "VARLEN", placement="HOST")
    _, code = _code_bytes(c)
    if n > 10_000:
        assert code < 0.8 * len(s.data), (code, len(s.data))
        assert c.info().compressed_bytes < v.info().compressed_bytes


def test_escapes_outside_the_sample(hctx):
    """Bytes that the chunk's sample never shows are escaped (code 255 then
    the byte) and still decode exactly."""
    rng = np.random.default_rng(3)
    letters = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz ", dtype=np.uint8)
    items = []
    for r in range(65536 + 300):
        b = letters[rng.integers(0, len(letters), rng.integers(10, 44))].tobytes()
        if r % 997 == 5:
            b = b[:3] + bytes([0xF0 + r % 16, 0]) + b[3:]
        items.append(b)
    s = to_strings(items)
    c = _col(hctx, s)
    _check(c, s)
    _, code = _code_bytes(c)
    assert code <= 2 * len(s.data)


def test_random_bytes_worst_case(hctx):
    rng = np.random.default_rng(4)
    s = to_strings([bytes(rng.integers(0, 256, 64).astype(np.uint8)) for _ in range(5000)])
    c = _col(hctx, s, chunk_rows=1024)
    _check(c, s)
    _, code = _code_bytes(c)
    assert code <= 2 * len(s.data)


def test_long_strings_past_the_sample_cut(hctx):
    rng = np.random.default_rng(5)
    base = b"the quick brown fox jumps over the lazy dog "
    items = [base * int(rng.integers(100, 300)) for _ in range(40)] + [b"z"]
    s = to_strings(items)
    c = _col(hctx, s, chunk_rows=256)
    _check(c, s)
    _, code = _code_bytes(c)
    assert code < len(s.data) / 3  # the repeated sentence is a handful of 8-byte symbols


def test_fsst_is_for_strings(hctx):
    with pytest.raises(dpf.DpfError):
        dpf.Column(hctx, np.arange(10, dtype=np.int64), "FSST", placement="HOST")
