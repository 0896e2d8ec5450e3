"""Pins of the edit-stream oracle (oracle/edits.py): the LEB128 varint and the
order-preserving keys against their definitions, a hand-written stream, and
exact round trips."""
import struct

import numpy as np
import pytest

from oracle import edits


@pytest.mark.parametrize("v,b", [(0, b"\x00"), (1, b"\x01"), (127, b"\x7f"), (128, b"\x80\x01"),
                                 (300, b"\xac\x02"), (16383, b"\xff\x7f"),
                                 (16384, b"\x80\x80\x01"), ((1 << 32) - 1, b"\xff\xff\xff\xff\x0f")])
def test_leb128_encoding(v, b):
    assert edits.leb128(v) == b


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_keys_count_representable_values(dtype):
    """key(b) - key(a) is the number of steps of nextafter from a up to b."""
    rng = np.random.default_rng(3)
    vals = np.concatenate([rng.standard_normal(50), [0.0, -0.0, 1e-40, -1e-40, 1.0, -1.0]]).astype(dtype)
    for a in vals[:20]:
        b = a
        for steps in range(1, 40):
            b = np.nextafter(b, dtype(np.inf))
            d = edits.keys(np.array([b], dtype)) - edits.keys(np.array([a], dtype))
            assert int(d[0]) == steps
    k = edits.keys(vals)
    # strictly larger values have strictly larger keys (-0 and +0 are equal
    # values with adjacent keys)
    for i in range(vals.size):
        for j in range(vals.size):
            if vals[i] < vals[j]:
                assert k[i] < k[j]
    back = edits.from_keys(k, dtype)
    assert np.array_equal(back.view(np.uint8), vals.view(np.uint8))


def test_hand_written_stream():
    fhat = np.array([1.0, 2.0, 3.0], np.float32)
    g = fhat.copy()
    g[1] = np.nextafter(np.float32(2.0), np.float32(0))
    g[2] = np.nextafter(np.nextafter(np.float32(3.0), np.float32(0)), np.float32(0))
    expect = (b"PMSE" + bytes([1, 0, 0, 0]) + struct.pack("<QQQII", 3, 2, 4, 4096, 1) +
              struct.pack("<QQ", 0, (1 << 64) - 1) + bytes([1, 1, 0, 2]))
    s = edits.encode(fhat, g)
    assert s == expect
    assert np.array_equal(edits.decode(fhat, s), g)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("frac", [0.0, 0.01, 0.5])
def test_round_trip(dtype, frac):
    rng = np.random.default_rng(11)
    fhat = (rng.standard_normal(20000) * 10).astype(dtype)
    g = fhat.copy()
    m = rng.uniform(size=g.size) < frac
    g[m] = (g[m].astype(np.float64) - rng.uniform(0, 1e-3, m.sum())).astype(dtype)
    g = np.minimum(g, fhat)
    s = edits.encode(fhat, g)
    h = edits.parse_header(s)
    assert h["edits"] == int(np.count_nonzero(g != fhat))
    assert h["chunks"] == (h["edits"] + edits.CHUNK - 1) // edits.CHUNK
    assert len(s) == h["header_bytes"] + h["payload_bytes"]
    assert np.array_equal(edits.decode(fhat, s).view(np.uint8), g.view(np.uint8))


def test_chunk_table_points_at_entries():
    fhat = np.arange(30000, dtype=np.float64)
    g = fhat.copy()
    g[::3] = np.nextafter(g[::3], -np.inf)
    s = edits.encode(fhat, g)
    h = edits.parse_header(s)
    assert h["chunks"] == 3
    base = 4 + struct.calcsize("<BBHQQQII")
    for c in range(h["chunks"]):
        off, prev = struct.unpack_from("<QQ", s, base + 16 * c)
        first = 3 * edits.CHUNK * c
        expect_prev = (1 << 64) - 1 if c == 0 else first - 3
        assert prev == expect_prev
        # the entry at `off` is the gap before vertex `first`
        gap = s[h["header_bytes"] + off]
        assert gap == (0 if c == 0 else 2)
