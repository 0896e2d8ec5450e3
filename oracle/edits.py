"""Edit stream: the storage the correction adds to a lossy-compressed field
(Sec. V-D counts it as the method's storage overhead; the paper fixes no
format, so this one is this project's reading).

TEST INFRASTRUCTURE ONLY (the oracle of the GPU encoder and decoder): only
tests, the smoke check and the benchmark's CPU-baseline leg use it.  It shares
no code with the GPU library.

Stream = header, chunk table, payload (all little-endian):
  header   'PMSE', u8 version (1), u8 dtype (0 binary32, 1 binary64),
           u16 0, u64 vertices, u64 edits, u64 payload bytes, u32 chunk
           (entries per chunk, 4096), u32 chunks
  table    per chunk: u64 payload offset of its first entry, u64 index of the
           edited vertex before it (2^64 - 1 when none)
  payload  per vertex i whose value changed, in ascending i:
           gap   = i - previous edited index - 1 (previous = -1 at the start)
           steps = key(fhat_i) - key(g_i) >= 1
           each as unsigned LEB128 (7 bits per byte, low groups first, top bit
           set on every byte but the last); key() maps a value to an integer
           in value order, so steps counts the representable values in
           (g_i, fhat_i].
"""
import struct

import numpy as np

CHUNK = 4096
MAGIC = b"PMSE"
NONE = (1 << 64) - 1


def keys(a):
    """Order-preserving integer keys of a float array (uint64)."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.float32:
        b = a.view(np.uint32).astype(np.uint64)
        sign = np.uint64(1 << 31)
        full = np.uint64((1 << 32) - 1)
    else:
        b = a.view(np.uint64).copy()
        sign = np.uint64(1 << 63)
        full = np.uint64((1 << 64) - 1)
    neg = (b & sign) != 0
    return np.where(neg, full ^ b, b | sign)


def from_keys(k, dtype):
    if dtype == np.float32:
        sign = np.uint64(1 << 31)
        full = np.uint64((1 << 32) - 1)
        b = np.where((k & sign) != 0, k ^ sign, full ^ k).astype(np.uint32)
        return b.view(np.float32)
    sign = np.uint64(1 << 63)
    full = np.uint64((1 << 64) - 1)
    b = np.where((k & sign) != 0, k ^ sign, full ^ k).astype(np.uint64)
    return b.view(np.float64)


def leb128(v):
    out = bytearray()
    v = int(v)
    while True:
        byte = v & 0x7F
        v >>= 7
        if v:
            out.append(byte | 0x80)
        else:
            out.append(byte)
            return bytes(out)


def encode(fhat, g):
    """Stream of the vertices where g's bits differ from fhat's."""
    fhat = np.ascontiguousarray(fhat).reshape(-1)
    g = np.ascontiguousarray(g).reshape(-1)
    assert fhat.dtype == g.dtype and fhat.size == g.size
    word = np.uint32 if g.dtype == np.float32 else np.uint64
    changed = np.flatnonzero(fhat.view(word) != g.view(word))
    steps = keys(fhat[changed]) - keys(g[changed])
    payload = bytearray()
    table = []
    prev = -1
    for n, (i, st) in enumerate(zip(changed.tolist(), steps.tolist())):
        if n % CHUNK == 0:
            table.append((len(payload), NONE if prev < 0 else prev))
        assert st >= 1
        payload += leb128(i - prev - 1)
        payload += leb128(st)
        prev = i
    dt = 0 if g.dtype == np.float32 else 1
    head = MAGIC + struct.pack("<BBHQQQII", 1, dt, 0, g.size, changed.size, len(payload), CHUNK,
                               len(table))
    body = b"".join(struct.pack("<QQ", o, p) for o, p in table)
    return head + body + bytes(payload)


def parse_header(stream):
    assert stream[:4] == MAGIC
    ver, dt, _, nv, ne, nb, chunk, nch = struct.unpack_from("<BBHQQQII", stream, 4)
    return {"version": ver, "dtype": dt, "vertices": nv, "edits": ne, "payload_bytes": nb,
            "chunk": chunk, "chunks": nch,
            "header_bytes": 4 + struct.calcsize("<BBHQQQII") + 16 * nch}


def decode(fhat, stream):
    """g from fhat and an edit stream."""
    h = parse_header(stream)
    fhat = np.ascontiguousarray(fhat)
    g = fhat.reshape(-1).copy()
    pos = h["header_bytes"]
    prev = -1
    idx, steps = [], []
    for _ in range(h["edits"]):
        vals = []
        for _k in range(2):
            v, shift = 0, 0
            while True:
                b = stream[pos]
                pos += 1
                v |= (b & 0x7F) << shift
                shift += 7
                if not b & 0x80:
                    break
            vals.append(v)
        i = prev + 1 + vals[0]
        idx.append(i)
        steps.append(vals[1])
        prev = i
    if idx:
        idx = np.asarray(idx, dtype=np.int64)
        k = keys(g[idx]) - np.asarray(steps, dtype=np.uint64)
        g[idx] = from_keys(k, g.dtype.type)
    return g.reshape(fhat.shape)
