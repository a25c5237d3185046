"""Oracle: the compressed phase-space format of Sec. 2.4, in plain numpy.

The paper's format: particles are bucketed into the cells of a cubic mesh of n_c^3
cells (n_c = half the neutrino lattice side) and written cell by cell in a fixed
order. For each cell, the particle count is one unsigned byte; a count of 255 or more
is written as 255 followed by the true count as a 4-byte integer (Sec. 2.4 footnote).
Each particle then takes one unsigned byte per axis for its position offset inside its
cell (precision L / (256 n_c)) and two bytes per axis for its velocity, the index of
one of 2^16 equal bins spanning [-v_max, v_max], with v_max the largest absolute
velocity of the species, kept per species in the file header.

Readings where the paper is silent (each listed in the design notes):
  * position code u = floor(x S) mod S with S = 256 n_c (exact: S is a power of two);
    cell = u >> 8, offset byte = u & 255; decoding returns the bin centre (u + 1/2)/S;
  * velocity code j = clamp(floor(v C + 32768), 0, 65535) with C = 32768 / v_max, both
    the product and the sum taken as separate IEEE float64 operations on the float32
    input; v_max = 0 gives j = 32768; decoding returns the bin centre
    (j - 32767.5) v_max / 32768 rounded once to float32;
  * v_max = max over particles and axes of |v_a| (per component);
  * cell order: bricks of B^3 cells in x-fastest order, cells x-fastest inside a brick
    (B = 1 is plain row-major); particles inside a cell keep input order;
  * byte stream: 64-byte little-endian header (magic, version, species, B, N, n_c,
    v_max, mass, checksum, body length), then every cell's count (with the escape)
    followed by its particles as x, y, z bytes and vx, vy, vz little-endian u16.

Pins: tests/golden/stream_escape.txt is a byte stream written by hand from the
paper's description; round trips encode(decode(s)) == s and the |dx| <= q/2,
|dv| <= v_max/65536 bounds; stream length formula; hand-checked sort order.
"""

from __future__ import annotations

import struct

import numpy as np

MAGIC = b"PMC1"
VERSION = 1
HEADER_BYTES = 64
ESCAPE = 255


def cell_keys(cell: np.ndarray, n_c: int, brick: int) -> np.ndarray:
    """Brick-major position in the stream of integer cell coords [n][3] (x, y, z)."""
    cell = np.asarray(cell, dtype=np.int64)
    nb = n_c // brick
    b = cell // brick
    loc = cell % brick
    bidx = (b[:, 2] * nb + b[:, 1]) * nb + b[:, 0]
    lidx = (loc[:, 2] * brick + loc[:, 1]) * brick + loc[:, 0]
    return bidx * brick ** 3 + lidx


def key_to_cell(key: np.ndarray, n_c: int, brick: int) -> np.ndarray:
    """Inverse of cell_keys: integer cell coords [n][3]."""
    key = np.asarray(key, dtype=np.int64)
    nb = n_c // brick
    b3 = brick ** 3
    bidx, lidx = key // b3, key % b3
    out = np.empty((key.shape[0], 3), dtype=np.int64)
    out[:, 0] = (bidx % nb) * brick + lidx % brick
    out[:, 1] = ((bidx // nb) % nb) * brick + (lidx // brick) % brick
    out[:, 2] = (bidx // (nb * nb)) * brick + lidx // (brick * brick)
    return out


def position_codes(x: np.ndarray, n_c: int) -> np.ndarray:
    """u = floor(x S) mod S per axis (int64), S = 256 n_c."""
    S = 256 * n_c
    u = np.floor(np.asarray(x, dtype=np.float64) * S).astype(np.int64)
    return np.mod(u, S)


def velocity_codes(v32: np.ndarray, v_max: np.float32) -> np.ndarray:
    """2^16-bin histogram index of each component over [-v_max, v_max]."""
    v = np.asarray(v32, dtype=np.float32).astype(np.float64)
    if float(v_max) == 0.0:
        return np.full(v.shape, 32768, dtype=np.int64)
    C = 32768.0 / np.float64(v_max)
    t = v * C
    t = t + 32768.0
    return np.clip(np.floor(t), 0, 65535).astype(np.int64)


def decode_velocity(j: np.ndarray, v_max: np.float32) -> np.ndarray:
    """Bin centre (j - 32767.5) * v_max / 32768, rounded once to float32."""
    if float(v_max) == 0.0:
        return np.zeros(np.shape(j), dtype=np.float32)
    w = np.float64(v_max) * 2.0 ** -15
    return ((np.asarray(j, dtype=np.float64) - 32767.5) * w).astype(np.float32)


def full_counts(state) -> np.ndarray:
    """Per-cell counts (int64, stream order) with the escapes resolved."""
    c = state["count"].astype(np.int64).copy()
    for cell, n in np.asarray(state["esc"], dtype=np.int64).reshape(-1, 2):
        c[cell] = n
    return c


def build_counts(keys_sorted: np.ndarray, n_c: int):
    """u8 count array (in stream order) plus the escape table for counts >= 255."""
    full = np.bincount(keys_sorted, minlength=n_c ** 3).astype(np.int64)
    count = np.minimum(full, ESCAPE).astype(np.uint8)
    big = np.nonzero(full >= ESCAPE)[0]
    esc = np.stack([big, full[big]], axis=1).astype(np.uint64) if big.size else \
        np.zeros((0, 2), dtype=np.uint64)
    return count, esc


def encode(x32: np.ndarray, v32: np.ndarray, n_c: int, brick: int,
           v_max: np.float32 | None = None):
    """Float particles -> compressed state dict (plus 'perm': stream -> input index)."""
    x32 = np.asarray(x32, dtype=np.float32)
    v32 = np.asarray(v32, dtype=np.float32)
    if v_max is None:
        v_max = np.float32(np.max(np.abs(v32))) if v32.size else np.float32(0.0)
    u = position_codes(x32, n_c)
    keys = cell_keys(u >> 8, n_c, brick)
    perm = np.argsort(keys, kind="stable")
    return assemble(u[perm], velocity_codes(v32, v_max)[perm], keys[perm], v_max,
                    n_c, brick, perm)


def assemble(u_sorted, j_sorted, keys_sorted, v_max, n_c, brick, perm=None):
    count, esc = build_counts(keys_sorted, n_c)
    st = {
        "n_c": n_c, "brick": brick,
        "count": count, "esc": esc,
        "pos": (u_sorted & 255).astype(np.uint8),
        "vel": j_sorted.astype(np.uint16),
        "v_max": np.float32(v_max),
    }
    if perm is not None:
        st["perm"] = perm
    return st


def stream_keys(state) -> np.ndarray:
    """Cell key of every particle in stream order."""
    full = full_counts(state)
    return np.repeat(np.arange(full.size, dtype=np.int64), full)


def decode_codes(state):
    """Integer position codes u [n][3] (int64) and velocity codes j [n][3]."""
    n_c, brick = state["n_c"], state["brick"]
    cell = key_to_cell(stream_keys(state), n_c, brick)
    u = cell * 256 + state["pos"].astype(np.int64)
    return u, state["vel"].astype(np.int64)


def decode(state):
    """Compressed state -> float32 x, v [n][3] in stream order (bin centres)."""
    u, j = decode_codes(state)
    S = 256 * state["n_c"]
    x = ((u.astype(np.float64) + 0.5) / S).astype(np.float32)
    v = decode_velocity(j, state["v_max"])
    return x, v


def cell_offsets(state) -> np.ndarray:
    """Stream offset of every cell key (int64 [n_c^3 + 1]): exclusive prefix of counts."""
    full = full_counts(state)
    off = np.zeros(full.size + 1, dtype=np.int64)
    np.cumsum(full, out=off[1:])
    return off


def decode_cells(state, keys, offsets=None):
    """Decoded (x, v) float32 and stream indices of the particles of the given cell keys
    only, with the same definitions as decode()."""
    off = cell_offsets(state) if offsets is None else offsets
    n_c, brick = state["n_c"], state["brick"]
    keys = np.asarray(keys, dtype=np.int64).reshape(-1)
    idx = np.concatenate([np.arange(off[k], off[k + 1]) for k in keys]) if keys.size else \
        np.zeros(0, dtype=np.int64)
    kk = np.repeat(keys, off[keys + 1] - off[keys])
    cell = key_to_cell(kk, n_c, brick)
    u = cell * 256 + state["pos"][idx].astype(np.int64)
    S = 256 * n_c
    x = ((u.astype(np.float64) + 0.5) / S).astype(np.float32)
    v = decode_velocity(state["vel"][idx].astype(np.int64), np.float32(state["v_max"]))
    return x, v, idx


def decoded_vmax(state) -> float:
    """Largest |decoded velocity component| (exact, float64)."""
    if state["vel"].size == 0:
        return 0.0
    _, v = decode(state)
    return float(np.max(np.abs(v.astype(np.float64))))


# ---------------------------------------------------------------- byte stream --

def checksum(body: bytes) -> int:
    """sum_i (2 i + 1) b_i mod 2^64: any single-byte change or unequal swap alters it."""
    b = np.frombuffer(body, dtype=np.uint8).astype(np.uint64)
    i = np.arange(b.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return int(np.sum((np.uint64(2) * i + np.uint64(1)) * b, dtype=np.uint64))


def pack(state, mass: float, species_id: int) -> bytes:
    """Cell-ordered byte stream: counts with the 255 escape, then 9-byte records."""
    full = full_counts(state)
    pos, vel = state["pos"], state["vel"]
    parts = []
    p = 0
    for c in range(full.size):
        n = int(full[c])
        if n >= ESCAPE:
            parts.append(bytes([ESCAPE]) + struct.pack("<I", n))
        else:
            parts.append(bytes([n]))
        if n:
            rec = np.zeros((n, 9), dtype=np.uint8)
            rec[:, 0:3] = pos[p:p + n]
            rec[:, 3:9] = vel[p:p + n].astype("<u2").view(np.uint8).reshape(n, 6)
            parts.append(rec.tobytes())
            p += n
    body = b"".join(parts)
    hdr = struct.pack("<4sIIIQQfIdQQ", MAGIC, VERSION, species_id, state["brick"],
                      int(pos.shape[0]), state["n_c"], float(state["v_max"]), 0,
                      float(mass), checksum(body), len(body))
    assert len(hdr) == HEADER_BYTES
    return hdr + body


class StreamError(ValueError):
    pass


def unpack(buf: bytes):
    """Inverse of pack with the integrity checks; returns (state, mass, species_id)."""
    if len(buf) < HEADER_BYTES:
        raise StreamError("truncated header")
    (magic, ver, sid, brick, n, n_c, v_max, _r, mass, csum, blen) = struct.unpack(
        "<4sIIIQQfIdQQ", buf[:HEADER_BYTES])
    if magic != MAGIC or ver != VERSION:
        raise StreamError("bad magic/version")
    body = buf[HEADER_BYTES:]
    if len(body) != blen:
        raise StreamError("body length mismatch")
    if checksum(body) != csum:
        raise StreamError("checksum mismatch")
    ncell = n_c ** 3
    count = np.zeros(ncell, dtype=np.uint8)
    esc = []
    pos = np.zeros((n, 3), dtype=np.uint8)
    vel = np.zeros((n, 3), dtype=np.uint16)
    off, p = 0, 0
    for c in range(ncell):
        if off >= len(body):
            raise StreamError("truncated body")
        k = body[off]
        off += 1
        if k == ESCAPE:
            (k,) = struct.unpack("<I", body[off:off + 4])
            off += 4
            esc.append((c, k))
        count[c] = min(k, ESCAPE)
        if p + k > n or off + 9 * k > len(body):
            raise StreamError("count exceeds N or body")
        rec = np.frombuffer(body[off:off + 9 * k], dtype=np.uint8).reshape(k, 9)
        pos[p:p + k] = rec[:, 0:3]
        vel[p:p + k] = rec[:, 3:9].copy().view("<u2").reshape(k, 3)
        off += 9 * k
        p += k
    if p != n or off != len(body):
        raise StreamError("sum of counts != N")
    st = {"n_c": n_c, "brick": brick, "count": count,
          "esc": np.array(esc, dtype=np.uint64).reshape(-1, 2),
          "pos": pos, "vel": vel, "v_max": np.float32(v_max)}
    return st, mass, sid


def stream_length(state) -> int:
    full = full_counts(state)
    return HEADER_BYTES + 9 * int(full.sum()) + full.size + 4 * int(np.sum(full >= ESCAPE))
