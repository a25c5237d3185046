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

Adjustable code widths (Sec. 2.4, closing remark: a memory-light variant stores
positions and velocities in 8 or 16 bits): a state may carry pos_bytes in {1, 2} and
vel_bytes in {1, 2} (absent: 1 and 2, the format above). With P position bytes the
offset inside a cell has 256^P steps, S = 256^P n_c and u = cell 256^P + offset; with V
velocity bytes the histogram has 2^(8V) bins over [-v_max, v_max] (half range H =
2^(8V - 1): j = clamp(floor(v H / v_max + H), 0, 2H - 1), bin centre (j - H + 1/2)
v_max / H). Multi-byte codes are little-endian in the stream, and the header's
otherwise reserved word holds P | V << 8 (0 for the paper's 1 and 2 bytes, so such
streams are unchanged).

Pins: tests/golden/stream_escape.txt is a byte stream written by hand from the
paper's description; round trips encode(decode(s)) == s and the |dx| <= q/2,
|dv| <= v_max/65536 bounds; stream length formula; hand-checked sort order; for the
other widths a hand-written stream, the same round-trip bounds with q = L / S and
v_max / 2^(8V), and the 1-byte code as the top byte of the 2-byte one.
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


def widths(state):
    """(position bytes, velocity bytes) of a state: (1, 2) unless it says otherwise."""
    return int(state.get("pos_bytes", 1)), int(state.get("vel_bytes", 2))


def pos_scale(n_c: int, pos_bytes: int = 1) -> int:
    """S = 256^P n_c position steps per box side."""
    return (256 ** pos_bytes) * n_c


def half_range(vel_bytes: int = 2) -> int:
    """H = 2^(8V - 1): half the number of velocity bins."""
    return 2 ** (8 * vel_bytes - 1)


def position_codes(x: np.ndarray, n_c: int, pos_bytes: int = 1) -> np.ndarray:
    """u = floor(x S) mod S per axis (int64), S = 256^P n_c."""
    S = pos_scale(n_c, pos_bytes)
    u = np.floor(np.asarray(x, dtype=np.float64) * S).astype(np.int64)
    return np.mod(u, S)


def velocity_codes(v32: np.ndarray, v_max: np.float32, vel_bytes: int = 2) -> np.ndarray:
    """2^(8V)-bin histogram index of each component over [-v_max, v_max]."""
    H = float(half_range(vel_bytes))
    v = np.asarray(v32, dtype=np.float32).astype(np.float64)
    if float(v_max) == 0.0:
        return np.full(v.shape, int(H), dtype=np.int64)
    C = H / np.float64(v_max)
    t = v * C
    t = t + H
    return np.clip(np.floor(t), 0, 2 * H - 1).astype(np.int64)


def decode_velocity(j: np.ndarray, v_max: np.float32, vel_bytes: int = 2) -> np.ndarray:
    """Bin centre (j - H + 1/2) * v_max / H, rounded once to float32."""
    if float(v_max) == 0.0:
        return np.zeros(np.shape(j), dtype=np.float32)
    H = float(half_range(vel_bytes))
    w = np.float64(v_max) / H
    return ((np.asarray(j, dtype=np.float64) - (H - 0.5)) * w).astype(np.float32)


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
           v_max: np.float32 | None = None, pos_bytes: int = 1, vel_bytes: int = 2):
    """Float particles -> compressed state dict (plus 'perm': stream -> input index)."""
    x32 = np.asarray(x32, dtype=np.float32)
    v32 = np.asarray(v32, dtype=np.float32)
    if v_max is None:
        v_max = np.float32(np.max(np.abs(v32))) if v32.size else np.float32(0.0)
    u = position_codes(x32, n_c, pos_bytes)
    keys = cell_keys(u >> (8 * pos_bytes), n_c, brick)
    perm = np.argsort(keys, kind="stable")
    return assemble(u[perm], velocity_codes(v32, v_max, vel_bytes)[perm], keys[perm], v_max,
                    n_c, brick, perm, pos_bytes, vel_bytes)


def assemble(u_sorted, j_sorted, keys_sorted, v_max, n_c, brick, perm=None, pos_bytes=1,
             vel_bytes=2):
    count, esc = build_counts(keys_sorted, n_c)
    st = {
        "n_c": n_c, "brick": brick,
        "count": count, "esc": esc,
        "pos": (u_sorted & (256 ** pos_bytes - 1)).astype(
            np.uint8 if pos_bytes == 1 else np.uint16),
        "vel": j_sorted.astype(np.uint16 if vel_bytes == 2 else np.uint8),
        "v_max": np.float32(v_max),
    }
    if (pos_bytes, vel_bytes) != (1, 2):
        st["pos_bytes"], st["vel_bytes"] = pos_bytes, vel_bytes
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
    pb, _ = widths(state)
    cell = key_to_cell(stream_keys(state), n_c, brick)
    u = cell * (256 ** pb) + state["pos"].astype(np.int64)
    return u, state["vel"].astype(np.int64)


def decode(state):
    """Compressed state -> float32 x, v [n][3] in stream order (bin centres)."""
    u, j = decode_codes(state)
    pb, vb = widths(state)
    S = pos_scale(state["n_c"], pb)
    x = ((u.astype(np.float64) + 0.5) / S).astype(np.float32)
    v = decode_velocity(j, state["v_max"], vb)
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
    pb, vb = widths(state)
    u = cell * (256 ** pb) + state["pos"][idx].astype(np.int64)
    S = pos_scale(n_c, pb)
    x = ((u.astype(np.float64) + 0.5) / S).astype(np.float32)
    v = decode_velocity(state["vel"][idx].astype(np.int64), np.float32(state["v_max"]), vb)
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


def width_word(pos_bytes: int, vel_bytes: int) -> int:
    """Header word of the code widths: 0 for the paper's (1, 2), else P | V << 8."""
    return 0 if (pos_bytes, vel_bytes) == (1, 2) else pos_bytes | (vel_bytes << 8)


def _le_bytes(a: np.ndarray, nbytes: int) -> np.ndarray:
    """[n][3] codes as little-endian bytes [n][3 nbytes]."""
    n = a.shape[0]
    if nbytes == 1:
        return a.astype(np.uint8).reshape(n, 3)
    return a.astype("<u2").view(np.uint8).reshape(n, 6)


def pack(state, mass: float, species_id: int) -> bytes:
    """Cell-ordered byte stream: counts with the 255 escape, then the particle records
    (3 P position bytes, then 3 V velocity bytes)."""
    full = full_counts(state)
    pos, vel = state["pos"], state["vel"]
    pb, vb = widths(state)
    rb = 3 * (pb + vb)
    parts = []
    p = 0
    for c in range(full.size):
        n = int(full[c])
        if n >= ESCAPE:
            parts.append(bytes([ESCAPE]) + struct.pack("<I", n))
        else:
            parts.append(bytes([n]))
        if n:
            rec = np.zeros((n, rb), dtype=np.uint8)
            rec[:, 0:3 * pb] = _le_bytes(pos[p:p + n], pb)
            rec[:, 3 * pb:rb] = _le_bytes(vel[p:p + n], vb)
            parts.append(rec.tobytes())
            p += n
    body = b"".join(parts)
    hdr = struct.pack("<4sIIIQQfIdQQ", MAGIC, VERSION, species_id, state["brick"],
                      int(pos.shape[0]), state["n_c"], float(state["v_max"]),
                      width_word(pb, vb), float(mass), checksum(body), len(body))
    assert len(hdr) == HEADER_BYTES
    return hdr + body


class StreamError(ValueError):
    pass


def unpack(buf: bytes):
    """Inverse of pack with the integrity checks; returns (state, mass, species_id)."""
    if len(buf) < HEADER_BYTES:
        raise StreamError("truncated header")
    (magic, ver, sid, brick, n, n_c, v_max, wword, mass, csum, blen) = struct.unpack(
        "<4sIIIQQfIdQQ", buf[:HEADER_BYTES])
    if magic != MAGIC or ver != VERSION:
        raise StreamError("bad magic/version")
    pb, vb = (1, 2) if wword == 0 else (wword & 255, wword >> 8)
    # (1, 2) is written as 0, so its explicit word is not a valid header either
    if pb not in (1, 2) or vb not in (1, 2) or wword == 0x201:
        raise StreamError("bad code widths")
    rb = 3 * (pb + vb)
    body = buf[HEADER_BYTES:]
    if len(body) != blen:
        raise StreamError("body length mismatch")
    if checksum(body) != csum:
        raise StreamError("checksum mismatch")
    ncell = n_c ** 3
    count = np.zeros(ncell, dtype=np.uint8)
    esc = []
    pos = np.zeros((n, 3), dtype=np.uint8 if pb == 1 else np.uint16)
    vel = np.zeros((n, 3), dtype=np.uint16 if vb == 2 else np.uint8)
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
        if p + k > n or off + rb * k > len(body):
            raise StreamError("count exceeds N or body")
        rec = np.frombuffer(body[off:off + rb * k], dtype=np.uint8).reshape(k, rb)
        rp, rv = rec[:, 0:3 * pb], rec[:, 3 * pb:rb]
        pos[p:p + k] = rp if pb == 1 else rp.copy().view("<u2").reshape(k, 3)
        vel[p:p + k] = rv if vb == 1 else rv.copy().view("<u2").reshape(k, 3)
        off += rb * k
        p += k
    if p != n or off != len(body):
        raise StreamError("sum of counts != N")
    st = {"n_c": n_c, "brick": brick, "count": count,
          "esc": np.array(esc, dtype=np.uint64).reshape(-1, 2),
          "pos": pos, "vel": vel, "v_max": np.float32(v_max)}
    if (pb, vb) != (1, 2):
        st["pos_bytes"], st["vel_bytes"] = pb, vb
    return st, mass, sid


def stream_length(state) -> int:
    full = full_counts(state)
    pb, vb = widths(state)
    return (HEADER_BYTES + 3 * (pb + vb) * int(full.sum()) + full.size +
            4 * int(np.sum(full >= ESCAPE)))
