"""Pins of the oracle's compressed format and compressed step (CPU only)."""

import struct

import numpy as np
import pytest

from golden_cases import load_stream_cases
from oracle import codec, mesh, step

CASES = {c["name"]: c for c in load_stream_cases()}


def _encode_case(c):
    return codec.encode(c["x"], c["v"], c["n_c"], c["brick"])


def test_golden_two_cells_stream_bytes():
    c = CASES["two_cells"]
    st = _encode_case(c)
    assert list(codec.full_counts(st)) == c["counts"]
    buf = codec.pack(st, mass=0.25, species_id=0)
    assert buf[codec.HEADER_BYTES:] == c["body"]
    magic, ver, sid, brick, n, n_c, v_max = struct.unpack("<4sIIIQQf", buf[:36])
    assert (magic, ver, sid, brick, n, n_c, v_max) == (b"PMC1", 1, 0, 1, 4, 2, 2.0)


def test_golden_escape_stream_bytes():
    c = CASES["escape_300"]
    st = _encode_case(c)
    assert st["count"][0] == 255 and st["esc"].tolist() == [[0, 300]]
    buf = codec.pack(st, mass=1.0, species_id=1)
    body = buf[codec.HEADER_BYTES:]
    assert body == c["body_prefix"] + c["record"] * 300
    assert len(buf) == codec.stream_length(st)


def test_golden_brick_order_keys():
    c = CASES["bricks_of_two"]
    u = codec.position_codes(c["x"], c["n_c"])
    keys = codec.cell_keys(u >> 8, c["n_c"], c["brick"])
    assert keys.tolist() == c["keys"]
    assert np.array_equal(codec.key_to_cell(keys, c["n_c"], c["brick"]), u >> 8)


def test_checksum_small_example():
    # sum (2i+1) b_i: 1*1 + 3*2 + 5*255 = 1282
    assert codec.checksum(bytes([1, 2, 255])) == 1282
    assert codec.checksum(b"") == 0


def _random_state(rng, n, n_c, brick, clump=0):
    x = rng.random((n, 3)).astype(np.float32)
    if clump:
        x[:clump] = np.float32(0.3)  # one cell with many particles (escape)
    x[x >= 1] = 0
    v = (rng.standard_normal((n, 3)) * 0.7).astype(np.float32)
    return x, v


@pytest.mark.parametrize("n,n_c,brick,clump", [(500, 4, 1, 0), (2000, 8, 2, 300),
                                                (3000, 8, 4, 600), (0, 4, 2, 0)])
def test_round_trips(n, n_c, brick, clump):
    rng = np.random.default_rng(n + n_c)
    x, v = _random_state(rng, n, n_c, brick, clump)
    st = codec.encode(x, v, n_c, brick)
    xd, vd = codec.decode(st)
    perm = st["perm"]
    q = 1.0 / (256 * n_c)
    if n:
        dx = np.abs(xd.astype(np.float64) - x[perm].astype(np.float64))
        dx = np.minimum(dx, 1.0 - dx)
        assert dx.max() <= q / 2 * (1 + 1e-12)
        # half a bin, plus the final rounding of the bin centre to float32
        err = np.abs(vd.astype(np.float64) - v[perm])
        assert np.all(err <= float(st["v_max"]) / 65536 + 2.0 ** -24 * np.abs(vd))
    # encode(decode(s)) == s byte for byte (same v_max)
    st2 = codec.encode(xd, vd, n_c, brick, v_max=st["v_max"])
    for k in ("count", "esc", "pos", "vel"):
        assert np.array_equal(st[k], st2[k]), k
    assert np.array_equal(st2["perm"], np.arange(n))
    buf = codec.pack(st, 0.5, 3)
    assert len(buf) == codec.stream_length(st)
    st3, mass, sid = codec.unpack(buf)
    assert (mass, sid) == (0.5, 3)
    for k in ("count", "esc", "pos", "vel", "v_max"):
        assert np.array_equal(st[k], st3[k]), k


def test_edge_codes():
    n_c = 2
    S = 256 * n_c
    x = np.array([[0.0, 1.0 - 2 ** -24, -1e-9], [1.0, 0.5, 0.25]], dtype=np.float32)
    u = codec.position_codes(x, n_c)
    assert u.tolist() == [[0, S - 1, S - 1], [0, S // 2, S // 4]]
    vm = np.float32(3.0)
    j = codec.velocity_codes(np.array([3.0, -3.0, 0.0, 2.9999998], np.float32), vm)
    assert j.tolist() == [65535, 0, 32768, 65535]
    assert codec.velocity_codes(np.array([0.0, 1.0], np.float32), np.float32(0)).tolist() \
        == [32768, 32768]
    assert codec.decode_velocity(np.array([32768]), np.float32(0)).tolist() == [0.0]


def test_stream_corruption_detected():
    rng = np.random.default_rng(9)
    x, v = _random_state(rng, 300, 4, 2, 0)
    st = codec.encode(x, v, 4, 2)
    buf = bytearray(codec.pack(st, 1.0, 0))
    with pytest.raises(codec.StreamError):
        codec.unpack(bytes(buf[:-1]))  # truncated
    bad = bytearray(buf)
    bad[codec.HEADER_BYTES + 10] ^= 0x01
    with pytest.raises(codec.StreamError):
        codec.unpack(bytes(bad))
    bad = bytearray(buf)
    bad[0] = ord("X")
    with pytest.raises(codec.StreamError):
        codec.unpack(bytes(bad))


# -------------------------------------------------------------- compressed step --

def _insertion_sort_perm(keys):
    """Pure-Python stable insertion sort: new index -> old index."""
    order = []
    for i, k in enumerate(keys):
        j = len(order)
        while j > 0 and keys[order[j - 1]] > k:
            j -= 1
        order.insert(j, i)
    return order


def test_compressed_step_properties():
    rng = np.random.default_rng(21)
    n_c, brick, n_g = 8, 2, 16
    S = 256 * n_c
    xc, vc = _random_state(rng, 400, n_c, brick)
    xn, vn = _random_state(rng, 900, n_c, brick)
    vn *= 20
    states = [codec.encode(xc, vc, n_c, brick), codec.encode(xn, vn, n_c, brick)]
    masses = [1.0 / 400, 0.01 / 900]
    dt = 0.01
    new, diag = step.step_compressed(states, masses, n_g, dt, dt)
    # the float step from the decoded state, re-encoded, must agree with the codes
    dec = [codec.decode(s) for s in states]
    out, fdiag = step.step_float([(x, v, m) for (x, v), m in zip(dec, masses)], n_g, dt, dt)
    assert abs(diag["a_max"] - np.max(np.abs(fdiag["a_mesh"]))) == 0
    for s, ns, d, (x1, v1), (x0, v0) in zip(states, new, diag["species"], out, dec):
        perm = d["perm"]
        xd, vd = codec.decode(ns)
        # positions: within half a position quantum of the float drift (mod 1)
        dx = np.abs(xd.astype(np.float64) - x1[perm])
        dx = np.minimum(dx, 1.0 - dx)
        assert dx.max() <= 0.5 / S * (1 + 1e-9)
        # velocities: within half a bin of the float kick, v_max' a power of two
        vmn = float(ns["v_max"])
        assert vmn > 0 and np.frexp(vmn)[0] == 0.5
        assert np.max(np.abs(v1)) <= vmn
        bound = np.max(np.abs(v0.astype(np.float64))) + dt * diag["a_max"]
        assert vmn / 2 < bound <= vmn
        err = np.abs(vd.astype(np.float64) - v1[perm])
        assert np.all(err <= vmn / 65536 + 2.0 ** -24 * np.abs(vd))
        # stream sorted by cell key, stable in old stream order
        keys_old = codec.cell_keys(d["u_new"] >> 8, n_c, brick).tolist()
        assert perm.tolist() == _insertion_sort_perm(keys_old)


def test_frozen_particles_do_not_move():
    # |v c_d S| < 1/2: the fixed-point drift rounds the displacement to zero
    n_c, brick, n_g = 4, 1, 8
    S = 256 * n_c
    x = np.array([[0.1, 0.2, 0.3], [0.6, 0.7, 0.8]], np.float32)
    v = np.array([[0.1, -0.1, 0.0], [0.0, 0.0, 0.0]], np.float32) * np.float32(0.4 / S / 0.01 / 0.1)
    st = codec.encode(x, v, n_c, brick)
    new, _ = step.step_compressed([st], [1e-12], n_g, 0.0, 0.01)
    assert np.array_equal(new[0]["pos"], st["pos"])
    assert np.array_equal(new[0]["count"], st["count"])


def test_float_step_single_particle_free_drift():
    # with negligible mass there is no force: x' = x + dt v exactly (mod 1)
    x = np.array([[0.95, 0.5, 0.01]])
    v = np.array([[10.0, -3.0, -2.0]])
    (out,), _ = step.step_float([(x, v, 0.0)], 8, 0.01, 0.01)
    assert np.allclose(out[0], np.mod(x + 0.01 * v, 1.0), atol=1e-15)
    assert np.allclose(out[1], v)


def test_decode_cells_matches_full_decode():
    rng = np.random.default_rng(9)
    x0, v0 = _random_state(rng, 2000, 8, 4, clump=300)
    st = codec.encode(x0, v0, 8, 4)
    x, v = codec.decode(st)
    keys = rng.choice(8 ** 3, size=40, replace=False)
    xs, vs, idx = codec.decode_cells(st, keys)
    assert np.array_equal(xs, x[idx]) and np.array_equal(vs, v[idx])
    sk = codec.stream_keys(st)
    assert np.array_equal(np.sort(idx), np.flatnonzero(np.isin(sk, keys)))
