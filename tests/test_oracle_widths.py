"""Pins of the oracle's adjustable code widths (Sec. 2.4, closing remark: 8- or 16-bit
positions and velocities): hand-written streams, hand-computed codes, round-trip
bounds, the 1-byte position code as the top byte of the 2-byte one, and the step with
2-byte positions moving particles that 1-byte positions freeze."""

import struct

import numpy as np
import pytest

from golden_cases import load_stream_cases
from oracle import codec, step

CASES = {c["name"]: c for c in load_stream_cases()}
WIDTHS = [(1, 2), (2, 2), (1, 1), (2, 1)]


@pytest.mark.parametrize("name", ["wide_positions_narrow_velocities", "narrow_velocities",
                                  "wide_positions"])
def test_golden_width_streams(name):
    c = CASES[name]
    pb, vb = c["widths"]
    st = codec.encode(c["x"], c["v"], c["n_c"], c["brick"], pos_bytes=pb, vel_bytes=vb)
    assert list(codec.full_counts(st)) == c["counts"]
    buf = codec.pack(st, mass=0.5, species_id=2)
    assert buf[codec.HEADER_BYTES:] == c["body"]
    assert len(buf) == codec.stream_length(st)
    word = struct.unpack("<I", buf[36:40])[0]
    assert word == pb | (vb << 8)
    back, mass, sid = codec.unpack(buf)
    assert (mass, sid) == (0.5, 2)
    for k in ("count", "pos", "vel"):
        assert np.array_equal(back[k], st[k]) and back[k].dtype == st[k].dtype
    assert codec.widths(back) == (pb, vb)


def test_velocity_codes_one_byte_hand_values():
    v = np.array([-1.0, -0.5, -1 / 256, 0.0, 1 / 128, 0.5, 0.99, 1.0, 2.0], np.float32)
    j = codec.velocity_codes(v, np.float32(1.0), vel_bytes=1)
    # floor(128 v + 128) clamped to [0, 255]
    assert j.tolist() == [0, 64, 127, 128, 129, 192, 254, 255, 255]
    d = codec.decode_velocity(np.array([0, 127, 128, 255]), np.float32(1.0), vel_bytes=1)
    assert d.tolist() == [-127.5 / 128, -0.5 / 128, 0.5 / 128, 127.5 / 128]
    assert codec.velocity_codes(v, np.float32(0.0), vel_bytes=1).tolist() == [128] * 9


def test_one_byte_code_is_the_top_byte_of_the_two_byte_code():
    rng = np.random.default_rng(1)
    x = rng.random((20000, 3)).astype(np.float32)
    x[:8] = np.float32([0.0, 0.5, 1.0 - 2 ** -24, 2 ** -20, 0.25, 0.75, 1e-30, 0.125])[:, None]
    for n_c in (1, 16, 512):
        u1 = codec.position_codes(x, n_c, 1)
        u2 = codec.position_codes(x, n_c, 2)
        assert np.array_equal(u2 >> 8, u1)


@pytest.mark.parametrize("pb,vb", WIDTHS)
def test_round_trip_bounds(pb, vb):
    rng = np.random.default_rng(2 + pb + 3 * vb)
    n_c, brick = 8, 2
    x = rng.random((5000, 3)).astype(np.float32)
    v = (rng.standard_normal((5000, 3)) * 0.7).astype(np.float32)
    st = codec.encode(x, v, n_c, brick, pos_bytes=pb, vel_bytes=vb)
    xd, vd = codec.decode(st)
    perm = st["perm"]
    S = codec.pos_scale(n_c, pb)
    dx = np.abs(xd.astype(np.float64) - x[perm].astype(np.float64))
    dx = np.minimum(dx, 1.0 - dx)
    assert np.all(dx <= 0.5 / S + 1e-7)
    assert np.max(dx) > 0.45 / S  # the bins are as wide as stated, not finer
    vmax = float(st["v_max"])
    dv = np.abs(vd.astype(np.float64) - v[perm].astype(np.float64))
    inside = np.abs(v[perm]) < vmax
    assert np.all(dv[inside] <= vmax / 2 ** (8 * vb) * (1 + 1e-6))
    # encoding the decoded particles gives back the same codes and order
    again = codec.encode(xd, vd, n_c, brick, v_max=st["v_max"], pos_bytes=pb, vel_bytes=vb)
    assert np.array_equal(again["perm"], np.arange(len(perm)))
    for k in ("count", "pos", "vel"):
        assert np.array_equal(again[k], st[k])


def test_default_widths_keep_the_paper_stream():
    # (1, 2) states carry no width keys and their header word is 0; an explicit 0x201
    # word is not accepted
    c = CASES["two_cells"]
    st = codec.encode(c["x"], c["v"], c["n_c"], c["brick"])
    assert "pos_bytes" not in st
    buf = bytearray(codec.pack(st, 0.25, 0))
    assert struct.unpack("<I", bytes(buf[36:40]))[0] == 0
    buf[36:40] = struct.pack("<I", 0x201)
    with pytest.raises(codec.StreamError):
        codec.unpack(bytes(buf))


def test_two_byte_positions_move_what_one_byte_positions_freeze():
    # a particle drifting 0.1 of a 1-byte position step per step stays put with 1-byte
    # codes (floor(0.1 + 1/2) = 0) and moves 25.6 -> 26 steps of 1/(65536 n_c) with
    # 2-byte codes, every step
    n_c = 4
    q1 = 1.0 / (256 * n_c)
    dt = 0.01
    vx = 0.1 * q1 / dt
    x = np.array([[0.3, 0.6, 0.9]], np.float32)
    v = np.array([[vx, 0.0, 0.0]], np.float32)
    for pb, moves in ((1, 0), (2, 26)):
        st = codec.encode(x, v, n_c, 1, pos_bytes=pb)
        u0, _ = codec.decode_codes(st)
        S = codec.pos_scale(n_c, pb)
        _, vd = codec.decode(st)
        u1, *_ = step.kick_codes(u0, vd, np.zeros((1, 3)), np.float32(1.0), S, 0.0, dt)
        assert (u1 - u0)[0].tolist() == [moves, 0, 0]


def test_compressed_step_with_two_byte_positions_tracks_the_float_step():
    # the compressed step with (2, 2) codes against the float step from the decoded
    # state: positions within half a 2-byte step, 256 times tighter than 1-byte codes
    rng = np.random.default_rng(3)
    n_c, n_g = 8, 16
    x = rng.random((3000, 3)).astype(np.float32)
    v = (rng.standard_normal((3000, 3)) * 0.05).astype(np.float32)
    st = codec.encode(x, v, n_c, 2, pos_bytes=2, vel_bytes=2)
    new, diag = step.step_compressed([st], [1.0 / 3000], n_g, 0.01, 0.01)
    xd, vd = codec.decode(st)
    ref, _ = step.step_float([(xd, vd, 1.0 / 3000)], n_g, 0.01, 0.01)
    x1 = ref[0][0]
    perm = diag["species"][0]["perm"]
    xn, _ = codec.decode(new[0])
    dx = np.abs(xn.astype(np.float64) - x1[perm])
    dx = np.minimum(dx, 1.0 - dx)
    S = codec.pos_scale(n_c, 2)
    assert np.all(dx <= 0.5 / S + 2e-7)
    assert codec.widths(new[0]) == (2, 2)
