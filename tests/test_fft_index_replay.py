"""CPU replay of the index arithmetic of the HIP FFT passes (no GPU, no library call).

The column passes (k_col_fft, k_col_zconv) give a workgroup W adjacent lines of N points
(from 2048 points on, each line as its even and odd halves on two thread groups);
thread (c, t) = (tid % W, tid / W) holds points t + T n1 of line c in registers, moves them
through a per-line LDS tile for the four-step exchange, and writes the result in the
transposed order k = (t + T v) + E k2. The row passes pair X[k] with X[M - k] by lane
shuffles. This module restates those formulas (Plan, col_cs, col_w, the z-blocked spectrum
layout, the Lines descriptors) and checks, for every mesh size and for the column widths
W = 1..16 that fit, what the kernels rely on:
  * every global read and write of a workgroup lies in the buffer, the per-thread 32-bit
    offsets do not wrap, and the 64-bit uniform base plus offset addresses the intended
    element of the intended line;
  * each line's N points are read once and written once, lines of one launch are
    disjoint and cover the buffer (exhaustively up to 128^3, on sampled workgroups above);
  * each LDS exchange phase writes every word of a line's tile once, reads only words
    written in that phase, and stays inside the line's padded column (no column overlaps
    another) and inside the workgroup's allocation;
  * the twiddle staging loop fills stw[0..N) exactly;
  * the row-pass shuffle partner of every lane is in the same wave and holds X[M - k].
"""

import numpy as np
import pytest


def ilog2(n):
    return n.bit_length() - 1


def plan(N):
    LG = ilog2(N)
    T = 1 << (LG // 2)
    E = N // T
    return T, E, E // T, T + 1


def line_plan(N):
    """(H, NH, T, E, V, TP): H thread groups of T threads per line, each group running
    the four-step plan of NH = N / H points (H = 2 from 2048 points on)."""
    H = 2 if N >= 2048 else 1
    NH = N // H
    T, E, V, TP = plan(NH)
    return H, NH, T, E, V, TP


def cmod(a, b):  # C++ remainder (sign of the dividend)
    r = abs(a) % b
    return -r if a < 0 else r


def col_cs(W, per_col):
    want = 32 // W
    r = per_col % 32
    return per_col + (cmod(want - r, 32) + 32) % 32


def col_w(N):
    w = 16384 // N
    w = min(w, 16, N // 2)
    return max(w, 1)


def zblk(n):
    if n >= 2048:
        return 64
    t = 1 << (ilog2(n) // 2)
    return min(t, 16)


def lines(kind, n):
    """(s1, s2h, s2l, sh2, es, esl, L1, L2) of the Lines descriptors in complex units."""
    M, ZB = n // 2, zblk(n)
    if kind == "y_main":   # l1 = kx, l2 = z, element = y
        return (1, n * ZB * M, M, ilog2(ZB), ZB * M, 0, M, n)
    if kind == "y_nyq":    # l1 = z, element = y
        return (n, 0, 0, 0, 1, 0, n, 1)
    if kind == "z_main":   # l1 = kx, l2 = y, element = z (blocked)
        return (1, ZB * M, 0, 0, n * ZB * M, M, M, n)
    if kind == "z_nyq":    # l1 = y, element = z
        return (1, 0, 0, 0, n, 0, n, 1)
    raise ValueError(kind)


def spectrum_index(kx, y, z, n):
    M, ZB = n // 2, zblk(n)
    return ((z // ZB) * n + y) * ZB * M + (z % ZB) * M + kx


def line_element(kind, n, l1, l2, e):
    """Address of element e of line (l1, l2) from the layout's definition."""
    if kind == "y_main":
        return spectrum_index(l1, e, l2, n)
    if kind == "z_main":
        return spectrum_index(l1, l2, e, n)
    if kind == "y_nyq":   # nyq[z][y]
        return l1 * n + e
    return e * n + l1     # z_nyq: nyq[z][y], l1 = y


def line_base(d, l1, l2):
    s1, s2h, s2l, sh2 = d[:4]
    return l1 * s1 + (l2 >> sh2) * s2h + (l2 & ((1 << sh2) - 1)) * s2l


def block_addresses(kind, n, W, bx, by, zpass):
    """Addresses read for element e by thread (c, tl = (t, h)), as the kernel computes
    them: [W][H T][E] arrays of (address, 32-bit offset, line l1, element e)."""
    H, NH, T, E, V, TP = line_plan(n)
    d = lines(kind, n)
    s1, es, esl = d[0], d[4], d[5]
    ubase = line_base(d, bx * W, by)
    c = np.arange(W)[:, None, None]
    tl = np.arange(H * T)[None, :, None]
    t, h = tl % T, tl // T
    n1 = np.arange(E)[None, None, :]
    e0 = H * t + h
    blk = zpass and kind == "z_main"
    if blk:
        ZB = zblk(n)
        LZB = ilog2(ZB)
        toff = c * s1 + (e0 >> LZB) * es + (e0 & (ZB - 1)) * esl
        step = ((H * T) >> LZB) * es
        addr = ubase + n1 * step + toff
    elif zpass:
        toff = c * s1 + e0 * es
        addr = ubase + n1 * (H * T * es) + toff
    else:
        toff = c * s1 + e0 * es
        addr = ubase + H * T * n1 * es + toff
    e = e0 + H * T * n1
    return addr, toff, bx * W + c + 0 * n1, e + 0 * c


def write_addresses(kind, n, W, bx, by, zpass):
    """Addresses written for output point k = (t + T v) + E k2 (column passes) or point
    t + T n1 (the z pass writes back in natural order)."""
    H, NH, T, E, V, TP = line_plan(n)
    if zpass:
        return block_addresses(kind, n, W, bx, by, zpass)
    d = lines(kind, n)
    s1, es = d[0], d[4]
    ubase = line_base(d, bx * W, by)
    c = np.arange(W)[:, None, None, None]
    tl = np.arange(H * T)[None, :, None, None]
    t, h = tl % T, tl // T
    v = np.arange(V)[None, None, :, None]
    k2 = np.arange(T)[None, None, None, :]
    shp = (W, H * T, V, T)
    off = np.broadcast_to(c * s1 + ((t + T * v) + h * NH) * es, shp)
    addr = ubase + E * k2 * es + off
    k = np.broadcast_to((t + T * v) + E * k2 + h * NH, shp)
    l1 = np.broadcast_to(bx * W + c, shp)
    r = (W, H * T, V * T)
    return addr.reshape(r), off.reshape(r), l1.reshape(r), k.reshape(r)


SIZES = [8, 16, 32, 64, 128, 256, 512, 1024, 2048]
LDS_MAX = 160 * 1024  # bytes of LDS one gfx950 workgroup may allocate


def widths(n):
    ws = {col_w(n)}
    for w in (1, 2, 4, 8, 16):
        H, NH, T, E, V, TP = line_plan(n)
        lds = w * col_cs(w, H * E * TP) * 4 + 8 * n  # exchange tiles + staged twiddles
        if w <= n // 2 and lds <= LDS_MAX:
            ws.add(w)
    return sorted(ws)


@pytest.mark.parametrize("n", SIZES)
def test_plan_and_lds_tiles(n):
    H, NH, T, E, V, TP = line_plan(n)
    assert H * T * E == n and V in (1, 2) and E % T == 0
    ZB = zblk(n)
    assert (H * T) % ZB == 0 and (H == 2 or E % ZB == 0)
    for W in widths(n):
        CS = col_cs(W, H * E * TP)
        assert CS >= H * E * TP
        nthreads = W * H * T
        assert nthreads <= 1024
        # the twiddle staging loop: i = tid, tid + W H T, ... < N fills stw once
        filled = np.zeros(n, dtype=np.int64)
        for tid in range(nthreads):
            filled[np.arange(tid, n, nthreads)] += 1
        assert np.all(filled == 1)
        # LDS exchange phases of nat_to_tr and tr_to_nat on each half's region
        t = np.arange(T)
        wr_nat = (np.arange(E)[:, None] * TP + t[None, :]).ravel()           # lds[k1 TP + t]
        rd_nat = ((t[:, None, None] + T * np.arange(V)[None, :, None]) * TP
                  + np.arange(T)[None, None, :]).ravel()                      # lds[(t+Tv)TP+k2]
        for wr, rd in ((wr_nat, rd_nat), (rd_nat, wr_nat)):  # tr_to_nat swaps the roles
            assert np.unique(wr).size == wr.size == E * T   # each word written once
            assert set(rd.tolist()) <= set(wr.tolist())      # reads only what was written
            assert wr.max() < E * TP and wr.min() >= 0       # inside the half's region
        if H == 2:
            # the radix-2 step: half h writes its region at q TP + t (q < E), reads the
            # other half's at the same place; the two regions do not overlap
            q = np.arange(E)[:, None]
            reg = [(hh * E * TP + q * TP + t[None, :]).ravel() for hh in (0, 1)]
            assert not set(reg[0].tolist()) & set(reg[1].tolist())
            assert max(r.max() for r in reg) < H * E * TP <= CS
            # every frequency k < N/2 is held once per half: (t + T v) + E k2
            kk = ((t[:, None, None] + T * np.arange(V)[None, :, None]) +
                  E * np.arange(T)[None, None, :]).ravel()
            assert np.array_equal(np.sort(kk), np.arange(NH))
        assert W * CS * 4 + 8 * n <= LDS_MAX


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["y_main", "y_nyq", "z_main", "z_nyq"])
def test_column_pass_addresses(n, kind):
    T, E, V, TP = plan(n)
    d = lines(kind, n)
    L1, L2 = d[6], d[7]
    size = n * n * (n // 2) if kind.endswith("main") else n * n
    for W in widths(n):
        if L1 % W:
            continue  # rejected on the host (PM_ERR_SHAPE)
        nbx = L1 // W
        if size <= 128 ** 3:
            blocks = [(bx, by) for bx in range(nbx) for by in range(L2)]
        else:
            rng = np.random.default_rng(n + W)
            blocks = [(0, 0), (nbx - 1, L2 - 1)] + [
                (int(rng.integers(nbx)), int(rng.integers(L2))) for _ in range(12)]
        # the y lines go through k_col_fft, the z lines through k_col_zconv
        for zpass in ((True,) if kind.startswith("z") else (False,)):
            seen_rd = np.zeros(size, dtype=np.int8) if size <= 128 ** 3 else None
            seen_wr = np.zeros(size, dtype=np.int8) if size <= 128 ** 3 else None
            for bx, by in blocks:
                addr, off, l1, e = block_addresses(kind, n, W, bx, by, zpass)
                assert off.max() < 2 ** 32 and off.min() >= 0      # 32-bit offsets
                assert addr.min() >= 0 and addr.max() < size        # in the buffer
                want = line_element(kind, n, l1, by, e)
                assert np.array_equal(addr, want)
                # each line's N points read once
                for c in range(W):
                    assert np.array_equal(np.sort(e[c].ravel()), np.arange(n))
                waddr, woff, wl1, k = write_addresses(kind, n, W, bx, by, zpass)
                assert woff.max() < 2 ** 32 and woff.min() >= 0
                wwant = line_element(kind, n, wl1, by, k)
                assert np.array_equal(waddr, wwant)
                for c in range(W):
                    assert np.array_equal(np.sort(k[c].ravel()), np.arange(n))
                # in-place passes: a workgroup writes only what it read
                assert set(waddr.ravel().tolist()) == set(addr.ravel().tolist())
                if seen_rd is not None:
                    np.add.at(seen_rd, addr.ravel(), 1)
                    np.add.at(seen_wr, waddr.ravel(), 1)
            if seen_rd is not None:
                assert np.all(seen_rd == 1) and np.all(seen_wr == 1)


def rows_per_wg(M):
    T, E, V, TP = plan(M)
    r = min(256 // T, 16)
    r = min(r, 20480 // (E * TP))
    return max(r, 1)


@pytest.mark.parametrize("n", SIZES)
def test_row_pass_shuffle_partners(n):
    M = n // 2
    T, E, V, TP = plan(M)
    R = rows_per_wg(M)
    assert 64 % T == 0 or T % 64 == 0
    assert (R * T) % 64 == 0 or R * T < 64
    for tid in range(R * T):
        t, rr = tid % T, tid // T
        lane = tid & 63
        src = (lane & ~(T - 1)) | ((T - t) & (T - 1))
        # the partner is the same row's lane (T - t) mod T, in the same wave
        partner_tid = (tid & ~63) | src
        assert partner_tid // T == rr and partner_tid % T == (T - t) % T
        # c2r: the partner's index E - 1 - j holds X[M - k] for k = t + T j (t > 0)
        if t > 0:
            tp = (T - t) % T
            for j in range(E):
                k = t + T * j
                assert tp + T * (E - 1 - j) == M - k
        # r2c: a[(V - 1 - v) T + (T - 1 - k2)] of the partner is Z[M - k]
        if t > 0:
            tp = (T - t) % T
            for v in range(V):
                for k2 in range(T):
                    k = (t + T * v) + E * k2
                    ip = (V - 1 - v) * T + (T - 1 - k2)
                    kp = (tp + T * (ip // T)) + E * (ip % T)
                    assert kp == M - k


def xcd_group(x, gx, G):
    """Tile of block x in a grid of gx blocks (the column passes' XCD-aware order): the G
    tiles G i .. G i + G - 1 of one 128-byte run go to blocks 8 G a + 8 b + r (b < G,
    r = i mod 8, a = i / 8); the identity unless 8 G divides gx."""
    if G == 1 or gx % (8 * G):
        return x
    a, b, r = x // (8 * G), (x // 8) % G, x % 8
    return 8 * G * a + G * r + b


def col_group(n, W):
    return 16 // W if n >= 2048 and W < 16 else 1


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("kind", ["y_main", "y_nyq", "z_main", "z_nyq"])
def test_xcd_tile_order(n, kind):
    # workgroups are dispatched round-robin over 8 XCDs (block x on XCD x mod 8 when 8
    # divides the grid's x extent); the reordered tiles must cover the lines once, and the
    # G tiles of a 128-byte run must share an XCD and be dispatched within 8 G blocks
    d = lines(kind, n)
    L1 = d[6]
    for W in widths(n):
        if L1 % W:
            continue
        gx, G = L1 // W, col_group(n, W)
        tiles = [xcd_group(x, gx, G) for x in range(gx)]
        assert sorted(tiles) == list(range(gx))
        if G > 1 and gx % (8 * G) == 0:
            blocks_of_run = {}
            for x, t in enumerate(tiles):
                blocks_of_run.setdefault(t // G, []).append(x)
            for xs in blocks_of_run.values():
                assert len(xs) == G
                assert len({x % 8 for x in xs}) == 1
                assert max(xs) - min(xs) < 8 * G
            # a run is G W columns of 8 bytes: 128 bytes
            assert G * W * 8 == 128


def col_thread(tid, W):
    """(c, t, h) of thread tid in a split-line column workgroup (T = 32 threads per half
    line), as the kernels compute it."""
    tl = tid // W
    return tid % W, tl % 32, tl // 32


@pytest.mark.parametrize("W", [1, 2, 4, 8, 16, 32])
def test_split_line_thread_mapping(W):
    # the mapping covers every (column, line thread, half) once, with the W columns of
    # one (t, h) in consecutive threads (a W x 8 byte run per access)
    n = 64 * W
    seen = {col_thread(tid, W) for tid in range(n)}
    assert seen == {(c, t, h) for c in range(W) for t in range(32) for h in range(2)}
    for tid in range(0, n, W):
        assert [col_thread(tid + c, W) for c in range(W)] == \
            [(c,) + col_thread(tid, W)[1:] for c in range(W)]
