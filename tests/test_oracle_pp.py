"""Pins of the oracle's cell-local particle-particle force (eq. (4)) on the CPU."""

import numpy as np
import pytest

from oracle import codec, pp

G = 1.0 / (4.0 * np.pi)


def test_two_particles_inverse_square():
    # one cell of an 8^3 mesh; r = 0.03 > r_soft: a_i = G m_j (x_j - x_i) / r^3
    x0 = np.array([[0.51, 0.52, 0.53]])
    x1 = np.array([[0.53, 0.52, 0.53]])
    a0, a1 = pp.pp_accel_positions([x0, x1], [2.0, 5.0], 8, 0.01, G)
    assert np.allclose(a0[0], [G * 5.0 / 0.02 ** 2, 0, 0], rtol=1e-12)
    assert np.allclose(a1[0], [-G * 2.0 / 0.02 ** 2, 0, 0], rtol=1e-12)


def test_softening_cut_and_cell_faces():
    # closer than r_soft: no force; in neighbouring cells (across x = 6/8): no force
    x = np.array([[0.51, 0.51, 0.51], [0.515, 0.51, 0.51],
                  [0.749, 0.9, 0.9], [0.751, 0.9, 0.9]])
    (a,) = pp.pp_accel_positions([x], [1.0], 8, 0.01, G)
    assert np.all(a == 0)


def test_newton_third_law_and_brute_force():
    rng = np.random.default_rng(1)
    n_g = 4
    xs = [rng.random((60, 3)), rng.random((90, 3))]
    ms = [1.0 / 60, 0.01 / 90]
    acc = pp.pp_accel_positions(xs, ms, n_g, 0.02, G)
    tot = sum(m * a.sum(0) for m, a in zip(ms, acc))
    scale = sum(m * np.abs(a).sum() for m, a in zip(ms, acc))
    assert scale > 0
    assert np.all(np.abs(tot) <= 1e-13 * scale)
    # brute force: every pair, same cell by floor, written as plain loops
    allx = np.concatenate(xs)
    allm = np.concatenate([np.full(60, ms[0]), np.full(90, ms[1])])
    want = np.zeros_like(allx)
    for i in range(allx.shape[0]):
        ci = [int(np.floor(allx[i, a] * n_g)) for a in range(3)]
        for j in range(allx.shape[0]):
            if j == i:
                continue
            cj = [int(np.floor(allx[j, a] * n_g)) for a in range(3)]
            if ci != cj:
                continue
            d = allx[j] - allx[i]
            r = float(np.sqrt(d @ d))
            if r >= 0.02:
                want[i] += G * allm[j] * d / r ** 3
    got = np.concatenate(acc)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def test_compressed_cut_on_integer_codes():
    # the compressed form decides the cut on code differences: a pair exactly r_soft apart
    # in codes interacts, a pair one code closer does not
    n_c, n_g = 4, 8
    S = 256 * n_c
    r_soft = 10.0 / S
    for du, interacts in ((10, True), (9, False)):
        u = np.array([[100, 300, 500], [100 + du, 300, 500]], dtype=np.float64)
        x = ((u + 0.5) / S).astype(np.float32)
        st = codec.encode(x, np.zeros_like(x), n_c, 1)
        (a,) = pp.pp_accel([st], [1.0], n_g, r_soft, G)
        if interacts:
            r = du / S
            assert np.allclose(np.sort(a[:, 0]), [-G / r ** 2, G / r ** 2], rtol=1e-12)
        else:
            assert np.all(a == 0)
