"""Pins of the two-level PM oracle (oracle.split): limits that reduce it to the pinned
one-level force, closed forms of the two parts of a point mass's force, the exact
periodic force for the sum, zero self-force and momentum conservation."""

import numpy as np
import pytest
import scipy.special

from oracle import codec, mesh, pp, split, step
from test_oracle_pins import G, ewald_newton, periodic_plummer

NF, NC = 64, 16
RS = split.default_r_split(NC)


def short_closed(d, rs):
    """Short-range acceleration of a unit mass at the origin (eps = 0, G = 1/4pi), at
    separation d with |d| << 1 (periodic images negligible): the erfc part of the Ewald
    split of Newton's force."""
    r = np.linalg.norm(d)
    f = G / r ** 2 * (scipy.special.erfc(r / (2 * rs))
                      + r / (rs * np.sqrt(np.pi)) * np.exp(-r * r / (4 * rs * rs)))
    return -f * np.asarray(d) / r


def point_mass_cases(rng, rc, nsrc=3, ndir=12):
    for _ in range(nsrc):
        src = rng.random(3)
        dirs = rng.standard_normal((ndir, 3))
        dirs[:6] = np.vstack([np.eye(3), -np.eye(3)])
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        xt = np.mod(src + dirs * rc / NF, 1.0)
        x = np.vstack([src[None, :], xt])
        m = np.concatenate([[1.0], np.zeros(len(xt))])
        yield x, m, xt, dirs * rc / NF


def rms(e):
    return float(np.sqrt(np.mean(np.square(e))))


def test_infinite_split_length_is_the_one_level_fine_force():
    # r_s -> infinity: the long-range kernel vanishes and the short-range one is the whole
    # kernel, so the two-level force is the pinned one-level force on the fine mesh
    rng = np.random.default_rng(1)
    xs = [(rng.random((300, 3)), 1.0 / 300), (rng.random((500, 3)), 0.01 / 500)]
    acc, a_s, a_l = split.accelerations_two_level(xs, 32, 8, 1e3)
    ref, a1, _ = mesh.accelerations(xs, 32)
    assert np.max(np.abs(a_l)) == 0.0
    np.testing.assert_allclose(a_s, a1, rtol=0, atol=1e-14 * np.max(np.abs(a1)))
    for a, b in zip(acc, ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.max(np.abs(a1)))


@pytest.mark.parametrize("rc,tol", [(4.0, 0.03), (6.0, 0.018), (8.0, 0.018), (12.0, 0.018)])
def test_short_range_point_mass_closed_form(rc, tol):
    # the fine mesh's short-range force of a point mass (eps = 0) against the erfc form;
    # errors relative to |Newton|, half the directions along the mesh axes (measured RMS
    # over 72 cases: 2.0% at 4 cells, 0.9-1.2% at 6, 0.7-1.0% at 8-12)
    rng = np.random.default_rng(2)
    errs = []
    for x, m, xt, d in point_mass_cases(rng, rc):
        _, a_s, _ = mesh.accelerations([(x, m)], NF, 0.0, G, (RS, "short"))
        ai = mesh.interpolate(a_s, xt)
        for p in range(len(xt)):
            errs.append(np.linalg.norm(ai[p] - short_closed(d[p], RS))
                        / np.linalg.norm(ewald_newton(d[p])))
    assert rms(errs) < tol, (rc, rms(errs))


@pytest.mark.parametrize("rc,tol", [(3.0, 0.01), (4.0, 0.01), (6.0, 0.01), (8.0, 0.012),
                                    (12.0, 0.025), (16.0, 0.025)])
def test_long_range_point_mass_is_newton_minus_short(rc, tol):
    # the coarse mesh's long-range force (eps = 0) against the exact periodic Newton force
    # minus the closed-form short range: independent of the mesh, the FFT and the filter's
    # code. Measured RMS 0.1-0.8% to 8 fine cells, 1-1.9% at 12-16. Without the window
    # division the errors are 0.7, 1.8, 3.2, 4.7, 4.0% at 4, 6, 8, 12, 16 cells.
    rng = np.random.default_rng(3)
    errs = []
    for x, m, xt, d in point_mass_cases(rng, rc):
        _, a_l, _ = mesh.accelerations([(x, m)], NC, 0.0, G, (RS, "long"))
        ai = mesh.interpolate(a_l, xt)
        for p in range(len(xt)):
            nw = ewald_newton(d[p])
            errs.append(np.linalg.norm(ai[p] - (nw - short_closed(d[p], RS))) / np.linalg.norm(nw))
    assert rms(errs) < tol, (rc, rms(errs))


@pytest.mark.parametrize("rc", [6.0, 8.0, 12.0, 16.0])
def test_two_level_point_mass_against_periodic_plummer(rc):
    # the sum of both levels (softening 1 fine cell on both) against the exact periodic
    # Plummer force: RMS <= 3%, no case above 6% from 6 fine cells to n/4 (measured RMS
    # 0.8-2.1%, largest 3.9%; the one-level fine force: 0.2-0.6%)
    rng = np.random.default_rng(4)
    errs = []
    for x, m, xt, d in point_mass_cases(rng, rc, nsrc=4):
        acc, _, _ = split.accelerations_two_level([(x, m)], NF, NC, RS, 1.0, G)
        for p in range(len(xt)):
            ref = periodic_plummer(d[p], 1.0 / NF)
            errs.append(np.linalg.norm(acc[0][1 + p] - ref) / np.linalg.norm(ref))
    assert rms(errs) < 0.03, (rc, rms(errs))
    assert max(errs) < 0.06, (rc, max(errs))


def test_zero_self_force_and_momentum():
    rng = np.random.default_rng(5)
    # one particle: no force on itself from either level
    x1 = rng.random((1, 3))
    acc, a_s, a_l = split.accelerations_two_level([(x1, 1.0)], 32, 8, split.default_r_split(8))
    scale = np.max(np.abs(a_s)) + np.max(np.abs(a_l)) + 1e-30
    assert np.max(np.abs(acc[0])) <= 1e-12 * max(scale, 1.0)
    # two species: sum m a = 0 (odd kernels, the same CIC weights for deposit and gather)
    xc, xn = rng.random((400, 3)), rng.random((900, 3))
    mc, mn = 1.0 / 400, 0.01 / 900
    acc, _, _ = split.accelerations_two_level([(xc, mc), (xn, mn)], 32, 8,
                                              split.default_r_split(8))
    p = mc * acc[0].sum(0) + mn * acc[1].sum(0)
    s = mc * np.abs(acc[0]).sum() + mn * np.abs(acc[1]).sum()
    assert np.max(np.abs(p)) <= 1e-13 * s


def _states(seed, n_c=8, brick=2):
    rng = np.random.default_rng(seed)
    xc = rng.random((200, 3)).astype(np.float32)
    vc = (rng.standard_normal((200, 3)) * 0.01).astype(np.float32)
    xn = rng.random((600, 3)).astype(np.float32)
    vn = (rng.standard_normal((600, 3)) * 0.3).astype(np.float32)
    st = [codec.encode(xc, vc, n_c, brick), codec.encode(xn, vn, n_c, brick)]
    return st, [1.0 / 200, 0.01 / 600]


def _same_states(a, b):
    for p, q in zip(a, b):
        for key in ("count", "pos", "vel"):
            np.testing.assert_array_equal(np.asarray(p[key]), np.asarray(q[key]))
        assert p["v_max"] == q["v_max"]


def test_step_infinite_split_length_is_the_one_level_step():
    st, ms = _states(6)
    new2, d2 = split.step_two_level(st, ms, 32, 8, 0.02, 0.02, 1e3)
    new1, d1 = step.step_compressed(st, ms, 32, 0.02, 0.02)
    _same_states(new2, new1)
    # with the PP force: equal to the one-level step with the PP term
    r_soft = 1.0 / (20 * 16)
    new2, _ = split.step_two_level(st, ms, 32, 8, 0.02, 0.02, 1e3, r_soft=r_soft)
    app = pp.pp_accel(st, ms, 32, r_soft, G)
    new1, _ = step.step_compressed(st, ms, 32, 0.02, 0.02, extra=app)
    _same_states(new2, new1)


def test_step_long_range_term_enters_the_kick():
    # the two-level step's velocities move by c_k (a_S + a_L) with the coarse-mesh max in
    # the velocity bound: compare the unquantised kicked velocities with the parts
    st, ms = _states(7)
    ck = 0.02
    new, d = split.step_two_level(st, ms, 32, 8, ck, ck, split.default_r_split(8))
    xs = [(codec.decode(s)[0].astype(np.float64), m) for s, m in zip(st, ms)]
    a_short, a_s, _ = mesh.accelerations(xs, 32, 1.0, G, (split.default_r_split(8), "short"))
    a_long, a_l, _ = mesh.accelerations(xs, 8, 0.25, G, (split.default_r_split(8), "long"))
    amax = np.max(np.abs(a_s)) + np.max(np.abs(a_l))
    assert d["a_max"] == pytest.approx(amax, rel=1e-15)
    for s, sp, al, ash in zip(st, d["species"], a_long, a_short):
        v0 = codec.decode(s)[1].astype(np.float64)
        np.testing.assert_allclose(sp["v_new"], v0 + ck * (ash + al), rtol=0, atol=1e-15)
