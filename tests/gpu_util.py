"""Shared helpers of the GPU parity tests: contexts, seeded loads, tie-zone checks."""

import numpy as np
import pytest
import torch

from oracle import codec
from pmsynth import make_workload


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"


def ctx(n_mesh, n_cell, brick=None, soft=1.0):
    from paper_1611_01545_amd import PMContext
    require_gpu()
    return PMContext(n_mesh, n_cell, brick=brick, soft_cells=soft)


def small_two_species(n_p_c=16, n_mesh=32, seed_offset=0, n_cell=None):
    """The two-species workload recipe at a reduced size (same generators)."""
    n_cell = n_cell or n_p_c
    return make_workload("two_species_256", seed_offset=seed_offset, n_p_c=n_p_c,
                         n_p_nu=2 * n_p_c, n_mesh=n_mesh, n_cell=n_cell)


def assert_state_equal(host, ref, keys=("count", "esc", "pos", "vel", "v_max")):
    for k in keys:
        a, b = np.asarray(host[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        assert np.array_equal(a, b), f"{k} differs in {np.count_nonzero(a != b)} places"


def density_close(rho_gpu, rho_ref, tol=1e-5):
    """|d rho| <= tol * max(|rho|, mean rho) at every node."""
    rho_gpu = np.asarray(rho_gpu, dtype=np.float64)
    scale = np.maximum(np.abs(rho_ref), np.abs(rho_ref).mean())
    err = np.abs(rho_gpu - rho_ref) / scale
    return float(err.max())


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))


def frac_dist(x):
    """Distance of x to the nearest integer."""
    return np.abs(x - np.round(x))


def _codes_old_order(host_state, perm):
    """Integer position codes u and velocity codes j of a state, in old stream order."""
    from oracle import codec
    u, j = codec.decode_codes(host_state)
    uo = np.empty_like(u)
    jo = np.empty_like(j)
    uo[perm] = u
    jo[perm] = j
    return uo, jo


def check_codes(c, out, perms, new, diag, n_cell, dt, a_rms=None):
    """GPU step outputs against oracle.step.step_compressed: position and velocity codes
    equal in old stream order except in the tie zone, counts and escapes consistent, the
    stream the stable cell sort of the new codes. Returns the number of tie-zone codes.
    a_rms: the force scale of the tolerance (default: RMS of the oracle's force mesh)."""
    from oracle import codec
    if a_rms is None:
        a_rms = np.sqrt(np.mean(diag["a_mesh"] ** 2))
    ties = 0
    for o, ns, d, perm in zip(out, new, diag["species"], perms):
        h = c.to_host(o)
        pb, vb = codec.widths(ns)
        assert codec.widths(h) == (pb, vb)
        S = codec.pos_scale(n_cell, pb)
        pm = perm.cpu().numpy()
        assert np.array_equal(np.sort(pm), np.arange(pm.size))
        ug, jg = _codes_old_order(h, pm)
        # tie zone: the oracle's pre-floor value lies within the propagated tolerance of
        # an integer. A force within the 1e-4 relative RMS tolerance differs at a particle
        # by at most 1e-4 (|a_i| + RMS(a)); v' = v + c_k a_i rounds once more in float32
        # (2^-23 |v'| + 2^-23 |c_k a_i|); the velocity code scales v' by a power of two
        # and the drift multiplies it by c_d S / L in float64.
        ai = np.abs(d["acc"])
        dv = abs(dt) * (1e-4 * (ai + a_rms) + 2.0 ** -23 * ai) + 2.0 ** -23 * np.abs(d["v_new"])
        tau_x = dt * S * dv + 1e-6 * np.maximum(1.0, np.abs(d["pos_pre"]))
        du = (ug - d["u_new"] + S // 2) % S - S // 2
        bad = du != 0
        assert np.all(np.abs(du[bad]) <= 1)
        assert np.all(frac_dist(d["pos_pre"][bad]) <= tau_x[bad])
        assert bad.mean() < 1e-3
        # velocity codes (same v_max' on both sides in these cases)
        assert float(h["v_max"]) == float(d["v_max_new"])
        C = codec.half_range(vb) / float(d["v_max_new"])
        tau_v = C * dv + 1e-6
        dj = jg - d["j_new"]
        badv = dj != 0
        assert np.all(np.abs(dj[badv]) <= 1)
        assert np.all(frac_dist(d["vel_pre"][badv]) <= tau_v[badv])
        assert badv.mean() < 1e-3
        ties += int(bad.sum() + badv.sum())
        # counts and escape table: the oracle's when every code agrees, and in any case
        # the counts of the GPU's own new codes (the escape rebuild after the kick)
        keys_new = codec.cell_keys(ug >> (8 * pb), n_cell, c.brick)
        cnt, esc = codec.build_counts(np.sort(keys_new), n_cell)
        assert np.array_equal(h["count"], cnt)
        assert np.array_equal(np.asarray(h["esc"], dtype=np.uint64).reshape(-1, 2), esc)
        if not bad.any():
            assert np.array_equal(h["count"], ns["count"])
            assert np.array_equal(np.asarray(h["esc"]).reshape(-1, 2).astype(np.uint64),
                                  np.asarray(ns["esc"]).reshape(-1, 2).astype(np.uint64))
        # the stream is the stable cell sort of the GPU's own new codes
        order = np.argsort(keys_new, kind="stable")
        assert np.array_equal(order, pm)
        assert np.array_equal(codec.full_counts(h),
                              np.bincount(keys_new, minlength=n_cell ** 3))
    return ties
