"""Oracle: one particle-mesh step, on float particles and on compressed particles.

A step deposits every species on one mesh, solves for the acceleration mesh, and then
for every particle interpolates the acceleration, kicks and drifts:
    v' = v + c_k a(x),   x' = x + c_d v'  (mod 1),
the kick-drift form of leapfrog with velocities at half steps. The paper does not
state its integrator, only that a particle's displacement per step is limited
(Sec. 3.2); the kick-drift form and the separate coefficients (c_k = c_d = dt for a
static box) are readings.

On compressed particles (Sec. 2.4 format) the step decodes the bin centres, runs the
same float64 step, and re-encodes:
  * positions in fixed point: u' = (u + floor(d + 1/2)) mod S with d = v' c_d S, which
    is the encoding of the decoded centre plus the displacement (S = 256^P n_c for P
    position bytes, oracle.codec);
  * velocities with a new v_max' = the smallest power of two >= V + |c_k| A_max, where
    V is the largest decoded |v_a| of the species and A_max the largest |a_a| over
    the acceleration mesh; CIC interpolation is a convex combination of mesh values,
    so no kicked component can exceed this bound (no clamping), and a power of two
    makes the choice robust to rounding in A_max;
  * the stream is re-sorted stably by the new cell key, particles keeping their old
    stream order inside a cell.

Pins: float step through the mesh pins; compressed step against the float step
(|dx| <= q/2 per axis, |dv| <= v_max'/65536 when the float step is re-encoded),
sorted-order checks against a pure-Python insertion sort on small cases.
"""

from __future__ import annotations

import numpy as np

from . import codec, mesh


def pow2_ceil(b: float) -> float:
    """Smallest power of two >= b (0 for b <= 0)."""
    if b <= 0.0:
        return 0.0
    m, e = np.frexp(b)
    if m == 0.5:
        return float(b)
    return float(np.ldexp(1.0, int(e)))


def step_float(species, n_g: int, c_k: float, c_d: float, soft_cells: float = 1.0,
               G: float = 1.0 / mesh.FOUR_PI):
    """species: list of (x, v, mass) float arrays -> list of (x', v') float64 + diag."""
    xs = [(np.asarray(x, dtype=np.float64), m) for x, _, m in species]
    acc, a_mesh, rho = mesh.accelerations(xs, n_g, soft_cells, G)
    out = []
    for (x, v, _), ai in zip(species, acc):
        v1 = np.asarray(v, dtype=np.float64) + c_k * ai
        x1 = np.mod(np.asarray(x, dtype=np.float64) + c_d * v1, 1.0)
        out.append((x1, v1))
    return out, {"acc": acc, "a_mesh": a_mesh, "rho": rho}


def kick_codes(u: np.ndarray, v_dec: np.ndarray, a_i: np.ndarray, v_max_new, S: int,
               c_k: float, c_d: float, vel_bytes: int = 2):
    """Kick, fixed-point drift and velocity re-binning of decoded particles.

    u: position codes [n][3] (S steps per box side); v_dec: decoded velocities; a_i:
    interpolated accelerations; v_max_new: the new bin range; vel_bytes: 2^(8 vel_bytes)
    velocity bins, half range H. Returns (u_new, j_new, v_new, pos_pre, vel_pre) with the
    pre-floor values d + 1/2 and v' C + H, C = H / v_max_new.
    """
    H = float(codec.half_range(vel_bytes))
    v1 = np.asarray(v_dec, dtype=np.float64) + c_k * np.asarray(a_i, dtype=np.float64)
    d = v1 * (c_d * S)
    pos_pre = d + 0.5
    u1 = np.mod(np.asarray(u, dtype=np.int64) + np.floor(pos_pre).astype(np.int64), S)
    if float(v_max_new) > 0:
        C = H / np.float64(v_max_new)
        vel_pre = v1 * C + H
        j1 = np.clip(np.floor(vel_pre), 0, 2 * H - 1).astype(np.int64)
    else:
        vel_pre = np.full(v1.shape, H)
        j1 = np.full(v1.shape, int(H), dtype=np.int64)
    return u1, j1, v1, pos_pre, vel_pre


def step_compressed(states, masses, n_g: int, c_k: float, c_d: float,
                    soft_cells: float = 1.0, G: float = 1.0 / mesh.FOUR_PI, extra=None,
                    extra_max=None, split=None):
    """states: list of codec state dicts (same n_c, brick) -> new states + diagnostics.

    extra (optional): per species an additional acceleration [n][3] in old stream order
    (the cell-local PP force of eq. (4), the long-range force of the two-level PM); it is
    added to the interpolated mesh force, and the velocity bound takes A_max + extra_max,
    by default max |extra_a| over all species and axes. split: the mesh kernel's part of
    the two-level split (oracle.mesh.split_factor).

    Diagnostics per species: 'perm' (new stream index -> old stream index), the
    pre-floor values 'pos_pre' = d + 1/2 and 'vel_pre' = v' C + 32768 in old stream
    order, 'v_max_new', 'acc' (interpolated accelerations, old order), 'v_new' (the
    unquantised float64 kicked velocities).
    """
    n_c = states[0]["n_c"]
    brick = states[0]["brick"]
    decoded = [codec.decode(st) for st in states]
    xs = [(x.astype(np.float64), m) for (x, _), m in zip(decoded, masses)]
    acc, a_mesh, rho = mesh.accelerations(xs, n_g, soft_cells, G, split)
    a_max = float(np.max(np.abs(a_mesh))) if a_mesh.size else 0.0
    if extra is not None:
        acc = [ai + np.asarray(e, dtype=np.float64) for ai, e in zip(acc, extra)]
        if extra_max is None:
            extra_max = max((float(np.max(np.abs(e))) for e in extra if np.size(e)),
                            default=0.0)
        a_max += extra_max
    new_states, diags = [], []
    for st, (x, v), ai in zip(states, decoded, acc):
        u, _ = codec.decode_codes(st)
        v_dec = v.astype(np.float64)
        V = float(np.max(np.abs(v_dec))) if v_dec.size else 0.0
        v_max_new = np.float32(pow2_ceil(V + abs(c_k) * a_max))
        pb, vb = codec.widths(st)
        S = codec.pos_scale(n_c, pb)
        u1, j1, v1, pos_pre, vel_pre = kick_codes(u, v_dec, ai, v_max_new, S, c_k, c_d, vb)
        keys = codec.cell_keys(u1 >> (8 * pb), n_c, brick)
        perm = np.argsort(keys, kind="stable")
        ns = codec.assemble(u1[perm], j1[perm], keys[perm], v_max_new, n_c, brick, None,
                            pb, vb)
        new_states.append(ns)
        diags.append({"perm": perm, "pos_pre": pos_pre, "vel_pre": vel_pre,
                      "v_max_new": v_max_new, "acc": ai, "v_new": v1,
                      "u_new": u1, "j_new": j1})
    return new_states, {"species": diags, "a_max": a_max, "a_mesh": a_mesh, "rho": rho}
