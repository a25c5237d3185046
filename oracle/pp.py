"""Oracle: the particle-particle (PP) force of eq. (4) inside the cells of the mesh.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.1: below the mesh scale the PM force is supplemented by a direct sum over the
particles that share particle i's cell of the (fine) interpolation mesh,
    F_i = G m_i sum_{j != i, same cell} m_j (x_j - x_i) / |x_j - x_i|^3,
truncated below the softening length r_soft (the paper uses r_soft = L / (20 n_p)).
Readings where the paper is silent:
  * the cell is a cell of the PM mesh (side Delta = L / n_g), the mesh the force is
    interpolated from; particles of every species in that cell take part;
  * "truncated" is read as a hard cut: a pair closer than r_soft exerts no force;
  * compressed particles sit at their bin centres; the cut is decided on the exact integer
    code differences du (|du|^2 >= (r_soft S / L)^2 with S = 256^P n_cell), so that it does not
    depend on rounding;
  * the acceleration is a_i = F_i / m_i.

Pins (tests/test_oracle_pp.py): two particles against the inverse-square law, the cut,
Newton's third law (sum m_i a_i = 0), no pair across a cell face, and the per-cell
grouping against a brute-force loop over all pairs of particles.
"""

from __future__ import annotations

import numpy as np

from . import codec


def pp_accel_positions(xs, masses, n_g: int, r_soft: float, G: float, box: float = 1.0,
                       codes=None, S: int | None = None):
    """PP accelerations of float64 particle positions xs (list of [n][3] in [0, box)).

    codes/S (optional): the integer position codes of the same particles, for the exact
    cut |du|^2 >= (r_soft S / box)^2; without them the cut is |x_j - x_i| >= r_soft."""
    allx = np.concatenate([np.asarray(x, dtype=np.float64) for x in xs]) if xs else \
        np.zeros((0, 3))
    allm = np.concatenate([np.full(np.asarray(x).shape[0], m, dtype=np.float64)
                           for x, m in zip(xs, masses)]) if xs else np.zeros(0)
    allu = np.concatenate([np.asarray(u, dtype=np.int64) for u in codes]) if codes else None
    cell = np.floor(allx * (n_g / box)).astype(np.int64) % n_g
    key = (cell[:, 2] * n_g + cell[:, 1]) * n_g + cell[:, 0]
    acc = np.zeros_like(allx)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    bounds = np.flatnonzero(np.diff(ks)) + 1
    groups = np.split(order, bounds)
    cut2 = (r_soft * S / box) ** 2 if allu is not None else r_soft ** 2
    for g in groups:
        if g.size < 2:
            continue
        x = allx[g]
        d = x[None, :, :] - x[:, None, :]          # x_j - x_i  [i][j][3]
        r2 = np.sum(d * d, axis=2)
        if allu is not None:
            du = allu[g][None, :, :] - allu[g][:, None, :]
            keep = np.sum(du * du, axis=2) >= cut2
        else:
            keep = r2 >= cut2
        np.fill_diagonal(keep, False)
        with np.errstate(divide="ignore", invalid="ignore"):
            w = np.where(keep, allm[g][None, :] / np.where(keep, r2, 1.0) ** 1.5, 0.0)
        acc[g] = G * np.sum(w[:, :, None] * d, axis=1)
    out, at = [], 0
    for x in xs:
        n = np.asarray(x).shape[0]
        out.append(acc[at:at + n])
        at += n
    return out


def pp_accel(states, masses, n_g: int, r_soft: float, G: float, box: float = 1.0):
    """PP accelerations of compressed states, per species in stream order."""
    xs, us = [], []
    pb = codec.widths(states[0])[0]
    assert all(codec.widths(st)[0] == pb for st in states), "one position width per call"
    S = codec.pos_scale(states[0]["n_c"], pb)
    for st in states:
        u, _ = codec.decode_codes(st)
        us.append(u)
        xs.append((u.astype(np.float64) + 0.5) * (box / S))
    return pp_accel_positions(xs, masses, n_g, r_soft, G, box, codes=us, S=S)
