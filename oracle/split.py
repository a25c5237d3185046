"""Oracle: the two-level particle-mesh force of Sec. 2.1, a long-range term on a coarse
global mesh plus a short-range term on a mesh four times finer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.1 computes the long-range force on a coarse mesh of (n_p/2)^3 cells spanning the
whole volume and the short-range force on a mesh 4 times finer per dimension, local to
each tile (with a buffer of n_buf = 24 fine cells around a tile, Sec. 3.1); both species
are interpolated to the same meshes. The paper gives no split kernel. Readings:
  * the split is a Gaussian filter of the softened Poisson kernel G(k) of oracle.mesh in
    Fourier space: G_L(k) = G(k) exp(-k^2 r_s^2) on the coarse mesh and G_S(k) = G(k)
    (1 - exp(-k^2 r_s^2)) on the fine mesh, with the same softening length eps (a
    length, not a cell count) on both, so that G_L + G_S = G;
  * r_s = 1.25 coarse cells by default. For eps = 0 the short-range acceleration of a
    point mass is G m / r^2 [erfc(r / 2 r_s) + r / (r_s sqrt(pi)) exp(-r^2 / 4 r_s^2)],
    below 1% of Newton's beyond 4.8 r_s = 24 fine cells: the paper's buffer width;
  * each level deposits with its own CIC weights, differentiates with its own mesh's
    gradient symbol and interpolates with its own CIC weights (oracle.mesh); a
    particle's acceleration is the sum of the two levels (plus the PP force of eq. (4)
    when asked for, oracle.pp, on the cells of the fine mesh);
  * the long-range kernel is also divided by the coarse mesh's deposit and interpolation
    windows, prod_a sinc(n_a / n_c)^4: at the split scale (k r_s ~ 1, about a coarse
    cell) the two CIC windows weaken the long-range force by several per cent, which the
    fine mesh, carrying only the short range, cannot make up (point-mass errors of the
    sum at 3-4 coarse cells fall from about 5% to 1-2%); the Gaussian filter keeps the
    divided kernel near 1e-4 of its peak or below wherever the windows are under 1/2;
  * the velocity bound of the compressed step (oracle.step) takes max |a| of the fine
    mesh plus max |a| of the coarse mesh (plus the largest PP component): interpolation
    is a convex combination of mesh values, so the sum bounds every component;
  * the paper's tiles keep the short-range solve inside one node's memory. With the
    whole box on one device the fine mesh is a single periodic tile spanning the box, so
    no buffer region is needed.

Pins (tests/test_oracle_split.py): r_s -> infinity reduces the force and the step to
the one-level ones on the fine mesh (with and without the PP force); the short-range
force of a point mass against its closed form; the long-range force against the exact
periodic Newton force minus that closed form (which fails without the window division);
the two-level sum against the exact periodic Plummer force; zero self-force and momentum
conservation.
"""

from __future__ import annotations

import numpy as np

from . import codec, mesh, pp, step

R_SPLIT_COARSE_CELLS = 1.25


def default_r_split(n_coarse: int) -> float:
    """The split length in box units: 1.25 coarse cells."""
    return R_SPLIT_COARSE_CELLS / n_coarse


def accelerations_two_level(species, n_fine: int, n_coarse: int, r_s: float,
                            soft_fine_cells: float = 1.0, G: float = 1.0 / mesh.FOUR_PI):
    """Two-level PM force of float64 particles (list of (x, mass), unit box).

    Returns (list of a_i [n][3], short-range mesh a_S [3][...] on the fine mesh,
    long-range mesh a_L [3][...] on the coarse mesh)."""
    eps_coarse_cells = soft_fine_cells * n_coarse / n_fine  # the same length on both
    _, a_s, _ = mesh.accelerations(species, n_fine, soft_fine_cells, G, (r_s, "short"))
    _, a_l, _ = mesh.accelerations(species, n_coarse, eps_coarse_cells, G, (r_s, "long"))
    acc = [mesh.interpolate(a_s, x) + mesh.interpolate(a_l, x) for x, _ in species]
    return acc, a_s, a_l


def long_range_accel(states, masses, n_coarse: int, r_s: float, eps: float,
                     G: float = 1.0 / mesh.FOUR_PI):
    """Long-range accelerations of compressed states (decoded positions) from the coarse
    mesh, per species in stream order, and the coarse force mesh. eps in box units."""
    xs = [(codec.decode(st)[0].astype(np.float64), m) for st, m in zip(states, masses)]
    acc, a_l, _ = mesh.accelerations(xs, n_coarse, eps * n_coarse, G, (r_s, "long"))
    return acc, a_l


def step_two_level(states, masses, n_fine: int, n_coarse: int, c_k: float, c_d: float,
                   r_s: float, soft_fine_cells: float = 1.0,
                   G: float = 1.0 / mesh.FOUR_PI, r_soft: float = 0.0):
    """One compressed kick-drift step with the two-level force (Sec. 2.1): the fine mesh
    carries the short-range kernel, the coarse mesh the long-range one; r_soft > 0 adds
    the PP force of eq. (4) truncated below r_soft. Returns (new states, diagnostics of
    oracle.step.step_compressed plus 'a_long' (coarse mesh) and 'pp' (per species or
    None))."""
    eps = soft_fine_cells / n_fine
    a_long, a_l = long_range_accel(states, masses, n_coarse, r_s, eps, G)
    extra = [np.asarray(a, dtype=np.float64) for a in a_long]
    extra_max = float(np.max(np.abs(a_l))) if a_l.size else 0.0
    app = None
    if r_soft > 0:
        app = pp.pp_accel(states, masses, n_fine, r_soft, G)
        extra = [e + a for e, a in zip(extra, app)]
        extra_max += max((float(np.max(np.abs(a))) for a in app if np.size(a)), default=0.0)
    new, diag = step.step_compressed(states, masses, n_fine, c_k, c_d, soft_fine_cells, G,
                                     extra=extra, extra_max=extra_max,
                                     split=(r_s, "short"))
    diag["a_long"] = a_l
    diag["pp"] = app
    return new, diag
