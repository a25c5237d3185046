"""Oracle: the adjoint (vector-Jacobian product) of one particle-mesh step.

For the step v' = v + c_k a(x), x' = x + c_d v', given lambda_x' = dL/dx' and
lambda_v' = dL/dv' the adjoint returns dL/dx and dL/dv:
    g_v      = lambda_v' + c_d lambda_x'
    lambda_v = g_v,   g_a = c_k g_v
    lambda_x = lambda_x'
             + sum_c grad W(x_i - x_c) [sum_a a_a(c) g_a,ia]           (direct term)
             + m_i Delta^-3 sum_c grad W(x_i - x_c) nu(c)               (through rho)
with mu_a(c) = sum_j W(x_j - x_c) g_a,ja (the transpose of the force interpolation is
a scatter) and nu = sum_a IDFT(+i D(k_a) G(k) DFT(mu_a)): the force operator a_a = K_a rho
is a real odd convolution, so its transpose is K_a^T = -K_a, i.e. the conjugate of
the spectral multiplier (D is odd and zero on the Nyquist index). The transpose of the CIC
deposit is the CIC gather scaled by Delta^-3 and the particle mass.

For compressed particles the quantisation of positions and velocities is treated as
the identity (straight-through); the adjoint is taken at the decoded state, and the
stream permutation of the re-sort maps the new-order cotangents back to old order.

Loss used by the differentiable workload: L = sum_c (rho(c) - rho_t(c))^2, with
dL/dx_i = 2 m_i Delta^-3 sum_c grad W(x_i - x_c) (rho(c) - rho_t(c)).

Pins: dot-product (transpose) identities of deposit/gather, interpolate/scatter and
K_a/K_a^T in float64; central finite differences of the whole step and of multi-step
losses on the float path.
"""

from __future__ import annotations

import numpy as np

from . import codec, mesh


def force_transpose(mu: np.ndarray, soft_cells: float = 1.0,
                    G: float = 1.0 / mesh.FOUR_PI) -> np.ndarray:
    """nu = sum_a K_a^T mu_a with K_a^T = IDFT(conj(-i D(k_a) G) DFT(.))."""
    n_g = mu.shape[1]
    g = mesh.green(n_g, soft_cells, G)
    acc_k = np.zeros((n_g, n_g, n_g // 2 + 1), dtype=np.complex128)
    for ax, fac in enumerate(mesh.gradient_factors(n_g)):
        acc_k += np.conj(fac) * g * np.fft.rfftn(mu[ax])
    return np.fft.irfftn(acc_k, s=(n_g, n_g, n_g), axes=(0, 1, 2))


def vjp_step_float(species, lam_x1, lam_v1, n_g: int, c_k: float, c_d: float,
                   soft_cells: float = 1.0, G: float = 1.0 / mesh.FOUR_PI):
    """species: list of (x, v, mass); lam_*1: lists of [n][3] -> (lam_x, lam_v) lists."""
    xs = [(np.asarray(x, dtype=np.float64), m) for x, _, m in species]
    rho = mesh.deposit_species(xs, n_g)
    a = mesh.force_mesh(rho, soft_cells, G)
    g_as, lam_vs = [], []
    mu = np.zeros((3, n_g, n_g, n_g))
    for (x, _), lx, lv in zip(xs, lam_x1, lam_v1):
        g_v = np.asarray(lv, dtype=np.float64) + c_d * np.asarray(lx, dtype=np.float64)
        lam_vs.append(g_v)
        g_a = c_k * g_v
        g_as.append(g_a)
        mu += mesh.scatter_vector(x, g_a, n_g)
    nu = force_transpose(mu, soft_cells, G)
    lam_xs = []
    for (x, m), lx, g_a in zip(xs, lam_x1, g_as):
        direct = np.zeros_like(g_a)
        for ax in range(3):
            # sum_c grad W [a_ax(c)] weighted by g_a,i,ax
            direct += mesh.gather_grad(a[ax], x) * g_a[:, ax:ax + 1]
        through = mesh.gather_grad(nu, x) * (m * float(n_g) ** 3)
        lam_xs.append(np.asarray(lx, dtype=np.float64) + direct + through)
    return lam_xs, lam_vs


def loss_density(species, rho_t: np.ndarray, n_g: int):
    """L = sum (rho - rho_t)^2 and dL/dx per species (dL/dv = 0)."""
    xs = [(np.asarray(x, dtype=np.float64), m) for x, m in species]
    rho = mesh.deposit_species(xs, n_g)
    r = rho - rho_t
    loss = float(np.sum(r * r))
    grads = [mesh.gather_grad(2.0 * r, x) * (m * float(n_g) ** 3) for x, m in xs]
    return loss, grads


def run_float(species, n_g, dt, steps, soft_cells=1.0, G=1.0 / mesh.FOUR_PI):
    """Forward K float steps; returns list of per-step states [(x, v, m) lists]."""
    from .step import step_float
    traj = [[(np.asarray(x, np.float64), np.asarray(v, np.float64), m)
             for x, v, m in species]]
    cur = traj[0]
    for _ in range(steps):
        out, _ = step_float(cur, n_g, dt, dt, soft_cells, G)
        cur = [(x1, v1, m) for (x1, v1), (_, _, m) in zip(out, cur)]
        traj.append(cur)
    return traj


def grad_float_loss(species, rho_t, n_g, dt, steps, soft_cells=1.0,
                    G=1.0 / mesh.FOUR_PI):
    """Loss after K float steps and its gradient w.r.t. the initial x and v."""
    traj = run_float(species, n_g, dt, steps, soft_cells, G)
    final = traj[-1]
    loss, lam_x = loss_density([(x, m) for x, _, m in final], rho_t, n_g)
    lam_v = [np.zeros_like(g) for g in lam_x]
    for k in range(steps - 1, -1, -1):
        lam_x, lam_v = vjp_step_float(traj[k], lam_x, lam_v, n_g, dt, dt, soft_cells, G)
    return loss, lam_x, lam_v


def vjp_step_compressed(states, masses, lam_x1, lam_v1, perms, n_g, c_k, c_d,
                        soft_cells=1.0, G=1.0 / mesh.FOUR_PI):
    """Straight-through adjoint at the decoded state.

    lam_*1 are in the NEW stream order of each species; perms[s][j] is the old stream
    index of new particle j. Returns (lam_x, lam_v) in the OLD stream order.
    """
    species = []
    lx_old, lv_old = [], []
    for st, m, lx, lv, perm in zip(states, masses, lam_x1, lam_v1, perms):
        x, v = codec.decode(st)
        species.append((x.astype(np.float64), v.astype(np.float64), m))
        a = np.empty_like(np.asarray(lx, dtype=np.float64))
        b = np.empty_like(a)
        a[perm] = lx
        b[perm] = lv
        lx_old.append(a)
        lv_old.append(b)
    return vjp_step_float(species, lx_old, lv_old, n_g, c_k, c_d, soft_cells, G)
