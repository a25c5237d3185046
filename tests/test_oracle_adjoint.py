"""Pins of the oracle adjoint: transpose identities and finite differences (CPU)."""

import numpy as np
import pytest

from oracle import adjoint, mesh


def test_deposit_gather_transpose():
    # <D m, f> = <m, D^T f> with D^T f = Delta^-3 sum_c W f(c)
    rng = np.random.default_rng(1)
    n = 8
    x = rng.random((50, 3))
    m = rng.standard_normal(50)
    f = rng.standard_normal((n, n, n))
    lhs = np.sum(mesh.deposit(x, m, n) * f)
    # gather of f via interpolate on a 3-component stack, first component
    g = mesh.interpolate(np.stack([f, f, f]), x)[:, 0] * n ** 3
    assert abs(lhs - np.sum(m * g)) <= 1e-12 * abs(lhs)


def test_interpolate_scatter_transpose():
    rng = np.random.default_rng(2)
    n = 8
    x = rng.random((40, 3))
    a = rng.standard_normal((3, n, n, n))
    g = rng.standard_normal((40, 3))
    lhs = np.sum(mesh.interpolate(a, x) * g)
    rhs = np.sum(a * mesh.scatter_vector(x, g, n))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_force_operator_transpose():
    # <K_a rho, mu_a> summed over a equals <rho, sum_a K_a^T mu_a>
    rng = np.random.default_rng(3)
    n = 8
    rho = rng.standard_normal((n, n, n))
    mu = rng.standard_normal((3, n, n, n))
    lhs = np.sum(mesh.force_mesh(rho) * mu)
    rhs = np.sum(rho * adjoint.force_transpose(mu))
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(rho ** 2) * np.sum(mu ** 2)) * 1e2


def test_gather_grad_matches_difference_of_deposit():
    # d/dx_i <deposit(x), f> = m Delta^-3 sum_c grad W f(c), checked by central FD
    rng = np.random.default_rng(4)
    n = 8
    x = rng.random((5, 3)) * 0.8 + 0.1
    f = rng.standard_normal((n, n, n))
    g = mesh.gather_grad(f, x) * n ** 3
    h = 1e-7
    for p in range(5):
        for a in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[p, a] += h
            xm[p, a] -= h
            fd = (np.sum(mesh.deposit(xp, 1.0, n) * f) - np.sum(mesh.deposit(xm, 1.0, n) * f)) / (2 * h)
            assert abs(fd - g[p, a]) <= 1e-6 * (abs(g[p, a]) + 1.0)


def _setup(seed, n=8, nc=30, nn=60):
    rng = np.random.default_rng(seed)
    xc = rng.random((nc, 3))
    vc = rng.standard_normal((nc, 3)) * 0.01
    xn = rng.random((nn, 3))
    vn = rng.standard_normal((nn, 3)) * 0.3
    return [(xc, vc, 1.0 / nc), (xn, vn, 0.01 / nn)], rng


def _cell_of(x, n):
    return np.floor(np.asarray(x) * n).astype(np.int64)


def test_step_vjp_finite_differences():
    # scalar L = <lx1, x'> + <lv1, v'> after one step; dL/dx, dL/dv by central FD
    n, dt = 8, 0.05
    species, rng = _setup(5, n)
    lx1 = [rng.standard_normal(s[0].shape) for s in species]
    lv1 = [rng.standard_normal(s[0].shape) for s in species]
    from oracle.step import step_float

    def L(sp):
        out, _ = step_float(sp, n, dt, dt)
        tot = 0.0
        for (x1, v1), (x0, _, _), a, b in zip(out, sp, lx1, lv1):
            # unwrap the periodic drift relative to the start so L is smooth
            d = np.mod(x1 - x0 + 0.5, 1.0) - 0.5
            tot += np.sum(a * (x0 + d)) + np.sum(b * v1)
        return tot

    gx, gv = adjoint.vjp_step_float(species, lx1, lv1, n, dt, dt)
    h = 1e-6
    checked = 0
    for s in range(2):
        for p in range(0, species[s][0].shape[0], 7):
            for a in range(3):
                for which in (0, 1):
                    sp_p = [(x.copy(), v.copy(), m) for x, v, m in species]
                    sp_m = [(x.copy(), v.copy(), m) for x, v, m in species]
                    sp_p[s][which][p, a] += h
                    sp_m[s][which][p, a] -= h
                    # skip stencils that cross a CIC kink (cell change) of any particle
                    if which == 0 and not np.array_equal(_cell_of(sp_p[s][0], n),
                                                         _cell_of(sp_m[s][0], n)):
                        continue
                    fd = (L(sp_p) - L(sp_m)) / (2 * h)
                    an = (gx if which == 0 else gv)[s][p, a]
                    assert abs(fd - an) <= 1e-5 * (abs(an) + 1.0), (s, p, a, which, fd, an)
                    checked += 1
    assert checked > 40


@pytest.mark.slow
def test_multistep_density_loss_gradient():
    n, dt, K = 8, 0.05, 3
    species, rng = _setup(6, n)
    rho_t = mesh.deposit_species([(x + 0.01, m) for x, _, m in species], n)
    loss, gx, gv = adjoint.grad_float_loss(species, rho_t, n, dt, K)

    def L(sp):
        traj = adjoint.run_float(sp, n, dt, K)
        return adjoint.loss_density([(x, m) for x, _, m in traj[-1]], rho_t, n)[0]

    assert abs(L(species) - loss) <= 1e-12 * loss
    h = 1e-6
    checked = 0
    for s in range(2):
        for p in range(0, species[s][0].shape[0], 9):
            for a in range(3):
                for which in (0, 1):
                    sp_p = [(x.copy(), v.copy(), m) for x, v, m in species]
                    sp_m = [(x.copy(), v.copy(), m) for x, v, m in species]
                    sp_p[s][which][p, a] += h
                    sp_m[s][which][p, a] -= h
                    tp = adjoint.run_float(sp_p, n, dt, K)
                    tm = adjoint.run_float(sp_m, n, dt, K)
                    same = all(np.array_equal(_cell_of(A[0], n), _cell_of(B[0], n))
                               for kp, km in zip(tp, tm) for A, B in zip(kp, km))
                    if not same:
                        continue
                    fd = (L(sp_p) - L(sp_m)) / (2 * h)
                    an = (gx if which == 0 else gv)[s][p, a]
                    assert abs(fd - an) <= 1e-4 * (abs(an) + 1e-3 * abs(loss)), (fd, an)
                    checked += 1
    assert checked > 20


# ------------------------------------------------ compressed adjoint: routing --

def _brick_key(cell, n_c, brick):
    """Stream key of a cell written out by hand: bricks x-fastest, cells x-fastest
    inside a brick."""
    nb = n_c // brick
    cx, cy, cz = (int(c) for c in cell)
    b = ((cz // brick) * nb + cy // brick) * nb + cx // brick
    local = ((cz % brick) * brick + cy % brick) * brick + cx % brick
    return b * brick ** 3 + local


def _stable_order(keys):
    """Pure-Python stable insertion sort: list of old indices in new order."""
    order = []
    for i, k in enumerate(keys):
        j = len(order)
        while j > 0 and keys[order[j - 1]] > k:
            j -= 1
        order.insert(j, i)
    return order


def _compressed_pair(seed, n_c=4, brick=2):
    from oracle import codec
    rng = np.random.default_rng(seed)
    states, masses = [], []
    for n, vs, m in ((40, 3.0, 1.0 / 40), (70, 9.0, 0.01 / 70)):
        x = rng.random((n, 3)).astype(np.float32)
        v = (rng.standard_normal((n, 3)) * vs).astype(np.float32)
        states.append(codec.encode(x, v, n_c, brick))
        masses.append(m)
    return states, masses


def _hand_routed_order(state, c_d, n_c, brick):
    """New stream order of a drift without kick (c_k = 0), by hand: decoded velocity,
    fixed-point displacement floor(v c_d S + 1/2), new cell, stable insertion sort."""
    from oracle import codec
    S = 256 * n_c
    u, j = codec.decode_codes(state)
    v = codec.decode_velocity(j, state["v_max"]).astype(np.float64)
    keys = []
    for p in range(u.shape[0]):
        cell = [((int(u[p, a]) + int(np.floor(v[p, a] * c_d * S + 0.5))) % S) >> 8
                for a in range(3)]
        keys.append(_brick_key(cell, n_c, brick))
    return np.array(_stable_order(keys), dtype=np.int64)


def test_vjp_step_compressed_routes_cotangents_through_the_resort():
    """With c_k = 0 the step is a pure drift: dL/dx = lambda_x' and dL/dv = lambda_v' +
    c_d lambda_x', each carried from the particle's new stream position back to its old
    one. The order is rebuilt here by hand; an inverted permutation fails."""
    from oracle import step
    n_c, brick, n_g, c_d = 4, 2, 8, 0.02
    states, masses = _compressed_pair(31, n_c, brick)
    rng = np.random.default_rng(32)
    orders = [_hand_routed_order(st, c_d, n_c, brick) for st in states]
    for o in orders:
        # the routing is not its own inverse, so getting its direction wrong is visible
        assert not np.array_equal(o[o], np.arange(o.size))
    # the oracle's re-sort is the same order
    _, diag = step.step_compressed(states, masses, n_g, 0.0, c_d)
    for o, d in zip(orders, diag["species"]):
        assert np.array_equal(d["perm"], o)
    lx1 = [rng.standard_normal((o.size, 3)) for o in orders]
    lv1 = [rng.standard_normal((o.size, 3)) for o in orders]
    gx, gv = adjoint.vjp_step_compressed(states, masses, lx1, lv1, orders, n_g, 0.0, c_d)
    for o, a, b, ex, ev in zip(orders, lx1, lv1, gx, gv):
        for new_pos, old_pos in enumerate(o):
            assert np.array_equal(ex[old_pos], a[new_pos])
            assert np.allclose(ev[old_pos], b[new_pos] + c_d * a[new_pos], rtol=0, atol=1e-15)


def test_vjp_step_compressed_equals_float_adjoint_on_routed_cotangents():
    """With a force (c_k != 0): the float adjoint at the decoded state, fed the
    cotangents routed to old order by the hand-built order."""
    from oracle import codec
    n_c, brick, n_g, dt = 4, 2, 8, 0.02
    states, masses = _compressed_pair(33, n_c, brick)
    rng = np.random.default_rng(34)
    from oracle import step
    _, diag = step.step_compressed(states, masses, n_g, dt, dt)
    orders = [d["perm"] for d in diag["species"]]
    lx1 = [rng.standard_normal((o.size, 3)) for o in orders]
    lv1 = [rng.standard_normal((o.size, 3)) for o in orders]
    gx, gv = adjoint.vjp_step_compressed(states, masses, lx1, lv1, orders, n_g, dt, dt)
    species, lxo, lvo = [], [], []
    for st, m, o, a, b in zip(states, masses, orders, lx1, lv1):
        x, v = codec.decode(st)
        species.append((x.astype(np.float64), v.astype(np.float64), m))
        ra = np.zeros_like(a)
        rb = np.zeros_like(b)
        for new_pos, old_pos in enumerate(o):
            ra[old_pos] = a[new_pos]
            rb[old_pos] = b[new_pos]
        lxo.append(ra)
        lvo.append(rb)
    fx, fv = adjoint.vjp_step_float(species, lxo, lvo, n_g, dt, dt)
    for a, b in zip(gx + gv, fx + fv):
        assert np.array_equal(a, b)
