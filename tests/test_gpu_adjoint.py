"""GPU parity of the adjoint calls (pm_step_vjp, pm_loss_density_vjp) against the oracle.

The oracle's adjoint is pinned by finite differences and transpose identities on the
CPU (test_oracle_adjoint.py); here the HIP path is compared with it on the same seeded
states and cotangents. Tolerance: the HIP path computes in float32 (density, force
meshes, the transposed force and the gathers); the gradient sums terms of both signs,
so the comparison is a relative RMS over all particles, 1e-3, with the velocity
cotangent (a plain axpy) held to 1e-6.
"""

import numpy as np
import pytest
import torch

from gpu_util import ctx, rel_rms, small_two_species
from oracle import adjoint, codec, step
from pmsynth import make_workload

pytestmark = pytest.mark.gpu

TOL = 1e-3


def _cotangents(ns, seed):
    rng = np.random.default_rng(seed)
    return ([rng.standard_normal((n, 3)).astype(np.float32) for n in ns],
            [rng.standard_normal((n, 3)).astype(np.float32) for n in ns])


def _dev(arrs, device):
    return [torch.from_numpy(a).to(device) for a in arrs]


# (16, 8): a 16^3 mesh runs every column pass at 8 columns per workgroup (as at 2048^3)
@pytest.mark.parametrize("n_mesh,n_p", [(16, 8), (32, 16), (64, 32)])
def test_step_vjp_float_matches_oracle(n_mesh, n_p):
    wl = make_workload("plain_cdm_64", n_p_c=n_p, n_mesh=n_mesh, n_cell=n_p // 2)
    c = ctx(wl.n_mesh, wl.n_cell)
    sp = [c.float_species(s.x, s.v, s.mass) for s in wl.species]
    lx1, lv1 = _cotangents([s.n for s in wl.species], 7)
    gx, gv = c.step_vjp(sp, wl.dt, _dev(lx1, c.device), _dev(lv1, c.device))
    rx, rv = adjoint.vjp_step_float([(s.x, s.v, s.mass) for s in wl.species], lx1, lv1,
                                    wl.n_mesh, wl.dt, wl.dt)
    for a, b in zip(gv, rv):
        assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-6 * np.max(np.abs(b))
    for a, b, l in zip(gx, rx, lx1):
        # compare the part the step adds to the passed-through cotangent
        e = rel_rms(a.cpu().numpy() - l, b - l)
        assert e <= TOL, e
    c.close()


# (n_mesh, n_cell): 16-node tiles of 8 cells (r = 2), of 4 cells (r = 4), and a shape
# that takes the per-particle fallback (r = 1)
@pytest.mark.parametrize("n_mesh,n_cell", [(16, 8), (32, 16), (64, 16), (32, 32)])
def test_step_vjp_compressed_two_species_matches_oracle(n_mesh, n_cell):
    wl = small_two_species(n_p_c=16, n_mesh=n_mesh, n_cell=n_cell)
    c = ctx(wl.n_mesh, wl.n_cell)
    st = [c.encode(c.float_species(s.x, s.v, s.mass)) for s in wl.species]
    host = [c.to_host(s) for s in st]
    masses = [s.mass for s in wl.species]
    # the oracle's re-sort; the GPU recomputes its own and must agree
    _, diag = step.step_compressed(host, masses, wl.n_mesh, wl.dt, wl.dt)
    perms = [d["perm"] for d in diag["species"]]
    acc, amax = c.force(c.deposit(st))
    _, gperms = c.kick_drift_perm(st, acc, amax, wl.dt, wl.dt)
    for p, g in zip(perms, gperms):
        assert np.array_equal(p, g.cpu().numpy())
    ns = [s.n for s in wl.species]
    lx1, lv1 = _cotangents(ns, 11)
    gx, gv = c.step_vjp(st, wl.dt, _dev(lx1, c.device), _dev(lv1, c.device))
    rx, rv = adjoint.vjp_step_compressed(host, masses, lx1, lv1, perms, wl.n_mesh,
                                         wl.dt, wl.dt)
    for a, b in zip(gv, rv):
        assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-6 * np.max(np.abs(b))
    for a, b, l, p in zip(gx, rx, lx1, perms):
        lo = np.empty_like(l)
        lo[p] = l  # passed-through cotangent in old order
        e = rel_rms(a.cpu().numpy() - lo, b - lo)
        assert e <= TOL, e
    c.close()


def test_step_vjp_compressed_dense_tile_matches_oracle():
    """Half of the neutrinos in a ball of radius 0.02: one tile holds far more particles
    than one batch of the tiled scatter, which then sizes its fixed-point unit from a
    pass of its own over the tile's cotangents."""
    import types
    wl = small_two_species(n_p_c=16, n_mesh=64, n_cell=16, seed_offset=3)
    rng = np.random.default_rng(21)
    nu = wl.species[1]
    x = nu.x.copy()
    h = x.shape[0] // 2
    x[:h] = (0.3 + 0.02 * rng.uniform(-1.0, 1.0, (h, 3))).astype(x.dtype)
    species = [wl.species[0], types.SimpleNamespace(x=x, v=nu.v, mass=nu.mass)]
    c = ctx(wl.n_mesh, wl.n_cell)
    st = [c.encode(c.float_species(s.x, s.v, s.mass)) for s in species]
    host = [c.to_host(s) for s in st]
    masses = [s.mass for s in species]
    _, diag = step.step_compressed(host, masses, wl.n_mesh, wl.dt, wl.dt)
    perms = [d["perm"] for d in diag["species"]]
    ns = [s.x.shape[0] for s in species]
    lx1, lv1 = _cotangents(ns, 13)
    gx, gv = c.step_vjp(st, wl.dt, _dev(lx1, c.device), _dev(lv1, c.device))
    rx, rv = adjoint.vjp_step_compressed(host, masses, lx1, lv1, perms, wl.n_mesh,
                                         wl.dt, wl.dt)
    for a, b, l, p in zip(gx, rx, lx1, perms):
        lo = np.empty_like(l)
        lo[p] = l
        e = rel_rms(a.cpu().numpy() - lo, b - lo)
        assert e <= TOL, e
    c.close()


def test_step_vjp_compressed_repeatable():
    """The tiled scatter sums fixed-point integers: two calls give the same bits."""
    wl = small_two_species(n_p_c=16, n_mesh=64, n_cell=16, seed_offset=5)
    c = ctx(wl.n_mesh, wl.n_cell)
    st = [c.encode(c.float_species(s.x, s.v, s.mass)) for s in wl.species]
    lx1, lv1 = _cotangents([s.n for s in wl.species], 19)
    a = c.step_vjp(st, wl.dt, _dev(lx1, c.device), _dev(lv1, c.device))
    b = c.step_vjp(st, wl.dt, _dev(lx1, c.device), _dev(lv1, c.device))
    for p, q in zip(a[0] + a[1], b[0] + b[1]):
        assert torch.equal(p, q)
    c.close()


def test_step_vjp_nan_cotangent_propagates():
    """A NaN velocity cotangent must not vanish in the fixed-point scatter: its tile is
    summed in float, so the position gradients come out NaN."""
    wl = small_two_species(n_p_c=16, n_mesh=64, n_cell=16, seed_offset=4)
    c = ctx(wl.n_mesh, wl.n_cell)
    st = [c.encode(c.float_species(s.x, s.v, s.mass)) for s in wl.species]
    ns = [s.n for s in wl.species]
    lx1, lv1 = _cotangents(ns, 17)
    lv1[1][5, 2] = np.nan
    gx, _ = c.step_vjp(st, wl.dt, _dev(lx1, c.device), _dev(lv1, c.device))
    assert np.isnan(gx[0].cpu().numpy()).any()
    c.close()


def test_step_vjp_rejects_aliased_results():
    wl = make_workload("plain_cdm_64", n_p_c=8, n_mesh=16, n_cell=8)
    c = ctx(wl.n_mesh, wl.n_cell)
    sp = [c.float_species(s.x, s.v, s.mass) for s in wl.species]
    lx = torch.zeros((sp[0].n, 3), dtype=torch.float32, device=c.device)
    lv = torch.zeros_like(lx)
    import ctypes

    from paper_1611_01545_amd import _lib
    from paper_1611_01545_amd.pm import _species_array
    arr = _species_array(sp)
    P = lambda t: (ctypes.c_void_p * 1)(t.data_ptr())
    st = c.lib.pm_step_vjp(c.h, arr, 1, 0.01, P(lx), P(lv), P(lx), P(torch.empty_like(lv)))
    assert _lib.STATUS[st] == "PM_ERR_ARG"
    c.close()


@pytest.mark.parametrize("layout", ["float", "compressed"])
def test_loss_density_vjp_matches_oracle(layout):
    wl = small_two_species(n_p_c=16, n_mesh=32)
    tgt = small_two_species(n_p_c=16, n_mesh=32, seed_offset=5)
    rho_t = sum(__import__("oracle").mesh.deposit(s.x, s.mass, wl.n_mesh)
                for s in tgt.species)
    c = ctx(wl.n_mesh, wl.n_cell)
    sp = [c.float_species(s.x, s.v, s.mass) for s in wl.species]
    if layout == "compressed":
        sp = [c.encode(s) for s in sp]
        xs = [codec.decode(c.to_host(s))[0] for s in sp]
    else:
        xs = [s.x for s in wl.species]
    loss, g = c.loss_density_vjp(sp, torch.from_numpy(rho_t.astype(np.float32)).to(c.device))
    rl, rg = adjoint.loss_density([(x, s.mass) for x, s in zip(xs, wl.species)], rho_t,
                                  wl.n_mesh)
    assert abs(float(loss.item()) - rl) <= 1e-4 * rl
    for a, b in zip(g, rg):
        e = rel_rms(a.cpu().numpy(), b)
        assert e <= TOL, e
    c.close()


@pytest.mark.parametrize("full", [False, True], ids=["32^3-mesh", "adjoint_128"])
def test_multistep_gradient_along_compressed_trajectory(full):
    """K compressed steps forward, then the chain of step VJPs backward from a density
    loss, against the float64 oracle's chain along the same (decoded) trajectory with
    the oracle's own re-sort permutations. Errors of the K chained float32 VJPs add, so
    the bound is K times the one-step tolerance.

    Also reported, not asserted: the gradient through K uncompressed float64 steps from
    the decoded initial state. The two trajectories differ (at this size most CDM
    particles move less than half a position quantum per step and stay frozen in the
    fixed-point drift), so the gradients differ by several per cent.

    Run at a 32^3 mesh for 3 steps and at the differentiable workload's full size
    (64^3 CDM, 128^3 mesh, 10 steps of dt 0.02)."""
    if full:
        wl = make_workload("adjoint_128")
        tgt = make_workload("adjoint_128", seed_offset=1)
        K = wl.steps
    else:
        wl = make_workload("adjoint_128", n_p_c=16, n_mesh=32, n_cell=16)
        tgt = make_workload("adjoint_128", seed_offset=1, n_p_c=16, n_mesh=32, n_cell=16)
        K = 3
    from oracle import mesh
    rho_t = sum(mesh.deposit(s.x, s.mass, wl.n_mesh) for s in tgt.species)
    masses = [s.mass for s in wl.species]
    c = ctx(wl.n_mesh, wl.n_cell)
    st = [c.encode(c.float_species(s.x, s.v, s.mass)) for s in wl.species]
    traj = [st]
    for _ in range(K):
        nxt = [c.empty_like(s) for s in traj[-1]]
        c.step(traj[-1], wl.dt, out=nxt)
        traj.append(nxt)
    rho_t_dev = torch.from_numpy(rho_t.astype(np.float32)).to(c.device)
    _, lx = c.loss_density_vjp(traj[-1], rho_t_dev)
    lv = [torch.zeros_like(t) for t in lx]
    for k in range(K - 1, -1, -1):
        lx, lv = c.step_vjp(traj[k], wl.dt, lx, lv)
    hosts = [[c.to_host(s) for s in states] for states in traj]
    xK = [codec.decode(h)[0] for h in hosts[K]]
    _, rx = adjoint.loss_density([(x, m) for x, m in zip(xK, masses)], rho_t, wl.n_mesh)
    rv = [np.zeros_like(g) for g in rx]
    for k in range(K - 1, -1, -1):
        _, diag = step.step_compressed(hosts[k], masses, wl.n_mesh, wl.dt, wl.dt)
        perms = [d["perm"] for d in diag["species"]]
        rx, rv = adjoint.vjp_step_compressed(hosts[k], masses, rx, rv, perms, wl.n_mesh,
                                             wl.dt, wl.dt)
    ex = rel_rms(lx[0].cpu().numpy(), rx[0])
    ev = rel_rms(lv[0].cpu().numpy(), rv[0])
    x0, v0 = codec.decode(hosts[0][0])
    _, fx, fv = adjoint.grad_float_loss([(x0, v0, masses[0])], rho_t, wl.n_mesh, wl.dt, K)
    print(f"{K} steps on {wl.n_mesh}^3: chain vs oracle: x {ex:.2e} v {ev:.2e}; "
          f"compressed vs float trajectory: "
          f"x {rel_rms(lx[0].cpu().numpy(), fx[0]):.3f} v {rel_rms(lv[0].cpu().numpy(), fv[0]):.3f}")
    assert ex <= K * TOL, ex
    assert ev <= K * TOL, ev
    c.close()
