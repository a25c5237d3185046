"""GPU: the torch.autograd wrapper over pm_step / pm_step_vjp (compressed checkpoints)."""

import numpy as np
import pytest
import torch

from gpu_util import ctx, rel_rms
from oracle import adjoint, mesh
from pmsynth import make_workload

pytestmark = pytest.mark.gpu


def _setup(K=2):
    wl = make_workload("adjoint_128", n_p_c=16, n_mesh=32, n_cell=16)
    tg = make_workload("adjoint_128", seed_offset=1, n_p_c=16, n_mesh=32, n_cell=16)
    rho_t = sum(mesh.deposit(s.x, s.mass, wl.n_mesh) for s in tg.species)
    return wl, rho_t, K


@pytest.mark.parametrize("full", [False, True], ids=["32^3-mesh", "adjoint_128"])
def test_float_trajectory_gradient_matches_oracle(full):
    """The autograd gradient through K float steps against the float64 oracle's
    adjoint: at a 32^3 mesh for 2 steps, and at the differentiable workload's full size
    (64^3 CDM, 128^3 mesh, 10 steps of dt 0.02). K chained float32 step adjoints, each
    within 1e-3 relative RMS, bound the error by K * 1e-3."""
    from paper_1611_01545_amd.autodiff import density_loss, trajectory
    if full:
        wl = make_workload("adjoint_128")
        tg = make_workload("adjoint_128", seed_offset=1)
        rho_t = sum(mesh.deposit(s.x, s.mass, wl.n_mesh) for s in tg.species)
        K = wl.steps
    else:
        wl, rho_t, K = _setup()
    sp = wl.species[0]
    c = ctx(wl.n_mesh, wl.n_cell)
    x0 = torch.from_numpy(sp.x).to(c.device).requires_grad_(True)
    v0 = torch.from_numpy(sp.v).to(c.device).requires_grad_(True)
    xs, vs = trajectory(c, [x0], [v0], [sp.mass], wl.dt, K, compressed=False)
    rt = torch.from_numpy(rho_t.astype(np.float32)).to(c.device)
    L = density_loss(c, [(xs[0], sp.mass)], rt)
    L.backward()
    rl, rx, rv = adjoint.grad_float_loss([(sp.x, sp.v, sp.mass)], rho_t, wl.n_mesh, wl.dt, K)
    assert abs(float(L.detach()) - rl) <= 1e-4 * rl
    ex = rel_rms(x0.grad.cpu().numpy(), rx[0])
    ev = rel_rms(v0.grad.cpu().numpy(), rv[0])
    print(f"float trajectory gradient vs oracle, {K} steps on {wl.n_mesh}^3: "
          f"x {ex:.2e} v {ev:.2e}", flush=True)
    assert ex <= K * 1e-3 and ev <= K * 1e-3, (ex, ev)
    c.close()


def test_compressed_trajectory_gradient_equals_manual_chain():
    from paper_1611_01545_amd.autodiff import density_loss, trajectory
    wl, rho_t, K = _setup()
    sp = wl.species[0]
    c = ctx(wl.n_mesh, wl.n_cell)
    x0 = torch.from_numpy(sp.x).to(c.device).requires_grad_(True)
    v0 = torch.from_numpy(sp.v).to(c.device).requires_grad_(True)
    xs, vs = trajectory(c, [x0], [v0], [sp.mass], wl.dt, K, compressed=True)
    rt = torch.from_numpy(rho_t.astype(np.float32)).to(c.device)
    L = density_loss(c, [(xs[0], sp.mass)], rt)
    L.backward()
    # the same chain through the raw calls
    st, perm = c.encode(c.float_species(sp.x, sp.v, sp.mass), want_perm=True)
    traj = [[st]]
    for _ in range(K):
        traj.append(c.step(traj[-1], wl.dt))
    loss, lx = c.loss_density_vjp(traj[-1], rt)
    lv = [torch.zeros_like(lx[0])]
    for k in range(K - 1, -1, -1):
        lx, lv = c.step_vjp(traj[k], wl.dt, lx, lv)
    gx = torch.empty_like(lx[0])
    gx[perm] = lx[0]
    gv = torch.empty_like(lv[0])
    gv[perm] = lv[0]
    assert abs(float(L.detach()) - float(loss.item())) <= 1e-6 * float(loss.item())
    assert rel_rms(x0.grad.cpu().numpy(), gx.cpu().numpy()) <= 1e-5
    assert rel_rms(v0.grad.cpu().numpy(), gv.cpu().numpy()) <= 1e-5
    c.close()


def test_gradient_matches_central_differences_adjoint_128():
    """The differentiable workload (64^3 CDM, 128^3 mesh, 10 steps of dt 0.02) on the
    float path: dL/dx0 and dL/dv0 from the adjoint chain against central differences
    with h = 1e-3 box units on 64 random components. A stencil whose perturbed particle
    sits in different mesh cells in the two runs at any step straddles a kink of the CIC
    weights (in the deposit or in the force gather) and is redrawn; on the remaining
    stencils the loss is smooth and the truncation error is O(h^2).

    Every component is held to |fd - g| <= 1e-2 max(|g|, g_rms), g_rms being the RMS of
    that gradient (dL/dx0 or dL/dv0) over all particles. The floor keeps components near
    zero from being judged on the rounding of the loss difference: the two runs round
    the float32 density and positions differently, and L(+h) - L(-h) divided by 2h
    carries that rounding whatever the size of the component."""
    from paper_1611_01545_amd.autodiff import density_loss, trajectory
    wl = make_workload("adjoint_128")
    tg = make_workload("adjoint_128", seed_offset=1)
    sp = wl.species[0]
    c = ctx(wl.n_mesh, wl.n_cell)
    rho_t = c.deposit([c.float_species(s.x, s.v, s.mass) for s in tg.species])
    K, h = wl.steps, 1e-3
    x0 = torch.from_numpy(sp.x).to(c.device).requires_grad_(True)
    v0 = torch.from_numpy(sp.v).to(c.device).requires_grad_(True)
    xs, _ = trajectory(c, [x0], [v0], [sp.mass], wl.dt, K, compressed=False)
    L = density_loss(c, [(xs[0], sp.mass)], rho_t)
    L.backward()
    gx, gv = x0.grad.double().cpu().numpy(), v0.grad.double().cpu().numpy()

    def final(x, v):
        st = [c.float_species(x, v, sp.mass)]
        cells = [np.floor(x[i] * wl.n_mesh)]
        for _ in range(K):
            st = c.step(st, wl.dt)
            cells.append(np.floor(st[0].x[i].cpu().numpy().astype(np.float64) * wl.n_mesh))
        loss, _ = c.loss_density_vjp(st, rho_t)
        return float(loss.item()), np.array(cells)

    rng = np.random.default_rng(17)
    rows = []
    while len(rows) < 64:
        i, a, which = int(rng.integers(sp.n)), int(rng.integers(3)), int(rng.integers(2))
        base = (sp.x.copy(), sp.v.copy())
        lp_in, lm_in = (base[0].copy(), base[1].copy()), (base[0].copy(), base[1].copy())
        lp_in[which][i, a] += np.float32(h)
        lm_in[which][i, a] -= np.float32(h)
        hp = float(lp_in[which][i, a]) - float(base[which][i, a])
        hm = float(base[which][i, a]) - float(lm_in[which][i, a])
        Lp, cp = final(*lp_in)
        Lm, cm = final(*lm_in)
        if np.any(cp != cm):
            continue  # the stencil straddles a CIC kink at some step
        fd = (Lp - Lm) / (hp + hm)
        g = (gx if which == 0 else gv)[i, a]
        rows.append((which, i, a, g, fd))
    g_rms = {0: float(np.sqrt(np.mean(gx ** 2))), 1: float(np.sqrt(np.mean(gv ** 2)))}
    errs = [abs(fd - g) / max(abs(g), g_rms[w]) for w, _, _, g, fd in rows]
    for w, i, a, g, fd in sorted(rows, key=lambda r: -abs(r[4] - r[3]))[:8]:
        print(f"  {'xv'[w]}[{i},{a}] adjoint {g:+.6e} fd {fd:+.6e} "
              f"|diff|/rms {abs(fd - g) / g_rms[w]:.2e}")
    print(f"FD check: L {float(L.detach()):.6e}, rms dL/dx {g_rms[0]:.3e}, "
          f"rms dL/dv {g_rms[1]:.3e}; median rel err {np.median(errs):.2e}, "
          f"max {np.max(errs):.2e}", flush=True)
    bad = [(r, e) for r, e in zip(rows, errs) if e > 1e-2]
    assert not bad, bad
    c.close()
