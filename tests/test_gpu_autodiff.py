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


def test_float_trajectory_gradient_matches_oracle():
    from paper_1611_01545_amd.autodiff import density_loss, trajectory
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
    print(f"float trajectory gradient vs oracle: x {ex:.2e} v {ev:.2e}")
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
    ends in a different mesh cell between the two runs straddles a kink of the CIC
    weights and is redrawn. The loss is evaluated in float64 from the float32 density,
    so the difference quotient carries about 1e-7 L / h of rounding; the tolerance is
    the survey's 1e-2 relative."""
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
        for _ in range(K):
            st = c.step(st, wl.dt)
        loss, _ = c.loss_density_vjp(st, rho_t)
        return float(loss.item()), st[0].x.cpu().numpy()

    rng = np.random.default_rng(17)
    checked, errs = 0, []
    while checked < 64:
        i, a, which = int(rng.integers(sp.n)), int(rng.integers(3)), int(rng.integers(2))
        base = (sp.x.copy(), sp.v.copy())
        lp_in, lm_in = (base[0].copy(), base[1].copy()), (base[0].copy(), base[1].copy())
        lp_in[which][i, a] += np.float32(h)
        lm_in[which][i, a] -= np.float32(h)
        hp = float(lp_in[which][i, a]) - float(base[which][i, a])
        hm = float(base[which][i, a]) - float(lm_in[which][i, a])
        Lp, xp = final(*lp_in)
        Lm, xm = final(*lm_in)
        if np.any(np.floor(xp[i] * wl.n_mesh) != np.floor(xm[i] * wl.n_mesh)):
            continue  # the stencil straddles a CIC kink
        fd = (Lp - Lm) / (hp + hm)
        g = (gx if which == 0 else gv)[i, a]
        errs.append(abs(fd - g) / max(abs(g), 1e-3 * np.abs(gx).max()))
        checked += 1
    print(f"FD check: median rel err {np.median(errs):.2e}, max {np.max(errs):.2e}")
    assert np.median(errs) <= 1e-2
    c.close()
