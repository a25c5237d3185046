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
