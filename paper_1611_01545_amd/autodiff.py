"""Differentiable K-step particle-mesh trajectories on top of pm_step / pm_step_vjp.

The forward pass encodes the initial float particles into the compressed format
(Sec. 2.4), runs K steps, keeps every intermediate state as a checkpoint (about 9 bytes
per particle each, instead of 24 for float positions and velocities), and returns the
decoded final positions and velocities. The backward pass chains pm_step_vjp from the
last checkpoint to the first; the quantisation of the format is treated as the
identity (straight-through), and the encoder's permutation maps the first checkpoint's
stream order back to the caller's particle order. With compressed=False the float
states are the checkpoints and no quantisation happens.

All arithmetic runs in libpm; this module only orders the calls and moves pointers.
"""

from __future__ import annotations

import torch

from .pm import FloatSpecies, PMContext


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(actx, pm: PMContext, masses, dt: float, steps: int, compressed: bool,
                *xv):
        ns = len(masses)
        xs, vs = xv[:ns], xv[ns:]
        fl = [pm.float_species(x.detach(), v.detach(), m) for x, v, m in zip(xs, vs, masses)]
        if compressed:
            enc = [pm.encode(f, want_perm=True) for f in fl]
            state = [e[0] for e in enc]
            perms = [e[1] for e in enc]
        else:
            state, perms = fl, None
        traj = [state]
        for _ in range(steps):
            traj.append(pm.step(traj[-1], dt))
        final = traj[-1]
        if compressed:
            dec = [pm.decode(s) for s in final]
            outs = [d.x for d in dec] + [d.v for d in dec]
        else:
            outs = [s.x.clone() for s in final] + [s.v.clone() for s in final]
        actx.pm, actx.dt, actx.traj, actx.perms = pm, dt, traj[:-1], perms
        actx.ns = ns
        return tuple(outs)

    @staticmethod
    def backward(actx, *grads):
        pm, ns = actx.pm, actx.ns
        lx = [g.contiguous() if g is not None else None for g in grads[:ns]]
        lv = [g.contiguous() if g is not None else None for g in grads[ns:]]
        for i, st in enumerate(actx.traj[-1] if actx.traj else []):
            if lx[i] is None:
                lx[i] = torch.zeros((st.n, 3), dtype=torch.float32, device=pm.device)
            if lv[i] is None:
                lv[i] = torch.zeros((st.n, 3), dtype=torch.float32, device=pm.device)
        for state in reversed(actx.traj):
            lx, lv = pm.step_vjp(state, actx.dt, lx, lv)
        if actx.perms is not None:
            gx, gv = [], []
            for a, b, p in zip(lx, lv, actx.perms):
                ga = torch.empty_like(a)
                gb = torch.empty_like(b)
                ga[p] = a  # stream position j holds input particle p[j]
                gb[p] = b
                gx.append(ga)
                gv.append(gb)
            lx, lv = gx, gv
        return (None, None, None, None, None, *lx, *lv)


def trajectory(pm: PMContext, xs, vs, masses, dt: float, steps: int,
               compressed: bool = True):
    """K steps from float initial conditions; returns (final x list, final v list).

    xs, vs: per species float32 [n][3] device tensors (may require grad); masses: per
    species particle mass. The outputs are in the final stream order (cell order for
    compressed states; input order for float states) and are differentiable with respect
    to xs and vs."""
    if steps < 1:
        raise ValueError("steps must be >= 1")
    out = _Trajectory.apply(pm, list(masses), float(dt), int(steps), bool(compressed),
                            *xs, *vs)
    ns = len(masses)
    return list(out[:ns]), list(out[ns:])


def density_loss(pm: PMContext, species, rho_target: torch.Tensor) -> torch.Tensor:
    """L = sum_c (rho(c) - rho_t(c))^2 of float species given as (x, mass) pairs, with
    dL/dx from pm_loss_density_vjp."""
    return _DensityLoss.apply(pm, [m for _, m in species], rho_target,
                              *[x for x, _ in species])


class _DensityLoss(torch.autograd.Function):
    @staticmethod
    def forward(actx, pm: PMContext, masses, rho_target, *xs):
        sp = [FloatSpecies(x.detach().contiguous(), torch.zeros_like(x), m)
              for x, m in zip(xs, masses)]
        loss, g = pm.loss_density_vjp(sp, rho_target)
        actx.g = g
        return loss.reshape(()).to(torch.float32)

    @staticmethod
    def backward(actx, gl):
        return (None, None, None, *[gl * g for g in actx.g])
