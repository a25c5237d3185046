"""Throughput of the particle-mesh step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config large_2048|tile_1024]

One "step" is one pass of the whole hot path over one batch of particles: cell
offsets, CIC deposit of both species, the fused FFT force solve, interpolate-kick-
drift-re-encode and the stable re-sort of both compressed streams (pm_step). Inputs
are resident in HBM before the timed region; W untimed warm-up steps are followed by
exactly K timed steps bracketed by device synchronisation.

The default workload is the largest that fits one GPU: 512^3 CDM + 1024^3 neutrinos
(1.21 G particles) on a 2048^3 mesh. Printed: one JSON line with the contract fields, a
roofline object for the dominant kernel and for the deposit and the interpolate-kick-
drift (algorithmic bytes per launch over the HIP-event launch duration measured on the
stream the kernels run on), the per-stage breakdown, the peak HBM footprint, the
fraction of particles whose position code does not change in a step, the comparison
of three compressed float32 steps with an all-float64 uncompressed run on the
[0, 128 Delta)^3 sub-box, the step with the two-level force of Sec. 2.1 (coarse
long-range mesh n/4, fine short-range mesh n, with and without the PP force), the step
and frozen fraction with 2-byte positions and with 1-byte velocities, the
1024^3 tile's step, PP, two-level and step-adjoint rates, and the oracle's own
throughput on a bounded sample (CPU baseline).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PM particle-updates/s (fwd and fwd+adjoint) at 1 GPU; % HBM roofline; err vs FP64"
HBM_PEAK_GBS = 8000.0

WORKLOAD_TEXT = {
    "large_2048": "the largest single-GPU workload: 512^3 CDM + 1024^3 neutrinos (1.21 G "
                  "particles), 2048^3 FP32 mesh, compressed particles (n_cell 512), dt "
                  "0.005, seed 11/111",
    "tile_1024": "one GPU's production-shaped tile: 256^3 CDM + 512^3 neutrinos, 1024^3 "
                 "FP32 mesh, compressed particles (n_cell 256), dt 0.005, seed 0",
    "two_species_256": "two-species step: 128^3 CDM + 256^3 neutrinos, 256^3 FP32 mesh, "
                       "compressed particles (n_cell 128), dt 0.01, seed 2/102",
}


# HBM bytes per launch of the dominant kernel from two rocprofv3 counter runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch; commands and calibration in
# profiles/hbm_traffic_<workload>.md), each scaled by what the counter reads for a kernel
# that reads and writes exactly 1 GiB. A record holds only for the kernel sources it was
# taken on (sha256 over `sources`); otherwise the traffic is reported as null.
MEASURED_TRAFFIC = {
    ("deposit", "tile_1024"): {
        "kernel": "k_deposit_tile<4, 1>",
        "sources": ["paper_1611_01545_amd/csrc/pm_deposit.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h",
                    "paper_1611_01545_amd/csrc/pm_codec.h",
                    "paper_1611_01545_amd/csrc/pm_scan.h"],
        "sha256": "b9a87e867dd2bf2cbf2a0cc2afdd62c96ded767a8296bfd572bb2c7e4006dc23",
        "fetch_kib": 509670.50, "fetch_factor": 1.99992,
        "write_kib": 4195298.69, "write_factor": 1.0,
    },
    ("fft_x_r2c", "tile_1024"): {
        "kernel": "k_row_r2c<512>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 2097307.62, "fetch_factor": 1.99992,
        "write_kib": 4202753.28, "write_factor": 1.0,
    },
    ("fft_y_fwd", "tile_1024"): {
        "kernel": "k_col_fft<1024, 16, -1, 0>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 2097320.19, "fetch_factor": 1.99992,
        "write_kib": 4194304.00, "write_factor": 1.0,
    },
    ("fft_z", "tile_1024"): {
        "kernel": "k_col_zconv<1024, 16, 0, true>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 2628255.31, "fetch_factor": 1.99992,
        "write_kib": 4194304.00, "write_factor": 1.0,
    },
    ("fft_y_inv", "tile_1024"): {
        "kernel": "k_col_fft<1024, 16, 1, 0>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 2097342.38, "fetch_factor": 1.99992,
        "write_kib": 4194304.12, "write_factor": 1.0,
    },
    ("fft_x_c2r", "tile_1024"): {
        "kernel": "k_row_c2r<512>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 2132485.69, "fetch_factor": 1.99992,
        "write_kib": 4194304.00, "write_factor": 1.0,
    },
    ("force_grad", "tile_1024"): {
        "kernel": "k_grad4",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 4654232.88, "fetch_factor": 1.99992,
        "write_kib": 12583241.62, "write_factor": 1.0,
    },
    ("interp_kick_drift", "tile_1024"): {
        "kernel": "k_kick_pair<256, 4, 1, 2>",
        "sources": ["paper_1611_01545_amd/csrc/pm_kick.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h",
                    "paper_1611_01545_amd/csrc/pm_codec.h",
                    "paper_1611_01545_amd/csrc/pm_scan.h"],
        "sha256": "b0a02528713e05ab4f8f47f7431efcc8e69725f6a97ff51bc2254cfa6440b90d",
        "fetch_kib": 8184960.06, "fetch_factor": 1.99992,
        "write_kib": 2258737.00, "write_factor": 1.0,
    },
    ("deposit", "large_2048"): {
        "kernel": "k_deposit_tile<4, 1>",
        "sources": ["paper_1611_01545_amd/csrc/pm_deposit.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h",
                    "paper_1611_01545_amd/csrc/pm_codec.h",
                    "paper_1611_01545_amd/csrc/pm_scan.h"],
        "sha256": "b9a87e867dd2bf2cbf2a0cc2afdd62c96ded767a8296bfd572bb2c7e4006dc23",
        "fetch_kib": 4074093.69, "fetch_factor": 1.99991,
        "write_kib": 33555662.69, "write_factor": 1.0,
    },
    ("fft_x_r2c", "large_2048"): {
        "kernel": "k_row_r2c<1024>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 16778414.75, "fetch_factor": 1.99991,
        "write_kib": 33587757.28, "write_factor": 1.0,
    },
    ("fft_y_fwd", "large_2048"): {
        "kernel": "k_col_fft<2048, 16, -1, 0>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 16817661.50, "fetch_factor": 1.99991,
        "write_kib": 33554432.00, "write_factor": 1.0,
    },
    ("fft_z", "large_2048"): {
        "kernel": "k_col_zconv<2048, 16, 0, true>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 24430745.19, "fetch_factor": 1.99991,
        "write_kib": 41418787.88, "write_factor": 1.0,
    },
    ("fft_y_inv", "large_2048"): {
        "kernel": "k_col_fft<2048, 16, 1, 0>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 16816735.56, "fetch_factor": 1.99991,
        "write_kib": 33554432.00, "write_factor": 1.0,
    },
    ("fft_x_c2r", "large_2048"): {
        "kernel": "k_row_c2r<1024>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 16794199.69, "fetch_factor": 1.99991,
        "write_kib": 33554432.50, "write_factor": 1.0,
    },
    ("force_grad", "large_2048"): {
        "kernel": "k_grad4",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "4e4f6cc89a2e2681720fffdfb260f2762f1fff1ff8fe8c7ac1a081a52cac4a3a",
        "fetch_kib": 37783092.44, "fetch_factor": 1.99991,
        "write_kib": 100666016.34, "write_factor": 1.0,
    },
    ("interp_kick_drift", "large_2048"): {
        "kernel": "k_kick_pair<256, 4, 1, 2>",
        "sources": ["paper_1611_01545_amd/csrc/pm_kick.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h",
                    "paper_1611_01545_amd/csrc/pm_codec.h",
                    "paper_1611_01545_amd/csrc/pm_scan.h"],
        "sha256": "b0a02528713e05ab4f8f47f7431efcc8e69725f6a97ff51bc2254cfa6440b90d",
        "fetch_kib": 66441099.62, "fetch_factor": 1.99991,
        "write_kib": 17960036.72, "write_factor": 1.0,
    },
}


def measured_traffic(stage: str, workload: str):
    import hashlib
    rec = MEASURED_TRAFFIC.get((stage, workload))
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != rec["sha256"]:
        return None  # the kernel changed since the counters were taken
    return (rec["fetch_kib"] * 1024 * rec["fetch_factor"] +
            rec["write_kib"] * 1024 * rec["write_factor"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def stage_bytes(name: str, n: int, wl) -> float:
    """Algorithmic HBM bytes of one launch of a stage (the byte model)."""
    n3 = float(n) ** 3
    n2 = float(n) ** 2
    N = float(wl.n_particles)
    ns = len(wl.species)
    nc3 = float(wl.n_cell) ** 3
    return {
        "fft_x_r2c": 8 * n3 + 8 * n2,          # real mesh in, half spectrum + Nyquist out
        "fft_y_fwd": 8 * n3,                    # half spectrum in and out
        "fft_z": 8 * n3,                        # the potential's spectrum, in place
        "fft_y_inv": 8 * n3,                    # in place
        "fft_x_c2r": 8 * n3 + 8 * n2,           # half spectrum + Nyquist in, real out
        "force_grad": 16 * n3,                  # the potential in, three components out
        "deposit": 3 * N + ns * nc3 + 4 * n3,   # positions, counts, density
        # one launch moves every species: codes in and out, counts, the 3 force meshes
        "interp_kick_drift": 9 * N + 9 * N + 2 * ns * nc3 + 12 * n3,
        "resort": (18 * N + 2 * ns * nc3) / ns,
        "cell_offsets": nc3 + 8 * nc3,          # counts in, offsets out (per species)
    }.get(name, 0.0)


def cpu_baseline_and_error(ctx_cls, make_workload, base: str):
    """The oracle (FP64, numpy, one thread) timed on a bounded sample of the workload:
    the same recipe at 1/4 of the linear size, five compressed steps. The GPU step on
    the same sample is compared with the oracle's first step."""
    import numpy as np

    from oracle import codec, step

    c = {"large_2048": dict(n_p_c=64, n_p_nu=128, n_mesh=256, n_cell=64),
         "tile_1024": dict(n_p_c=64, n_p_nu=128, n_mesh=256, n_cell=64),
         "two_species_256": dict(n_p_c=32, n_p_nu=64, n_mesh=64, n_cell=32)}[base]
    frac = {"large_2048": "1/8", "tile_1024": "1/4", "two_species_256": "1/4"}[base]
    wl = make_workload(base, **c)
    ctx = ctx_cls(wl.n_mesh, wl.n_cell)
    dev = [ctx.encode(ctx.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    states = [ctx.to_host(d) for d in dev]
    masses = [sp.mass for sp in wl.species]
    n_steps = 5
    t0 = time.perf_counter()
    new, diag = step.step_compressed(states, masses, wl.n_mesh, wl.dt, wl.dt)
    cur = new
    for _ in range(n_steps - 1):
        cur, _ = step.step_compressed(cur, masses, wl.n_mesh, wl.dt, wl.dt)
    t_cpu = time.perf_counter() - t0
    # GPU on the same sample
    rho = ctx.deposit(dev)
    rho_h = rho.cpu().numpy().astype(np.float64)
    acc, amax = ctx.force(rho)
    acc_h = acc.cpu().numpy()
    out, perms = ctx.kick_drift_perm(dev, acc, amax, wl.dt, wl.dt)
    ctx.sync()
    ref_rho = diag["rho"]
    scale = np.maximum(np.abs(ref_rho), np.abs(ref_rho).mean())
    rho_err = float(np.max(np.abs(rho_h - ref_rho) / scale))
    am = diag["a_mesh"]
    f_err = float(np.sqrt(np.mean((acc_h - am) ** 2) / np.mean(am ** 2)))
    mism = 0
    tot = 0
    for o, d, p in zip(out, diag["species"], perms):
        h = ctx.to_host(o)
        u, _ = codec.decode_codes(h)
        uo = np.empty_like(u)
        uo[p.cpu().numpy()] = u
        mism += int(np.count_nonzero(uo != d["u_new"]))
        tot += u.size
    ctx.close()
    n = wl.n_particles
    return ({"value": n * n_steps / t_cpu, "unit": "particle-updates/s", "cores": 1,
             "kind": "oracle",
             "sample": f"{base} recipe at {frac} linear size ({c['n_p_c']}^3 CDM + "
                       f"{c['n_p_nu']}^3 nu, {c['n_mesh']}^3 mesh, n_cell {c['n_cell']}), "
                       f"{n_steps} compressed steps, numpy float64, one thread",
             "seconds": t_cpu},
            {"sample": f"{c['n_mesh']}^3 mesh, {n} particles, first step",
             "density_max_rel": rho_err, "force_rel_rms": f_err,
             "position_code_mismatch_frac": mism / max(1, tot)})


def adjoint_rates(ctx_cls, make_workload, torch, name: str, reps: int = 3):
    """Forward K compressed steps (keeping every state as a checkpoint), then the density
    loss and K step adjoints backward. Returns the median forward and backward times."""
    wl = make_workload(name)
    tg = make_workload(name, seed_offset=1)
    K = wl.steps
    ctx = ctx_cls(wl.n_mesh, wl.n_cell)
    tgt = [ctx.float_species(sp.x, sp.v, sp.mass) for sp in tg.species]
    rho_t = ctx.deposit(tgt)
    st0 = [ctx.encode(ctx.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    traj = [st0] + [[ctx.empty_like(s) for s in st0] for _ in range(K)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    t_f, t_b = [], []
    for r in range(reps + 1):
        ctx.sync()
        ev[0].record()
        for k in range(K):
            ctx.step(traj[k], wl.dt, out=traj[k + 1])
        ev[1].record()
        _, lx = ctx.loss_density_vjp(traj[K], rho_t)
        lv = [torch.zeros_like(t) for t in lx]
        for k in range(K - 1, -1, -1):
            lx, lv = ctx.step_vjp(traj[k], wl.dt, lx, lv)
        ev[2].record()
        torch.cuda.synchronize()
        if r > 0:  # the first repetition warms up
            t_f.append(ev[0].elapsed_time(ev[1]))
            t_b.append(ev[1].elapsed_time(ev[2]))
    ctx.close()
    t_f = sorted(t_f)[len(t_f) // 2]
    t_b = sorted(t_b)[len(t_b) // 2]
    N = wl.n_particles
    return {"workload": name, "particles": N, "n_mesh": wl.n_mesh, "steps": K,
            "fwd_ms": t_f, "bwd_ms": t_b, "bwd_over_fwd": t_b / t_f,
            "fwd_updates_per_s": N * K / (t_f * 1e-3),
            "fwd_adjoint_updates_per_s": N * K / ((t_f + t_b) * 1e-3)}


def mem_used(torch) -> int:
    free, total = torch.cuda.mem_get_info()
    return total - free


def timed_steps(ctx, A, B, wl, torch, steps, warmup):
    """W warm-up steps, then K timed steps of pm_step (ping-pong A <-> B) with the stage
    profiler on. Returns (ms_step, value, stages, cur)."""
    cur, nxt = A, B
    for _ in range(warmup):
        ctx.step(cur, wl.dt, out=nxt)
        cur, nxt = nxt, cur
    ctx.sync()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step(cur, wl.dt, out=nxt)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_step = (t1 - t0) * 1e3 / steps
    value = wl.n_particles * steps / (t1 - t0)
    stages = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        per = ms / cnt
        b = stage_bytes(name, wl.n_mesh, wl)
        stages[name] = {"ms_per_step": ms / steps, "launches_per_step": cnt / steps,
                        "ms_per_launch": per,
                        "gbs": (b / (per * 1e-3) / 1e9) if b else None}
    return ms_step, value, stages, cur


def stage_kernel(name: str, n: int):
    """The one kernel template a stage's launches run at mesh side n (the bench workloads:
    4 mesh cells per compression cell, bricks of 4^3 cells), or None when the stage runs
    several: a kernel's roofline needs that kernel's own launch duration. The force takes
    one transform of the potential (one launch per pass) and the stencil pass for its
    three components."""
    return {
        "deposit": "k_deposit_tile<4, 1>",
        "fft_x_r2c": f"k_row_r2c<{n // 2}>",
        "fft_y_fwd": f"k_col_fft<{n}, 16, -1, 0>",
        "fft_z": f"k_col_zconv<{n}, 16, 0, true>",
        "fft_y_inv": f"k_col_fft<{n}, 16, 1, 0>",
        "fft_x_c2r": f"k_row_c2r<{n // 2}>",
        "force_grad": "k_grad4",
        "interp_kick_drift": "k_kick_pair<256, 4, 1, 2>",
    }.get(name)


def dominant_kernel_stage(stages, n: int, wl) -> str:
    """The stage of the kernel with the largest time per step, among the stages that run
    one kernel template."""
    return max((k for k in stages if stage_bytes(k, n, wl) > 0 and stage_kernel(k, n)),
               key=lambda k: stages[k]["ms_per_step"])


def roofline_of(stages, name, wl, config):
    st = stages[name]
    return {"bound": "hbm", "kernel": stage_kernel(name, wl.n_mesh) or name, "stage": name,
            "achieved": st["gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": st["gbs"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(name, config),
            "bytes_per_launch": stage_bytes(name, wl.n_mesh, wl),
            "ms_per_launch": st["ms_per_launch"]}


def stream_cells(cs, torch):
    """Cell key of every particle of a compressed stream, in stream order (int32)."""
    nc3 = cs.count.numel()
    cnt = cs.count.to(torch.int64)
    ne = int(cs.header()["n_esc"])
    if ne:
        e = cs.esc[:ne]
        cnt[e[:, 0]] = e[:, 1]
    keys = torch.arange(nc3, dtype=torch.int32, device=cs.count.device)
    return torch.repeat_interleave(keys, cnt, output_size=cs.n)


def moved_fraction(old, new, perm, torch):
    """Fraction of particles whose position code changed in a step: new stream
    particle j was old stream particle perm[j]."""
    c_old = stream_cells(old, torch)
    c_new = stream_cells(new, torch)
    moved = c_new != c_old[perm]
    del c_old, c_new
    moved |= (new.pos != old.pos[perm]).any(dim=1)
    return float(moved.float().mean().item())


SUB = 128  # side of the comparison sub-box in mesh nodes


def large_comparison(ctx, wl, torch, log):
    """Three compressed float32 steps from the encoded initial state, through the
    separate calls (pm_deposit, pm_force, pm_kick_drift_perm) so that the density, the
    force and the particle identities can be read: the sub-box of the first density and
    force, the fraction of frozen position codes per step and species, the final
    positions of the particles that start in the sub-box. Returns a dict of host arrays
    and figures; frees its device buffers."""
    import numpy as np
    n = wl.n_mesh
    dev = ctx.device
    A, perm0 = [], []
    for sp in wl.species:
        fs = ctx.float_species(sp.x, sp.v, sp.mass)
        cs, p = ctx.encode(fs, want_perm=True)
        del fs
        A.append(cs)
        perm0.append(p)
    B = [ctx.empty_like(s) for s in A]
    acc = torch.empty((3, n, n, n), dtype=torch.float32, device=dev)
    a_max = torch.zeros(1, dtype=torch.float32, device=dev)
    peak = mem_used(torch)
    idx = perm0  # stream position -> input index
    frozen = []
    rho_sub = a_sub = None
    cur, nxt = A, B
    for k in range(wl.steps):
        ctx.deposit(cur, rho=acc[0])
        if k == 0:
            rho_sub = acc[0, :SUB, :SUB, :SUB].cpu().numpy()
        ctx.force(acc[0], acc=acc, a_max=a_max)
        if k == 0:
            a_sub = acc[:, :SUB, :SUB, :SUB].cpu().numpy()
        nxt, perms = ctx.kick_drift_perm(cur, acc, a_max, wl.dt, wl.dt, out=nxt)
        peak = max(peak, mem_used(torch))
        frozen.append([1.0 - moved_fraction(o, q, p, torch) for o, q, p in zip(cur, nxt, perms)])
        idx = [i[p] for i, p in zip(idx, perms)]
        del perms
        cur, nxt = nxt, cur
        log(f"[bench] comparison step {k + 1}: frozen fraction {frozen[-1]}")
    del acc, nxt, A, B, perm0
    torch.cuda.empty_cache()
    final = {}
    for s_, (cs, ix, sp) in enumerate(zip(cur, idx, wl.species)):
        sel = np.flatnonzero(np.all(sp.x < np.float32(SUB / n), axis=1))
        fs = ctx.decode(cs)
        inv = torch.empty(cs.n, dtype=torch.int64, device=dev)
        inv[ix] = torch.arange(cs.n, dtype=torch.int64, device=dev)
        j = inv[torch.from_numpy(sel).to(dev)]
        final[s_] = (sel, fs.x[j].cpu().numpy().astype(np.float64))
        del fs, inv, j
    del cur, idx
    torch.cuda.empty_cache()
    return {"rho_sub": rho_sub, "a_sub": a_sub, "frozen": frozen, "final": final,
            "peak_used": peak}


def window_density_oracle(wl):
    """CPU oracle density on the sub-box nodes from the decoded (bin-centre) initial
    positions of the particles that reach them: the GPU deposit's own input."""
    import numpy as np

    from oracle import codec, mesh
    n = wl.n_mesh
    lo, hi = np.float32(SUB / n), np.float32((n - 1) / n)
    rho = np.zeros((SUB, SUB, SUB))
    for sp in wl.species:
        near = np.all((sp.x < lo) | (sp.x >= hi), axis=1)
        x = sp.x[near]
        u = codec.position_codes(x, wl.n_cell)
        xd = (u.astype(np.float64) + 0.5) / (256 * wl.n_cell)
        rho += mesh.deposit_window(xd, sp.mass, n, (0, 0, 0), SUB)
    return rho


def fp64_reference(wl, torch, log):
    """The uncompressed float64 run (oracle.fp64_torch) of the same workload from the
    generator's float32 positions and velocities: sub-box density and force of the first
    step, positions after all steps, and its own time per step."""
    import numpy as np

    from oracle import fp64_torch
    dev = torch.device("cuda")
    sp = [(torch.from_numpy(s.x).to(dev).to(torch.float64),
           torch.from_numpy(s.v).to(dev).to(torch.float64), s.mass) for s in wl.species]
    kept = {}

    def keep(key, m):
        if "first" not in kept:
            kept[key] = m[:SUB, :SUB, :SUB].cpu().numpy()

    times = []
    for k in range(wl.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fp64_torch.step_float(sp, wl.n_mesh, wl.dt, wl.dt, keep=keep)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        kept["first"] = True
        log(f"[bench] float64 reference step {k + 1}: {times[-1]:.1f} s")
    peak = mem_used(torch)
    final = {}
    for s_, (x, _, _) in enumerate(sp):
        sel = np.flatnonzero(np.all(wl.species[s_].x < np.float32(SUB / wl.n_mesh), axis=1))
        final[s_] = x[torch.from_numpy(sel).to(dev)].cpu().numpy()
    del sp
    torch.cuda.empty_cache()
    return {"rho_sub": kept["rho"], "a_sub": np.stack([kept[0], kept[1], kept[2]]),
            "final": final, "s_per_step": float(np.median(times)), "peak_used": peak}


def compare_figures(gpu, ref, rho_oracle, wl):
    import numpy as np
    mean = sum(sp.mass * sp.n for sp in wl.species)  # mean density (unit box)
    scale = np.maximum(np.abs(ref["rho_sub"]), mean)
    out = {
        "sub_box": f"[0, {SUB} Delta)^3 of the {wl.n_mesh}^3 mesh",
        "density_max_rel_vs_fp64": float(np.max(np.abs(gpu["rho_sub"] - ref["rho_sub"]) / scale)),
        "density_rel_rms_vs_fp64": float(np.sqrt(np.mean((gpu["rho_sub"] - ref["rho_sub"]) ** 2)
                                                 / np.mean(ref["rho_sub"] ** 2))),
        "density_max_rel_vs_oracle_same_input": float(np.max(
            np.abs(gpu["rho_sub"] - rho_oracle) / np.maximum(np.abs(rho_oracle), mean))),
        "force_rel_rms_vs_fp64": float(np.sqrt(np.mean((gpu["a_sub"] - ref["a_sub"]) ** 2) /
                                               np.mean(ref["a_sub"] ** 2))),
    }
    q = 1.0 / (256 * wl.n_cell)
    for s_, name in enumerate(sp.name for sp in wl.species):
        sel_g, xg = gpu["final"][s_]
        xr = ref["final"][s_]
        d = np.abs(xg - xr)
        d = np.minimum(d, 1.0 - d)
        out[f"position_{name}_particles"] = int(sel_g.size)
        out[f"position_{name}_max_abs"] = float(d.max()) if d.size else 0.0
        out[f"position_{name}_rms_abs"] = float(np.sqrt(np.mean(d ** 2))) if d.size else 0.0
    out["position_quantum"] = q
    out["after_steps"] = wl.steps
    out["note"] = ("float32 mesh and FFT with compressed fixed-point positions, against "
                   "float64 throughout from the uncompressed initial state: the position "
                   "differences include the compression's quantisation (at most q/2 per "
                   "axis at the start, q = L / (256 n_cell)) and its frozen drifts")
    return out


def two_level_rates(PMContext, wl, cur, brick, torch, log, steps, warmup, ms_one):
    """The two-level force of Sec. 2.1 (pm_step_p3m): coarse long-range mesh n/4, r_s =
    1.25 coarse cells, fine short-range mesh n, on the compressed states cur; timed
    without and with the PP force (r_soft = L / (20 n_p)), stage times of both meshes."""
    fine, coarse = PMContext.two_level(wl.n_mesh, wl.n_cell, brick=brick)
    nxt = [fine.empty_like(s) for s in cur]
    r_soft = 1.0 / (20 * 2 * wl.n_cell)
    res = {"coarse_mesh": coarse.n_mesh, "r_split_coarse_cells": 1.25,
           "r_split": fine.r_split}
    for tag, rs in (("p3m_step", 0.0), ("p3m_step_with_pp", r_soft)):
        for _ in range(max(1, warmup)):
            fine.step_p3m(coarse, cur, wl.dt, r_soft=rs, out=nxt)
        fine.sync()
        fine.profile(True)
        coarse.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fine.step_p3m(coarse, cur, wl.dt, r_soft=rs, out=nxt)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        pf, pc = fine.profile_read(), coarse.profile_read()
        fine.profile(False)
        coarse.profile(False)
        res[tag] = {
            "ms_per_step": ms, "value": wl.n_particles / (ms * 1e-3),
            "over_one_level_step": ms / ms_one,
            "fine_stage_ms": {k: v[0] / steps for k, v in pf.items() if v[1]},
            "coarse_stage_ms": {k: v[0] / steps for k, v in pc.items() if v[1]}}
        if rs > 0:
            res[tag]["r_soft"] = rs
        log(f"[bench] two-level {tag}: {ms:.3f} ms/step ({ms / ms_one:.2f}x the one-level "
            "step)")
    fine.close()
    coarse.close()
    del nxt
    torch.cuda.empty_cache()
    return res


def width_rates(PMContext, wl, torch, log, steps, warmup, ms_one,
                pairs=((2, 2), (1, 1))):
    """Adjustable code widths (Sec. 2.4, closing remark: 8- or 16-bit positions and
    velocities): for each (position bytes, velocity bytes) pair, the pm_step rate on the
    same particles and, per species, the fraction of position codes one step leaves
    unchanged (from a step with the PP force cut everywhere, r_soft = L, which is pm_step
    with the re-sort reported)."""
    from paper_1611_01545_amd import widths_word
    res = {}
    for pb, vb in pairs:
        ctx = PMContext(wl.n_mesh, wl.n_cell)
        w = widths_word(pb, vb)
        A = []
        for sp in wl.species:
            fs = ctx.float_species(sp.x, sp.v, sp.mass)
            A.append(ctx.encode(fs, widths=w))
            del fs
        B = [ctx.empty_like(s) for s in A]
        B, perms = ctx.step_pp(A, wl.dt, ctx.box, out=B, want_perm=True)
        frozen = {sp.name: 1.0 - moved_fraction(a, b, p, torch)
                  for sp, a, b, p in zip(wl.species, A, B, perms)}
        del perms
        ms, value, _, cur = timed_steps(ctx, A, B, wl, torch, steps, warmup)
        res[f"{pb}_{vb}"] = {
            "position_bytes": pb, "velocity_bytes": vb,
            "bytes_per_particle": 3 * (pb + vb),
            "ms_per_step": ms, "value": value, "over_paper_widths": ms / ms_one,
            "frozen_fraction": frozen}
        log(f"[bench] code widths ({pb}, {vb}): {ms:.3f} ms/step, frozen "
            + ", ".join(f"{k} {v:.4f}" for k, v in frozen.items()))
        ctx.close()
        del A, B, cur
        torch.cuda.empty_cache()
    return res


def tile_extra(PMContext, make_workload, torch, log, steps, warmup, adjoint=True):
    """The 1024^3 tile (256^3 + 512^3): step rate over its 8 seeds, the PP, two-level and
    code-width steps, and the step adjoint at that size."""
    import numpy as np
    wl = make_workload("tile_1024")
    ctx = PMContext(wl.n_mesh, wl.n_cell)
    A = [ctx.encode(ctx.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    B = [ctx.empty_like(s) for s in A]
    ctx.sync()
    ms_step, value, stages, cur = timed_steps(ctx, A, B, wl, torch, steps, warmup)
    out = {"workload": WORKLOAD_TEXT["tile_1024"], "particles": wl.n_particles,
           "ms_per_step": ms_step, "value": value,
           "deposit_frac": stages["deposit"]["gbs"] / HBM_PEAK_GBS,
           "interp_kick_drift_frac": stages["interp_kick_drift"]["gbs"] / HBM_PEAK_GBS}
    log(f"[bench] tile_1024: {ms_step:.3f} ms/step, {value:.3e} particle-updates/s")
    # the tile's 8 random seeds (seed 0 above): each re-generated, encoded and stepped
    # `steps` times on the same context
    per_seed = [ms_step]
    for seed in range(1, 8):
        w2 = make_workload("tile_1024", seed_offset=seed)
        A2 = [ctx.encode(ctx.float_species(sp.x, sp.v, sp.mass)) for sp in w2.species]
        B2 = [ctx.empty_like(s_) for s_ in A2]
        ms2, _, _, _ = timed_steps(ctx, A2, B2, w2, torch, steps, min(warmup, 1))
        per_seed.append(ms2)
        del w2, A2, B2
    torch.cuda.empty_cache()
    out["seeds"] = {"ms_per_step": per_seed, "mean_ms": float(np.mean(per_seed)),
                    "min_ms": float(np.min(per_seed)), "max_ms": float(np.max(per_seed)),
                    "mean_value": wl.n_particles / (float(np.mean(per_seed)) * 1e-3)}
    log(f"[bench] tile_1024 over 8 seeds: {np.mean(per_seed):.3f} ms/step "
        f"({np.min(per_seed):.3f}-{np.max(per_seed):.3f})")
    # the same step with the cell-local PP force of eq. (4), r_soft = L / (20 n_p)
    r_soft = 1.0 / (20 * 2 * wl.n_cell)
    nxt = [ctx.empty_like(s) for s in cur]
    ctx.step_pp(cur, wl.dt, r_soft, out=nxt)
    ctx.sync()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.step_pp(cur, wl.dt, r_soft, out=nxt)
    torch.cuda.synchronize()
    t_pp = (time.perf_counter() - t0) * 1e3 / steps
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_pp, n_pp = prof["pp"]
    out["pp_step"] = {"ms_per_step": t_pp, "pp_kernel_ms": ms_pp / max(1, n_pp),
                      "r_soft": r_soft,
                      "note": "pm_step_pp: the step with the cell-local PP force added"}
    del nxt
    log(f"[bench] tile_1024 with the PP force: {t_pp:.3f} ms/step "
        f"(PP kernel {ms_pp / max(1, n_pp):.3f} ms)")
    out["two_level"] = two_level_rates(PMContext, wl, cur, ctx.brick, torch, log, steps,
                                       warmup, ms_step)
    out["code_widths"] = width_rates(PMContext, wl, torch, log, steps, warmup, ms_step)
    if adjoint:
        lx = [torch.ones((sp.n, 3), dtype=torch.float32, device=ctx.device) for sp in cur]
        lv = [torch.ones_like(t) for t in lx]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        t_vjp = []
        for r in range(3):
            ev[0].record()
            gx, gv = ctx.step_vjp(cur, wl.dt, lx, lv)
            ev[1].record()
            torch.cuda.synchronize()
            if r > 0:
                t_vjp.append(ev[0].elapsed_time(ev[1]))
        del gx, gv, lx, lv
        t_vjp = min(t_vjp)
        out.update({"step_vjp_ms": t_vjp, "vjp_over_step": t_vjp / ms_step,
                    "fwd_adjoint_updates_per_s": wl.n_particles / ((ms_step + t_vjp) * 1e-3)})
        log(f"[bench] tile_1024 step adjoint {t_vjp:.3f} ms ({t_vjp / ms_step:.2f}x the step)")
    ctx.close()
    del A, B, cur
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="large_2048", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the step-adjoint timings (fwd+adjoint rates)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the float64 sub-box comparison of the large workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 1024^3 tile measured beside the large workload")
    ap.add_argument("--no-two-level", action="store_true",
                    help="skip the two-level force (pm_step_p3m) timings")
    ap.add_argument("--no-widths", action="store_true",
                    help="skip the 2-byte-position and 1-byte-velocity code widths")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, run one elementwise kernel that reads and "
                         "writes exactly 1 GiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this "
              "single-GPU build (the path's sharding is described in DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1611_01545_amd import PMContext
    from pmsynth import make_workload

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    t = time.perf_counter()
    wl = make_workload(args.config)
    log(f"[bench] workload {args.config}: {wl.n_particles} particles, mesh {wl.n_mesh}^3 "
        f"({time.perf_counter() - t:.1f} s to generate)")
    used0 = mem_used(torch)
    ctx = PMContext(wl.n_mesh, wl.n_cell)
    n_tot = wl.n_particles
    sizes = PMContext.query_sizes(wl.n_mesh, wl.n_cell, ctx.brick, n_tot, len(wl.species))
    large = args.config == "large_2048"
    cmp_gpu = None
    if large and not args.no_compare:
        log("[bench] comparison run: 3 compressed steps through the separate calls")
        cmp_gpu = large_comparison(ctx, wl, torch, log)
    A = [ctx.encode(ctx.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    B = [ctx.empty_like(s) for s in A]
    ctx.sync()
    log("[bench] encoded; warming up")
    ms_step, value, stages, cur = timed_steps(ctx, A, B, wl, torch, args.steps, args.warmup)
    peak_step = mem_used(torch) - used0
    log(f"[bench] {ms_step:.3f} ms/step, {value:.3e} particle-updates/s")
    dom = dominant_kernel_stage(stages, wl.n_mesh, wl)
    roofline = roofline_of(stages, dom, wl, args.config)
    for k, st in stages.items():
        if st["gbs"] is not None:
            st["frac"] = st["gbs"] / HBM_PEAK_GBS
            st["traffic"] = measured_traffic(k, args.config)
    total_model = sum(stage_bytes(k, wl.n_mesh, wl) * stages[k]["launches_per_step"]
                      for k in stages)
    step_frac = total_model / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=ctx.device)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b

    adj = None
    if not large and not args.no_adjoint:
        log("[bench] step adjoint at the same workload")
        lx = [torch.ones((sp.n, 3), dtype=torch.float32, device=ctx.device) for sp in cur]
        lv = [torch.ones_like(t) for t in lx]
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        t_vjp = []
        for r in range(3):
            ev[0].record()
            gx, gv = ctx.step_vjp(cur, wl.dt, lx, lv)
            ev[1].record()
            torch.cuda.synchronize()
            if r > 0:
                t_vjp.append(ev[0].elapsed_time(ev[1]))
        del gx, gv, lx, lv
        t_vjp = min(t_vjp)
        adj = {"step_vjp_ms": t_vjp, "vjp_over_step": t_vjp / ms_step,
               "fwd_adjoint_updates_per_s": wl.n_particles / ((ms_step + t_vjp) * 1e-3)}
        log(f"[bench] step adjoint {t_vjp:.3f} ms ({t_vjp / ms_step:.2f}x the step)")
    brick = ctx.brick
    ctx.close()
    two_level = None
    if not args.no_two_level:
        # the one-level context is gone; the compressed states stay on the device
        log("[bench] two-level force (pm_step_p3m)")
        two_level = two_level_rates(PMContext, wl, cur, brick, torch, log, args.steps,
                                    args.warmup, ms_step)
    del A, B, cur
    torch.cuda.empty_cache()
    widths = None
    if not args.no_widths:
        log("[bench] adjustable code widths")
        widths = width_rates(PMContext, wl, torch, log, args.steps, args.warmup, ms_step)

    footprint = {"timed_steps_gb": peak_step / 1e9,
                 "query_sizes_gb": {k: v / 1e9 for k, v in sizes.items()},
                 "note": "device memory in use (hipMemGetInfo) above the level before the "
                         "context: after the timed steps (context tables and meshes, grown "
                         "scratch, two compressed copies of every species), and at the "
                         "peak of the comparison run (which also holds a caller-owned "
                         "force mesh, permutations and the frozen-fraction counts)"}
    if cmp_gpu is not None:
        footprint["comparison_run_gb"] = (cmp_gpu["peak_used"] - used0) / 1e9

    compare, frozen = None, None
    if cmp_gpu is not None:
        frozen = {"per_step": [dict(zip((sp.name for sp in wl.species), f))
                               for f in cmp_gpu["frozen"]],
                  "definition": "fraction of particles whose position code is unchanged "
                                "by the step (|v' c_d S / L| < 1/2 on every axis)"}
        log("[bench] oracle density on the sub-box (CPU)")
        rho_or = window_density_oracle(wl)
        log("[bench] float64 reference run")
        ref = fp64_reference(wl, torch, log)
        compare = compare_figures(cmp_gpu, ref, rho_or, wl)
        compare["fp64_reference_s_per_step"] = ref["s_per_step"]
        footprint["fp64_reference_peak_gb"] = (ref["peak_used"] - used0) / 1e9

    extra = None
    if large and not args.no_extra:
        log("[bench] the 1024^3 tile")
        extra = tile_extra(PMContext, make_workload, torch, log, args.steps, args.warmup,
                           adjoint=not args.no_adjoint)
        if not args.no_adjoint:
            adj = {"tile_1024": {k: extra[k] for k in ("step_vjp_ms", "vjp_over_step",
                                                      "fwd_adjoint_updates_per_s")}}
    if not args.no_adjoint:
        a128 = adjoint_rates(PMContext, make_workload, torch, "adjoint_128")
        adj = adj or {}
        adj["adjoint_128"] = a128
        log(f"[bench] adjoint_128: fwd {a128['fwd_ms']:.2f} ms, bwd {a128['bwd_ms']:.2f} ms "
            f"for {a128['steps']} steps")

    cpu, err = None, None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline + error vs FP64 on a sample")
        cpu, err = cpu_baseline_and_error(PMContext, make_workload, args.config)

    out = {
        "metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.config], "name": args.config,
                   "particles": wl.n_particles, "n_mesh": wl.n_mesh, "n_cell": wl.n_cell,
                   "brick": PMContext.default_brick(wl.n_mesh, wl.n_cell),
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "roofline_deposit": roofline_of(stages, "deposit", wl, args.config),
        "roofline_interp_kick_drift": roofline_of(stages, "interp_kick_drift", wl, args.config),
        "step_hbm_frac_model": step_frac,
        "stages": stages,
        "hbm_footprint": footprint,
        "frozen_fraction": frozen,
        "vs_fp64_sub_box": compare,
        "two_level": two_level,
        "code_widths": widths,
        "tile_1024": extra,
        "adjoint": adj,
        "err_vs_fp64": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
