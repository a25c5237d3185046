"""Throughput of the particle-mesh step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config tile_1024]

One "step" is one pass of the whole hot path over one batch of particles: cell
offsets, CIC deposit of both species, the fused FFT force solve, interpolate-kick-
drift-re-encode and the stable re-sort of both compressed streams (pm_step). Inputs
are resident in HBM before the timed region; W untimed warm-up steps are followed by
exactly K timed steps bracketed by device synchronisation.

Printed: one JSON line with the contract fields, a roofline object for the dominant
kernel (algorithmic bytes per launch over the HIP-event launch duration measured on
the stream the kernel runs on), the per-stage breakdown, the error of the same path
against the FP64 oracle on a small sample of the workload, and the oracle's own
throughput on that sample (CPU baseline).
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
    ("interp_kick_drift", "tile_1024"): {
        "kernel": "k_kick_pair<256, 4>",
        "sources": ["paper_1611_01545_amd/csrc/pm_kick.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h",
                    "paper_1611_01545_amd/csrc/pm_codec.h"],
        "sha256": "1dc0117ead72af659fd28f6f6dc1cfa1f50eabd20de7c5455a87155bccba33e1",
        "fetch_kib": 8164916.25, "fetch_factor": 1.99988,
        "write_kib": 2200561.28, "write_factor": 1.0,
    },
    ("fft_x_c2r", "tile_1024"): {
        "kernel": "k_row_c2r<512>",
        "sources": ["paper_1611_01545_amd/csrc/pm_fft.hip",
                    "paper_1611_01545_amd/csrc/pm_common.h"],
        "sha256": "b4c65a62e4abf37a64be1ac3a81a194d3b65c53b2a438f4e666e0963fe4c84fc",
        "fetch_kib": 2101697.0, "fetch_factor": 1.99988,
        "write_kib": 4196763.0, "write_factor": 1.0,
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
        "fft_z": 12 * n3,                       # fused z pass, one in, two out
        "fft_y_inv": 10 * n3,                   # 2 launches: one in two out, one in one out
        "fft_x_c2r": 8 * n3 + 8 * n2,           # half spectrum + Nyquist in, real out
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

    c = {"tile_1024": dict(n_p_c=64, n_p_nu=128, n_mesh=256, n_cell=64),
         "two_species_256": dict(n_p_c=32, n_p_nu=64, n_mesh=64, n_cell=32)}[base]
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
             "sample": f"{base} recipe at 1/4 linear size ({c['n_p_c']}^3 CDM + "
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="tile_1024", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the step-adjoint timings (fwd+adjoint rates)")
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
    ctx = PMContext(wl.n_mesh, wl.n_cell)
    A = [ctx.encode(ctx.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    B = [ctx.empty_like(s) for s in A]
    ctx.sync()
    log("[bench] encoded; warming up")
    cur, nxt = A, B
    for _ in range(args.warmup):
        ctx.step(cur, wl.dt, out=nxt)
        cur, nxt = nxt, cur
    ctx.sync()
    log("[bench] timed steps")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.step(cur, wl.dt, out=nxt)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = wl.n_particles * args.steps / (t1 - t0)
    log(f"[bench] {ms_step:.3f} ms/step, {value:.3e} particle-updates/s")

    stages = {}
    for name, (ms, cnt) in prof.items():
        if cnt == 0:
            continue
        per = ms / cnt
        b = stage_bytes(name, wl.n_mesh, wl)
        stages[name] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps,
                        "ms_per_launch": per,
                        "gbs": (b / (per * 1e-3) / 1e9) if b else None}
    dom = max((k for k in stages if stage_bytes(k, wl.n_mesh, wl) > 0),
              key=lambda k: stages[k]["ms_per_step"])
    ach = stages[dom]["gbs"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": measured_traffic(dom, args.config),
                "bytes_per_launch": stage_bytes(dom, wl.n_mesh, wl),
                "ms_per_launch": stages[dom]["ms_per_launch"]}
    # the same figures for every stage with a byte model (the particle kernels included)
    for k, st in stages.items():
        if st["gbs"] is not None:
            st["frac"] = st["gbs"] / HBM_PEAK_GBS
            st["traffic"] = measured_traffic(k, args.config)
    total_model = sum(stage_bytes(k, wl.n_mesh, wl) * stages[k]["launches_per_step"]
                      for k in stages)
    step_frac = total_model / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    adj = None
    if not args.no_adjoint:
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
        a128 = adjoint_rates(PMContext, make_workload, torch, "adjoint_128")
        adj["adjoint_128"] = a128
        log(f"[bench] adjoint_128: fwd {a128['fwd_ms']:.2f} ms, bwd {a128['bwd_ms']:.2f} ms "
            f"for {a128['steps']} steps")

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=ctx.device)
        b = torch.empty_like(a)
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b

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
                   "brick": ctx.brick, "parallelism": "single GPU"},
        "roofline": roofline,
        "step_hbm_frac_model": step_frac,
        "stages": stages,
        "adjoint": adj,
        "err_vs_fp64": err,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
