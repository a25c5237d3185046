"""Host-side logic of bench.py: the byte model, the measured-traffic record, the
single-GPU guard (no GPU needed)."""

import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from pmsynth import make_workload  # noqa: E402


def test_byte_model_headline_totals():
    wl = make_workload("plain_cdm_64")  # shape only; the model is linear in N and n^3
    n = 1024
    n3 = float(n) ** 3
    assert bench.stage_bytes("fft_z", n, wl) == 8 * n3
    assert bench.stage_bytes("fft_y_fwd", n, wl) == 8 * n3
    assert bench.stage_bytes("force_grad", n, wl) == 16 * n3  # 4 n^3 in, 12 n^3 out
    assert bench.stage_bytes("unknown", n, wl) == 0.0
    N = wl.n_particles
    assert bench.stage_bytes("interp_kick_drift", n, wl) == 18 * N + 2 * wl.n_cell ** 3 + 12 * n3


def test_measured_traffic_is_tied_to_the_kernel_sources():
    rec = bench.MEASURED_TRAFFIC[("interp_kick_drift", "tile_1024")]
    t = bench.measured_traffic("interp_kick_drift", "tile_1024")
    want = rec["fetch_kib"] * 1024 * rec["fetch_factor"] + rec["write_kib"] * 1024 * rec["write_factor"]
    assert t is None or abs(t - want) < 1.0
    assert bench.measured_traffic("resort", "tile_1024") is None  # no record
    # a record taken on other sources is not used
    bad = dict(rec, sha256="0" * 64)
    saved = bench.MEASURED_TRAFFIC[("interp_kick_drift", "tile_1024")]
    try:
        bench.MEASURED_TRAFFIC[("interp_kick_drift", "tile_1024")] = bad
        assert bench.measured_traffic("interp_kick_drift", "tile_1024") is None
    finally:
        bench.MEASURED_TRAFFIC[("interp_kick_drift", "tile_1024")] = saved


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_dominant_kernel_is_one_template():
    # the roofline goes to the single-template stage with the largest time per step; the
    # re-sort (several templates) is never picked, even when it takes longest
    wl = types.SimpleNamespace(n_particles=10 ** 9, species=[0, 1], n_cell=512, n_mesh=2048)
    st = {k: {"ms_per_step": ms} for k, ms in (("fft_z", 27.8), ("fft_y_inv", 14.8),
                                               ("fft_x_c2r", 12.5), ("interp_kick_drift", 38.0),
                                               ("force_grad", 27.2), ("deposit", 23.1),
                                               ("resort", 40.0))}
    assert bench.dominant_kernel_stage(st, 2048, wl) == "interp_kick_drift"
    assert bench.stage_kernel("fft_z", 2048) == "k_col_zconv<2048, 16, 0, true>"
    assert bench.stage_kernel("fft_y_inv", 2048) == "k_col_fft<2048, 16, 1, 0>"
    assert bench.stage_kernel("force_grad", 2048) == "k_grad4"
    assert bench.stage_kernel("resort", 2048) is None
    st["force_grad"]["ms_per_step"] = 50.0
    assert bench.dominant_kernel_stage(st, 2048, wl) == "force_grad"
