"""Shared helpers of the GPU parity tests: contexts, seeded loads, tie-zone checks."""

import numpy as np
import pytest
import torch

from oracle import codec
from pmsynth import make_workload


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"


def ctx(n_mesh, n_cell, brick=None, soft=1.0):
    from paper_1611_01545_amd import PMContext
    require_gpu()
    return PMContext(n_mesh, n_cell, brick=brick, soft_cells=soft)


def small_two_species(n_p_c=16, n_mesh=32, seed_offset=0, n_cell=None):
    """The two-species workload recipe at a reduced size (same generators)."""
    n_cell = n_cell or n_p_c
    return make_workload("two_species_256", seed_offset=seed_offset, n_p_c=n_p_c,
                         n_p_nu=2 * n_p_c, n_mesh=n_mesh, n_cell=n_cell)


def assert_state_equal(host, ref, keys=("count", "esc", "pos", "vel", "v_max")):
    for k in keys:
        a, b = np.asarray(host[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        assert np.array_equal(a, b), f"{k} differs in {np.count_nonzero(a != b)} places"


def density_close(rho_gpu, rho_ref, tol=1e-5):
    """|d rho| <= tol * max(|rho|, mean rho) at every node."""
    rho_gpu = np.asarray(rho_gpu, dtype=np.float64)
    scale = np.maximum(np.abs(rho_ref), np.abs(rho_ref).mean())
    err = np.abs(rho_gpu - rho_ref) / scale
    return float(err.max())


def rel_rms(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))


def frac_dist(x):
    """Distance of x to the nearest integer."""
    return np.abs(x - np.round(x))
