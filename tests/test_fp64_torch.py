"""Pins of the torch float64 restatement of the oracle (oracle.fp64_torch) against the
numpy oracle on the CPU: density, force mesh, interpolation and a float step agree to
rounding, with slab sizes that do and do not divide the mesh."""

import numpy as np
import pytest
import torch

from oracle import fp64_torch, mesh, step


def _particles(seed, n):
    rng = np.random.default_rng(seed)
    return [(rng.random((n, 3)), rng.standard_normal((n, 3)) * 0.3, 1.0 / n),
            (rng.random((2 * n, 3)), rng.standard_normal((2 * n, 3)) * 3.0, 0.01 / (2 * n))]


@pytest.mark.parametrize("n,slab", [(8, 3), (16, 32), (16, 5)])
def test_force_mesh_and_interpolation_match_oracle(n, slab):
    sp = _particles(n + slab, 300)
    dev = torch.device("cpu")
    xs = [(torch.from_numpy(x), m) for x, _, m in sp]
    rho = fp64_torch.deposit(xs, n, dev)
    rho_o = mesh.deposit_species([(x, m) for x, _, m in sp], n)
    assert np.allclose(rho.numpy(), rho_o, rtol=1e-13, atol=1e-13 * rho_o.max())
    a_o = mesh.force_mesh(rho_o)
    rhok = fp64_torch.spectrum(rho.clone(), slab)
    assert np.allclose(rhok.numpy(), np.fft.rfftn(rho_o), rtol=0,
                       atol=1e-12 * np.abs(np.fft.rfftn(rho_o)).max())
    scale = np.abs(a_o).max()
    for axis in range(3):
        a = fp64_torch.force_component(rhok, axis, slab=slab)
        assert np.allclose(a.numpy(), a_o[axis], rtol=0, atol=1e-12 * scale)
        x = sp[1][0]
        got = fp64_torch.interpolate(a, torch.from_numpy(x)).numpy()
        want = mesh.interpolate(a_o, x)[:, axis]
        assert np.allclose(got, want, rtol=0, atol=1e-12 * scale)


def test_gradient_symbol_and_kernel_match_oracle():
    n = 32
    k = np.arange(-n // 2, n // 2, dtype=np.float64)
    assert np.array_equal(fp64_torch.gradient_symbol(torch.from_numpy(k), n).numpy(),
                          mesh.gradient_symbol(k, n))
    k2 = np.arange(0, 3 * 16 * 16 + 1, dtype=np.float64)
    got = fp64_torch.kernel(torch.from_numpy(k2), n, 1.0, 1.0 / (4 * np.pi)).numpy()
    want = mesh.plummer_kernel_k(2 * np.pi * np.sqrt(k2), 1.0 / n, 1.0 / (4 * np.pi))
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_float_step_matches_oracle():
    n, dt = 16, 0.01
    sp = _particles(3, 400)
    out_o, _ = step.step_float(sp, n, dt, dt)
    t = [(torch.from_numpy(x.copy()), torch.from_numpy(v.copy()), m) for x, v, m in sp]
    fp64_torch.step_float(t, n, dt, dt, slab=5)
    for (x, v, _), (xo, vo) in zip(t, out_o):
        dx = np.abs(x.numpy() - xo)
        assert np.minimum(dx, 1 - dx).max() <= 1e-13
        assert np.allclose(v.numpy(), vo, rtol=1e-12, atol=1e-14)
