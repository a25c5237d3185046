"""Oracle, float64 on any torch device: the uncompressed particle-mesh step at sizes the
CPU oracle cannot hold (2048^3 meshes, 1.2 G particles).

TEST INFRASTRUCTURE ONLY, like the rest of this package: it restates the numpy oracle's
definitions (oracle.mesh, oracle.step.step_float) with torch float64 tensor operations so
that the largest workload can be compared with an all-float64, uncompressed reference on
the same GPU. It shares no code with the HIP library and calls none of it. Library
primitives serve as steps: torch.fft for the discrete Fourier transforms,
Tensor.index_add_ for the CIC scatter-adds, torch.special.modified_bessel_k1 for K1.

Definitions (Sec. 2.1 and the readings of oracle.mesh): node-centred CIC weights,
rho(c) = n^3 sum_i m_i W(x_i - x_c) in the unit box; a_a = IDFT(-i D(k_a) G(|k|)
DFT(rho)) with the Plummer kernel G(k) = -4 pi G eps K1(k eps)/k, G(0) = 0, and the
fourth-order central-difference symbol D; CIC interpolation; kick v' = v + c_k a_i, drift
x' = x + c_d v' (mod 1).

Memory: the transforms run in slabs, and each force component is made in the storage of
one half-spectrum (its rows hold n + 2 reals), so that a step at 2048^3 needs the
particles, the density spectrum and one component: about 200 GB with 1.2 G particles.

Pins (tests/test_fp64_torch.py, CPU): deposit, force mesh, interpolation and the float
step equal the numpy oracle's to rounding on small meshes, slab sizes that do not
divide the mesh included.
"""

from __future__ import annotations

import math

import torch

FOUR_PI = 4.0 * math.pi
CHUNK = 1 << 24  # particles per scatter / gather batch


def _cic(x: torch.Tensor, n: int):
    """Lower node index (int64, per axis, mod n) and fractional offset of each particle."""
    u = x * n
    fl = torch.floor(u)
    return torch.remainder(fl.to(torch.int64), n), u - fl


def _corners(i: torch.Tensor, f: torch.Tensor, n: int):
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((f[:, 0] if dx else 1.0 - f[:, 0]) * (f[:, 1] if dy else 1.0 - f[:, 1]) *
                     (f[:, 2] if dz else 1.0 - f[:, 2]))
                idx = ((((i[:, 2] + dz) % n) * n + (i[:, 1] + dy) % n) * n +
                       (i[:, 0] + dx) % n)
                yield idx, w


def deposit(species, n: int, device) -> torch.Tensor:
    """species: list of (x [N][3] float tensor, mass). Returns rho [n][n][n] float64."""
    rho = torch.zeros(n ** 3, dtype=torch.float64, device=device)
    for x, m in species:
        for s in range(0, x.shape[0], CHUNK):
            xs = x[s:s + CHUNK].to(device=device, dtype=torch.float64)
            i, f = _cic(xs, n)
            for idx, w in _corners(i, f, n):
                rho.index_add_(0, idx, w * float(m))
            del xs, i, f
    rho *= float(n) ** 3
    return rho.view(n, n, n)


def spectrum(rho: torch.Tensor, slab: int = 32) -> torch.Tensor:
    """Unnormalised forward DFT of a real [n][n][n] mesh as the half spectrum
    [z][y][x <= n/2] (complex128), in slabs: (y, x) transforms of z slabs, then z
    transforms of y slabs. rho is consumed (freed by the caller afterwards)."""
    n = rho.shape[0]
    out = torch.empty((n, n, n // 2 + 1), dtype=torch.complex128, device=rho.device)
    for z0 in range(0, n, slab):
        out[z0:z0 + slab] = torch.fft.rfft2(rho[z0:z0 + slab])
    for y0 in range(0, n, slab):
        out[:, y0:y0 + slab] = torch.fft.fft(out[:, y0:y0 + slab], dim=0)
    return out


def _signed(n: int, m: int, device) -> torch.Tensor:
    k = torch.arange(m, device=device, dtype=torch.float64)
    return torch.where(k < n / 2, k, k - n)


def gradient_symbol(k: torch.Tensor, n: int) -> torch.Tensor:
    """D(k) = (8 sin(2 pi k / n) - sin(4 pi k / n)) n / 6 for integer wave numbers k,
    each sine exactly 0 where its angle is a multiple of pi."""
    t = 2.0 * math.pi * k / n
    s1 = torch.where(torch.remainder(2.0 * k, n) == 0, torch.zeros_like(t), torch.sin(t))
    s2 = torch.where(torch.remainder(4.0 * k, n) == 0, torch.zeros_like(t), torch.sin(2.0 * t))
    return (8.0 * s1 - s2) * (n / 6.0)


def kernel(k2: torch.Tensor, n: int, soft_cells: float, G: float) -> torch.Tensor:
    """G(|k|) on integer |n|^2 values: -4 pi G eps K1(k eps) / k, 0 at k = 0."""
    k = 2.0 * math.pi * torch.sqrt(k2)
    eps = soft_cells / n
    safe = torch.where(k > 0, k, torch.ones_like(k))
    if eps > 0:
        g = -FOUR_PI * G * eps * torch.special.modified_bessel_k1(safe * eps) / safe
    else:
        g = -FOUR_PI * G / (safe * safe)
    return torch.where(k > 0, g, torch.zeros_like(g))


def force_component(rhok: torch.Tensor, axis: int, soft_cells: float = 1.0,
                    G: float = 1.0 / FOUR_PI, slab: int = 32) -> torch.Tensor:
    """a_axis = IDFT(-i D(k_axis) G(|k|) rho~) as a float64 view [n][n][n] of a padded
    [n][n][n + 2] array (the storage of one half spectrum). axis 0, 1, 2 = x, y, z."""
    n = rhok.shape[0]
    dev = rhok.device
    h = n // 2 + 1
    kz = _signed(n, n, dev)
    ky = kz
    kx = torch.arange(h, device=dev, dtype=torch.float64)
    P = torch.empty_like(rhok)
    for y0 in range(0, n, slab):
        y1 = min(n, y0 + slab)
        k2 = (kz[:, None, None] ** 2 + ky[None, y0:y1, None] ** 2 + kx[None, None, :] ** 2)
        g = kernel(k2, n, soft_cells, G)
        if axis == 0:
            d = gradient_symbol(kx, n)[None, None, :]
        elif axis == 1:
            d = gradient_symbol(ky[y0:y1], n)[None, :, None]
        else:
            d = gradient_symbol(kz, n)[:, None, None]
        blk = rhok[:, y0:y1] * (-1j * (d * g))
        P[:, y0:y1] = torch.fft.ifft(blk, dim=0)
        del blk, g, k2
    real = P.view(torch.float64).view(n, n, 2 * h)
    for z0 in range(0, n, slab):
        z1 = min(n, z0 + slab)
        r = torch.fft.irfft(torch.fft.ifft(P[z0:z1], dim=1), n=n, dim=2)
        real[z0:z1, :, :n] = r
        del r
    return real[:, :, :n]


def interpolate(a: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """CIC gather of one component mesh (a [n][n][n] view, any strides) at x [N][3]."""
    n = a.shape[0]
    sz, sy, sx = a.stride()
    flat = a.as_strided((a.untyped_storage().nbytes() // 8,), (1,), a.storage_offset())
    out = torch.zeros(x.shape[0], dtype=torch.float64, device=a.device)
    for s in range(0, x.shape[0], CHUNK):
        xs = x[s:s + CHUNK].to(device=a.device, dtype=torch.float64)
        i, f = _cic(xs, n)
        acc = torch.zeros(xs.shape[0], dtype=torch.float64, device=a.device)
        for idx, w in _corners(i, f, n):
            iz, rem = idx // (n * n), idx % (n * n)
            iy, ix = rem // n, rem % n
            acc += w * flat[iz * sz + iy * sy + ix * sx]
        out[s:s + xs.shape[0]] = acc
    return out


def step_float(species, n: int, c_k: float, c_d: float, soft_cells: float = 1.0,
               G: float = 1.0 / FOUR_PI, slab: int = 32, keep=None):
    """One kick-drift step of float64 particles in place: species is a list of
    (x [N][3] float64, v [N][3] float64, mass) on the device. keep(axis, a_mesh) is called
    with each force component mesh before it is freed (to sample it), and keep('rho',
    rho) with the density."""
    dev = species[0][0].device
    rho = deposit([(x, m) for x, _, m in species], n, dev)
    if keep is not None:
        keep("rho", rho)
    rhok = spectrum(rho, slab)
    del rho
    for axis in range(3):
        a = force_component(rhok, axis, soft_cells, G, slab)
        if keep is not None:
            keep(axis, a)
        for x, v, _ in species:
            v[:, axis] += c_k * interpolate(a, x)
        del a
    del rhok
    for x, v, _ in species:
        x += c_d * v
        torch.remainder(x, 1.0, out=x)
