"""Oracle: the particle-mesh gravity operators in float64.

Follows Sec. 2.1 of the paper: the density is interpolated onto a uniform cubic mesh
(cloud-in-cell, "CIC", Sec. 2.3), Fourier transformed, multiplied by the Poisson
kernel of eq. (2), differentiated in Fourier space as in eq. (3) (with the discrete
gradient symbol below in place of k), transformed back, and the force is interpolated
back to the particles with the same CIC weights ("inverse force interpolation",
Fig. 2).

Readings where the paper is silent:
  * CIC is node-centred: u = x n_g, i = floor(u), f = u - i, weights (1 - f, f) on
    nodes i and i+1 (mod n_g) per axis, product over the three axes;
  * the Poisson kernel carries Plummer softening of eps = soft_cells mesh cells:
    G(k) = -4 pi G eps K1(k eps) / k, the Fourier transform of -G / sqrt(r^2 + eps^2);
    it tends to eq. (2)'s -4 pi G / k^2 as eps -> 0; G(0) = 0 removes the mean density;
  * the gradient factor of eq. (3) is -i D(k_a) with the symbol of the fourth-order
    central difference, D(k) = (8 sin(k Delta) - sin(2 k Delta)) / (6 Delta), equal to k
    up to O((k Delta)^4) and zero on the Nyquist index. The bare -i k truncated at the
    Nyquist cube rings (Gibbs) along the mesh axes: a point mass then pulls 20-66% too
    weakly at 4-16 cells along an axis; D keeps the operator real and odd (exact zero
    self-force and momentum conservation) without the ringing.

Pins (tests/test_oracle_pins.py): kernel against the Fourier transform of the Plummer
density computed by quadrature and against the eps -> 0 limit; FFT path against
explicit DFT sums; mass conservation; zero self-force; momentum conservation; inverse
square law against the exact periodic Plummer force; Zel'dovich plane-wave response and growth.
"""

from __future__ import annotations

import numpy as np
import scipy.special

FOUR_PI = 4.0 * np.pi


def _corner_weights(x: np.ndarray, n_g: int):
    """Yield (flat node index, weight, per-axis (w, sign)) for the 8 CIC corners."""
    u = np.asarray(x, dtype=np.float64) * n_g
    i = np.floor(u)
    f = u - i
    i = i.astype(np.int64) % n_g
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                d = (dx, dy, dz)
                ws = []
                for a in range(3):
                    ws.append(f[:, a] if d[a] else 1.0 - f[:, a])
                idx = (((i[:, 2] + dz) % n_g) * n_g + (i[:, 1] + dy) % n_g) * n_g \
                    + (i[:, 0] + dx) % n_g
                yield idx, ws, d


def deposit(x: np.ndarray, mass, n_g: int) -> np.ndarray:
    """CIC mass density rho(c) = Delta^-3 sum_i m_i W(x_i - x_c); returns [z][y][x]."""
    x = np.asarray(x, dtype=np.float64)
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (x.shape[0],))
    rho = np.zeros(n_g ** 3, dtype=np.float64)
    for idx, ws, _ in _corner_weights(x, n_g):
        rho += np.bincount(idx, weights=m * ws[0] * ws[1] * ws[2], minlength=n_g ** 3)
    return rho.reshape(n_g, n_g, n_g) * float(n_g) ** 3


def density_at(x: np.ndarray, mass, n_g: int, nodes: np.ndarray) -> np.ndarray:
    """CIC density at the given nodes [k][3] (integer x, y, z) only.

    By the definition of the weight: W is the product over axes of the tent
    max(0, 1 - |u - c|) in mesh units (u = x n_g, c the node), with the periodic
    (nearest image) distance; rho(c) = n_g^3 sum_i m_i W. For particles far from the
    nodes this never forms the mesh, so it serves single nodes of large meshes.
    """
    u = np.asarray(x, dtype=np.float64) * n_g
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (u.shape[0],))
    nodes = np.asarray(nodes, dtype=np.int64).reshape(-1, 3)
    out = np.zeros(nodes.shape[0], dtype=np.float64)
    for k, c in enumerate(nodes):
        d = u - c
        d -= n_g * np.round(d / n_g)  # nearest periodic image
        w = np.prod(np.clip(1.0 - np.abs(d), 0.0, None), axis=1)
        out[k] = float(np.sum(m * w)) * float(n_g) ** 3
    return out


def deposit_window(x: np.ndarray, mass, n_g: int, lo, size: int) -> np.ndarray:
    """CIC density on the window of nodes lo_a <= c_a < lo_a + size (mod n_g) of the
    periodic n_g^3 mesh, from the given particles only; returns [z][y][x] of side size.
    The same weights as deposit(); a particle contributes to a window node when one of
    its 8 corner nodes is that node. For the nodes of a large mesh that only the
    particles near the window reach."""
    x = np.asarray(x, dtype=np.float64)
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (x.shape[0],))
    lo = np.asarray(lo, dtype=np.int64).reshape(3)
    out = np.zeros(size ** 3, dtype=np.float64)
    u = x * n_g
    i = np.floor(u)
    f = u - i
    i = i.astype(np.int64) % n_g
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                d = (dx, dy, dz)
                w = m.copy()
                inside = np.ones(x.shape[0], dtype=bool)
                loc = []
                for a in range(3):
                    w = w * (f[:, a] if d[a] else 1.0 - f[:, a])
                    c = (i[:, a] + d[a] - lo[a]) % n_g
                    inside &= c < size
                    loc.append(c)
                idx = (loc[2] * size + loc[1]) * size + loc[0]
                out += np.bincount(idx[inside], weights=w[inside], minlength=size ** 3)
    return out.reshape(size, size, size) * float(n_g) ** 3


def deposit_species(species, n_g: int) -> np.ndarray:
    """Both species onto the same mesh (Sec. 2.1 footnote): list of (x, mass)."""
    rho = np.zeros((n_g, n_g, n_g), dtype=np.float64)
    for x, m in species:
        rho += deposit(x, m, n_g)
    return rho


def wave_numbers(n_g: int):
    """Integer wave numbers on numpy's rfft grid: (nz, ny, nx) broadcastable."""
    f = np.fft.fftfreq(n_g, d=1.0 / n_g)
    fx = np.fft.rfftfreq(n_g, d=1.0 / n_g)
    return f[:, None, None], f[None, :, None], fx[None, None, :]


def plummer_kernel_k(k: np.ndarray, eps: float, G: float) -> np.ndarray:
    """-4 pi G eps K1(k eps) / k for k > 0 (eps > 0), -4 pi G / k^2 for eps = 0; 0 at k=0."""
    k = np.asarray(k, dtype=np.float64)
    out = np.zeros_like(k)
    pos = k > 0
    if eps > 0:
        out[pos] = -FOUR_PI * G * eps * scipy.special.k1(k[pos] * eps) / k[pos]
    else:
        out[pos] = -FOUR_PI * G / (k[pos] * k[pos])
    return out


def split_factor(k: np.ndarray, split) -> np.ndarray:
    """Gaussian force split of the two-level PM (oracle.split): split = (r_s, part) with
    the split length r_s in box units; part 'long' gives exp(-k^2 r_s^2), 'short' gives
    1 - exp(-k^2 r_s^2); None gives 1 (the one-level kernel)."""
    k = np.asarray(k, dtype=np.float64)
    if split is None:
        return np.ones_like(k)
    r_s, part = split
    q = (k * r_s) ** 2
    if part == "long":
        return np.exp(-q)
    if part == "short":
        return -np.expm1(-q)
    raise ValueError(f"unknown split part {part!r}")


def cic_window2(nz, ny, nx, n_g: int) -> np.ndarray:
    """Product of the CIC deposit and interpolation windows at integer wave numbers:
    prod_a sinc(n_a / n_g)^4, sinc(t) = sin(pi t) / (pi t)."""
    return (np.sinc(nx / n_g) * np.sinc(ny / n_g) * np.sinc(nz / n_g)) ** 4


def green(n_g: int, soft_cells: float = 1.0, G: float = 1.0 / FOUR_PI,
          split=None) -> np.ndarray:
    """Kernel on the rfft grid [z][y][x<=n/2]. One level: a function of |n|^2 only.
    split (see split_factor): the long-range part is also divided by the mesh's CIC
    window product (oracle.split)."""
    nz, ny, nx = wave_numbers(n_g)
    k = 2.0 * np.pi * np.sqrt(nz * nz + ny * ny + nx * nx)
    g = plummer_kernel_k(k, soft_cells / n_g, G) * split_factor(k, split)
    if split is not None and split[1] == "long":
        g = g / cic_window2(nz, ny, nx, n_g)
    return g


def gradient_symbol(nn, n_g: int):
    """D(k) = (8 sin(k Delta) - sin(2 k Delta)) / (6 Delta) at k = 2 pi nn, Delta = 1/n_g;
    each sine is taken as exactly 0 where its angle is a multiple of pi."""
    nn = np.asarray(nn, dtype=np.float64)
    t = 2.0 * np.pi * nn / n_g
    s1 = np.where(np.mod(2.0 * nn, n_g) == 0, 0.0, np.sin(t))
    s2 = np.where(np.mod(4.0 * nn, n_g) == 0, 0.0, np.sin(2.0 * t))
    return (8.0 * s1 - s2) * (n_g / 6.0)


def gradient_factors(n_g: int):
    """-i D(k_a) per axis on the rfft grid (zero on the Nyquist index)."""
    nz, ny, nx = wave_numbers(n_g)
    return [-1j * gradient_symbol(nn, n_g) for nn in (nx, ny, nz)]  # x, y, z


def force_mesh(rho: np.ndarray, soft_cells: float = 1.0, G: float = 1.0 / FOUR_PI,
               split=None) -> np.ndarray:
    """Acceleration mesh a[3][z][y][x] from density: eqs. (2)-(3) with F = m a and the
    discrete gradient symbol (split: one part of the two-level kernel, see green)."""
    n_g = rho.shape[0]
    phi_k = green(n_g, soft_cells, G, split) * np.fft.rfftn(rho)
    a = np.empty((3, n_g, n_g, n_g), dtype=np.float64)
    for ax, fac in enumerate(gradient_factors(n_g)):
        a[ax] = np.fft.irfftn(fac * phi_k, s=(n_g, n_g, n_g), axes=(0, 1, 2))
    return a


def interpolate(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """CIC gather a_i = sum_c W(x_i - x_c) a(c) for each component; returns [n][3]."""
    n_g = a.shape[1]
    flat = a.reshape(3, -1)
    out = np.zeros((x.shape[0], 3), dtype=np.float64)
    for idx, ws, _ in _corner_weights(x, n_g):
        w = ws[0] * ws[1] * ws[2]
        for c in range(3):
            out[:, c] += w * flat[c, idx]
    return out


def scatter_vector(x: np.ndarray, g: np.ndarray, n_g: int) -> np.ndarray:
    """Transpose of interpolate: mu_a(c) = sum_i W(x_i - x_c) g_ia; returns [3][z][y][x]."""
    mu = np.zeros((3, n_g ** 3), dtype=np.float64)
    for idx, ws, _ in _corner_weights(x, n_g):
        w = ws[0] * ws[1] * ws[2]
        for c in range(3):
            mu[c] += np.bincount(idx, weights=w * g[:, c], minlength=n_g ** 3)
    return mu.reshape(3, n_g, n_g, n_g)


def gather_grad(mesh: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_c grad_x W(x_i - x_c) f(c) for a scalar mesh f; returns [n][3].

    The weight per axis is (1 - f) or f with f = u - floor(u), so its derivative with
    respect to x is -n_g or +n_g; the derivative at f = 0 is taken one-sided, with the
    node assignment that floor gives.
    """
    n_g = mesh.shape[0]
    flat = mesh.reshape(-1)
    out = np.zeros((x.shape[0], 3), dtype=np.float64)
    for idx, ws, d in _corner_weights(x, n_g):
        val = flat[idx]
        for a in range(3):
            s = n_g if d[a] else -n_g
            prod = s * val
            for b in range(3):
                if b != a:
                    prod = prod * ws[b]
            out[:, a] += prod
    return out


def accelerations(species, n_g: int, soft_cells: float = 1.0,
                  G: float = 1.0 / FOUR_PI, split=None):
    """Full PM force: list of (x, mass) -> (list of a_i [n][3], mesh a[3][...])."""
    rho = deposit_species(species, n_g)
    a = force_mesh(rho, soft_cells, G, split)
    return [interpolate(a, x) for x, _ in species], a, rho
