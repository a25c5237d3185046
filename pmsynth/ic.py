"""Synthetic initial conditions for the particle-mesh step.

The paper's workloads (Sec. 2.4 compression test, Sec. 3 TianNu and the weak-scaling
runs) start from cosmological initial conditions that are not available here, so these
seeded generators stand in for them with the same structure:

* cold dark matter (CDM): a cubic lattice of n_p^3 particles displaced by the
  Zel'dovich approximation from a Gaussian random field with a power-law spectrum
  P(k) ~ k^n_s, cut at the lattice Nyquist sphere, scaled to a stated RMS
  displacement measured in particle-mesh cells; velocities follow the static
  growing mode v = psi (time unit 1/sqrt(4 pi G rho_cdm) = 1);
* neutrinos: uniform random positions, isotropic directions and speeds drawn from
  the relativistic Fermi-Dirac momentum distribution p^2/(e^p+1), scaled so that the
  mean speed is a stated multiple of the CDM RMS speed (Sec. 3.2 describes neutrinos
  as fast, thermally supported and initialised later than CDM); the paper's 8:1
  neutrino-to-CDM particle-count ratio is kept (Sec. 2.1 footnote).

Units: box side 1, total CDM mass 1 (mean CDM density 1). The neutrino particle mass
is m_cdm / 8 * (Omega_nu / Omega_cdm) with Omega_nu / Omega_cdm = 0.01.

All randomness comes from numpy's PCG64 generator: one independent stream per fixed
chunk of 2^22 values (SeedSequence.spawn), each chunk drawing its quantities in a fixed
order, so that results do not depend on the machine or on how many threads fill the
chunks. Every array is returned as float32, the precision the step consumes.
"""

from __future__ import annotations

import concurrent.futures
import dataclasses
import os

import numpy as np
import scipy.fft

CHUNK = 1 << 22  # fixed draw granularity (part of the definition of the streams)
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))

OMEGA_NU_OVER_OMEGA_C = 0.01
NU_PER_CDM_SIDE = 2  # 8:1 in count


@dataclasses.dataclass
class SpeciesLoad:
    name: str
    x: np.ndarray  # float32 [n][3], box units in [0, 1)
    v: np.ndarray  # float32 [n][3], box units per unit time
    mass: float

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclasses.dataclass
class PMWorkload:
    name: str
    n_mesh: int
    n_cell: int
    dt: float
    steps: int
    species: list  # list[SpeciesLoad]
    soft_cells: float = 1.0

    @property
    def n_particles(self) -> int:
        return sum(s.n for s in self.species)


# The five workloads the step is measured and tested on. 'n_cell' is the side of the
# compression mesh: half the neutrino lattice side (Sec. 2.4 uses (n_p/2)^3 cells with
# n_p the neutrino count per side, Sec. 2.1 footnote), or half the CDM side when there
# are no neutrinos.
CONFIGS = {
    "plain_cdm_64": dict(n_p_c=32, n_p_nu=0, n_mesh=64, n_cell=16, n_s=-2.0, sigma=0.2,
                         dt=0.01, steps=1, seed_c=1, seed_nu=101, layout="float"),
    "two_species_256": dict(n_p_c=128, n_p_nu=256, n_mesh=256, n_cell=128, n_s=-1.5,
                            sigma=0.3, dt=0.01, steps=1, seed_c=2, seed_nu=102,
                            layout="compressed"),
    "tile_1024": dict(n_p_c=256, n_p_nu=512, n_mesh=1024, n_cell=256, n_s=-1.0, sigma=0.3,
                      dt=0.005, steps=5, seed_c=0, seed_nu=100, layout="compressed"),
    "adjoint_128": dict(n_p_c=64, n_p_nu=0, n_mesh=128, n_cell=32, n_s=-2.0, sigma=0.2,
                        dt=0.02, steps=10, seed_c=4, seed_nu=104, layout="compressed",
                        seed_target=5),
    "large_2048": dict(n_p_c=512, n_p_nu=1024, n_mesh=2048, n_cell=512, n_s=-1.0,
                       sigma=0.3, dt=0.005, steps=3, seed_c=11, seed_nu=111,
                       layout="compressed"),
}


def _chunk_streams(seed: int, n: int):
    """One PCG64 stream per chunk of CHUNK values of an n-value quantity."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn((n + CHUNK - 1) // CHUNK)]


def _fill_chunks(n: int, seed: int, fill):
    """Call fill(rng, start, end) for every chunk, the chunks spread over threads (numpy's
    generators release the GIL while they fill)."""
    rngs = _chunk_streams(seed, n)
    with concurrent.futures.ThreadPoolExecutor(WORKERS) as ex:
        list(ex.map(lambda k: fill(rngs[k], k * CHUNK, min(n, (k + 1) * CHUNK)),
                    range(len(rngs))))


def cdm_zeldovich(n_p: int, n_mesh: int, n_s: float, sigma_cells: float, seed: int):
    """Lattice + Zel'dovich displacement from a power-law Gaussian random field.

    Returns (x, v) float32 [n_p^3][3]; particle index (iz*n_p + iy)*n_p + ix,
    columns (x, y, z). The RMS of |psi| equals sigma_cells / n_mesh.
    """
    n3 = n_p ** 3
    white = np.empty(n3, dtype=np.float64)

    def fill(r, a, b):
        white[a:b] = r.standard_normal(b - a)

    _fill_chunks(n3, seed, fill)
    white = white.reshape(n_p, n_p, n_p)  # [z][y][x]
    dk = scipy.fft.rfftn(white, workers=WORKERS)
    del white
    fz = np.fft.fftfreq(n_p, d=1.0 / n_p)  # integer wave numbers
    fx = np.fft.rfftfreq(n_p, d=1.0 / n_p)
    nz = fz[:, None, None]
    ny = fz[None, :, None]
    nx = fx[None, None, :]
    n2 = nz * nz + ny * ny + nx * nx
    keep = (n2 > 0) & (n2 < (n_p / 2.0) ** 2)  # drop k=0 and the Nyquist sphere
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where(keep, np.power(np.where(n2 > 0, n2, 1.0), n_s / 4.0), 0.0)
        inv_k2 = np.where(keep, 1.0 / np.where(n2 > 0, n2, 1.0), 0.0)
    dk *= amp
    psi = np.empty((n3, 3), dtype=np.float64)
    for col, nn in ((0, nx), (1, ny), (2, nz)):
        comp = scipy.fft.irfftn(1j * nn * inv_k2 * dk, s=(n_p, n_p, n_p), axes=(0, 1, 2),
                                workers=WORKERS)
        psi[:, col] = comp.reshape(-1)
        del comp
    del dk
    rms = np.sqrt(np.mean(np.sum(psi * psi, axis=1)))
    if rms > 0:
        psi *= (sigma_cells / n_mesh) / rms
    i = np.arange(n_p, dtype=np.float64) / n_p
    qz, qy, qx = np.meshgrid(i, i, i, indexing="ij")
    q = np.stack([qx.reshape(-1), qy.reshape(-1), qz.reshape(-1)], axis=1)
    x = np.mod(q + psi, 1.0)
    x32 = x.astype(np.float32)
    x32[x32 >= np.float32(1.0)] = np.float32(0.0)  # wrap values that round up to 1
    v32 = psi.astype(np.float32)
    return x32, v32


def fd_speed_table(n: int = 1 << 16, p_max: float = 40.0):
    """Inverse-CDF table of the relativistic Fermi-Dirac magnitude p^2/(e^p+1).

    Returns (cdf, p) float64 arrays for np.interp; the distribution's mean is
    (7/8) 6 zeta(4) / ((3/4) 2 zeta(3)) = 3.15137.
    """
    p = np.linspace(0.0, p_max, n + 1)
    f = p * p / (np.exp(p) + 1.0)
    # trapezoid cumulative integral
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(p))])
    cdf /= cdf[-1]
    return cdf, p


FD_MEAN = 3.15137


def neutrinos_fermi_dirac(n_p: int, mean_speed: float, seed: int):
    """Uniform positions, isotropic directions, Fermi-Dirac speeds with the given mean.
    Each chunk draws its positions, then directions, then speeds from its own stream."""
    n = n_p ** 3
    x = np.empty((n, 3), dtype=np.float32)
    v = np.empty((n, 3), dtype=np.float32)
    cdf, p = fd_speed_table()
    scale = mean_speed / FD_MEAN

    def fill(r, s, e):
        m = e - s
        xs32 = r.random((m, 3)).astype(np.float32)
        xs32[xs32 >= np.float32(1.0)] = np.float32(0.0)
        x[s:e] = xs32
        d = r.standard_normal((m, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        t = np.interp(r.random(m), cdf, p)
        v[s:e] = (d * (t * scale)[:, None]).astype(np.float32)

    _fill_chunks(n, seed, fill)
    return x, v


def make_workload(name: str, seed_offset: int = 0, n_p_c: int | None = None,
                  n_p_nu: int | None = None, n_mesh: int | None = None,
                  n_cell: int | None = None) -> PMWorkload:
    """Build one of CONFIGS, optionally shrunk (same recipe, smaller sides)."""
    c = dict(CONFIGS[name])
    if n_p_c is not None:
        c["n_p_c"] = n_p_c
    if n_p_nu is not None:
        c["n_p_nu"] = n_p_nu
    if n_mesh is not None:
        c["n_mesh"] = n_mesh
    if n_cell is not None:
        c["n_cell"] = n_cell
    xc, vc = cdm_zeldovich(c["n_p_c"], c["n_mesh"], c["n_s"], c["sigma"],
                           c["seed_c"] + seed_offset)
    n_c = c["n_p_c"] ** 3
    m_c = 1.0 / n_c
    species = [SpeciesLoad("cdm", xc, vc, m_c)]
    if c["n_p_nu"] > 0:
        v_rms = float(np.sqrt(np.mean(np.sum(vc.astype(np.float64) ** 2, axis=1))))
        xn, vn = neutrinos_fermi_dirac(c["n_p_nu"], 50.0 * v_rms, c["seed_nu"] + seed_offset)
        n_nu = c["n_p_nu"] ** 3
        species.append(SpeciesLoad("nu", xn, vn, OMEGA_NU_OVER_OMEGA_C * 1.0 / n_nu))
    return PMWorkload(name=name, n_mesh=c["n_mesh"], n_cell=c["n_cell"], dt=c["dt"],
                      steps=c["steps"], species=species)
