"""GPU parity of the cell-local particle-particle force (eq. (4)) and of the step that
adds it (pm_pp_accel, pm_step_pp) against the oracle (oracle.pp, oracle.step)."""

import types

import numpy as np
import pytest
import torch

from gpu_util import check_codes, ctx, small_two_species
from oracle import pp, step

pytestmark = pytest.mark.gpu


def _clustered(seed, n_mesh=64, n_cell=16):
    """The two-species recipe with CDM clumps a third of a mesh cell across, so that many
    mesh cells hold several particles; neutrinos stream through them."""
    wl = small_two_species(16, n_mesh, seed_offset=seed, n_cell=n_cell)
    rng = np.random.default_rng(seed)
    cdm, nu = wl.species
    x = cdm.x.copy()
    q = 1.0 / (256 * n_cell)
    at = 0
    for k in (300, 200, 120, 60, 30):
        centre = rng.random(3)
        x[at:at + k] = np.mod(centre + q * rng.uniform(-20, 20, (k, 3)), 1.0).astype(np.float32)
        at += k
    x[x >= 1] = 0
    return wl, [types.SimpleNamespace(x=x, v=cdm.v, mass=cdm.mass), nu]


def _r_soft(wl):
    return 1.0 / (20 * 2 * wl.n_cell)  # L / (20 n_p), n_p = 2 n_cell (Sec. 2.1, Sec. 2.4)


@pytest.mark.parametrize("seed,n_mesh,n_cell", [(1, 64, 16), (2, 32, 16), (3, 64, 32)])
def test_pp_accel_matches_oracle(seed, n_mesh, n_cell):
    wl, species = _clustered(seed, n_mesh, n_cell)
    _check_pp(wl, species, n_mesh, n_cell)


def test_pp_accel_dense_brick_matches_oracle():
    # a brick whose codes exceed what a wave stages in LDS (4 KB: 1365 particles with
    # 1-byte codes) reads its partners from the stream: a clump of 2400 CDM particles
    # in one mesh cell
    wl = small_two_species(16, 64, seed_offset=8, n_cell=16)
    cdm, nu = wl.species
    rng = np.random.default_rng(8)
    x = cdm.x.copy()
    q = 1.0 / (256 * 16)
    x[:2400] = np.mod(rng.random(3) + q * rng.uniform(-20, 20, (2400, 3)), 1.0).astype(np.float32)
    x[x >= 1] = 0
    species = [types.SimpleNamespace(x=x, v=cdm.v, mass=cdm.mass), nu]
    _check_pp(wl, species, 64, 16, min_pairs=2000)


def _check_pp(wl, species, n_mesh, n_cell, min_pairs=100):
    c = ctx(n_mesh, n_cell)
    st = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    pmax = torch.zeros(1, dtype=torch.float32, device=c.device)
    app = c.pp_accel(st, _r_soft(wl), pmax)
    c.sync()
    hosts = [c.to_host(s) for s in st]
    masses = [sp.mass for sp in species]
    want = pp.pp_accel(hosts, masses, n_mesh, _r_soft(wl), c.G)
    got = [a.cpu().numpy().astype(np.float64) for a in app]
    scale = max(np.sqrt(np.mean(w ** 2)) for w in want)
    assert scale > 0
    pairs = 0
    for g_, w in zip(got, want):
        err = np.abs(g_ - w)
        assert np.all(err <= 1e-5 * (np.abs(w) + scale)), err.max()
        assert np.array_equal(g_ == 0, w == 0)  # the same particles have partners
        pairs += int(np.count_nonzero(np.any(w != 0, axis=1)))
    assert pairs > min_pairs
    assert float(pmax.item()) == max(float(np.max(np.abs(a.cpu().numpy()))) for a in app)
    # Newton's third law: sum m a = 0 up to float32 rounding
    tot = sum(m * g_.sum(0) for m, g_ in zip(masses, got))
    mag = sum(m * np.abs(g_).sum() for m, g_ in zip(masses, got))
    assert np.all(np.abs(tot) <= 1e-5 * mag)
    print(f"[pp] {pairs} particles with partners, |a_pp| up to {float(pmax.item()):.3e}",
          flush=True)
    c.close()


def test_step_pp_matches_oracle():
    wl, species = _clustered(4)
    c = ctx(64, 16)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    out, perms = c.step_pp(dev, wl.dt, _r_soft(wl), want_perm=True)
    c.sync()
    states = [c.to_host(d) for d in dev]
    masses = [sp.mass for sp in species]
    extra = pp.pp_accel(states, masses, 64, _r_soft(wl), c.G)
    new, diag = step.step_compressed(states, masses, 64, wl.dt, wl.dt, extra=extra)
    ties = check_codes(c, out, perms, new, diag, 16, wl.dt)
    print(f"[pp] step with the PP force: {ties} codes in the tie zone", flush=True)
    c.close()


def test_step_pp_without_pairs_equals_step():
    """With r_soft above every in-cell distance no pair interacts: the same bits as pm_step."""
    wl, species = _clustered(5)
    c = ctx(64, 16)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    a = c.step(dev, wl.dt)
    b = c.step_pp(dev, wl.dt, 1.0)
    c.sync()
    for x, y in zip(a, b):
        for f in ("count", "pos", "vel", "hdr"):
            assert torch.equal(getattr(x, f), getattr(y, f)), f
    c.close()
