"""Parity of the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: the compressed codec, stream order, counts and byte streams are bit-exact;
density |d rho| <= 1e-5 max(|rho|, mean rho); forces relative RMS <= 1e-4; float-path
positions <= 1e-6 box units; compressed codes equal except in the tie zone where the
oracle's pre-floor value lies within the propagated force tolerance of an integer.
"""

import types

import numpy as np
import pytest
import torch

from gpu_util import (_codes_old_order, assert_state_equal, check_codes, ctx,
                      density_close, frac_dist, rel_rms,
                      small_two_species)
from oracle import codec, mesh, step

pytestmark = pytest.mark.gpu


def _encode_both(c, wl, brick):
    states, dev = [], []
    for sp in wl.species:
        st = codec.encode(sp.x, sp.v, wl.n_cell, brick)
        fs = c.float_species(sp.x, sp.v, sp.mass)
        cs, perm = c.encode(fs, want_perm=True)
        states.append(st)
        dev.append((cs, perm))
    return states, dev


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_kernel_table(n):
    c = ctx(n, n // 2)
    t = c.kernel_table().cpu().numpy().astype(np.float64)
    q = np.arange(t.size, dtype=np.float64)
    ref = mesh.plummer_kernel_k(2 * np.pi * np.sqrt(q), 1.0 / n, 1 / (4 * np.pi)) / n ** 3
    nz = ref != 0
    assert t[0] == 0.0
    assert np.max(np.abs(t[nz] / ref[nz] - 1)) < 2e-7


@pytest.mark.parametrize("n_p_c,n_mesh,brick", [(16, 32, 4), (16, 32, 1), (32, 64, 8)])
def test_encode_decode_bit_exact(n_p_c, n_mesh, brick):
    wl = small_two_species(n_p_c, n_mesh)
    c = ctx(n_mesh, wl.n_cell, brick)
    states, dev = _encode_both(c, wl, brick)
    for st, (cs, perm) in zip(states, dev):
        h = c.to_host(cs)
        assert_state_equal(h, st)
        assert np.array_equal(perm.cpu().numpy(), st["perm"])
        fs = c.decode(cs)
        c.sync()
        xo, vo = codec.decode(st)
        assert np.array_equal(fs.x.cpu().numpy(), xo)
        assert np.array_equal(fs.v.cpu().numpy(), vo)


def test_encode_escape_and_edges():
    rng = np.random.default_rng(3)
    n_c, n_mesh, brick = 8, 32, 2
    n = 5000
    x = rng.random((n, 3)).astype(np.float32)
    x[:700] = np.float32(0.51)             # one cell with 700 particles
    x[700:1000] = np.float32(0.0)          # 300 at the origin corner
    x[1000, :] = np.float32(1.0 - 2 ** -24)
    x[1001, :] = np.float32(-1e-9)
    x[1002, :] = np.float32(1.0)
    v = rng.standard_normal((n, 3)).astype(np.float32)
    v[5] = [3.5, -3.5, 0.0]
    c = ctx(n_mesh, n_c, brick)
    st = codec.encode(x, v, n_c, brick)
    cs, perm = c.encode(c.float_species(x, v, 1.0 / n), want_perm=True)
    h = c.to_host(cs)
    assert st["esc"].shape[0] == 2
    assert_state_equal(h, st)
    assert np.array_equal(perm.cpu().numpy(), st["perm"])
    assert (h["j_min"], h["j_max"]) == (int(st["vel"].min()), int(st["vel"].max()))


def test_encode_capacity_error():
    from paper_1611_01545_amd._lib import PMError
    n_c = 4
    x = np.full((600, 3), 0.3, np.float32)
    v = np.zeros((600, 3), np.float32)
    c = ctx(16, n_c, 1)
    cs = c.encode(c.float_species(x, v, 1.0), cap_esc=0)
    with pytest.raises(PMError) as e:
        c.sync()
    assert "CAPACITY" in str(e.value)
    assert c.last_error_detail() == 1


def test_empty_species():
    c = ctx(16, 8, 2)
    x = np.zeros((0, 3), np.float32)
    cs = c.encode(c.float_species(x, x, 1.0))
    h = c.to_host(cs)
    assert h["count"].sum() == 0 and h["v_max"] == 0


@pytest.mark.parametrize("n_p_c,n_mesh", [(16, 32), (16, 64), (32, 64)])
def test_deposit_compressed(n_p_c, n_mesh):
    wl = small_two_species(n_p_c, n_mesh)
    c = ctx(n_mesh, wl.n_cell)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    rho = c.deposit(dev).cpu().numpy()
    c.sync()
    sts = [c.to_host(d) for d in dev]
    ref = mesh.deposit_species([(codec.decode(s)[0].astype(np.float64), sp.mass)
                                for s, sp in zip(sts, wl.species)], n_mesh)
    assert density_close(rho, ref) <= 1e-5
    # deterministic: a second deposit is bit-identical
    rho2 = c.deposit(dev).cpu().numpy()
    assert np.array_equal(rho, rho2)


def test_deposit_compressed_dense_cell():
    """15000 of 20000 particles inside one mesh cell: each of its eight nodes sums
    thousands of CIC weights, far past 2^32 units of 2^-27 (the integer sums carry)."""
    rng = np.random.default_rng(41)
    n_mesh, n_c, n = 32, 8, 20000
    x = rng.random((n, 3)).astype(np.float32)
    x[:15000] = (0.3 + rng.uniform(0.0, 1.0 / n_mesh, (15000, 3))).astype(np.float32)
    v = np.zeros((n, 3), np.float32)
    x2 = rng.random((3000, 3)).astype(np.float32)
    c = ctx(n_mesh, n_c)
    dev = [c.encode(c.float_species(x, v, 1.0 / n)),
           c.encode(c.float_species(x2, v[:3000], 0.25 / 3000))]
    rho = c.deposit(dev).cpu().numpy()
    c.sync()
    sts = [c.to_host(d) for d in dev]
    ref = mesh.deposit_species([(codec.decode(sts[0])[0].astype(np.float64), 1.0 / n),
                                (codec.decode(sts[1])[0].astype(np.float64), 0.25 / 3000)],
                               n_mesh)
    assert ref.max() > 2000.0 * ref.mean()
    assert density_close(rho, ref) <= 1e-5
    assert np.array_equal(rho, c.deposit(dev).cpu().numpy())


def test_deposit_compressed_tile_past_carry_range():
    """2.2 M particles in one compression cell: more than 2^21 in one deposit tile, so
    its per-node integer sums are flushed in several segments."""
    rng = np.random.default_rng(43)
    n_mesh, n_c, n = 16, 4, 2_300_000
    x = rng.random((n, 3)).astype(np.float32)
    x[:2_200_000] = (0.55 + rng.uniform(0.0, 0.2, (2_200_000, 3))).astype(np.float32)
    v = np.zeros((n, 3), np.float32)
    c = ctx(n_mesh, n_c)
    dev = [c.encode(c.float_species(x, v, 1.0 / n))]
    rho = c.deposit(dev).cpu().numpy()
    c.sync()
    h = c.to_host(dev[0])
    assert int(codec.full_counts(h).max()) >= 2_200_000
    ref = mesh.deposit_species([(codec.decode(h)[0].astype(np.float64), 1.0 / n)], n_mesh)
    assert density_close(rho, ref) <= 1e-5


def test_deposit_float():
    wl = make_plain()
    c = ctx(wl.n_mesh, wl.n_cell)
    sp = wl.species[0]
    rho = c.deposit([c.float_species(sp.x, sp.v, sp.mass)]).cpu().numpy()
    ref = mesh.deposit(sp.x.astype(np.float64), sp.mass, wl.n_mesh)
    assert density_close(rho, ref) <= 1e-5


def make_plain():
    from pmsynth import make_workload
    return make_workload("plain_cdm_64")


@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256])
def test_force_random_density(n):
    rng = np.random.default_rng(n)
    rho = (1.0 + 0.5 * rng.standard_normal((n, n, n))).astype(np.float32)
    c = ctx(n, n // 2)
    acc, amax = c.force(torch.from_numpy(rho).cuda())
    a = acc.cpu().numpy()
    ref = mesh.force_mesh(rho.astype(np.float64))
    for ax in range(3):
        assert rel_rms(a[ax], ref[ax]) <= 1e-4, (ax, rel_rms(a[ax], ref[ax]))
    assert abs(float(amax.item()) / np.max(np.abs(ref)) - 1) < 1e-4


def test_force_in_place_alias():
    n = 32
    rng = np.random.default_rng(1)
    rho = rng.random((n, n, n)).astype(np.float32)
    c = ctx(n, 16)
    buf = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
    buf[0].copy_(torch.from_numpy(rho))
    acc, _ = c.force(buf[0], acc=buf)
    ref = mesh.force_mesh(rho.astype(np.float64))
    for ax in range(3):
        assert rel_rms(acc[ax].cpu().numpy(), ref[ax]) <= 1e-4


def test_float_step_plain():
    wl = make_plain()
    c = ctx(wl.n_mesh, wl.n_cell)
    sp = wl.species[0]
    fs = c.float_species(sp.x, sp.v, sp.mass)
    (out,) = c.step([fs], wl.dt)
    c.sync()
    (ref,), diag = step.step_float([(sp.x, sp.v, sp.mass)], wl.n_mesh, wl.dt, wl.dt)
    dx = np.abs(out.x.cpu().numpy().astype(np.float64) - ref[0])
    dx = np.minimum(dx, 1 - dx)
    assert dx.max() <= 1e-6
    # particle accelerations through the kick: a = (v' - v) / dt
    a_gpu = (out.v.cpu().numpy().astype(np.float64) - sp.v) / wl.dt
    assert rel_rms(a_gpu, diag["acc"][0]) <= 1e-4


# kick variants: two-brick z-half tiles (16 nodes per brick side: 4 cells at r = 4,
# 2 cells at r = 8), one-brick 16-node tiles (8 cells at r = 2), 8-node tiles (2 cells
# at r = 4) and the per-particle gather from the mesh (1 cell at r = 2)
@pytest.mark.parametrize("n_p_c,n_mesh,seed,brick", [(16, 64, 4, None), (16, 128, 5, 2),
                                                     (16, 32, 0, None), (32, 64, 1, None),
                                                     (16, 64, 2, 2), (16, 32, 3, 1)])
def test_compressed_step_tie_zone(n_p_c, n_mesh, seed, brick):
    wl = small_two_species(n_p_c, n_mesh, seed_offset=seed)
    c = ctx(n_mesh, wl.n_cell, brick=brick)
    _step_against_oracle(c, wl.species, n_mesh, wl.n_cell, wl.dt)


# one to four species (the most a step takes) through the two-brick kick tiles (r = 4)
# and the one-brick 16-node tiles (r = 2)
@pytest.mark.parametrize("n_sp,n_mesh", [(1, 64), (3, 64), (4, 64), (4, 32)])
def test_compressed_step_species_count(n_sp, n_mesh):
    a = small_two_species(16, n_mesh, seed_offset=6)
    b = small_two_species(16, n_mesh, seed_offset=7)
    species = [a.species[0], a.species[1], b.species[0], b.species[1]][:n_sp]
    # distinct masses, so a species mix-up shows in the density and force
    species = [types.SimpleNamespace(x=sp.x, v=sp.v, mass=sp.mass * (1.0 + 0.25 * i))
               for i, sp in enumerate(species)]
    c = ctx(n_mesh, a.n_cell)
    _step_against_oracle(c, species, n_mesh, a.n_cell, a.dt)


def _dense_species(seed):
    """The two-species recipe at 64^3 with four CDM clumps: cells holding 600, 256, 255
    and 254 particles, nearly at rest, so that they keep >= 255 (escape) or < 255 through
    the step; the neutrinos stream through the same cells."""
    wl = small_two_species(16, 64, seed_offset=seed)
    rng = np.random.default_rng(seed)
    cdm, nu = wl.species
    x = cdm.x.copy()
    v = cdm.v.copy()
    q = 1.0 / (256 * wl.n_cell)
    at = 0
    for cell, k in (((3, 4, 5), 600), ((10, 2, 7), 256), ((0, 15, 15), 255), ((8, 8, 8), 254)):
        centre = (np.array(cell) + 0.5) / wl.n_cell
        x[at:at + k] = (centre + q * rng.uniform(-20, 20, (k, 3))).astype(np.float32)
        v[at:at + k] *= np.float32(1e-3)
        at += k
    return wl, [types.SimpleNamespace(x=x, v=v, mass=cdm.mass), nu]


def test_compressed_step_dense_cells_match_oracle():
    """Cells at and above the escape count (>= 255) before and after a step: counts,
    escape table, codes (tie-zone rule) and the re-sort permutation against the oracle."""
    wl, species = _dense_species(8)
    c = ctx(64, wl.n_cell)
    _step_against_oracle(c, species, 64, wl.n_cell, wl.dt)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    # the clumps share their cells with lattice particles: count with the oracle
    want = codec.encode(species[0].x, species[0].v, wl.n_cell, c.brick)["esc"].shape[0]
    assert int(dev[0].header()["n_esc"]) == want >= 3
    c.close()


def test_compressed_step_escape_capacity_latched():
    """An output escape table too small for the step's cells >= 255: pm_sync reports
    PM_ERR_CAPACITY with the entries needed, and the context keeps working."""
    from paper_1611_01545_amd._lib import PMError
    wl, species = _dense_species(9)
    c = ctx(64, wl.n_cell)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    c.sync()
    ok = c.step(dev, wl.dt)  # default capacity
    c.sync()
    need = int(ok[0].header()["n_esc"])
    assert need >= 2
    out = [c.empty_compressed(d.n, d.mass, cap_esc=1) for d in dev]
    c.step(dev, wl.dt, out=out)
    with pytest.raises(PMError) as e:
        c.sync()
    assert e.value.code == 5  # PM_ERR_CAPACITY
    assert c.last_error_detail() == need
    again = c.step(dev, wl.dt)  # the latch is cleared: the context works on
    c.sync()
    for a, b in zip(again, ok):
        assert torch.equal(a.pos, b.pos) and torch.equal(a.count, b.count)
    c.close()


def _step_against_oracle(c, species, n_mesh, n_cell, dt, out=None):
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    rho = c.deposit(dev)
    acc, amax = c.force(rho)
    out, perms = c.kick_drift_perm(dev, acc, amax, dt, dt, out=out)
    c.sync()
    states = [c.to_host(d) for d in dev]
    masses = [sp.mass for sp in species]
    new, diag = step.step_compressed(states, masses, n_mesh, dt, dt)
    assert density_close(rho.cpu().numpy(), diag["rho"]) <= 1e-5
    assert rel_rms(acc.cpu().numpy(), diag["a_mesh"]) <= 1e-4
    return check_codes(c, out, perms, new, diag, n_cell, dt)


@pytest.mark.parametrize("dense", [False, True])
def test_compressed_step_without_movers_matches_oracle(dense):
    """A step too short for any position code to change: no particle leaves its cell, so
    the movers' sort is empty, every brick's run of arrivals is empty and each brick's new
    particle count is its old one (the re-sort's brick totals); with the dense clumps the
    escape table carries through unchanged as well."""
    if dense:
        wl, species = _dense_species(12)
    else:
        wl = small_two_species(16, 64, seed_offset=10)
        species = wl.species
    c = ctx(64, wl.n_cell)
    dt = wl.dt * 1e-6
    _step_against_oracle(c, species, 64, wl.n_cell, dt)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    out = c.step(dev, dt)
    c.sync()
    for a, b in zip(dev, out):
        assert_state_equal(c.to_host(b), c.to_host(a), keys=("count", "esc", "pos"))


def test_step_equals_pieces_and_is_deterministic():
    wl = small_two_species(16, 32, seed_offset=5)
    c = ctx(32, wl.n_cell)
    dev = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    out1 = c.step(dev, wl.dt)
    out2 = c.step(dev, wl.dt)
    rho = c.deposit(dev)
    acc, amax = c.force(rho)
    out3 = c.kick_drift(dev, acc, amax, wl.dt, wl.dt)
    c.sync()
    for a, b, d in zip(out1, out2, out3):
        ha, hb, hd = c.to_host(a), c.to_host(b), c.to_host(d)
        assert_state_equal(ha, hb)
        assert_state_equal(ha, hd)


def test_multi_step_chain_conserves_particles():
    wl = small_two_species(16, 32, seed_offset=6)
    c = ctx(32, wl.n_cell)
    cur = [c.encode(c.float_species(sp.x, sp.v, sp.mass)) for sp in wl.species]
    for _ in range(5):
        cur = c.step(cur, wl.dt * 5)
    c.sync()
    for cs, sp in zip(cur, wl.species):
        h = c.to_host(cs)
        assert codec.full_counts(h).sum() == sp.x.shape[0]


def test_pack_unpack_bytes():
    wl = small_two_species(16, 32, seed_offset=2)
    c = ctx(32, wl.n_cell)
    for sid, sp in enumerate(wl.species):
        cs = c.encode(c.float_species(sp.x, sp.v, sp.mass))
        buf = c.pack(cs, sid)
        st = c.to_host(cs)
        ref = codec.pack(st, sp.mass, sid)
        assert buf == ref
        back, sid2 = c.unpack(buf, cs.n)
        assert sid2 == sid and back.mass == sp.mass
        assert_state_equal(c.to_host(back), st)


def test_pack_escape_and_corruption():
    from paper_1611_01545_amd._lib import PMError
    n_c = 4
    rng = np.random.default_rng(4)
    x = rng.random((2000, 3)).astype(np.float32)
    x[:400] = np.float32(0.6)
    v = rng.standard_normal((2000, 3)).astype(np.float32)
    c = ctx(16, n_c, 2)
    cs = c.encode(c.float_species(x, v, 0.5))
    buf = c.pack(cs, 1)
    st = c.to_host(cs)
    assert buf == codec.pack(st, 0.5, 1)
    bad = bytearray(buf)
    bad[100] ^= 0x10
    with pytest.raises(PMError):
        c.unpack(bytes(bad), cs.n)
    with pytest.raises(PMError):
        c.unpack(buf[:-3], cs.n)


@pytest.mark.parametrize("layout", ["compressed", "float"])
def test_reduce_mass_momentum_force(layout):
    """pm_reduce against the oracle: mass, per-species momentum m sum v and m sum a with a
    the CIC interpolation of the force mesh; the total sum m a vanishes (momentum
    conservation, Sec. 2.1) up to the float32 rounding of the mesh force."""
    wl = small_two_species(16, 32, seed_offset=3)
    c = ctx(32, wl.n_cell)
    fl = [c.float_species(sp.x, sp.v, sp.mass) for sp in wl.species]
    dev = [c.encode(f) for f in fl] if layout == "compressed" else fl
    rho = c.deposit(dev)
    acc, _ = c.force(c.deposit(dev))
    out = c.reduce(dev, rho, acc)
    mtot = sum(sp.mass * sp.x.shape[0] for sp in wl.species)
    assert abs(out[1] - mtot) <= 1e-14 * mtot
    assert abs(out[0] - mtot) <= 1e-6 * mtot  # float32 mesh summed in float64
    xs, vs, masses = [], [], []
    for d, sp in zip(dev, wl.species):
        if layout == "compressed":
            x, v = codec.decode(c.to_host(d))
        else:
            x, v = sp.x, sp.v
        xs.append(x.astype(np.float64))
        vs.append(v.astype(np.float64))
        masses.append(sp.mass)
    acc_o, _, _ = mesh.accelerations(list(zip(xs, masses)), 32)
    scale = sum(m * np.abs(a).sum() for m, a in zip(masses, acc_o))
    ptot, ftot = np.zeros(3), np.zeros(3)
    for s_, (x, v, m, ai) in enumerate(zip(xs, vs, masses, acc_o)):
        per = out[8 + 6 * s_: 14 + 6 * s_]
        p = m * v.sum(0)
        f = m * ai.sum(0)
        assert np.allclose(per[:3], p, rtol=1e-12, atol=1e-15)
        assert np.all(np.abs(per[3:] - f) <= 1e-4 * scale), (per[3:], f)
        ptot += p
        ftot += f
    assert np.allclose(out[2:5], ptot, rtol=1e-12, atol=1e-15)
    # the two species pull on each other: each has a net force, the total has none
    assert np.max(np.abs(out[5:8])) <= 1e-5 * scale, (out[5:8], scale)
    assert np.max(np.abs(ftot)) <= 1e-12 * scale
    c.close()


def test_bad_shapes_rejected():
    from paper_1611_01545_amd._lib import PMError
    for args in [(48, 16), (64, 128), (4096, 256), (64, 2)]:
        with pytest.raises(PMError):
            ctx(*args)


def test_compressed_step_many_movers_matches_oracle():
    """A step in which nearly every particle of a 5 M-particle species changes cell: the
    movers' radix sort (at most 1024 workgroups) then takes several 4096-pair tiles per
    workgroup, the scatter's multi-tile path, and the stayer placement sees bricks whose
    particles mostly arrive from elsewhere."""
    rng = np.random.default_rng(31)
    n = 5 * 2 ** 20
    x = rng.random((n, 3)).astype(np.float32)
    x[x >= 1] = 0
    v = (0.5 * rng.standard_normal((n, 3))).astype(np.float32)
    sp = types.SimpleNamespace(x=x, v=v, mass=1.0 / n)
    n_mesh, n_cell = 128, 64
    dt = 3.0 / n_cell / 0.5  # about three cells per step at the RMS speed
    c = ctx(n_mesh, n_cell)
    ties = _step_against_oracle(c, [sp], n_mesh, n_cell, dt)
    print(f"[parity] 5 M particles, most of them moving: {ties} codes in the tie zone",
          flush=True)
    c.close()
