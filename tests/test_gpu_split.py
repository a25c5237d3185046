"""GPU parity of the two-level PM force of Sec. 2.1 (contexts with the long- and
short-range kernel parts, pm_interp_accel, pm_step_p3m) against the oracle
(oracle.split, oracle.mesh, oracle.step)."""

import numpy as np
import pytest
import torch

from gpu_util import check_codes, ctx, rel_rms, small_two_species
from oracle import codec, mesh, pp, split
from paper_1611_01545_amd import PMContext

pytestmark = pytest.mark.gpu

G = 1.0 / (4.0 * np.pi)
LONG, SHORT = PMContext.KERNEL_LONG, PMContext.KERNEL_SHORT


def _encode(c, wl):
    return [c.encode(c.float_species(s.x, s.v, s.mass)) for s in wl.species]


@pytest.mark.parametrize("n,kernel", [(8, LONG), (32, LONG), (16, SHORT), (64, SHORT)])
def test_kernel_table(n, kernel):
    r_s = (1.25 if kernel == LONG else 5.0) / n
    c = PMContext(n, n // 2 if n > 8 else n, soft_cells=1.0, kernel=kernel, r_split=r_s)
    t = c.kernel_table().cpu().numpy().astype(np.float64)
    q = np.arange(t.size, dtype=np.float64)
    k = 2 * np.pi * np.sqrt(q)
    ref = mesh.plummer_kernel_k(k, 1.0 / n, G) * mesh.split_factor(
        k, (r_s, "long" if kernel == LONG else "short")) / n ** 3
    assert t[0] == 0.0
    assert np.all(np.abs(t - ref) <= 2e-7 * np.abs(ref) + 1e-44)
    c.close()


@pytest.mark.parametrize("n,n_cell,kernel", [(8, 8, LONG), (16, 16, LONG), (32, 16, LONG),
                                             (32, 16, SHORT), (64, 16, SHORT)])
def test_force_mesh_matches_oracle(n, n_cell, kernel):
    # the filtered (and, for the long part, window-divided) kernel through the whole FFT
    # path, on the two-species recipe's density
    wl = small_two_species(16, 64, seed_offset=3, n_cell=16)
    r_s = 1.25 / (n if kernel == LONG else n // 4)
    soft = 0.25 if kernel == LONG else 1.0
    c = PMContext(n, n_cell, soft_cells=soft, kernel=kernel, r_split=r_s)
    f = ctx(64, 16)
    st = _encode(f, wl)
    hosts = [f.to_host(s) for s in st]
    xs = [(codec.decode(h)[0].astype(np.float64), sp.mass) for h, sp in zip(hosts, wl.species)]
    rho = mesh.deposit_species(xs, n)
    acc, amax = c.force(torch.tensor(rho, dtype=torch.float32, device=c.device))
    want = mesh.force_mesh(rho.astype(np.float32).astype(np.float64), soft, G,
                           (r_s, "long" if kernel == LONG else "short"))
    got = acc.cpu().numpy()
    for a in range(3):
        assert rel_rms(got[a], want[a]) < 1e-4, (a, rel_rms(got[a], want[a]))
    assert abs(float(amax.item()) - np.max(np.abs(want))) <= 1e-4 * np.max(np.abs(want))
    c.close()
    f.close()


@pytest.mark.parametrize("n_mesh,n_cell", [(16, 16), (64, 16), (32, 8)])
def test_interp_accel_matches_oracle(n_mesh, n_cell):
    wl = small_two_species(16, 64, seed_offset=4, n_cell=n_cell)
    c = ctx(n_mesh, n_cell)
    st = _encode(c, wl)
    acc, _ = c.force(c.deposit(st))
    out = c.interp_accel(st, acc)
    twice = c.interp_accel(st, acc, out=[o.clone() for o in out], accumulate=True)
    c.sync()
    acc_h = acc.cpu().numpy().astype(np.float64)
    scale = np.max(np.abs(acc_h))
    for s, o, o2 in zip(st, out, twice):
        x = codec.decode(c.to_host(s))[0].astype(np.float64)
        want = mesh.interpolate(acc_h, x)
        got = o.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(got - want)) <= 2e-6 * scale
        assert torch.equal(o2, o + o)
    c.close()


def test_step_p3m_matches_oracle():
    wl = small_two_species(16, 64, seed_offset=5, n_cell=16)
    fine, coarse = PMContext.two_level(64, 16)
    st = _encode(fine, wl)
    out, perms = fine.step_p3m(coarse, st, wl.dt, want_perm=True)
    fine.sync()
    states = [fine.to_host(s) for s in st]
    masses = [sp.mass for sp in wl.species]
    new, diag = split.step_two_level(states, masses, 64, 16, wl.dt, wl.dt, fine.r_split,
                                     1.0, G)
    a_rms = np.sqrt(np.mean(diag["a_mesh"] ** 2) + np.mean(diag["a_long"] ** 2))
    ties = check_codes(fine, out, perms, new, diag, 16, wl.dt, a_rms=a_rms)
    print(f"[split] two-level step: {ties} codes in the tie zone", flush=True)
    fine.close()
    coarse.close()


def test_step_p3m_with_pp_matches_oracle():
    from test_gpu_pp import _clustered, _r_soft
    wl, species = _clustered(6)
    fine, coarse = PMContext.two_level(64, 16)
    st = [fine.encode(fine.float_species(sp.x, sp.v, sp.mass)) for sp in species]
    out, perms = fine.step_p3m(coarse, st, wl.dt, r_soft=_r_soft(wl), want_perm=True)
    fine.sync()
    states = [fine.to_host(s) for s in st]
    masses = [sp.mass for sp in species]
    new, diag = split.step_two_level(states, masses, 64, 16, wl.dt, wl.dt, fine.r_split,
                                     1.0, G, r_soft=_r_soft(wl))
    assert sum(int(np.count_nonzero(np.any(a != 0, axis=1))) for a in diag["pp"]) > 100
    a_rms = np.sqrt(np.mean(diag["a_mesh"] ** 2) + np.mean(diag["a_long"] ** 2))
    ties = check_codes(fine, out, perms, new, diag, 16, wl.dt, a_rms=a_rms)
    print(f"[split] two-level step with PP: {ties} codes in the tie zone", flush=True)
    fine.close()
    coarse.close()


def test_step_p3m_infinite_split_is_the_one_level_step():
    # r_split -> infinity: the long-range kernel is 0 and the short-range one is the
    # one-level kernel, so the step has the same bits as pm_step
    wl = small_two_species(16, 64, seed_offset=7, n_cell=16)
    fine, coarse = PMContext.two_level(64, 16, r_split=1e6)
    one = ctx(64, 16)
    st = _encode(one, wl)
    a = one.step(st, wl.dt)
    b = fine.step_p3m(coarse, st, wl.dt)
    one.sync()
    fine.sync()
    for x, y in zip(a, b):
        for f in ("count", "pos", "vel", "hdr"):
            assert torch.equal(getattr(x, f), getattr(y, f)), f
    for c in (fine, coarse, one):
        c.close()


def test_step_p3m_rejects_a_mismatched_pair():
    wl = small_two_species(8, 32, seed_offset=8, n_cell=8)
    fine, coarse = PMContext.two_level(32, 8)
    st = _encode(fine, wl)
    with pytest.raises(RuntimeError):
        coarse.step_p3m(fine, st, wl.dt)  # roles swapped
    other = PMContext(8, 8, fine.brick, soft_cells=0.25, kernel=LONG,
                      r_split=2 * fine.r_split)
    with pytest.raises(RuntimeError):
        fine.step_p3m(other, st, wl.dt)  # another split length
    full = PMContext(8, 8, fine.brick, soft_cells=0.25)
    with pytest.raises(RuntimeError):
        fine.step_p3m(full, st, wl.dt)  # not a long-range context
    soft = PMContext(8, 8, fine.brick, soft_cells=1.0, kernel=LONG, r_split=fine.r_split)
    with pytest.raises(RuntimeError):
        fine.step_p3m(soft, st, wl.dt)  # another softening length
    with pytest.raises(RuntimeError):
        PMContext(16, 8, kernel=LONG, r_split=0.0)
    for c in (fine, coarse, other, full, soft):
        c.close()


def test_step_p3m_with_two_byte_positions_matches_oracle():
    # the two-level step on (2, 2)-byte codes (the adjustable widths of Sec. 2.4)
    from paper_1611_01545_amd import widths_word
    wl = small_two_species(16, 64, seed_offset=9, n_cell=16)
    fine, coarse = PMContext.two_level(64, 16)
    st = [fine.encode(fine.float_species(s.x, s.v, s.mass), widths=widths_word(2, 2))
          for s in wl.species]
    out, perms = fine.step_p3m(coarse, st, wl.dt, want_perm=True)
    fine.sync()
    states = [fine.to_host(s) for s in st]
    masses = [sp.mass for sp in wl.species]
    new, diag = split.step_two_level(states, masses, 64, 16, wl.dt, wl.dt, fine.r_split,
                                     1.0, G)
    a_rms = np.sqrt(np.mean(diag["a_mesh"] ** 2) + np.mean(diag["a_long"] ** 2))
    ties = check_codes(fine, out, perms, new, diag, 16, wl.dt, a_rms=a_rms)
    print(f"[split] two-level step, 2-byte positions: {ties} codes in the tie zone",
          flush=True)
    fine.close()
    coarse.close()
