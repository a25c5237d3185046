"""pm_reduce_noalloc (the entry point for callers that cannot allocate) against pm_reduce:
the same results on two calls in a row, the second with a smaller input, with nothing
allocated by the library (a fresh context holds no scratch afterwards)."""

import numpy as np
import pytest
import torch

from gpu_util import ctx, small_two_species

pytestmark = pytest.mark.gpu


def _inputs(c, n_p_c, seed, layout):
    wl = small_two_species(n_p_c, c.n_mesh, seed_offset=seed, n_cell=c.n_cell)
    fl = [c.float_species(sp.x, sp.v, sp.mass) for sp in wl.species]
    return [c.encode(f) for f in fl] if layout == "compressed" else fl


@pytest.mark.parametrize("layout", ["compressed", "float"])
def test_noalloc_reduce_equals_reduce(layout):
    from paper_1611_01545_amd import PMContext
    c = ctx(32, 16)
    ref = ctx(32, 16)
    for n_p_c, seed in ((16, 1), (8, 2)):  # the second call with a smaller input
        sp = _inputs(ref, n_p_c, seed, layout)
        rho = ref.deposit(sp)
        acc, _ = ref.force(ref.deposit(sp))
        want = ref.reduce(sp, rho, acc)
        # the same device buffers through the context that never allocated scratch
        out = torch.full((8 + 6 * len(sp),), float("nan"), dtype=torch.float64,
                         device=c.device)
        c.reduce_noalloc(sp, out, rho, acc)
        c.sync()
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (got, want)
        assert c.scratch_bytes() == 0
        # without meshes, and with the momentum only
        out2 = torch.zeros(8 + 6 * len(sp), dtype=torch.float64, device=c.device)
        c.reduce_noalloc(sp, out2)
        c.sync()
        assert np.array_equal(out2.cpu().numpy(), ref.reduce(sp))
    c.close()
    ref.close()


def test_noalloc_reduce_rejects_cells_beyond_its_array():
    from paper_1611_01545_amd._lib import PMError
    c = ctx(128, 64)  # 64^3 cells > 32^3
    sp = _inputs(c, 16, 3, "compressed")
    out = torch.zeros(8 + 6 * len(sp), dtype=torch.float64, device=c.device)
    with pytest.raises(PMError) as e:
        c.reduce_noalloc(sp, out)
    assert e.value.code == 2  # PM_ERR_SHAPE
    # float species of the same context are not limited
    fl = [c.float_species(s.x, s.v, s.mass) for s in
          small_two_species(16, 128, seed_offset=3, n_cell=64).species]
    c.reduce_noalloc(fl, out)
    c.sync()
    assert np.isclose(out[1].item(), sum(f.mass * f.n for f in fl))
    c.close()
