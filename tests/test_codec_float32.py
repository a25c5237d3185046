"""The float32 forms of the velocity codec that the kick uses (CPU only).

The kick evaluates the velocity code of Sec. 2.4 in float32 when v_max' is a power of
two in [2^-90, 2^90], and the decode in float32 when v_max is in that range. These
tests restate those two formulas with numpy float32 arithmetic (IEEE, like the GPU's)
and check them against the oracle's float64 definitions on the values where a
float32 evaluation could plausibly go wrong: bin edges, the |x| < 2^-15 region where
the float64 sum x + 32768 rounds, the clamps, overflow to infinity, subnormals.
"""

import numpy as np
import pytest

from oracle import codec

F = np.float32


def code_p2(v: np.ndarray, v_max: float) -> np.ndarray:
    """The kernel's float32 velocity code for a power-of-two v_max."""
    C = F(2.0 ** 15 / v_max)  # exact: a power of two
    with np.errstate(over="ignore", invalid="ignore"):
        x = np.asarray(v, dtype=F) * C
    fl = np.floor(x)
    fl = np.where((x < 0) & (x >= F(-2.0 ** -39)), F(0), fl)
    out = np.where(fl >= F(32767), 65535, 0)
    mid = (fl >= F(-32768)) & (fl < F(32767))
    out[mid] = fl[mid].astype(np.int64) + 32768
    return out.astype(np.int64)


def decode_w(j: np.ndarray, v_max: np.float32) -> np.ndarray:
    """The kernel's float32 velocity decode."""
    w = F(v_max) * F(2.0 ** -15)
    return (np.asarray(j, dtype=np.uint32).astype(F) - F(32767.5)) * w


def _adversarial_x() -> np.ndarray:
    k = np.arange(-32770, 32771, dtype=np.float64)
    ulp = np.spacing(np.abs(k).astype(F)).astype(np.float64)
    edges = np.concatenate([k, k - ulp, k + ulp, k + 0.5])
    tiny = []
    for e in range(-160, -10):
        for m in (1.0, 1.0 - 2.0 ** -24, 1.0 + 2.0 ** -23, 1.5):
            tiny += [m * 2.0 ** e, -m * 2.0 ** e]
    tiny += [2.0 ** -39, -2.0 ** -39, -(2.0 ** -39) * (1 + 2.0 ** -23),
             -(2.0 ** -39) * (1 - 2.0 ** -24), 0.0, -0.0, 1e-45, -1e-45]
    big = [32767.0, 32767.5, 32768.0, -32768.0, -32768.5, -32769.0, 1e30, -1e30]
    return np.concatenate([edges, np.array(tiny), np.array(big)])


@pytest.mark.parametrize("e", [-90, -40, -7, -1, 0, 1, 5, 17, 60, 90])
def test_velocity_code_float32_matches_float64_definition(e):
    v_max = F(2.0 ** e)
    rng = np.random.default_rng(100 + e)
    x = _adversarial_x()
    with np.errstate(over="ignore"):
        v = (x * 2.0 ** (e - 15)).astype(F)  # v = x / C, exact unless it leaves float32 range
    v = np.concatenate([
        v,
        (rng.uniform(-1.5, 1.5, 200000) * float(v_max)).astype(F),
        (rng.standard_normal(50000) * 2.0 ** rng.integers(-140, 120, 50000)).astype(F),
        np.array([np.inf, -np.inf, np.finfo(F).max, -np.finfo(F).max,
                  np.finfo(F).tiny, -np.finfo(F).tiny], dtype=F),
    ])
    v = v[np.isfinite(v) | np.isinf(v)]
    want = codec.velocity_codes(v, v_max)
    got = code_p2(v, float(v_max))
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (v[bad[:5]], got[bad[:5]], want[bad[:5]])


def test_velocity_code_tiny_negative_rounds_like_float64():
    # x + 32768 in float64 rounds to 32768 for -2^-39 <= x < 0, and to just below it
    # for x < -2^-39: the float32 form must reproduce both sides of that edge
    v_max = F(1.0)
    x = np.array([-(2.0 ** -39), -(2.0 ** -39) * (1 + 2.0 ** -23), -(2.0 ** -40)])
    v = (x * 2.0 ** -15).astype(F)
    assert list(codec.velocity_codes(v, v_max)) == [32768, 32767, 32768]
    assert list(code_p2(v, 1.0)) == [32768, 32767, 32768]


@pytest.mark.parametrize("seed", range(6))
def test_velocity_decode_float32_matches_float64_definition(seed):
    rng = np.random.default_rng(seed)
    j = np.arange(65536, dtype=np.int64)
    for v_max in [F(2.0 ** -90), F(2.0 ** 90), F(1.0)] + list(
            (2.0 ** rng.uniform(-90, 90, 8)).astype(F)):
        got = decode_w(j, v_max)
        want = codec.decode_velocity(j, v_max)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), float(v_max)
