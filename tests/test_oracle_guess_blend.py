"""Pins of the oracle's blended extrapolation guess (oracle/guess_blend.py),
all on the CPU.

* the blend's weights sum to 1 for any (a, b) and give the damped cubic, the
  linear and the previous-step guess at (0, 0), (1, 0) and (0, 1); on a
  history sampled from a cubic the damped cubic (a = b = 0) is exact;
* optimal_blend recovers planted coefficients exactly, agrees with NumPy's
  least squares on random complex data, and its guess is never worse than the
  damped cubic; a constant history gives no target;
* the features on simple cases.
"""

import math

import numpy as np
import pytest

from oracle import guess_blend as gb


@pytest.mark.parametrize("a,b", [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (0.3, -0.7), (-2.5, 1.5)])
def test_weights(a, b):
    w = gb.blend_weights(a, b)
    assert w.sum() == pytest.approx(1.0, abs=1e-14)
    if (a, b) == (0.0, 0.0):
        np.testing.assert_array_equal(w, gb.C_DC)
    if (a, b) == (1.0, 0.0):
        np.testing.assert_allclose(w, [2.0, -1.0, 0.0, 0.0, 0.0], atol=1e-15)
    if (a, b) == (0.0, 1.0):
        np.testing.assert_allclose(w, [1.0, 0.0, 0.0, 0.0, 0.0], atol=1e-15)


def test_damped_cubic_exact_on_cubics():
    # u(t) = cubic in t, sampled at t = -1 .. -5: the damped cubic reproduces
    # u(0) (a polynomial of degree <= 3 is extrapolated exactly)
    rng = np.random.default_rng(1)
    coef = rng.standard_normal((4, 7)) + 1j * rng.standard_normal((4, 7))
    u = lambda t: sum(coef[p] * t ** p for p in range(4))  # noqa: E731
    hist = [u(-1.0 - k) for k in range(5)]
    np.testing.assert_allclose(gb.guess(hist, 0.0, 0.0), u(0.0), rtol=1e-12, atol=1e-12)


def test_optimal_blend_recovers_planted():
    rng = np.random.default_rng(2)
    hist = [rng.standard_normal(40) + 1j * rng.standard_normal(40) for _ in range(5)]
    for a, b in ((0.2, -0.1), (-1.3, 2.0), (0.0, 0.0)):
        un = gb.guess(hist, a, b)
        got = gb.optimal_blend(hist, un)
        assert got == pytest.approx((a, b), abs=1e-10)


def test_optimal_blend_is_least_squares():
    rng = np.random.default_rng(3)
    for trial in range(5):
        hist = [rng.standard_normal(30) + 1j * rng.standard_normal(30) for _ in range(5)]
        un = rng.standard_normal(30) + 1j * rng.standard_normal(30)
        x_dc = gb.guess(hist, 0.0, 0.0)
        d1 = (2 * hist[0] - hist[1]) - x_dc
        d2 = hist[0] - x_dc
        # real least squares over the stacked real and imaginary parts
        M = np.stack([np.concatenate([d1.real, d1.imag]), np.concatenate([d2.real, d2.imag])], 1)
        rhs = np.concatenate([(un - x_dc).real, (un - x_dc).imag])
        ref, *_ = np.linalg.lstsq(M, rhs, rcond=None)
        ref = np.clip(ref, -gb.CLIP, gb.CLIP)
        got = gb.optimal_blend(hist, un)
        assert got == pytest.approx(tuple(ref), rel=1e-9, abs=1e-12)
        e_opt = np.linalg.norm(gb.guess(hist, *got) - un)
        assert e_opt <= np.linalg.norm(x_dc - un) * (1 + 1e-12)


def test_constant_history_has_no_target():
    v = np.full(12, 2.0 + 1j)
    assert gb.optimal_blend([v] * 5, v) is None


def test_features():
    x = gb.features(2e-4, [5000.0, 4900.0, 4800.0, 4700.0, 4600.0, 4500.0], 0.5, 100.0, 0.5,
                    3e-3, 1e-4, [0.0, 3.0, 4.0])
    np.testing.assert_allclose(x[:6], 2e-4 * 0.5 * np.array([5000, 4900, 4800, 4700, 4600, 4500.0]))
    assert x[6] == pytest.approx(math.log(0.5 * 100 * 3e-3 / 0.25))
    gf = 2e-4 * 5000.0
    assert x[7] == pytest.approx(math.log1p(50 * 3e-3 * gf * gf))
    assert x[8] == pytest.approx(math.log1p(50 * 3e-3 * gf / 0.5))
    assert x[9] == pytest.approx(math.log1p(50 * 1e-4 / 0.5))
    np.testing.assert_allclose(x[10:13], [0.0, 0.6, 0.8])
    assert not x[13:].any()
