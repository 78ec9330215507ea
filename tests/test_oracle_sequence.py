"""Pins of the oracle's PGSE profile and b-value conversion.

Sec. 2, eq. pgse (profile) and eq. b_value (b = gamma^2 |g|^2 int F^2). The
closed form of int F^2 is checked against adaptive quadrature of F(t)^2, and F
against quadrature of f, so a wrong ramp, plateau or sign fails here.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import sequence as sq

CASES = [(10600.0, 13400.0), (10600.0, 43100.0), (10000.0, 10000.0), (3000.0, 25000.0)]


@pytest.mark.parametrize("delta,Delta", CASES)
def test_F_is_integral_of_f(delta, Delta):
    T = Delta + delta
    for t in np.linspace(0.0, T, 37):
        pts = [p for p in (delta, Delta) if 0 < p < t]
        val, _ = integrate.quad(lambda s: float(sq.pgse_f(s, delta, Delta)), 0.0, t,
                                points=pts or None, limit=200)
        assert abs(float(sq.pgse_F(t, delta, Delta)) - val) < 1e-7 * max(1.0, delta)


@pytest.mark.parametrize("delta,Delta", CASES)
def test_int_F2_closed_form(delta, Delta):
    T = Delta + delta
    val, _ = integrate.quad(lambda s: float(sq.pgse_F(s, delta, Delta)) ** 2, 0.0, T,
                            points=[delta, Delta], limit=200)
    assert sq.pgse_int_F2(delta, Delta) == pytest.approx(val, rel=1e-10)


def test_F_vanishes_at_echo():
    # F(T) = 0 at T = Delta + delta: the transformed and physical fields agree.
    for delta, Delta in CASES:
        assert float(sq.pgse_F(Delta + delta, delta, Delta)) == 0.0


def test_profile_edges():
    # eq. pgse: closed at delta, open at Delta, closed at Delta + delta.
    d, D = 10600.0, 13400.0
    f = sq.pgse_f(np.array([0.0, d, d + 1e-6, D, D + 1e-6, D + d, D + d + 1e-6]), d, D)
    assert list(f) == [1.0, 1.0, 0.0, 0.0, -1.0, -1.0, 0.0]


def test_b_to_G_roundtrip_and_units():
    d, D = 10600.0, 13400.0
    G = float(sq.b_to_G(1000.0, d, D))
    # b = G^2 int F^2 (eq. b_value with G = gamma |g|).
    assert G * G * sq.pgse_int_F2(d, D) == pytest.approx(1000.0, rel=1e-14)
    # Config-0 values: G = 3.00337e-5 rad/(um us), |g| = 112.27 mT/m.
    assert G == pytest.approx(3.00337e-5, rel=1e-5)
    assert float(sq.G_to_tesla_per_m(G)) == pytest.approx(0.11227, rel=1e-4)


def test_interval_f_matches_one_sided_limits():
    d, D, dt = 10600.0, 13400.0, 100.0
    fi = sq.interval_f(d, D, dt)
    t = sq.time_grid(d, D, dt)
    eps = 1e-7
    left = sq.pgse_f(t[:-1] + eps, d, D)     # f(t^{n-1}+)
    right = sq.pgse_f(t[1:] - eps, d, D)     # f(t^n-)
    assert np.array_equal(fi, left) and np.array_equal(fi, right)
    assert len(fi) == 240
    assert math.isclose(fi.sum() * dt, 0.0, abs_tol=1e-9)
