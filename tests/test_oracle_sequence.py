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


# --------------------------------------------------------------- general profiles
# Sec. 3 ("General diffusion-encoding sequence": the cos-OGSE definition) and
# Sec. 4 (PGSE, double PGSE, cos-OGSE, sin-OGSE, trapezoidal and double
# trapezoidal profiles). Readings are listed in oracle/sequence.py.

GENERAL = [
    ("pgse", (10600.0, 13400.0)),
    ("double_pgse", (2000.0, 4000.0, 1000.0)),
    ("double_pgse", (10000.0, 10000.0, 0.0)),
    ("cos_ogse", (10000.0, 10000.0, 2.0)),
    ("cos_ogse", (6000.0, 9000.0, 3.0)),
    ("sin_ogse", (10000.0, 14000.0, 1.0)),
    ("trap_pgse", (10600.0, 13400.0, 1000.0)),
    ("double_trap_pgse", (2000.0, 4000.0, 400.0, 0.0)),
]


def _fine_F(prof, n=400001):
    # Independent of the closed forms: cumulative midpoint rule for f on a
    # fine grid (f sampled inside the cells, so jumps on nodes are exact).
    pts = sorted(set([0.0, prof.T] + [p for p in prof.breakpoints() if 0 < p < prof.T]))
    t = np.unique(np.concatenate([
        np.linspace(a, b, max(2, int(n * (b - a) / prof.T))) for a, b in zip(pts[:-1], pts[1:])]))
    mid = 0.5 * (t[1:] + t[:-1])
    f = np.array([prof.f(v) for v in mid])
    F = np.concatenate([[0.0], np.cumsum(f * np.diff(t))])
    return t, F


@pytest.mark.parametrize("kind,params", GENERAL)
def test_general_F_is_integral_of_f_and_vanishes_at_echo(kind, params):
    prof = sq.Profile(kind, params)
    pts = prof.breakpoints()
    for t in np.linspace(0.0, prof.T, 29):
        inner = [p for p in pts if 0 < p < t]
        val, _ = integrate.quad(prof.f, 0.0, t, points=inner or None, limit=400,
                                epsabs=1e-9)
        assert abs(prof.F(t) - val) < 1e-7 * params[0]
    assert abs(prof.F(prof.T)) < 1e-9 * params[0]


@pytest.mark.parametrize("kind,params", GENERAL)
def test_general_int_F2_against_fine_grid(kind, params):
    prof = sq.Profile(kind, params)
    t, F = _fine_F(prof)
    val = np.trapezoid(F * F, t)
    assert prof.int_F2() == pytest.approx(val, rel=2e-6)


def test_general_int_F2_closed_forms():
    d, D = 10600.0, 13400.0
    assert sq.Profile("pgse", (d, D)).int_F2() == pytest.approx(sq.pgse_int_F2(d, D), rel=1e-12)
    # a double profile without gap: F returns to 0 between the blocks
    assert sq.Profile("double_pgse", (d, D, 700.0)).int_F2() == pytest.approx(
        2 * sq.pgse_int_F2(d, D), rel=1e-12)
    for n in (1, 2, 3):
        w = 2 * n * math.pi / 10000.0
        # cos lobe: F = sin(w t)/w, int = delta/(2 w^2) per lobe
        assert sq.Profile("cos_ogse", (10000.0, 12000.0, n)).int_F2() == pytest.approx(
            10000.0 / w ** 2, rel=1e-11)
        # sin lobe: F = (1 - cos(w t))/w, int = 3 delta/(2 w^2) per lobe
        assert sq.Profile("sin_ogse", (10000.0, 12000.0, n)).int_F2() == pytest.approx(
            3 * 10000.0 / w ** 2, rel=1e-11)


def test_trapezoid_tends_to_pgse():
    d, D = 10600.0, 13400.0
    ref = sq.pgse_int_F2(d, D)
    errs = [abs(sq.Profile("trap_pgse", (d, D, e)).int_F2() - ref) / ref for e in (400, 200, 100)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-2
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05)   # first order in the ramp


def test_general_pgse_equals_pgse_functions():
    d, D = 10600.0, 13400.0
    prof = sq.Profile("pgse", (d, D))
    for t in np.linspace(0, d + D, 61):
        assert prof.F(t) == pytest.approx(float(sq.pgse_F(t, d, D)), abs=1e-9)
        assert prof.f(t) == float(sq.pgse_f(t, d, D))


@pytest.mark.parametrize("kind,params", GENERAL)
def test_one_sided_limits(kind, params):
    prof = sq.Profile(kind, params)
    dt = 200.0
    if not prof.on_grid(dt):
        pytest.skip("breakpoints off the 200 us grid")
    n = int(round(prof.T / dt))
    e = 1e-6
    for k in range(1, n + 1):
        lo, hi = prof.f_limits((k - 1) * dt, k * dt)
        assert lo == pytest.approx(prof.f((k - 1) * dt + e), abs=1e-6)
        assert hi == pytest.approx(prof.f(k * dt - e), abs=1e-6)
