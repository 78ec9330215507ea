"""PGSE gradient profile and b-value conversion (oracle, FP64).

Test infrastructure only (see the package header).

* f(t): Sec. 2, eq. pgse -- +1 on [0, delta], -1 on (Delta, Delta+delta],
  0 otherwise.
* F(t) = int_0^t f(s) ds: Sec. 2, definition under eq. btpde_bc.
* b = gamma^2 |g|^2 int_0^T F(s)^2 ds: Sec. 2, eq. b_value. The solver needs
  only G = gamma |g| (rad per um per us), so b -> G = sqrt(b / int F^2).

Pins: the closed form of int F^2 is checked against adaptive quadrature of
F^2, and F against quadrature of f (tests/test_oracle_sequence.py).
"""

from __future__ import annotations

import math

import numpy as np

GAMMA = 2.67513e8  # rad s^-1 T^-1, the water-proton value the paper states (Sec. 2)


def pgse_f(t, delta, Delta):
    """PGSE temporal profile, eq. pgse."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    out[(t >= 0.0) & (t <= delta)] = 1.0
    out[(t > Delta) & (t <= Delta + delta)] = -1.0
    return out


def pgse_F(t, delta, Delta):
    """F(t) = int_0^t f: a ramp up to delta, flat, then a ramp back to 0."""
    t = np.asarray(t, dtype=np.float64)
    up = np.clip(t, 0.0, delta)
    down = np.clip(t - Delta, 0.0, delta)
    return up - down


def pgse_int_F2(delta, Delta):
    """int_0^T F(s)^2 ds for PGSE with T = Delta + delta.

    Ramp 0..delta contributes delta^3/3, the plateau delta^2 (Delta - delta),
    the ramp down another delta^3/3: total delta^2 (Delta - delta/3).
    """
    return delta * delta * (Delta - delta / 3.0)


def b_to_G(b, delta, Delta):
    """gamma*|g| in rad/(um us) for a b-value in us/um^2 (== s/mm^2)."""
    b = np.asarray(b, dtype=np.float64)
    return np.sqrt(b / pgse_int_F2(delta, Delta))


def G_to_tesla_per_m(G):
    """|g| in T/m from G = gamma |g| in rad/(um us)."""
    # rad/(um us) = 1e12 rad/(m s); divide by gamma [rad/(s T)].
    return np.asarray(G) * 1e12 / GAMMA


def time_grid(delta, Delta, dt):
    """t^n = n dt, n = 0..N with N = (Delta + delta)/dt (must be an integer)."""
    T = Delta + delta
    N = int(round(T / dt))
    if abs(N * dt - T) > 1e-9 * T:
        raise ValueError("echo time must be a multiple of dt")
    return np.arange(N + 1, dtype=np.float64) * dt


def interval_f(delta, Delta, dt):
    """f on each step interval (t^{n-1}, t^n), n = 1..N (midpoint value).

    Pulse edges on the grid make f constant on every open interval, so the
    one-sided limits f(t^{n-1}+) and f(t^n-) both equal this value.
    """
    t = time_grid(delta, Delta, dt)
    mid = 0.5 * (t[:-1] + t[1:])
    return pgse_f(mid, delta, Delta)


def check_grid(delta, Delta, dt):
    """Pulse edges delta and Delta must be multiples of dt."""
    for v in (delta, Delta):
        r = v / dt
        if abs(r - round(r)) > 1e-9 * max(1.0, abs(r)):
            return False
    return math.isfinite(dt) and dt > 0
