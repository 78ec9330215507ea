"""Gradient profiles and b-value conversion (oracle, FP64).

Test infrastructure only (see the package header).

PGSE (below) and general piecewise profiles (class Profile, further down).

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


# ---------------------------------------------------------------------------
# General temporal profiles (Sec. 3, "General diffusion-encoding sequence";
# Sec. 4, the comparison of PGSE, double PGSE, cos-OGSE, sin-OGSE,
# trapezoidal and double trapezoidal profiles).
#
# A profile is a list of pieces (a, b, shape) on which f is smooth; f is 0
# outside them. Shapes, with s = +-1 the lobe sign:
#   ("const", s)            f = s
#   ("cos", s, t0, w)       f = s cos(w (t - t0))
#   ("sin", s, t0, w)       f = s sin(w (t - t0))
#   ("ramp", s, t0, eps)    f = s (t - t0) / eps          (linear ramp)
# F(t) = int_0^t f is taken piece by piece in closed form; int_0^T F^2 by
# adaptive quadrature over the pieces (closed forms for PGSE and OGSE are
# used by the pins). Readings (the paper gives the cos-OGSE formula and
# names the others):
#  * cos/sin-OGSE: n periods per lobe, w = 2 n pi / delta, the second lobe
#    (sign -1) starts at tau = (delta + Delta) / 2, echo T = delta + Delta
#    (as in the paper's cos-OGSE definition);
#  * trapezoidal PGSE: each pulse of total length delta rises linearly over
#    eps, stays at 1, falls linearly over eps; second pulse (sign -1) starts
#    at Delta; T = Delta + delta;
#  * double profiles: the single profile followed, after a mixing time t_m,
#    by the same profile again; T = 2 (Delta + delta) + t_m.
# ---------------------------------------------------------------------------

KINDS = ("pgse", "double_pgse", "cos_ogse", "sin_ogse", "trap_pgse", "double_trap_pgse")


def _pieces_single(kind, p):
    d, D = float(p[0]), float(p[1])
    if kind == "pgse":
        return [(0.0, d, ("const", 1.0)), (D, D + d, ("const", -1.0))], D + d
    if kind in ("cos_ogse", "sin_ogse"):
        n = float(p[2])
        w = 2.0 * n * math.pi / d
        tau = 0.5 * (d + D)
        sh = "cos" if kind == "cos_ogse" else "sin"
        return [(0.0, d, (sh, 1.0, 0.0, w)), (tau, tau + d, (sh, -1.0, tau, w))], d + D
    if kind == "trap_pgse":
        eps = float(p[2])
        out = []
        for start, s in ((0.0, 1.0), (D, -1.0)):
            out.append((start, start + eps, ("ramp", s, start, eps)))
            if d - 2 * eps > 0:
                out.append((start + eps, start + d - eps, ("const", s)))
            out.append((start + d - eps, start + d, ("ramp", -s, start + d, eps)))
        return out, D + d
    raise ValueError(kind)


class Profile:
    """Temporal profile f, its integral F and int_0^T F^2 (oracle, FP64)."""

    def __init__(self, kind, params):
        kind = str(kind)
        self.kind = kind
        self.params = tuple(float(v) for v in params)
        if kind.startswith("double_"):
            base = kind[len("double_"):]
            pcs, T1 = _pieces_single(base, self.params)
            tm = self.params[-1]
            shift = T1 + tm
            self.pieces = list(pcs) + [(a + shift, b + shift, _shift(sh, shift)) for a, b, sh in pcs]
            self.T = 2.0 * T1 + tm
        else:
            self.pieces, self.T = _pieces_single(kind, self.params)
        self.pieces.sort(key=lambda x: x[0])
        # F at the start of every piece (F is 0 before the first).
        self._F0 = []
        acc = 0.0
        for a, b, sh in self.pieces:
            self._F0.append(acc)
            acc += _piece_int(sh, a, b)
        self._F_end = acc

    def breakpoints(self):
        pts = set()
        for a, b, _ in self.pieces:
            pts.add(a)
            pts.add(b)
        return sorted(pts)

    def f(self, t):
        """f(t); at a breakpoint the value of the piece that ends there."""
        t = float(t)
        for a, b, sh in self.pieces:
            if a < t <= b or (a == 0.0 and t == 0.0):
                return _piece_f(sh, t)
        return 0.0

    def f_limits(self, t0, t1):
        """One-sided limits (f(t0+), f(t1-)) on an interval (t0, t1) that lies
        inside one piece or between pieces."""
        for a, b, sh in self.pieces:
            if a <= t0 and t1 <= b:
                return _piece_f(sh, t0), _piece_f(sh, t1)
        return 0.0, 0.0

    def F(self, t):
        t = float(t)
        acc = 0.0
        for (a, b, sh), F0 in zip(self.pieces, self._F0):
            if t <= a:
                return F0  # f = 0 between the previous piece and this one
            if t <= b:
                return F0 + _piece_int(sh, a, t)
            acc = F0 + _piece_int(sh, a, b)
        return acc

    def int_F2(self):
        """int_0^T F^2 by adaptive quadrature between the breakpoints."""
        from scipy import integrate
        pts = [0.0] + [p for p in self.breakpoints() if 0.0 < p < self.T] + [self.T]
        total = 0.0
        for lo, hi in zip(pts[:-1], pts[1:]):
            if hi > lo:
                v, _ = integrate.quad(lambda s: self.F(s) ** 2, lo, hi, epsabs=0.0,
                                      epsrel=1e-13, limit=400)
                total += v
        return total

    def on_grid(self, dt):
        """Every breakpoint is a multiple of dt (within 1e-9) and T too."""
        for p in self.breakpoints() + [self.T]:
            r = p / dt
            if abs(r - round(r)) > 1e-9 * max(1.0, r):
                return False
        return True


def _shift(sh, s):
    if sh[0] == "const":
        return sh
    return (sh[0], sh[1], sh[2] + s, sh[3])


def _piece_f(sh, t):
    if sh[0] == "const":
        return sh[1]
    if sh[0] == "cos":
        return sh[1] * math.cos(sh[3] * (t - sh[2]))
    if sh[0] == "sin":
        return sh[1] * math.sin(sh[3] * (t - sh[2]))
    if sh[0] == "ramp":
        return sh[1] * (t - sh[2]) / sh[3]
    raise ValueError(sh)


def _piece_int(sh, a, t):
    """int_a^t f over one piece, in closed form."""
    if sh[0] == "const":
        return sh[1] * (t - a)
    if sh[0] == "cos":
        s, t0, w = sh[1], sh[2], sh[3]
        return s * (math.sin(w * (t - t0)) - math.sin(w * (a - t0))) / w
    if sh[0] == "sin":
        s, t0, w = sh[1], sh[2], sh[3]
        return s * (math.cos(w * (a - t0)) - math.cos(w * (t - t0))) / w
    if sh[0] == "ramp":
        s, t0, e = sh[1], sh[2], sh[3]
        return s * ((t - t0) ** 2 - (a - t0) ** 2) / (2.0 * e)
    raise ValueError(sh)


def profile_of(seq):
    """The Profile of a sequence description: a PGSE (delta, Delta, dt, theta)
    record, or one with kind and params."""
    kind = getattr(seq, "kind", "pgse")
    params = getattr(seq, "params", None)
    if params is None:
        params = (seq.delta, seq.Delta)
    return Profile(kind, params)
