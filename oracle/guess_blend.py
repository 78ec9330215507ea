"""Learned blend of extrapolations for the initial guess (oracle, FP64).

Test infrastructure only (see the package header).

Each theta-step (Appendix A, eq. theta_discretization) may start its Krylov
solve from any guess; the paper solves each step from scratch. The guess
here blends three extrapolations of the solution history u_k = u^{n-1-k},
k = 0..4, with two coefficients per system and step:

    x_dc  = sum_k c_k u_k,  c = (49, -36, -26, 44, -15) / 16  (damped cubic)
    x_lin = 2 u_0 - u_1                                       (linear)
    x_0   = x_dc + a (x_lin - x_dc) + b (u_0 - x_dc)

i.e. weights w = (1 - a - b) c + a (2, -1, 0, 0, 0) + b (1, 0, 0, 0, 0),
which sum to 1 for every (a, b) (a constant history is reproduced), and
(a, b) = (0, 0) is the damped cubic itself. A network predicts (a, b) from
per-system features; its training targets are the (a, b) that minimise
||x_0 - u^n||^2 over the real span (real inner products of the complex
vectors) once u^n is known:

    [d1.d1  d1.d2] [a]   [-d1.e]      d1 = x_lin - x_dc, d2 = u_0 - x_dc,
    [d2.d1  d2.d2] [b] = [-d2.e],     e = x_dc - u^n.

Features (16): G h v(t^{n-k}) for k = 0..5 (v = F for the transformed form,
the one-sided f for the U-form; h the longest edge), log(theta dt D/h^2),
log(1 + theta dt D (G v_n)^2), log(1 + theta dt D |G v_n| / h),
log(1 + theta dt kappa / h), |q_x|, |q_y|, |q_z|, three zeros.

Pins (tests/test_oracle_guess_blend.py): the weights sum to 1 and give the
damped cubic, linear and previous-step guesses at (0,0), (1,0), (0,1);
optimal_blend recovers planted (a, b) exactly, equals NumPy's least squares
on random data and never does worse than the damped cubic; the features on
simple cases.
"""

from __future__ import annotations

import math

import numpy as np

C_DC = np.array([49.0, -36.0, -26.0, 44.0, -15.0]) / 16.0
C_LIN = np.array([2.0, -1.0, 0.0, 0.0, 0.0])
C_PREV = np.array([1.0, 0.0, 0.0, 0.0, 0.0])
CLIP = 4.0  # |a|, |b| above this are clipped (targets and predictions)


def blend_weights(a: float, b: float) -> np.ndarray:
    """Weights of u^{n-1} .. u^{n-5} for the blend (a, b)."""
    return (1.0 - a - b) * C_DC + a * C_LIN + b * C_PREV


def guess(hist, a: float, b: float):
    """x_0 from the history [u^{n-1}, ..., u^{n-5}]."""
    w = blend_weights(a, b)
    return sum(wk * uk for wk, uk in zip(w, hist))


def optimal_blend(hist, un):
    """(a, b) minimising ||x_0 - u^n|| (real coefficients), or None when the
    2 x 2 system is singular (a history without change)."""
    u0, u1 = hist[0], hist[1]
    x_dc = sum(c * u for c, u in zip(C_DC, hist))
    d1 = (2.0 * u0 - u1) - x_dc
    d2 = u0 - x_dc
    e = x_dc - un
    g11 = np.vdot(d1, d1).real
    g12 = np.vdot(d1, d2).real
    g22 = np.vdot(d2, d2).real
    r1 = -np.vdot(d1, e).real
    r2 = -np.vdot(d2, e).real
    det = g11 * g22 - g12 * g12
    if not (g11 > 0 and g22 > 0 and det > 1e-12 * g11 * g22):
        return None
    a = (r1 * g22 - r2 * g12) / det
    b = (g11 * r2 - g12 * r1) / det
    return float(np.clip(a, -CLIP, CLIP)), float(np.clip(b, -CLIP, CLIP))


def features(G: float, v_hist, h: float, dt: float, theta: float, d_max: float,
             kappa: float, q) -> np.ndarray:
    """Sixteen inputs for one system at step n; v_hist = [v(t^n), ...,
    v(t^{n-5})]."""
    q = np.asarray(q, dtype=np.float64)
    nq = np.linalg.norm(q)
    qn = q / nq if nq > 0 else np.array([1.0, 0.0, 0.0])
    x = np.zeros(16)
    for k in range(6):
        x[k] = G * h * v_hist[k]
    k_ = theta * dt
    gf = abs(G * v_hist[0])
    x[6] = math.log(k_ * d_max / (h * h))
    x[7] = math.log1p(k_ * d_max * gf * gf)
    x[8] = math.log1p(k_ * d_max * gf / h)
    x[9] = math.log1p(k_ * kappa / h)
    x[10:13] = np.abs(qn)
    return x
