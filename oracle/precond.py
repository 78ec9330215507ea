"""Polynomial preconditioning inside flexible CG, and the spectral data that
trains its learned interval (oracle, FP64).

Test infrastructure only (see the package header).

The paper leaves the Krylov method of each theta-step unnamed (Sec. 3,
"Diffusion MRI simulation library"); the step systems are those of
Appendix A, eq. theta_discretization, whose transformed-form matrix
A = M/k + theta L(F^n) is Hermitian positive definite. With D = diag(A)
(real and positive), this module states:

* chebyshev_apply: z = p(D^-1 A) D^-1 r, the Chebyshev acceleration of
  Jacobi (Saad, Iterative Methods for Sparse Linear Systems, 2nd ed.,
  Sec. 12.3, three-term recurrence) on an interval [a, b] with m terms,
  started from zero. Its polynomial satisfies
      1 - lam p(lam) = T_m((b + a - 2 lam) / (b - a)) / T_m((b + a) / (b - a)),
  which is positive on (0, b] for every 0 < a < b, so z is a Hermitian
  positive definite preconditioner whenever b bounds the spectrum of D^-1 A.
  m = 1 is Jacobi scaled by 2 / (a + b).
* fcg: flexible CG, Notay (2000) FCG(1): the new direction is the
  preconditioned residual made A-orthogonal to the previous direction,
  beta = -(q^H z) / (p^H q) with q = A p; alpha = (r^H z) / (p^H q). With a
  fixed Hermitian positive definite preconditioner it equals preconditioned
  CG in exact arithmetic; with any preconditioner the exact line search keeps
  the A-norm of the error from growing.
* pcg_coefficients / ritz_extremes: Jacobi-preconditioned CG recording its
  alpha_k and beta_k, and the extreme eigenvalues of the Lanczos tridiagonal
  they define (Saad, Sec. 6.7.3): diagonal 1/alpha_0, 1/alpha_k +
  beta_{k-1}/alpha_{k-1}; off-diagonal sqrt(beta_{k-1})/alpha_{k-1}. Their
  eigenvalues (Ritz values) lie inside the spectrum of D^-1 A and reach its
  ends as the iteration proceeds.
* features / interval_from_output / targets_from_ritz: the per-system,
  per-step inputs of the interval network (dimensionless ratios of the
  operator's terms to the mass term M/k), the interval its two outputs give,
  and the outputs a PCG run's Ritz values ask for.

Pins (tests/test_oracle_precond.py): the Chebyshev residual polynomial
against its closed form in the eigenbasis of D^-1/2 A D^-1/2; FCG with m = 1 against SciPy's
Jacobi-preconditioned CG (same iterates, same count); FCG solutions against
a direct solve; Ritz values of a full-length Lanczos run against the
eigenvalues of D^-1 A, and interlacing inside the spectrum for short runs.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from . import sequence as seqmod
from .timestep import _n_steps, _qB, _unit


def step_operator(asm, seq, b: float, q, n: int):
    """Left matrix A_n and the right operator R_n of transformed-form step n
    (Appendix A, eq. theta_discretization): A_n u^n = R_n u^{n-1}."""
    k = float(seq.dt)
    th = float(seq.theta)
    prof = seqmod.profile_of(seq)
    N = _n_steps(prof, k)
    if not 1 <= n <= N:
        raise ValueError("step out of range")
    G = math.sqrt(b / prof.int_F2()) if b > 0 else 0.0
    qn = _unit(q)
    base = (asm.S + asm.IG + asm.R2).tocsr()
    Mk = (asm.M / k).tocsr()
    qB = _qB(asm, qn).tocsr()
    qq = (qn[0] ** 2, qn[1] ** 2, qn[2] ** 2, 2 * qn[0] * qn[1], 2 * qn[0] * qn[2],
          2 * qn[1] * qn[2])
    Mq = sum(c * m for c, m in zip(qq, asm.MDab)).tocsr()

    def L(Fv):
        return base + (G * Fv) ** 2 * Mq + 1j * (G * Fv) * qB

    Fn, Fp = prof.F(n * k), prof.F((n - 1) * k)
    A = (Mk + th * L(Fn)).tocsr().astype(np.complex128)
    R = (Mk - (1.0 - th) * L(Fp)).tocsr().astype(np.complex128)
    return A, R


def chebyshev_apply(A, dinv, r, a: float, b: float, m: int):
    """z = p(D^-1 A) D^-1 r after m Chebyshev terms on [a, b] from y = 0."""
    if not (0.0 < a < b) or m < 1:
        raise ValueError("need 0 < a < b and m >= 1")
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = (dinv * r) / theta
    y = d.copy()
    for _ in range(1, m):
        w = dinv * (r - A @ y)
        rho_next = 1.0 / (2.0 * sigma - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * w
        y = y + d
        rho = rho_next
    return y


def chebyshev_residual_poly(lam, a: float, b: float, m: int):
    """Closed form of 1 - lam p(lam) for the m-term Chebyshev polynomial."""
    lam = np.asarray(lam, dtype=np.float64)

    def T(m_, x):
        x = np.asarray(x, dtype=np.float64)
        out = np.empty_like(x)
        inside = np.abs(x) <= 1.0
        out[inside] = np.cos(m_ * np.arccos(x[inside]))
        xo = x[~inside]
        out[~inside] = np.sign(xo) ** m_ * np.cosh(m_ * np.arccosh(np.abs(xo)))
        return out

    return T(m, (b + a - 2.0 * lam) / (b - a)) / T(m, np.array([(b + a) / (b - a)]))[0]


def fcg(A, rhs, x0, rtol: float, precond, max_iter: int = 5000):
    """Flexible CG (FCG(1)) on Hermitian positive definite A; precond(r)
    returns z. Stops when ||r|| <= rtol ||rhs||. Returns (x, iterations)."""
    x = np.array(x0, dtype=np.complex128)
    r = rhs - A @ x
    bb = np.vdot(rhs, rhs).real
    if np.vdot(r, r).real <= rtol * rtol * bb:
        return x, 0
    z = precond(r)
    p = z.copy()
    rho = np.vdot(r, z)
    for it in range(1, max_iter + 1):
        q = A @ p
        sigma = np.vdot(p, q)
        alpha = rho / sigma
        x = x + alpha * p
        r = r - alpha * q
        if np.vdot(r, r).real <= rtol * rtol * bb:
            return x, it
        z = precond(r)
        beta = -np.vdot(q, z) / sigma
        rho = np.vdot(r, z)
        p = z + beta * p
    raise RuntimeError("fcg did not converge")


def pcg_coefficients(A, rhs, x0, rtol: float, max_iter: int = 5000):
    """Jacobi-preconditioned CG; returns (x, alphas, betas) with
    beta_k = rho_{k+1} / rho_k for every iteration that continued."""
    dinv = 1.0 / A.diagonal().real
    x = np.array(x0, dtype=np.complex128)
    r = rhs - A @ x
    bb = np.vdot(rhs, rhs).real
    alphas, betas = [], []
    if np.vdot(r, r).real <= rtol * rtol * bb:
        return x, alphas, betas
    z = dinv * r
    p = z.copy()
    rho = np.vdot(r, z)
    for _ in range(max_iter):
        q = A @ p
        alpha = rho / np.vdot(p, q)
        alphas.append(alpha)
        x = x + alpha * p
        r = r - alpha * q
        if np.vdot(r, r).real <= rtol * rtol * bb:
            return x, alphas, betas
        z = dinv * r
        rho_new = np.vdot(r, z)
        beta = rho_new / rho
        betas.append(beta)
        rho = rho_new
        p = z + beta * p
    raise RuntimeError("pcg did not converge")


def lanczos_tridiagonal(alphas, betas):
    """Tridiagonal matrix of the Lanczos process behind PCG's coefficients
    (real parts: for Hermitian positive definite systems they are real)."""
    al = np.real(np.asarray(alphas, dtype=np.complex128))
    be = np.real(np.asarray(betas, dtype=np.complex128))[: max(0, len(al) - 1)]
    n = len(al)
    T = np.zeros((n, n))
    for k in range(n):
        T[k, k] = 1.0 / al[k] + (be[k - 1] / al[k - 1] if k > 0 else 0.0)
        if k + 1 < n:
            T[k, k + 1] = T[k + 1, k] = math.sqrt(be[k]) / al[k]
    return T


def ritz_extremes(alphas, betas):
    """(smallest, largest) Ritz value of the PCG run."""
    ev = np.linalg.eigvalsh(lanczos_tridiagonal(alphas, betas))
    return float(ev[0]), float(ev[-1])


def features(dt: float, theta: float, d_max: float, h: float, kappa: float, gG: float,
             F: float, q) -> np.ndarray:
    """Sixteen inputs of the interval network for one system at one step:
    log(theta k D/h^2) (stiffness / mass), log(1 + theta k D (G F)^2) (the
    g.Dg mass term / mass), log(1 + theta k D |G F| / h) (first-order term /
    mass), log(1 + theta k kappa / h) (membranes / mass), |q_x|, |q_y|, |q_z|
    of the unit direction, then zeros. gG is the gyromagnetic ratio times the
    gradient amplitude, F the profile integral at t^n."""
    qn = _unit(q)
    gf = abs(gG * F)
    x = np.zeros(16)
    x[0] = math.log(theta * dt * d_max / (h * h))
    x[1] = math.log1p(theta * dt * d_max * gf * gf)
    x[2] = math.log1p(theta * dt * d_max * gf / h)
    x[3] = math.log1p(theta * dt * kappa / h)
    x[4:7] = np.abs(qn)
    return x


# The network predicts the interval relative to a reference interval, so an
# all-zero network gives the reference itself; the upper end gets a margin
# over the largest Ritz value, which approaches lam_max from below.
A_REF = 0.5
B_REF = 1.5
MARGIN = 1.1


def interval_from_output(y0: float, y1: float):
    """Interval used by the preconditioner from the network output:
    [A_REF e^y0, B_REF e^y1] with y clipped to [-20, 20], or the reference
    interval when that is not finite or not an interval (a (1 + 1e-3) >= b)."""
    if not (math.isfinite(y0) and math.isfinite(y1)):
        return A_REF, B_REF
    a = A_REF * math.exp(min(20.0, max(-20.0, y0)))
    b = B_REF * math.exp(min(20.0, max(-20.0, y1)))
    if not a * 1.001 < b:
        return A_REF, B_REF
    return a, b


def targets_from_ritz(lo: float, hi: float):
    """Training targets of one PCG run: (log(lo / A_REF), log(MARGIN hi / B_REF))."""
    return math.log(lo / A_REF), math.log(MARGIN * hi / B_REF)


def jacobi_spectrum(A):
    """Eigenvalues of D^-1 A (dense; small matrices only)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    d = np.real(np.diag(Ad))
    s = 1.0 / np.sqrt(d)
    return np.linalg.eigvalsh((s[:, None] * Ad) * s[None, :])
