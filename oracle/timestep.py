"""Theta-method time stepping with exact sparse solves (oracle, FP64).

Test infrastructure only (see the package header).

Transformed (strong pseudo-periodic) form, Appendix A,
eq. theta_discretization and eq. linear_billinear. With
  L(F) = S + I_Gamma + R2 + (G F)^2 M_D + i G F (q . B)
each step n = 1..N solves
  (M/k + theta L(F^n)) u^n = (M/k - (1 - theta) L(F^{n-1})) u^{n-1}.

U-form (Neumann walls), Appendix B, eq. matrix_form with eq. loadvec, with
the T2 term on the mass matrix (the printed A multiplies 1/T2 by J, which
conflicts with eq. loadvec where it multiplies the plain mass):
  L(f) = S + I_Gamma + R2 + i G f (q . J),
  (M/k + theta L(f(t^n-))) U^n = (M/k - (1 - theta) L(f(t^{n-1}+))) U^{n-1},
with the one-sided limits of f on the step interval (profile breakpoints lie
on the grid; for PGSE both limits are the interval's constant value).

Any temporal profile of oracle.sequence.Profile (PGSE, double PGSE, cos- and
sin-OGSE, trapezoidal, double trapezoidal) enters through F(t^n) (transformed
form) or the one-sided limits of f (U-form), and int_0^T F^2 in b -> G.

Signal (Sec. 2, eq. signal): S = int U(T) = sum_i w_i u_i^N, because
F(T) = 0 at T = Delta + delta makes u(T) = U(T).

Each step is solved exactly with SuperLU (scipy.sparse.linalg.splu, minimum
degree ordering on A + A^T). The left operator depends on the step only
through F^n (or f_n), so factorizations are cached by that value. For meshes
where sparse LU fill makes that impractical (tens of thousands of 3-D DOFs),
solver="krylov" solves each step with SciPy's conjugate gradient (Hermitian
transformed operator) or GMRES (complex-symmetric U-form) to a relative
residual of 1e-13, i.e. exact up to rounding; tests pin it to SuperLU.

Pins (tests/test_oracle_*.py): free diffusion closed-form recurrence and the
Stejskal-Tanner limit exp(-D b) with second-order time convergence; mass
conservation at b = 0; kappa -> 0 decoupling and kappa -> inf
single-compartment limit; S(-q) = conj S(q); 1-D slab matrix formalism for
both forms; the two forms agree on a non-symmetric case; dense solves equal
SuperLU.

Parity unpinned: signals of the staircase compartment geometries with the
gradient across the membranes (e.g. q perpendicular to the cylinder) have no
closed form; there the oracle rests on the invariants and limits above.
"""

from __future__ import annotations

import math
from collections import OrderedDict
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import sequence as seqmod
from .fem import Assembly, assemble


class _LUCache:
    def __init__(self, size: int):
        self.size = int(size)
        self.d: "OrderedDict[float, object]" = OrderedDict()

    def get(self, key, build):
        if key in self.d:
            self.d.move_to_end(key)
            return self.d[key]
        lu = build()
        if self.size > 0:
            self.d[key] = lu
            while len(self.d) > self.size:
                self.d.popitem(last=False)
        return lu


def _qB(asm: Assembly, q):
    return q[0] * asm.B[0] + q[1] * asm.B[1] + q[2] * asm.B[2]


def _qJ(asm: Assembly, q):
    return q[0] * asm.J[0] + q[1] * asm.J[1] + q[2] * asm.J[2]


KRYLOV_RTOL = 1e-13


def _splu(A):
    return spla.splu(A.tocsc().astype(np.complex128), permc_spec="MMD_AT_PLUS_A")


def _krylov(A, rhs, x0, hermitian):
    A = A.tocsr().astype(np.complex128)
    dinv = 1.0 / A.diagonal()
    P = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v, dtype=np.complex128)
    if hermitian:
        x, info = spla.cg(A, rhs, x0=x0, rtol=KRYLOV_RTOL, atol=0.0, maxiter=20000, M=P)
    else:
        x, info = spla.gmres(A, rhs, x0=x0, rtol=KRYLOV_RTOL, atol=0.0, restart=60,
                             maxiter=2000, M=P)
    if info != 0:
        raise RuntimeError("oracle Krylov solve did not reach rtol=%g (info=%d)"
                           % (KRYLOV_RTOL, info))
    return x


def _n_steps(prof, k):
    """N = T / k; the profile's breakpoints and T must lie on the time grid."""
    if not prof.on_grid(k):
        raise ValueError("profile breakpoints and the echo time must be multiples of dt")
    return int(round(prof.T / k))


def _unit(q):
    q = np.asarray(q, dtype=np.float64)
    nq = np.linalg.norm(q)
    return q / nq if nq > 0 else np.array([1.0, 0.0, 0.0])


def solve_transformed(asm: Assembly, seq, b: float, q, n_steps: Optional[int] = None,
                      cache_size: int = 256, return_u: bool = False, solver: str = "splu",
                      start_step: int = 0):
    """Signal of one (b, q) system with the transformed operator.

    n_steps limits the run to the first n steps (for timing samples and
    intermediate checks); the signal is then sum w u^n at that step, which is
    the physical signal only when F(t^n) = 0. start_step = s > 0 starts the
    recurrence at t^s from the initial magnetization instead of t^0 and takes
    steps s+1 .. s+n_steps (a timing sample of later steps; not a physical
    trajectory).
    """
    k = float(seq.dt)
    th = float(seq.theta)
    prof = seqmod.profile_of(seq)
    N_all = _n_steps(prof, k)
    t = np.arange(N_all + 1, dtype=np.float64) * k
    F = np.array([prof.F(v) for v in t])
    G = math.sqrt(b / prof.int_F2())
    qn = _unit(q)
    s0 = int(start_step)
    N = len(t) - 1 if n_steps is None else min(len(t) - 1, s0 + int(n_steps))

    base = (asm.S + asm.IG + asm.R2).tocsr()
    Mk = (asm.M / k).tocsr()
    qB = _qB(asm, qn).tocsr()
    # g.Dg mass term for the direction q: sum_ab q_a q_b int D_ab phi_i phi_j
    qq = (qn[0] ** 2, qn[1] ** 2, qn[2] ** 2, 2 * qn[0] * qn[1], 2 * qn[0] * qn[2],
          2 * qn[1] * qn[2])
    Mq = sum(c * m for c, m in zip(qq, asm.MDab)).tocsr()

    def L(Fv):
        return base + (G * Fv) ** 2 * Mq + 1j * (G * Fv) * qB

    def L_apply(Fv, v):
        return base @ v + (G * Fv) ** 2 * (Mq @ v) + 1j * (G * Fv) * (qB @ v)

    cache = _LUCache(cache_size)
    u = asm.u0.astype(np.complex128)
    for n in range(s0 + 1, N + 1):
        rhs = Mk @ u - (1.0 - th) * L_apply(F[n - 1], u)
        Fn = float(F[n])
        if solver == "dense":
            A = (Mk + th * L(Fn)).toarray()
            u = np.linalg.solve(A, rhs)
        elif solver == "krylov":
            u = _krylov(Mk + th * L(Fn), rhs, u, hermitian=True)
        else:
            lu = cache.get(Fn, lambda: _splu(Mk + th * L(Fn)))
            u = lu.solve(rhs)
    s = complex(asm.w @ u)
    return (s, u) if return_u else s


def solve_uform(asm: Assembly, seq, b: float, q, n_steps: Optional[int] = None,
                cache_size: int = 8, return_u: bool = False, solver: str = "splu"):
    """Signal of one (b, q) system with the untransformed U-form (Neumann box)."""
    k = float(seq.dt)
    th = float(seq.theta)
    prof = seqmod.profile_of(seq)
    N_all = _n_steps(prof, k)
    # one-sided limits f(t^{n-1}+) (right side) and f(t^n-) (left side)
    lim = [prof.f_limits((n - 1) * k, n * k) for n in range(1, N_all + 1)]
    G = math.sqrt(b / prof.int_F2())
    qn = _unit(q)
    N = N_all if n_steps is None else int(n_steps)

    base = (asm.S + asm.IG + asm.R2).tocsr()
    Mk = (asm.M / k).tocsr()
    qJ = _qJ(asm, qn).tocsr()
    # weak pseudo-periodic faces (Appendix B, a* and L*): theta kappa_e face
    # mass on the left, the lagged partner with the phase of t^n on the right
    weak = asm.weak if asm.weak else ()
    if weak:
        if abs(th - 0.5) > 1e-12:
            raise ValueError("the weak pseudo-periodic scheme is the Crank-Nicolson one")
        Mk = (Mk + th * asm.KB).tocsr()
        Fg = [prof.F(v * k) for v in range(N_all + 1)]
    cache = _LUCache(cache_size)
    U = asm.u0.astype(np.complex128)
    for n in range(1, N + 1):
        f_prev, fn = lim[n - 1]
        rhs = (Mk @ U - (th * asm.KB @ U if weak else 0.0)
               - (1.0 - th) * (base @ U + 1j * (G * f_prev) * (qJ @ U)))
        for a, Cms, Csm, La in weak:
            ph = G * Fg[n] * qn[a] * La          # theta_ms = gamma g.(x_s - x_m) F(t^n)
            rhs = rhs + (1.0 - th) * (np.exp(1j * ph) * (Cms @ U) + np.exp(-1j * ph) * (Csm @ U))
        if solver == "dense":
            U = np.linalg.solve((Mk + th * (base + 1j * (G * fn) * qJ)).toarray(), rhs)
        elif solver == "krylov":
            U = _krylov(Mk + th * (base + 1j * (G * fn) * qJ), rhs, U, hermitian=False)
        else:
            lu = cache.get(fn, lambda: _splu(Mk + th * (base + 1j * (G * fn) * qJ)))
            U = lu.solve(rhs)
    s = complex(asm.w @ U)
    return (s, U) if return_u else s


def signals(prob, seq, b, q, form: str = "auto", asm: Optional[Assembly] = None, **kw):
    """Signals of every (b_s, q_s) pair on one problem, in input order.

    form: "transformed", "uform", or "auto" (U-form when the box has no
    periodic axis, transformed otherwise).
    """
    if asm is None:
        asm = assemble(prob)
    if form == "auto":
        pm = int(prob.periodic_mask)
        form = "uform" if (pm & 7) == 0 or (pm & 8) else "transformed"
    fn = solve_transformed if form == "transformed" else solve_uform
    b = np.atleast_1d(np.asarray(b, dtype=np.float64))
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    return np.array([fn(asm, seq, float(b[i]), q[i], **kw) for i in range(len(b))],
                    dtype=np.complex128)


def _simplex_rule(n):
    """Barycentric points [P, 4] and weights [P] (summing to 1/6) of a
    collapsed (Duffy) Gauss-Legendre rule with n points per direction on the
    unit tetrahedron."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    xi, eta, zeta = np.meshgrid(g, g, g, indexing="ij")
    wx, we, wz = np.meshgrid(w, w, w, indexing="ij")
    l1 = xi
    l2 = (1.0 - xi) * eta
    l3 = (1.0 - xi) * (1.0 - eta) * zeta
    l0 = 1.0 - l1 - l2 - l3
    lam = np.stack([l0, l1, l2, l3], axis=-1).reshape(-1, 4)
    wt = (wx * we * wz * (1.0 - xi) ** 2 * (1.0 - eta)).reshape(-1)
    return lam, wt


def physical_signal(prob, asm: Assembly, u, kvec, n_gauss: int = 8):
    """S = int U dx with U = u exp(-i k . (x - c)) (Sec. 2, eq. signal; the
    substitution of Appendix A with x from the box centre c): the P1 field
    u_h of the transformed form times the plane wave, integrated over every
    tetrahedron with a collapsed Gauss rule (n_gauss points per direction;
    for |k| h of order 1 the rule is exact to rounding). k = G F(t) q.
    With k = 0 this is sum_i w_i u_i."""
    xyz = np.asarray(prob.xyz, dtype=np.float64)
    tets = np.asarray(prob.tets, dtype=np.int64)
    c = 0.5 * (np.asarray(prob.box_lo, dtype=np.float64) + np.asarray(prob.box_hi, dtype=np.float64))
    X = xyz[tets] - c[None, None, :]                     # [m, 4, 3]
    vol6 = np.abs(np.linalg.det(X[:, 1:, :] - X[:, :1, :]))   # 6 |e|
    lam, wt = _simplex_rule(n_gauss)                     # [P, 4], [P]
    k = np.asarray(kvec, dtype=np.float64)
    uv = np.asarray(u)[asm.tet_dof]                      # [m, 4]
    total = 0.0 + 0.0j
    for s0 in range(0, X.shape[0], 4096):                # bounded memory
        Xs = X[s0:s0 + 4096]
        xq = np.einsum("pl,mla->mpa", lam, Xs)           # [m, P, 3]
        wave = np.exp(-1j * (xq @ k))                    # [m, P]
        uq = uv[s0:s0 + 4096] @ lam.T                    # [m, P]
        total += np.sum(vol6[s0:s0 + 4096, None] * wt[None, :] * uq * wave)
    return complex(total)
