"""Pins of the oracle's polynomial preconditioner, flexible CG and Ritz
extraction (oracle/precond.py), all on the CPU.

* the Chebyshev preconditioner's residual polynomial, measured in the
  eigenbasis of D^-1/2 A D^-1/2, equals the closed form
  T_m((b + a - 2 lam)/(b - a)) / T_m((b + a)/(b - a)) (a wrong recurrence
  coefficient, sign or starting term changes it);
* FCG with one Chebyshev term (scaled Jacobi) takes the iterations of SciPy's
  Jacobi-preconditioned CG and reaches its solution; FCG with several terms
  reaches the direct solution of a theta-step system;
* Ritz values of a PCG run that explores the whole space equal the
  eigenvalues of D^-1 A; a short run's lie inside the spectrum
  (interlacing);
* the step operator is Hermitian and one solve with it reproduces the
  oracle's first time step;
* features and the network-output-to-interval map on simple cases.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import dmri_inputs as di
from oracle import fem, precond, timestep

SEQ = di.Sequence(delta=10600.0, Delta=13400.0, dt=200.0)


def _hpd(n, seed, spread=30.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, spread, n)
    A = (Q * lam) @ Q.conj().T
    d = rng.uniform(0.5, 4.0, n)  # uneven diagonal scaling
    A = (np.sqrt(d)[:, None] * A) * np.sqrt(d)[None, :]
    return 0.5 * (A + A.conj().T)


@pytest.fixture(scope="module")
def step_system():
    prob = di.cylinder_box(n=8, half=6.0, r=4.0, D_in=1.5e-3, kappa=1e-4)
    asm = fem.assemble(prob)
    A, R = precond.step_operator(asm, SEQ, 3000.0, [0.3, 0.5, 0.8], 12)
    rng = np.random.default_rng(3)
    u = asm.u0 * np.exp(1j * rng.uniform(0, 0.3, asm.u0.shape))
    return prob, asm, A, R @ u


@pytest.mark.parametrize("m", [1, 2, 5])
def test_chebyshev_polynomial_closed_form(m):
    A = _hpd(12, seed=m)
    d = np.real(np.diag(A))
    s = 1.0 / np.sqrt(d)
    B = (s[:, None] * A) * s[None, :]
    lam, V = np.linalg.eigh(B)
    a, b = 0.5 * lam[0], 1.2 * lam[-1]
    rng = np.random.default_rng(10 + m)
    r = rng.standard_normal(12) + 1j * rng.standard_normal(12)
    z = precond.chebyshev_apply(A, 1.0 / d, r, a, b, m)
    # D^-1/2 (r - A z) = (I - B p(B)) D^-1/2 r, coordinate by coordinate in V
    c_in = V.conj().T @ (s * r)
    c_out = V.conj().T @ (s * (r - A @ z))
    want = precond.chebyshev_residual_poly(lam, a, b, m)
    np.testing.assert_allclose(c_out, want * c_in, rtol=1e-9, atol=1e-12 * np.abs(c_in).max())
    # the polynomial is positive on the spectrum: z is a descent direction
    assert np.vdot(r, z).real > 0


def test_fcg_one_term_is_jacobi_cg(step_system):
    _, _, A, rhs = step_system
    x0 = np.zeros_like(rhs)
    dinv = 1.0 / A.diagonal().real
    x, it = precond.fcg(A, rhs, x0, 1e-10,
                        lambda r: precond.chebyshev_apply(A, dinv, r, 0.2, 1.8, 1))
    count = [0]

    def cb(_):
        count[0] += 1

    M = spla.LinearOperator(A.shape, matvec=lambda v: dinv * v, dtype=np.complex128)
    xs, info = spla.cg(A, rhs, x0=x0, rtol=1e-10, atol=0.0, M=M, callback=cb, maxiter=5000)
    assert info == 0
    assert abs(it - count[0]) <= 1, (it, count[0])
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


@pytest.mark.parametrize("m,interval", [(3, (0.1, 2.5)), (6, (0.3, 2.0)), (4, (0.05, 1.2))])
def test_fcg_reaches_direct_solution(step_system, m, interval):
    # the last interval cuts the top of the spectrum: the preconditioner is
    # then not positive there, and FCG must still converge
    _, _, A, rhs = step_system
    dinv = 1.0 / A.diagonal().real
    x, it = precond.fcg(A, rhs, np.zeros_like(rhs), 1e-12,
                        lambda r: precond.chebyshev_apply(A, dinv, r, *interval, m))
    xd = spla.spsolve(A.tocsc(), rhs)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert it > 0


def test_chebyshev_cuts_iterations(step_system):
    _, _, A, rhs = step_system
    lam = precond.jacobi_spectrum(A)
    dinv = 1.0 / A.diagonal().real
    x0 = np.zeros_like(rhs)
    _, it1 = precond.fcg(A, rhs, x0, 1e-10,
                         lambda r: precond.chebyshev_apply(A, dinv, r, lam[0], lam[-1], 1))
    _, it4 = precond.fcg(A, rhs, x0, 1e-10,
                         lambda r: precond.chebyshev_apply(A, dinv, r, lam[0], lam[-1], 4))
    assert it4 < it1 / 2, (it1, it4)


def test_ritz_full_run_equals_spectrum():
    A = sp.csr_matrix(_hpd(8, seed=21, spread=6.0))
    rng = np.random.default_rng(5)
    rhs = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    x, al, be = precond.pcg_coefficients(A, rhs, np.zeros(8), 1e-15)
    assert len(al) == 8
    lo, hi = precond.ritz_extremes(al, be)
    lam = precond.jacobi_spectrum(A)
    assert abs(lo - lam[0]) <= 1e-8 * lam[-1]
    assert abs(hi - lam[-1]) <= 1e-8 * lam[-1]
    T = precond.lanczos_tridiagonal(al, be)
    np.testing.assert_allclose(np.linalg.eigvalsh(T), lam, rtol=1e-8)


def test_ritz_short_run_interlaces(step_system):
    _, _, A, rhs = step_system
    lam = precond.jacobi_spectrum(A)
    _, al, be = precond.pcg_coefficients(A, rhs, np.zeros_like(rhs), 1e-2)
    assert 2 <= len(al) < 40
    lo, hi = precond.ritz_extremes(al, be)
    assert lam[0] * (1 - 1e-12) <= lo <= hi <= lam[-1] * (1 + 1e-12)
    # coefficients of a Hermitian positive definite run are real
    assert max(abs(np.imag(v)) for v in al) <= 1e-10 * max(abs(v) for v in al)


def test_step_operator_matches_time_step():
    prob = di.free_box(n=5, half=2.5)
    asm = fem.assemble(prob)
    q = [0.2, -0.4, 0.9]
    A, R = precond.step_operator(asm, SEQ, 2000.0, q, 1)
    assert abs(A - A.conj().T).max() <= 1e-12 * abs(A).max()
    u1 = spla.spsolve(A.tocsc(), R @ asm.u0.astype(np.complex128))
    s, u = timestep.solve_transformed(asm, SEQ, 2000.0, q, n_steps=1, return_u=True)
    np.testing.assert_allclose(u1, u, rtol=1e-12, atol=1e-14)


def test_features_and_interval_map():
    x = precond.features(100.0, 0.5, 3e-3, 1.0, 0.0, 0.0, 0.0, [0.0, 0.0, 2.0])
    assert x[0] == pytest.approx(math.log(0.5 * 100.0 * 3e-3))
    assert x[1] == 0.0 and x[2] == 0.0 and x[3] == 0.0
    np.testing.assert_array_equal(x[4:7], [0.0, 0.0, 1.0])
    assert not x[7:].any()
    gG, F = 2e-4, 5000.0
    x = precond.features(100.0, 0.5, 3e-3, 0.5, 1e-3, gG, F, [1.0, 1.0, 0.0])
    assert x[1] == pytest.approx(math.log1p(0.5 * 100 * 3e-3 * (gG * F) ** 2))
    assert x[2] == pytest.approx(math.log1p(0.5 * 100 * 3e-3 * gG * F / 0.5))
    assert x[3] == pytest.approx(math.log1p(0.5 * 100 * 1e-3 / 0.5))
    ar, br = precond.A_REF, precond.B_REF
    assert precond.interval_from_output(math.log(0.2), math.log(2.0)) == \
        pytest.approx((0.2 * ar, 2.0 * br))
    assert precond.interval_from_output(0.0, 0.0) == (ar, br)
    assert precond.interval_from_output(float("nan"), 1.0) == (ar, br)
    assert precond.interval_from_output(1.0, -1.0) == (ar, br)
    assert precond.interval_from_output(-1e9, 1e9) == pytest.approx(
        (ar * math.exp(-20.0), br * math.exp(20.0)))
    t0, t1 = precond.targets_from_ritz(0.7, 1.3)
    assert precond.interval_from_output(t0, t1) == pytest.approx((0.7, 1.3 * precond.MARGIN))
