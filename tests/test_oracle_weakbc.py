"""Pins of the oracle's weak pseudo-periodic faces (Appendix B, artificial
permeability; oracle/weakbc.py), all on the CPU.

* the partner couplings integrate products of linear fields exactly over
  matching and non-matching faces (closed-form rectangle moments), and the
  face mass does the same on both faces;
* C_sm is the transpose of C_ms, and each face is tiled completely (row
  sums of the couplings equal row sums of the face mass);
* kappa_e = max{D / h} on a Kuhn box (D / (sqrt(3) h)) and with a tensor
  (largest eigenvalue);
* with g = 0 a constant field stays constant to rounding (the flux
  kappa_e (U_partner - U) vanishes), and a theta other than 1/2 is refused;
* on a thin slab the weak U-form tends to the exact free-diffusion signal
  exp(-b D) as kappa_e grows and dt shrinks, and the paper's kappa_e at a
  coarse step sits between that and the walled (Neumann) signal.
"""

import dataclasses
import math

import numpy as np
import pytest

import dmri_inputs as di
from oracle import fem, timestep, weakbc

SEQ = di.Sequence(delta=10600.0, Delta=13400.0, dt=100.0)


def _rect_int(lo, hi, u, v):
    """int over [lo0, hi0] x [lo1, hi1] of (u0 + u1 s + u2 t)(v0 + v1 s + v2 t)."""
    (a0, b0), (a1, b1) = (lo[0], hi[0]), (lo[1], hi[1])
    L0, L1 = b0 - a0, b1 - a1
    m1 = L0 * L1
    ms = (b0 ** 2 - a0 ** 2) / 2 * L1
    mt = L0 * (b1 ** 2 - a1 ** 2) / 2
    mss = (b0 ** 3 - a0 ** 3) / 3 * L1
    mtt = L0 * (b1 ** 3 - a1 ** 3) / 3
    mst = (b0 ** 2 - a0 ** 2) / 2 * (b1 ** 2 - a1 ** 2) / 2
    return (u[0] * v[0] * m1 + (u[0] * v[1] + u[1] * v[0]) * ms + (u[0] * v[2] + u[2] * v[0]) * mt
            + u[1] * v[1] * mss + u[2] * v[2] * mtt + (u[1] * v[2] + u[2] * v[1]) * mst)


def _dof_xyz(prob, asm):
    # coordinates of each DOF's node (dof_node numbers the mesh's distinct
    # node positions; weak faces are not identified)
    tn, nt = fem.torus_nodes(prob.xyz, prob.box_lo, prob.box_hi, prob.periodic_mask)
    c = np.zeros((nt, 3))
    c[tn] = prob.xyz
    return c[asm.dof_node]


CASES = {
    "matching": lambda: di.free_box(n=4, half=2.0, periodic_mask=15),
    "nonmatching": lambda: di.nonmatching_faces(di.free_box(n=5, half=2.5, periodic_mask=15),
                                                amount=0.3, seed=4),
    "nonmatching_cylinder": lambda: di.nonmatching_faces(
        di.conforming_cylinder_box(n=6, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3,
                                   periodic_mask=13, seed=1), axes=(0, 2), amount=0.25, seed=7),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_couplings_integrate_linear_products(name):
    prob = CASES[name]()
    asm = fem.assemble(prob)
    x = _dof_xyz(prob, asm)
    lo, hi = np.asarray(prob.box_lo), np.asarray(prob.box_hi)
    rng = np.random.default_rng(3)
    ke = asm.kappa_e
    assert asm.weak
    for a, Cms, Csm, L in asm.weak:
        b, c = [k for k in range(3) if k != a]
        assert L == pytest.approx(hi[a] - lo[a])
        for _ in range(3):
            u, v = rng.normal(size=3), rng.normal(size=3)
            uf = u[0] + u[1] * x[:, b] + u[2] * x[:, c]
            vf = v[0] + v[1] * x[:, b] + v[2] * x[:, c]
            # restricted per compartment: a DOF only meets its own tet's faces,
            # and every compartment's faces tile its share of the box face
            want = ke * _rect_int((lo[b], lo[c]), (hi[b], hi[c]), u, v)
            assert uf @ (Cms @ vf) == pytest.approx(want, rel=1e-11)
            assert vf @ (Csm @ uf) == pytest.approx(want, rel=1e-11)
        assert abs(Csm - Cms.T).max() <= 1e-15 * abs(Cms).max()
        assert Cms.sum() == pytest.approx(ke * (hi[b] - lo[b]) * (hi[c] - lo[c]), rel=1e-12)


@pytest.mark.parametrize("name", sorted(CASES))
def test_face_mass_and_tiling(name):
    prob = CASES[name]()
    asm = fem.assemble(prob)
    x = _dof_xyz(prob, asm)
    lo, hi = np.asarray(prob.box_lo), np.asarray(prob.box_hi)
    ke = asm.kappa_e
    n = asm.n_dof
    dof = asm.tet_dof
    total = 0.0
    for a, Cms, Csm, L in asm.weak:
        _, _, Kf = weakbc.coupling(prob, dof, a, ke, L)
        # both faces tiled: coupling row sums equal face-mass row sums
        rs = np.asarray(Kf.sum(axis=1)).ravel()
        cs = np.asarray((Cms + Csm).sum(axis=1)).ravel()
        assert np.abs(rs - cs).max() <= 1e-13 * rs.max()
        # the face mass integrates products of 3-D linear fields on both faces
        b, c = [k for k in range(3) if k != a]
        u = np.array([0.3, -0.7, 0.2, 0.5])  # 1, x, y, z
        v = np.array([1.1, 0.4, -0.6, 0.9])
        f = lambda w: w[0] + w[1] * x[:, 0] + w[2] * x[:, 1] + w[3] * x[:, 2]  # noqa: E731
        want = 0.0
        for plane in (lo[a], hi[a]):
            uu = [u[0] + u[1 + a] * plane, u[1 + b], u[1 + c]]
            vv = [v[0] + v[1 + a] * plane, v[1 + b], v[1 + c]]
            want += _rect_int((lo[b], lo[c]), (hi[b], hi[c]), uu, vv)
        assert f(u) @ (Kf @ f(v)) == pytest.approx(ke * want, rel=1e-11)
        total += Kf
    assert abs(asm.KB - total).max() <= 1e-15 * abs(total).max()
    assert asm.KB.shape == (n, n)


def test_kappa_e_is_max_D_over_h():
    prob = di.free_box(n=4, half=2.0, periodic_mask=9)        # h = 1, longest edge sqrt(3)
    asm = fem.assemble(prob)
    assert asm.kappa_e == pytest.approx(di.D_FREE / math.sqrt(3.0), rel=1e-14)
    D = di.tensor([3e-3, 1e-3, 2e-3], (0.4, 0.9, -0.3))
    pt = dataclasses.replace(prob, D=D[None])
    assert fem.assemble(pt).kappa_e == pytest.approx(3e-3 / math.sqrt(3.0), rel=1e-12)
    # scaling only multiplies the arrays
    a2 = fem.assemble(prob, weak_kappa=4.0)
    assert a2.kappa_e == asm.kappa_e
    assert abs(a2.KB - 4.0 * asm.KB).max() <= 1e-15 * abs(asm.KB).max() * 4


def test_constant_field_stays_constant():
    prob = CASES["nonmatching_cylinder"]()
    asm = fem.assemble(prob, weak_kappa=5.0)
    seq = di.Sequence(2000.0, 4000.0, 200.0)
    s, u = timestep.solve_uform(asm, seq, 0.0, [1.0, 0.0, 0.0], return_u=True)
    assert np.abs(u - 1.0).max() < 1e-12
    assert s.real == pytest.approx(np.prod(np.asarray(prob.box_hi) - prob.box_lo), rel=1e-12)
    with pytest.raises(ValueError, match="Crank-Nicolson"):
        timestep.solve_uform(asm, di.Sequence(2000.0, 4000.0, 200.0, theta=0.75), 0.0,
                             [1.0, 0.0, 0.0])


def test_weak_slab_tends_to_free_diffusion():
    # A thin slab along x (24 cells, one cell across), weak faces on x only,
    # walls on y and z; free diffusion with b = 1000 along x.
    prob = di.slab_box(n=24, half=5.0, split=10.0, cross=(0.5, 1), periodic_mask=9)
    vol = 10.0 * 0.25
    exact = math.exp(-1000.0 * di.D_FREE)
    neumann = abs(timestep.signals(dataclasses.replace(prob, periodic_mask=0), SEQ, 1000.0,
                                   [1.0, 0.0, 0.0])[0]) / vol

    def weak(scale, dt):
        asm = fem.assemble(prob, weak_kappa=scale)
        seq = di.Sequence(SEQ.delta, SEQ.Delta, dt)
        return abs(timestep.solve_uform(asm, seq, 1000.0, [1.0, 0.0, 0.0])) / vol

    coarse = weak(1.0, 20.0)
    fine = weak(16.0, 0.5)
    assert exact < coarse < neumann
    assert abs(fine - exact) < 0.05 * exact
    assert abs(fine - exact) < 0.25 * abs(coarse - exact)
