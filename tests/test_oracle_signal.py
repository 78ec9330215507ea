"""Pins of the oracle's time stepping and signal against closed forms.

Each test ties the FP64 oracle to something other than itself:

* free diffusion on a torus: a constant field stays constant, so the
  theta-scheme collapses to a scalar recurrence written out here; its limit
  is the Stejskal-Tanner attenuation exp(-D b) with O(dt^2) error
  (Sec. 2 eq. b_value; Appendix A eq. theta_discretization);
* mass conservation at b = 0 with permeable membranes (Sec. 2 eq. btpde_ic:
  the flux is continuous, so no magnetization is lost);
* kappa -> 0 decouples compartments (equals a run on the sub-mesh alone) and
  kappa -> infinity merges them (equals the single-compartment run);
* a gradient parallel to voxel-staircase prisms keeps each compartment
  constant: per-compartment scalar recurrences;
* a 1-D slab against the matrix formalism (the paper's reference method,
  Sec. 4), for both the transformed (Appendix A) and the U-form
  (Appendix B) discretizations, at second order in (h, dt);
* the two forms agree on a non-symmetric case with a complex signal, which
  fixes the sign of the first-order term;
* S(-q) = conj S(q); dense, SuperLU and Krylov solves agree.
"""

import math

import numpy as np
import pytest

import dmri_inputs as di
from oracle import fem, mf1d, sequence as sq, timestep

PGSE = di.Sequence(10600.0, 13400.0, 100.0, 0.5)


def recurrence(D, b, seq, T2=None, G=None):
    """c^n = c^{n-1} (1/k - (1-th) a^{n-1}) / (1/k + th a^n), a = D (G F)^2 + 1/T2."""
    T = seq.Delta + seq.delta
    N = int(round(T / seq.dt))
    if G is None:
        G = math.sqrt(b / (seq.delta ** 2 * (seq.Delta - seq.delta / 3.0)))

    def F(t):
        return min(max(t, 0.0), seq.delta) - min(max(t - seq.Delta, 0.0), seq.delta)

    r2 = 0.0 if T2 is None else 1.0 / T2
    c = 1.0
    for n in range(1, N + 1):
        a0 = D * (G * F((n - 1) * seq.dt)) ** 2 + r2
        a1 = D * (G * F(n * seq.dt)) ** 2 + r2
        c *= (1.0 / seq.dt - (1.0 - seq.theta) * a0) / (1.0 / seq.dt + seq.theta * a1)
    return c


def test_free_diffusion_box_closed_form():
    prob, seq, sysl = di.free_diffusion_10()
    s = timestep.signals(prob, seq, sysl.b, sysl.q)[0]
    vol = 1000.0
    c = recurrence(3e-3, 1000.0, seq)
    assert s.real / vol == pytest.approx(c, rel=1e-12)
    assert abs(s.imag) < 1e-12 * vol
    # The value quoted for this workload (discrete CN, dt = 100 us).
    assert s.real / vol == pytest.approx(0.049775509970, abs=5e-13)


def test_stejskal_tanner_second_order():
    prob = di.free_box(n=4, half=5.0)
    asm = fem.assemble(prob)
    D, b = 3e-3, 1000.0
    st = math.exp(-D * b)
    errs = []
    for dt in (100.0, 50.0, 25.0):
        seq = di.Sequence(10600.0, 13400.0, dt, 0.5)
        s = timestep.signals(prob, seq, [b], [[1, 0, 0]], asm=asm, solver="krylov")[0]
        errs.append(s.real / 1000.0 / st - 1.0)
    assert errs[0] == pytest.approx(-2.32e-4, rel=5e-3)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.9 < r1 < 4.1 and 3.9 < r2 < 4.1


def test_free_diffusion_oblique_with_T2():
    prob = di.free_box(n=5, half=5.0)
    prob.T2 = np.array([4.0e4])
    q = np.array([0.3, -0.5, 0.7])
    s = timestep.signals(prob, PGSE, [2500.0], [q], solver="krylov")[0]
    assert s.real / 1000.0 == pytest.approx(recurrence(3e-3, 2500.0, PGSE, T2=4.0e4), rel=1e-11)


def test_mass_conservation_b0_permeable():
    prob = di.cylinder_box(n=10, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3, D_out=3e-3,
                           u0=(0.3, 1.7))
    asm = fem.assemble(prob)
    s = timestep.signals(prob, PGSE, [0.0], [[1, 0, 0]], asm=asm, solver="krylov")[0]
    expect = 0.3 * asm.comp_volume[0] + 1.7 * asm.comp_volume[1]
    assert s.real == pytest.approx(expect, rel=1e-11)
    assert abs(s.imag) < 1e-11 * expect


def _submesh(prob, label):
    keep = prob.tet_label == label
    return di.Problem(prob.xyz, prob.tets[keep], np.zeros(keep.sum(), np.int32), 1,
                      np.array([prob.D[label]]), None, None, 0.0, prob.box_lo, prob.box_hi,
                      prob.periodic_mask)


def test_kappa_zero_decouples():
    prob = di.cylinder_box(n=10, half=6.0, r=4.0, kappa=0.0, D_in=1e-3, D_out=3e-3,
                           u0=(0.0, 1.0))
    q = np.array([1.0, 0.4, 0.2])
    s2 = timestep.signals(prob, PGSE, [2000.0], [q], solver="krylov")[0]
    s1 = timestep.signals(_submesh(prob, 1), PGSE, [2000.0], [q], solver="krylov")[0]
    assert s2 == pytest.approx(s1, rel=1e-11, abs=1e-11)


def test_kappa_infinity_merges():
    base = di.cylinder_box(n=8, half=6.0, r=4.0, kappa=0.0)
    single = di.Problem(base.xyz, base.tets, np.zeros(base.n_tets, np.int32), 1,
                        np.array([3e-3]), None, None, 0.0, base.box_lo, base.box_hi, 7)
    q = [[1.0, 0.0, 0.0]]
    ref = timestep.signals(single, PGSE, [3000.0], q, solver="krylov")[0]
    errs = []
    for kappa in (0.1, 1.0, 10.0):
        p = di.cylinder_box(n=8, half=6.0, r=4.0, kappa=kappa)
        s = timestep.signals(p, PGSE, [3000.0], q, solver="krylov")[0]
        errs.append(abs(s - ref) / abs(ref))
    # O(1/kappa): each decade of kappa removes about a decade of error.
    assert errs[0] > 5 * errs[1] > 25 * errs[2]
    assert errs[2] < 3e-4


def test_axial_gradient_staircase_prisms():
    # Voxel labels make every membrane face vertical: with q along z and no
    # exchange each compartment keeps a constant field.
    D_in, D_out = 1e-3, 3e-3
    prob = di.cylinder_box(n=9, half=6.0, r=4.0, kappa=0.0, D_in=D_in, D_out=D_out,
                           mode="cube")
    asm = fem.assemble(prob)
    b = 2000.0
    s = timestep.signals(prob, PGSE, [b], [[0, 0, 1]], asm=asm, solver="krylov")[0]
    expect = (asm.comp_volume[0] * recurrence(D_out, b, PGSE)
              + asm.comp_volume[1] * recurrence(D_in, b, PGSE))
    assert s.real == pytest.approx(expect, rel=1e-11)
    # Equal diffusivities: one recurrence even with exchange.
    prob2 = di.cylinder_box(n=9, half=6.0, r=4.0, kappa=0.05, mode="cube")
    s2 = timestep.signals(prob2, PGSE, [b], [[0, 0, 1]], solver="krylov")[0]
    assert s2.real == pytest.approx(1728.0 * recurrence(3e-3, b, PGSE), rel=1e-11)


@pytest.mark.parametrize("form,mask", [("uform", 0), ("transformed", 0), ("transformed", 6)])
def test_slab_matches_matrix_formalism(form, mask):
    L, D, b = 10.0, 3e-3, 3000.0
    G = float(sq.b_to_G(b, PGSE.delta, PGSE.Delta))
    ref = mf1d.slab_signal(L, D, G, PGSE.delta, PGSE.Delta, n_modes=96)
    # The truncated expansion has converged.
    assert abs(ref - mf1d.slab_signal(L, D, G, PGSE.delta, PGSE.Delta, n_modes=48)) < 1e-8
    errs = []
    for n, dt in ((10, 200.0), (20, 100.0), (40, 50.0)):
        seq = di.Sequence(PGSE.delta, PGSE.Delta, dt, 0.5)
        p = di.slab_box(n=n, half=L / 2, split=99.0, cross=(1.0, 1), periodic_mask=mask)
        s = timestep.signals(p, seq, [b], [[1, 0, 0]], form=form, solver="krylov")[0]
        errs.append(abs(s - ref) / abs(ref))
    assert errs[2] < 5e-3
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_forms_agree_on_complex_signal():
    # Asymmetric two-compartment slab with exchange and unequal initial
    # values: the signal has a large imaginary part, whose sign depends on
    # the sign convention of the first-order term.
    prev = None
    vals = []
    for n, dt in ((10, 200.0), (20, 100.0), (40, 50.0)):
        seq = di.Sequence(PGSE.delta, PGSE.Delta, dt, 0.5)
        p = di.slab_box(n=n, half=5.0, split=-1.0, D=(3e-3, 1e-3), kappa=1e-3, u0=(1.0, 0.2),
                        cross=(1.0, 1), periodic_mask=0)
        asm = fem.assemble(p)
        su = timestep.signals(p, seq, [3000.0], [[1, 0, 0]], form="uform", asm=asm,
                              solver="krylov")[0]
        st = timestep.signals(p, seq, [3000.0], [[1, 0, 0]], form="transformed", asm=asm,
                              solver="krylov")[0]
        vals.append((su, st))
        d = abs(su - st)
        if prev is not None:
            assert prev / d > 3.5
        prev = d
    su, st = vals[-1]
    assert su.imag > 0.5 and st.imag > 0.5
    assert abs(su - st) / abs(su) < 1e-2


def test_conjugate_symmetry():
    p = di.slab_box(n=12, half=5.0, split=-1.0, D=(3e-3, 1e-3), kappa=1e-3, u0=(1.0, 0.2),
                    cross=(1.0, 1), periodic_mask=0b110)
    asm = fem.assemble(p)
    q = np.array([0.8, 0.36, 0.48])
    sp_, sm = timestep.signals(p, PGSE, [1500.0, 1500.0], [q, -q], form="transformed",
                               asm=asm, solver="krylov")
    assert abs(sp_.imag) > 0.1
    assert abs(sp_ - np.conj(sm)) < 1e-11 * abs(sp_)


def test_dense_splu_krylov_agree():
    prob = di.cylinder_box(n=4, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3)
    asm = fem.assemble(prob)
    seq = di.Sequence(2000.0, 3000.0, 250.0, 0.5)
    q = [[0.6, 0.0, 0.8]]
    vals = [timestep.signals(prob, seq, [4000.0], q, asm=asm, solver=s)[0]
            for s in ("dense", "splu", "krylov")]
    assert abs(vals[0] - vals[1]) < 1e-12 * abs(vals[0])
    assert abs(vals[0] - vals[2]) < 1e-11 * abs(vals[0])
    p0 = di.slab_box(n=6, half=3.0, split=0.5, D=(3e-3, 2e-3), kappa=1e-3, periodic_mask=0)
    a0 = fem.assemble(p0)
    vu = [timestep.signals(p0, seq, [4000.0], [[1, 0, 0]], asm=a0, form="uform", solver=s)[0]
          for s in ("dense", "splu", "krylov")]
    assert abs(vu[0] - vu[1]) < 1e-12 * abs(vu[0])
    assert abs(vu[0] - vu[2]) < 1e-11 * abs(vu[0])


# ------------------------------------------------- general temporal profiles
# Free diffusion on the torus for every profile: the FE signal equals the
# scalar theta recurrence with the profile's F at the grid points, and tends
# to exp(-D b) (b = G^2 int F^2) at second order in dt. For the U-form (walls)
# the one-sided limits of f are pinned by the two forms converging to each
# other at second order on the asymmetric exchange slab.

PROFILES = [
    ("double_pgse", (2000.0, 4000.0, 1000.0)),
    ("cos_ogse", (4000.0, 6000.0, 2.0)),
    ("sin_ogse", (4000.0, 6000.0, 1.0)),
    ("trap_pgse", (4000.0, 6000.0, 1000.0)),
    ("double_trap_pgse", (2000.0, 4000.0, 500.0, 500.0)),
]


def _profile_recurrence(D, b, prof, dt, theta=0.5):
    N = int(round(prof.T / dt))
    F = [prof.F(n * dt) for n in range(N + 1)]
    G2 = b / prof.int_F2()
    c = 1.0
    for n in range(1, N + 1):
        a0, a1 = D * G2 * F[n - 1] ** 2, D * G2 * F[n] ** 2
        c *= (1.0 / dt - (1.0 - theta) * a0) / (1.0 / dt + theta * a1)
    return c


@pytest.mark.parametrize("kind,params", PROFILES)
def test_free_diffusion_general_profile(kind, params):
    prob = di.free_box(n=4, half=5.0)
    asm = fem.assemble(prob)
    prof = sq.Profile(kind, params)
    D, b = 3e-3, 1500.0
    errs = []
    for dt in (100.0, 50.0, 25.0):
        seq = di.GeneralSequence(kind, params, dt, 0.5)
        s = timestep.signals(prob, seq, [b], [[0.6, 0.0, 0.8]], asm=asm, solver="splu")[0]
        c = _profile_recurrence(D, b, prof, dt)
        assert s.real / 1000.0 == pytest.approx(c, rel=1e-11)
        assert abs(s.imag) < 1e-11 * 1000.0
        errs.append(c / math.exp(-D * b) - 1.0)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.8 < r1 < 4.2 and 3.8 < r2 < 4.2, (errs, r1, r2)


@pytest.mark.parametrize("kind,params", [("cos_ogse", (4000.0, 6000.0, 1.0)),
                                         ("trap_pgse", (4000.0, 6000.0, 1000.0))])
def test_forms_agree_general_profile(kind, params):
    prev = None
    for n, dt in ((10, 200.0), (20, 100.0), (40, 50.0)):
        seq = di.GeneralSequence(kind, params, dt, 0.5)
        p = di.slab_box(n=n, half=5.0, split=-1.0, D=(3e-3, 1e-3), kappa=1e-3, u0=(1.0, 0.2),
                        cross=(1.0, 1), periodic_mask=0)
        asm = fem.assemble(p)
        su = timestep.signals(p, seq, [3000.0], [[1, 0, 0]], form="uform", asm=asm,
                              solver="splu")[0]
        st = timestep.signals(p, seq, [3000.0], [[1, 0, 0]], form="transformed", asm=asm,
                              solver="splu")[0]
        d = abs(su - st)
        if prev is not None:
            assert prev / d > 3.5, (prev, d)
        prev = d
    # (the OGSE signal is small here, 0.23 of the slab's 1.8, so the
    # relative gap at n = 40 is larger than for PGSE)
    assert abs(su - st) / abs(su) < 5e-2


# --------------------------------------- physical signal when F(t) != 0
# S(t) = int u_h exp(-i k.(x - c)) (Sec. 2, eq. signal; Appendix A's
# substitution). Pinned against exact box integrals of the plane wave times a
# constant and times a linear field (both represented exactly by P1), against
# sum w u at k = 0, and by the two forms converging to each other when the
# run stops mid-sequence (F != 0, the U-form needs no phase).

def _box_wave(L, k):
    # int_{-L/2}^{L/2} exp(-i k x) dx and int x exp(-i k x) dx (= i d/dk of it)
    if k == 0.0:
        return L, 0.0
    I = 2.0 * math.sin(0.5 * k * L) / k
    dI = L * math.cos(0.5 * k * L) / k - 2.0 * math.sin(0.5 * k * L) / k ** 2
    return I, 1j * dI


@pytest.mark.parametrize("k", [(0.0, 0.0, 0.0), (0.3, -0.2, 0.5), (1.1, 0.4, -0.7)])
def test_physical_signal_box_integrals(k):
    p = di.free_box(n=5, half=2.5, periodic_mask=0)
    p.xyz = p.xyz + np.array([0.7, -0.3, 0.2])           # box not centred at 0
    p.box_lo = p.box_lo + np.array([0.7, -0.3, 0.2])
    p.box_hi = p.box_hi + np.array([0.7, -0.3, 0.2])
    asm = fem.assemble(p)
    c = 0.5 * (p.box_lo + p.box_hi)
    L = 5.0
    Ix, Jx = _box_wave(L, k[0])
    Iy, Jy = _box_wave(L, k[1])
    Iz, Jz = _box_wave(L, k[2])
    ones = np.ones(asm.n_dof)
    s1 = timestep.physical_signal(p, asm, ones, k)
    assert abs(s1 - Ix * Iy * Iz) < 1e-12 * L ** 3
    tn, nt = fem.torus_nodes(p.xyz, p.box_lo, p.box_hi, p.periodic_mask)
    node_xyz = np.zeros((nt, 3))
    node_xyz[tn] = p.xyz                                  # dof_node numbers these
    ynode = node_xyz[asm.dof_node, 1] - c[1]              # linear field y - c_y
    s2 = timestep.physical_signal(p, asm, ynode, k)
    assert abs(s2 - Ix * Jy * Iz) < 1e-12 * L ** 4
    xnode = node_xyz[asm.dof_node, 0] - c[0]              # and x - c_x
    s3 = timestep.physical_signal(p, asm, xnode, k)
    assert abs(s3 - Jx * Iy * Iz) < 1e-12 * L ** 4
    if k == (0.0, 0.0, 0.0):
        u = np.random.default_rng(1).normal(size=asm.n_dof)
        assert timestep.physical_signal(p, asm, u, k) == pytest.approx(asm.w @ u, rel=1e-13)


def test_physical_signal_forms_agree_mid_sequence():
    # Stop at step n where F != 0: the U-form signal sum w U^n and the
    # transformed form's physical signal converge to each other at second
    # order (fixes the sign and the origin of the phase).
    prev = None
    for n, dt in ((10, 200.0), (20, 100.0), (40, 50.0)):
        seq = di.Sequence(2000.0, 4000.0, dt, 0.5)
        stop = int(round(3000.0 / dt))                   # t = 3 ms: F = delta
        p = di.slab_box(n=n, half=5.0, split=-1.0, D=(3e-3, 1e-3), kappa=1e-3, u0=(1.0, 0.2),
                        cross=(1.0, 1), periodic_mask=0)
        asm = fem.assemble(p)
        G = float(sq.b_to_G(3000.0, seq.delta, seq.Delta))
        su = timestep.solve_uform(asm, seq, 3000.0, [1, 0, 0], n_steps=stop, solver="splu")
        _, u = timestep.solve_transformed(asm, seq, 3000.0, [1, 0, 0], n_steps=stop,
                                          solver="splu", return_u=True)
        F = float(sq.pgse_F(stop * dt, seq.delta, seq.Delta))
        st = timestep.physical_signal(p, asm, u, G * F * np.array([1.0, 0.0, 0.0]))
        naive = asm.w @ u
        d = abs(su - st)
        if prev is not None:
            assert prev / d > 3.5, (prev, d)
        prev = d
    assert abs(su - st) / abs(su) < 2e-2
    assert abs(naive - su) / abs(su) > 0.1                 # the phase matters here


def test_free_diffusion_tensor_closed_form():
    # one compartment with a tensor on the torus: u stays uniform, so the
    # scalar recurrence holds with a = (q.D q) (G F)^2, and the signal tends
    # to exp(-b q.D q) at second order
    Dt = di.tensor([3e-3, 1e-3, 2e-3], (0.4, 0.9, -0.3))
    q = np.array([0.6, 0.0, 0.8])
    b = 1200.0
    errs = []
    for dt in (100.0, 50.0, 25.0):
        prob = di.free_box(n=4, half=5.0)
        prob.D = Dt[None]
        seq = di.Sequence(10600.0, 13400.0, dt, 0.5)
        asm = fem.assemble(prob)
        s = timestep.signals(prob, seq, [b], [q], asm=asm, solver="splu")[0]
        c = recurrence(float(q @ Dt @ q), b, seq)
        assert s.real / 1000.0 == pytest.approx(c, rel=1e-11)
        assert abs(s.imag) < 1e-11 * 1000.0
        errs.append(c / math.exp(-b * q @ Dt @ q) - 1.0)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.9 < r1 < 4.1 and 3.9 < r2 < 4.1


def test_uform_slab_with_tensor_equals_scalar_Dxx():
    # a slab invariant in y and z, gradient along x: only D_xx acts (the
    # off-diagonal couplings integrate to zero over the periodic cross
    # section), so the full-tensor U-form signal equals the scalar one
    Dt = di.tensor([3e-3, 1e-3, 2e-3], (0.5, 0.7, 0.1))
    seq = di.Sequence(2000.0, 4000.0, 200.0, 0.5)
    ps = di.slab_box(n=12, half=4.0, split=10.0, D=(float(Dt[0, 0]),), cross=(1.0, 1),
                     periodic_mask=0b110)
    pt = di.slab_box(n=12, half=4.0, split=10.0, D=(float(Dt[0, 0]),), cross=(1.0, 1),
                     periodic_mask=0b110)
    pt.D = Dt[None]
    for mask in (0b110,):
        ss = timestep.signals(ps, seq, [2500.0], [[1, 0, 0]], form="uform", solver="splu")[0]
        st = timestep.signals(pt, seq, [2500.0], [[1, 0, 0]], form="uform", solver="splu")[0]
        assert abs(st - ss) < 1e-12 * abs(ss)
