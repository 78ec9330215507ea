"""Pins of the oracle's P1/PUFEM assembly.

* Element integrals (mass, stiffness, the skew first-order term, the
  x-weighted mass of the U-form, the interface face mass) are recomputed on
  random tetrahedra with an independent collapsed-coordinate Gauss rule and
  barycentric functions obtained by solving the 4x4 vertex system.
* Global invariants: total mass = volume, stiffness and the skew term
  annihilate constants on a torus, the face term sums to kappa |Gamma| with
  |Gamma| counted independently from voxel faces, DOF counts follow the PUFEM
  rule (one DOF per compartment touching a node, Appendix A eq. phase_func).
"""

import numpy as np
import pytest

import dmri_inputs as di
from oracle import fem

RNG = np.random.default_rng(1234)


def _single_tet_problem(v, D=1.7):
    xyz = np.asarray(v, dtype=np.float64)
    tets = np.array([[0, 1, 2, 3]], dtype=np.int32)
    lo = xyz.min(axis=0) - 1.0
    hi = xyz.max(axis=0) + 1.0
    return di.Problem(xyz, tets, np.zeros(1, np.int32), 1, np.array([D]), None, None, 0.0,
                      lo, hi, 0)


def _gauss_tet(v, n=6):
    """Collapsed (Duffy) tensor Gauss rule on a tetrahedron: points, weights."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            for c, wc in zip(g, w):
                l1 = a
                l2 = b * (1 - a)
                l3 = c * (1 - a) * (1 - b)
                jac = (1 - a) ** 2 * (1 - b)
                lam = np.array([1 - l1 - l2 - l3, l1, l2, l3])
                pts.append(lam @ v)
                wts.append(wa * wb * wc * jac)
    vol = abs(np.linalg.det(v[1:] - v[0])) / 6.0
    return np.array(pts), np.array(wts) * 6.0 * vol


def _barycentric(v):
    """Coefficients (c0, grad) of each lambda_i from [1 x y z] lambda = e_i."""
    A = np.hstack([np.ones((4, 1)), v])          # rows: vertices
    C = np.linalg.inv(A)                          # column i: coefficients of lambda_i
    return C[0, :], C[1:, :].T                    # c0[i], grad[i, :]


@pytest.mark.parametrize("trial", range(5))
def test_element_integrals_vs_quadrature(trial):
    v = RNG.normal(size=(4, 3)) * RNG.uniform(0.3, 3.0)
    if np.linalg.det(v[1:] - v[0]) < 0:
        v[[1, 2]] = v[[2, 1]]
    D = 1.7
    prob = _single_tet_problem(v, D)
    centre = np.array([0.3, -0.2, 0.5])
    asm = fem.assemble(prob, centre=centre)
    assert asm.n_dof == 4
    # Map mesh vertex i to its DOF.
    tn, _ = fem.torus_nodes(prob.xyz, prob.box_lo, prob.box_hi, 0)
    order = np.array([int(np.nonzero(asm.dof_node == tn[i])[0][0]) for i in range(4)])
    P = lambda A: A.toarray()[np.ix_(order, order)]  # noqa: E731

    x, w = _gauss_tet(v)
    c0, gr = _barycentric(v)
    lam = c0[None, :] + x @ gr.T                  # [nq, 4]
    mass = np.einsum("q,qi,qj->ij", w, lam, lam)
    stiff = w.sum() * gr @ gr.T
    np.testing.assert_allclose(P(asm.M), mass, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(P(asm.S), D * stiff, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(P(asm.MD), D * mass, rtol=1e-12, atol=1e-14)
    for a in range(3):
        # B_a[i,j] = D int (phi_i d_a phi_j - phi_j d_a phi_i)
        t1 = np.einsum("q,qi->i", w, lam)[:, None] * gr[None, :, a]
        Bq = D * (t1 - t1.T)
        np.testing.assert_allclose(P(asm.B[a]), Bq, rtol=1e-11, atol=1e-13)
        Jq = np.einsum("q,q,qi,qj->ij", w, x[:, a] - centre[a], lam, lam)
        np.testing.assert_allclose(P(asm.J[a]), Jq, rtol=1e-11, atol=1e-13)


def _gauss_tri(p, n=6):
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts, lams = [], [], []
    area = 0.5 * np.linalg.norm(np.cross(p[1] - p[0], p[2] - p[0]))
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            l1 = a
            l2 = b * (1 - a)
            lam = np.array([1 - l1 - l2, l1, l2])
            lams.append(lam)
            pts.append(lam @ p)
            wts.append(wa * wb * (1 - a))
    return np.array(lams), np.array(wts) * 2.0 * area


def test_interface_face_mass_vs_quadrature():
    # Two tets sharing the face (0,1,2) with different labels.
    v = np.array([[0.0, 0, 0], [1.3, 0.1, 0], [0.2, 0.9, 0.1], [0.3, 0.2, 1.1],
                  [0.4, 0.3, -0.9]])
    tets = np.array([[0, 1, 2, 3], [0, 2, 1, 4]], dtype=np.int32)
    kappa = 0.37
    prob = di.Problem(v, tets, np.array([0, 1], np.int32), 2, np.array([1.0, 2.0]), None, None,
                      kappa, v.min(0) - 1, v.max(0) + 1, 0)
    asm = fem.assemble(prob)
    assert asm.n_dof == 8
    lam, w = _gauss_tri(v[:3])
    Mf = np.einsum("q,qi,qj->ij", w, lam, lam)
    IG = asm.IG.toarray()
    tn, _ = fem.torus_nodes(v, prob.box_lo, prob.box_hi, 0)
    back = {int(t): i for i, t in enumerate(tn)}
    idx = {(int(c), back[int(nd)]): i for i, (c, nd) in enumerate(zip(asm.dof_comp, asm.dof_node))}
    for i in range(3):
        for j in range(3):
            a_i, a_j = idx[(0, i)], idx[(0, j)]
            b_i, b_j = idx[(1, i)], idx[(1, j)]
            assert IG[a_i, a_j] == pytest.approx(kappa * Mf[i, j], rel=1e-12)
            assert IG[b_i, b_j] == pytest.approx(kappa * Mf[i, j], rel=1e-12)
            assert IG[a_i, b_j] == pytest.approx(-kappa * Mf[i, j], rel=1e-12)
    # Vertices off the face carry no face term.
    assert abs(IG[idx[(0, 3)]]).sum() == 0 and abs(IG[idx[(1, 4)]]).sum() == 0
    assert asm.interface_area == pytest.approx(w.sum(), rel=1e-12)


def test_torus_invariants_free_box():
    prob = di.free_box(n=6, half=2.5)
    asm = fem.assemble(prob)
    assert asm.n_dof == 6 ** 3 == asm.n_torus_nodes
    one = np.ones(asm.n_dof)
    assert asm.M.sum() == pytest.approx(125.0, rel=1e-13)
    assert asm.w.sum() == pytest.approx(125.0, rel=1e-13)
    assert np.abs(asm.S @ one).max() < 1e-14
    for a in range(3):
        Ba = asm.B[a]
        assert abs(Ba + Ba.T).max() < 1e-15
        # On a torus the skew term also annihilates constants.
        assert np.abs(Ba @ one).max() < 1e-14
    # Kuhn lattice: every torus node has 14 neighbours plus itself.
    assert np.all(np.diff(asm.M.indptr) == 15)
    # M_D = D M for one compartment.
    assert abs(asm.MD - prob.D[0] * asm.M).max() < 1e-16


def test_neumann_box_x_weighted_mass():
    # int (x_a - c_a) over a box centred at c vanishes; shifting the centre
    # by s gives -s |Omega|.
    prob = di.free_box(n=4, half=1.5, periodic_mask=0)
    asm = fem.assemble(prob, centre=np.array([0.5, -0.25, 0.0]))
    one = np.ones(asm.n_dof)
    vol = 27.0
    assert one @ (asm.J[0] @ one) == pytest.approx(-0.5 * vol, rel=1e-12)
    assert one @ (asm.J[1] @ one) == pytest.approx(0.25 * vol, rel=1e-12)
    assert abs(one @ (asm.J[2] @ one)) < 1e-12


def _voxel_interface_area(n, half, r):
    """Count axis-aligned voxel faces between inside and outside cubes."""
    h = 2 * half / n
    c = -half + h * (np.arange(n) + 0.5)
    X, Y = np.meshgrid(c, c, indexing="ij")
    inside = X ** 2 + Y ** 2 < r * r
    faces = 0
    faces += np.count_nonzero(inside != np.roll(inside, 1, axis=0))
    faces += np.count_nonzero(inside != np.roll(inside, 1, axis=1))
    return faces * h * (2 * half)  # every column spans the full z extent


def test_pufem_dofs_and_interface_area_cube_labels():
    n, half, r = 12, 6.0, 4.0
    kappa = 0.25
    prob = di.cylinder_box(n=n, half=half, r=r, kappa=kappa, mode="cube")
    asm = fem.assemble(prob)
    area = _voxel_interface_area(n, half, r)
    assert asm.interface_area == pytest.approx(area, rel=1e-12)
    # 1_k^T I_Gamma 1_k = kappa |Gamma| for each side, -kappa |Gamma| across.
    e0 = (asm.dof_comp == 0).astype(float)
    e1 = (asm.dof_comp == 1).astype(float)
    assert e0 @ (asm.IG @ e0) == pytest.approx(kappa * area, rel=1e-12)
    assert e1 @ (asm.IG @ e1) == pytest.approx(kappa * area, rel=1e-12)
    assert e0 @ (asm.IG @ e1) == pytest.approx(-kappa * area, rel=1e-12)
    # Conservation structure: columns of I_Gamma sum to zero.
    assert np.abs(np.asarray(asm.IG.sum(axis=0))).max() < 1e-14
    # DOFs: torus nodes + nodes touched by both compartments.
    lab = prob.tet_label
    tn, ntor = fem.torus_nodes(prob.xyz, prob.box_lo, prob.box_hi, 7)
    touch = np.zeros((ntor, 2), bool)
    for k in range(2):
        touch[np.unique(tn[prob.tets[lab == k]]), k] = True
    assert asm.n_dof == touch.sum()
    assert ntor == n ** 3
    # Compartment volumes from the labels.
    h3 = (2 * half / n) ** 3
    ncube_in = np.count_nonzero(lab == 1) // 6
    assert asm.comp_volume[1] == pytest.approx(ncube_in * h3, rel=1e-12)


def test_transformed_operator_is_hermitian():
    prob = di.cylinder_box(n=8, half=6.0, r=4.0, kappa=1e-3, D_in=2e-3, D_out=3e-3)
    asm = fem.assemble(prob)
    q = np.array([0.3, -0.5, 0.8])
    q /= np.linalg.norm(q)
    GF, k, th = 0.37, 100.0, 0.5
    qB = q[0] * asm.B[0] + q[1] * asm.B[1] + q[2] * asm.B[2]
    A = asm.M / k + th * (asm.S + asm.IG + GF ** 2 * asm.MD + 1j * GF * qB)
    Ad = A.toarray()
    assert np.abs(Ad - Ad.conj().T).max() < 1e-15 * np.abs(Ad).max()
    ev = np.linalg.eigvalsh(Ad)
    assert ev.min() > 0


# ------------------------------------------- diffusion tensors (Sec. 2, Sec. 3)
# Per-compartment symmetric positive definite tensors on an unstructured,
# interface-conforming mesh: each assembled array against an exact integral
# of a function P1 represents exactly.

def _dof_xyz(p, asm):
    # coordinates of each DOF's node (dof_node numbers the identified nodes)
    tn, nt = fem.torus_nodes(p.xyz, p.box_lo, p.box_hi, p.periodic_mask)
    c = np.zeros((nt, 3))
    c[tn] = p.xyz
    return c[asm.dof_node]


def _tensor_prob(mask=0):
    return di.conforming_cylinder_box(
        n=6, half=6.0, r=4.0, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
        D_out=di.tensor([2e-3, 2.5e-3, 1.5e-3], (1.0, -0.4, 0.7)), kappa=5e-3,
        periodic_mask=mask, jitter=0.2, seed=4)


def test_tensor_stiffness_of_linear_field():
    # u = a.x is P1-exact on each compartment's copy: u^T S u = sum_k |Om_k| a^T D_k a
    p = _tensor_prob()
    asm = fem.assemble(p)
    a = np.array([0.3, -1.1, 0.7])
    u = _dof_xyz(p, asm) @ a
    want = sum(asm.comp_volume[k] * a @ p.D[k] @ a for k in range(2))
    assert u @ (asm.S @ u) == pytest.approx(want, rel=1e-12)


def test_tensor_mass_term_and_first_order_term():
    p = _tensor_prob()
    asm = fem.assemble(p)
    q = np.array([0.48, 0.6, 0.64])
    qq = (q[0] ** 2, q[1] ** 2, q[2] ** 2, 2 * q[0] * q[1], 2 * q[0] * q[2], 2 * q[1] * q[2])
    Mq = sum(c * m for c, m in zip(qq, asm.MDab))
    one = np.ones(asm.n_dof)
    assert one @ (Mq @ one) == pytest.approx(
        sum(asm.comp_volume[k] * q @ p.D[k] @ q for k in range(2)), rel=1e-12)
    # 1^T B_q u = int (D q).grad u - u (D q).grad 1 = sum_k |Om_k| (D_k q).a
    a = np.array([0.3, -1.1, 0.7])
    u = _dof_xyz(p, asm) @ a
    Bq = q[0] * asm.B[0] + q[1] * asm.B[1] + q[2] * asm.B[2]
    assert one @ (Bq @ u) == pytest.approx(
        sum(asm.comp_volume[k] * (p.D[k] @ q) @ a for k in range(2)), rel=1e-11)
    # a scalar D gives MDab = D delta_ab M
    ps = di.conforming_cylinder_box(n=5, D_in=1e-3, D_out=3e-3, periodic_mask=0)
    asms = fem.assemble(ps)
    assert abs(asms.MDab[0] - asms.MD).max() < 1e-15 and asms.MDab[3].nnz == 0 or \
        abs(asms.MDab[3]).max() == 0.0
