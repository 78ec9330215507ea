"""P1 finite-element assembly with PUFEM compartments (oracle, FP64).

Test infrastructure only (see the package header).

Follows:
* Appendix A (strong pseudo-periodic imposition): the unknown
  u = U exp(i gamma F g.x) satisfies plain periodic conditions, so opposite
  box faces are identified (a torus mesh) and the operator gains a
  first-order term and a (gamma F)^2 g.Dg mass term (eq. trBlo).
* Appendix A, eq. theta_discretization and eq. phase_func: one P1 field per
  compartment; an element of compartment k contributes only to the DOFs of
  compartment k (the phase function Phi_h selects the field).
* Sec. 2, eq. btpde_ic: permeable interface, flux = -kappa [[u]], giving the
  face term kappa <[[u]], [[v]]>_Gamma (also in eq. loadvec).
* Appendix B, eq. loadvec / eq. matrix_form: the untransformed U-form with
  the (g.x)-weighted mass matrix J, used for boxes with Neumann walls.
* Appendix B, eq. bjump1/bjump2/weak_periodic, forms a* and L*: with bit 3
  of periodic_mask set, the axes in bits 0-2 get weak pseudo-periodic faces
  (artificial permeability, oracle/weakbc.py) on the U-form; their faces
  are not identified.

Reading of the first-order term. Substituting U = u exp(-i phi) and the
test function exp(+i phi) v (phi = gamma F g.x) into the bilinear U weak
form turns -(D grad U, grad V) into
  -(D grad u, grad v) - i gamma F [(Dg.grad u, v) - (u, Dg.grad v)]
  - (gamma F)^2 (g.Dg u, v),
which is the paper's weak form of Appendix A after integration by parts with
the interface terms absorbed. With g = G q (G = gamma |g|) and isotropic D_k
per compartment this gives, for test index i and trial index j,
  B_a[i, j] = sum_k D_k int_{Omega_k} (phi_i d_a phi_j - phi_j d_a phi_i)
(real, skew) and M_D = sum_k D_k int_{Omega_k} phi_i phi_j.

Element integrals (textbook P1 on a tetrahedron e with barycentric
coordinates lambda, volume |e|, face area |f|):
  int_e phi_i phi_j      = |e| (1 + delta_ij) / 20
  int_e grad phi_i . grad phi_j = |e| grad lambda_i . grad lambda_j
  int_e phi_i d_a phi_j  = |e| d_a lambda_j / 4
  int_e x_a phi_i phi_j  = |e| (1 + delta_ij)/120 (sum_l x_a,l + x_a,i + x_a,j)
  int_f phi_i phi_j      = |f| (1 + delta_ij) / 12
These are pinned against an independent collapsed-coordinate Gauss
quadrature in tests/test_oracle_fem.py.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class Assembly:
    """Real sparse operators on the DOF set, in the oracle's own DOF order."""

    n_dof: int
    dof_comp: np.ndarray      # [n_dof] compartment of each DOF
    dof_node: np.ndarray      # [n_dof] torus node of each DOF
    M: sp.csr_matrix          # mass
    S: sp.csr_matrix          # sum_k D_k stiffness
    MD: sp.csr_matrix         # sum_k D_k mass (trace(D)/3 for tensors)
    B: tuple                  # (Bx, By, Bz) real skew
    R2: sp.csr_matrix         # sum_k (1/T2_k) mass
    IG: sp.csr_matrix         # kappa * interface jump face mass
    J: tuple                  # (Jx, Jy, Jz): int (x_a - c_a) phi_i phi_j
    w: np.ndarray             # signal weights int phi_i over its compartment
    u0: np.ndarray            # initial value per DOF
    comp_volume: np.ndarray   # |Omega_k|
    interface_area: float     # |Gamma| (sum of interface face areas)
    n_torus_nodes: int
    tet_dof: np.ndarray = None  # [n_tets, 4] DOF of each vertex (its tet's compartment)
    MDab: tuple = None        # int D_ab phi_i phi_j for ab = xx, yy, zz, xy, xz, yz
    # weak pseudo-periodic faces (Appendix B): kappa_e face mass on the faces
    # of the weak axes, and per axis (C_ms, C_sm, L_a) partner couplings
    KB: sp.csr_matrix = None
    weak: tuple = ()
    kappa_e: float = 0.0      # max{D / h} before the weak_kappa scale


def torus_nodes(xyz, box_lo, box_hi, periodic_mask, rel_tol=1e-9):
    """Identify nodes on opposite faces of the box along periodic axes.

    Returns (node -> torus id, number of torus nodes). Coordinates are
    rounded to a grid of rel_tol * box size; a node on the upper face of a
    periodic axis is moved to the lower face before matching. Weak
    pseudo-periodic faces (bit 3 of the mask) are never identified.
    """
    if periodic_mask & 8:
        periodic_mask = 0
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    L = hi - lo
    scale = 1.0 / rel_tol
    key = np.rint((xyz - lo) / L * scale).astype(np.int64)
    top = int(round(scale))
    for a in range(3):
        if periodic_mask >> a & 1:
            key[key[:, a] == top, a] = 0
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    return inv.reshape(-1).astype(np.int64), int(uniq.shape[0])


def tet_geometry(xyz, tets):
    """Volumes [m] and barycentric gradients [m, 4, 3] of each tetrahedron."""
    v = xyz[tets]                                   # [m, 4, 3]
    E = v[:, 1:, :] - v[:, :1, :]                   # rows: edges from vertex 0
    det = np.linalg.det(E)
    vol = np.abs(det) / 6.0
    # lambda_j(x) = lambda_j(v0) + g_j . (x - v0); for j=1..3 the gradients are
    # the rows of inv(E)^T, i.e. E^{-1} columns; lambda_0 = 1 - sum.
    Einv = np.linalg.inv(E)                         # [m, 3, 3]
    g123 = np.transpose(Einv, (0, 2, 1))            # g_j = column j of E^{-1}
    g0 = -g123.sum(axis=1, keepdims=True)
    grads = np.concatenate([g0, g123], axis=1)      # [m, 4, 3]
    return vol, grads, det


def _coo(rows, cols, vals, n):
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(n, n)).tocsr()


def assemble(prob, centre: Optional[np.ndarray] = None, weak_kappa: float = 1.0) -> Assembly:
    """Assemble every real operator of the method on the PUFEM DOF set."""
    xyz = np.asarray(prob.xyz, dtype=np.float64)
    tets = np.asarray(prob.tets, dtype=np.int64)
    lab = np.asarray(prob.tet_label, dtype=np.int64)
    K = int(prob.n_comp)
    # D: a scalar per compartment, or a symmetric 3x3 tensor per compartment
    # (Sec. 2: D(x) symmetric positive definite; Sec. 3, "Diffusion
    # coefficients and tensors": piecewise constant per partition marker).
    D = np.asarray(prob.D, dtype=np.float64)
    if D.ndim == 1:
        Dt = D[:, None, None] * np.eye(3)[None]
    else:
        Dt = D.reshape(K, 3, 3)
    invT2 = np.zeros(K) if prob.T2 is None else 1.0 / np.asarray(prob.T2, dtype=np.float64)
    u0c = np.ones(K) if prob.u0 is None else np.asarray(prob.u0, dtype=np.float64)
    if centre is None:
        centre = 0.5 * (np.asarray(prob.box_lo) + np.asarray(prob.box_hi))

    pmask = int(prob.periodic_mask)
    weak_axes = [a for a in range(3) if pmask & 8 and pmask >> a & 1]
    # weakly periodic axes are not identified (the U-form on the open box)
    tnode, n_torus = torus_nodes(xyz, prob.box_lo, prob.box_hi, pmask)
    tt = tnode[tets]                                # [m, 4] torus nodes
    # PUFEM DOF (k, torus node) exists iff the node touches a tet of label k.
    key = lab[:, None] * n_torus + tt               # [m, 4]
    ukeys, dof_of = np.unique(key.ravel(), return_inverse=True)
    dof = dof_of.reshape(tets.shape)
    n_dof = int(ukeys.shape[0])
    dof_comp = ukeys // n_torus
    dof_node = ukeys % n_torus

    vol, grads, _ = tet_geometry(xyz, tets)
    m = tets.shape[0]
    eye = np.eye(4)
    R = np.repeat(dof[:, :, None], 4, axis=2)       # row = test index i
    C = np.repeat(dof[:, None, :], 4, axis=1)       # col = trial index j

    Me = vol[:, None, None] * (1.0 + eye)[None] / 20.0
    De = Dt[lab]                                       # [m, 3, 3] tensor of each tet
    # stiffness: int grad phi_i . D grad phi_j = |e| grad lambda_i^T D grad lambda_j
    Se = vol[:, None, None] * np.einsum("mia,mab,mjb->mij", grads, De, grads)
    M = _coo(R, C, Me, n_dof)
    S = _coo(R, C, Se, n_dof)
    # (gamma F)^2 g.Dg mass term: g.Dg = G^2 sum_ab q_a q_b D_ab, so six arrays
    # int D_ab phi_i phi_j; for a scalar D they are D delta_ab times the mass.
    pairs_ab = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    MDab = tuple(_coo(R, C, De[:, a, b][:, None, None] * Me, n_dof) for a, b in pairs_ab)
    MD = _coo(R, C, (np.trace(De, axis1=1, axis2=2) / 3.0)[:, None, None] * Me, n_dof)
    R2 = _coo(R, C, invT2[lab][:, None, None] * Me, n_dof)
    B = []
    J = []
    xs = xyz[tets] - np.asarray(centre)[None, None, :]   # [m, 4, 3]
    for a in range(3):
        # first-order term (D g).grad with g = G q: int (phi_i d_b phi_j - phi_j
        # d_b phi_i) (D q)_b = sum_a q_a [sum_b D_ba int (phi_i d_b phi_j - ...)]
        gDa = np.einsum("mib,mb->mi", grads, De[:, :, a])   # sum_b D_ba d_b lambda_i
        Be = vol[:, None, None] * (gDa[:, None, :] - gDa[:, :, None]) / 4.0
        B.append(_coo(R, C, Be, n_dof))
        xa = xs[:, :, a]
        ssum = xa.sum(axis=1)
        Je = (vol[:, None, None] * (1.0 + eye)[None] / 120.0
              * (ssum[:, None, None] + xa[:, :, None] + xa[:, None, :]))
        J.append(_coo(R, C, Je, n_dof))

    w = np.asarray(M.sum(axis=1)).ravel()
    comp_volume = np.bincount(lab, weights=vol, minlength=K)

    # Interface faces: a face (three torus nodes) shared by tets of different
    # labels. Local faces opposite vertex 0..3.
    faces_local = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    ft = tt[:, faces_local]                          # [m, 4, 3] torus ids
    fkey = np.sort(ft, axis=2).reshape(-1, 3)
    owner = np.repeat(np.arange(m), 4)
    local = np.tile(np.arange(4), m)
    order = np.lexsort((fkey[:, 2], fkey[:, 1], fkey[:, 0]))
    fk = fkey[order]
    same = np.all(fk[1:] == fk[:-1], axis=1)
    pairs = np.nonzero(same)[0]
    IG_rows, IG_cols, IG_vals = [], [], []
    area_total = 0.0
    kappa = float(prob.kappa)
    for p in pairs:
        a_idx, b_idx = order[p], order[p + 1]
        ta, tb = owner[a_idx], owner[b_idx]
        if lab[ta] == lab[tb]:
            continue
        # Face vertices in tet a's coordinates and their DOFs on both sides,
        # matched through the torus node ids.
        la = faces_local[local[a_idx]]
        lb = faces_local[local[b_idx]]
        pa = xyz[tets[ta, la]]
        area = 0.5 * np.linalg.norm(np.cross(pa[1] - pa[0], pa[2] - pa[0]))
        area_total += area
        na = tt[ta, la]
        nb = tt[tb, lb]
        da = dof[ta, la]
        perm = [int(np.nonzero(nb == x)[0][0]) for x in na]
        db = dof[tb, lb][perm]
        Mf = area * (1.0 + np.eye(3)) / 12.0
        for i in range(3):
            for j in range(3):
                for (r, c, s) in ((da[i], da[j], 1.0), (db[i], db[j], 1.0),
                                  (da[i], db[j], -1.0), (db[i], da[j], -1.0)):
                    IG_rows.append(r)
                    IG_cols.append(c)
                    IG_vals.append(s * kappa * Mf[i, j])
    if IG_rows:
        IG = sp.coo_matrix((IG_vals, (IG_rows, IG_cols)), shape=(n_dof, n_dof)).tocsr()
    else:
        IG = sp.csr_matrix((n_dof, n_dof))

    KB = None
    weak = ()
    ke0 = 0.0
    if weak_axes:
        from . import weakbc
        Dmax = np.array([np.linalg.eigvalsh(Dt[k])[-1] for k in range(K)])
        ke0 = weakbc.kappa_e(prob, Dmax[lab], weak_axes)
        ke = weak_kappa * ke0
        KB = sp.csr_matrix((n_dof, n_dof))
        wl = []
        for a in weak_axes:
            La = float(prob.box_hi[a] - prob.box_lo[a])
            Cms, Csm, Kf = weakbc.coupling(prob, dof, a, ke, La)
            KB = KB + Kf
            wl.append((a, Cms, Csm, La))
        weak = tuple(wl)

    return Assembly(n_dof=n_dof, dof_comp=dof_comp, dof_node=dof_node, M=M, S=S, MD=MD,
                    B=tuple(B), R2=R2, MDab=MDab, IG=IG, J=tuple(J), w=w, u0=u0c[dof_comp],
                    comp_volume=comp_volume, interface_area=area_total,
                    n_torus_nodes=n_torus, tet_dof=dof, KB=KB, weak=weak,
                    kappa_e=ke0)
