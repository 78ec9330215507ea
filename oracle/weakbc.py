"""Weak pseudo-periodic conditions by artificial permeability (oracle, FP64).

Test infrastructure only (see the package header).

Appendix B (eq. bjump1, eq. bjump2, eq. weak_periodic and the modified
forms a*, L* after eq. matrix_form): on a box whose opposite faces are not
identified, the flux through a face point x_m of the master face
(x_a = lo_a) is kappa_e (U_s e^{i theta_ms} - U_m) with U_s the field at the
opposite point x_s = x_m + L_a e_a of the slave face (x_a = hi_a), and
symmetrically on the slave face, theta_ms = -theta_sm = gamma g.(x_s - x_m)
F(t) = G F q_a L_a. The operator splitting of eq. weak_periodic lags the
partner by one step, and the forms become
  a*(U^n, v) = a + theta kappa_e (<U^n, v>_{Gamma_m} + <U^n, v>_{Gamma_s})
  L*(v)      = L + (1 - theta) kappa_e (<U_s^{n-1} e^{i theta_ms^n}, v>_{Gamma_m}
                                        + <U_m^{n-1} e^{i theta_sm^n}, v>_{Gamma_s}).
kappa_e = max{D / h} (the Nitsche-consistent choice after eq. bjump2):
one constant per problem, the largest D_k / h_e over the tetrahedra that
have a face on a weakly periodic box face, with D_k the largest eigenvalue
of the element's compartment tensor (the scalar itself when isotropic) and
h_e the element's longest edge.

The coupling integrals int_{Gamma_m} phi_i(x) phi_j(x + L e_a) dx are exact:
every master face triangle is intersected with every translated slave face
triangle whose bounding box overlaps it (convex polygon clipping), the
intersection fanned into triangles and the product of the two linear
functions integrated with the edge-midpoint rule (exact for degree 2). The
faces need not match node for node (non-matching meshes).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _boundary_faces(xyz, tets, axis, value, tol):
    """Faces of tets lying in the plane x_axis = value: (tet, local vertex ids)."""
    local = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    out = []
    on = np.abs(xyz[:, axis] - value) <= tol
    onv = on[tets]                                        # [m, 4]
    cand = np.nonzero(onv.sum(axis=1) >= 3)[0]
    for e in cand:
        for f in range(4):
            if np.all(onv[e, local[f]]):
                out.append((e, local[f]))
    return out


def _clip(poly, tri):
    """Sutherland-Hodgman: convex polygon `poly` [k,2] clipped by the
    counter-clockwise triangle `tri` [3,2]."""
    out = list(poly)
    for i in range(3):
        a, b = tri[i], tri[(i + 1) % 3]
        inp, out = out, []
        if not inp:
            break
        def inside(p):
            return (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0]) >= -1e-15

        def cut(p, q):
            d1 = (b[0] - a[0]) * (p[1] - a[1]) - (b[1] - a[1]) * (p[0] - a[0])
            d2 = (b[0] - a[0]) * (q[1] - a[1]) - (b[1] - a[1]) * (q[0] - a[0])
            t = d1 / (d1 - d2)
            return p + t * (q - p)
        for k in range(len(inp)):
            p, q = inp[k], inp[(k + 1) % len(inp)]
            if inside(q):
                if not inside(p):
                    out.append(cut(p, q))
                out.append(q)
            elif inside(p):
                out.append(cut(p, q))
    return np.array(out) if out else np.zeros((0, 2))


def _ccw(t):
    t = np.asarray(t, dtype=np.float64)
    area2 = (t[1, 0] - t[0, 0]) * (t[2, 1] - t[0, 1]) - (t[1, 1] - t[0, 1]) * (t[2, 0] - t[0, 0])
    return (t[[0, 2, 1]], -area2) if area2 < 0 else (t, area2)


def _bary(t, p):
    """Barycentric coordinates of points p [k,2] in triangle t [3,2]."""
    T = np.array([[t[0, 0] - t[2, 0], t[1, 0] - t[2, 0]], [t[0, 1] - t[2, 1], t[1, 1] - t[2, 1]]])
    l01 = np.linalg.solve(T, (p - t[2]).T).T
    return np.column_stack([l01, 1.0 - l01.sum(axis=1)])


def coupling(prob, dof, axis, ke, L):
    """Coupling matrices of one axis: (C_ms, C_sm, face mass on both faces)
    with kappa_e folded in. dof: [m, 4] DOF of each tet vertex."""
    xyz = np.asarray(prob.xyz, dtype=np.float64)
    tets = np.asarray(prob.tets, dtype=np.int64)
    lo, hi = float(prob.box_lo[axis]), float(prob.box_hi[axis])
    tol = 1e-9 * L
    other = [b for b in range(3) if b != axis]
    faces = {0: _boundary_faces(xyz, tets, axis, lo, tol), 1: _boundary_faces(xyz, tets, axis, hi, tol)}
    n = int(dof.max()) + 1
    rows, cols, vals = {0: [], 1: []}, {0: [], 1: []}, {0: [], 1: []}
    mrows, mcols, mvals = [], [], []
    tri2d = {s: [xyz[tets[e, lv]][:, other] for e, lv in faces[s]] for s in (0, 1)}
    # face mass kappa_e |f| (1 + delta_ij)/12 on both faces (implicit term)
    for s in (0, 1):
        for (e, lv), t in zip(faces[s], tri2d[s]):
            _, a2 = _ccw(t)
            area = 0.5 * a2
            d = dof[e, lv]
            for i in range(3):
                for j in range(3):
                    mrows.append(d[i])
                    mcols.append(d[j])
                    mvals.append(ke * area * (2.0 if i == j else 1.0) / 12.0)
    # partner coupling: rows on side s, columns on the opposite side
    for s in (0, 1):
        o = 1 - s
        otri = [(_ccw(t)[0], e, lv) for (e, lv), t in zip(faces[o], tri2d[o])]
        obox = np.array([[t[:, 0].min(), t[:, 1].min(), t[:, 0].max(), t[:, 1].max()]
                         for t, _, _ in otri])
        for (e, lv), t in zip(faces[s], tri2d[s]):
            tm, _ = _ccw(t)
            # vertex order of tm matches lv after the possible swap
            lvm = lv if np.allclose(tm, t) else lv[[0, 2, 1]]
            dm = dof[e, lvm]
            bb = (tm[:, 0].min(), tm[:, 1].min(), tm[:, 0].max(), tm[:, 1].max())
            hit = np.nonzero((obox[:, 0] <= bb[2] + tol) & (obox[:, 2] >= bb[0] - tol) &
                             (obox[:, 1] <= bb[3] + tol) & (obox[:, 3] >= bb[1] - tol))[0]
            for h in hit:
                ts, es, lvs = otri[h]
                ts0 = xyz[tets[es, lvs]][:, other]
                lvs2 = lvs if np.allclose(ts, ts0) else lvs[[0, 2, 1]]
                ds = dof[es, lvs2]
                poly = _clip(tm, ts)
                if len(poly) < 3:
                    continue
                for k in range(1, len(poly) - 1):
                    sub = np.array([poly[0], poly[k], poly[k + 1]])
                    _, a2 = _ccw(sub)
                    if a2 <= 1e-30:
                        continue
                    mids = 0.5 * (sub + sub[[1, 2, 0]])
                    bm = _bary(tm, mids)                 # master basis at the midpoints
                    bs = _bary(ts, mids)                 # partner basis at the same points
                    w = (0.5 * a2) / 3.0
                    for i in range(3):
                        for j in range(3):
                            rows[s].append(dm[i])
                            cols[s].append(ds[j])
                            vals[s].append(ke * w * np.sum(bm[:, i] * bs[:, j]))
    mk = lambda r, c, v: sp.coo_matrix((v, (r, c)), shape=(n, n)).tocsr()  # noqa: E731
    return mk(rows[0], cols[0], vals[0]), mk(rows[1], cols[1], vals[1]), mk(mrows, mcols, mvals)


def kappa_e(prob, tet_D, axes):
    """The constant kappa_e = max D_e / h_e over the tetrahedra with a face on
    a face of the weak axes; tet_D [m] the largest eigenvalue of each tet's
    diffusivity."""
    xyz = np.asarray(prob.xyz, dtype=np.float64)
    tets = np.asarray(prob.tets, dtype=np.int64)
    v = xyz[tets]
    h = np.zeros(v.shape[0])
    for a in range(4):
        for b in range(a + 1, 4):
            h = np.maximum(h, np.linalg.norm(v[:, a] - v[:, b], axis=1))
    best = 0.0
    for a in axes:
        L = float(prob.box_hi[a] - prob.box_lo[a])
        for value in (float(prob.box_lo[a]), float(prob.box_hi[a])):
            for e, _ in _boundary_faces(xyz, tets, a, value, 1e-9 * L):
                best = max(best, tet_D[e] / h[e])
    return best
