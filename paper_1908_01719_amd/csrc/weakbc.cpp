// Weak pseudo-periodic box faces by an artificial permeability (Appendix B,
// eq. bjump1, eq. bjump2, eq. weak_periodic and the forms a*, L*).
//
// For every weak axis a the face x_a = lo_a (master) and the face
// x_a = hi_a (slave) exchange flux kappa_e (U_partner e^{+-i phi_a} - U).
// The operator splitting lags the partner by one step, so the library needs
//   * the face mass  kappa_e <phi_i, phi_j> on both faces, added to the
//     left operator with theta (a*), stored on the CSR pattern (a face's
//     three DOFs belong to one tetrahedron, so the pattern holds them);
//   * the couplings  kappa_e int_{Gamma_m} phi_i(x) phi_j(x + L_a e_a)
//     (rows on the master face, columns on the slave face) and their
//     transposes (rows on the slave face), applied to the previous step
//     with (1 - theta) and the phase of t^n (L*).
// The faces need not match: each master triangle is intersected with the
// slave triangles that overlap it (both projected on the face plane), the
// convex intersection is split into triangles and the product of the two
// linear basis functions is integrated exactly with the vertex rule
//   int_T f g = |T| / 12 (sum_v f_v g_v + (sum_v f_v)(sum_v g_v)).
// kappa_e = max{D / h} (the Nitsche-consistent choice of Appendix B): one
// constant, the largest lambda_max(D_k) / h_e over the tetrahedra with a
// face on a weak face (h_e = longest edge), times a user scale.
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include "assembly.hpp"

namespace dmri {
namespace {

struct P2 {
    double u, v;
};

inline double orient(const P2& a, const P2& b, const P2& p) {
    return (b.u - a.u) * (p.v - a.v) - (b.v - a.v) * (p.u - a.u);
}

struct FaceTri {
    P2 p[3];          // counter-clockwise in the (b, c) plane
    int32_t dof[3];   // DOF of each vertex (in the order of p)
    double area;
    int64_t tet;
};

// Barycentric coordinates of x in triangle t.
inline void bary(const FaceTri& t, const P2& x, double l[3]) {
    const double a2 = orient(t.p[0], t.p[1], t.p[2]);
    l[0] = orient(t.p[1], t.p[2], x) / a2;
    l[1] = orient(t.p[2], t.p[0], x) / a2;
    l[2] = 1.0 - l[0] - l[1];
}

// Clip convex polygon poly (counter-clockwise) by the triangle t.
void clip(std::vector<P2>& poly, const FaceTri& t, double eps) {
    std::vector<P2> out;
    for (int e = 0; e < 3 && !poly.empty(); ++e) {
        const P2 a = t.p[e], b = t.p[(e + 1) % 3];
        out.clear();
        const size_t n = poly.size();
        for (size_t k = 0; k < n; ++k) {
            const P2 cur = poly[k], nxt = poly[(k + 1) % n];
            const double dc = orient(a, b, cur), dn = orient(a, b, nxt);
            const bool ic = dc >= -eps, in_ = dn >= -eps;
            if (ic) out.push_back(cur);
            if (ic != in_) {
                const double s = dc / (dc - dn);
                out.push_back({cur.u + s * (nxt.u - cur.u), cur.v + s * (nxt.v - cur.v)});
            }
        }
        poly.swap(out);
    }
}

struct Coo {
    int32_t row, code, col;
    double val;
    bool operator<(const Coo& o) const {
        if (row != o.row) return row < o.row;
        if (code != o.code) return code < o.code;
        return col < o.col;
    }
};

}  // namespace

double lambda_max(double A[3][3]) {
    for (int sweep = 0; sweep < 32; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        const double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {  // A = J^T A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
            }
    }
    return std::max(A[0][0], std::max(A[1][1], A[2][2]));
}

void add_weak_faces(const MeshInput& in, const std::vector<int32_t>& tdof, HostOperator& op) {
    static const int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    const int64_t nT = in.n_tets;
    double L[3];
    for (int a = 0; a < 3; ++a) L[a] = in.hi[a] - in.lo[a];
    auto pos = [&](int32_t r, int32_t c) -> int64_t {
        const int32_t* b = op.col.data() + op.row_ptr[r];
        const int32_t* e = op.col.data() + op.row_ptr[r + 1];
        const int32_t* p = std::lower_bound(b, e, c);
        if (p == e || *p != c) throw Error(DMRI_E_INVALID, "internal: face entry off the pattern");
        return p - op.col.data();
    };
    // largest eigenvalue of each compartment's diffusivity
    std::vector<double> dmax(in.n_comp);
    for (int32_t k = 0; k < in.n_comp; ++k) {
        if (in.Dt) {
            const double* t = in.Dt + 6 * k;
            double A[3][3] = {{t[0], t[3], t[4]}, {t[3], t[1], t[5]}, {t[4], t[5], t[2]}};
            dmax[k] = lambda_max(A);
        } else {
            dmax[k] = in.D[k];
        }
    }
    // faces on the planes of the weak axes: side 0 = lo (master), 1 = hi
    std::array<std::array<std::vector<FaceTri>, 2>, 3> faces;
    double kappa_e = 0.0;
    for (int64_t e = 0; e < nT; ++e) {
        const int32_t* tv = in.tets + 4 * e;
        for (int a = 0; a < 3; ++a) {
            if (!(in.periodic_mask >> a & 1)) continue;
            const int b = (a + 1) % 3, c = (a + 2) % 3;
            const double tol = 1e-9 * L[a];
            for (int f = 0; f < 4; ++f) {
                for (int side = 0; side < 2; ++side) {
                    const double plane = side ? in.hi[a] : in.lo[a];
                    bool on = true;
                    for (int i = 0; i < 3 && on; ++i)
                        on = std::fabs(in.xyz[3 * tv[kFace[f][i]] + a] - plane) <= tol;
                    if (!on) continue;
                    FaceTri t;
                    for (int i = 0; i < 3; ++i) {
                        const double* x = in.xyz + 3 * tv[kFace[f][i]];
                        t.p[i] = {x[b], x[c]};
                        t.dof[i] = tdof[4 * e + kFace[f][i]];
                    }
                    double a2 = orient(t.p[0], t.p[1], t.p[2]);
                    if (a2 < 0) {
                        std::swap(t.p[1], t.p[2]);
                        std::swap(t.dof[1], t.dof[2]);
                        a2 = -a2;
                    }
                    t.area = 0.5 * a2;
                    t.tet = e;
                    faces[a][side].push_back(t);
                    double h2 = 0.0;
                    for (int i = 0; i < 4; ++i)
                        for (int j = i + 1; j < 4; ++j) {
                            double s = 0.0;
                            for (int cc = 0; cc < 3; ++cc) {
                                const double d = in.xyz[3 * tv[i] + cc] - in.xyz[3 * tv[j] + cc];
                                s += d * d;
                            }
                            h2 = std::max(h2, s);
                        }
                    kappa_e = std::max(kappa_e, dmax[in.label[e]] / std::sqrt(h2));
                }
            }
        }
    }
    op.kappa_e = kappa_e;
    op.KB.assign(op.nnz, 0.0);
    std::vector<Coo> coo;
    for (int a = 0; a < 3; ++a) {
        if (!(in.periodic_mask >> a & 1)) continue;
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        const double want = L[b] * L[c];
        for (int side = 0; side < 2; ++side) {
            double area = 0.0;
            for (const FaceTri& t : faces[a][side]) {
                area += t.area;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        op.KB[pos(t.dof[i], t.dof[j])] +=
                            kappa_e * t.area * (i == j ? 2.0 : 1.0) / 12.0;
            }
            if (!(std::fabs(area - want) <= 1e-8 * want))
                throw Error(DMRI_E_INVALID,
                            "weakly periodic axis: a box face is not fully covered by mesh faces");
        }
        // bucket grid of the slave triangles
        const std::vector<FaceTri>& ms = faces[a][0];
        const std::vector<FaceTri>& sl = faces[a][1];
        const int nb = std::max(1, static_cast<int>(std::sqrt(static_cast<double>(sl.size()))));
        auto cell = [&](double x, int axis) {
            const double r = (x - in.lo[axis]) / L[axis] * nb;
            return std::min(nb - 1, std::max(0, static_cast<int>(std::floor(r))));
        };
        std::vector<std::vector<int32_t>> bucket(static_cast<size_t>(nb) * nb);
        for (size_t s = 0; s < sl.size(); ++s) {
            double u0 = sl[s].p[0].u, u1 = u0, v0 = sl[s].p[0].v, v1 = v0;
            for (int i = 1; i < 3; ++i) {
                u0 = std::min(u0, sl[s].p[i].u);
                u1 = std::max(u1, sl[s].p[i].u);
                v0 = std::min(v0, sl[s].p[i].v);
                v1 = std::max(v1, sl[s].p[i].v);
            }
            for (int i = cell(u0, b); i <= cell(u1, b); ++i)
                for (int j = cell(v0, c); j <= cell(v1, c); ++j)
                    bucket[static_cast<size_t>(i) * nb + j].push_back(static_cast<int32_t>(s));
        }
        std::vector<int64_t> stamp(sl.size(), -1);
        const double eps = 1e-13 * want;
        double covered = 0.0;
        std::vector<P2> poly;
        for (size_t m = 0; m < ms.size(); ++m) {
            const FaceTri& tm = ms[m];
            double u0 = tm.p[0].u, u1 = u0, v0 = tm.p[0].v, v1 = v0;
            for (int i = 1; i < 3; ++i) {
                u0 = std::min(u0, tm.p[i].u);
                u1 = std::max(u1, tm.p[i].u);
                v0 = std::min(v0, tm.p[i].v);
                v1 = std::max(v1, tm.p[i].v);
            }
            for (int i = cell(u0, b); i <= cell(u1, b); ++i)
                for (int j = cell(v0, c); j <= cell(v1, c); ++j)
                    for (int32_t s : bucket[static_cast<size_t>(i) * nb + j]) {
                        if (stamp[s] == static_cast<int64_t>(m)) continue;
                        stamp[s] = static_cast<int64_t>(m);
                        const FaceTri& ts = sl[s];
                        poly.assign(tm.p, tm.p + 3);
                        clip(poly, ts, eps);
                        if (poly.size() < 3) continue;
                        double mm[3][3] = {};  // int phi^m_i phi^s_j over the overlap
                        for (size_t k = 1; k + 1 < poly.size(); ++k) {
                            const P2 q[3] = {poly[0], poly[k], poly[k + 1]};
                            const double ar = 0.5 * orient(q[0], q[1], q[2]);
                            if (!(ar > 0.0)) continue;
                            covered += ar;
                            double lm[3][3], ls[3][3];  // [vertex][basis]
                            for (int v = 0; v < 3; ++v) {
                                bary(tm, q[v], lm[v]);
                                bary(ts, q[v], ls[v]);
                            }
                            for (int ii = 0; ii < 3; ++ii)
                                for (int jj = 0; jj < 3; ++jj) {
                                    double s1 = 0.0, fi = 0.0, gj = 0.0;
                                    for (int v = 0; v < 3; ++v) {
                                        s1 += lm[v][ii] * ls[v][jj];
                                        fi += lm[v][ii];
                                        gj += ls[v][jj];
                                    }
                                    mm[ii][jj] += ar / 12.0 * (s1 + fi * gj);
                                }
                        }
                        for (int ii = 0; ii < 3; ++ii)
                            for (int jj = 0; jj < 3; ++jj) {
                                const double v = kappa_e * mm[ii][jj];
                                if (v == 0.0) continue;
                                coo.push_back({tm.dof[ii], a, ts.dof[jj], v});      // master row
                                coo.push_back({ts.dof[jj], 3 + a, tm.dof[ii], v});  // slave row
                            }
                    }
        }
        if (!(std::fabs(covered - want) <= 1e-8 * want))
            throw Error(DMRI_E_INVALID,
                        "weakly periodic axis: the opposite box faces do not cover each other");
    }
    // merge duplicates into rows of (code, col)
    std::sort(coo.begin(), coo.end());
    op.wk_rows.clear();
    op.wk_ptr.assign(1, 0);
    op.wk_col.clear();
    op.wk_code.clear();
    op.wk_val.clear();
    for (size_t i = 0; i < coo.size();) {
        size_t j = i;
        double v = 0.0;
        while (j < coo.size() && coo[j].row == coo[i].row && coo[j].code == coo[i].code &&
               coo[j].col == coo[i].col)
            v += coo[j++].val;
        if (op.wk_rows.empty() || op.wk_rows.back() != coo[i].row) {
            if (!op.wk_rows.empty()) op.wk_ptr.push_back(static_cast<int32_t>(op.wk_col.size()));
            op.wk_rows.push_back(coo[i].row);
        }
        op.wk_col.push_back(coo[i].col);
        op.wk_code.push_back(coo[i].code);
        op.wk_val.push_back(v);
        i = j;
    }
    if (!op.wk_rows.empty()) op.wk_ptr.push_back(static_cast<int32_t>(op.wk_col.size()));
    for (int a = 0; a < 3; ++a) op.box_len[a] = L[a];
}

}  // namespace dmri
