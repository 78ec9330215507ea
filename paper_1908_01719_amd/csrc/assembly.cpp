// Host-side mesh processing and operator assembly (see assembly.hpp).
#include "assembly.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace dmri {
namespace {

// Coordinates are matched on a grid of 2^-32 of the box length per axis.
constexpr double kQuant = 4294967296.0;
constexpr int64_t kQuantI = 4294967296LL;

struct Key3 {
    int64_t a, b, c;
    bool operator==(const Key3& o) const { return a == o.a && b == o.b && c == o.c; }
};

struct Key3Hash {
    size_t operator()(const Key3& k) const {
        uint64_t h = static_cast<uint64_t>(k.a) * 0x9E3779B97F4A7C15ULL;
        h ^= static_cast<uint64_t>(k.b) + 0xC2B2AE3D27D4EB4FULL + (h << 6) + (h >> 2);
        h ^= static_cast<uint64_t>(k.c) + 0x165667B19E3779F9ULL + (h << 6) + (h >> 2);
        return static_cast<size_t>(h ^ (h >> 29));
    }
};

// Interleave the low 21 bits of v with two zero bits between each.
uint64_t spread3(uint64_t v) {
    v &= 0x1FFFFF;
    v = (v | v << 32) & 0x1F00000000FFFFULL;
    v = (v | v << 16) & 0x1F0000FF0000FFULL;
    v = (v | v << 8) & 0x100F00F00F00F00FULL;
    v = (v | v << 4) & 0x10C30C30C30C30C3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

inline bool finite(double v) { return std::isfinite(v); }

void fail(dmri_status c, const std::string& m) { throw Error(c, m); }

struct Vec3 {
    double x, y, z;
};
inline Vec3 sub(const double* a, const double* b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline Vec3 cross(const Vec3& a, const Vec3& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double dot(const Vec3& a, const Vec3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(const Vec3& a) { return std::sqrt(dot(a, a)); }

}  // namespace

HostOperator assemble(const MeshInput& in) {
    // ---------------------------------------------------------------- checks
    if (in.n_nodes < 4 || in.n_tets < 1 || in.n_comp < 1)
        fail(DMRI_E_INVALID, "need n_nodes >= 4, n_tets >= 1, n_comp >= 1");
    if (!in.xyz || !in.tets || !in.label || (!in.D && !in.Dt))
        fail(DMRI_E_INVALID, "xyz, tets, tet_label and D must not be NULL");
    if (in.n_nodes > (int64_t(1) << 31) - 1 || in.n_tets > (int64_t(1) << 31) / 4)
        fail(DMRI_E_INVALID, "mesh too large for 32-bit indices");
    const bool weak = (in.periodic_mask & 8u) != 0;
    if (weak ? (in.periodic_mask > 15u || (in.periodic_mask & 7u) == 0)
             : (in.periodic_mask != 0 && in.periodic_mask != 7))
        fail(DMRI_E_UNSUPPORTED,
             "periodic_mask must be 0 (Neumann walls), 7 (periodic box) or 8 plus the "
             "weakly periodic axes (bits 0-2)");
    if (!finite(in.kappa) || in.kappa < 0) fail(DMRI_E_INVALID, "kappa must be finite and >= 0");
    for (int a = 0; a < 3; ++a)
        if (!finite(in.lo[a]) || !finite(in.hi[a]) || !(in.lo[a] < in.hi[a]))
            fail(DMRI_E_INVALID, "box_lo < box_hi must hold on every axis");
    for (int32_t k = 0; k < in.n_comp; ++k) {
        if (in.Dt) {
            const double* t = in.Dt + 6 * k;
            for (int c = 0; c < 6; ++c)
                if (!finite(t[c])) fail(DMRI_E_INVALID, "diffusion tensors must be finite");
            // positive definite: leading principal minors (Sylvester)
            const double m1 = t[0], m2 = t[0] * t[1] - t[3] * t[3];
            const double m3 = t[0] * (t[1] * t[2] - t[5] * t[5]) - t[3] * (t[3] * t[2] - t[5] * t[4]) +
                              t[4] * (t[3] * t[5] - t[1] * t[4]);
            if (!(m1 > 0) || !(m2 > 0) || !(m3 > 0))
                fail(DMRI_E_INVALID, "diffusion tensors must be positive definite");
        } else if (!finite(in.D[k]) || in.D[k] <= 0) {
            fail(DMRI_E_INVALID, "D must be finite and > 0");
        }
        if (in.T2 && (!finite(in.T2[k]) || in.T2[k] <= 0))
            fail(DMRI_E_INVALID, "T2 must be finite and > 0");
        if (in.u0 && !finite(in.u0[k])) fail(DMRI_E_INVALID, "u0 must be finite");
    }
    const int64_t nN = in.n_nodes, nT = in.n_tets;
    for (int64_t i = 0; i < 3 * nN; ++i)
        if (!finite(in.xyz[i])) fail(DMRI_E_INVALID, "node coordinates must be finite");
    for (int64_t e = 0; e < nT; ++e) {
        for (int v = 0; v < 4; ++v) {
            int32_t id = in.tets[4 * e + v];
            if (id < 0 || id >= nN) fail(DMRI_E_INVALID, "tetrahedron node index out of range");
        }
        if (in.label[e] < 0 || in.label[e] >= in.n_comp)
            fail(DMRI_E_INVALID, "tet_label out of range");
    }

    HostOperator op;
    op.form = in.periodic_mask == 7 ? FORM_TRANSFORMED : FORM_UFORM;
    // strong identification of opposite faces (weak faces stay apart)
    const uint32_t ident = weak ? 0u : in.periodic_mask;
    op.n_comp = in.n_comp;
    const double L[3] = {in.hi[0] - in.lo[0], in.hi[1] - in.lo[1], in.hi[2] - in.lo[2]};
    const double centre[3] = {0.5 * (in.lo[0] + in.hi[0]), 0.5 * (in.lo[1] + in.hi[1]),
                              0.5 * (in.lo[2] + in.hi[2])};

    // --------------------------------------------- periodic identification
    std::vector<uint8_t> used(nN, 0);
    for (int64_t i = 0; i < 4 * nT; ++i) used[in.tets[i]] = 1;
    std::vector<std::array<int64_t, 3>> qk(nN);
    for (int64_t n = 0; n < nN; ++n) {
        for (int a = 0; a < 3; ++a) {
            double r = (in.xyz[3 * n + a] - in.lo[a]) / L[a];
            qk[n][a] = std::llround(r * kQuant);
        }
    }
    for (int a = 0; a < 3; ++a) {
        if (!(ident >> a & 1)) continue;
        const int b = (a + 1) % 3, c = (a + 2) % 3;
        std::vector<std::pair<int64_t, int64_t>> lo_face, hi_face;
        for (int64_t n = 0; n < nN; ++n) {
            if (!used[n]) continue;
            if (qk[n][a] < 0 || qk[n][a] > kQuantI)
                fail(DMRI_E_INVALID, "node outside the periodic box");
            if (qk[n][a] == 0) lo_face.push_back({qk[n][b], qk[n][c]});
            if (qk[n][a] == kQuantI) hi_face.push_back({qk[n][b], qk[n][c]});
        }
        std::sort(lo_face.begin(), lo_face.end());
        lo_face.erase(std::unique(lo_face.begin(), lo_face.end()), lo_face.end());
        std::sort(hi_face.begin(), hi_face.end());
        hi_face.erase(std::unique(hi_face.begin(), hi_face.end()), hi_face.end());
        // Edge/corner nodes wrap along other axes too; compare wrapped keys.
        auto wrap = [&](std::vector<std::pair<int64_t, int64_t>>& v) {
            for (auto& p : v) {
                if ((ident >> b & 1) && p.first == kQuantI) p.first = 0;
                if ((ident >> c & 1) && p.second == kQuantI) p.second = 0;
            }
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
        };
        wrap(lo_face);
        wrap(hi_face);
        if (lo_face.empty() || lo_face != hi_face)
            fail(DMRI_E_INVALID, "periodic box: opposite faces do not match node for node");
    }
    for (int64_t n = 0; n < nN; ++n)
        for (int a = 0; a < 3; ++a)
            if ((ident >> a & 1) && qk[n][a] == kQuantI) qk[n][a] = 0;

    std::unordered_map<Key3, int64_t, Key3Hash> tmap;
    tmap.reserve(static_cast<size_t>(nN * 1.3) + 16);
    std::vector<int64_t> tnode(nN, -1);
    std::vector<int32_t> rep;  // representative (lowest) mesh node per torus node
    std::vector<std::array<int64_t, 3>> tkey;
    for (int64_t n = 0; n < nN; ++n) {
        if (!used[n]) continue;
        Key3 k{qk[n][0], qk[n][1], qk[n][2]};
        auto it = tmap.find(k);
        if (it == tmap.end()) {
            int64_t id = static_cast<int64_t>(rep.size());
            tmap.emplace(k, id);
            rep.push_back(static_cast<int32_t>(n));
            tkey.push_back(qk[n]);
            tnode[n] = id;
        } else {
            tnode[n] = it->second;
        }
    }
    const int64_t nTor = static_cast<int64_t>(rep.size());
    op.n_torus_nodes = nTor;

    // Spatial order of torus nodes: consecutive DOFs are mesh neighbours.
    std::vector<int64_t> rank(nTor);
    {
        std::vector<std::pair<uint64_t, int64_t>> code(nTor);
        if (in.ordering == 0) {
            for (int64_t t = 0; t < nTor; ++t) {
                uint64_t c = spread3(static_cast<uint64_t>(tkey[t][0]) >> 11) |
                             spread3(static_cast<uint64_t>(tkey[t][1]) >> 11) << 1 |
                             spread3(static_cast<uint64_t>(tkey[t][2]) >> 11) << 2;
                code[t] = {c, t};
            }
        } else {
            // Cell size estimate: mean edge length of (up to) 4096 tetrahedra.
            double hsum = 0.0;
            int64_t hn = 0;
            const int64_t stride = std::max<int64_t>(1, nT / 4096);
            for (int64_t e = 0; e < nT; e += stride) {
                const int32_t* tv = in.tets + 4 * e;
                for (int a = 0; a < 4; ++a)
                    for (int b = a + 1; b < 4; ++b) {
                        hsum += norm(sub(in.xyz + 3 * tv[a], in.xyz + 3 * tv[b]));
                        ++hn;
                    }
            }
            // A Kuhn cube of edge h splits into tetrahedra whose six edges are
            // h, h, h, sqrt2 h, sqrt2 h, sqrt3 h (mean 1.26 h); for other meshes
            // any estimate of the right order serves the ordering.
            const double h = std::max(1e-300, hsum / std::max<int64_t>(1, hn) / 1.26008);
            const int64_t w = std::max<int32_t>(1, in.pencil);
            for (int64_t t = 0; t < nTor; ++t) {
                uint64_t gxyz[3];
                for (int a = 0; a < 3; ++a) {
                    double gv = (tkey[t][a] / kQuant) * L[a] / h;
                    int64_t gi = std::llround(gv);
                    gi = std::min<int64_t>(std::max<int64_t>(gi, 0), (1 << 12) - 1);
                    gxyz[a] = static_cast<uint64_t>(gi);
                }
                const uint64_t bx = gxyz[0] / w, by = gxyz[1] / w;
                const uint64_t c = (by << 44) | (bx << 36) | (gxyz[2] << 24) | (gxyz[1] << 12) |
                                   gxyz[0];
                code[t] = {c, t};
            }
        }
        std::sort(code.begin(), code.end());
        for (int64_t r = 0; r < nTor; ++r) rank[code[r].second] = r;
    }

    // ----------------------------------------------------------- PUFEM DOFs
    std::vector<uint64_t> pairs;
    pairs.reserve(static_cast<size_t>(4 * nT));
    for (int64_t e = 0; e < nT; ++e) {
        uint64_t k = static_cast<uint64_t>(in.label[e]);
        for (int v = 0; v < 4; ++v)
            pairs.push_back(static_cast<uint64_t>(rank[tnode[in.tets[4 * e + v]]]) << 20 | k);
    }
    if (in.n_comp >= (1 << 20)) fail(DMRI_E_INVALID, "too many compartments");
    std::sort(pairs.begin(), pairs.end());
    pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
    const int64_t nD = static_cast<int64_t>(pairs.size());
    if (nD > (int64_t(1) << 31) - 1) fail(DMRI_E_INVALID, "too many DOFs");
    op.n_dof = nD;
    std::vector<int64_t> dstart(nTor + 1, 0);
    for (uint64_t p : pairs) dstart[(p >> 20) + 1]++;
    for (int64_t r = 0; r < nTor; ++r) dstart[r + 1] += dstart[r];
    std::vector<int64_t> rank_to_t(nTor);
    for (int64_t t = 0; t < nTor; ++t) rank_to_t[rank[t]] = t;
    op.dof_comp.resize(nD);
    op.dof_node.resize(nD);
    op.dof_xyz.resize(3 * nD);
    op.dof_membrane.resize(nD);
    for (int64_t d = 0; d < nD; ++d) {
        int64_t r = static_cast<int64_t>(pairs[d] >> 20);
        int64_t t = rank_to_t[r];
        op.dof_comp[d] = static_cast<int32_t>(pairs[d] & 0xFFFFF);
        op.dof_node[d] = rep[t];
        for (int a = 0; a < 3; ++a)
            op.dof_xyz[3 * d + a] =
                static_cast<float>(in.lo[a] + L[a] * (tkey[t][a] / kQuant) - centre[a]);
        op.dof_membrane[d] = (dstart[r + 1] - dstart[r] > 1) ? 1.0f : 0.0f;
    }
    auto dof_of = [&](int64_t t, int32_t k) -> int32_t {
        int64_t r = rank[t];
        for (int64_t d = dstart[r]; d < dstart[r + 1]; ++d)
            if (static_cast<int32_t>(pairs[d] & 0xFFFFF) == k) return static_cast<int32_t>(d);
        throw Error(DMRI_E_INVALID, "internal: missing DOF");
    };

    // Per-tet DOFs; reject tets whose vertices collapse under identification.
    std::vector<int32_t> tdof(static_cast<size_t>(4 * nT));
    for (int64_t e = 0; e < nT; ++e) {
        int64_t t4[4];
        for (int v = 0; v < 4; ++v) t4[v] = tnode[in.tets[4 * e + v]];
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b)
                if (t4[a] == t4[b])
                    fail(DMRI_E_INVALID,
                         "a tetrahedron has two vertices identified by periodicity "
                         "(the mesh needs at least 2 cells per periodic axis)");
        for (int v = 0; v < 4; ++v) tdof[4 * e + v] = dof_of(t4[v], in.label[e]);
    }

    // ------------------------------------------------------ interface faces
    static const int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    struct FaceRec {
        int64_t k0, k1, k2;
        int64_t tet;
        int32_t local;
        bool operator<(const FaceRec& o) const {
            if (k0 != o.k0) return k0 < o.k0;
            if (k1 != o.k1) return k1 < o.k1;
            if (k2 != o.k2) return k2 < o.k2;
            return tet < o.tet;
        }
    };
    std::vector<FaceRec> cand;
    for (int64_t e = 0; e < nT; ++e) {
        for (int f = 0; f < 4; ++f) {
            int64_t r[3];
            bool multi = true;
            for (int i = 0; i < 3; ++i) {
                int64_t t = tnode[in.tets[4 * e + kFace[f][i]]];
                r[i] = rank[t];
                if (dstart[r[i] + 1] - dstart[r[i]] < 2) multi = false;
            }
            if (!multi) continue;
            std::sort(r, r + 3);
            cand.push_back({r[0], r[1], r[2], e, f});
        }
    }
    std::sort(cand.begin(), cand.end());
    struct IFace {
        int32_t da[3], db[3];
        double area;
    };
    std::vector<IFace> ifaces;
    for (size_t i = 0; i < cand.size();) {
        size_t j = i + 1;
        while (j < cand.size() && cand[j].k0 == cand[i].k0 && cand[j].k1 == cand[i].k1 &&
               cand[j].k2 == cand[i].k2)
            ++j;
        if (j - i > 2) fail(DMRI_E_INVALID, "non-manifold mesh: a face shared by >2 tetrahedra");
        if (j - i == 2) {
            const FaceRec& A = cand[i];
            const FaceRec& B = cand[i + 1];
            int32_t ka = in.label[A.tet], kb = in.label[B.tet];
            if (ka != kb) {
                IFace fc;
                const double* p[3];
                for (int v = 0; v < 3; ++v) {
                    int32_t node = in.tets[4 * A.tet + kFace[A.local][v]];
                    p[v] = in.xyz + 3 * node;
                    int64_t t = tnode[node];
                    fc.da[v] = dof_of(t, ka);
                    fc.db[v] = dof_of(t, kb);
                }
                fc.area = 0.5 * norm(cross(sub(p[1], p[0]), sub(p[2], p[0])));
                ifaces.push_back(fc);
            }
        }
        i = j;
    }
    op.n_interface_faces = static_cast<int64_t>(ifaces.size());

    // ------------------------------------------------------------ CSR pattern
    std::vector<int64_t> cnt(nD + 1, 0);
    for (int64_t e = 0; e < nT; ++e)
        for (int v = 0; v < 4; ++v) cnt[tdof[4 * e + v] + 1] += 4;
    for (const IFace& f : ifaces)
        for (int v = 0; v < 3; ++v) {
            cnt[f.da[v] + 1] += 3;
            cnt[f.db[v] + 1] += 3;
        }
    for (int64_t d = 0; d < nD; ++d) cnt[d + 1] += cnt[d];
    std::vector<int32_t> raw(static_cast<size_t>(cnt[nD]));
    {
        std::vector<int64_t> fillp(cnt.begin(), cnt.end() - 1);
        for (int64_t e = 0; e < nT; ++e)
            for (int i = 0; i < 4; ++i) {
                int32_t r = tdof[4 * e + i];
                for (int j = 0; j < 4; ++j) raw[fillp[r]++] = tdof[4 * e + j];
            }
        for (const IFace& f : ifaces)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    raw[fillp[f.da[i]]++] = f.db[j];
                    raw[fillp[f.db[i]]++] = f.da[j];
                }
    }
    op.row_ptr.assign(nD + 1, 0);
    op.col.clear();
    op.col.reserve(static_cast<size_t>(16 * nD));
    for (int64_t d = 0; d < nD; ++d) {
        auto b = raw.begin() + cnt[d], e = raw.begin() + cnt[d + 1];
        std::sort(b, e);
        auto u = std::unique(b, e);
        op.col.insert(op.col.end(), b, u);
        op.row_ptr[d + 1] = static_cast<int32_t>(op.col.size());
        if (op.col.size() > static_cast<size_t>((int64_t(1) << 31) - 1))
            fail(DMRI_E_INVALID, "too many nonzeros for 32-bit indices");
    }
    raw.clear();
    raw.shrink_to_fit();
    const int64_t nnz = static_cast<int64_t>(op.col.size());
    op.nnz = nnz;
    op.M.assign(nnz, 0.0);
    op.R.assign(nnz, 0.0);
    op.MD.assign(nnz, 0.0);
    for (int a = 0; a < 3; ++a) op.V[a].assign(nnz, 0.0);
    op.w.assign(nD, 0.0);
    op.comp_volume.assign(in.n_comp, 0.0);
    op.diag_pos.resize(nD);
    auto pos = [&](int32_t r, int32_t c) -> int64_t {
        const int32_t* b = op.col.data() + op.row_ptr[r];
        const int32_t* e = op.col.data() + op.row_ptr[r + 1];
        const int32_t* p = std::lower_bound(b, e, c);
        return p - op.col.data();
    };
    for (int64_t d = 0; d < nD; ++d) op.diag_pos[d] = static_cast<int32_t>(pos(d, d));

    // ------------------------------------------------------- element values
    for (int64_t e = 0; e < nT; ++e) {
        const int32_t* tv = in.tets + 4 * e;
        const double* v[4] = {in.xyz + 3 * tv[0], in.xyz + 3 * tv[1], in.xyz + 3 * tv[2],
                              in.xyz + 3 * tv[3]};
        Vec3 e1 = sub(v[1], v[0]), e2 = sub(v[2], v[0]), e3 = sub(v[3], v[0]);
        double det = dot(e1, cross(e2, e3));
        double hbar = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) hbar += norm(sub(v[a], v[b]));
        hbar /= 6.0;
        double vol = std::fabs(det) / 6.0;
        if (!(vol >= 1e-12 * hbar * hbar * hbar)) fail(DMRI_E_INVALID, "degenerate tetrahedron");
        Vec3 g[4];
        g[1] = cross(e2, e3);
        g[2] = cross(e3, e1);
        g[3] = cross(e1, e2);
        for (int a = 1; a < 4; ++a) g[a] = {g[a].x / det, g[a].y / det, g[a].z / det};
        g[0] = {-(g[1].x + g[2].x + g[3].x), -(g[1].y + g[2].y + g[3].y),
                -(g[1].z + g[2].z + g[3].z)};
        const int32_t k = in.label[e];
        // D as a 3x3 matrix (a scalar times the identity without tensors)
        double Dm[3][3];
        if (in.Dt) {
            const double* t = in.Dt + 6 * k;
            Dm[0][0] = t[0]; Dm[1][1] = t[1]; Dm[2][2] = t[2];
            Dm[0][1] = Dm[1][0] = t[3];
            Dm[0][2] = Dm[2][0] = t[4];
            Dm[1][2] = Dm[2][1] = t[5];
        } else {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Dm[a][b] = a == b ? in.D[k] : 0.0;
        }
        const double Dk = in.Dt ? (Dm[0][0] + Dm[1][1] + Dm[2][2]) / 3.0 : in.D[k];  // trace/3
        Vec3 Dg[4];  // D grad lambda_i
        for (int i = 0; i < 4; ++i)
            Dg[i] = {Dm[0][0] * g[i].x + Dm[0][1] * g[i].y + Dm[0][2] * g[i].z,
                     Dm[1][0] * g[i].x + Dm[1][1] * g[i].y + Dm[1][2] * g[i].z,
                     Dm[2][0] * g[i].x + Dm[2][1] * g[i].y + Dm[2][2] * g[i].z};
        const double r2 = in.T2 ? 1.0 / in.T2[k] : 0.0;
        op.comp_volume[k] += vol;
        double xs[4][3];
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) xs[a][c] = v[a][c] - centre[c];
        double xsum[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) xsum[c] += xs[a][c];
        const int32_t* d = tdof.data() + 4 * e;
        for (int i = 0; i < 4; ++i) {
            op.w[d[i]] += 0.25 * vol;
            const double gi[3] = {g[i].x, g[i].y, g[i].z};
            for (int j = 0; j < 4; ++j) {
                const double gj[3] = {g[j].x, g[j].y, g[j].z};
                const int64_t p = pos(d[i], d[j]);
                const double mass = vol * (i == j ? 2.0 : 1.0) / 20.0;
                op.M[p] += mass;
                op.MD[p] += Dk * mass;
                // grad phi_i . D grad phi_j
                op.R[p] += vol * dot(g[i], Dg[j]) + r2 * mass;
                const double Dgi[3] = {Dg[i].x, Dg[i].y, Dg[i].z};
                const double Dgj[3] = {Dg[j].x, Dg[j].y, Dg[j].z};
                for (int c = 0; c < 3; ++c) {
                    // (phi_i (D q).grad phi_j - phi_j (D q).grad phi_i) per q_c
                    if (op.form == FORM_TRANSFORMED)
                        op.V[c][p] += vol * (Dgj[c] - Dgi[c]) * 0.25;
                    else
                        op.V[c][p] += vol * (i == j ? 2.0 : 1.0) / 120.0 *
                                      (xsum[c] + xs[i][c] + xs[j][c]);
                }
            }
        }
    }
    // ------------------------------------------------------ membrane terms
    double area_total = 0.0;
    for (const IFace& f : ifaces) {
        area_total += f.area;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double m = in.kappa * f.area * (i == j ? 2.0 : 1.0) / 12.0;
                op.R[pos(f.da[i], f.da[j])] += m;
                op.R[pos(f.db[i], f.db[j])] += m;
                op.R[pos(f.da[i], f.db[j])] -= m;
                op.R[pos(f.db[i], f.da[j])] -= m;
            }
    }
    op.interface_area = area_total;
    op.u0.resize(nD);
    op.dof_D.resize(nD);
    for (int64_t dd = 0; dd < nD; ++dd) {
        const int32_t k = op.dof_comp[dd];
        op.u0[dd] = in.u0 ? in.u0[k] : 1.0;
        op.dof_D[dd] = static_cast<float>(
            in.Dt ? (in.Dt[6 * k] + in.Dt[6 * k + 1] + in.Dt[6 * k + 2]) / 3.0 : in.D[k]);
    }
    op.aniso = in.Dt != nullptr;
    if (op.aniso) {
        op.MT = op.M;
        op.comp_tensor.assign(in.Dt, in.Dt + 6 * in.n_comp);
    } else {
        op.MT = op.MD;
    }
    op.volume = 0.0;
    for (double v : op.comp_volume) op.volume += v;
    // Geometry of the tetrahedra for the phase-weighted signal.
    op.tet_dof = tdof;
    op.tet_node.assign(in.tets, in.tets + 4 * nT);
    op.node_xyz.resize(static_cast<size_t>(3 * in.n_nodes));
    for (int64_t i = 0; i < in.n_nodes; ++i)
        for (int a = 0; a < 3; ++a) op.node_xyz[3 * i + a] = in.xyz[3 * i + a] - centre[a];
    double emax = 0.0;
    for (int64_t e = 0; e < nT; ++e) {
        const int32_t* tv = in.tets + 4 * e;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                double l2 = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double d = in.xyz[3 * tv[a] + c] - in.xyz[3 * tv[b] + c];
                    l2 += d * d;
                }
                emax = std::max(emax, l2);
            }
    }
    op.max_edge = std::sqrt(emax);
    op.kappa = in.kappa;
    for (int32_t k = 0; k < in.n_comp; ++k) {
        double dk = in.Dt ? 0.0 : in.D[k];
        if (in.Dt) {
            const double* t = in.Dt + 6 * k;
            double A[3][3] = {{t[0], t[3], t[4]}, {t[3], t[1], t[5]}, {t[4], t[5], t[2]}};
            dk = lambda_max(A);
        }
        op.d_max = std::max(op.d_max, dk);
    }
    if (weak) add_weak_faces(in, tdof, op);
    return op;
}

}  // namespace dmri
