// Host-only driver of libdmri's C++ mesh and sequence code, built by
// tests/test_host_sanitize.py with AddressSanitizer and UndefinedBehavior-
// Sanitizer (g++, no device code). It feeds caller-style inputs, including
// invalid ones, to dmri::assemble and dmri::make_sequence: a validation
// failure must come back as dmri::Error, never as a memory error.
//
//   host_driver mesh FILE      assemble the mesh in FILE (format below)
//   host_driver seq KIND DT THETA P...   build a sequence
//
// Mesh file (little endian): int64 n_nodes, n_tets, n_comp, has_tensor,
// has_T2, has_u0; uint32 periodic_mask; double kappa, lo[3], hi[3];
// double xyz[n_nodes][3]; int32 tets[n_tets][4]; int32 label[n_tets];
// double D[n_comp] or D_tensor[n_comp][6]; double T2[n_comp] if has_T2;
// double u0[n_comp] if has_u0.
// Prints one line: "ok n_dof nnz sum_M sum_R kappa_e n_slots" / "ok N F_N int_F2"
// or "error CODE MESSAGE".
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1908_01719_amd/csrc/assembly.hpp"
#include "../../paper_1908_01719_amd/csrc/sequence.hpp"

namespace {

template <typename T>
bool rd(FILE* f, T* p, size_t n) {
    return std::fread(p, sizeof(T), n, f) == n;
}

int run_mesh(const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return 2;
    int64_t hdr[6];
    uint32_t mask = 0;
    double kappa = 0, lo[3], hi[3];
    if (!rd(f, hdr, 6) || !rd(f, &mask, 1) || !rd(f, &kappa, 1) || !rd(f, lo, 3) ||
        !rd(f, hi, 3))
        return 3;
    const int64_t nn = hdr[0], nt = hdr[1], nc = hdr[2];
    if (nn < 0 || nt < 0 || nc < 0 || nn > (1 << 26) || nt > (1 << 26) || nc > 1024) return 3;
    std::vector<double> xyz(3 * nn), D(nc * (hdr[3] ? 6 : 1)), T2(nc), u0(nc);
    std::vector<int32_t> tets(4 * nt), label(nt);
    if (!rd(f, xyz.data(), xyz.size()) || !rd(f, tets.data(), tets.size()) ||
        !rd(f, label.data(), label.size()) || !rd(f, D.data(), D.size()))
        return 3;
    if (hdr[4] && !rd(f, T2.data(), T2.size())) return 3;
    if (hdr[5] && !rd(f, u0.data(), u0.size())) return 3;
    std::fclose(f);
    dmri::MeshInput in;
    in.n_nodes = nn;
    in.xyz = xyz.data();
    in.n_tets = nt;
    in.tets = tets.data();
    in.label = label.data();
    in.n_comp = static_cast<int32_t>(nc);
    if (hdr[3]) in.Dt = D.data(); else in.D = D.data();
    in.T2 = hdr[4] ? T2.data() : nullptr;
    in.u0 = hdr[5] ? u0.data() : nullptr;
    in.kappa = kappa;
    for (int a = 0; a < 3; ++a) {
        in.lo[a] = lo[a];
        in.hi[a] = hi[a];
    }
    in.periodic_mask = mask;
    try {
        const dmri::HostOperator op = dmri::assemble(in);
        double sm = 0, sr = 0;
        for (double v : op.M) sm += v;
        for (double v : op.R) sr += v;
        std::printf("ok %lld %lld %.17g %.17g %.17g %zu\n", static_cast<long long>(op.n_dof),
                    static_cast<long long>(op.nnz), sm, sr, op.kappa_e, op.wk_rows.size());
    } catch (const dmri::Error& e) {
        std::printf("error %d %s\n", static_cast<int>(e.code), e.what());
    }
    return 0;
}

int run_seq(int argc, char** argv) {
    const int32_t kind = std::atoi(argv[2]);
    const double dt = std::atof(argv[3]), theta = std::atof(argv[4]);
    std::vector<double> p;
    for (int i = 5; i < argc; ++i) p.push_back(std::atof(argv[i]));
    try {
        const dmri::SequenceTables s =
            dmri::make_sequence(kind, p.data(), static_cast<int32_t>(p.size()), dt, theta);
        std::printf("ok %d %.17g %.17g\n", s.n_steps, s.F.back(), s.int_F2);
    } catch (const dmri::Error& e) {
        std::printf("error %d %s\n", static_cast<int>(e.code), e.what());
    }
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc >= 3 && std::string(argv[1]) == "mesh") return run_mesh(argv[2]);
    if (argc >= 5 && std::string(argv[1]) == "seq") return run_seq(argc, argv);
    std::fprintf(stderr, "usage: host_driver mesh FILE | seq KIND DT THETA P...\n");
    return 2;
}
