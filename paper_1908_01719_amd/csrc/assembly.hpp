// Host-side mesh processing and operator assembly for libdmri.
//
// Builds, once per mesh, the time-independent real sparse operators of the
// P1 / PUFEM discretization (Appendix A, eq. theta_discretization and
// eq. phase_func; Appendix B, eq. loadvec):
//   M   = sum_k int_{Omega_k} phi_i phi_j
//   R   = sum_k D_k int grad phi_i . grad phi_j              (stiffness)
//         + kappa int_Gamma [[phi_i]] [[phi_j]]              (membranes)
//         + sum_k (1/T2_k) int_{Omega_k} phi_i phi_j          (relaxation)
//   M_D = sum_k D_k int_{Omega_k} phi_i phi_j
//   V_a = B_a = sum_k D_k int (phi_i d_a phi_j - phi_j d_a phi_i)   (periodic box)
//   V_a = J_a = sum_k int (x_a - c_a) phi_i phi_j                   (Neumann box)
// on the DOF set "one P1 field per compartment": DOF (k, node) exists iff the
// node touches a tetrahedron of compartment k. Periodic boxes identify the
// nodes of opposite faces (strong pseudo-periodic imposition, Appendix A).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dmri.h"

namespace dmri {

struct Error : std::runtime_error {
    dmri_status code;
    Error(dmri_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum Form : int32_t { FORM_TRANSFORMED = 1, FORM_UFORM = 2 };

struct MeshInput {
    int64_t n_nodes = 0;
    const double* xyz = nullptr;
    int64_t n_tets = 0;
    const int32_t* tets = nullptr;
    const int32_t* label = nullptr;
    int32_t n_comp = 0;
    const double* D = nullptr;
    // Optional diffusion tensors per compartment, [n_comp][6] = xx, yy, zz,
    // xy, xz, yz (symmetric positive definite); D is then ignored.
    const double* Dt = nullptr;
    const double* T2 = nullptr;   // may be null
    const double* u0 = nullptr;   // may be null
    double kappa = 0.0;
    double lo[3] = {0, 0, 0};
    double hi[3] = {0, 0, 0};
    // 0 = Neumann walls, 7 = periodic box (strong), 8 | axes = weak
    // pseudo-periodic faces on those axes (U-form, Appendix B)
    uint32_t periodic_mask = 0;
    // DOF ordering: 0 = Morton (Z-order) of node positions; 1 = pencils:
    // columns of pencil x pencil cells in (x, y), each swept z-, y-, x-major,
    // which bounds the index distance between mesh neighbours by about
    // pencil^2 rows.
    int32_t ordering = 1;
    int32_t pencil = 12;
};

// Assembled operators in the library's DOF order (spatially sorted).
struct HostOperator {
    int32_t form = FORM_TRANSFORMED;
    int64_t n_dof = 0;
    int64_t nnz = 0;
    int32_t n_comp = 0;
    std::vector<int32_t> row_ptr, col, diag_pos;
    std::vector<double> M, R, MD, V[3];
    // Array of the (gamma F)^2 g.Dg mass term on the device: M_D for scalar
    // diffusivities; for tensors the plain mass M, scaled per row by the
    // row's compartment factor q.D_k q (mass entries never join compartments).
    std::vector<double> MT;
    bool aniso = false;
    std::vector<double> comp_tensor;  // [n_comp][6] when aniso
    std::vector<double> w, u0;
    std::vector<int32_t> dof_comp, dof_node;
    std::vector<double> comp_volume;
    double volume = 0.0;
    double interface_area = 0.0;
    int64_t n_torus_nodes = 0;
    int64_t n_interface_faces = 0;
    // Extra per-DOF geometry used by the learned guess features.
    std::vector<float> dof_xyz;      // [n_dof][3] position relative to box centre
    std::vector<float> dof_membrane; // [n_dof] 1 if the node also belongs to another compartment
    std::vector<float> dof_D;        // [n_dof] diffusivity of the DOF's compartment
    // Per tetrahedron (for the signal of the physical field when F(t) != 0):
    // its four DOFs and its vertices' mesh nodes; node positions relative
    // to the box centre.
    std::vector<int32_t> tet_dof;    // [n_tets][4]
    std::vector<int32_t> tet_node;   // [n_tets][4]
    std::vector<double> node_xyz;    // [n_nodes][3]
    double max_edge = 0.0;           // longest tetrahedron edge
    // Weak pseudo-periodic faces (Appendix B; periodic_mask bit 3 with the
    // axes in bits 0-2, U-form, no identification): KB [nnz] the face mass
    // kappa_e <phi_i, phi_j> on the weak faces (empty otherwise); the
    // partner couplings in rows wk_rows (ascending), entries
    // wk_ptr[r]..wk_ptr[r+1] with column wk_col, value wk_val (kappa_e
    // folded in) and wk_code = a (row on the face x_a = lo, phase
    // e^{+i G F q_a L_a}) or 3 + a (row on x_a = hi, phase e^{-i ...}).
    std::vector<double> KB;
    double kappa_e = 0.0;
    std::vector<int32_t> wk_rows, wk_ptr, wk_col, wk_code;
    std::vector<double> wk_val;
    double box_len[3] = {0.0, 0.0, 0.0};
    // Scales of the operator's terms (inputs of the preconditioner's
    // interval network): the largest compartment diffusivity (largest
    // eigenvalue for tensors) and the membrane permeability.
    double d_max = 0.0;
    double kappa = 0.0;
};

// Largest eigenvalue of a symmetric 3x3 matrix (cyclic Jacobi rotations;
// A is overwritten).
double lambda_max(double A[3][3]);

// Fill the weak-face arrays of op (called by assemble once the pattern
// exists); tdof [n_tets][4] holds the DOF of every tetrahedron vertex.
void add_weak_faces(const MeshInput& in, const std::vector<int32_t>& tdof, HostOperator& op);

// Validate the input and assemble. Throws dmri::Error.
HostOperator assemble(const MeshInput& in);

}  // namespace dmri
