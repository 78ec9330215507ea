/*
 * dmri.h -- C ABI of libdmri: finite-element Bloch-Torrey simulation of the
 * diffusion MRI signal on one AMD Instinct MI355X (gfx950).
 *
 * The library computes, for every (b-value, gradient direction) pair, the
 * complex signal S = int_Omega U(x, T) dx at echo time T (Sec. 2, eq. signal)
 * of the Bloch-Torrey equation (Sec. 2, eq. strong_BT) with permeable
 * membranes between compartments (Sec. 2, eq. btpde_ic), discretized with P1
 * tetrahedra, one field per compartment (Appendix A, eq. phase_func) and the
 * theta-method in time (Appendix A, eq. theta_discretization; Appendix B,
 * eq. matrix_form). Boxes that are periodic along every axis use the strong
 * imposition of the pseudo-periodic conditions of Sec. 2 (eq. btpde_bc)
 * through the transformation of Appendix A (eq. trBlo); boxes with walls use
 * homogeneous Neumann conditions (Sec. 2) on the untransformed U-form of
 * Appendix B (eq. loadvec). The gradient profile is the PGSE sequence of
 * Sec. 2 (eq. pgse); b and the gradient strength are related by
 * eq. b_value.
 *
 * Units: micrometres and microseconds throughout. D in um^2/us (== mm^2/s),
 * b in us/um^2 (== s/mm^2), kappa in um/us (== m/s), T2 in us, signals in
 * um^3 (volume-weighted magnetization).
 *
 * Conventions
 *  - Every function returns a dmri_status; the library never aborts and no
 *    C++ exception crosses this interface. dmri_last_error() gives the text
 *    of the last failure on a handle.
 *  - All input arrays are owned by the caller and are copied (or fully
 *    consumed) before the call returns. Outputs go to caller-allocated
 *    buffers. A handle owns every device allocation it makes until
 *    dmri_destroy().
 *  - One handle per host thread at a time; several handles may coexist.
 *  - Sizes are int64_t, mesh indices int32_t (0-based), reals double.
 */
#ifndef DMRI_H
#define DMRI_H

#include <stdint.h>

/* Every entry point below is exported from libdmri.so; the library is built
 * with hidden default visibility, so nothing else is. */
#define DMRI_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmri_ctx* dmri_handle;

typedef enum {
    DMRI_OK = 0,
    DMRI_NOT_CONVERGED = 1,   /* warning: results written, some systems hit max_iter */
    DMRI_E_INVALID = -1,      /* bad argument (NaN/Inf, out of range, degenerate mesh...) */
    DMRI_E_STATE = -2,        /* call out of order (no sequence, no device, bad id) */
    DMRI_E_NOMEM = -3,        /* host or device allocation failed */
    DMRI_E_DEVICE = -4,       /* HIP runtime error */
    DMRI_E_UNSUPPORTED = -5   /* valid request this build does not implement */
} dmri_status;

/* Per-run statistics. Array members are caller-owned, length n_sys (the
 * n_pairs of the run), and may be NULL. Scalars are always written. The
 * first seven members are the minimal set (sizes, per-system results, the
 * three wall times); the rest are work counters and kernel timing. */
typedef struct {
    int64_t  n_sys;
    int32_t* iters_total;     /* Krylov iterations summed over all time steps */
    uint8_t* converged;       /* 1 if every step reached rtol */
    double*  final_rel_res;   /* ||r|| / ||b|| of the last step */
    double   t_setup_s;       /* host+device set-up inside the run */
    double   t_solve_s;       /* time loop */
    double   t_signal_s;      /* signal quadrature and copy-out */
    int64_t  total_iterations;/* sum over systems and steps */
    int64_t  spmv_rows;       /* matrix rows applied (all systems), work counter */
    int64_t  n_steps;         /* time steps taken */
    int64_t  n_kernel_launches; /* launches of the kernel chosen by option "time_kernel" */
    double   t_kernel_s;      /* their summed durations (HIP events on the run's stream) */
} dmri_stats;

/* Create a context on HIP device `device_ordinal`. device_ordinal = -1
 * creates a host-only context: problems can be added and their assembled
 * operators exported (dmri_export_operator), but dmri_run* return
 * DMRI_E_STATE. On failure *out is NULL and dmri_last_error(NULL) has the
 * reason. */
DMRI_API dmri_status dmri_create(int device_ordinal, dmri_handle* out);

/* Free every host and device resource of h. NULL-safe. */
DMRI_API void dmri_destroy(dmri_handle h);

/* Text of the last error on h (or of the last failed dmri_create for
 * h == NULL). Valid until the next call on h. Never NULL. */
DMRI_API const char* dmri_last_error(dmri_handle h);

/* Add one mesh with its compartments (Sec. 2: compartments Omega_k with
 * diffusivity D_k, relaxation T2_k, permeability kappa on the interfaces
 * Gamma; Sec. 3 "Initial conditions" per compartment).
 *   xyz        [n_nodes][3] node coordinates
 *   tets       [n_tets][4] node indices (any orientation)
 *   tet_label  [n_tets] compartment of each tetrahedron, in [0, n_comp)
 *   D          [n_comp] > 0
 *   T2         [n_comp] > 0, or NULL for no relaxation
 *   u0         [n_comp] initial magnetization per compartment, or NULL (1)
 *   kappa      >= 0, applied on every face between different labels
 *   box_lo/hi  the box Omega = [lo, hi] (lo < hi on every axis)
 *   periodic_mask  7 = periodic along x, y and z: pseudo-periodic
 *              conditions imposed strongly (Appendix A); opposite faces must
 *              match node for node. 0 = homogeneous Neumann walls (U-form,
 *              Appendix B). 8 + axes (9..15, bit a = axis a): pseudo-periodic
 *              conditions imposed weakly on those axes by an artificial
 *              permeability (Appendix B, eq. bjump1, eq. bjump2,
 *              eq. weak_periodic, forms a* and L*), U-form, other axes
 *              Neumann walls. Opposite faces need not match: the coupling
 *              integrals are exact over the overlaps of face triangles.
 *              kappa_e = max{D / h}, the largest lambda_max(D_k) / h_e over
 *              the tetrahedra with a face on a weak face (h_e the longest
 *              edge), times option "weak_kappa"; runs need theta = 1/2.
 *              Other values: DMRI_E_UNSUPPORTED.
 * Interior interfaces are found from the labels: a face shared by two
 * tetrahedra with different labels carries the kappa jump term.
 * Validation (DMRI_E_INVALID): non-finite values, D <= 0, T2 <= 0,
 * kappa < 0, a label or node index out of range, a degenerate tetrahedron
 * (|volume| < 1e-12 h^3 with h the mean edge length), a periodic face that
 * does not match its opposite face, a weakly periodic box face not fully
 * covered by mesh faces.
 * On success *problem_id receives the new id (0, 1, ...). */
DMRI_API dmri_status dmri_add_problem(dmri_handle h,
                             int64_t n_nodes, const double* xyz,
                             int64_t n_tets, const int32_t* tets,
                             const int32_t* tet_label, int32_t n_comp,
                             const double* D, const double* T2, const double* u0,
                             double kappa,
                             const double box_lo[3], const double box_hi[3],
                             uint32_t periodic_mask,
                             int32_t* problem_id);

/* Same as dmri_add_problem with an intrinsic diffusion tensor per
 * compartment (Sec. 2: D(x) symmetric positive definite; Sec. 3, "Diffusion
 * coefficients and tensors": cell-based, piecewise constant per partition
 * marker, i.e. per compartment here):
 *   D_tensor [n_comp][6] = D_xx, D_yy, D_zz, D_xy, D_xz, D_yz (um^2/us)
 * The stiffness takes grad phi_i . D_k grad phi_j, the transformed form's
 * first-order term (D_k q) . grad and its mass term (gamma F)^2 q . D_k q
 * (Appendix A, eq. trBlo); the U-form is unchanged apart from the
 * stiffness. Validation as dmri_add_problem, plus DMRI_E_INVALID for a
 * tensor that is not positive definite (leading principal minors). The
 * exported M_D (dmri_export_operator) holds trace(D_k)/3 times the mass;
 * dmri_apply_operator's c then multiplies the plain mass matrix. */
DMRI_API dmri_status dmri_add_problem_tensor(dmri_handle h,
                             int64_t n_nodes, const double* xyz,
                             int64_t n_tets, const int32_t* tets,
                             const int32_t* tet_label, int32_t n_comp,
                             const double* D_tensor, const double* T2, const double* u0,
                             double kappa,
                             const double box_lo[3], const double box_hi[3],
                             uint32_t periodic_mask,
                             int32_t* problem_id);

/* Number of DOFs (one per compartment touching a node, after periodic
 * identification) and stored nonzeros of problem `problem_id`. */
DMRI_API dmri_status dmri_problem_info(dmri_handle h, int32_t problem_id,
                              int64_t* n_dof, int64_t* nnz);

/* Copy the assembled real operators of a problem (host data, no device).
 * Every output pointer may be NULL to skip it.
 *   row_ptr [n_dof+1], col [nnz]: CSR pattern shared by every array
 *   vals    [6][nnz]: M (mass), R (stiffness + interface + relaxation),
 *           M_D (D-weighted mass), V_x, V_y, V_z, where V is the skew
 *           first-order operator B of Appendix A (periodic boxes) or the
 *           x-weighted mass J of Appendix B (Neumann boxes, x measured
 *           from the box centre)
 *   w       [n_dof] signal weights int phi_i over its compartment
 *   u0      [n_dof] initial magnetization per DOF
 *   dof_comp [n_dof] compartment, dof_node [n_dof] a mesh node of the DOF
 *           (the lowest-index node among periodically identified copies). */
DMRI_API dmri_status dmri_export_operator(dmri_handle h, int32_t problem_id,
                                 int32_t* row_ptr, int32_t* col, double* vals,
                                 double* w, double* u0,
                                 int32_t* dof_comp, int32_t* dof_node);

/* Weak pseudo-periodic faces of a problem (periodic_mask 9..15; host
 * data). *n_slots receives the number of DOFs on a weak face, *n_entries
 * the number of coupling entries, *kappa_e the artificial permeability
 * (before the "weak_kappa" scale); both are 0 for other problems. Arrays
 * (each may be NULL):
 *   rows [n_slots]       DOF of each slot, ascending
 *   ptr  [n_slots + 1]   entries of slot s: ptr[s] .. ptr[s+1]
 *   col, code, val [n_entries]: partner DOF, code and
 *        kappa_e int_{face} phi_row(x) phi_col(x +- L_a e_a) dx;
 *        code a in 0..2: the row lies on the face x_a = lo_a and the
 *        partner term carries e^{+i G F q_a L_a}; code 3 + a: the row lies
 *        on x_a = hi_a, phase e^{-i G F q_a L_a} (Appendix B, theta_ms =
 *        -theta_sm = gamma g.(x_s - x_m) F)
 *   face_mass [nnz]      kappa_e <phi_i, phi_j> over the weak faces on the
 *        CSR pattern of dmri_export_operator (added with theta to the
 *        left operator only). */
DMRI_API dmri_status dmri_export_weak(dmri_handle h, int32_t problem_id, int64_t* n_slots,
                             int64_t* n_entries, double* kappa_e, int32_t* rows,
                             int32_t* ptr, int32_t* col, int32_t* code, double* val,
                             double* face_mass);

/* PGSE sequence (Sec. 2, eq. pgse) with pulse length delta and pulse
 * spacing Delta (us), fixed time step dt (us) and theta in [1/2, 1]
 * (theta = 1/2 is Crank-Nicolson). The echo time is T = Delta + delta.
 * delta/dt and Delta/dt must be integers (within 1e-9) so pulse edges
 * fall on the grid; 0 < delta <= Delta. */
DMRI_API dmri_status dmri_set_sequence_pgse(dmri_handle h, double delta_us, double Delta_us,
                                   double dt_us, double theta);

/* General temporal profiles f(t) (Sec. 3, "General diffusion-encoding
 * sequence", which defines cos-OGSE; Sec. 4, which compares PGSE, double
 * PGSE, cos-OGSE, sin-OGSE, trapezoidal and double trapezoidal profiles).
 * All times in us; lobes of sign +1 then -1:
 *   DMRI_SEQ_PGSE           {delta, Delta}: as dmri_set_sequence_pgse
 *   DMRI_SEQ_DOUBLE_PGSE    {delta, Delta, t_mix}: a PGSE, t_mix, a PGSE;
 *                           T = 2 (Delta + delta) + t_mix
 *   DMRI_SEQ_COS_OGSE       {delta, Delta, n}: cos(w t) on [0, delta],
 *                           -cos(w (t - tau)) on (tau, tau + delta],
 *                           w = 2 n pi / delta, tau = (delta + Delta) / 2,
 *                           n >= 1 whole periods; T = delta + Delta
 *   DMRI_SEQ_SIN_OGSE       {delta, Delta, n}: the same with sin
 *   DMRI_SEQ_TRAP_PGSE      {delta, Delta, ramp}: PGSE pulses of length delta
 *                           with linear ramps of length ramp (0 < ramp <=
 *                           delta/2) up and down; T = Delta + delta
 *   DMRI_SEQ_DOUBLE_TRAP_PGSE {delta, Delta, ramp, t_mix}
 * Every edge of f (pulse starts and ends, ramp corners, lobe starts) and the
 * echo time T must be a multiple of dt (within 1e-9), 0 < delta <= Delta.
 * F(t) = int_0^t f is evaluated in closed form at the grid points, the
 * U-form uses the one-sided limits f(t^{n-1}+), f(t^n-) of each step, and
 * b = G^2 int_0^T F^2 (eq. b_value) with the integral in closed form for
 * PGSE and by Gauss-Legendre quadrature between the edges otherwise. Every
 * profile here has F(T) = 0, so the returned S is the signal at echo time.
 * Errors: DMRI_E_INVALID (unknown kind, wrong n_params, bad values). */
#define DMRI_SEQ_PGSE 0
#define DMRI_SEQ_DOUBLE_PGSE 1
#define DMRI_SEQ_COS_OGSE 2
#define DMRI_SEQ_SIN_OGSE 3
#define DMRI_SEQ_TRAP_PGSE 4
#define DMRI_SEQ_DOUBLE_TRAP_PGSE 5
DMRI_API dmri_status dmri_set_sequence(dmri_handle h, int32_t kind, const double* params,
                              int32_t n_params, double dt_us, double theta);

/* Arbitrary profile given on the time grid t^n = n dt, n = 0..n_steps (the
 * C analogue of giving any expression f(s), Sec. 3):
 *   F       [n_steps + 1] F(t^n), F[0] = 0 (transformed form)
 *   f_start [n_steps] f(t^n+), f_end [n_steps] f(t^{n+1}-) for the step
 *           (t^n, t^{n+1}) (U-form; both NULL if only periodic problems run)
 *   int_F2  int_0^T F^2 > 0, with T = n_steps dt (b = G^2 int_F2)
 * The arrays are copied. The returned S is sum_i w_i u_i^N, the signal when
 * F(T) = 0. Errors: DMRI_E_INVALID (non-finite values, F[0] != 0, one f
 * array without the other, int_F2 <= 0); a run of a Neumann problem without
 * f gives DMRI_E_STATE. */
DMRI_API dmri_status dmri_set_sequence_table(dmri_handle h, int64_t n_steps, double dt_us,
                                    double theta, const double* F, const double* f_start,
                                    const double* f_end, double int_F2);

/* Solver options (all have defaults):
 *  "precision"  0 = all FP64 (default), 1 = FP32 matrices and Krylov
 *               vectors with FP64 reductions and FP64 residual refinement
 *  "krylov"     0 = auto (CG on the Hermitian transformed operator, COCG on
 *               the complex-symmetric U-form), 1 = CG, 2 = COCG, 3 = restarted
 *               GMRES(m) with right Jacobi preconditioning (either form; a
 *               cross-check and fallback for COCG, whose bilinear form can
 *               break down on the U-form; precision 0 only, else
 *               DMRI_E_UNSUPPORTED). Every system stops at the same
 *               ||b - A x|| <= rtol ||b|| test
 *  "gmres_m"    GMRES restart length m, 1..32 (default 30)
 *  "dir_bf16"   1 (default): the FP32 inner solves on 128-system paired
 *               tiles (precision 1, batches above 64 systems) store their
 *               search directions in BF16, halving the SpMV's gathered bytes;
 *               every recurrence uses the stored direction, so the residual
 *               stays consistent and the FP64 refinement sets the accuracy.
 *               0: FP32 directions
 *  "spmv_rows"  2 (default): a wavefront of the paired BF16 SpMV takes its
 *               rows two at a time, both rows' gathers in flight together (the
 *               kernel is bound by the latency of each row's dependent loads);
 *               1: one row at a time
 *  "markers"    1: roctx ranges ("dmri batch <systems>", "dmri step <n>")
 *               around each batch and time step, for profiler timelines
 *               (rocprofv3 --marker-trace); 0 (default): none
 *  "weak_kappa" scale of kappa_e on weak pseudo-periodic faces, (0, 1e6]
 *               (default 1: the paper's max{D / h}). Larger values couple
 *               the faces more tightly and need a smaller dt (the partner
 *               term is lagged by one step).
 *  "rtol"       per-step relative residual ||b - A x|| <= rtol ||b||
 *               (default 1e-10)
 *  "inner_rtol" FP32 inner solve reduction in mixed precision (1e-4)
 *  "mesh_merge" 1: a dmri_run over pairs of several problems solves them as
 *               one batch: the problems' operators concatenated block-
 *               diagonally, each problem's pairs (ordered by cost) padded
 *               with b = 0 systems to whole tiles, so each tile holds one
 *               mesh's systems; every kernel launch then covers the tiles of
 *               all meshes, each over its own mesh's rows; a batch of at most
 *               64 systems can run the persistent Krylov kernel (options
 *               persistent, graph: one launch per solve over all meshes, the
 *               time loop captured in a HIP graph). Any precision and
 *               Krylov method, guess 0/1, signal at echo (or option
 *               signal = 0); one form for all problems, no tensors, weak
 *               faces, LDS SpMV, polynomial preconditioner or sample
 *               recording; other combinations end in DMRI_E_UNSUPPORTED. The concatenated
 *               operator is built once per list of problems and kept (host
 *               and device copies) until dmri_destroy. 0 (default): one
 *               batch per problem (option concurrency). Applies to dmri_run
 *               and to dmri_run_device over several problems.
 *  "inner_floor" fraction f in (0, 1] of the outer target below which an
 *               FP32 inner solve does not go: it stops once ||r|| <=
 *               max(inner_rtol ||r64||, f rtol ||b||) (default 0.25). A
 *               larger f saves inner iterations; the FP64 refinement still
 *               ends every step at ||b - A x|| <= rtol ||b||
 *  "max_iter"   Krylov iterations per step and system (default 2000)
 *  "guess"      0 = previous step, 1 = polynomial extrapolation of the
 *               past solutions (default), 2 = learned correction of the
 *               damped cubic extrapolation (needs network parameters;
 *               precision 0 or 1)
 *  "extrap_order" order p of the extrapolation (1..4, default 3): the
 *               polynomial through u^{n-1}, ..., u^{n-1-p} at t^n, i.e.
 *               x0 = sum_k (-1)^k C(p+1, k+1) u^{n-1-k}; early steps use the
 *               history available
 *  "extrap_damp" 1 = use p + 2 past solutions with weights that reproduce
 *               polynomials of degree <= p and cancel a sign-alternating
 *               sequence (the components the theta = 1/2 scheme barely
 *               damps, which plain extrapolation amplifies by 2^(p+1))
 *               (default); 0 = plain polynomial extrapolation
 *  "sys_tile"   systems per lane group: 0 = auto, or 8, 16, 32, 64
 *  "graph"      1 = when the Krylov solves run in the persistent kernel
 *               (no host decisions inside the time loop), capture the whole
 *               time loop in a HIP graph and replay it; the graph is kept in
 *               the handle (one per kind of batch, up to 8 per lane) and
 *               replayed while the batch, buffers and options are unchanged;
 *               any device reallocation since the capture forces a new one
 *               (default 0; not with time_kernel or sample recording)
 *  "n_steps"    0 = full echo (default); n > 0 stops after n steps and
 *               returns the signal at t^n (see "signal")
 *  "signal"     what is returned when a run stops where F(t) != 0 on a
 *               periodic problem (n_steps, or a table sequence with
 *               F(T) != 0): 1 = the physical signal S(t) = int U(x, t) dx
 *               with U = u exp(-i G F q . x), x from the box centre
 *               (Appendix A's substitution; Sec. 2, eq. signal), integrated
 *               exactly per tetrahedron for the P1 field u (default;
 *               DMRI_E_UNSUPPORTED if G |F| times the longest edge exceeds
 *               16 rad); 0 = sum_i w_i u_i (the transformed field's
 *               integral). Both are the same when F = 0; for walls (U-form)
 *               the unknown is U and sum_i w_i U_i is returned
 *  "time_kernel" 0 = off, 1 = SpMV+dot, 2 = CG update, 3 = direction
 *               update, 4 = step start, 5 = learned-guess network, 6 =
 *               extrapolation, 7 = polynomial preconditioner (its terms and
 *               direction update): bracket every launch of that kernel
 *               with HIP events and report the summed time in dmri_stats
 *  "precond"    preconditioner of the Krylov solves (the paper leaves the
 *               solver open, Sec. 3): 0 = Jacobi (default); 1 = Chebyshev
 *               polynomial in D^-1 A (D = diag A) on the spectral interval
 *               [a, b] that the preconditioner network predicts for each
 *               system and step (dmri_precond_set_params); 2 = the same on
 *               the fixed interval [cheb_a, cheb_b]. 1 and 2 run flexible CG
 *               (FCG(1): each direction is the preconditioned residual made
 *               A-orthogonal to the previous one) to the same ||b - A x|| <=
 *               rtol ||b|| test; a step in which a system ends with a new
 *               flag (max_iter, non-finite) is solved again by Jacobi CG
 *               from the flexible solve's x. CG on the transformed form in
 *               precision 0 only, static sweeps (queue 0); otherwise
 *               DMRI_E_UNSUPPORTED
 *  "cheb_terms" m, terms of the polynomial (1..16, default 4): m - 1
 *               products with A per application; m = 1 is Jacobi
 *  "cheb_a", "cheb_b" fixed interval of precond = 2 (defaults 0.5, 1.5;
 *               0 < a, 1.001 a < b <= 1e6)
 *  "pc_fallback_steps" read-only: steps re-solved by Jacobi CG since the
 *               handle was created
 *  "blocks_per_xcd" workgroups per XCD sweeping the rows (default 512)
 *  "max_outer"  FP64 refinement passes per step in mixed precision (8)
 *  "queue"      1 = gather kernels take rows from a per-XCD queue,
 *               0 = static chunks (default)
 *  "grab"       rows per queue grab, in units of 2 wavefront passes (4)
 *  "nt"         1 = SpMV results stored non-temporally (default)
 *  "lds"        1 = SpMV stages matrix chunks in LDS for tiles of 32/64
 *               systems (default 0)
 *  "persistent" Krylov iterations of a step in one persistent launch with
 *               grid barriers: 0 = off, 1 = on (batches of <= 64 systems),
 *               2 = auto (default: on when rows x systems <= 131072)
 *  "autotune"   1 = before the first run of a kind of batch (problem,
 *               number of systems, precision, solver), time its first steps
 *               under each candidate launch configuration (tile width,
 *               blocks per XCD, persistent kernel, LDS SpMV) and use the
 *               fastest; the choice is cached in the handle (default 0). A
 *               several-mesh batch (mesh_merge) is one kind of batch per list
 *               of problems and pair counts; its candidates are the tile
 *               width, blocks per XCD and the persistent kernel
 *  "tuned_sys_tile", "tuned_blocks_per_xcd", "tuned_persistent",
 *  "tuned_lds", "tuned_trials"  read-only (dmri_get_option): the
 *               configuration the autotuner applied last (-1 before any)
 *  "progress"   k > 0 prints one line to stderr every k time steps
 *  "ordering"   DOF order of problems added afterwards: 0 = Morton curve,
 *               1 = pencils (default): columns of "pencil" x "pencil" cells
 *               swept z-, y-, x-major, bounding the index distance between
 *               mesh neighbours
 *  "pencil"     pencil width in cells (default 12)
 *  "sort_systems" 1 = order the systems of a batch before tiling, so tiles
 *               of similar systems converge and leave the Krylov loop
 *               together (default): by the iterations each (problem, b, q)
 *               needed in its last run in this handle when all are known,
 *               else by b; 0 = input order. Results are returned in input
 *               order and do not depend on the setting
 *  "xcd_split"  1 = every tile of systems is split into 8 row parts, one
 *               per XCD, so the tiles still iterating keep the whole chip
 *               busy; 0 = tiles split only as far as needed for a multiple
 *               of 8 work items (default)
 *  "tile_sched" 1 = each chunk of Krylov iterations is launched over the
 *               tiles still active (as of the last counts the host read),
 *               each split into enough row parts that all XCDs get the same
 *               work (default); 0 = every launch covers every tile and
 *               converged tiles only exit early. Results do not depend on it
 *  "pair_lanes" 1 = the FP32 inner solves of mixed precision on batches of
 *               more than 64 systems use tiles of 128 systems with two
 *               systems per lane (16-byte vector accesses, half the memory
 *               instructions per system) (default); 0 = 64-system tiles
 *  "concurrency" k > 1: a dmri_run over several problems runs up to k of
 *               them at once, each on its own stream and workspace driven by
 *               its own host thread with its own copy of the options (meshes
 *               of uneven size share the GPU; the autotuner tunes one batch
 *               at a time); 1 = one after another (default). Runs with
 *               sample recording use one lane
 * Unknown keys or out-of-range values: DMRI_E_INVALID. */
DMRI_API dmri_status dmri_set_option(dmri_handle h, const char* key, double value);
DMRI_API dmri_status dmri_get_option(dmri_handle h, const char* key, double* value);

/* ---- Learned initial guess (option "guess" = 2) ----------------------
 * A per-element network corrects the damped cubic extrapolation of the next
 * time step's solution (the theta-scheme of Appendix A marches u^{n-1} ->
 * u^n; the network only moves the Krylov starting point, the solve and its
 * stopping test are unchanged). With u_k = u^{n-1-k} (k = 0..4), the base is
 * x_dc = (49 u_0 - 36 u_1 - 26 u_2 + 44 u_3 - 15 u_4) / 16 (option guess = 1's
 * default) and the scale is s = |u_0 - u_1|. For element (DOF i, system s)
 * the 16 features are: (u_k - u_{k+1}) / s for k = 0..3 (Re, Im), the phase
 * u_0 / |u_0| (Re, Im), the changes of G F(t) over the last two steps (x10),
 * G F(t^n), dt D (G F(t^n))^2, (q . x) / 10 with x from the box centre in um,
 * the membrane flag; all zero where s or |u_0| is 0. The network 16 -> 64 ->
 * 64 -> 2 (ReLU) predicts 100 (u^n - x_dc) / s (Re, Im; recorded targets
 * clipped to [-100, 100]); the guess is x_dc + s y / 100, so an element
 * whose history did not change gets no correction. Layers run as BF16
 * matrix-core products with FP32 accumulation; the parameters are FP32,
 * packed W1[16][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2]
 * (row-major, x W + b). Non-finite predictions fall back to x_dc element by
 * element; the first four steps use the extrapolation of guess = 1. */
#define DMRI_GUESS_N_FEATURES 16
#define DMRI_GUESS_N_PARAMS 5378

/* Set the network parameters from host memory (n_params must equal
 * DMRI_GUESS_N_PARAMS); restarts the Adam moments. */
DMRI_API dmri_status dmri_guess_set_params(dmri_handle h, const float* params, int64_t n_params);
/* Copy the current parameters to host memory. DMRI_E_STATE if none set. */
DMRI_API dmri_status dmri_guess_get_params(dmri_handle h, float* params, int64_t n_params);
/* Load / save parameters as a file: 8 bytes "DMRIMLP1", int32 16, 64, 2,
 * then DMRI_GUESS_N_PARAMS little-endian float32. A wrong header gives
 * DMRI_E_INVALID. */
DMRI_API dmri_status dmri_load_guess_model(dmri_handle h, const char* path);
DMRI_API dmri_status dmri_save_guess_model(dmri_handle h, const char* path);

/* Autotuner cache (option "autotune"; Sec. 5 "Parallelization": many runs of
 * the same meshes): the launch configuration chosen for each (device
 * architecture and CU count, mesh structure hash, number of systems,
 * precision, krylov, sys_tile) is kept in the handle; these calls write it
 * to a text file and merge a file into the handle, so later processes skip
 * the trial runs. A loaded entry reports option "tuned_trials" 0. Malformed
 * files (header "dmri-tuning-v1", then "key sys_tile blocks_per_xcd
 * persistent lds seconds" per line, values in their option ranges) give
 * DMRI_E_INVALID and change nothing. Host-only handles may load and save. */
DMRI_API dmri_status dmri_save_tuning(dmri_handle h, const char* path);
DMRI_API dmri_status dmri_load_tuning(dmri_handle h, const char* path);

/* Record training samples during later dmri_run / dmri_run_device calls:
 * at every step n >= 5, every stride-th element of the batch (a different
 * offset each step) appends its features to d_features ([capacity][16]
 * float32, device) and its target to d_targets ([capacity][2] float32,
 * device) until capacity samples are held; capacity = 0 stops recording.
 * The buffers are the caller's and must stay valid while recording is on.
 * Resets the sample count. Recording needs precision 0 or 1. */
DMRI_API dmri_status dmri_guess_record(dmri_handle h, float* d_features, float* d_targets,
                              int64_t capacity, int64_t stride);
/* Samples recorded so far (<= capacity). */
DMRI_API dmri_status dmri_guess_record_count(dmri_handle h, int64_t* count);

/* Evaluate the network on n samples (device buffers): outputs d_out[n][2]
 * (may be NULL), the gradient of the mean squared error
 * L = sum((y - t)^2) / n with respect to the packed parameters into
 * d_grad[DMRI_GUESS_N_PARAMS] (may be NULL) and L into *loss (may be NULL).
 * Gradient and loss need d_targets. Returns after the results are written. */
DMRI_API dmri_status dmri_guess_eval(dmri_handle h, int64_t n, const float* d_features,
                            const float* d_targets, float* d_out, float* d_grad, double* loss);
/* n_iters full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, step
 * size lr) on the mean squared error over n device samples. *loss_first is
 * L before the first step, *loss_last L before the last step (either may be
 * NULL). */
DMRI_API dmri_status dmri_guess_train(dmri_handle h, int64_t n, const float* d_features,
                             const float* d_targets, int32_t n_iters, double lr,
                             double* loss_first, double* loss_last);

/* Preconditioner network (option "precond" = 1; the learned preconditioner
 * that goes with the learned guess). Same shape and parameter layout as the
 * guess network (16 -> 64 -> 64 -> 2, BF16 matrix-core layers, FP32
 * parameters), one sample per system and time step. Inputs: log(theta dt
 * D/h^2), log(1 + theta dt D (G F)^2), log(1 + theta dt D |G F| / h),
 * log(1 + theta dt kappa / h), |q_x|, |q_y|, |q_z|, then nine zeros (D the
 * largest compartment diffusivity, h the longest edge, F = F(t^n)). Outputs
 * y give the interval [0.5 e^y0, 1.5 e^y1] (y clipped to [-20, 20]; the
 * reference interval [0.5, 1.5] where that is not finite or not an interval,
 * so a zero network gives the reference). */
#define DMRI_PRECOND_N_FEATURES 16
#define DMRI_PRECOND_N_PARAMS 5378
DMRI_API dmri_status dmri_precond_set_params(dmri_handle h, const float* params,
                                             int64_t n_params);
DMRI_API dmri_status dmri_precond_get_params(dmri_handle h, float* params, int64_t n_params);
/* Record training samples during later runs with precond = 0 (Jacobi CG,
 * precision 0, transformed form, static sweeps): after every time step,
 * each system that took 2..64 iterations without a flag appends its 16
 * features to d_features ([capacity][16] float32, device) and the targets
 * {log(r_min / 0.5), log(1.1 r_max / 1.5)} to d_targets ([capacity][2]),
 * where r_min, r_max are the extreme Ritz values of the step's CG run (the
 * eigenvalues of the Lanczos tridiagonal its alpha_k and beta_k define:
 * estimates of the ends of the spectrum of D^-1 A that the residual
 * explored; 1.1 is the margin over the largest). Samples go in system order
 * until capacity are held; capacity = 0 stops recording. Resets the count.
 * The buffers are the caller's and must stay valid while recording is on. */
DMRI_API dmri_status dmri_precond_record(dmri_handle h, float* d_features, float* d_targets,
                                         int64_t capacity);
DMRI_API dmri_status dmri_precond_record_count(dmri_handle h, int64_t* count);
/* n_iters full-batch Adam steps on the mean squared error of the
 * preconditioner network over n device samples (as dmri_guess_train). */
DMRI_API dmri_status dmri_precond_train(dmri_handle h, int64_t n, const float* d_features,
                                        const float* d_targets, int32_t n_iters, double lr,
                                        double* loss_first, double* loss_last);

/* Simulate n_pairs (problem, b, direction) systems and write their signals.
 *   problem_id [n_pairs] ids from dmri_add_problem
 *   b          [n_pairs] >= 0
 *   q          [n_pairs][3] gradient direction, normalized inside; ignored
 *              when b == 0; must be nonzero when b > 0
 *   signal_out [n_pairs][2] Re, Im of S (um^3)
 *   stats      may be NULL
 * The pairs of each problem are solved as one batch on the device (all
 * systems of a mesh share every matrix read); batches of different
 * problems run one after another, or several at once on their own streams
 * with option "concurrency" > 1, or all problems form one batch with option
 * "mesh_merge" = 1. Results agree to rounding across these choices.
 * n_pairs = 0 is an empty run: DMRI_OK, stats zeroed, nothing read or written.
 * Returns DMRI_NOT_CONVERGED (results still written) when any system hit
 * max_iter in some step. */
DMRI_API dmri_status dmri_run(dmri_handle h, int64_t n_pairs,
                     const int32_t* problem_id, const double* b, const double* q,
                     double* signal_out, dmri_stats* stats);

/* Same as dmri_run with device-resident inputs and output (e.g. from
 * PyTorch tensors): d_problem_id [n_pairs] (int32), d_b [n_pairs],
 * d_q [n_pairs][3], d_signal [n_pairs][2] are device pointers. Work is
 * enqueued on hip_stream (NULL = the handle's own stream), after the work
 * already queued there; the call reads the (small) pair list to the host to
 * check it and form the batches, synchronizes that stream to poll
 * convergence, and returns after the signals have been written. When every
 * pair names the same problem its b and q are used in place; otherwise the
 * batches are formed as in dmri_run. n_pairs = 0: DMRI_OK, stats zeroed. */
DMRI_API dmri_status dmri_run_device(dmri_handle h, void* hip_stream, int64_t n_pairs,
                            const int32_t* d_problem_id, const double* d_b, const double* d_q,
                            double* d_signal, dmri_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run as dmri_run_device, with every buffer of the run (solution history,
 * Krylov vectors, partial sums, counters, per-system scalars, grid barrier)
 * taken from a fixed 64 MiB device array that the library holds on each
 * device it runs on until the process ends. The call makes no hipMalloc,
 * hipFree, pinned-host or other device allocation; state is cleared with
 * fill kernels. The caller still passes the inputs and the output.
 * Limits: 1..64 pairs, all on one problem; precision 0 (FP64) with the
 * persistent Krylov kernel (one launch per step); guess 0 or 1; no sample
 * recording; no weak pseudo-periodic faces (DMRI_E_UNSUPPORTED). The
 * problem's operators must already be on the device for the
 * current sequence (any earlier dmri_run / dmri_run_device of the problem
 * uploads them), else DMRI_E_STATE. A run that needs more scratch than the
 * array holds (n_dof x padded systems x (history + 4) x 16 bytes plus
 * partials) gives DMRI_E_INVALID with the size in the message; other
 * violated limits DMRI_E_INVALID or DMRI_E_UNSUPPORTED. Systems are tiled in
 * input order (option "sort_systems" is not applied); a run that would need
 * the phase-weighted signal (option "signal", F != 0 at its last step) gives
 * DMRI_E_UNSUPPORTED. Every call on a device
 * uses that device's one array and leaves its contents there: calls that
 * overlap on one device (other threads, other handles, or work still queued
 * on another stream) race and corrupt each other; serialize them. Same
 * arguments, statistics and status as dmri_run_device; returns after the
 * signals are written. */
DMRI_API dmri_status dmri_run_device_noalloc(dmri_handle h, void* hip_stream, int64_t n_pairs,
                                    const int32_t* d_problem_id, const double* d_b,
                                    const double* d_q, double* d_signal, dmri_stats* stats);

/* Apply one step operator of problem `problem_id` to host vectors
 * (kernel check): y = (Base + c M_D + i (d . V)) x with Base = M/dt +
 * theta R when which = 0 (left side) or M/dt - (1-theta) R when which = 1
 * (right side, without the sign flip of the time-dependent parts: the
 * coefficients are taken as given). x, y: [n_dof][n_sys][2] doubles;
 * c [n_sys], d [n_sys][3]. Uses the precision of option "precision". With
 * weak pseudo-periodic faces the left Base also holds theta times the
 * scaled face mass (dmri_export_weak); the partner term is not applied. */
DMRI_API dmri_status dmri_apply_operator(dmri_handle h, int32_t problem_id, int32_t which,
                                int64_t n_sys, const double* c, const double* d,
                                const double* x, double* y);

#ifdef __cplusplus
}
#endif

#endif /* DMRI_H */
