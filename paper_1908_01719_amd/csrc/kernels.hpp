// Device kernels of libdmri (gfx950 / CDNA4) and their host launchers.
//
// Data layout in HBM (one problem = one mesh):
//   CSR pattern      row_ptr[n+1], col[nnz]                        int32
//                    every row padded to a multiple of kRowPad entries
//                    (padding: column = the row itself, all values 0), so
//                    the gather kernels fetch kRowPad column indices with one
//                    scalar load and issue kRowPad gathers back to back
//   matrix values    K0[nnz], Kr[nnz]                               T
//                    aux[nnz] = {M_D, V_x, V_y, V_z}                T4 (16/32 B)
//                    dK0[n], daux[n] (the diagonal, for Jacobi)
//   vectors          [n_tiles][n_rows][S] complex (T2): tile-major, systems
//                    fastest inside a tile, so a tile's rows are contiguous
//                    (S complex values per row); ld = n_tiles * S
//   per system       gq[ld] = {G, q_x, q_y, q_z} (double4)
// K0 = M/dt + theta R is the constant part of the left operator,
// Kr = M/dt - (1-theta) R the constant part of the right operator
// (Appendix A, eq. linear_billinear). The time-dependent parts are built on
// the fly per system: c = cm (G F)^2 on M_D and i d . V with d = cd G F q.
//
// Work decomposition ("XCD sweep"). A tile is S consecutive systems (S = 128
// for the paired FP32 layout, two systems per lane). Work items are (tile,
// row part) pairs, numbered so that their count is a multiple of 8; XCD x
// (blocks with blockIdx % 8 == x, which the hardware places on XCD x) owns
// items x, x+8, ... A Krylov launch may cover only the tiles still active
// (Geom::sched), each split into enough parts that every XCD gets the same
// number of items. Inside an item block j takes the row chunks j, j+B, ...;
// the gather kernels can instead take rows from a per-item queue (one atomic
// per wavefront grab, option). Every block keeps one FP64 partial per system
// for each item; small finalize kernels add the partials in a fixed order
// (deterministic), update the per-system Krylov scalars and reset the queues.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmri {

constexpr int kRowPad = 8;
// Most tiles a Krylov launch can be restricted to (the tiles still active).
constexpr int kMaxSched = 32;

template <typename T> struct Vec2Of;
template <> struct Vec2Of<double> { using type = double2; };
template <> struct Vec2Of<float> { using type = float2; };
template <typename T> struct Vec4Of;
template <> struct Vec4Of<double> { using type = double4; };
template <> struct Vec4Of<float> { using type = float4; };

template <typename T>
struct MatView {
    const int32_t* row_ptr;
    const int32_t* col;
    const T* K0;
    const T* Kr;
    const typename Vec4Of<T>::type* aux;
    const T* dK0;
    const typename Vec4Of<T>::type* daux;
    int32_t n_rows;
};

// Coefficients of one operator application: F value of the step and the
// multipliers of (G F)^2 (on M_D) and G F q (on V).
struct Coef {
    double F;
    double cm;
    double cd;
};

// Per-system Krylov state, all FP64.
struct SolverState {
    double2* rho;
    double2* alpha;
    double2* beta;
    double* bb;         // ||b||^2
    double* rr;         // ||r||^2
    int32_t* active;    // 1 while iterating
    int32_t* iters;     // iterations this step
    int32_t* iters_total;
    int32_t* flags;     // bit 0: hit max_iter, bit 1: non-finite residual
    int32_t* n_active;  // [n_tiles] systems still iterating per tile
    int32_t n_sys;
    int32_t max_iter;
    double rtol2;
    // Optional floor of the reference norm: a solve starts with
    // bb = max(||b||^2, floor_scale * floor_bb[sys]) (the FP32 inner solves
    // of mixed precision stop once they reach the outer tolerance).
    const double* floor_bb;
    double floor_scale;
    // Optional record of the CG coefficients of the current step for the
    // Ritz values that train the preconditioner's interval network:
    // ab_hist[sys * kRitzMax + k] = {Re alpha_k, Re beta_k}.
    double2* ab_hist;
};

constexpr int kRitzMax = 64;  // CG coefficients kept per system and step

// Launch geometry shared by every kernel of a problem.
struct Geom {
    int32_t n_rows;
    int32_t ld;          // leading dimension (systems, padded)
    int32_t S;           // systems per lane group (tile width)
    int32_t n_tiles;     // ld / S
    int32_t n_parts;     // row parts per tile
    int32_t n_items;     // n_tiles * n_parts (a multiple of 8)
    int32_t part_rows;   // rows per part (multiple of chunk_rows)
    int32_t chunk_rows;  // rows per block chunk of the streaming kernels
    int32_t B;           // blocks per XCD
    int32_t queue;       // gather kernels: 1 = per-item row queue, 0 = static chunks
    int32_t grab;        // queue grabs per wavefront take grab * 2 * 64/S rows
    int32_t tile_bytes_ok;  // a 64-system FP64 tile is below 2^31 bytes (buffer gathers)
    int32_t dx_pair;        // refinement: dx is stored in the 128-system paired layout
    int32_t nt;          // 1 = SpMV output stored non-temporally
    int32_t lds;         // 1 = LDS-staged SpMV for tiles of 32 or 64 systems
    int32_t dir16;       // paired layout: search directions p stored as BF16 (8 B per lane)
    int32_t rows2;       // paired SpMV with BF16 directions: 2 = a wavefront takes two rows at once
    int32_t bpx;         // blocks per XCD asked for (B = min(bpx, chunks of a part))
    int32_t n_sched;     // 0: items cover tiles 0..n_tiles-1; else tiles sched[0..n_sched)
    int32_t sched[kMaxSched];
    // Anisotropic problems (a diffusion tensor per compartment): the mass
    // term's coefficient of a row is scaled by q.D_k q of the row's
    // compartment k: comp[row] = k, acomp[k * ld + sys] = q_sys . D_k q_sys.
    // Both null for scalar diffusivities (the factor is then in M_D itself).
    const int32_t* comp;
    const double* acomp;
    int32_t acomp_ld;    // row stride of acomp (>= ld)
    // Batches over several meshes (the meshes' rows concatenated, each tile
    // holding systems of one mesh): per tile {first row, end row, element
    // base, rows per part} in device memory, where element (row, system) of
    // tile t sits at base + row * S + (system - t S) for the tile's rows
    // only and each tile's n_parts parts split its own rows; part_rows is
    // then the longest part. vlen is the elements of one vector (the sum
    // over tiles of rows * S). Null and 0 for one mesh (element base
    // tile * n_rows * S, vlen n_rows * ld).
    const int64_t* mtab;
    int64_t vlen;
};

inline int64_t vec_elems(const Geom& g) {
    return g.vlen ? g.vlen : static_cast<int64_t>(g.n_rows) * g.ld;
}

struct Scratch {
    double* partial;     // [n_tiles * n_parts][B][S][4], item = tile * n_parts + part
    int32_t* ctr_spmv;   // [n_tiles * n_parts] chunk queues of the gather kernels,
    int32_t* ctr_init;   // [n_tiles * n_parts] zero between launches
    // [n_tiles][kFinGroups][S][4] group sums of a two-stage finalize, or null
    // (the finalize then adds every partial itself)
    double* stage = nullptr;
};

// Groups of the first stage of a finalize over many partials per tile.
constexpr int kFinGroups = 64;

Geom make_geom(int32_t n_rows, int32_t n_sys, int32_t S, int32_t blocks_per_xcd, int32_t queue,
               int32_t grab, bool xcd_split = false);
// Geometry of g restricted to the n tiles listed (the tiles that may still
// be active): each is split into enough row parts that every XCD gets the
// same number of items. Returns g itself when the list is empty, covers
// every tile, is longer than kMaxSched, or g uses row queues or spans
// several meshes (whose tiles keep their own row parts). Partials and
// queue counters of the restricted launches stay addressed by
// (tile * n_parts + part), so buffers sized for n_tiles * 8 parts serve both.
Geom sched_geom(const Geom& g, const int32_t* tiles, int n);

// guess_mode: 0 x0 = u_prev, 1 x0 = 2 u_prev - u_prev2 (x0 written to x),
// 2 x0 given in x, 3 x0 = x + dx (mixed-precision correction, written to
// x_out, which must not alias x; b read from bvec), 4 r -= A dx, x_out =
// x + dx (refinement pass keeping the step's ||b||^2). In modes 0-2 p = D^-1 r
// is written when p is not null (the mixed-precision outer level passes null:
// its inner solves form their own directions).
template <typename T>
void launch_init(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                 Coef lhs, Coef rhs, bool herm, int guess_mode,
                 const typename Vec2Of<T>::type* u_prev, const typename Vec2Of<T>::type* u_prev2,
                 typename Vec2Of<T>::type* x, typename Vec2Of<T>::type* r,
                 typename Vec2Of<T>::type* p, const float2* dx, typename Vec2Of<T>::type* x_out,
                 typename Vec2Of<T>::type* bvec, SolverState s, Scratch sc,
                 const int32_t* wmap = nullptr, const typename Vec2Of<T>::type* wb = nullptr);

// Weak pseudo-periodic faces (Appendix B, the partner term of L*): for every
// DOF on a weak face (slot), wb[slot * ld + sys] =
//   c sum_k val_k e^{i s_k phi_a} u_prev[col_k][sys],  phi_a = G F q_a L_a,
// a = code_k % 3, s_k = +1 for code_k < 3 (row on the face x_a = lo), -1
// otherwise; G, q from gq, F = F(t^n), c = (1 - theta) times the kappa_e
// scale. k_init adds wb to the right-hand side of the rows wmap maps to a
// slot (wmap[row] = slot or -1).
struct WeakView {
    const int32_t* ptr;   // [n_slots + 1]
    const int32_t* col;
    const int32_t* code;
    const double* val;
    const int32_t* map;   // [n_rows]
    int32_t n_slots;
    double L[3];
};
template <typename T>
void launch_weak_rhs(hipStream_t st, const Geom& g, const WeakView& w, const double4* gq,
                     int32_t n_sys, double F, double c, const typename Vec2Of<T>::type* u_prev,
                     typename Vec2Of<T>::type* wb);

// Start of an FP32 inner solve on the FP64 residual r64 of the systems still
// active in `outer`: r = (float) r64, dx = 0, p = D^-1 r (FP32 operator).
void launch_inner_start(hipStream_t st, const Geom& g, const MatView<float>& A,
                        const double4* gq, Coef lhs, bool herm, const double2* r64,
                        const int32_t* outer_active, float2* r, float2* dx, float2* p,
                        SolverState s, Scratch sc);

template <typename T>
void launch_spmv_dot(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                     Coef lhs, bool herm, const typename Vec2Of<T>::type* p,
                     typename Vec2Of<T>::type* q, SolverState s, Scratch sc);

// r -= alpha q with the convergence decision on ||r||^2; check_only keeps
// beta and rho (flexible CG forms them from the preconditioned residual).
template <typename T>
void launch_update(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                   Coef lhs, bool herm, typename Vec2Of<T>::type* x,
                   typename Vec2Of<T>::type* r, const typename Vec2Of<T>::type* p,
                   const typename Vec2Of<T>::type* q, SolverState s, Scratch sc,
                   bool check_only = false);

// ---- polynomial preconditioner inside flexible CG (FP64, Hermitian) ----
// z = p(D^-1 A) D^-1 r by m terms of the Chebyshev recurrence on each
// system's interval ab[sys] = {a, b} (0 < a < b), for the systems active in
// s: term 0 writes y[0] (and d), term j reads y[(j-1) & 1] and writes
// y[j & 1]; returns z = y[(m-1) & 1]. The last term also forms r^H z and
// q^H z, and a finalize sets rho = r^H z and beta = -(q^H z) / (p^H q) (or
// beta = 0 when start is set). Needs static sweeps (g.queue == 0).
const double2* launch_cheb(hipStream_t st, const Geom& g, const MatView<double>& A,
                           const double4* gq, Coef lhs, const double2* ab, int m, bool start,
                           const double2* r, const double2* q, double2* const y[2], double2* d,
                           SolverState s, Scratch sc);

// End of flexible-CG iteration k_iter: x += alpha p for the systems that took
// part in it (none when k_iter < 0), p = z + beta p for the systems active.
void launch_pupdate_z(hipStream_t st, const Geom& g, const double2* z, double2* p, double2* x,
                      int32_t k_iter, SolverState s);

// Scalars of one step for the interval network's features.
struct PcScalars {
    double dt, theta, d_max, h, kappa;
    double F;  // F(t^n)
};
// Interval per system: features X[ld][16] -> network (theta, the packed
// 16-64-64-2 parameters) -> Y[ld][2] -> ab[sys] = {A_ref e^Y0, B_ref e^Y1}
// (clipped exponents; the reference interval where that is not finite or
// not an interval). theta = NULL gives every system the interval {a, b}.
constexpr double kPcARef = 0.5, kPcBRef = 1.5, kPcMargin = 1.1;
void launch_pc_interval(hipStream_t st, int32_t n_sys, int32_t ld, const double4* gq,
                        PcScalars ps, const float* theta, double a, double b, float* X, float* Y,
                        double2* ab);
// Training samples of a Jacobi-CG step (coefficients in s.ab_hist): every
// system that took 2 to kRitzMax iterations and ended without a flag appends
// its features and targets {log(ritz_min / A_ref), log(margin ritz_max /
// B_ref)}, in system order, at *count while *count < cap.
void launch_pc_record(hipStream_t st, int32_t n_sys, const double4* gq, PcScalars ps,
                      SolverState s, float* X, float* T, int64_t* count, int64_t cap);

template <typename T>
// End of Krylov iteration k_iter (1-based within the solve): x += alpha p
// for the systems that took part in it, p = D^-1 r + beta p for the systems
// still active.
void launch_pupdate(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                    Coef lhs, const typename Vec2Of<T>::type* r, typename Vec2Of<T>::type* p,
                    typename Vec2Of<T>::type* x, int32_t k_iter, SolverState s);

template <typename T>
void launch_signal(hipStream_t st, const Geom& g, const double* w,
                   const typename Vec2Of<T>::type* x, double2* out, int32_t n_sys, Scratch sc);

// Tetrahedra of a mesh on the device: DOFs and mesh nodes of the four
// vertices, node positions relative to the box centre.
struct TetView {
    const int4* dof;
    const int4* node;
    const double* xyz;  // [n_nodes][3]
    int32_t n_tets;
};

// Signal of the physical field U = u exp(-i k_s . x) with k_s = G_s F q_s at a
// time where F != 0 (transformed form): S_s = sum over tetrahedra of the exact
// integral of the P1 field u_s times the plane wave. g is the vector layout
// (rows = DOFs), gt the same tiles with rows = tetrahedra (work items).
template <typename T>
void launch_signal_phase(hipStream_t st, const Geom& g, const Geom& gt, const TetView& tv,
                         const double4* gq, double F, const typename Vec2Of<T>::type* x,
                         double2* out, int32_t n_sys, Scratch sc);

// y = (Base + c M_D + i d.V) x for explicit per-system c and d (kernel check).
template <typename T>
void launch_apply(hipStream_t st, const Geom& g, const MatView<T>& A, int which,
                  const double* c, const double3* d, const typename Vec2Of<T>::type* x,
                  typename Vec2Of<T>::type* y);

// acomp[k * ld + s] = q_s . D_k q_s for every compartment k < n_comp and
// system s < ld (q from gq; padding systems have q = x). tensors [n_comp][6]
// = xx, yy, zz, xy, xz, yz.
void launch_aniso_params(hipStream_t st, int32_t n_comp, int32_t ld, const double4* gq,
                         const double* tensors, double* acomp);

// Fill: x = u0 per DOF for every system < n_sys, 0 for padding.
template <typename T>
void launch_set_initial(hipStream_t st, const Geom& g, const double* u0, int32_t n_sys,
                        typename Vec2Of<T>::type* x);
// The same for one tile block of a several-mesh batch: rows * S elements
// from x, row r of lane l set to u0[r] for lanes l < n_live, 0 otherwise.
template <typename T>
void launch_set_initial_block(hipStream_t st, int64_t rows, int32_t S, int32_t n_live,
                              const double* u0, typename Vec2Of<T>::type* x);

// Per-system parameters from b and q on the device: G = sqrt(b / intF2),
// q normalised; padding systems get G = 0.
void launch_sys_params(hipStream_t st, int32_t n_sys, int32_t ld, const double* b,
                       const double* q, double int_F2, double4* gq, int32_t* bad);

// Grid-wide barrier state for the persistent solver (zero-initialised once).
struct GridBarrier {
    uint32_t* count;  // [32 * 9]: global counter at 0, XCD-group counters at 32*(x+1)
    uint32_t* gen;
    int32_t* err;     // set to 1 if a barrier wait timed out
};

// Krylov iterations of one step in a single launch of 8 * g.B blocks, all of
// which must be co-resident (the host sizes g.B from the CU count). The
// per-system scalars are recomputed redundantly in every block from the
// partials after each grid barrier, so a batch may hold at most 64 systems
// (g.ld <= 64). Requires g.queue == 0 and a partial buffer of twice the
// usual size (2 * n_items * B * S * 4 doubles).
template <typename T>
void launch_krylov_persistent(hipStream_t st, const Geom& g, const MatView<T>& A,
                              const double4* gq, Coef lhs, bool herm,
                              typename Vec2Of<T>::type* x, typename Vec2Of<T>::type* r,
                              typename Vec2Of<T>::type* p, typename Vec2Of<T>::type* q,
                              SolverState s, Scratch sc, GridBarrier bar);

// True when the 8 * g.B blocks of the persistent solver can all be resident
// at once on a device with n_cu compute units (occupancy of the kernel that
// launch_krylov_persistent would pick); the grid barrier needs that.
template <typename T>
bool persistent_fits(const Geom& g, bool herm, int n_cu);

// ---- restarted GMRES(m) with right Jacobi preconditioning (FP64) ----
constexpr int kGmMax = 32;                      // longest cycle (restart length)
constexpr int kGmVals = 2 * (kGmMax + 1) + 2;   // reduction values per system
// Krylov basis: v_i = base + i * stride (batch-layout FP64 vectors).
struct GmresBasis {
    double2* base;
    size_t stride;
};
// Per-system state of the cycles (FP64), indexed by system < ld.
struct GmresState {
    double* partial;   // [items][B][S][kGmVals] block partials
    double* hout;      // [ld][kGmVals] reduced values
    double2* H;        // [ld][(kGmMax + 1) * kGmMax] Hessenberg, row-major
    double* cs;        // [ld][kGmMax] Givens cosines
    double2* sn;       // [ld][kGmMax] Givens sines
    double2* g;        // [ld][kGmMax + 1] rotated right-hand side
    double2* y;        // [ld][kGmMax] small solution
    double* hnorm;     // [ld] last norm (beta, then h_{j+1,j})
    int32_t* cycle;    // [ld] 1 while the system iterates in the current cycle
    int32_t* dim;      // [ld] columns of the current cycle
};
// A cycle's kernels take a SolverState whose `active` points at gm.cycle.
void gmres_cycle_start(hipStream_t st, const Geom& g, const GmresState& gm, const SolverState& s);
void gmres_count(hipStream_t st, const Geom& g, const GmresState& gm, const SolverState& s);
void gmres_scale(hipStream_t st, const Geom& g, const MatView<double>& A, const double4* gq,
                 Coef lhs, const double2* w, double2* v, double2* z, const GmresState& gm,
                 const SolverState& cyc);
void gmres_orthogonalize(hipStream_t st, const Geom& g, double2* w, GmresBasis V, int nv, int col,
                         int32_t n_sys, const GmresState& gm, const SolverState& cyc);
void gmres_givens(hipStream_t st, int32_t n_sys, int col, int m, bool use_rr,
                  const GmresState& gm, const SolverState& s);
void gmres_update(hipStream_t st, const Geom& g, const MatView<double>& A, const double4* gq,
                  Coef lhs, double2* x, GmresBasis V, int32_t n_sys, const GmresState& gm);
void gmres_residual(hipStream_t st, const Geom& g, const double2* b, const double2* q, double2* r,
                    const GmresState& gm, const SolverState& cyc);

// Zero n int32 values (a kernel, so it may be captured in a graph).
void launch_zero_i32(hipStream_t st, int32_t* p, int64_t n);

// Up to kMaxHist vectors and FP64 weights of a linear combination.
constexpr int kMaxHist = 7;
template <typename T>
struct ExtrapTerms {
    const typename Vec2Of<T>::type* u[kMaxHist];
    double c[kMaxHist];
    int32_t m;
};

// x = sum_k c[k] u[k] over all n_rows * ld elements of the batch.
template <typename T>
void launch_combine(hipStream_t st, const Geom& g, const ExtrapTerms<T>& t,
                    typename Vec2Of<T>::type* x);

}  // namespace dmri
