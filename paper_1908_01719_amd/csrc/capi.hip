// C ABI of libdmri and the host orchestration of the time loop.
//
// One run = all (b, q) systems of the requested problems. Per problem the
// systems form one batch on the device ([n_dof][ld] complex vectors, systems
// fastest) and each theta-step is (Appendix A, eq. linear_billinear):
//   b = (Kr + c_r M_D + i d_r . V) u^{n-1}               right-hand side
//   x0 = guess; r = b - A x0                             k_init
//   Krylov iterations on A x = b                         k_spmv_dot, k_update, k_pupdate
//   u^n = x
// and after the last step S = sum_i w_i u_i^N (Sec. 2, eq. signal).
// The host never waits on a single iteration: it enqueues chunks of
// iterations, copies the per-tile active counts to pinned memory behind each
// chunk, and checks the previous chunk's counts while the next one runs.
// Converged systems drop out inside the kernels (per-system masks).
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <string>
#include <vector>

#include "../../include/dmri.h"
#include "assembly.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "sequence.hpp"

namespace dmri {
namespace {

thread_local std::string g_create_error = "no error";

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            if (e_ == hipErrorOutOfMemory)                                             \
                throw Error(DMRI_E_NOMEM, std::string("device allocation failed: ") + \
                                              hipGetErrorString(e_));                  \
            throw Error(DMRI_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
        }                                                                              \
    } while (0)

// Bumped by every device (re)allocation of a DevBuf. A captured graph bakes
// device addresses into its launches, so its cache key includes this count:
// any reallocation since the capture forces a new capture.
std::atomic<uint64_t> g_alloc_gen{0};

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        if (count <= n && p) return;
        release();
        if (count == 0) count = 1;
        HIPCHK(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
        n = count;
        g_alloc_gen.fetch_add(1);
    }
    void upload(const T* h, size_t count, hipStream_t st) {
        alloc(count);
        HIPCHK(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, st));
    }
};

template <typename T>
struct DevMatrix {
    DevBuf<T> K0, Kr, dK0;
    DevBuf<typename Vec4Of<T>::type> aux, daux;
    bool ready = false;
};

struct ProblemRec {
    HostOperator op;
    DevBuf<int32_t> row_ptr, col;
    DevBuf<double> w, u0;
    DevMatrix<double> A64;
    DevMatrix<float> A32;
    double dt_up = -1, theta_up = -1;  // sequence the K0/Kr on device were built for
    bool pattern_up = false;
    // Device pattern: CSR rows padded to a multiple of kRowPad; pad_src maps
    // a padded entry to its stored entry (-1 for padding).
    std::vector<int32_t> pad_row_ptr, pad_col;
    std::vector<int64_t> pad_src;
    // Per-DOF inputs of the learned-guess features (uploaded on first use).
    DevBuf<float4> feat_geo;
    DevBuf<float2> feat_flags;
    bool feat_up = false;
    // Anisotropic problems: compartment of each row, tensors [n_comp][6].
    DevBuf<int32_t> row_comp;
    DevBuf<double> comp_tensor;
    // Tetrahedra for the phase-weighted signal (uploaded on first use).
    DevBuf<int4> tet_dof, tet_node;
    DevBuf<double> node_xyz;
    bool tets_up = false;
    // Weak pseudo-periodic faces: partner couplings (rows = slots) and the
    // row -> slot map; the kappa_e scale the device K0 was built with.
    DevBuf<int32_t> wk_ptr, wk_col, wk_code, wk_map;
    DevBuf<double> wk_val;
    double wk_scale_up = -1;
    // Hash of the sparsity structure (form, DOF count, CSR pattern): the
    // problem's part of the autotuner cache key, stable across processes.
    uint64_t fingerprint = 0;
};

uint64_t fnv1a(uint64_t h, const void* data, size_t n) {
    const unsigned char* p = static_cast<const unsigned char*>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001B3ULL;
    }
    return h;
}

uint64_t structure_fingerprint(const HostOperator& op) {
    uint64_t h = 0xCBF29CE484222325ULL;
    h = fnv1a(h, &op.form, sizeof op.form);
    h = fnv1a(h, &op.n_dof, sizeof op.n_dof);
    h = fnv1a(h, op.row_ptr.data(), op.row_ptr.size() * sizeof(int32_t));
    h = fnv1a(h, op.col.data(), op.col.size() * sizeof(int32_t));
    return h;
}

void build_padded(ProblemRec& P) {
    const HostOperator& op = P.op;
    const int64_t n = op.n_dof;
    P.pad_row_ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t len = op.row_ptr[i + 1] - op.row_ptr[i];
        const int64_t padded = (len + kRowPad - 1) / kRowPad * kRowPad;
        P.pad_row_ptr[i + 1] = static_cast<int32_t>(P.pad_row_ptr[i] + padded);
    }
    const int64_t total = P.pad_row_ptr[n];
    P.pad_col.assign(total, 0);
    P.pad_src.assign(total, -1);
    for (int64_t i = 0; i < n; ++i) {
        int64_t d = P.pad_row_ptr[i];
        for (int64_t k = op.row_ptr[i]; k < op.row_ptr[i + 1]; ++k, ++d) {
            P.pad_col[d] = op.col[k];
            P.pad_src[d] = k;
        }
        for (; d < P.pad_row_ptr[i + 1]; ++d) P.pad_col[d] = static_cast<int32_t>(i);
    }
}

struct Options {
    int precision = 0;
    int krylov = 0;
    double rtol = 1e-10;
    double inner_rtol = 1e-4;
    double inner_floor = 0.25;  // inner FP32 solves stop at inner_floor * rtol ||b|| at the latest
    int max_iter = 2000;
    int guess = 1;
    int extrap_order = 3;
    int extrap_damp = 1;
    int sys_tile = 0;
    int graph = 0;
    int autotune = 0;
    int n_steps = 0;
    int blocks_per_xcd = 512;
    int max_outer = 8;
    int queue = 0;
    int grab = 4;
    int nt = 1;
    int lds = 0;
    int persistent = 2;
    int time_kernel = 0;
    int progress = 0;
    int ordering = 1;
    int pencil = 12;
    int concurrency = 1;
    int sort_systems = 1;
    int xcd_split = 0;
    int tile_sched = 1;
    int pair_lanes = 1;
    int signal = 1;
    int gmres_m = 30;
    double weak_kappa = 1.0;  // scale of kappa_e on weak pseudo-periodic faces
    int markers = 0;          // 1: roctx ranges around runs, batches and time steps
    int dir_bf16 = 1;         // paired FP32 inner solves keep their directions in BF16
    int spmv_rows = 2;        // rows a wavefront of the paired BF16 SpMV takes at once (1, 2)
    int mesh_merge = 0;       // runs over several meshes: 1 = one batch, each launch over all meshes
    // Krylov preconditioner of the FP64 Hermitian solves: 0 Jacobi (CG), 1
    // Chebyshev polynomial in D^-1 A on the interval the preconditioner
    // network predicts, 2 the same on the fixed interval [cheb_a, cheb_b];
    // 1 and 2 run flexible CG with Jacobi CG as the fallback.
    int precond = 0;
    int cheb_terms = 4;
    double cheb_a = kPcARef, cheb_b = kPcBRef;
};

// Per-system Krylov state arrays of one solver level.
struct StateBufs {
    DevBuf<double2> rho, alpha, beta;
    DevBuf<double> bb, rr;
    DevBuf<int32_t> active, iters, iters_total, flags, n_active;
    void alloc(size_t ld, size_t n_tiles) {
        rho.alloc(ld);
        alpha.alloc(ld);
        beta.alloc(ld);
        bb.alloc(ld);
        rr.alloc(ld);
        active.alloc(ld);
        iters.alloc(ld);
        iters_total.alloc(ld);
        flags.alloc(ld);
        n_active.alloc(n_tiles);
    }
    void reset(size_t ld, hipStream_t st) {
        HIPCHK(hipMemsetAsync(rho.p, 0, sizeof(double2) * ld, st));
        HIPCHK(hipMemsetAsync(alpha.p, 0, sizeof(double2) * ld, st));
        HIPCHK(hipMemsetAsync(beta.p, 0, sizeof(double2) * ld, st));
        HIPCHK(hipMemsetAsync(bb.p, 0, sizeof(double) * ld, st));
        HIPCHK(hipMemsetAsync(rr.p, 0, sizeof(double) * ld, st));
        HIPCHK(hipMemsetAsync(active.p, 0, sizeof(int32_t) * ld, st));
        HIPCHK(hipMemsetAsync(iters.p, 0, sizeof(int32_t) * ld, st));
        HIPCHK(hipMemsetAsync(iters_total.p, 0, sizeof(int32_t) * ld, st));
        HIPCHK(hipMemsetAsync(flags.p, 0, sizeof(int32_t) * ld, st));
    }
    SolverState view(int32_t n_sys, int32_t max_iter, double rtol2) {
        SolverState s{};
        s.rho = rho.p;
        s.alpha = alpha.p;
        s.beta = beta.p;
        s.bb = bb.p;
        s.rr = rr.p;
        s.active = active.p;
        s.iters = iters.p;
        s.iters_total = iters_total.p;
        s.flags = flags.p;
        s.n_active = n_active.p;
        s.n_sys = n_sys;
        s.max_iter = max_iter;
        s.rtol2 = rtol2;
        s.floor_bb = nullptr;
        s.floor_scale = 0.0;
        return s;
    }
};

// Per-batch device workspace (grow-only, reused across runs).
struct Workspace {
    DevBuf<double> vec64[kMaxHist + 5];
    DevBuf<float> vec32[kMaxHist + 5];
    DevBuf<double4> gq;
    DevBuf<double2> sig;
    DevBuf<double> partial, b_in, q_in;
    DevBuf<double> fin_stage;  // group sums of the two-stage finalize
    DevBuf<int32_t> ctr, bad;
    DevBuf<uint32_t> barrier;  // count, generation, error flag of the persistent solver
    StateBufs outer, inner;
    // GMRES(m): Krylov basis and per-system cycle state
    DevBuf<double2> gm_basis, gm_H, gm_sn, gm_g, gm_y;
    DevBuf<double> gm_partial, gm_hout, gm_cs, gm_hnorm;
    DevBuf<double> acomp;  // [n_comp][ld] q.D_k q per system (anisotropic problems)
    DevBuf<double> wb;     // [slots][ld] complex partner terms of weak faces
    // Polynomial preconditioner: two term vectors y, the update d, the
    // per-system interval, the network's inputs and outputs, and the CG
    // coefficients of the recorder.
    DevBuf<double> pc_y[2], pc_d;
    DevBuf<double2> pc_ab, pc_hist;
    DevBuf<float> pc_X, pc_Y;
    DevBuf<int32_t> gm_cycle, gm_dim;
    DevBuf<int64_t> mtab;  // per tile {first row, end row, element base, part rows}, several meshes
    int32_t* h_active[2] = {nullptr, nullptr};  // pinned
    size_t h_active_n = 0;
    ~Workspace() {
        for (auto& p : h_active)
            if (p) (void)hipHostFree(p);
    }
    void pinned(size_t n) {
        if (n <= h_active_n) return;
        for (auto& p : h_active) {
            if (p) (void)hipHostFree(p);
            p = nullptr;
            HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&p), n * sizeof(int32_t), 0));
        }
        h_active_n = n;
    }
};

// Captured time loop of the persistent path, replayed while its key (every
// pointer and scalar baked into the launches) is unchanged.
struct GraphCache {
    std::vector<uint64_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* final_u = nullptr;  // u^N after the loop
    uint64_t last_use = 0;
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
        final_u = nullptr;
    }
    ~GraphCache() { reset(); }
};

// One execution lane: a stream with its own workspace, polling events,
// timing-event pool and captured graph.
// Row layout of a batch over several meshes (their rows concatenated): per
// tile {first row, end row, element base, rows per part} (also uploaded to
// Workspace::mtab), the elements of one vector, and the largest mesh's row
// count.
struct MeshLayout {
    std::vector<int64_t> tab;
    int64_t vlen = 0;
    int64_t max_rows = 0;
};

struct Lane {
    hipStream_t stream = nullptr;
    Workspace ws;
    const MeshLayout* layout = nullptr;  // set while a several-mesh batch runs
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> tpool;  // timing events, reused across runs
    // Captured time loops (one per kind of batch, e.g. per mesh of a
    // multi-mesh run); the least recently used is replaced.
    static constexpr int kGraphs = 8;
    GraphCache graphs[kGraphs];
    uint64_t graph_clock = 0;
    GraphCache& graph_for(const std::vector<uint64_t>& key, bool& hit) {
        GraphCache* victim = &graphs[0];
        for (GraphCache& gc : graphs) {
            if (gc.exec && gc.key == key) {
                hit = true;
                gc.last_use = ++graph_clock;
                return gc;
            }
            if (gc.last_use < victim->last_use) victim = &gc;
        }
        hit = false;
        victim->reset();
        victim->last_use = ++graph_clock;
        return *victim;
    }
    void create() {
        HIPCHK(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    }
    ~Lane() {
        if (stream) (void)hipStreamSynchronize(stream);
        for (GraphCache& gc : graphs) gc.reset();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : tpool) (void)hipEventDestroy(e);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

// Launch configuration picked by the autotuner for one kind of batch.
struct TuneChoice {
    int sys_tile = -1, blocks_per_xcd = -1, persistent = -1, lds = -1;
    double seconds = 0.0;  // trial time of the chosen configuration
    int trials = 0;
};

// Learned-guess network: FP32 parameters, Adam moments, gradient scratch,
// and the sample recorder registered by dmri_guess_record.
struct GuessModel {
    DevBuf<float> theta, adam_m, adam_v, grad, partial, loss_hist;
    int adam_t = 0;
    bool set = false;
    float* rec_X = nullptr;
    float* rec_T = nullptr;
    int64_t rec_cap = 0, rec_count = 0;
    int64_t rec_stride = 1;
    DevBuf<int64_t> rec_count_dev;  // sample count kept on the device (preconditioner)
};

}  // namespace
}  // namespace dmri

struct dmri_ctx {
    int device = -1;
    bool host_only = true;
    std::string last_error = "no error";
    std::vector<std::unique_ptr<dmri::ProblemRec>> problems;
    bool seq_set = false;
    double dt = 0, theta = 0.5;
    int n_steps = 0;
    dmri::SequenceTables seq;  // F, one-sided f and int F^2 on the time grid
    uint64_t seq_gen = 0;      // bumped by every sequence change
    dmri::Options opt;
    dmri::GuessModel model;
    // Network of the preconditioner's interval (same shape as the guess
    // network) and its recorder of Ritz-value samples.
    dmri::GuessModel pcmodel;
    std::atomic<int64_t> pc_fallbacks{0};  // steps re-solved by Jacobi CG
    std::map<std::string, dmri::TuneChoice> tuned;  // autotuner cache
    std::string device_tag = "host";  // architecture and CU count, in cache keys
    dmri::TuneChoice last_tune;
    std::mutex tuned_mu;  // the cache and last_tune (lanes tune one at a time)
    // Krylov iterations each (problem, b, q) system needed in its last run:
    // the order in which later batches tile their systems.
    std::map<std::string, int64_t> sys_cost;
    std::mutex sys_cost_mu;
    // Execution lanes: lane 0 serves the calling thread; runs over several
    // problems may use more lanes, one host thread each.
    std::vector<std::unique_ptr<dmri::Lane>> lanes;
    // Problems formed by concatenating several problems' operators (block
    // diagonal), keyed by the member ids: the operator of a several-mesh batch.
    std::map<std::vector<int32_t>, std::unique_ptr<dmri::ProblemRec>> merged;
    // Device address of this device's copy of the file-scope scratch array
    // (the buffers of dmri_run_device_noalloc), looked up at creation.
    void* scratch_dev = nullptr;
};

namespace dmri {
namespace {

// The lane of the calling thread (set by the multi-problem scheduler).
thread_local Lane* tl_lane = nullptr;

Lane& lane(dmri_ctx* h) { return tl_lane ? *tl_lane : *h->lanes[0]; }

// Options of the calling thread's run: the handle's, or a private copy in the
// lane threads of a multi-problem run, so concurrent lanes (and the
// autotuner's trial settings inside one of them) never share one.
thread_local Options* tl_opt = nullptr;
Options& opts(dmri_ctx* h) { return tl_opt ? *tl_opt : h->opt; }
const Options& opts(const dmri_ctx* h) { return tl_opt ? *tl_opt : h->opt; }

std::string sys_key(int32_t pid, double b, const double* q) {
    std::string k(reinterpret_cast<const char*>(&pid), sizeof pid);
    k.append(reinterpret_cast<const char*>(&b), sizeof b);
    k.append(reinterpret_cast<const char*>(q), 3 * sizeof(double));
    return k;
}

// Order of the systems of a batch for tiling: by the iterations each needed
// in its last run when every system has one, otherwise by b (larger b needs
// more iterations). Stable, so ties keep the input order.
void order_systems(dmri_ctx* h, int32_t pid, const double* b, const double* q,
                   std::vector<int64_t>& idx) {
    std::vector<int64_t> cost(idx.size(), -1);
    bool all = true;
    {
        std::lock_guard<std::mutex> lock(h->sys_cost_mu);
        for (size_t i = 0; i < idx.size(); ++i) {
            auto it = h->sys_cost.find(sys_key(pid, b[idx[i]], q + 3 * idx[i]));
            if (it == h->sys_cost.end()) {
                all = false;
                break;
            }
            cost[i] = it->second;
        }
    }
    std::vector<size_t> perm(idx.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = i;
    if (all)
        std::stable_sort(perm.begin(), perm.end(),
                         [&](size_t a, size_t c) { return cost[a] < cost[c]; });
    else
        std::stable_sort(perm.begin(), perm.end(),
                         [&](size_t a, size_t c) { return b[idx[a]] < b[idx[c]]; });
    std::vector<int64_t> out(idx.size());
    for (size_t i = 0; i < perm.size(); ++i) out[i] = idx[perm[i]];
    idx.swap(out);
}

void remember_costs(dmri_ctx* h, int32_t pid, const double* b, const double* q,
                    const std::vector<int64_t>& idx, const std::vector<int32_t>& iters) {
    std::lock_guard<std::mutex> lock(h->sys_cost_mu);
    for (size_t i = 0; i < idx.size() && i < iters.size(); ++i)
        h->sys_cost[sys_key(pid, b[idx[i]], q + 3 * idx[i])] = iters[i];
}

}  // namespace
}  // namespace dmri

namespace dmri {
namespace {

void need_device(dmri_ctx* h) {
    if (h->host_only) throw Error(DMRI_E_STATE, "host-only context (created with device -1)");
    HIPCHK(hipSetDevice(h->device));
}

// Build K0 = M/dt + theta R, Kr = M/dt - (1-theta) R, aux = {M_D, V} and the
// diagonal, in precision T, and upload them. Weak pseudo-periodic faces add
// kb K_B to K0 only (kb = theta times the kappa_e scale; the form a*), the
// right side keeps no face mass (L*).
template <typename T>
void upload_matrix(const ProblemRec& P, double dt, double th, double kb, DevMatrix<T>& A,
                   hipStream_t st) {
    using T4 = typename Vec4Of<T>::type;
    const HostOperator& op = P.op;
    const size_t total = P.pad_col.size(), n = static_cast<size_t>(op.n_dof);
    std::vector<T> K0(total, T(0)), Kr(total, T(0)), dK0(n);
    std::vector<T4> aux(total), daux(n);
    for (size_t d = 0; d < total; ++d) {
        const int64_t k = P.pad_src[d];
        T4 a;
        a.x = a.y = a.z = a.w = T(0);
        if (k >= 0) {
            K0[d] = static_cast<T>(op.M[k] / dt + th * op.R[k] + (op.KB.empty() ? 0.0 : kb * op.KB[k]));
            Kr[d] = static_cast<T>(op.M[k] / dt - (1.0 - th) * op.R[k]);
            a.x = static_cast<T>(op.MT[k]);
            a.y = static_cast<T>(op.V[0][k]);
            a.z = static_cast<T>(op.V[1][k]);
            a.w = static_cast<T>(op.V[2][k]);
        }
        aux[d] = a;
    }
    for (size_t i = 0; i < n; ++i) {
        const int64_t k = op.diag_pos[i];
        dK0[i] = static_cast<T>(op.M[k] / dt + th * op.R[k] + (op.KB.empty() ? 0.0 : kb * op.KB[k]));
        daux[i].x = static_cast<T>(op.MT[k]);
        daux[i].y = static_cast<T>(op.V[0][k]);
        daux[i].z = static_cast<T>(op.V[1][k]);
        daux[i].w = static_cast<T>(op.V[2][k]);
    }
    A.K0.upload(K0.data(), total, st);
    A.Kr.upload(Kr.data(), total, st);
    A.dK0.upload(dK0.data(), n, st);
    A.aux.upload(aux.data(), total, st);
    A.daux.upload(daux.data(), n, st);
    HIPCHK(hipStreamSynchronize(st));  // host staging vectors go out of scope
    A.ready = true;
}

void ensure_uploaded(dmri_ctx* h, ProblemRec& P, bool need32) {
    hipStream_t st = lane(h).stream;
    if (!P.pattern_up) {
        build_padded(P);
        P.row_ptr.upload(P.pad_row_ptr.data(), P.pad_row_ptr.size(), st);
        P.col.upload(P.pad_col.data(), P.pad_col.size(), st);
        P.w.upload(P.op.w.data(), P.op.w.size(), st);
        P.u0.upload(P.op.u0.data(), P.op.u0.size(), st);
        if (P.op.aniso) {
            P.row_comp.upload(P.op.dof_comp.data(), P.op.dof_comp.size(), st);
            P.comp_tensor.upload(P.op.comp_tensor.data(), P.op.comp_tensor.size(), st);
        }
        std::vector<int32_t> wmap;
        if (!P.op.wk_rows.empty()) {
            const HostOperator& op = P.op;
            wmap.assign(static_cast<size_t>(op.n_dof), -1);
            for (size_t sl = 0; sl < op.wk_rows.size(); ++sl)
                wmap[op.wk_rows[sl]] = static_cast<int32_t>(sl);
            P.wk_ptr.upload(op.wk_ptr.data(), op.wk_ptr.size(), st);
            P.wk_col.upload(op.wk_col.data(), op.wk_col.size(), st);
            P.wk_code.upload(op.wk_code.data(), op.wk_code.size(), st);
            P.wk_val.upload(op.wk_val.data(), op.wk_val.size(), st);
            P.wk_map.upload(wmap.data(), wmap.size(), st);
        }
        HIPCHK(hipStreamSynchronize(st));
        P.pattern_up = true;
    }
    const double wks = P.op.KB.empty() ? 1.0 : opts(h).weak_kappa;
    if (P.dt_up != h->dt || P.theta_up != h->theta || P.wk_scale_up != wks) {
        P.A64.ready = false;
        P.A32.ready = false;
        P.dt_up = h->dt;
        P.theta_up = h->theta;
        P.wk_scale_up = wks;
    }
    const double kb = h->theta * wks;
    if (!P.A64.ready) upload_matrix<double>(P, h->dt, h->theta, kb, P.A64, st);
    if (need32 && !P.A32.ready) upload_matrix<float>(P, h->dt, h->theta, kb, P.A32, st);
}

template <typename T>
MatView<T> view(ProblemRec& P, DevMatrix<T>& A) {
    MatView<T> v;
    v.row_ptr = P.row_ptr.p;
    v.col = P.col.p;
    v.K0 = A.K0.p;
    v.Kr = A.Kr.p;
    v.aux = A.aux.p;
    v.dK0 = A.dK0.p;
    v.daux = A.daux.p;
    v.n_rows = static_cast<int32_t>(P.op.n_dof);
    return v;
}

// Device view of a problem's weak pseudo-periodic faces (n_slots = 0 when
// it has none). The scheme of Appendix B keeps a constant field constant
// only with theta = 1/2 (implicit face mass theta, lagged partner 1 -
// theta), so other theta values are refused.
WeakView weak_view(const dmri_ctx* h, const ProblemRec& P) {
    WeakView w{};
    if (P.op.wk_rows.empty()) return w;
    if (std::fabs(h->theta - 0.5) > 1e-12)
        throw Error(DMRI_E_UNSUPPORTED,
                    "weak pseudo-periodic faces need the Crank-Nicolson scheme (theta = 1/2)");
    w.ptr = P.wk_ptr.p;
    w.col = P.wk_col.p;
    w.code = P.wk_code.p;
    w.val = P.wk_val.p;
    w.map = P.wk_map.p;
    w.n_slots = static_cast<int32_t>(P.op.wk_rows.size());
    for (int a = 0; a < 3; ++a) w.L[a] = P.op.box_len[a];
    return w;
}

int auto_tile(int64_t n_sys) {
    if (n_sys >= 64) return 64;
    if (n_sys >= 32) return 32;
    if (n_sys >= 16) return 16;
    return 8;
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// F(t^n) for n = 0..N (transformed form) and f(t^n-) for n = 1..N (U-form
// left side) of the current sequence.
void step_tables(const dmri_ctx* h, std::vector<double>& F, std::vector<double>& f) {
    F = h->seq.F;
    f = h->seq.f_end;
}

// Learned-guess inputs of step n (n >= 2): F (or f) at the last three
// levels and the step length.
MlpStep mlp_step(const dmri_ctx* h, bool tr, const std::vector<double>& F,
                 const std::vector<double>& f, int n) {
    const std::vector<double>& v = tr ? F : f;
    return MlpStep{v[n], v[n - 1], v[n - 2], h->dt};
}

MlpDofs ensure_features(dmri_ctx* h, ProblemRec& P) {
    if (!P.feat_up) {
        const HostOperator& op = P.op;
        const size_t n = static_cast<size_t>(op.n_dof);
        std::vector<float4> geo(n);
        std::vector<float2> fl(n);
        for (size_t i = 0; i < n; ++i) {
            geo[i] = make_float4(op.dof_xyz[3 * i], op.dof_xyz[3 * i + 1], op.dof_xyz[3 * i + 2],
                                 op.dof_D[i]);
            fl[i] = make_float2(static_cast<float>(op.dof_comp[i]), op.dof_membrane[i]);
        }
        P.feat_geo.upload(geo.data(), n, lane(h).stream);
        P.feat_flags.upload(fl.data(), n, lane(h).stream);
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        P.feat_up = true;
    }
    return MlpDofs{P.feat_geo.p, P.feat_flags.p};
}

// Solution history of the initial guess. ring[0..nh-1] hold u^{n-1},
// u^{n-2}, ... (newest first; `avail` of them are filled) and ring[nh] is the
// next solution x. After a step x becomes u^{n-1} and the oldest slot is
// reused for the next x.
template <typename V2>
struct History {
    std::vector<V2*> ring;
    int nh = 2, avail = 1;
    V2* u(int k) const { return ring[k]; }
    V2* x() const { return ring[nh]; }
    void advance() {
        V2* oldest = ring[nh - 1];
        for (int k = nh - 1; k >= 1; --k) ring[k] = ring[k - 1];
        ring[0] = ring[nh];
        ring[nh] = oldest;
        avail = std::min(avail + 1, nh);
    }
};

// History length needed by the guess options: polynomial extrapolation of
// order p uses p + 1 past solutions (p + 2 damped); the learned guess
// corrects the damped cubic and uses five.
int history_len(const dmri_ctx* h) {
    if (opts(h).guess == 2) return kMlpHist;
    if (opts(h).guess != 1) return 2;
    return std::min(kMaxHist, std::max(2, opts(h).extrap_order + 1 + (opts(h).extrap_damp ? 1 : 0)));
}

// Weights of the order-p polynomial through u^{n-1}, ..., u^{n-1-p} on equal
// steps, evaluated one step ahead: c_k = (-1)^k C(p+1, k+1).
void extrap_weights(int p, double* c) {
    for (int k = 0; k <= p; ++k) {
        double bin = 1.0;  // C(p+1, k+1)
        for (int i = 1; i <= k + 1; ++i) bin = bin * (p + 2 - i) / i;
        c[k] = (k & 1) ? -bin : bin;
    }
}

// Damped extrapolation over p + 2 past solutions: the weights c_0..c_{p+1}
// reproduce every polynomial of degree <= p one step ahead and give zero
// response to a sequence alternating in sign from step to step (the
// components the theta = 1/2 scheme barely damps, which the plain
// extrapolation amplifies by 2^(p+1)). Solves the (p+2) x (p+2) system
//   sum_k c_k k^j = (-1)^j (j = 0..p),  sum_k c_k (-1)^k = 0.
void extrap_weights_damped(int p, double* c) {
    const int n = p + 2;
    double A[kMaxHist][kMaxHist + 1];
    for (int j = 0; j <= p; ++j) {
        for (int k = 0; k < n; ++k) A[j][k] = std::pow(static_cast<double>(k), j);
        A[j][n] = (j & 1) ? -1.0 : 1.0;
    }
    for (int k = 0; k < n; ++k) A[p + 1][k] = (k & 1) ? -1.0 : 1.0;
    A[p + 1][n] = 0.0;
    for (int col = 0; col < n; ++col) {  // Gaussian elimination, partial pivoting
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        for (int k = 0; k <= n; ++k) std::swap(A[col][k], A[piv][k]);
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[r][col] / A[col][col];
            for (int k = col; k <= n; ++k) A[r][k] -= f * A[col][k];
        }
    }
    // The exact weights are dyadic rationals with denominator 2^(p+1) (for
    // p = 3: 49/16, -9/4, -13/8, 11/4, -15/16). Snapping the eliminated values
    // to that grid makes them exact, so they sum to exactly 1: a constant
    // history is then reproduced without a bias that a loose solve would keep.
    for (int k = 0; k < n; ++k) {
        const double v = A[k][n] / A[k][k];
        c[k] = std::round(v * 1024.0) / 1024.0;
    }
}

// Start of step n: writes the guess into hist.x() when it is not formed
// inside k_init, and returns k_init's guess mode (0 = u^{n-1}, 1 = linear
// extrapolation inside k_init, 2 = x already holds the guess).
template <typename T, typename Timer>
int prepare_guess(dmri_ctx* h, const Geom& g, const MlpDofs& dofs, bool tr,
                  const std::vector<double>& F, const std::vector<double>& f, int n,
                  int64_t n_sys, const History<typename Vec2Of<T>::type>& hs, Timer& timer) {
    const int og = opts(h).guess;
    if (og == 2 && hs.avail >= kMlpHist) {
        if constexpr (sizeof(T) == 8) {
            MlpHist mh{};
            extrap_weights_damped(3, mh.c);
            for (int k = 0; k < kMlpHist; ++k) mh.u[k] = hs.u(k);
            timer.run(5, [&] {
                launch_mlp_guess(lane(h).stream, g, h->model.theta.p, dofs, lane(h).ws.gq.p,
                                 mlp_step(h, tr, F, f, n), static_cast<int32_t>(n_sys), mh,
                                 hs.x());
            });
            return 2;
        }
    }
    // The first steps of the learned guess (history shorter than five) use
    // the same extrapolation as guess = 1 with the default cubic order.
    if (og == 1 || og == 2) {
        const int p = og == 1 ? opts(h).extrap_order : 3;
        ExtrapTerms<T> t{};
        if ((og == 2 || opts(h).extrap_damp) && hs.avail >= p + 2 && p + 2 <= kMaxHist) {
            t.m = p + 2;
            extrap_weights_damped(p, t.c);
        } else {
            const int m = std::min(p, hs.avail - 1);
            if (m <= 0) return 0;
            if (m == 1) return 1;
            t.m = m + 1;
            extrap_weights(m, t.c);
        }
        for (int k = 0; k < t.m; ++k) t.u[k] = hs.u(k);
        timer.run(6, [&] { launch_combine<T>(lane(h).stream, g, t, hs.x()); });
        return 2;
    }
    return 0;
}

// Append training samples of step n (history u^{n-1} .. u^{n-5}, solved
// un = u^n) while the registered recorder has room.
void record_samples(dmri_ctx* h, const Geom& g, const MlpDofs& dofs, bool tr,
                    const std::vector<double>& F, const std::vector<double>& f, int n,
                    int64_t n_sys, const History<double2>& hs, const double2* un) {
    GuessModel& M = h->model;
    if (n < 2 || hs.avail < kMlpHist || M.rec_cap <= 0 || M.rec_count >= M.rec_cap) return;
    MlpHist mh{};
    extrap_weights_damped(3, mh.c);
    for (int k = 0; k < kMlpHist; ++k) mh.u[k] = hs.u(k);
    const int64_t nv = static_cast<int64_t>(g.n_rows) * g.ld;
    const int64_t offset = static_cast<int64_t>((static_cast<uint64_t>(n) * 2654435761u) %
                                                static_cast<uint64_t>(M.rec_stride));
    if (offset >= nv) return;
    const int64_t cnt = (nv - offset + M.rec_stride - 1) / M.rec_stride;
    launch_mlp_record(lane(h).stream, g, dofs, lane(h).ws.gq.p, mlp_step(h, tr, F, f, n),
                      static_cast<int32_t>(n_sys), mh, un, M.rec_stride, offset, M.rec_count,
                      M.rec_cap, M.rec_X, M.rec_T);
    M.rec_count = std::min(M.rec_cap, M.rec_count + cnt);
}

void check_guess_setup(dmri_ctx* h, bool fp64_vectors) {
    const bool rec = h->model.rec_cap > 0;
    if (opts(h).guess == 2 && !h->model.set)
        throw Error(DMRI_E_STATE,
                    "guess = 2 needs network parameters (dmri_guess_set_params or "
                    "dmri_load_guess_model)");
    if ((opts(h).guess == 2 || rec) && !fp64_vectors)
        throw Error(DMRI_E_UNSUPPORTED,
                    "the learned guess and sample recording need FP64 solution vectors "
                    "(precision 0 or 1)");
}

// u^0 = u0 per DOF for every system (0 for padding systems): over the whole
// vector for one mesh, tile by tile (each over its own mesh's rows) for a
// several-mesh batch.
template <typename T>
void fill_initial(dmri_ctx* h, const Geom& g, const ProblemRec& P, int32_t n_sys,
                  typename Vec2Of<T>::type* x) {
    hipStream_t st = lane(h).stream;
    const MeshLayout* ml = lane(h).layout;
    if (!ml || !g.mtab) {
        launch_set_initial<T>(st, g, P.u0.p, n_sys, x);
        return;
    }
    for (int32_t t = 0; t < g.n_tiles; ++t) {
        const int64_t lo = ml->tab[4 * t], hi = ml->tab[4 * t + 1], base = ml->tab[4 * t + 2];
        const int32_t live = std::max(0, std::min(g.S, n_sys - t * g.S));
        launch_set_initial_block<T>(st, hi - lo, g.S, live, P.u0.p + lo, x + (base + lo * g.S));
    }
}

struct BatchResult {
    std::vector<double> sig;       // [n_sys][2]
    std::vector<int32_t> iters, flags;
    std::vector<double> rr, bb;
    int64_t total_iters = 0;
    int64_t spmv_rows = 0;
    int steps = 0;
    double t_solve = 0, t_signal = 0;
    int64_t n_timed = 0;
    double t_timed = 0;
};

// Brackets launches of one kernel with timing events from the context's pool.
struct KernelTimer {
    dmri_ctx* h;
    hipStream_t st;
    int which;
    size_t used = 0;
    KernelTimer(dmri_ctx* hh, hipStream_t s, int w) : h(hh), st(s), which(w) {}
    template <typename L>
    void run(int kind, L&& launch) {
        if (kind != which) {
            launch();
            return;
        }
        while (lane(h).tpool.size() < used + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            lane(h).tpool.push_back(e);
        }
        HIPCHK(hipEventRecord(lane(h).tpool[used], st));
        launch();
        HIPCHK(hipEventRecord(lane(h).tpool[used + 1], st));
        used += 2;
    }
    void collect(BatchResult& res) {
        HIPCHK(hipStreamSynchronize(st));
        double tot = 0.0;
        for (size_t i = 0; i + 1 < used; i += 2) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, lane(h).tpool[i], lane(h).tpool[i + 1]));
            tot += ms;
        }
        res.n_timed += static_cast<int64_t>(used / 2);
        res.t_timed += tot * 1e-3;
        used = 0;
    }
};

// Common set-up of a batch: geometry, per-system parameters, scratch.
// Row parts of a several-mesh batch: each tile's mesh in kMeshParts parts of
// whole chunks (chunk_rows rows, the streaming kernels' block chunk).
constexpr int kMeshParts = 8;
int64_t mesh_part_rows(int64_t rows, int64_t chunk_rows) {
    int64_t pr = (rows + kMeshParts - 1) / kMeshParts;
    pr = (pr + chunk_rows - 1) / chunk_rows * chunk_rows;
    return std::max<int64_t>(pr, chunk_rows);
}
int64_t mesh_chunk_rows(int S) { return make_geom(1, S, S, 1, 0, 1).chunk_rows; }

// A second geometry of a several-mesh batch (the persistent solver's, or
// GMRES's with fewer blocks per XCD) takes the batch's row layout: the same
// tile table and row parts, its own blocks per XCD.
void follow_mesh_layout(Geom& d, const Geom& g) {
    if (!g.mtab) return;
    d.mtab = g.mtab;
    d.vlen = g.vlen;
    d.tile_bytes_ok = 0;
    d.n_parts = g.n_parts;
    d.n_items = d.n_tiles * d.n_parts;
    d.part_rows = g.part_rows;
    const int32_t chunks = (d.part_rows + d.chunk_rows - 1) / d.chunk_rows;
    d.B = std::max(1, std::min(d.bpx, chunks));
}

struct BatchSetup {
    Geom g;
    Geom gi;        // geometry of the FP32 inner solves (g, or 128-system paired tiles)
    bool pair;      // inner solves use the paired-lane layout
    Geom gp;        // geometry of the persistent solver (one block per CU)
    bool persist;   // Krylov loop in one persistent launch per solve
    bool herm;
    Scratch sc;
    GridBarrier bar;
    int32_t ld_aniso = 0;  // row stride of the q.D_k q table (anisotropic problems)
};

BatchSetup setup_batch(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b,
                       const double* d_q, bool want_pair = false) {
    hipStream_t st = lane(h).stream;
    Workspace& W = lane(h).ws;
    BatchSetup bs{};
    bs.herm = (P.op.form == FORM_TRANSFORMED) ? (opts(h).krylov != 2) : false;
    if (P.op.form == FORM_UFORM && opts(h).krylov == 1)
        throw Error(DMRI_E_INVALID, "CG needs the Hermitian (periodic-box) operator; use COCG");
    const int S = opts(h).sys_tile ? opts(h).sys_tile : auto_tile(n_sys);
    bs.g = make_geom(static_cast<int32_t>(P.op.n_dof), static_cast<int32_t>(n_sys), S,
                     opts(h).blocks_per_xcd, opts(h).queue, opts(h).grab, opts(h).xcd_split != 0);
    bs.g.nt = opts(h).nt;
    bs.g.lds = opts(h).lds;
    if (const MeshLayout* ml = lane(h).layout) {
        // Several meshes: every tile is split into 8 parts of its own mesh's
        // rows (so every XCD takes an eighth of every mesh), vectors hold
        // only each tile's rows, and the kernels' paths that assume one row
        // range per launch stay off. part_rows and B follow the largest mesh.
        Geom& gm = bs.g;
        if (static_cast<int64_t>(gm.n_tiles) * 4 != static_cast<int64_t>(ml->tab.size()))
            throw Error(DMRI_E_STATE, "several-mesh layout does not match the batch");
        if (gm.lds || want_pair)
            throw Error(DMRI_E_UNSUPPORTED, "several-mesh batches: no LDS SpMV or paired tiles");
        gm.mtab = lane(h).ws.mtab.p;
        gm.vlen = ml->vlen;
        gm.tile_bytes_ok = 0;
        gm.n_parts = kMeshParts;
        gm.n_items = gm.n_tiles * gm.n_parts;
        gm.part_rows = static_cast<int32_t>(mesh_part_rows(ml->max_rows, gm.chunk_rows));
        const int32_t chunks = (gm.part_rows + gm.chunk_rows - 1) / gm.chunk_rows;
        gm.B = std::max(1, std::min(gm.bpx, chunks));
    }
    const Geom& g = bs.g;
    const size_t ld = static_cast<size_t>(g.ld);
    int n_cu = 0;
    HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
    bs.gp = make_geom(g.n_rows, static_cast<int32_t>(n_sys), S, std::max(1, n_cu / 8), 0, 1);
    bs.gp.nt = g.nt;
    bs.gp.lds = 0;
    follow_mesh_layout(bs.gp, g);  // the persistent solver's items follow a several-mesh layout
    // Auto: the persistent solver wins where launch latency dominates (small
    // batches on small meshes); chunked launches win once a phase has enough
    // work to hide the per-launch cost.
    const bool small = vec_elems(g) <= 131072;
    if (opts(h).krylov == 3 && opts(h).precision != 0)
        throw Error(DMRI_E_UNSUPPORTED, "GMRES (krylov = 3) runs in precision 0 (FP64)");
    bs.persist = (opts(h).persistent == 1 || (opts(h).persistent == 2 && small)) && g.ld <= 64 &&
                 opts(h).krylov != 3 && opts(h).precond == 0 && h->pcmodel.rec_cap == 0;
    // The grid barrier needs every block resident: otherwise chunked launches.
    if (bs.persist) {
        const bool fits = opts(h).precision != 0 ? persistent_fits<float>(bs.gp, bs.herm, n_cu)
                                                : persistent_fits<double>(bs.gp, bs.herm, n_cu);
        if (!fits) bs.persist = false;
    }
    // FP32 inner solves of wide batches: 128-system tiles, two systems per lane.
    bs.pair = want_pair && !bs.persist && S == 64 && n_sys > 64 && !g.queue &&
              static_cast<int64_t>(g.n_rows) * 1024 < (int64_t(1) << 31);
    bs.gi = g;
    if (bs.pair) {
        bs.gi = make_geom(g.n_rows, static_cast<int32_t>(n_sys), 128, opts(h).blocks_per_xcd, 0, 1,
                          opts(h).xcd_split != 0);
        bs.gi.nt = g.nt;
        bs.gi.lds = 0;
        bs.gi.dir16 = opts(h).dir_bf16;
        bs.gi.rows2 = opts(h).spmv_rows;
    }
    const Geom& gi = bs.gi;
    const size_t ld_max = std::max<size_t>(ld, static_cast<size_t>(gi.ld));
    // Launches restricted to the active tiles split a tile into up to 8 parts
    // (sched_geom); partials and counters are addressed by tile * n_parts + part.
    const int32_t items_max =
        std::max({g.n_items, gi.n_items, 8 * g.n_tiles, 8 * gi.n_tiles});
    W.gq.alloc(ld_max);
    const size_t part_n = std::max<size_t>(
        std::max<size_t>(static_cast<size_t>(std::max(g.n_items, 8 * g.n_tiles)) * g.B * S * 4,
                         static_cast<size_t>(std::max(gi.n_items, 8 * gi.n_tiles)) * gi.B *
                             gi.S * 4),
        2 * static_cast<size_t>(bs.gp.n_items) * bs.gp.B * S * 4);
    W.partial.alloc(part_n);
    {
        size_t cols = 0;  // tiles x tile width of the widest geometry
        for (const Geom* gg : {&g, &gi, static_cast<const Geom*>(&bs.gp)})
            cols = std::max(cols, static_cast<size_t>(gg->n_tiles) * gg->S);
        W.fin_stage.alloc(cols * kFinGroups * 4);
    }
    W.barrier.alloc(32 * 11);
    HIPCHK(hipMemsetAsync(W.barrier.p, 0, sizeof(uint32_t) * 32 * 11, st));
    bs.bar.count = W.barrier.p;
    bs.bar.gen = W.barrier.p + 32 * 9;
    bs.bar.err = reinterpret_cast<int32_t*>(W.barrier.p + 32 * 10);
    W.ctr.alloc(2 * static_cast<size_t>(items_max));
    W.bad.alloc(1);
    W.pinned(static_cast<size_t>(std::max(g.n_tiles, gi.n_tiles)));
    HIPCHK(hipMemsetAsync(W.ctr.p, 0, sizeof(int32_t) * 2 * items_max, st));
    HIPCHK(hipMemsetAsync(W.bad.p, 0, sizeof(int32_t), st));
    if (P.op.form == FORM_UFORM && !h->seq.has_f)
        throw Error(DMRI_E_STATE, "the U-form (walls) needs f on the time grid: the sequence "
                                  "table was given without f_start / f_end");
    const double intF2 = h->seq.int_F2;
    launch_sys_params(st, static_cast<int32_t>(n_sys), static_cast<int32_t>(ld_max), d_b, d_q,
                      intF2, W.gq.p, W.bad.p);
    if (P.op.aniso) {
        // q.D_k q per (compartment, system); layout [k][ld] of the vector layout
        // in use (the paired inner tiles have ld_max >= ld columns: one table of
        // ld_max per compartment serves both, systems index it directly).
        W.acomp.alloc(static_cast<size_t>(P.op.n_comp) * ld_max);
        launch_aniso_params(st, P.op.n_comp, static_cast<int32_t>(ld_max), W.gq.p,
                            P.comp_tensor.p, W.acomp.p);
        for (Geom* gg : {&bs.g, &bs.gi, &bs.gp}) {
            gg->comp = P.row_comp.p;
            gg->acomp = W.acomp.p;
            gg->acomp_ld = static_cast<int32_t>(ld_max);
        }
        bs.ld_aniso = static_cast<int32_t>(ld_max);
    }
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, W.bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) throw Error(DMRI_E_INVALID, "b must be finite and >= 0, q finite and nonzero when b > 0");
    bs.sc.partial = W.partial.p;
    bs.sc.ctr_spmv = W.ctr.p;
    bs.sc.ctr_init = W.ctr.p + items_max;
    bs.sc.stage = W.fin_stage.p;
    return bs;
}

// Sum of the per-tile active counts after the work enqueued so far.
int poll_active(dmri_ctx* h, const Geom& g, const SolverState& s) {
    HIPCHK(hipMemcpyAsync(lane(h).ws.h_active[0], s.n_active, sizeof(int32_t) * g.n_tiles,
                          hipMemcpyDeviceToHost, lane(h).stream));
    HIPCHK(hipStreamSynchronize(lane(h).stream));
    int tot = 0;
    for (int t = 0; t < g.n_tiles; ++t) tot += lane(h).ws.h_active[0][t];
    return tot;
}

// Host driver of a chunked Krylov loop: enqueues `iterate(gk, k)` for
// iterations k = done + 1, ... in chunks (the first of first_chunk, then 2),
// each followed by a copy of the per-tile active counts to pinned memory;
// the host reads chunk k's counts while chunk k + 1 runs, restricts later
// chunks to the tiles still active (option tile_sched) and stops when none
// is. Returns the iterations enqueued.
template <typename Iterate>
int chunked_loop(dmri_ctx* h, const Geom& g, const SolverState& s, int first_chunk,
                 int max_iter, Iterate&& iterate) {
    hipStream_t st = lane(h).stream;
    int done = 0, slot = 0;
    bool pending = false;
    int chunk = std::max(1, first_chunk);
    Geom gk = g;  // geometry of the next chunk: every tile, or the tiles still active
    std::vector<int32_t> live;
    for (;;) {
        for (int i = 0; i < chunk; ++i) iterate(gk, done + i + 1);
        done += chunk;
        HIPCHK(hipMemcpyAsync(lane(h).ws.h_active[slot], s.n_active, sizeof(int32_t) * g.n_tiles,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(lane(h).ev[slot], st));
        if (pending) {
            HIPCHK(hipEventSynchronize(lane(h).ev[slot ^ 1]));
            int tot = 0;
            live.clear();
            for (int t = 0; t < g.n_tiles; ++t) {
                const int32_t a = lane(h).ws.h_active[slot ^ 1][t];
                tot += a;
                if (a > 0) live.push_back(t);
            }
            if (tot == 0) {
                done -= chunk;  // the chunk just enqueued only early-exits
                break;
            }
            // A tile that has left the loop never re-enters it, so the tiles
            // active in these (older) counts cover the ones still active.
            if (opts(h).tile_sched)
                gk = sched_geom(g, live.data(), static_cast<int>(live.size()));
        }
        pending = true;
        slot ^= 1;
        chunk = 2;
        if (done > max_iter + 4) {
            HIPCHK(hipStreamSynchronize(st));
            break;
        }
    }
    return done;
}

// Krylov iterations on the systems active in s until none is left.
// Chunks of iterations are enqueued back to back; behind each chunk the
// per-tile active counts are copied to pinned memory, and the host checks
// chunk k's counts while chunk k+1 runs. Returns the iterations enqueued.
template <typename T>
int krylov_loop(dmri_ctx* h, const BatchSetup& bs, const MatView<T>& Av, const double4* gq,
                Coef lhs, typename Vec2Of<T>::type* x, typename Vec2Of<T>::type* r,
                typename Vec2Of<T>::type* p, typename Vec2Of<T>::type* q, SolverState s,
                KernelTimer& timer, int first_chunk, int max_iter) {
    hipStream_t st = lane(h).stream;
    if (bs.persist) {
        timer.run(1, [&] {
            launch_krylov_persistent<T>(st, bs.gp, Av, gq, lhs, bs.herm, x, r, p, q, s, bs.sc,
                                        bs.bar);
        });
        return 0;
    }
    return chunked_loop(h, bs.g, s, first_chunk, max_iter, [&](const Geom& gk, int32_t k_iter) {
        timer.run(1, [&] { launch_spmv_dot<T>(st, gk, Av, gq, lhs, bs.herm, p, q, s, bs.sc); });
        timer.run(2, [&] { launch_update<T>(st, gk, Av, gq, lhs, bs.herm, x, r, p, q, s, bs.sc); });
        timer.run(3, [&] { launch_pupdate<T>(st, gk, Av, gq, lhs, r, p, x, k_iter, s); });
    });
}

// Buffers of the polynomial preconditioner.
struct PcBufs {
    double2* y[2];
    double2* d;
    double2* ab;
};

// Flexible CG (Notay's FCG(1)) with the Chebyshev polynomial preconditioner
// on the systems active in s after the step start (k_init has formed r and
// p = D^-1 r): z0 = P(r0), p0 = z0, then per iteration q = A p, alpha =
// rho / (p^H q), x += alpha p, r -= alpha q, z = P(r), beta = -(q^H z) /
// (p^H q), rho = r^H z, p = z + beta p. Chunks and polling as krylov_loop.
// Returns the iterations enqueued.
int fcg_loop(dmri_ctx* h, const BatchSetup& bs, const MatView<double>& Av, const double4* gq,
             Coef lhs, double2* x, double2* r, double2* p, double2* q, const PcBufs& pb,
             SolverState s, KernelTimer& timer, int max_iter) {
    hipStream_t st = lane(h).stream;
    const int m = opts(h).cheb_terms;
    timer.run(7, [&] {
        // (no q yet: the start's q^H z is not used, r stands in for q)
        const double2* z = launch_cheb(st, bs.g, Av, gq, lhs, pb.ab, m, true, r, r, pb.y, pb.d, s,
                                       bs.sc);
        launch_pupdate_z(st, bs.g, z, p, x, -1, s);
    });
    return chunked_loop(h, bs.g, s, 2, max_iter, [&](const Geom& gk, int32_t k_iter) {
        timer.run(1, [&] { launch_spmv_dot<double>(st, gk, Av, gq, lhs, true, p, q, s, bs.sc); });
        timer.run(2, [&] {
            launch_update<double>(st, gk, Av, gq, lhs, true, x, r, p, q, s, bs.sc, true);
        });
        timer.run(7, [&] {
            const double2* z =
                launch_cheb(st, gk, Av, gq, lhs, pb.ab, m, false, r, q, pb.y, pb.d, s, bs.sc);
            launch_pupdate_z(st, gk, z, p, x, k_iter, s);
        });
    });
}

// Coefficients of step n: the left operator at t^n, the right one at
// t^{n-1} (transformed form: F at the grid points; U-form: the one-sided
// limits f(t^n-) and f(t^{n-1}+) on the step interval).
Coef lhs_coef(const dmri_ctx* h, bool tr, const std::vector<double>& F,
              const std::vector<double>& f, int n) {
    const double th = h->theta;
    return tr ? Coef{F[n], th, th} : Coef{f[n], 0.0, th};
}
Coef rhs_coef(const dmri_ctx* h, bool tr, const std::vector<double>& F,
              const std::vector<double>& f, int n) {
    (void)f;
    const double th = h->theta;
    return tr ? Coef{F[n - 1], -(1.0 - th), -(1.0 - th)}
              : Coef{h->seq.f_start[n], 0.0, -(1.0 - th)};
}

// roctx range for profiler timelines (option "markers"), popped on scope exit.
struct Marker {
    bool on;
    Marker(const dmri_ctx* h, const char* what, int64_t k = -1) : on(opts(h).markers != 0) {
        if (!on) return;
        char buf[64];
        if (k >= 0) std::snprintf(buf, sizeof buf, "dmri %s %lld", what, static_cast<long long>(k));
        else std::snprintf(buf, sizeof buf, "dmri %s", what);
        roctxRangePush(buf);
    }
    ~Marker() {
        if (on) roctxRangePop();
    }
    Marker(const Marker&) = delete;
    Marker& operator=(const Marker&) = delete;
};

void progress_line(dmri_ctx* h, int n, int N, int iters, double t0) {
    if (opts(h).progress > 0 && (n % opts(h).progress == 0 || n == N)) {
        std::fprintf(stderr, "[dmri] step %d/%d: %d iterations, %.2fs\n", n, N, iters,
                     now_s() - t0);
        std::fflush(stderr);
    }
}

TetView ensure_tets(dmri_ctx* h, ProblemRec& P) {
    if (!P.tets_up) {
        const HostOperator& op = P.op;
        const size_t m = op.tet_dof.size() / 4;
        hipStream_t st = lane(h).stream;
        P.tet_dof.upload(reinterpret_cast<const int4*>(op.tet_dof.data()), m, st);
        P.tet_node.upload(reinterpret_cast<const int4*>(op.tet_node.data()), m, st);
        P.node_xyz.upload(op.node_xyz.data(), op.node_xyz.size(), st);
        HIPCHK(hipStreamSynchronize(st));
        P.tets_up = true;
    }
    return TetView{P.tet_dof.p, P.tet_node.p, P.node_xyz.p,
                   static_cast<int32_t>(P.op.tet_dof.size() / 4)};
}

// Signal of the last step: S = sum_i w_i u_i when F(t^N) = 0 (or for the
// U-form, whose unknown is U itself); otherwise, with option "signal" = 1,
// the exact integral of u_h exp(-i G F q . x) over every tetrahedron (the
// physical field of the transformed form, Appendix A, at that time).
template <typename T>
void launch_step_signal(dmri_ctx* h, const BatchSetup& bs, ProblemRec& P,
                        const typename Vec2Of<T>::type* u, double2* d_sig, int64_t n_sys,
                        double F_end) {
    hipStream_t st = lane(h).stream;
    const bool phase = P.op.form == FORM_TRANSFORMED && F_end != 0.0 && opts(h).signal == 1;
    if (!phase) {
        launch_signal<T>(st, bs.g, P.w.p, u, d_sig, static_cast<int32_t>(n_sys), bs.sc);
        return;
    }
    // |k.x_l - mean| <= |k| (longest edge): the series needs it moderate.
    std::vector<double4> gq(static_cast<size_t>(n_sys));
    HIPCHK(hipMemcpyAsync(gq.data(), lane(h).ws.gq.p, sizeof(double4) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double gmax = 0.0;
    for (const double4& v : gq) gmax = std::max(gmax, v.x);
    if (gmax * std::fabs(F_end) * P.op.max_edge > 16.0)
        throw Error(DMRI_E_UNSUPPORTED,
                    "phase-weighted signal: |k| h above 16 rad (mesh too coarse for the "
                    "gradient); use option signal = 0 for sum w u");
    const TetView tv = ensure_tets(h, P);
    Geom gt = make_geom(tv.n_tets, static_cast<int32_t>(n_sys), bs.g.S, opts(h).blocks_per_xcd,
                        0, 1);
    Workspace& W = lane(h).ws;
    const size_t need = static_cast<size_t>(std::max(gt.n_items, 8 * gt.n_tiles)) * gt.B *
                        gt.S * 4;
    W.partial.alloc(need);
    Scratch sc = bs.sc;
    sc.partial = W.partial.p;
    launch_signal_phase<T>(st, bs.g, gt, tv, W.gq.p, F_end, u, d_sig, static_cast<int32_t>(n_sys),
                           sc);
}

template <typename T>
void collect_result(dmri_ctx* h, const BatchSetup& bs, ProblemRec& P, StateBufs& sb,
                    const typename Vec2Of<T>::type* u, double2* d_sig, int64_t n_sys,
                    BatchResult& res, double F_end) {
    hipStream_t st = lane(h).stream;
    const double t0 = now_s();
    launch_step_signal<T>(h, bs, P, u, d_sig, n_sys, F_end);
    res.iters.resize(n_sys);
    res.flags.resize(n_sys);
    res.rr.resize(n_sys);
    res.bb.resize(n_sys);
    HIPCHK(hipMemcpyAsync(res.flags.data(), sb.flags.p, sizeof(int32_t) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(res.rr.data(), sb.rr.p, sizeof(double) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(res.bb.data(), sb.bb.p, sizeof(double) * n_sys, hipMemcpyDeviceToHost, st));
    int32_t bar_err = 0;
    HIPCHK(hipMemcpyAsync(&bar_err, lane(h).ws.barrier.p + 32 * 10, sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bar_err != 0)
        throw Error(DMRI_E_DEVICE, "persistent solver: a grid barrier wait timed out");
    res.t_signal = now_s() - t0;
}

// Restarted GMRES(m) on the systems active in s after the step start
// (k_init has formed r = b - A x0, ||b||^2 and ||r||^2): cycles of up to m
// Arnoldi steps with right Jacobi preconditioning, each system leaving its
// cycle when |g_{j+1}| <= rtol ||b||; x += D^-1 V y after every cycle, the
// true residual b - A x restarts the next. Returns the Arnoldi steps taken.
int gmres_loop(dmri_ctx* h, const BatchSetup& bs, const MatView<double>& Av, const double4* gq,
               Coef lhs, double2* x, double2* r, double2* z, double2* w, const double2* b,
               SolverState s, int64_t n_sys) {
    hipStream_t st = lane(h).stream;
    Workspace& W = lane(h).ws;
    const Geom& g = bs.g;
    const int m = std::max(1, std::min(opts(h).gmres_m, kGmMax));
    const size_t ld = static_cast<size_t>(g.ld), nv = static_cast<size_t>(vec_elems(g));
    Geom gg = make_geom(g.n_rows, static_cast<int32_t>(n_sys), g.S,
                        std::min(64, opts(h).blocks_per_xcd), 0, 1);
    follow_mesh_layout(gg, g);
    gg.comp = g.comp;
    gg.acomp = g.acomp;
    gg.acomp_ld = g.acomp_ld;
    W.gm_basis.alloc(static_cast<size_t>(m + 1) * nv);
    W.gm_partial.alloc(static_cast<size_t>(std::max(gg.n_items, 8 * gg.n_tiles)) * gg.B * gg.S *
                       kGmVals);
    W.gm_hout.alloc(ld * kGmVals);
    W.gm_H.alloc(ld * (kGmMax + 1) * kGmMax);
    W.gm_cs.alloc(ld * kGmMax);
    W.gm_sn.alloc(ld * kGmMax);
    W.gm_g.alloc(ld * (kGmMax + 1));
    W.gm_y.alloc(ld * kGmMax);
    W.gm_hnorm.alloc(ld);
    W.gm_cycle.alloc(ld);
    W.gm_dim.alloc(ld);
    GmresState gm{W.gm_partial.p, W.gm_hout.p, W.gm_H.p,    W.gm_cs.p,    W.gm_sn.p,
                  W.gm_g.p,       W.gm_y.p,    W.gm_hnorm.p, W.gm_cycle.p, W.gm_dim.p};
    const GmresBasis V{W.gm_basis.p, nv};
    SolverState cyc = s;
    cyc.active = gm.cycle;
    const int32_t ns = static_cast<int32_t>(n_sys);
    int steps = 0;
    for (int cycle = 0;; ++cycle) {
        gmres_cycle_start(st, g, gm, s);
        if (poll_active(h, g, s) == 0) break;
        if (cycle > 0) {  // true residual of the updated x
            launch_spmv_dot<double>(st, g, Av, gq, lhs, bs.herm, x, w, cyc, bs.sc);
            gmres_residual(st, gg, b, w, r, gm, cyc);
        }
        gmres_givens(st, ns, -1, m, cycle == 0, gm, s);
        for (int col = 0; col < m; ++col) {
            gmres_scale(st, gg, Av, gq, lhs, col == 0 ? r : w, V.base + col * nv, z, gm, cyc);
            launch_spmv_dot<double>(st, g, Av, gq, lhs, bs.herm, z, w, cyc, bs.sc);
            gmres_orthogonalize(st, gg, w, V, col + 1, col, ns, gm, cyc);
            gmres_givens(st, ns, col, m, false, gm, s);
            ++steps;
            if ((col & 3) == 3 || col == m - 1) {
                gmres_count(st, g, gm, s);
                if (poll_active(h, g, s) == 0) break;
            }
        }
        gmres_update(st, gg, Av, gq, lhs, x, V, ns, gm);
        if (steps > opts(h).max_iter + m) break;
    }
    return steps;
}

// Solve one batch of systems on one problem in precision T throughout
// (all-FP64, or all-FP32 for testing). b/q are device pointers ([n_sys],
// [n_sys][3]); the signals go to d_sig ([n_sys] double2, device).
template <typename T>
void solve_batch(dmri_ctx* h, ProblemRec& P, DevMatrix<T>& A, int64_t n_sys, const double* d_b,
                 const double* d_q, double2* d_sig, BatchResult& res) {
    using V2 = typename Vec2Of<T>::type;
    hipStream_t st = lane(h).stream;
    Workspace& W = lane(h).ws;
    const BatchSetup bs = setup_batch(h, P, n_sys, d_b, d_q);
    const Geom& g = bs.g;
    const size_t nv = static_cast<size_t>(vec_elems(g)), ld = static_cast<size_t>(g.ld);
    DevBuf<T>* vecs;
    if constexpr (sizeof(T) == 8) vecs = W.vec64; else vecs = W.vec32;
    History<V2> hs;
    hs.nh = history_len(h);
    const bool gmres = opts(h).krylov == 3;
    for (int i = 0; i < hs.nh + (gmres ? 5 : 4); ++i) vecs[i].alloc(2 * nv);
    for (int i = 0; i <= hs.nh; ++i) hs.ring.push_back(reinterpret_cast<V2*>(vecs[i].p));
    V2* r = reinterpret_cast<V2*>(vecs[hs.nh + 1].p);
    V2* p = reinterpret_cast<V2*>(vecs[hs.nh + 2].p);
    V2* q = reinterpret_cast<V2*>(vecs[hs.nh + 3].p);
    V2* bv = gmres ? reinterpret_cast<V2*>(vecs[hs.nh + 4].p) : nullptr;  // b, for restarts
    W.outer.alloc(ld, g.n_tiles);
    W.outer.reset(ld, st);
    SolverState s = W.outer.view(static_cast<int32_t>(n_sys), opts(h).max_iter,
                                 opts(h).rtol * opts(h).rtol);
    const MatView<T> Av = view<T>(P, A);
    const WeakView wv = weak_view(h, P);
    V2* wb = nullptr;
    if (wv.n_slots > 0) {
        W.wb.alloc(2 * static_cast<size_t>(wv.n_slots) * ld);
        wb = reinterpret_cast<V2*>(W.wb.p);
    }
    const double wc = (1.0 - h->theta) * opts(h).weak_kappa;
    fill_initial<T>(h, g, P, s.n_sys, hs.u(0));
    std::vector<double> F, f;
    step_tables(h, F, f);
    const bool tr = P.op.form == FORM_TRANSFORMED;
    const int N = opts(h).n_steps > 0 ? std::min(opts(h).n_steps, h->n_steps) : h->n_steps;

    constexpr bool kF64 = sizeof(T) == 8;
    check_guess_setup(h, kF64);
    const bool learn = opts(h).guess == 2 || h->model.rec_cap > 0;
    const MlpDofs dofs = learn ? ensure_features(h, P) : MlpDofs{nullptr, nullptr};

    // Polynomial preconditioner (flexible CG) and its sample recorder.
    const bool pc = opts(h).precond != 0;
    GuessModel& PM = h->pcmodel;
    const bool pc_rec = PM.rec_cap > 0;
    PcBufs pb{};
    PcScalars ps{h->dt, h->theta, P.op.d_max, P.op.max_edge, P.op.kappa, 0.0};
    if (pc || pc_rec) {
        if (!kF64 || gmres || !bs.herm || g.queue)
            throw Error(DMRI_E_UNSUPPORTED,
                        "the polynomial preconditioner and its recorder run with CG on the "
                        "Hermitian (transformed) form in precision 0, without row queues");
        if (pc && pc_rec)
            throw Error(DMRI_E_UNSUPPORTED,
                        "preconditioner samples come from Jacobi CG runs (precond = 0)");
        if (opts(h).precond == 1 && !PM.set)
            throw Error(DMRI_E_STATE, "precond = 1 needs network parameters "
                                      "(dmri_precond_set_params)");
    }
    std::vector<int32_t> pc_prev, pc_cur;
    if (pc) {
        for (auto& v : W.pc_y) v.alloc(2 * nv);
        W.pc_d.alloc(2 * nv);
        W.pc_ab.alloc(ld);
        W.pc_X.alloc(ld * 16);
        W.pc_Y.alloc(ld * 2);
        pb.y[0] = reinterpret_cast<double2*>(W.pc_y[0].p);
        pb.y[1] = reinterpret_cast<double2*>(W.pc_y[1].p);
        pb.d = reinterpret_cast<double2*>(W.pc_d.p);
        pb.ab = W.pc_ab.p;
        pc_prev.assign(static_cast<size_t>(n_sys), 0);
        pc_cur.resize(static_cast<size_t>(n_sys));
    }
    if (pc_rec) {
        W.pc_hist.alloc(ld * kRitzMax);
        s.ab_hist = W.pc_hist.p;
    }

    KernelTimer timer(h, st, opts(h).time_kernel);
    const double t0 = now_s();
    int last_iters = 8;
    auto step = [&](int n) {
        const Marker mk(h, "step", n);
        const Coef lhs = lhs_coef(h, tr, F, f, n), rhs = rhs_coef(h, tr, F, f, n);
        const int gm = prepare_guess<T>(h, g, dofs, tr, F, f, n, n_sys, hs, timer);
        timer.run(4, [&] {
            if (wb) launch_weak_rhs<T>(st, g, wv, W.gq.p, s.n_sys, F[n], wc, hs.u(0), wb);
            launch_init<T>(st, g, Av, W.gq.p, lhs, rhs, bs.herm, gm, hs.u(0), hs.u(1), hs.x(), r,
                           p, nullptr, nullptr, bv, s, bs.sc, wb ? wv.map : nullptr, wb);
        });
        int done = 0;
        if constexpr (sizeof(T) == 8) {
            if (gmres)
                done = gmres_loop(h, bs, Av, W.gq.p, lhs, hs.x(), r, p, q, bv, s, n_sys);
        }
        if (!gmres && !pc)
            done = krylov_loop<T>(h, bs, Av, W.gq.p, lhs, hs.x(), r, p, q, s, timer,
                                  last_iters - 2, opts(h).max_iter);
        if constexpr (kF64) {
            if (pc) {
                ps.F = lhs.F;
                launch_pc_interval(st, static_cast<int32_t>(n_sys), static_cast<int32_t>(ld),
                                   W.gq.p, ps, opts(h).precond == 1 ? PM.theta.p : nullptr,
                                   opts(h).cheb_a, opts(h).cheb_b, W.pc_X.p, W.pc_Y.p, pb.ab);
                done = fcg_loop(h, bs, Av, W.gq.p, lhs, hs.x(), r, p, q, pb, s, timer,
                                opts(h).max_iter);
                // Jacobi CG re-solves the step from the flexible solve's x
                // when a system ended with a flag it did not have before.
                HIPCHK(hipMemcpyAsync(pc_cur.data(), s.flags, sizeof(int32_t) * n_sys,
                                      hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                if (pc_cur != pc_prev) {
                    HIPCHK(hipMemcpyAsync(s.flags, pc_prev.data(), sizeof(int32_t) * n_sys,
                                          hipMemcpyHostToDevice, st));
                    launch_init<T>(st, g, Av, W.gq.p, lhs, rhs, bs.herm, 2, hs.u(0), hs.u(1),
                                   hs.x(), r, p, nullptr, nullptr, bv, s, bs.sc,
                                   wb ? wv.map : nullptr, wb);
                    done += krylov_loop<T>(h, bs, Av, W.gq.p, lhs, hs.x(), r, p, q, s, timer,
                                           8, opts(h).max_iter);
                    HIPCHK(hipMemcpyAsync(pc_cur.data(), s.flags, sizeof(int32_t) * n_sys,
                                          hipMemcpyDeviceToHost, st));
                    HIPCHK(hipStreamSynchronize(st));
                    h->pc_fallbacks.fetch_add(1);
                }
                pc_prev.swap(pc_cur);
            }
            if (pc_rec) {
                ps.F = lhs.F;
                launch_pc_record(st, static_cast<int32_t>(n_sys), W.gq.p, ps, s, PM.rec_X,
                                 PM.rec_T, PM.rec_count_dev.p, PM.rec_cap);
            }
        }
        last_iters = done;
        if constexpr (kF64) {
            record_samples(h, g, dofs, tr, F, f, n, n_sys, hs, hs.x());
        }
        progress_line(h, n, N, done, t0);
        hs.advance();
    };
    // With the persistent solver no host decision is needed inside the time
    // loop, so the whole loop can be captured once and replayed.
    const bool use_graph = opts(h).graph && bs.persist && opts(h).time_kernel == 0 &&
                           h->model.rec_cap == 0 && opts(h).progress == 0;
    V2* u_final = nullptr;
    if (use_graph) {
        std::vector<uint64_t> key;
        auto kp = [&](const void* ptr) { key.push_back(reinterpret_cast<uintptr_t>(ptr)); };
        auto kd = [&](double v) {
            uint64_t bits;
            std::memcpy(&bits, &v, sizeof bits);
            key.push_back(bits);
        };
        key.push_back(g_alloc_gen.load());
        kp(&P);
        kp(Av.K0);
        kp(Av.aux);
        kp(W.gq.p);
        kp(bs.sc.partial);
        kp(bs.bar.count);
        kp(s.rho);
        kp(h->model.theta.p);
        for (V2* v : hs.ring) kp(v);
        kp(r);
        kp(p);
        kp(q);
        kp(wb);
        kd(wc);
        for (double v : {double(n_sys), double(N), double(sizeof(T)), double(bs.herm),
                         double(g.S), double(bs.gp.B), opts(h).rtol, double(opts(h).max_iter),
                         double(opts(h).guess), double(opts(h).extrap_order),
                         double(opts(h).extrap_damp), h->dt, h->theta,
                         double(h->seq_gen)})
            kd(v);
        if (const MeshLayout* ml = lane(h).layout)  // the tiles' meshes and rows
            for (int64_t v : ml->tab) key.push_back(static_cast<uint64_t>(v));
        bool hit = false;
        GraphCache& gc = lane(h).graph_for(key, hit);
        if (hit) {
            HIPCHK(hipGraphLaunch(gc.exec, st));
            u_final = static_cast<V2*>(gc.final_u);
        } else {
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                for (int n = 1; n <= N; ++n) step(n);
            } catch (...) {
                hipGraph_t broken = nullptr;
                (void)hipStreamEndCapture(st, &broken);
                if (broken) (void)hipGraphDestroy(broken);
                throw;
            }
            HIPCHK(hipStreamEndCapture(st, &gc.graph));
            HIPCHK(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
            gc.key = key;
            gc.final_u = hs.u(0);
            HIPCHK(hipGraphLaunch(gc.exec, st));
            u_final = hs.u(0);
        }
    } else {
        for (int n = 1; n <= N; ++n) step(n);
        u_final = hs.u(0);
    }
    HIPCHK(hipStreamSynchronize(st));
    res.t_solve = now_s() - t0;
    res.steps = N;
    timer.collect(res);
    collect_result<T>(h, bs, P, W.outer, u_final, d_sig, n_sys, res, h->seq.F[N]);
    HIPCHK(hipMemcpyAsync(res.iters.data(), W.outer.iters_total.p, sizeof(int32_t) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n_sys; ++i) res.total_iters += res.iters[i];
    res.spmv_rows = res.total_iters * g.n_rows;
}

// Geometries of one refinement pass from the outer per-tile active counts
// `cnt`: the FP64 tiles with a system above rtol (g_ref) and the inner tiles
// that hold their systems (g_in; the inner tiles may be wider).
void refine_sched(const int32_t* cnt, const Geom& g, const Geom& gi, int64_t n_sys, Geom& g_ref,
                  Geom& g_in) {
    std::vector<int32_t> live, live_in;
    for (int t = 0; t < g.n_tiles; ++t) {
        if (cnt[t] <= 0) continue;
        live.push_back(t);
        const int64_t s0 = static_cast<int64_t>(t) * g.S;
        const int64_t s1 = std::min(n_sys, s0 + g.S) - 1;
        for (int64_t ti = s0 / gi.S; ti <= s1 / gi.S; ++ti)
            if (live_in.empty() || live_in.back() < ti) live_in.push_back(static_cast<int32_t>(ti));
    }
    g_ref = sched_geom(g, live.data(), static_cast<int>(live.size()));
    g_in = sched_geom(gi, live_in.data(), static_cast<int>(live_in.size()));
}

// Mixed precision: FP64 time stepping (right-hand side, residual, solution,
// signal) around FP32 Krylov solves of the correction equation
//   A dx = r64,  x64 += dx,  r64 = b - A x64  (FP64 operator)
// repeated until ||r64|| <= rtol ||b|| (iterative refinement). The inner
// solves reduce the residual by inner_rtol and use FP32 matrices and vectors
// with FP64 dot products.
void solve_batch_mixed(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b,
                       const double* d_q, double2* d_sig, BatchResult& res) {
    hipStream_t st = lane(h).stream;
    Workspace& W = lane(h).ws;
    const BatchSetup bs = setup_batch(h, P, n_sys, d_b, d_q, opts(h).pair_lanes != 0);
    const Geom& g = bs.g;
    // Inner (FP32) solves run on bsi: the same geometry, or paired tiles.
    BatchSetup bsi = bs;
    bsi.g = bs.gi;
    Geom gr = g;  // refinement residual: dx in the inner layout
    gr.dx_pair = bs.pair ? 1 : 0;
    const size_t nv = static_cast<size_t>(vec_elems(g)), ld = static_cast<size_t>(g.ld);
    const size_t ldi = std::max(ld, static_cast<size_t>(bs.gi.ld));
    const size_t nvi = bs.pair ? static_cast<size_t>(g.n_rows) * ldi : nv;
    History<double2> hs;
    hs.nh = history_len(h);
    // FP64 level: history ring, r64, b64 (no FP64 direction vector: the
    // inner solves form their own). The refinement passes update x in place.
    for (int i = 0; i < hs.nh + 3; ++i) W.vec64[i].alloc(2 * nv);
    for (int i = 0; i < 4; ++i) W.vec32[i].alloc(2 * nvi);
    for (int i = 0; i <= hs.nh; ++i) hs.ring.push_back(reinterpret_cast<double2*>(W.vec64[i].p));
    double2* r64 = reinterpret_cast<double2*>(W.vec64[hs.nh + 1].p);
    double2* b64 = reinterpret_cast<double2*>(W.vec64[hs.nh + 2].p);  // right-hand side of the step
    float2* r32 = reinterpret_cast<float2*>(W.vec32[0].p);
    float2* dx = reinterpret_cast<float2*>(W.vec32[1].p);
    float2* p32 = reinterpret_cast<float2*>(W.vec32[2].p);
    float2* q32 = reinterpret_cast<float2*>(W.vec32[3].p);
    W.outer.alloc(ld, g.n_tiles);
    W.inner.alloc(ldi, std::max(g.n_tiles, bs.gi.n_tiles));
    W.outer.reset(ld, st);
    W.inner.reset(ldi, st);
    SolverState so = W.outer.view(static_cast<int32_t>(n_sys), opts(h).max_outer,
                                  opts(h).rtol * opts(h).rtol);
    SolverState si = W.inner.view(static_cast<int32_t>(n_sys), opts(h).max_iter,
                                  opts(h).inner_rtol * opts(h).inner_rtol);
    // An inner solve need not reduce its residual below a fraction f of the
    // outer target: ||r|| <= max(inner_rtol ||r64||, f rtol ||b||).
    si.floor_bb = W.outer.bb.p;
    {
        const double k = opts(h).inner_floor * opts(h).rtol / opts(h).inner_rtol;
        si.floor_scale = k * k;
    }
    const MatView<double> A64 = view<double>(P, P.A64);
    const MatView<float> A32 = view<float>(P, P.A32);
    const WeakView wv = weak_view(h, P);
    double2* wb = nullptr;
    if (wv.n_slots > 0) {
        W.wb.alloc(2 * static_cast<size_t>(wv.n_slots) * ld);
        wb = reinterpret_cast<double2*>(W.wb.p);
    }
    const double wc = (1.0 - h->theta) * opts(h).weak_kappa;
    fill_initial<double>(h, g, P, so.n_sys, hs.u(0));
    std::vector<double> F, f;
    step_tables(h, F, f);
    const bool tr = P.op.form == FORM_TRANSFORMED;
    const int N = opts(h).n_steps > 0 ? std::min(opts(h).n_steps, h->n_steps) : h->n_steps;
    std::vector<int32_t> flag_or(n_sys, 0);
    check_guess_setup(h, true);
    const bool learn = opts(h).guess == 2 || h->model.rec_cap > 0;
    const MlpDofs dofs = learn ? ensure_features(h, P) : MlpDofs{nullptr, nullptr};

    KernelTimer timer(h, st, opts(h).time_kernel);
    const double t0 = now_s();
    int last_first_pass = 8;
    for (int n = 1; n <= N; ++n) {
        const Marker mk(h, "step", n);
        const Coef lhs = lhs_coef(h, tr, F, f, n), rhs = rhs_coef(h, tr, F, f, n);
        const int gm = prepare_guess<double>(h, g, dofs, tr, F, f, n, n_sys, hs, timer);
        timer.run(4, [&] {
            if (wb) launch_weak_rhs<double>(st, g, wv, W.gq.p, so.n_sys, F[n], wc, hs.u(0), wb);
            launch_init<double>(st, g, A64, W.gq.p, lhs, rhs, bs.herm, gm, hs.u(0), hs.u(1),
                                hs.x(), r64, nullptr, nullptr, nullptr, b64, so, bs.sc,
                                wb ? wv.map : nullptr, wb);
        });
        int step_iters = 0;
        for (int pass = 0; pass < opts(h).max_outer; ++pass) {
            const int still = poll_active(h, g, so);
            if (opts(h).progress > 0 && n % opts(h).progress == 0) {
                std::fprintf(stderr, "[dmri] step %d refinement pass %d: %d systems above rtol\n",
                             n, pass, still);
                std::fflush(stderr);
            }
            if (still == 0) break;
            // Only the tiles that hold a system above rtol take part in the
            // pass (later passes typically have a handful of such systems):
            // the others keep x and r64, and their inner tiles stay idle.
            Geom g_ref = gr, g_in = bsi.g;
            if (opts(h).tile_sched)
                refine_sched(lane(h).ws.h_active[0], gr, bsi.g, so.n_sys, g_ref, g_in);
            launch_inner_start(st, g_in, A32, W.gq.p, lhs, bs.herm, r64, W.outer.active.p, r32, dx,
                               p32, si, bs.sc);
            const int it = krylov_loop<float>(h, bsi, A32, W.gq.p, lhs, dx, r32, p32, q32, si,
                                              timer, pass == 0 ? last_first_pass - 2 : 2,
                                              opts(h).max_iter);
            if (pass == 0) last_first_pass = it;
            step_iters += it;
            timer.run(4, [&] {
                launch_init<double>(st, g_ref, A64, W.gq.p, lhs, rhs, bs.herm, 4, hs.u(0), hs.u(1),
                                    hs.x(), r64, nullptr, dx, hs.x(), b64, so, bs.sc);
            });
        }
        if (poll_active(h, g, so) != 0) {
            // Outer refinement did not reach rtol within max_outer passes.
            std::vector<int32_t> act(n_sys);
            HIPCHK(hipMemcpy(act.data(), W.outer.active.p, sizeof(int32_t) * n_sys,
                             hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n_sys; ++i)
                if (act[i]) flag_or[i] |= 1;
        }
        record_samples(h, g, dofs, tr, F, f, n, n_sys, hs, hs.x());
        progress_line(h, n, N, step_iters, t0);
        hs.advance();
    }
    HIPCHK(hipStreamSynchronize(st));
    res.t_solve = now_s() - t0;
    res.steps = N;
    timer.collect(res);
    collect_result<double>(h, bs, P, W.outer, hs.u(0), d_sig, n_sys, res, h->seq.F[N]);
    std::vector<int32_t> inner_flags(n_sys);
    HIPCHK(hipMemcpyAsync(res.iters.data(), W.inner.iters_total.p, sizeof(int32_t) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(inner_flags.data(), W.inner.flags.p, sizeof(int32_t) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int64_t i = 0; i < n_sys; ++i) {
        res.total_iters += res.iters[i];
        // Inner max_iter hits are recovered by the next outer pass; only
        // non-finite inner residuals and outer failures are reported.
        res.flags[i] |= flag_or[i] | (inner_flags[i] & 2);
    }
    res.spmv_rows = res.total_iters * g.n_rows;
}

void fill_stats(dmri_stats* stats, const std::vector<int64_t>& owner_idx, const BatchResult& R,
                int64_t n_total) {
    if (!stats) return;
    for (size_t i = 0; i < owner_idx.size(); ++i) {
        const int64_t o = owner_idx[i];
        if (o < 0 || o >= n_total) continue;
        if (stats->iters_total) stats->iters_total[o] = R.iters[i];
        if (stats->converged) stats->converged[o] = R.flags[i] == 0 ? 1 : 0;
        if (stats->final_rel_res)
            stats->final_rel_res[o] = R.bb[i] > 0 ? std::sqrt(R.rr[i] / R.bb[i]) : 0.0;
    }
    stats->total_iterations += R.total_iters;
    stats->spmv_rows += R.spmv_rows;
    stats->n_steps = R.steps;
    stats->t_solve_s += R.t_solve;
    stats->t_signal_s += R.t_signal;
    stats->n_kernel_launches += R.n_timed;
    stats->t_kernel_s += R.t_timed;
}

void run_batch_with(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b,
                    const double* d_q, double2* d_sig, BatchResult& R) {
    if ((opts(h).precond != 0 || h->pcmodel.rec_cap > 0) && opts(h).precision != 0)
        throw Error(DMRI_E_UNSUPPORTED,
                    "the polynomial preconditioner and its recorder run in precision 0");
    if (opts(h).precision == 0) {
        solve_batch<double>(h, P, P.A64, n_sys, d_b, d_q, d_sig, R);
    } else if (opts(h).precision == 2) {
        solve_batch<float>(h, P, P.A32, n_sys, d_b, d_q, d_sig, R);
    } else {
        solve_batch_mixed(h, P, n_sys, d_b, d_q, d_sig, R);
    }
}

// Restores the context's options (and the sample recorder) on scope exit.
struct OptionGuard {
    dmri_ctx* h;
    Options saved;
    int64_t rec_cap, pc_rec_cap;
    explicit OptionGuard(dmri_ctx* hh)
        : h(hh), saved(opts(hh)), rec_cap(hh->model.rec_cap), pc_rec_cap(hh->pcmodel.rec_cap) {}
    ~OptionGuard() {
        opts(h) = saved;
        h->model.rec_cap = rec_cap;
        h->pcmodel.rec_cap = pc_rec_cap;
    }
};

// Autotuner: times the first few steps of the batch under each candidate
// launch configuration (tile width, blocks per XCD, persistent Krylov
// kernel, LDS-staged SpMV) and keeps the fastest. Trials write their
// signals to scratch and record no training samples.
TuneChoice autotune(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b,
                    const double* d_q) {
    OptionGuard guard(h);
    h->model.rec_cap = 0;
    h->pcmodel.rec_cap = 0;
    const int total = opts(h).n_steps > 0 ? std::min(opts(h).n_steps, h->n_steps) : h->n_steps;
    opts(h).n_steps = std::max(1, std::min(4, total));
    opts(h).signal = 0;  // trial signals are discarded
    opts(h).progress = 0;
    opts(h).time_kernel = 0;
    DevBuf<double2> sig;
    sig.alloc(static_cast<size_t>(n_sys));
    const int s0 = guard.saved.sys_tile ? guard.saved.sys_tile : auto_tile(n_sys);
    std::vector<TuneChoice> cands;
    for (int S : {s0, s0 / 2}) {
        if (S < 8) continue;
        for (int bpx : {256, 512, 1024}) {
            TuneChoice c;
            c.sys_tile = S;
            c.blocks_per_xcd = bpx;
            c.persistent = 0;
            c.lds = 0;
            cands.push_back(c);
        }
        if (S >= 32) {
            TuneChoice c;
            c.sys_tile = S;
            c.blocks_per_xcd = 512;
            c.persistent = 0;
            c.lds = 1;
            cands.push_back(c);
        }
        if ((n_sys + S - 1) / S * S <= 64) {
            TuneChoice c;
            c.sys_tile = S;
            c.blocks_per_xcd = 512;
            c.persistent = 1;
            c.lds = 0;
            cands.push_back(c);
        }
    }
    auto apply = [&](const TuneChoice& c) {
        opts(h).sys_tile = c.sys_tile;
        opts(h).blocks_per_xcd = c.blocks_per_xcd;
        opts(h).persistent = c.persistent;
        opts(h).lds = c.lds;
    };
    TuneChoice best;
    best.seconds = 1e300;
    {  // warm-up: allocations and first-touch costs stay out of the trials
        apply(cands.front());
        BatchResult R;
        run_batch_with(h, P, n_sys, d_b, d_q, sig.p, R);
    }
    int trials = 0;
    for (const TuneChoice& c : cands) {
        apply(c);
        BatchResult R;
        const double t0 = now_s();
        run_batch_with(h, P, n_sys, d_b, d_q, sig.p, R);
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        const double t = now_s() - t0;
        ++trials;
        if (t < best.seconds) {
            best = c;
            best.seconds = t;
        }
    }
    best.trials = trials;
    return best;
}

void run_batch(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b, const double* d_q,
               double2* d_sig, BatchResult& R) {
    const Marker mk(h, "batch", n_sys);
    if (!opts(h).autotune) {
        run_batch_with(h, P, n_sys, d_b, d_q, d_sig, R);
        return;
    }
    // Content-based key (device, mesh structure, batch shape, solver), so a
    // cache saved by dmri_save_tuning serves later processes.
    char fp[17];
    std::snprintf(fp, sizeof fp, "%016llx", static_cast<unsigned long long>(P.fingerprint));
    const std::string key = h->device_tag + "/" + fp + "/" + std::to_string(n_sys) + "/" +
                            std::to_string(opts(h).precision) + "/" +
                            std::to_string(opts(h).krylov) + "/" + std::to_string(opts(h).sys_tile);
    TuneChoice c;
    {
        std::lock_guard<std::mutex> lock(h->tuned_mu);
        auto it = h->tuned.find(key);
        if (it == h->tuned.end())
            it = h->tuned.emplace(key, autotune(h, P, n_sys, d_b, d_q)).first;
        c = it->second;
        h->last_tune = c;
    }
    OptionGuard guard(h);
    opts(h).sys_tile = c.sys_tile;
    opts(h).blocks_per_xcd = c.blocks_per_xcd;
    opts(h).persistent = c.persistent;
    opts(h).lds = c.lds;
    run_batch_with(h, P, n_sys, d_b, d_q, d_sig, R);
}

dmri_status set_err(dmri_ctx* h, dmri_status c, const std::string& m) {
    if (h) h->last_error = m;
    else g_create_error = m;
    return c;
}

template <typename Fn>
dmri_status guarded(dmri_ctx* h, Fn fn) {
    try {
        return fn();
    } catch (const Error& e) {
        return set_err(h, e.code, e.what());
    } catch (const std::bad_alloc&) {
        return set_err(h, DMRI_E_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_err(h, DMRI_E_DEVICE, e.what());
    } catch (...) {
        return set_err(h, DMRI_E_DEVICE, "unknown error");
    }
}

ProblemRec& get_problem(dmri_ctx* h, int32_t id) {
    if (id < 0 || id >= static_cast<int32_t>(h->problems.size()))
        throw Error(DMRI_E_STATE, "unknown problem id");
    return *h->problems[id];
}

void need_sequence(dmri_ctx* h) {
    if (!h->seq_set)
        throw Error(DMRI_E_STATE, "no sequence: call dmri_set_sequence_pgse, dmri_set_sequence or "
                                  "dmri_set_sequence_table first");
}

constexpr char kModelMagic[8] = {'D', 'M', 'R', 'I', 'M', 'L', 'P', '1'};

// New parameters; the Adam moments restart from zero.
void set_model_params(dmri_ctx* h, GuessModel& M, const float* host_theta) {
    hipStream_t st = lane(h).stream;
    M.theta.alloc(kMlpParams);
    M.adam_m.alloc(kMlpParams);
    M.adam_v.alloc(kMlpParams);
    M.grad.alloc(kMlpParams + 1);
    HIPCHK(hipMemcpyAsync(M.theta.p, host_theta, sizeof(float) * kMlpParams,
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(M.adam_m.p, 0, sizeof(float) * kMlpParams, st));
    HIPCHK(hipMemsetAsync(M.adam_v.p, 0, sizeof(float) * kMlpParams, st));
    HIPCHK(hipStreamSynchronize(st));
    M.adam_t = 0;
    M.set = true;
}

// Gradient and loss of the current parameters over n samples into M.grad.
void grad_pass(dmri_ctx* h, GuessModel& M, int64_t n, const float* X, const float* T) {
    int n_cu = 0;
    HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
    const int waves = std::max(4, 4 * n_cu);  // one block of four waves per CU
    M.partial.alloc(static_cast<size_t>(waves) * (kMlpParams + 1));
    launch_mlp_grad(lane(h).stream, n, X, T, M.theta.p, M.partial.p, waves, M.grad.p);
}


// n_iters full-batch Adam steps of network M on n device samples.
void train_model(dmri_ctx* h, GuessModel& M, int64_t n, const float* X, const float* T,
                 int32_t n_iters, double lr, double* loss_first, double* loss_last) {
    if (n < 1 || !X || !T || n_iters < 1)
        throw Error(DMRI_E_INVALID, "need n >= 1, n_iters >= 1 and sample buffers");
    if (!(lr > 0.0) || !std::isfinite(lr)) throw Error(DMRI_E_INVALID, "lr must be > 0");
    hipStream_t st = lane(h).stream;
    M.loss_hist.alloc(2);
    for (int32_t it = 0; it < n_iters; ++it) {
        grad_pass(h, M, n, X, T);
        if (it == 0)
            HIPCHK(hipMemcpyAsync(M.loss_hist.p, M.grad.p + kMlpParams, sizeof(float),
                                  hipMemcpyDeviceToDevice, st));
        if (it == n_iters - 1)
            HIPCHK(hipMemcpyAsync(M.loss_hist.p + 1, M.grad.p + kMlpParams, sizeof(float),
                                  hipMemcpyDeviceToDevice, st));
        ++M.adam_t;
        launch_adam(st, M.theta.p, M.adam_m.p, M.adam_v.p, M.grad.p, static_cast<float>(lr), 0.9f,
                    0.999f, 1e-8f, M.adam_t);
    }
    float lh[2] = {0.0f, 0.0f};
    HIPCHK(hipMemcpyAsync(lh, M.loss_hist.p, sizeof(lh), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (loss_first) *loss_first = lh[0];
    if (loss_last) *loss_last = lh[1];
}

}  // namespace
}  // namespace dmri

// Buffers of dmri_run_device_noalloc: every vector, partial sum, counter and
// per-system scalar of that entry point lives in this array, of which each
// device the library runs on holds one copy until the process ends. Host
// code never uses the name itself as an address (it is a host-side stand-in):
// it uses the device address looked up once per device with
// hipGetSymbolAddress (scratch_address below).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace dmri {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Makes S the handle's sequence.
void install_sequence(dmri_ctx* h, SequenceTables S) {
    h->dt = S.dt;
    h->theta = S.theta;
    h->n_steps = S.n_steps;
    h->seq = std::move(S);
    h->seq_set = true;
    ++h->seq_gen;
}

// Device address of `scratch` on `device`, which must be current. Looked up
// on the first call for a device and kept.
void* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices)
        throw Error(DMRI_E_UNSUPPORTED, "device ordinal above 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error(DMRI_E_DEVICE, "hipGetSymbolAddress gave a null address");
        g_scratch_ptr[device] = ptr;
    }
    return g_scratch_ptr[device];
}

}  // namespace
}  // namespace dmri

using namespace dmri;

extern "C" {

dmri_status dmri_create(int device_ordinal, dmri_handle* out) {
    if (!out) return set_err(nullptr, DMRI_E_INVALID, "out must not be NULL");
    *out = nullptr;
    return guarded(nullptr, [&]() -> dmri_status {
        std::unique_ptr<dmri_ctx> h(new dmri_ctx());
        if (device_ordinal >= 0) {
            int count = 0;
            HIPCHK(hipGetDeviceCount(&count));
            if (device_ordinal >= count) throw Error(DMRI_E_INVALID, "no such HIP device");
            HIPCHK(hipSetDevice(device_ordinal));
            h->device = device_ordinal;
            h->host_only = false;
            h->scratch_dev = scratch_address(device_ordinal);
            hipDeviceProp_t prop;
            HIPCHK(hipGetDeviceProperties(&prop, device_ordinal));
            std::string arch(prop.gcnArchName);
            for (char& c : arch)
                if (c == ' ' || c == '/') c = '_';
            h->device_tag = arch + "_cu" + std::to_string(prop.multiProcessorCount);
            h->lanes.push_back(std::make_unique<Lane>());
            h->lanes.back()->create();
        } else if (device_ordinal != -1) {
            throw Error(DMRI_E_INVALID, "device_ordinal must be >= 0 or -1 (host only)");
        }
        *out = h.release();
        return DMRI_OK;
    });
}

void dmri_destroy(dmri_handle h) {
    if (!h) return;
    try {
        if (!h->host_only) (void)hipSetDevice(h->device);
        h->lanes.clear();  // synchronizes and frees each lane's stream and workspace
        h->problems.clear();
    } catch (...) {
    }
    delete h;
}

const char* dmri_last_error(dmri_handle h) {
    return h ? h->last_error.c_str() : g_create_error.c_str();
}

}  // extern "C"

namespace dmri {
namespace {

dmri_status add_problem_impl(dmri_handle h, int64_t n_nodes, const double* xyz, int64_t n_tets,
                             const int32_t* tets, const int32_t* tet_label, int32_t n_comp,
                             const double* D, const double* Dt, const double* T2, const double* u0,
                             double kappa, const double box_lo[3], const double box_hi[3],
                             uint32_t periodic_mask, int32_t* problem_id) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!problem_id || !box_lo || !box_hi) throw Error(DMRI_E_INVALID, "NULL argument");
        MeshInput in;
        in.n_nodes = n_nodes;
        in.xyz = xyz;
        in.n_tets = n_tets;
        in.tets = tets;
        in.label = tet_label;
        in.n_comp = n_comp;
        in.D = D;
        in.Dt = Dt;
        in.T2 = T2;
        in.u0 = u0;
        in.kappa = kappa;
        for (int a = 0; a < 3; ++a) {
            in.lo[a] = box_lo[a];
            in.hi[a] = box_hi[a];
        }
        in.periodic_mask = periodic_mask;
        in.ordering = opts(h).ordering;
        in.pencil = opts(h).pencil;
        auto rec = std::make_unique<ProblemRec>();
        rec->op = assemble(in);
        rec->fingerprint = structure_fingerprint(rec->op);
        h->problems.push_back(std::move(rec));
        *problem_id = static_cast<int32_t>(h->problems.size() - 1);
        return DMRI_OK;
    });
}

}  // namespace
}  // namespace dmri

extern "C" {

dmri_status dmri_add_problem(dmri_handle h, int64_t n_nodes, const double* xyz, int64_t n_tets,
                             const int32_t* tets, const int32_t* tet_label, int32_t n_comp,
                             const double* D, const double* T2, const double* u0, double kappa,
                             const double box_lo[3], const double box_hi[3],
                             uint32_t periodic_mask, int32_t* problem_id) {
    if (!D) return set_err(h, DMRI_E_INVALID, "D must not be NULL");
    return add_problem_impl(h, n_nodes, xyz, n_tets, tets, tet_label, n_comp, D, nullptr, T2, u0,
                            kappa, box_lo, box_hi, periodic_mask, problem_id);
}

dmri_status dmri_add_problem_tensor(dmri_handle h, int64_t n_nodes, const double* xyz,
                                    int64_t n_tets, const int32_t* tets, const int32_t* tet_label,
                                    int32_t n_comp, const double* D_tensor, const double* T2,
                                    const double* u0, double kappa, const double box_lo[3],
                                    const double box_hi[3], uint32_t periodic_mask,
                                    int32_t* problem_id) {
    if (!D_tensor) return set_err(h, DMRI_E_INVALID, "D_tensor must not be NULL");
    return add_problem_impl(h, n_nodes, xyz, n_tets, tets, tet_label, n_comp, nullptr, D_tensor,
                            T2, u0, kappa, box_lo, box_hi, periodic_mask, problem_id);
}

dmri_status dmri_problem_info(dmri_handle h, int32_t problem_id, int64_t* n_dof, int64_t* nnz) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        ProblemRec& P = get_problem(h, problem_id);
        if (n_dof) *n_dof = P.op.n_dof;
        if (nnz) *nnz = P.op.nnz;
        return DMRI_OK;
    });
}

dmri_status dmri_export_operator(dmri_handle h, int32_t problem_id, int32_t* row_ptr, int32_t* col,
                                 double* vals, double* w, double* u0, int32_t* dof_comp,
                                 int32_t* dof_node) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        const HostOperator& op = get_problem(h, problem_id).op;
        const size_t nnz = static_cast<size_t>(op.nnz), n = static_cast<size_t>(op.n_dof);
        if (row_ptr) std::memcpy(row_ptr, op.row_ptr.data(), (n + 1) * sizeof(int32_t));
        if (col) std::memcpy(col, op.col.data(), nnz * sizeof(int32_t));
        if (vals) {
            const std::vector<double>* arr[6] = {&op.M, &op.R, &op.MD, &op.V[0], &op.V[1], &op.V[2]};
            for (int a = 0; a < 6; ++a) std::memcpy(vals + a * nnz, arr[a]->data(), nnz * sizeof(double));
        }
        if (w) std::memcpy(w, op.w.data(), n * sizeof(double));
        if (u0) std::memcpy(u0, op.u0.data(), n * sizeof(double));
        if (dof_comp) std::memcpy(dof_comp, op.dof_comp.data(), n * sizeof(int32_t));
        if (dof_node) std::memcpy(dof_node, op.dof_node.data(), n * sizeof(int32_t));
        return DMRI_OK;
    });
}

dmri_status dmri_export_weak(dmri_handle h, int32_t problem_id, int64_t* n_slots,
                             int64_t* n_entries, double* kappa_e, int32_t* rows, int32_t* ptr,
                             int32_t* col, int32_t* code, double* val, double* face_mass) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        const HostOperator& op = get_problem(h, problem_id).op;
        const size_t ns = op.wk_rows.size(), ne = op.wk_col.size();
        if (n_slots) *n_slots = static_cast<int64_t>(ns);
        if (n_entries) *n_entries = static_cast<int64_t>(ne);
        if (kappa_e) *kappa_e = op.kappa_e;
        if (ns == 0) return DMRI_OK;
        if (rows) std::memcpy(rows, op.wk_rows.data(), ns * sizeof(int32_t));
        if (ptr) std::memcpy(ptr, op.wk_ptr.data(), (ns + 1) * sizeof(int32_t));
        if (col) std::memcpy(col, op.wk_col.data(), ne * sizeof(int32_t));
        if (code) std::memcpy(code, op.wk_code.data(), ne * sizeof(int32_t));
        if (val) std::memcpy(val, op.wk_val.data(), ne * sizeof(double));
        if (face_mass) std::memcpy(face_mass, op.KB.data(), op.KB.size() * sizeof(double));
        return DMRI_OK;
    });
}

dmri_status dmri_set_sequence_pgse(dmri_handle h, double delta_us, double Delta_us, double dt_us,
                                   double theta) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        const double p[2] = {delta_us, Delta_us};
        install_sequence(h, make_sequence(DMRI_SEQ_PGSE, p, 2, dt_us, theta));
        return DMRI_OK;
    });
}

dmri_status dmri_set_sequence(dmri_handle h, int32_t kind, const double* params,
                              int32_t n_params, double dt_us, double theta) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        install_sequence(h, make_sequence(kind, params, n_params, dt_us, theta));
        return DMRI_OK;
    });
}

dmri_status dmri_set_sequence_table(dmri_handle h, int64_t n_steps, double dt_us, double theta,
                                    const double* F, const double* f_start, const double* f_end,
                                    double int_F2) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (n_steps < 1 || n_steps > 10000000) throw Error(DMRI_E_INVALID, "need 1 <= n_steps <= 1e7");
        if (!F) throw Error(DMRI_E_INVALID, "NULL F");
        if ((f_start == nullptr) != (f_end == nullptr))
            throw Error(DMRI_E_INVALID, "give both f_start and f_end, or neither");
        if (!std::isfinite(dt_us) || !(dt_us > 0)) throw Error(DMRI_E_INVALID, "need dt > 0");
        if (!std::isfinite(theta) || theta < 0.5 || theta > 1.0)
            throw Error(DMRI_E_INVALID, "theta must be in [1/2, 1]");
        if (!std::isfinite(int_F2) || !(int_F2 > 0)) throw Error(DMRI_E_INVALID, "need int_F2 > 0");
        SequenceTables S;
        S.dt = dt_us;
        S.theta = theta;
        S.n_steps = static_cast<int>(n_steps);
        S.F.assign(F, F + n_steps + 1);
        S.f_start.assign(n_steps + 1, 0.0);
        S.f_end.assign(n_steps + 1, 0.0);
        for (double v : S.F)
            if (!std::isfinite(v)) throw Error(DMRI_E_INVALID, "F must be finite");
        if (S.F[0] != 0.0) throw Error(DMRI_E_INVALID, "F(0) must be 0");
        if (f_start) {
            for (int64_t n = 0; n < n_steps; ++n) {
                if (!std::isfinite(f_start[n]) || !std::isfinite(f_end[n]))
                    throw Error(DMRI_E_INVALID, "f must be finite");
                S.f_start[n + 1] = f_start[n];
                S.f_end[n + 1] = f_end[n];
            }
            S.has_f = true;
        }
        S.int_F2 = int_F2;
        install_sequence(h, std::move(S));
        return DMRI_OK;
    });
}

dmri_status dmri_set_option(dmri_handle h, const char* key, double v) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!key) throw Error(DMRI_E_INVALID, "NULL key");
        if (!std::isfinite(v)) throw Error(DMRI_E_INVALID, "option value must be finite");
        const std::string k(key);
        auto as_int = [&](int lo, int hi) {
            if (v != std::floor(v) || v < lo || v > hi)
                throw Error(DMRI_E_INVALID, "option " + k + " out of range");
            return static_cast<int>(v);
        };
        Options& o = h->opt;
        if (k == "precision") o.precision = as_int(0, 2);
        else if (k == "krylov") o.krylov = as_int(0, 3);
        else if (k == "rtol") {
            if (!(v > 0 && v < 1)) throw Error(DMRI_E_INVALID, "rtol must be in (0, 1)");
            o.rtol = v;
        } else if (k == "inner_rtol") {
            if (!(v > 0 && v < 1)) throw Error(DMRI_E_INVALID, "inner_rtol must be in (0, 1)");
            o.inner_rtol = v;
        } else if (k == "inner_floor") {
            if (!(v > 0 && v <= 1)) throw Error(DMRI_E_INVALID, "inner_floor must be in (0, 1]");
            o.inner_floor = v;
        } else if (k == "max_iter") o.max_iter = as_int(1, 1000000);
        else if (k == "guess") o.guess = as_int(0, 2);
        else if (k == "extrap_order") o.extrap_order = as_int(1, kMaxHist - 1);
        else if (k == "extrap_damp") o.extrap_damp = as_int(0, 1);
        else if (k == "sys_tile") {
            int t = as_int(0, 64);
            if (t != 0 && t != 8 && t != 16 && t != 32 && t != 64)
                throw Error(DMRI_E_INVALID, "sys_tile must be 0, 8, 16, 32 or 64");
            o.sys_tile = t;
        } else if (k == "graph") o.graph = as_int(0, 1);
        else if (k == "autotune") o.autotune = as_int(0, 1);
        else if (k == "n_steps") o.n_steps = as_int(0, 10000000);
        else if (k == "blocks_per_xcd") o.blocks_per_xcd = as_int(1, 4096);
        else if (k == "max_outer") o.max_outer = as_int(1, 1000);
        else if (k == "queue") o.queue = as_int(0, 1);
        else if (k == "grab") o.grab = as_int(1, 1024);
        else if (k == "nt") o.nt = as_int(0, 1);
        else if (k == "lds") o.lds = as_int(0, 1);
        else if (k == "persistent") o.persistent = as_int(0, 2);
        else if (k == "time_kernel") o.time_kernel = as_int(0, 7);
        else if (k == "progress") o.progress = as_int(0, 1000000);
        else if (k == "ordering") o.ordering = as_int(0, 1);
        else if (k == "pencil") o.pencil = as_int(1, 4096);
        else if (k == "concurrency") o.concurrency = as_int(1, 16);
        else if (k == "sort_systems") o.sort_systems = as_int(0, 1);
        else if (k == "xcd_split") o.xcd_split = as_int(0, 1);
        else if (k == "tile_sched") o.tile_sched = as_int(0, 1);
        else if (k == "pair_lanes") o.pair_lanes = as_int(0, 1);
        else if (k == "signal") o.signal = as_int(0, 1);
        else if (k == "gmres_m") o.gmres_m = as_int(1, kGmMax);
        else if (k == "weak_kappa") {
            if (!(v > 0 && v <= 1e6)) throw Error(DMRI_E_INVALID, "weak_kappa must be in (0, 1e6]");
            o.weak_kappa = v;
        } else if (k == "markers") o.markers = as_int(0, 1);
        else if (k == "dir_bf16") o.dir_bf16 = as_int(0, 1);
        else if (k == "spmv_rows") o.spmv_rows = as_int(1, 2);
        else if (k == "mesh_merge") o.mesh_merge = as_int(0, 1);
        else if (k == "precond") o.precond = as_int(0, 2);
        else if (k == "cheb_terms") o.cheb_terms = as_int(1, 16);
        else if (k == "cheb_a" || k == "cheb_b") {
            const double a = k == "cheb_a" ? v : o.cheb_a, b = k == "cheb_b" ? v : o.cheb_b;
            if (!(a > 0.0 && b <= 1e6 && a * 1.001 < b))
                throw Error(DMRI_E_INVALID, "need 0 < cheb_a, cheb_a * 1.001 < cheb_b <= 1e6");
            o.cheb_a = a;
            o.cheb_b = b;
        } else throw Error(DMRI_E_INVALID, "unknown option " + k);
        return DMRI_OK;
    });
}

dmri_status dmri_get_option(dmri_handle h, const char* key, double* value) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!key || !value) throw Error(DMRI_E_INVALID, "NULL argument");
        const std::string k(key);
        const Options& o = h->opt;
        if (k == "precision") *value = o.precision;
        else if (k == "krylov") *value = o.krylov;
        else if (k == "rtol") *value = o.rtol;
        else if (k == "inner_rtol") *value = o.inner_rtol;
        else if (k == "inner_floor") *value = o.inner_floor;
        else if (k == "max_iter") *value = o.max_iter;
        else if (k == "guess") *value = o.guess;
        else if (k == "extrap_order") *value = o.extrap_order;
        else if (k == "extrap_damp") *value = o.extrap_damp;
        else if (k == "sys_tile") *value = o.sys_tile;
        else if (k == "graph") *value = o.graph;
        else if (k == "autotune") *value = o.autotune;
        else if (k == "n_steps") *value = o.n_steps;
        else if (k == "blocks_per_xcd") *value = o.blocks_per_xcd;
        else if (k == "max_outer") *value = o.max_outer;
        else if (k == "queue") *value = o.queue;
        else if (k == "grab") *value = o.grab;
        else if (k == "nt") *value = o.nt;
        else if (k == "lds") *value = o.lds;
        else if (k == "persistent") *value = o.persistent;
        else if (k == "time_kernel") *value = o.time_kernel;
        else if (k == "progress") *value = o.progress;
        else if (k == "ordering") *value = o.ordering;
        else if (k == "pencil") *value = o.pencil;
        else if (k == "concurrency") *value = o.concurrency;
        else if (k == "sort_systems") *value = o.sort_systems;
        else if (k == "xcd_split") *value = o.xcd_split;
        else if (k == "tile_sched") *value = o.tile_sched;
        else if (k == "pair_lanes") *value = o.pair_lanes;
        else if (k == "signal") *value = o.signal;
        else if (k == "gmres_m") *value = o.gmres_m;
        else if (k == "weak_kappa") *value = o.weak_kappa;
        else if (k == "markers") *value = o.markers;
        else if (k == "dir_bf16") *value = o.dir_bf16;
        else if (k == "spmv_rows") *value = o.spmv_rows;
        else if (k == "mesh_merge") *value = o.mesh_merge;
        else if (k == "precond") *value = o.precond;
        else if (k == "cheb_terms") *value = o.cheb_terms;
        else if (k == "cheb_a") *value = o.cheb_a;
        else if (k == "cheb_b") *value = o.cheb_b;
        else if (k == "pc_fallback_steps") *value = static_cast<double>(h->pc_fallbacks.load());
        else if (k == "tuned_sys_tile") *value = h->last_tune.sys_tile;
        else if (k == "tuned_blocks_per_xcd") *value = h->last_tune.blocks_per_xcd;
        else if (k == "tuned_persistent") *value = h->last_tune.persistent;
        else if (k == "tuned_lds") *value = h->last_tune.lds;
        else if (k == "tuned_trials") *value = h->last_tune.trials;
        else throw Error(DMRI_E_INVALID, "unknown option " + k);
        return DMRI_OK;
    });
}

dmri_status dmri_guess_set_params(dmri_handle h, const float* params, int64_t n_params) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!params || n_params != kMlpParams)
            throw Error(DMRI_E_INVALID, "params must hold DMRI_GUESS_N_PARAMS floats");
        set_model_params(h, h->model, params);
        return DMRI_OK;
    });
}

dmri_status dmri_guess_get_params(dmri_handle h, float* params, int64_t n_params) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!params || n_params != kMlpParams)
            throw Error(DMRI_E_INVALID, "params must hold DMRI_GUESS_N_PARAMS floats");
        if (!h->model.set) throw Error(DMRI_E_STATE, "no guess network parameters set");
        HIPCHK(hipMemcpyAsync(params, h->model.theta.p, sizeof(float) * kMlpParams,
                              hipMemcpyDeviceToHost, lane(h).stream));
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        return DMRI_OK;
    });
}

dmri_status dmri_load_guess_model(dmri_handle h, const char* path) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!path) throw Error(DMRI_E_INVALID, "NULL path");
        std::FILE* fp = std::fopen(path, "rb");
        if (!fp) throw Error(DMRI_E_INVALID, std::string("cannot open ") + path);
        char magic[8];
        int32_t dims[3];
        std::vector<float> theta(kMlpParams);
        const bool ok = std::fread(magic, 1, 8, fp) == 8 && std::fread(dims, 4, 3, fp) == 3 &&
                        std::fread(theta.data(), 4, kMlpParams, fp) ==
                            static_cast<size_t>(kMlpParams);
        std::fclose(fp);
        if (!ok || std::memcmp(magic, kModelMagic, 8) != 0 || dims[0] != kMlpIn ||
            dims[1] != kMlpHid || dims[2] != kMlpOut)
            throw Error(DMRI_E_INVALID, std::string("not a guess-network file: ") + path);
        set_model_params(h, h->model, theta.data());
        return DMRI_OK;
    });
}

// Autotuner cache file: a header line, then one line per entry
//   key sys_tile blocks_per_xcd persistent lds seconds
constexpr const char* kTuneHeader = "dmri-tuning-v1";

dmri_status dmri_save_tuning(dmri_handle h, const char* path) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!path) throw Error(DMRI_E_INVALID, "NULL path");
        std::lock_guard<std::mutex> lock(h->tuned_mu);
        std::FILE* fp = std::fopen(path, "w");
        if (!fp) throw Error(DMRI_E_INVALID, std::string("cannot create ") + path);
        bool ok = std::fprintf(fp, "%s\n", kTuneHeader) > 0;
        for (const auto& kv : h->tuned) {
            const TuneChoice& c = kv.second;
            ok = ok && std::fprintf(fp, "%s %d %d %d %d %.9g\n", kv.first.c_str(), c.sys_tile,
                                    c.blocks_per_xcd, c.persistent, c.lds, c.seconds) > 0;
        }
        const bool closed = std::fclose(fp) == 0;
        if (!ok || !closed) throw Error(DMRI_E_INVALID, std::string("write failed: ") + path);
        return DMRI_OK;
    });
}

dmri_status dmri_load_tuning(dmri_handle h, const char* path) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!path) throw Error(DMRI_E_INVALID, "NULL path");
        std::FILE* fp = std::fopen(path, "r");
        if (!fp) throw Error(DMRI_E_INVALID, std::string("cannot open ") + path);
        std::map<std::string, TuneChoice> got;
        char line[1024];
        bool header = false, bad = false;
        while (std::fgets(line, sizeof line, fp)) {
            std::string ln(line);
            while (!ln.empty() && (ln.back() == '\n' || ln.back() == '\r')) ln.pop_back();
            if (ln.empty()) continue;
            if (!header) {
                header = ln == kTuneHeader;
                if (!header) {
                    bad = true;
                    break;
                }
                continue;
            }
            char key[512];
            TuneChoice c;
            int used = 0;
            if (ln.size() >= sizeof key ||
                std::sscanf(ln.c_str(), "%511s %d %d %d %d %lf%n", key, &c.sys_tile,
                            &c.blocks_per_xcd, &c.persistent, &c.lds, &c.seconds, &used) != 6 ||
                used != static_cast<int>(ln.size()) ||
                !(c.sys_tile == 8 || c.sys_tile == 16 || c.sys_tile == 32 || c.sys_tile == 64) ||
                c.blocks_per_xcd < 1 || c.blocks_per_xcd > 4096 || c.persistent < 0 ||
                c.persistent > 2 || c.lds < 0 || c.lds > 1 || !std::isfinite(c.seconds)) {
                bad = true;
                break;
            }
            c.trials = 0;  // served from the file: no trial run in this process
            got[key] = c;
        }
        std::fclose(fp);
        if (bad || !header) throw Error(DMRI_E_INVALID, std::string("not a tuning file: ") + path);
        std::lock_guard<std::mutex> lock(h->tuned_mu);
        for (auto& kv : got) h->tuned[kv.first] = kv.second;
        return DMRI_OK;
    });
}

dmri_status dmri_save_guess_model(dmri_handle h, const char* path) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!path) throw Error(DMRI_E_INVALID, "NULL path");
        if (!h->model.set) throw Error(DMRI_E_STATE, "no guess network parameters set");
        std::vector<float> theta(kMlpParams);
        HIPCHK(hipMemcpyAsync(theta.data(), h->model.theta.p, sizeof(float) * kMlpParams,
                              hipMemcpyDeviceToHost, lane(h).stream));
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        std::FILE* fp = std::fopen(path, "wb");
        if (!fp) throw Error(DMRI_E_INVALID, std::string("cannot create ") + path);
        const int32_t dims[3] = {kMlpIn, kMlpHid, kMlpOut};
        const bool ok = std::fwrite(kModelMagic, 1, 8, fp) == 8 && std::fwrite(dims, 4, 3, fp) == 3 &&
                        std::fwrite(theta.data(), 4, kMlpParams, fp) ==
                            static_cast<size_t>(kMlpParams);
        const bool closed = std::fclose(fp) == 0;
        if (!ok || !closed) throw Error(DMRI_E_INVALID, std::string("write failed: ") + path);
        return DMRI_OK;
    });
}

dmri_status dmri_guess_record(dmri_handle h, float* d_features, float* d_targets,
                              int64_t capacity, int64_t stride) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (capacity < 0 || stride < 1) throw Error(DMRI_E_INVALID, "need capacity >= 0, stride >= 1");
        if (capacity > 0 && (!d_features || !d_targets))
            throw Error(DMRI_E_INVALID, "NULL sample buffer");
        GuessModel& M = h->model;
        M.rec_X = capacity > 0 ? d_features : nullptr;
        M.rec_T = capacity > 0 ? d_targets : nullptr;
        M.rec_cap = capacity;
        M.rec_stride = stride;
        M.rec_count = 0;
        return DMRI_OK;
    });
}

dmri_status dmri_guess_record_count(dmri_handle h, int64_t* count) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!count) throw Error(DMRI_E_INVALID, "NULL argument");
        *count = h->model.rec_count;
        return DMRI_OK;
    });
}

dmri_status dmri_guess_eval(dmri_handle h, int64_t n, const float* d_features,
                            const float* d_targets, float* d_out, float* d_grad, double* loss) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!h->model.set) throw Error(DMRI_E_STATE, "no guess network parameters set");
        if (n < 1 || !d_features) throw Error(DMRI_E_INVALID, "need n >= 1 and features");
        if ((d_grad || loss) && !d_targets)
            throw Error(DMRI_E_INVALID, "gradient and loss need targets");
        hipStream_t st = lane(h).stream;
        GuessModel& M = h->model;
        if (d_out) launch_mlp_forward(st, n, d_features, M.theta.p, d_out);
        if (d_grad || loss) {
            grad_pass(h, h->model, n, d_features, d_targets);
            if (d_grad)
                HIPCHK(hipMemcpyAsync(d_grad, M.grad.p, sizeof(float) * kMlpParams,
                                      hipMemcpyDeviceToDevice, st));
            if (loss) {
                float l = 0.0f;
                HIPCHK(hipMemcpyAsync(&l, M.grad.p + kMlpParams, sizeof(float),
                                      hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                *loss = l;
            }
        }
        HIPCHK(hipStreamSynchronize(st));
        return DMRI_OK;
    });
}

dmri_status dmri_guess_train(dmri_handle h, int64_t n, const float* d_features,
                             const float* d_targets, int32_t n_iters, double lr,
                             double* loss_first, double* loss_last) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!h->model.set) throw Error(DMRI_E_STATE, "no guess network parameters set");
        train_model(h, h->model, n, d_features, d_targets, n_iters, lr, loss_first, loss_last);
        return DMRI_OK;
    });
}

dmri_status dmri_precond_set_params(dmri_handle h, const float* params, int64_t n_params) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!params || n_params != kMlpParams)
            throw Error(DMRI_E_INVALID, "params must hold DMRI_PRECOND_N_PARAMS floats");
        set_model_params(h, h->pcmodel, params);
        return DMRI_OK;
    });
}

dmri_status dmri_precond_get_params(dmri_handle h, float* params, int64_t n_params) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!params || n_params != kMlpParams)
            throw Error(DMRI_E_INVALID, "params must hold DMRI_PRECOND_N_PARAMS floats");
        if (!h->pcmodel.set) throw Error(DMRI_E_STATE, "no preconditioner network parameters set");
        HIPCHK(hipMemcpyAsync(params, h->pcmodel.theta.p, sizeof(float) * kMlpParams,
                              hipMemcpyDeviceToHost, lane(h).stream));
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        return DMRI_OK;
    });
}

dmri_status dmri_precond_record(dmri_handle h, float* d_features, float* d_targets,
                                int64_t capacity) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (capacity < 0) throw Error(DMRI_E_INVALID, "need capacity >= 0");
        if (capacity > 0 && (!d_features || !d_targets))
            throw Error(DMRI_E_INVALID, "NULL sample buffer");
        GuessModel& M = h->pcmodel;
        M.rec_X = capacity > 0 ? d_features : nullptr;
        M.rec_T = capacity > 0 ? d_targets : nullptr;
        M.rec_cap = capacity;
        M.rec_count_dev.alloc(1);
        const int64_t zero = 0;
        HIPCHK(hipMemcpyAsync(M.rec_count_dev.p, &zero, sizeof zero, hipMemcpyHostToDevice,
                              lane(h).stream));
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        return DMRI_OK;
    });
}

dmri_status dmri_precond_record_count(dmri_handle h, int64_t* count) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!count) throw Error(DMRI_E_INVALID, "NULL argument");
        *count = 0;
        GuessModel& M = h->pcmodel;
        if (M.rec_count_dev.p) {
            need_device(h);
            HIPCHK(hipMemcpyAsync(count, M.rec_count_dev.p, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, lane(h).stream));
            HIPCHK(hipStreamSynchronize(lane(h).stream));
        }
        return DMRI_OK;
    });
}

dmri_status dmri_precond_train(dmri_handle h, int64_t n, const float* d_features,
                               const float* d_targets, int32_t n_iters, double lr,
                               double* loss_first, double* loss_last) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        if (!h->pcmodel.set) throw Error(DMRI_E_STATE, "no preconditioner network parameters set");
        train_model(h, h->pcmodel, n, d_features, d_targets, n_iters, lr, loss_first, loss_last);
        return DMRI_OK;
    });
}

// The scalar members of a run's statistics, zeroed for a run of n pairs; the
// caller-owned array pointers are left as they are.
static void reset_stats(dmri_stats* st, int64_t n) {
    if (!st) return;
    st->n_sys = n;
    st->total_iterations = 0;
    st->spmv_rows = 0;
    st->n_steps = 0;
    st->t_setup_s = st->t_solve_s = st->t_signal_s = 0.0;
    st->n_kernel_launches = 0;
    st->t_kernel_s = 0.0;
}

}  // extern "C"

namespace dmri {
namespace {

// Validates host pairs (problem ids, b >= 0, q nonzero when b > 0).
void check_pairs(dmri_ctx* h, int64_t n_pairs, const int32_t* problem_id, const double* b,
                 const double* q) {
    for (int64_t i = 0; i < n_pairs; ++i) {
        get_problem(h, problem_id[i]);
        const double nq = std::sqrt(q[3 * i] * q[3 * i] + q[3 * i + 1] * q[3 * i + 1] +
                                    q[3 * i + 2] * q[3 * i + 2]);
        if (!std::isfinite(b[i]) || b[i] < 0 || !std::isfinite(nq) || (b[i] > 0 && !(nq > 0)))
            throw Error(DMRI_E_INVALID, "b must be finite and >= 0, q finite and nonzero");
    }
}

// The block-diagonal concatenation of the listed problems (rows and
// columns of problem k shifted by the DOFs of problems 0..k-1), built once
// per list and kept in the handle: the operator of a several-mesh batch.
// Its members must share the form; diffusion tensors and weak faces are not
// supported here.
ProblemRec& merged_problem(dmri_ctx* h, const std::vector<int32_t>& pids) {
    auto it = h->merged.find(pids);
    if (it != h->merged.end()) return *it->second;
    auto M = std::make_unique<ProblemRec>();
    HostOperator& op = M->op;
    const HostOperator& first = get_problem(h, pids.front()).op;
    op.form = first.form;
    uint64_t fp = 0xCBF29CE484222325ULL;
    int64_t rows = 0, nnz = 0;
    for (int32_t pid : pids) {
        const ProblemRec& P = get_problem(h, pid);
        const HostOperator& m = P.op;
        if (m.form != op.form)
            throw Error(DMRI_E_UNSUPPORTED, "several-mesh batches need one form (all periodic "
                                            "boxes, or all walls)");
        if (m.aniso || !m.wk_rows.empty())
            throw Error(DMRI_E_UNSUPPORTED, "several-mesh batches: no diffusion tensors or weak "
                                            "pseudo-periodic faces");
        const int64_t mnz = static_cast<int64_t>(m.col.size());
        if (rows + m.n_dof > (int64_t(1) << 31) - 1 || nnz + mnz > (int64_t(1) << 31) - 1)
            throw Error(DMRI_E_UNSUPPORTED, "several-mesh batch too large for 32-bit indices");
        for (int64_t i = 0; i < m.n_dof; ++i) {
            op.row_ptr.push_back(static_cast<int32_t>(m.row_ptr[i] + nnz));
            op.diag_pos.push_back(static_cast<int32_t>(m.diag_pos[i] + nnz));
        }
        for (int32_t c : m.col) op.col.push_back(static_cast<int32_t>(c + rows));
        op.M.insert(op.M.end(), m.M.begin(), m.M.end());
        op.R.insert(op.R.end(), m.R.begin(), m.R.end());
        op.MT.insert(op.MT.end(), m.MT.begin(), m.MT.end());
        for (int a = 0; a < 3; ++a) op.V[a].insert(op.V[a].end(), m.V[a].begin(), m.V[a].end());
        op.w.insert(op.w.end(), m.w.begin(), m.w.end());
        op.u0.insert(op.u0.end(), m.u0.begin(), m.u0.end());
        fp = fnv1a(fp, &P.fingerprint, sizeof P.fingerprint);
        rows += m.n_dof;
        nnz += mnz;
    }
    op.row_ptr.push_back(static_cast<int32_t>(nnz));
    op.n_dof = rows;
    op.nnz = nnz;
    M->fingerprint = fp;
    ProblemRec& ref = *M;
    h->merged.emplace(pids, std::move(M));
    return ref;
}

// Several problems as one batch (option mesh_merge): the problems' operators
// concatenated block-diagonally, each problem's pairs ordered by cost and
// padded with b = 0 systems to whole tiles, so every tile belongs to one
// mesh. Each kernel launch then covers the tiles of all meshes, every tile
// over its own mesh's rows only (vectors hold just those rows). FP64 and
// mixed precision with CG/COCG and the polynomial-extrapolation guesses.
// Slots of a several-mesh batch at tile width S: per problem its pairs
// (cost order) then b = 0 padding to whole tiles, with the row layout.
struct MergedSlots {
    MeshLayout ml;
    std::vector<int64_t> owner;  // caller's pair index per slot, -1 for padding
    std::vector<double> b, q;
    std::vector<std::vector<int64_t>> order;  // per problem, its pairs in slot order
};

MergedSlots merged_slots(dmri_ctx* h,
                         const std::vector<std::pair<int32_t, std::vector<int64_t>>>& groups,
                         const double* b, const double* q, int S) {
    MergedSlots m;
    m.order.resize(groups.size());
    int64_t row0 = 0, elems = 0;
    const int64_t chunk_rows = mesh_chunk_rows(S);
    for (size_t k = 0; k < groups.size(); ++k) {
        const int32_t pid = groups[k].first;
        std::vector<int64_t> idx = groups[k].second;
        if (opts(h).sort_systems) order_systems(h, pid, b, q, idx);
        const int64_t rows = get_problem(h, pid).op.n_dof;
        const int64_t nt = (static_cast<int64_t>(idx.size()) + S - 1) / S;
        for (int64_t t = 0; t < nt; ++t) {
            m.ml.tab.push_back(row0);
            m.ml.tab.push_back(row0 + rows);
            m.ml.tab.push_back(elems - row0 * S);
            m.ml.tab.push_back(mesh_part_rows(rows, chunk_rows));
            elems += rows * S;
        }
        for (int64_t i = 0; i < nt * S; ++i) {
            const bool real = i < static_cast<int64_t>(idx.size());
            m.owner.push_back(real ? idx[i] : -1);
            m.b.push_back(real ? b[idx[i]] : 0.0);
            for (int a = 0; a < 3; ++a)
                m.q.push_back(real ? q[3 * idx[i] + a] : (a == 0 ? 1.0 : 0.0));
        }
        m.ml.max_rows = std::max(m.ml.max_rows, rows);
        row0 += rows;
        m.order[k] = std::move(idx);
    }
    m.ml.vlen = elems;
    if (static_cast<int64_t>(m.owner.size()) / S > 4096)
        throw Error(DMRI_E_UNSUPPORTED, "several-mesh batch: over 4096 tiles");
    return m;
}

// One run of a several-mesh batch with tile width S, blocks per XCD and the
// persistent-kernel option as given (the options are restored afterwards).
void run_merged_with(dmri_ctx* h, ProblemRec& M, const MergedSlots& m, int S, int bpx,
                     int persistent, double2* d_sig, BatchResult& R) {
    hipStream_t st = lane(h).stream;
    Workspace& W = lane(h).ws;
    const int64_t ns = static_cast<int64_t>(m.owner.size());
    W.mtab.upload(m.ml.tab.data(), m.ml.tab.size(), st);
    W.b_in.upload(m.b.data(), ns, st);
    W.q_in.upload(m.q.data(), 3 * ns, st);
    HIPCHK(hipStreamSynchronize(st));
    OptionGuard guard(h);
    opts(h).sys_tile = S;
    opts(h).blocks_per_xcd = bpx;
    opts(h).persistent = persistent;
    opts(h).pair_lanes = 0;
    struct LayoutScope {
        Lane& l;
        LayoutScope(Lane& ln, const MeshLayout* ml) : l(ln) { l.layout = ml; }
        ~LayoutScope() { l.layout = nullptr; }
    } scope(lane(h), &m.ml);
    const Marker mk(h, "batch", ns);
    run_batch_with(h, M, ns, W.b_in.p, W.q_in.p, d_sig, R);
}

// Autotuner of several-mesh batches: the first steps under each candidate
// (tile width S0 or S0 / 2, 256/512/1024 blocks per XCD, and the persistent
// kernel when all slots fit it), fastest kept; trials record nothing and
// write their signals to scratch.
TuneChoice autotune_merged(dmri_ctx* h, ProblemRec& M,
                           const std::vector<std::pair<int32_t, std::vector<int64_t>>>& groups,
                           const double* b, const double* q, int S0) {
    OptionGuard guard(h);
    const int total = opts(h).n_steps > 0 ? std::min(opts(h).n_steps, h->n_steps) : h->n_steps;
    opts(h).n_steps = std::max(1, std::min(4, total));
    opts(h).signal = 0;
    opts(h).progress = 0;
    opts(h).time_kernel = 0;
    opts(h).graph = 0;
    std::vector<TuneChoice> cands;
    for (int S : {S0, S0 / 2}) {
        if (S < 8 || (S != S0 && opts(h).sys_tile)) continue;
        for (int bpx : {256, 512, 1024}) {
            TuneChoice c;
            c.sys_tile = S;
            c.blocks_per_xcd = bpx;
            c.persistent = 0;
            c.lds = 0;
            cands.push_back(c);
        }
        size_t slots = 0;
        for (const auto& gr : groups) slots += (gr.second.size() + S - 1) / S * S;
        if (slots <= 64) {
            TuneChoice c;
            c.sys_tile = S;
            c.blocks_per_xcd = 512;
            c.persistent = 1;
            c.lds = 0;
            cands.push_back(c);
        }
    }
    TuneChoice best;
    best.seconds = 1e300;
    DevBuf<double2> sig;
    bool warm = false;
    int trials = 0;
    for (const TuneChoice& c : cands) {
        const MergedSlots m = merged_slots(h, groups, b, q, c.sys_tile);
        sig.alloc(m.owner.size());
        if (!warm) {  // allocations and first-touch costs stay out of the trials
            BatchResult R0;
            run_merged_with(h, M, m, c.sys_tile, c.blocks_per_xcd, c.persistent, sig.p, R0);
            warm = true;
        }
        BatchResult R;
        const double t0 = now_s();
        run_merged_with(h, M, m, c.sys_tile, c.blocks_per_xcd, c.persistent, sig.p, R);
        HIPCHK(hipStreamSynchronize(lane(h).stream));
        const double t = now_s() - t0;
        ++trials;
        if (t < best.seconds) {
            best = c;
            best.seconds = t;
        }
    }
    best.trials = trials;
    return best;
}

// Several problems as one batch (option mesh_merge): the problems' operators
// concatenated block-diagonally, each problem's pairs ordered by cost and
// padded with b = 0 systems to whole tiles, so every tile belongs to one
// mesh. Each kernel launch then covers the tiles of all meshes, every tile
// over its own mesh's rows only (vectors hold just those rows). FP64 and
// mixed precision with CG/COCG and the polynomial-extrapolation guesses;
// with option autotune the tile width, blocks per XCD and persistent kernel
// are tuned per kind of batch (cached with the other choices).
bool run_merged(dmri_ctx* h, const std::vector<std::pair<int32_t, std::vector<int64_t>>>& groups,
                int64_t n_pairs, const double* b, const double* q, double* signal_out,
                dmri_stats* stats) {
    const Options& o = opts(h);
    if (o.precond != 0 || o.guess == 2 || o.lds || h->model.rec_cap > 0 ||
        h->pcmodel.rec_cap > 0)
        throw Error(DMRI_E_UNSUPPORTED,
                    "several-mesh batches run without the LDS SpMV, the learned guess or "
                    "preconditioner, and sample recording");
    std::vector<int32_t> pids;
    size_t max_ns = 0;
    for (const auto& gr : groups) {
        pids.push_back(gr.first);
        max_ns = std::max(max_ns, gr.second.size());
    }
    int S = o.sys_tile ? o.sys_tile : auto_tile(static_cast<int64_t>(max_ns));
    int bpx = o.blocks_per_xcd, persistent = o.persistent;
    hipStream_t st = lane(h).stream;
    const double ts = now_s();
    ProblemRec& M = merged_problem(h, pids);
    ensure_uploaded(h, M, o.precision != 0);
    if (M.op.form == FORM_TRANSFORMED && o.signal == 1) {
        const int N = o.n_steps > 0 ? std::min(o.n_steps, h->n_steps) : h->n_steps;
        if (h->seq.F[N] != 0.0)
            throw Error(DMRI_E_UNSUPPORTED, "several-mesh batches return sum w u (F(t) != 0 at "
                                            "the last step needs option signal = 0)");
    }
    if (o.autotune) {
        char fp[17];
        std::snprintf(fp, sizeof fp, "%016llx", static_cast<unsigned long long>(M.fingerprint));
        std::string key = h->device_tag + "/merged-" + fp + "/";
        for (const auto& gr : groups) key += std::to_string(gr.second.size()) + ",";
        key += "/" + std::to_string(o.precision) + "/" + std::to_string(o.krylov) + "/" +
               std::to_string(o.sys_tile);
        TuneChoice c;
        {
            std::lock_guard<std::mutex> lock(h->tuned_mu);
            auto it = h->tuned.find(key);
            if (it == h->tuned.end())
                it = h->tuned.emplace(key, autotune_merged(h, M, groups, b, q, S)).first;
            c = it->second;
            h->last_tune = c;
        }
        S = c.sys_tile;
        bpx = c.blocks_per_xcd;
        persistent = c.persistent;
    }
    const MergedSlots m = merged_slots(h, groups, b, q, S);
    const int64_t ns = static_cast<int64_t>(m.owner.size());
    Workspace& W = lane(h).ws;
    W.sig.alloc(ns);
    const double t_up = now_s() - ts;
    BatchResult R;
    run_merged_with(h, M, m, S, bpx, persistent, W.sig.p, R);
    std::vector<double> sig(2 * ns);
    HIPCHK(hipMemcpyAsync(sig.data(), W.sig.p, sizeof(double2) * ns, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool any_nc = false;
    for (int64_t i = 0; i < ns; ++i) {
        if (m.owner[i] < 0) continue;
        signal_out[2 * m.owner[i]] = sig[2 * i];
        signal_out[2 * m.owner[i] + 1] = sig[2 * i + 1];
        if (R.flags[i]) any_nc = true;
    }
    // Totals over the caller's pairs only (not the b = 0 padding), each
    // system's products over its own mesh's rows.
    R.total_iters = 0;
    R.spmv_rows = 0;
    for (int64_t i = 0; i < ns; ++i) {
        if (m.owner[i] < 0) continue;
        const int64_t t = i / S;
        R.total_iters += R.iters[i];
        R.spmv_rows += static_cast<int64_t>(R.iters[i]) * (m.ml.tab[4 * t + 1] - m.ml.tab[4 * t]);
    }
    if (stats) stats->t_setup_s += t_up;
    fill_stats(stats, m.owner, R, n_pairs);
    // Costs per problem, in the order its pairs took in the slots.
    int64_t slot = 0;
    for (size_t k = 0; k < groups.size(); ++k) {
        const std::vector<int64_t>& idx = m.order[k];
        std::vector<int32_t> it(idx.size());
        for (size_t i = 0; i < idx.size(); ++i) it[i] = R.iters[slot + static_cast<int64_t>(i)];
        remember_costs(h, groups[k].first, b, q, idx, it);
        slot += (static_cast<int64_t>(idx.size()) + S - 1) / S * S;
    }
    return any_nc;
}

// Runs host pairs grouped by problem: one batch per problem, in sequence or
// (option "concurrency") on several lanes at once. Signals go to host memory
// in input order. Returns true when some system did not converge.
bool run_host_pairs(dmri_ctx* h, int64_t n_pairs, const int32_t* problem_id, const double* b,
                    const double* q, double* signal_out, dmri_stats* stats) {
    // Group pairs by problem, keeping input order inside each group.
    std::vector<std::pair<int32_t, std::vector<int64_t>>> groups;
    for (int32_t pid = 0; pid < static_cast<int32_t>(h->problems.size()); ++pid) {
        std::vector<int64_t> idx;
        for (int64_t i = 0; i < n_pairs; ++i)
            if (problem_id[i] == pid) idx.push_back(i);
        if (!idx.empty()) groups.emplace_back(pid, std::move(idx));
    }
    if (opts(h).mesh_merge && groups.size() > 1)
        return run_merged(h, groups, n_pairs, b, q, signal_out, stats);
    std::atomic<bool> any_nc{false};
    std::mutex mu;
    auto run_group = [&](int32_t pid, std::vector<int64_t> idx) {
        // Tiles of systems with similar b converge together, so whole tiles
        // drop out of the Krylov loop early (results do not depend on the
        // position of a system in the batch).
        if (opts(h).sort_systems) order_systems(h, pid, b, q, idx);
        hipStream_t st = lane(h).stream;
        ProblemRec& P = get_problem(h, pid);
        const double ts = now_s();
        ensure_uploaded(h, P, opts(h).precision != 0);
        const int64_t ns = static_cast<int64_t>(idx.size());
        std::vector<double> hb(ns), hq(3 * ns);
        for (int64_t i = 0; i < ns; ++i) {
            hb[i] = b[idx[i]];
            for (int a = 0; a < 3; ++a) hq[3 * i + a] = q[3 * idx[i] + a];
        }
        Workspace& W = lane(h).ws;
        W.b_in.upload(hb.data(), ns, st);
        W.q_in.upload(hq.data(), 3 * ns, st);
        W.sig.alloc(ns);
        const double t_up = now_s() - ts;
        BatchResult R;
        run_batch(h, P, ns, W.b_in.p, W.q_in.p, W.sig.p, R);
        std::vector<double> hs(2 * ns);
        HIPCHK(hipMemcpyAsync(hs.data(), W.sig.p, sizeof(double2) * ns, hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipStreamSynchronize(st));
        std::lock_guard<std::mutex> lock(mu);
        for (int64_t i = 0; i < ns; ++i) {
            signal_out[2 * idx[i]] = hs[2 * i];
            signal_out[2 * idx[i] + 1] = hs[2 * i + 1];
            if (R.flags[i]) any_nc = true;
        }
        if (stats) stats->t_setup_s += t_up;
        fill_stats(stats, idx, R, n_pairs);
        remember_costs(h, pid, b, q, idx, R.iters);
    };
    // Several problems run concurrently, one lane (stream, workspace, host
    // thread) each, unless a feature shares state across batches.
    int n_lanes = std::min<int>(opts(h).concurrency, static_cast<int>(groups.size()));
    if (h->model.rec_cap > 0 || h->pcmodel.rec_cap > 0) n_lanes = 1;  // one sample recorder
    if (n_lanes <= 1) {
        for (const auto& gr : groups) run_group(gr.first, gr.second);
    } else {
        while (static_cast<int>(h->lanes.size()) < n_lanes) {
            h->lanes.push_back(std::make_unique<Lane>());
            h->lanes.back()->create();
        }
        std::atomic<int> next{0};
        std::exception_ptr first_error;
        std::vector<std::thread> pool;
        for (int t = 0; t < n_lanes; ++t) {
            pool.emplace_back([&, t] {
                // Lane 0 keeps the stream the caller's thread set on it.
                tl_lane = t == 0 ? &lane(h) : h->lanes[t].get();
                Options mine = h->opt;
                tl_opt = &mine;
                try {
                    HIPCHK(hipSetDevice(h->device));
                    for (int gi = next++; gi < static_cast<int>(groups.size()); gi = next++)
                        run_group(groups[gi].first, groups[gi].second);
                } catch (...) {
                    std::lock_guard<std::mutex> lock(mu);
                    if (!first_error) first_error = std::current_exception();
                    next = static_cast<int>(groups.size());
                }
                tl_lane = nullptr;
                tl_opt = nullptr;
            });
        }
        for (auto& th : pool) th.join();
        if (first_error) std::rethrow_exception(first_error);
    }
    return any_nc.load();
}

// Sets the lane's stream for the duration of a call and restores it.
struct StreamOverride {
    dmri_ctx* h;
    hipStream_t saved;
    StreamOverride(dmri_ctx* hh, void* s) : h(hh), saved(lane(hh).stream) {
        if (s) lane(h).stream = static_cast<hipStream_t>(s);
    }
    ~StreamOverride() { lane(h).stream = saved; }
};

// Bump allocator over a fixed device region (256-byte aligned pieces). With
// base == nullptr it only measures.
struct Arena {
    char* base;
    size_t cap;
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        const size_t off = (used + 255) & ~static_cast<size_t>(255);
        used = off + std::max<size_t>(1, count) * sizeof(T);
        if (base && used > cap) throw Error(DMRI_E_INVALID, "scratch region overflow");
        return base ? reinterpret_cast<T*>(base + off) : nullptr;
    }
};

// Device buffers of one no-allocation run.
struct NoAllocBufs {
    double2* vec[kMaxHist + 4];
    double4* gq;
    double* partial;
    int32_t* ctr;
    int32_t* bad;
    uint32_t* barrier;
    double2 *rho, *alpha, *beta;
    double *bb, *rr;
    int32_t *active, *iters, *iters_total, *flags, *n_active;
    // zero-filled at the start of a run: [zero_from, zero_to) in int32 words
    int32_t* zero_from;
    int32_t* zero_to;
    double* acomp;  // q.D_k q per (compartment, system), anisotropic problems
    void carve(Arena& a, int n_vec, size_t nv, size_t ld, size_t n_tiles, size_t part_n,
               size_t items_max, size_t n_acomp) {
        for (int i = 0; i < n_vec; ++i) vec[i] = a.take<double2>(nv);
        gq = a.take<double4>(ld);
        acomp = n_acomp ? a.take<double>(n_acomp) : nullptr;
        partial = a.take<double>(part_n);
        // The state below is contiguous so one fill clears it.
        rho = a.take<double2>(ld);
        alpha = a.take<double2>(ld);
        beta = a.take<double2>(ld);
        bb = a.take<double>(ld);
        rr = a.take<double>(ld);
        active = a.take<int32_t>(ld);
        iters = a.take<int32_t>(ld);
        iters_total = a.take<int32_t>(ld);
        flags = a.take<int32_t>(ld);
        n_active = a.take<int32_t>(n_tiles);
        ctr = a.take<int32_t>(2 * items_max);
        bad = a.take<int32_t>(1);
        barrier = a.take<uint32_t>(32 * 11);
        zero_from = reinterpret_cast<int32_t*>(rho);
        zero_to = reinterpret_cast<int32_t*>(barrier + 32 * 11);
    }
};

// All-FP64 run of n_sys <= 64 systems of one problem with the persistent
// Krylov kernel, every buffer taken from this device's scratch array. No
// device or pinned memory is allocated: the problem's operators must already
// be on the device (uploaded by an earlier run with the same sequence), and
// state is cleared with fill kernels, not memset nodes.
void run_noalloc(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b, const double* d_q,
                 double2* d_sig, dmri_stats* stats) {
    const Options& o = opts(h);
    hipStream_t st = lane(h).stream;
    if (o.precision != 0)
        throw Error(DMRI_E_UNSUPPORTED, "the no-allocation entry point runs precision 0 (FP64)");
    if (o.guess == 2)
        throw Error(DMRI_E_UNSUPPORTED, "the no-allocation entry point has no learned guess");
    if (o.krylov == 3)
        throw Error(DMRI_E_UNSUPPORTED, "the no-allocation entry point runs CG or COCG");
    if (h->model.rec_cap > 0 || h->pcmodel.rec_cap > 0)
        throw Error(DMRI_E_UNSUPPORTED, "sample recording allocates; not with this entry point");
    if (o.precond != 0)
        throw Error(DMRI_E_UNSUPPORTED,
                    "the no-allocation entry point runs Jacobi CG or COCG (precond = 0)");
    if (!P.op.wk_rows.empty())
        throw Error(DMRI_E_UNSUPPORTED,
                    "the no-allocation entry point has no weak pseudo-periodic faces");
    if (!P.pattern_up || !P.A64.ready || P.dt_up != h->dt || P.theta_up != h->theta)
        throw Error(DMRI_E_STATE,
                    "the problem's operators are not on the device for this sequence: run it "
                    "once through dmri_run or dmri_run_device first");
    const bool herm = (P.op.form == FORM_TRANSFORMED) ? (o.krylov != 2) : false;
    if (P.op.form == FORM_UFORM && o.krylov == 1)
        throw Error(DMRI_E_INVALID, "CG needs the Hermitian (periodic-box) operator; use COCG");
    const int S = o.sys_tile ? o.sys_tile : auto_tile(n_sys);
    const int32_t n_rows = static_cast<int32_t>(P.op.n_dof);
    Geom g = make_geom(n_rows, static_cast<int32_t>(n_sys), S, o.blocks_per_xcd, 0, o.grab,
                       o.xcd_split != 0);
    g.nt = o.nt;
    g.lds = 0;
    if (g.ld > 64)
        throw Error(DMRI_E_INVALID, "the no-allocation entry point takes at most 64 systems");
    int n_cu = 0;
    HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
    Geom gp = make_geom(n_rows, static_cast<int32_t>(n_sys), S, std::max(1, n_cu / 8), 0, 1);
    gp.nt = g.nt;
    gp.lds = 0;
    if (!persistent_fits<double>(gp, herm, n_cu))
        throw Error(DMRI_E_UNSUPPORTED, "the persistent Krylov grid does not fit on this device");
    const size_t ld = static_cast<size_t>(g.ld), nv = static_cast<size_t>(n_rows) * ld;
    const int32_t items_max = std::max(g.n_items, 8 * g.n_tiles);
    const size_t part_n =
        std::max(static_cast<size_t>(items_max) * g.B * S * 4,
                 2 * static_cast<size_t>(gp.n_items) * gp.B * S * 4);
    History<double2> hs;
    hs.nh = history_len(h);
    const int n_vec = hs.nh + 4;
    Arena probe{nullptr, 0};
    NoAllocBufs B{};
    const size_t n_acomp = P.op.aniso ? static_cast<size_t>(P.op.n_comp) * ld : 0;
    B.carve(probe, n_vec, nv, ld, static_cast<size_t>(g.n_tiles), part_n,
            static_cast<size_t>(items_max), n_acomp);
    if (probe.used > kNoAllocScratchBytes)
        throw Error(DMRI_E_INVALID,
                    "the run needs " + std::to_string(probe.used) + " bytes of scratch; the "
                    "no-allocation entry point has " + std::to_string(kNoAllocScratchBytes) +
                    " (fewer systems or a smaller mesh)");
    Arena arena{static_cast<char*>(h->scratch_dev), kNoAllocScratchBytes};
    B.carve(arena, n_vec, nv, ld, static_cast<size_t>(g.n_tiles), part_n,
            static_cast<size_t>(items_max), n_acomp);
    // The array keeps the previous call's contents: clear the state, the
    // queue counters, the invalid-input flag and the grid barrier.
    launch_zero_i32(st, B.zero_from, B.zero_to - B.zero_from);
    if (P.op.form == FORM_UFORM && !h->seq.has_f)
        throw Error(DMRI_E_STATE, "the U-form (walls) needs f on the time grid");
    launch_sys_params(st, static_cast<int32_t>(n_sys), static_cast<int32_t>(ld), d_b, d_q,
                      h->seq.int_F2, B.gq, B.bad);
    if (P.op.aniso) {
        launch_aniso_params(st, P.op.n_comp, static_cast<int32_t>(ld), B.gq, P.comp_tensor.p,
                            B.acomp);
        for (Geom* gg : {&g, &gp}) {
            gg->comp = P.row_comp.p;
            gg->acomp = B.acomp;
            gg->acomp_ld = static_cast<int32_t>(ld);
        }
    }
    SolverState s{};
    s.rho = B.rho;
    s.alpha = B.alpha;
    s.beta = B.beta;
    s.bb = B.bb;
    s.rr = B.rr;
    s.active = B.active;
    s.iters = B.iters;
    s.iters_total = B.iters_total;
    s.flags = B.flags;
    s.n_active = B.n_active;
    s.n_sys = static_cast<int32_t>(n_sys);
    s.max_iter = o.max_iter;
    s.rtol2 = o.rtol * o.rtol;
    s.floor_bb = nullptr;
    s.floor_scale = 0.0;
    Scratch sc{B.partial, B.ctr, B.ctr + items_max};
    GridBarrier bar{B.barrier, B.barrier + 32 * 9, reinterpret_cast<int32_t*>(B.barrier + 32 * 10)};
    for (int i = 0; i <= hs.nh; ++i) hs.ring.push_back(B.vec[i]);
    double2* r = B.vec[hs.nh + 1];
    double2* p = B.vec[hs.nh + 2];
    double2* q = B.vec[hs.nh + 3];
    const MatView<double> Av = view<double>(P, P.A64);
    launch_set_initial<double>(st, g, P.u0.p, s.n_sys, hs.u(0));
    std::vector<double> F, f;
    step_tables(h, F, f);
    const bool tr = P.op.form == FORM_TRANSFORMED;
    const int N = o.n_steps > 0 ? std::min(o.n_steps, h->n_steps) : h->n_steps;
    if (P.op.form == FORM_TRANSFORMED && h->seq.F[N] != 0.0 && o.signal == 1)
        throw Error(DMRI_E_UNSUPPORTED,
                    "the no-allocation entry point returns sum w u only: stop where F = 0 or "
                    "set option signal = 0");
    KernelTimer timer(h, st, 0);
    const MlpDofs no_dofs{nullptr, nullptr};
    const double t0 = now_s();
    for (int n = 1; n <= N; ++n) {
        const Coef lhs = lhs_coef(h, tr, F, f, n), rhs = rhs_coef(h, tr, F, f, n);
        const int gm = prepare_guess<double>(h, g, no_dofs, tr, F, f, n, n_sys, hs, timer);
        launch_init<double>(st, g, Av, B.gq, lhs, rhs, herm, gm, hs.u(0), hs.u(1), hs.x(), r, p,
                            nullptr, nullptr, nullptr, s, sc);
        launch_krylov_persistent<double>(st, gp, Av, B.gq, lhs, herm, hs.x(), r, p, q, s, sc, bar);
        hs.advance();
    }
    launch_signal<double>(st, g, P.w.p, hs.u(0), d_sig, s.n_sys, sc);
    // Results for the statistics and the status (n_sys <= 64: stack arrays).
    int32_t bad = 0, bar_err = 0;
    int32_t fl[64], it[64];
    double rr[64], bb[64];
    HIPCHK(hipMemcpyAsync(&bad, B.bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&bar_err, bar.err, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(fl, B.flags, sizeof(int32_t) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(it, B.iters_total, sizeof(int32_t) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(rr, B.rr, sizeof(double) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(bb, B.bb, sizeof(double) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) throw Error(DMRI_E_INVALID, "b must be finite and >= 0, q finite and nonzero when b > 0");
    if (bar_err) throw Error(DMRI_E_DEVICE, "persistent solver: a grid barrier wait timed out");
    bool nc = false;
    int64_t tot = 0;
    for (int64_t i = 0; i < n_sys; ++i) {
        nc |= fl[i] != 0;
        tot += it[i];
        if (stats && stats->iters_total) stats->iters_total[i] = it[i];
        if (stats && stats->converged) stats->converged[i] = fl[i] == 0 ? 1 : 0;
        if (stats && stats->final_rel_res)
            stats->final_rel_res[i] = bb[i] > 0 ? std::sqrt(rr[i] / bb[i]) : 0.0;
    }
    if (stats) {
        stats->t_solve_s = now_s() - t0;
        stats->total_iterations = tot;
        stats->spmv_rows = tot * n_rows;
        stats->n_steps = N;
    }
    if (nc) throw Error(DMRI_NOT_CONVERGED, "some systems hit max_iter");
}

}  // namespace
}  // namespace dmri

extern "C" {

dmri_status dmri_run(dmri_handle h, int64_t n_pairs, const int32_t* problem_id, const double* b,
                     const double* q, double* signal_out, dmri_stats* stats) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        need_sequence(h);
        if (n_pairs < 0) throw Error(DMRI_E_INVALID, "n_pairs must be >= 0");
        if (n_pairs > 0 && (!problem_id || !b || !q || !signal_out))
            throw Error(DMRI_E_INVALID, "NULL argument");
        check_pairs(h, n_pairs, problem_id, b, q);
        reset_stats(stats, n_pairs);
        if (n_pairs == 0) return DMRI_OK;
        const bool nc = run_host_pairs(h, n_pairs, problem_id, b, q, signal_out, stats);
        return nc ? DMRI_NOT_CONVERGED : DMRI_OK;
    });
}

dmri_status dmri_run_device(dmri_handle h, void* hip_stream, int64_t n_pairs,
                            const int32_t* d_problem_id, const double* d_b, const double* d_q,
                            double* d_signal, dmri_stats* stats) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        need_sequence(h);
        if (n_pairs < 0) throw Error(DMRI_E_INVALID, "n_pairs must be >= 0");
        if (n_pairs == 0) {
            reset_stats(stats, 0);
            return DMRI_OK;
        }
        if (!d_problem_id || !d_b || !d_q || !d_signal)
            throw Error(DMRI_E_INVALID, "NULL argument");
        StreamOverride so(h, hip_stream);
        hipStream_t st = lane(h).stream;
        // The pair list is small: read it (and b, q for the checks and the
        // tile order) to the host, in stream order after the caller's work.
        std::vector<int32_t> hp(n_pairs);
        std::vector<double> hb(n_pairs), hq(3 * n_pairs);
        HIPCHK(hipMemcpyAsync(hp.data(), d_problem_id, sizeof(int32_t) * n_pairs,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hb.data(), d_b, sizeof(double) * n_pairs, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hq.data(), d_q, sizeof(double) * 3 * n_pairs, hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipStreamSynchronize(st));
        check_pairs(h, n_pairs, hp.data(), hb.data(), hq.data());
        reset_stats(stats, n_pairs);
        bool one = true;
        for (int64_t i = 1; i < n_pairs; ++i) one &= hp[i] == hp[0];
        if (!one) {
            // Several problems: one batch per problem (as dmri_run), signals
            // copied to the caller's buffer in input order.
            std::vector<double> sig(2 * n_pairs);
            const bool nc = run_host_pairs(h, n_pairs, hp.data(), hb.data(), hq.data(),
                                           sig.data(), stats);
            HIPCHK(hipMemcpyAsync(d_signal, sig.data(), sizeof(double2) * n_pairs,
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
            return nc ? DMRI_NOT_CONVERGED : DMRI_OK;
        }
        const int32_t problem_id = hp[0];
        ProblemRec& P = get_problem(h, problem_id);
        const double ts = now_s();
        ensure_uploaded(h, P, opts(h).precision != 0);
        if (stats) stats->t_setup_s = now_s() - ts;
        BatchResult R;
        std::vector<int64_t> idx(n_pairs);
        for (int64_t i = 0; i < n_pairs; ++i) idx[i] = i;
        if (opts(h).sort_systems) order_systems(h, problem_id, hb.data(), hq.data(), idx);
        bool identity = true;
        for (int64_t i = 0; i < n_pairs; ++i) identity &= idx[i] == i;
        if (identity) {
            run_batch(h, P, n_pairs, d_b, d_q, reinterpret_cast<double2*>(d_signal), R);
        } else {
            // Sorted copies of b and q in the lane's workspace; signals are
            // scattered back to the caller's order.
            std::vector<double> sb(n_pairs), sq(3 * n_pairs);
            for (int64_t i = 0; i < n_pairs; ++i) {
                sb[i] = hb[idx[i]];
                for (int a = 0; a < 3; ++a) sq[3 * i + a] = hq[3 * idx[i] + a];
            }
            Workspace& W = lane(h).ws;
            W.b_in.upload(sb.data(), n_pairs, st);
            W.q_in.upload(sq.data(), 3 * n_pairs, st);
            W.sig.alloc(n_pairs);
            run_batch(h, P, n_pairs, W.b_in.p, W.q_in.p, W.sig.p, R);
            std::vector<double> ss(2 * n_pairs), out(2 * n_pairs);
            HIPCHK(hipMemcpyAsync(ss.data(), W.sig.p, sizeof(double2) * n_pairs,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t i = 0; i < n_pairs; ++i) {
                out[2 * idx[i]] = ss[2 * i];
                out[2 * idx[i] + 1] = ss[2 * i + 1];
            }
            HIPCHK(hipMemcpyAsync(d_signal, out.data(), sizeof(double2) * n_pairs,
                                  hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        fill_stats(stats, idx, R, n_pairs);
        if (opts(h).sort_systems) remember_costs(h, problem_id, hb.data(), hq.data(), idx, R.iters);
        for (int32_t fl : R.flags)
            if (fl) return DMRI_NOT_CONVERGED;
        return DMRI_OK;
    });
}

dmri_status dmri_run_device_noalloc(dmri_handle h, void* hip_stream, int64_t n_pairs,
                                    const int32_t* d_problem_id, const double* d_b,
                                    const double* d_q, double* d_signal, dmri_stats* stats) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        need_sequence(h);
        if (n_pairs < 0 || n_pairs > 64)
            throw Error(DMRI_E_INVALID, "the no-allocation entry point takes 0..64 pairs");
        reset_stats(stats, n_pairs);
        if (n_pairs == 0) return DMRI_OK;
        if (!d_problem_id || !d_b || !d_q || !d_signal)
            throw Error(DMRI_E_INVALID, "NULL argument");
        StreamOverride so(h, hip_stream);
        hipStream_t st = lane(h).stream;
        // At most 64 pairs: the pair list is checked on the host in stack arrays.
        int32_t ids[64];
        double hb[64], hq[3 * 64];
        HIPCHK(hipMemcpyAsync(ids, d_problem_id, sizeof(int32_t) * n_pairs, hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipMemcpyAsync(hb, d_b, sizeof(double) * n_pairs, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(hq, d_q, sizeof(double) * 3 * n_pairs, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        check_pairs(h, n_pairs, ids, hb, hq);
        for (int64_t i = 1; i < n_pairs; ++i)
            if (ids[i] != ids[0])
                throw Error(DMRI_E_INVALID,
                            "the no-allocation entry point runs the pairs of one problem");
        ProblemRec& P = get_problem(h, ids[0]);
        try {
            run_noalloc(h, P, n_pairs, d_b, d_q, reinterpret_cast<double2*>(d_signal), stats);
        } catch (const Error& e) {
            if (e.code == DMRI_NOT_CONVERGED) return DMRI_NOT_CONVERGED;
            throw;
        }
        return DMRI_OK;
    });
}

dmri_status dmri_apply_operator(dmri_handle h, int32_t problem_id, int32_t which, int64_t n_sys,
                                const double* c, const double* d, const double* x, double* y) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        need_sequence(h);
        if (which != 0 && which != 1) throw Error(DMRI_E_INVALID, "which must be 0 or 1");
        if (n_sys <= 0 || !c || !d || !x || !y) throw Error(DMRI_E_INVALID, "bad arguments");
        ProblemRec& P = get_problem(h, problem_id);
        const bool f32 = opts(h).precision != 0;
        ensure_uploaded(h, P, f32);
        hipStream_t st = lane(h).stream;
        const int S = opts(h).sys_tile ? opts(h).sys_tile : auto_tile(n_sys);
        const Geom g = make_geom(static_cast<int32_t>(P.op.n_dof), static_cast<int32_t>(n_sys), S,
                                 opts(h).blocks_per_xcd, opts(h).queue, opts(h).grab);
        const size_t nrow = static_cast<size_t>(g.n_rows), ld = static_cast<size_t>(g.ld);
        std::vector<double> hc(ld, 0.0), hd(3 * ld, 0.0);
        for (int64_t s = 0; s < n_sys; ++s) {
            hc[s] = c[s];
            for (int a = 0; a < 3; ++a) hd[3 * s + a] = d[3 * s + a];
        }
        DevBuf<double> dc, dd;
        dc.upload(hc.data(), ld, st);
        dd.upload(hd.data(), 3 * ld, st);
        // Device vectors are tile-major: element (row, s) at
        // ((s / S) * n_rows + row) * S + s % S.
        auto didx = [&](size_t row, int64_t sy) -> size_t {
            return (static_cast<size_t>(sy / S) * nrow + row) * S + static_cast<size_t>(sy % S);
        };
        if (!f32) {
            std::vector<double> hx(2 * nrow * ld, 0.0), hy(2 * nrow * ld);
            for (size_t i = 0; i < nrow; ++i)
                for (int64_t sy = 0; sy < n_sys; ++sy)
                    for (int k = 0; k < 2; ++k) hx[2 * didx(i, sy) + k] = x[2 * (i * n_sys + sy) + k];
            DevBuf<double> dx, dy;
            dx.upload(hx.data(), hx.size(), st);
            dy.alloc(hy.size());
            launch_apply<double>(st, g, view<double>(P, P.A64), which, dc.p,
                                 reinterpret_cast<const double3*>(dd.p),
                                 reinterpret_cast<const double2*>(dx.p),
                                 reinterpret_cast<double2*>(dy.p));
            HIPCHK(hipMemcpyAsync(hy.data(), dy.p, hy.size() * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (size_t i = 0; i < nrow; ++i)
                for (int64_t sy = 0; sy < n_sys; ++sy)
                    for (int k = 0; k < 2; ++k) y[2 * (i * n_sys + sy) + k] = hy[2 * didx(i, sy) + k];
        } else {
            std::vector<float> hx(2 * nrow * ld, 0.0f), hy(2 * nrow * ld);
            for (size_t i = 0; i < nrow; ++i)
                for (int64_t sy = 0; sy < n_sys; ++sy)
                    for (int k = 0; k < 2; ++k)
                        hx[2 * didx(i, sy) + k] = static_cast<float>(x[2 * (i * n_sys + sy) + k]);
            DevBuf<float> dx, dy;
            dx.upload(hx.data(), hx.size(), st);
            dy.alloc(hy.size());
            launch_apply<float>(st, g, view<float>(P, P.A32), which, dc.p,
                                reinterpret_cast<const double3*>(dd.p),
                                reinterpret_cast<const float2*>(dx.p),
                                reinterpret_cast<float2*>(dy.p));
            HIPCHK(hipMemcpyAsync(hy.data(), dy.p, hy.size() * sizeof(float), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (size_t i = 0; i < nrow; ++i)
                for (int64_t sy = 0; sy < n_sys; ++sy)
                    for (int k = 0; k < 2; ++k) y[2 * (i * n_sys + sy) + k] = hy[2 * didx(i, sy) + k];
        }
        return DMRI_OK;
    });
}

}  // extern "C"
