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

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/dmri.h"
#include "assembly.hpp"
#include "kernels.hpp"

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
};

struct Options {
    int precision = 0;
    int krylov = 0;
    double rtol = 1e-10;
    double inner_rtol = 1e-4;
    int max_iter = 2000;
    int guess = 1;
    int sys_tile = 0;
    int graph = 0;
    int autotune = 0;
    int n_steps = 0;
    int blocks_per_xcd = 256;
    int chunk_passes = 1;
    int time_kernel = 0;
    int progress = 0;
};

// Per-batch device workspace (grow-only, reused across runs).
struct Workspace {
    DevBuf<double> vec64[6];
    DevBuf<float> vec32[6];
    DevBuf<double4> gq;
    DevBuf<double2> rho, alpha, beta, sig;
    DevBuf<double> bb, rr, partial, b_in, q_in;
    DevBuf<int32_t> active, iters, iters_total, flags, n_active, bad;
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

}  // namespace
}  // namespace dmri

struct dmri_ctx {
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    std::string last_error = "no error";
    std::vector<std::unique_ptr<dmri::ProblemRec>> problems;
    bool seq_set = false;
    double delta = 0, Delta = 0, dt = 0, theta = 0.5;
    int n_steps = 0;
    dmri::Options opt;
    dmri::Workspace ws;
    hipEvent_t ev[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> tpool;  // timing events, reused across runs
};

namespace dmri {
namespace {

void need_device(dmri_ctx* h) {
    if (h->host_only) throw Error(DMRI_E_STATE, "host-only context (created with device -1)");
    HIPCHK(hipSetDevice(h->device));
}

// Build K0 = M/dt + theta R, Kr = M/dt - (1-theta) R, aux = {M_D, V} and the
// diagonal, in precision T, and upload them.
template <typename T>
void upload_matrix(const HostOperator& op, double dt, double th, DevMatrix<T>& A,
                   hipStream_t st) {
    using T4 = typename Vec4Of<T>::type;
    const size_t nnz = static_cast<size_t>(op.nnz), n = static_cast<size_t>(op.n_dof);
    std::vector<T> K0(nnz), Kr(nnz), dK0(n);
    std::vector<T4> aux(nnz), daux(n);
    for (size_t k = 0; k < nnz; ++k) {
        K0[k] = static_cast<T>(op.M[k] / dt + th * op.R[k]);
        Kr[k] = static_cast<T>(op.M[k] / dt - (1.0 - th) * op.R[k]);
        aux[k].x = static_cast<T>(op.MD[k]);
        aux[k].y = static_cast<T>(op.V[0][k]);
        aux[k].z = static_cast<T>(op.V[1][k]);
        aux[k].w = static_cast<T>(op.V[2][k]);
    }
    for (size_t i = 0; i < n; ++i) {
        dK0[i] = K0[op.diag_pos[i]];
        daux[i] = aux[op.diag_pos[i]];
    }
    A.K0.upload(K0.data(), nnz, st);
    A.Kr.upload(Kr.data(), nnz, st);
    A.dK0.upload(dK0.data(), n, st);
    A.aux.upload(aux.data(), nnz, st);
    A.daux.upload(daux.data(), n, st);
    HIPCHK(hipStreamSynchronize(st));  // host staging vectors go out of scope
    A.ready = true;
}

void ensure_uploaded(dmri_ctx* h, ProblemRec& P, bool need32) {
    hipStream_t st = h->stream;
    if (!P.pattern_up) {
        P.row_ptr.upload(P.op.row_ptr.data(), P.op.row_ptr.size(), st);
        P.col.upload(P.op.col.data(), P.op.col.size(), st);
        P.w.upload(P.op.w.data(), P.op.w.size(), st);
        P.u0.upload(P.op.u0.data(), P.op.u0.size(), st);
        HIPCHK(hipStreamSynchronize(st));
        P.pattern_up = true;
    }
    if (P.dt_up != h->dt || P.theta_up != h->theta) {
        P.A64.ready = false;
        P.A32.ready = false;
        P.dt_up = h->dt;
        P.theta_up = h->theta;
    }
    if (!P.A64.ready) upload_matrix<double>(P.op, h->dt, h->theta, P.A64, st);
    if (need32 && !P.A32.ready) upload_matrix<float>(P.op, h->dt, h->theta, P.A32, st);
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

// F(t^n) for n = 0..N (transformed form) or f on (t^{n-1}, t^n] for n = 1..N
// (U-form, index n), from the PGSE profile of Sec. 2 eq. pgse.
void step_tables(const dmri_ctx* h, std::vector<double>& F, std::vector<double>& f) {
    const int N = h->n_steps;
    F.assign(N + 1, 0.0);
    f.assign(N + 1, 0.0);
    for (int n = 0; n <= N; ++n) {
        const double t = n * h->dt;
        const double up = std::min(std::max(t, 0.0), h->delta);
        const double down = std::min(std::max(t - h->Delta, 0.0), h->delta);
        F[n] = up - down;
        if (n >= 1) {
            const double tm = (n - 0.5) * h->dt;
            f[n] = (tm <= h->delta) ? 1.0 : ((tm > h->Delta && tm <= h->Delta + h->delta) ? -1.0 : 0.0);
        }
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
        while (h->tpool.size() < used + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            h->tpool.push_back(e);
        }
        HIPCHK(hipEventRecord(h->tpool[used], st));
        launch();
        HIPCHK(hipEventRecord(h->tpool[used + 1], st));
        used += 2;
    }
    void collect(BatchResult& res) {
        HIPCHK(hipStreamSynchronize(st));
        double tot = 0.0;
        for (size_t i = 0; i + 1 < used; i += 2) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, h->tpool[i], h->tpool[i + 1]));
            tot += ms;
        }
        res.n_timed += static_cast<int64_t>(used / 2);
        res.t_timed += tot * 1e-3;
        used = 0;
    }
};

// Solve one batch of systems on one problem in precision T (FP64 or FP32
// throughout). b/q are device pointers ([n_sys], [n_sys][3]); the signals
// are written to d_sig ([n_sys] double2, device).
template <typename T>
void solve_batch(dmri_ctx* h, ProblemRec& P, DevMatrix<T>& A, int64_t n_sys, const double* d_b,
                 const double* d_q, double2* d_sig, BatchResult& res) {
    using V2 = typename Vec2Of<T>::type;
    hipStream_t st = h->stream;
    Workspace& W = h->ws;
    const bool herm = (P.op.form == FORM_TRANSFORMED) ? (h->opt.krylov != 2) : false;
    if (P.op.form == FORM_UFORM && h->opt.krylov == 1)
        throw Error(DMRI_E_INVALID, "CG needs the Hermitian (periodic-box) operator; use COCG");
    const int S = h->opt.sys_tile ? h->opt.sys_tile : auto_tile(n_sys);
    const Geom g = make_geom(static_cast<int32_t>(P.op.n_dof), static_cast<int32_t>(n_sys), S,
                             h->opt.blocks_per_xcd, h->opt.chunk_passes);
    const size_t nv = static_cast<size_t>(g.n_rows) * g.ld;
    DevBuf<T>* vecs;
    if constexpr (sizeof(T) == 8) vecs = W.vec64; else vecs = W.vec32;
    for (int i = 0; i < 6; ++i) vecs[i].alloc(2 * nv);
    V2* bufs[3] = {reinterpret_cast<V2*>(vecs[0].p), reinterpret_cast<V2*>(vecs[1].p),
                   reinterpret_cast<V2*>(vecs[2].p)};
    V2* r = reinterpret_cast<V2*>(vecs[3].p);
    V2* p = reinterpret_cast<V2*>(vecs[4].p);
    V2* q = reinterpret_cast<V2*>(vecs[5].p);
    const size_t ld = static_cast<size_t>(g.ld);
    W.gq.alloc(ld);
    W.rho.alloc(ld);
    W.alpha.alloc(ld);
    W.beta.alloc(ld);
    W.bb.alloc(ld);
    W.rr.alloc(ld);
    W.active.alloc(ld);
    W.iters.alloc(ld);
    W.iters_total.alloc(ld);
    W.flags.alloc(ld);
    W.n_active.alloc(static_cast<size_t>(g.n_tiles));
    W.partial.alloc(static_cast<size_t>(g.n_items) * g.B * S * 4);
    W.bad.alloc(1);
    W.pinned(static_cast<size_t>(g.n_tiles));
    HIPCHK(hipMemsetAsync(W.iters_total.p, 0, sizeof(int32_t) * ld, st));
    HIPCHK(hipMemsetAsync(W.flags.p, 0, sizeof(int32_t) * ld, st));
    HIPCHK(hipMemsetAsync(W.active.p, 0, sizeof(int32_t) * ld, st));
    HIPCHK(hipMemsetAsync(W.iters.p, 0, sizeof(int32_t) * ld, st));
    HIPCHK(hipMemsetAsync(W.bad.p, 0, sizeof(int32_t), st));
    HIPCHK(hipMemsetAsync(W.rho.p, 0, sizeof(double2) * ld, st));
    HIPCHK(hipMemsetAsync(W.alpha.p, 0, sizeof(double2) * ld, st));
    HIPCHK(hipMemsetAsync(W.beta.p, 0, sizeof(double2) * ld, st));
    HIPCHK(hipMemsetAsync(W.bb.p, 0, sizeof(double) * ld, st));
    HIPCHK(hipMemsetAsync(W.rr.p, 0, sizeof(double) * ld, st));

    const double intF2 = h->delta * h->delta * (h->Delta - h->delta / 3.0);
    launch_sys_params(st, static_cast<int32_t>(n_sys), g.ld, d_b, d_q, intF2, W.gq.p, W.bad.p);
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, W.bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) throw Error(DMRI_E_INVALID, "b must be finite and >= 0, q finite and nonzero when b > 0");

    SolverState s{};
    s.rho = W.rho.p;
    s.alpha = W.alpha.p;
    s.beta = W.beta.p;
    s.bb = W.bb.p;
    s.rr = W.rr.p;
    s.active = W.active.p;
    s.iters = W.iters.p;
    s.iters_total = W.iters_total.p;
    s.flags = W.flags.p;
    s.n_active = W.n_active.p;
    s.n_sys = static_cast<int32_t>(n_sys);
    s.max_iter = h->opt.max_iter;
    s.rtol2 = h->opt.rtol * h->opt.rtol;
    Scratch sc{W.partial.p};
    const MatView<T> Av = view<T>(P, A);

    launch_set_initial<T>(st, g, P.u0.p, s.n_sys, bufs[0]);
    std::vector<double> F, f;
    step_tables(h, F, f);
    const bool tr = P.op.form == FORM_TRANSFORMED;
    const double th = h->theta;
    const int N = h->opt.n_steps > 0 ? std::min(h->opt.n_steps, h->n_steps) : h->n_steps;

    KernelTimer timer(h, st, h->opt.time_kernel);
    double t0 = now_s();
    int cur = 0, prev2 = 1, nxt = 2;  // indices into bufs: u_prev, u_prev2, x
    int last_iters = 8;
    for (int n = 1; n <= N; ++n) {
        Coef lhs, rhs;
        if (tr) {
            lhs = Coef{F[n], th, th};
            rhs = Coef{F[n - 1], -(1.0 - th), -(1.0 - th)};
        } else {
            lhs = Coef{f[n], 0.0, th};
            rhs = Coef{f[n], 0.0, -(1.0 - th)};
        }
        const int gm = (h->opt.guess == 1 && n >= 2) ? 1 : 0;
        timer.run(4, [&] {
            launch_init<T>(st, g, Av, W.gq.p, lhs, rhs, herm, gm, bufs[cur], bufs[prev2],
                           bufs[nxt], r, p, s, sc);
        });
        // Pipelined chunks: enqueue chunk k+1 before checking chunk k.
        int done = 0, slot = 0;
        bool pending = false;
        int first = std::max(1, last_iters - 2);
        int chunk = first;
        for (;;) {
            for (int i = 0; i < chunk; ++i) {
                timer.run(1, [&] { launch_spmv_dot<T>(st, g, Av, W.gq.p, lhs, herm, p, q, s, sc); });
                timer.run(2, [&] {
                    launch_update<T>(st, g, Av, W.gq.p, lhs, herm, bufs[nxt], r, p, q, s, sc);
                });
                timer.run(3, [&] { launch_pupdate<T>(st, g, Av, W.gq.p, lhs, r, p, s); });
            }
            done += chunk;
            HIPCHK(hipMemcpyAsync(W.h_active[slot], W.n_active.p, sizeof(int32_t) * g.n_tiles,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipEventRecord(h->ev[slot], st));
            if (pending) {
                HIPCHK(hipEventSynchronize(h->ev[slot ^ 1]));
                int tot = 0;
                for (int t = 0; t < g.n_tiles; ++t) tot += W.h_active[slot ^ 1][t];
                if (tot == 0) {
                    done -= chunk;  // the chunk just enqueued only early-exits
                    break;
                }
            }
            pending = true;
            slot ^= 1;
            chunk = 2;
            if (done > h->opt.max_iter + 4) {
                HIPCHK(hipStreamSynchronize(st));
                break;
            }
        }
        last_iters = done;
        if (h->opt.progress > 0 && (n % h->opt.progress == 0 || n == N)) {
            std::fprintf(stderr, "[dmri] step %d/%d: %d iterations, %.2fs\n", n, N, done,
                         now_s() - t0);
            std::fflush(stderr);
        }
        res.spmv_rows += static_cast<int64_t>(done) * g.n_rows * n_sys;
        const int old_prev2 = prev2;
        prev2 = cur;
        cur = nxt;
        nxt = old_prev2;
    }
    HIPCHK(hipStreamSynchronize(st));
    res.t_solve = now_s() - t0;
    res.steps = N;
    timer.collect(res);
    t0 = now_s();
    launch_signal<T>(st, g, P.w.p, bufs[cur], d_sig, s.n_sys, sc);
    res.iters.resize(n_sys);
    res.flags.resize(n_sys);
    res.rr.resize(n_sys);
    res.bb.resize(n_sys);
    HIPCHK(hipMemcpyAsync(res.iters.data(), W.iters_total.p, sizeof(int32_t) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(res.flags.data(), W.flags.p, sizeof(int32_t) * n_sys,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(res.rr.data(), W.rr.p, sizeof(double) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(res.bb.data(), W.bb.p, sizeof(double) * n_sys, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    res.t_signal = now_s() - t0;
    for (int64_t i = 0; i < n_sys; ++i) res.total_iters += res.iters[i];
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

void run_batch(dmri_ctx* h, ProblemRec& P, int64_t n_sys, const double* d_b, const double* d_q,
               double2* d_sig, BatchResult& R) {
    if (h->opt.precision == 0) {
        solve_batch<double>(h, P, P.A64, n_sys, d_b, d_q, d_sig, R);
    } else if (h->opt.precision == 2) {
        solve_batch<float>(h, P, P.A32, n_sys, d_b, d_q, d_sig, R);
    } else {
        throw Error(DMRI_E_UNSUPPORTED, "mixed precision with FP64 refinement is not built yet");
    }
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
    if (!h->seq_set) throw Error(DMRI_E_STATE, "no sequence: call dmri_set_sequence_pgse first");
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
            HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming));
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
        if (!h->host_only) {
            (void)hipSetDevice(h->device);
            (void)hipStreamSynchronize(h->stream);
        }
        h->problems.clear();
        h->ws.~Workspace();
        new (&h->ws) Workspace();
        if (!h->host_only) {
            for (auto& e : h->ev)
                if (e) (void)hipEventDestroy(e);
            for (auto& e : h->tpool) (void)hipEventDestroy(e);
            (void)hipStreamDestroy(h->stream);
        }
    } catch (...) {
    }
    delete h;
}

const char* dmri_last_error(dmri_handle h) {
    return h ? h->last_error.c_str() : g_create_error.c_str();
}

dmri_status dmri_add_problem(dmri_handle h, int64_t n_nodes, const double* xyz, int64_t n_tets,
                             const int32_t* tets, const int32_t* tet_label, int32_t n_comp,
                             const double* D, const double* T2, const double* u0, double kappa,
                             const double box_lo[3], const double box_hi[3],
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
        in.T2 = T2;
        in.u0 = u0;
        in.kappa = kappa;
        for (int a = 0; a < 3; ++a) {
            in.lo[a] = box_lo[a];
            in.hi[a] = box_hi[a];
        }
        in.periodic_mask = periodic_mask;
        auto rec = std::make_unique<ProblemRec>();
        rec->op = assemble(in);
        h->problems.push_back(std::move(rec));
        *problem_id = static_cast<int32_t>(h->problems.size() - 1);
        return DMRI_OK;
    });
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

dmri_status dmri_set_sequence_pgse(dmri_handle h, double delta_us, double Delta_us, double dt_us,
                                   double theta) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        if (!std::isfinite(delta_us) || !std::isfinite(Delta_us) || !std::isfinite(dt_us) ||
            !std::isfinite(theta))
            throw Error(DMRI_E_INVALID, "sequence parameters must be finite");
        if (!(dt_us > 0) || !(delta_us > 0) || !(Delta_us >= delta_us))
            throw Error(DMRI_E_INVALID, "need dt > 0 and 0 < delta <= Delta");
        if (theta < 0.5 || theta > 1.0) throw Error(DMRI_E_INVALID, "theta must be in [1/2, 1]");
        for (double v : {delta_us, Delta_us}) {
            const double r = v / dt_us;
            if (std::fabs(r - std::round(r)) > 1e-9 * std::max(1.0, r))
                throw Error(DMRI_E_INVALID, "delta/dt and Delta/dt must be integers");
        }
        const double steps = std::round((Delta_us + delta_us) / dt_us);
        if (steps > 1e7) throw Error(DMRI_E_INVALID, "too many time steps");
        h->delta = delta_us;
        h->Delta = Delta_us;
        h->dt = dt_us;
        h->theta = theta;
        h->n_steps = static_cast<int>(steps);
        h->seq_set = true;
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
        else if (k == "krylov") o.krylov = as_int(0, 2);
        else if (k == "rtol") {
            if (!(v > 0 && v < 1)) throw Error(DMRI_E_INVALID, "rtol must be in (0, 1)");
            o.rtol = v;
        } else if (k == "inner_rtol") {
            if (!(v > 0 && v < 1)) throw Error(DMRI_E_INVALID, "inner_rtol must be in (0, 1)");
            o.inner_rtol = v;
        } else if (k == "max_iter") o.max_iter = as_int(1, 1000000);
        else if (k == "guess") o.guess = as_int(0, 2);
        else if (k == "sys_tile") {
            int t = as_int(0, 64);
            if (t != 0 && t != 8 && t != 16 && t != 32 && t != 64)
                throw Error(DMRI_E_INVALID, "sys_tile must be 0, 8, 16, 32 or 64");
            o.sys_tile = t;
        } else if (k == "graph") o.graph = as_int(0, 1);
        else if (k == "autotune") o.autotune = as_int(0, 1);
        else if (k == "n_steps") o.n_steps = as_int(0, 10000000);
        else if (k == "blocks_per_xcd") o.blocks_per_xcd = as_int(1, 4096);
        else if (k == "chunk_passes") o.chunk_passes = as_int(1, 64);
        else if (k == "time_kernel") o.time_kernel = as_int(0, 4);
        else if (k == "progress") o.progress = as_int(0, 1000000);
        else throw Error(DMRI_E_INVALID, "unknown option " + k);
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
        else if (k == "max_iter") *value = o.max_iter;
        else if (k == "guess") *value = o.guess;
        else if (k == "sys_tile") *value = o.sys_tile;
        else if (k == "graph") *value = o.graph;
        else if (k == "autotune") *value = o.autotune;
        else if (k == "n_steps") *value = o.n_steps;
        else if (k == "blocks_per_xcd") *value = o.blocks_per_xcd;
        else if (k == "chunk_passes") *value = o.chunk_passes;
        else if (k == "time_kernel") *value = o.time_kernel;
        else if (k == "progress") *value = o.progress;
        else throw Error(DMRI_E_INVALID, "unknown option " + k);
        return DMRI_OK;
    });
}

dmri_status dmri_load_guess_model(dmri_handle h, const char* path) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        (void)path;
        throw Error(DMRI_E_UNSUPPORTED, "learned guess model not built yet");
    });
}

dmri_status dmri_run(dmri_handle h, int64_t n_pairs, const int32_t* problem_id, const double* b,
                     const double* q, double* signal_out, dmri_stats* stats) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        need_sequence(h);
        if (n_pairs < 0) throw Error(DMRI_E_INVALID, "n_pairs must be >= 0");
        if (n_pairs == 0) return DMRI_OK;
        if (!problem_id || !b || !q || !signal_out) throw Error(DMRI_E_INVALID, "NULL argument");
        for (int64_t i = 0; i < n_pairs; ++i) {
            get_problem(h, problem_id[i]);
            const double nq = std::sqrt(q[3 * i] * q[3 * i] + q[3 * i + 1] * q[3 * i + 1] +
                                        q[3 * i + 2] * q[3 * i + 2]);
            if (!std::isfinite(b[i]) || b[i] < 0 || !std::isfinite(nq) || (b[i] > 0 && !(nq > 0)))
                throw Error(DMRI_E_INVALID, "b must be finite and >= 0, q finite and nonzero");
        }
        const double t_start = now_s();
        if (stats) {
            stats->n_sys = n_pairs;
            stats->total_iterations = 0;
            stats->spmv_rows = 0;
            stats->n_steps = 0;
            stats->t_setup_s = stats->t_solve_s = stats->t_signal_s = 0.0;
            stats->n_kernel_launches = 0;
            stats->t_kernel_s = 0.0;
        }
        bool any_nc = false;
        hipStream_t st = h->stream;
        // Group pairs by problem, keeping input order inside each group.
        for (int32_t pid = 0; pid < static_cast<int32_t>(h->problems.size()); ++pid) {
            std::vector<int64_t> idx;
            for (int64_t i = 0; i < n_pairs; ++i)
                if (problem_id[i] == pid) idx.push_back(i);
            if (idx.empty()) continue;
            ProblemRec& P = get_problem(h, pid);
            const double ts = now_s();
            ensure_uploaded(h, P, h->opt.precision != 0);
            const int64_t ns = static_cast<int64_t>(idx.size());
            std::vector<double> hb(ns), hq(3 * ns);
            for (int64_t i = 0; i < ns; ++i) {
                hb[i] = b[idx[i]];
                for (int a = 0; a < 3; ++a) hq[3 * i + a] = q[3 * idx[i] + a];
            }
            h->ws.b_in.upload(hb.data(), ns, st);
            h->ws.q_in.upload(hq.data(), 3 * ns, st);
            h->ws.sig.alloc(ns);
            if (stats) stats->t_setup_s += now_s() - ts;
            BatchResult R;
            run_batch(h, P, ns, h->ws.b_in.p, h->ws.q_in.p, h->ws.sig.p, R);
            std::vector<double> hs(2 * ns);
            HIPCHK(hipMemcpyAsync(hs.data(), h->ws.sig.p, sizeof(double2) * ns,
                                  hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t i = 0; i < ns; ++i) {
                signal_out[2 * idx[i]] = hs[2 * i];
                signal_out[2 * idx[i] + 1] = hs[2 * i + 1];
                if (R.flags[i]) any_nc = true;
            }
            fill_stats(stats, idx, R, n_pairs);
        }
        (void)t_start;
        return any_nc ? DMRI_NOT_CONVERGED : DMRI_OK;
    });
}

dmri_status dmri_run_device(dmri_handle h, void* hip_stream, int32_t problem_id, int64_t n_pairs,
                            const double* d_b, const double* d_q, double* d_signal,
                            dmri_stats* stats) {
    if (!h) return set_err(nullptr, DMRI_E_INVALID, "NULL handle");
    return guarded(h, [&]() -> dmri_status {
        need_device(h);
        need_sequence(h);
        if (n_pairs <= 0) return n_pairs == 0 ? DMRI_OK : set_err(h, DMRI_E_INVALID, "n_pairs < 0");
        if (!d_b || !d_q || !d_signal) throw Error(DMRI_E_INVALID, "NULL argument");
        ProblemRec& P = get_problem(h, problem_id);
        hipStream_t saved = h->stream;
        if (hip_stream) h->stream = static_cast<hipStream_t>(hip_stream);
        struct Restore {
            dmri_ctx* h;
            hipStream_t s;
            ~Restore() { h->stream = s; }
        } restore{h, saved};
        const double ts = now_s();
        ensure_uploaded(h, P, h->opt.precision != 0);
        if (stats) {
            stats->n_sys = n_pairs;
            stats->total_iterations = 0;
            stats->spmv_rows = 0;
            stats->n_steps = 0;
            stats->t_setup_s = now_s() - ts;
            stats->t_solve_s = stats->t_signal_s = 0.0;
            stats->n_kernel_launches = 0;
            stats->t_kernel_s = 0.0;
        }
        BatchResult R;
        run_batch(h, P, n_pairs, d_b, d_q, reinterpret_cast<double2*>(d_signal), R);
        std::vector<int64_t> idx(n_pairs);
        for (int64_t i = 0; i < n_pairs; ++i) idx[i] = i;
        fill_stats(stats, idx, R, n_pairs);
        for (int32_t fl : R.flags)
            if (fl) return DMRI_NOT_CONVERGED;
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
        const bool f32 = h->opt.precision != 0;
        ensure_uploaded(h, P, f32);
        hipStream_t st = h->stream;
        const int S = h->opt.sys_tile ? h->opt.sys_tile : auto_tile(n_sys);
        const Geom g = make_geom(static_cast<int32_t>(P.op.n_dof), static_cast<int32_t>(n_sys), S,
                                 h->opt.blocks_per_xcd, h->opt.chunk_passes);
        const size_t nrow = static_cast<size_t>(g.n_rows), ld = static_cast<size_t>(g.ld);
        std::vector<double> hc(ld, 0.0), hd(3 * ld, 0.0);
        for (int64_t s = 0; s < n_sys; ++s) {
            hc[s] = c[s];
            for (int a = 0; a < 3; ++a) hd[3 * s + a] = d[3 * s + a];
        }
        DevBuf<double> dc, dd;
        dc.upload(hc.data(), ld, st);
        dd.upload(hd.data(), 3 * ld, st);
        if (!f32) {
            std::vector<double> hx(2 * nrow * ld, 0.0), hy(2 * nrow * ld);
            for (size_t i = 0; i < nrow; ++i)
                for (int64_t s = 0; s < n_sys; ++s)
                    for (int k = 0; k < 2; ++k) hx[2 * (i * ld + s) + k] = x[2 * (i * n_sys + s) + k];
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
                for (int64_t s = 0; s < n_sys; ++s)
                    for (int k = 0; k < 2; ++k) y[2 * (i * n_sys + s) + k] = hy[2 * (i * ld + s) + k];
        } else {
            std::vector<float> hx(2 * nrow * ld, 0.0f), hy(2 * nrow * ld);
            for (size_t i = 0; i < nrow; ++i)
                for (int64_t s = 0; s < n_sys; ++s)
                    for (int k = 0; k < 2; ++k)
                        hx[2 * (i * ld + s) + k] = static_cast<float>(x[2 * (i * n_sys + s) + k]);
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
                for (int64_t s = 0; s < n_sys; ++s)
                    for (int k = 0; k < 2; ++k) y[2 * (i * n_sys + s) + k] = hy[2 * (i * ld + s) + k];
        }
        return DMRI_OK;
    });
}

}  // extern "C"
