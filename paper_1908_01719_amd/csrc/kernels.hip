// Device kernels of libdmri for gfx950 (see kernels.hpp for the layouts).
//
// Work decomposition. A launch covers n_chunks x n_tiles blocks of 256
// threads (4 wavefronts of 64 lanes). A tile is S consecutive systems; a
// chunk is a contiguous range of matrix rows. Inside a wavefront, lane l
// works on system (tile*S + l % S) and on row sub-slot l / S, so a wavefront
// covers 64/S rows x S systems per pass: for S = 64 every lane reads the
// same matrix row (scalar loads, broadcast) and the vector gathers are
// 64 consecutive complex values (1 KiB in FP64); for small batches S = 8
// keeps lanes busy with 8 rows at a time. Consecutive block ids are dealt
// round-robin to the 8 XCDs by the hardware; the block id is remapped so that
// each XCD works on a contiguous part of the mesh and its L2 holds the
// neighbourhood the gathers need.
//
// Reductions (per-system dot products) are FP64 in every precision: lanes
// accumulate their rows, wavefront shuffles and LDS combine a block, each
// block writes one partial per system, and the last block of a tile to
// finish (atomic ticket) adds the partials in chunk order -- deterministic,
// no floating-point atomics -- and updates the per-system Krylov scalars.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

namespace dmri {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

template <typename T> using V2 = typename Vec2Of<T>::type;
template <typename T> using V4 = typename Vec4Of<T>::type;

__device__ __forceinline__ void block_coords(const Geom& g, int& chunk, int& tile) {
    int L = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0) L = (L & 7) * (nb >> 3) + (L >> 3);
    chunk = L / g.n_tiles;
    tile = L - chunk * g.n_tiles;
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-lane coefficients of one operator: c on M_D, (d0, d1, d2) on V.
template <typename T>
struct LaneCoef {
    T c, d0, d1, d2;
    __device__ __forceinline__ LaneCoef(const double4 gg, const Coef k) {
        const double gf = gg.x * k.F;
        c = static_cast<T>(k.cm * gf * gf);
        const double s = k.cd * gf;
        d0 = static_cast<T>(s * gg.y);
        d1 = static_cast<T>(s * gg.z);
        d2 = static_cast<T>(s * gg.w);
    }
};

// Reduce K doubles over the lanes sharing a system, then over the block.
// Result valid in threads [0, S).
template <int S, int K>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* lds) {
#pragma unroll
    for (int off = S; off < 64; off <<= 1) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += __shfl_xor(v[k], off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < S) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds[(wave * S + lane) * K + k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < S) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += lds[(w * S + threadIdx.x) * K + k];
            v[k] = t;
        }
    }
}

// Publish this block's partials (threads [0, S) hold them); the last block
// of the tile to arrive adds all partials in chunk order and runs
// fin(sys, tot) in threads [0, S). Returns true in that last block.
template <int S, int K, typename Fin>
__device__ __forceinline__ bool publish_finalize(const Geom& g, int chunk, int tile,
                                                 double (&v)[K], Scratch sc, Fin fin) {
    __shared__ int is_last;
    if (threadIdx.x < S) {
        const size_t base = (static_cast<size_t>(chunk) * g.ld + tile * S + threadIdx.x) * 4;
#pragma unroll
        for (int k = 0; k < K; ++k) st_agent(sc.partial + base + k, v[k]);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = atomicAdd(&sc.counters[tile], 1);
        is_last = (t == g.n_chunks - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    if (threadIdx.x < S) {
        const int sys = tile * S + threadIdx.x;
        double tot[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tot[k] = 0.0;
        for (int c = 0; c < g.n_chunks; ++c) {
            const size_t base = (static_cast<size_t>(c) * g.ld + sys) * 4;
#pragma unroll
            for (int k = 0; k < K; ++k) tot[k] += ld_agent(sc.partial + base + k);
        }
        fin(sys, tot);
    }
    if (threadIdx.x == 0)
        __hip_atomic_store(&sc.counters[tile], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// Store the number of active systems of a tile (only in the last block).
template <int S>
__device__ __forceinline__ void recount_tile(int tile, SolverState s) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (threadIdx.x < S) {
        const int sys = tile * S + threadIdx.x;
        if (sys < s.n_sys && s.active[sys]) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) s.n_active[tile] = cnt;
}

// Row range of a chunk and the first row / stride of this lane.
template <int S>
struct RowIter {
    int begin, end, stride;
    __device__ __forceinline__ RowIter(const Geom& g, int chunk) {
        constexpr int R = 64 / S;
        const int row0 = chunk * g.chunk_rows;
        int wave = threadIdx.x >> 6;
        if (S == 64) wave = __builtin_amdgcn_readfirstlane(wave);
        const int rs = (threadIdx.x & 63) / S;
        begin = row0 + wave * R + rs;
        end = min(g.n_rows, row0 + g.chunk_rows);
        stride = kWaves * R;
    }
};

// Jacobi diagonal of A_s at a row: dK0 + c dM_D + i d . dV.
template <typename T>
__device__ __forceinline__ void diag_at(const MatView<T>& A, int row, const LaneCoef<T>& lc,
                                        T& dr, T& di) {
    const V4<T> a = A.daux[row];
    dr = A.dK0[row] + lc.c * a.x;
    di = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
}

template <typename T>
__device__ __forceinline__ V2<T> cdivT(V2<T> a, T dr, T di) {
    const T den = dr * dr + di * di;
    V2<T> o;
    o.x = (a.x * dr + a.y * di) / den;
    o.y = (a.y * dr - a.x * di) / den;
    return o;
}

template <typename T>
__device__ __forceinline__ V2<T> mk2(T a, T b) {
    V2<T> o;
    o.x = a;
    o.y = b;
    return o;
}

// Accumulate a dot product term: conj(a) b (Hermitian) or a b (bilinear).
template <bool HERM, typename T>
__device__ __forceinline__ void dot_acc(double& re, double& im, V2<T> a, V2<T> b) {
    if (HERM) {
        re += double(a.x) * b.x + double(a.y) * b.y;
        im += double(a.x) * b.y - double(a.y) * b.x;
    } else {
        re += double(a.x) * b.x - double(a.y) * b.y;
        im += double(a.x) * b.y + double(a.y) * b.x;
    }
}

// --------------------------------------------------------------- kernels

// q = A p and sigma = p^H q (or p^T q); finalize alpha = rho / sigma.
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_spmv_dot(Geom g, MatView<T> A, const double4* gq,
                                                     Coef lhs, const V2<T>* __restrict__ p,
                                                     V2<T>* __restrict__ q, SolverState s,
                                                     Scratch sc) {
    __shared__ double lds[kWaves * S * 2];
    int chunk, tile;
    block_coords(g, chunk, tile);
    const int sys = tile * S + (threadIdx.x & 63) % S;
    const bool act = sys < s.n_sys && s.active[sys];
    if (!__syncthreads_or(act)) return;
    const LaneCoef<T> lc(gq[sys], lhs);
    double acc[2] = {0.0, 0.0};
    if (act) {
        const RowIter<S> it(g, chunk);
        for (int row = it.begin; row < it.end; row += it.stride) {
            const int kb = A.row_ptr[row], ke = A.row_ptr[row + 1];
            T yr = 0, yi = 0;
#pragma unroll 4
            for (int k = kb; k < ke; ++k) {
                const int j = A.col[k];
                const V4<T> a = A.aux[k];
                const T ar = A.K0[k] + lc.c * a.x;
                const T ai = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
                const V2<T> xv = p[static_cast<size_t>(j) * g.ld + sys];
                yr += ar * xv.x - ai * xv.y;
                yi += ar * xv.y + ai * xv.x;
            }
            const size_t idx = static_cast<size_t>(row) * g.ld + sys;
            q[idx] = mk2<T>(yr, yi);
            dot_acc<HERM, T>(acc[0], acc[1], p[idx], mk2<T>(yr, yi));
        }
    }
    block_reduce<S, 2>(acc, lds);
    publish_finalize<S, 2>(g, chunk, tile, acc, sc, [&](int sy, double* tot) {
        if (sy < s.n_sys && s.active[sy]) s.alpha[sy] = cdiv(s.rho[sy], make_double2(tot[0], tot[1]));
    });
}

// x += alpha p, r -= alpha q, z = D^-1 r; rho' = r^H z, ||r||^2; finalize
// convergence, beta = rho'/rho.
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_update(Geom g, MatView<T> A, const double4* gq,
                                                   Coef lhs, V2<T>* __restrict__ x,
                                                   V2<T>* __restrict__ r,
                                                   const V2<T>* __restrict__ p,
                                                   const V2<T>* __restrict__ q, SolverState s,
                                                   Scratch sc) {
    __shared__ double lds[kWaves * S * 3];
    int chunk, tile;
    block_coords(g, chunk, tile);
    const int sys = tile * S + (threadIdx.x & 63) % S;
    const bool act = sys < s.n_sys && s.active[sys];
    if (!__syncthreads_or(act)) return;
    const LaneCoef<T> lc(gq[sys], lhs);
    const double2 al = act ? s.alpha[sys] : make_double2(0.0, 0.0);
    const T ar = static_cast<T>(al.x), ai = static_cast<T>(al.y);
    double acc[3] = {0.0, 0.0, 0.0};
    if (act) {
        const RowIter<S> it(g, chunk);
        for (int row = it.begin; row < it.end; row += it.stride) {
            const size_t idx = static_cast<size_t>(row) * g.ld + sys;
            const V2<T> pv = p[idx], qv = q[idx];
            V2<T> xv = x[idx], rv = r[idx];
            xv.x += ar * pv.x - ai * pv.y;
            xv.y += ar * pv.y + ai * pv.x;
            rv.x -= ar * qv.x - ai * qv.y;
            rv.y -= ar * qv.y + ai * qv.x;
            x[idx] = xv;
            r[idx] = rv;
            T dr, di;
            diag_at(A, row, lc, dr, di);
            dot_acc<HERM, T>(acc[0], acc[1], rv, cdivT<T>(rv, dr, di));
            acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
        }
    }
    block_reduce<S, 3>(acc, lds);
    const bool last = publish_finalize<S, 3>(g, chunk, tile, acc, sc, [&](int sy, double* tot) {
        if (sy >= s.n_sys || !s.active[sy]) return;
        const double2 rho_new = make_double2(tot[0], tot[1]);
        const double rr = tot[2];
        s.rr[sy] = rr;
        const int it_now = s.iters[sy] + 1;
        s.iters[sy] = it_now;
        s.iters_total[sy] += 1;
        bool stop = false;
        if (!isfinite(rr) || !isfinite(rho_new.x) || !isfinite(rho_new.y)) {
            s.flags[sy] |= 2;
            stop = true;
        } else if (rr <= s.rtol2 * s.bb[sy]) {
            stop = true;
        } else if (it_now >= s.max_iter) {
            s.flags[sy] |= 1;
            stop = true;
        }
        if (stop) {
            s.active[sy] = 0;
        } else {
            s.beta[sy] = cdiv(rho_new, s.rho[sy]);
            s.rho[sy] = rho_new;
        }
    });
    if (last) recount_tile<S>(tile, s);
}

// p = D^-1 r + beta p.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_pupdate(Geom g, MatView<T> A, const double4* gq,
                                                    Coef lhs, const V2<T>* __restrict__ r,
                                                    V2<T>* __restrict__ p, SolverState s) {
    int chunk, tile;
    block_coords(g, chunk, tile);
    const int sys = tile * S + (threadIdx.x & 63) % S;
    const bool act = sys < s.n_sys && s.active[sys];
    if (!__syncthreads_or(act)) return;
    if (!act) return;
    const LaneCoef<T> lc(gq[sys], lhs);
    const double2 be = s.beta[sys];
    const T br = static_cast<T>(be.x), bi = static_cast<T>(be.y);
    const RowIter<S> it(g, chunk);
    for (int row = it.begin; row < it.end; row += it.stride) {
        const size_t idx = static_cast<size_t>(row) * g.ld + sys;
        T dr, di;
        diag_at(A, row, lc, dr, di);
        const V2<T> z = cdivT<T>(r[idx], dr, di);
        const V2<T> pv = p[idx];
        p[idx] = mk2<T>(z.x + br * pv.x - bi * pv.y, z.y + br * pv.y + bi * pv.x);
    }
}

// Start of a time step: b = Right(u_prev), x0 = guess, r = b - A x0,
// p = z = D^-1 r; finalize ||b||^2, ||r||^2, rho and the active flags.
template <typename T, int S, bool HERM, int GM>
__global__ __launch_bounds__(kBlock) void k_init(Geom g, MatView<T> A, const double4* gq,
                                                 Coef lhs, Coef rhs,
                                                 const V2<T>* __restrict__ u_prev,
                                                 const V2<T>* __restrict__ u_prev2,
                                                 V2<T>* __restrict__ x, V2<T>* __restrict__ r,
                                                 V2<T>* __restrict__ p, SolverState s,
                                                 Scratch sc) {
    __shared__ double lds[kWaves * S * 4];
    int chunk, tile;
    block_coords(g, chunk, tile);
    const int sys = tile * S + (threadIdx.x & 63) % S;
    const bool act = sys < s.n_sys;
    if (!__syncthreads_or(act)) return;
    const double4 gg = gq[sys];
    const LaneCoef<T> ll(gg, lhs), lr(gg, rhs);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (act) {
        const RowIter<S> it(g, chunk);
        for (int row = it.begin; row < it.end; row += it.stride) {
            const int kb = A.row_ptr[row], ke = A.row_ptr[row + 1];
            T br = 0, bi = 0, axr = 0, axi = 0;
            V2<T> x0_own = mk2<T>(0, 0);
#pragma unroll 2
            for (int k = kb; k < ke; ++k) {
                const int j = A.col[k];
                const V4<T> a = A.aux[k];
                const T vl = ll.d0 * a.y + ll.d1 * a.z + ll.d2 * a.w;
                const T vr = lr.d0 * a.y + lr.d1 * a.z + lr.d2 * a.w;
                const T al = A.K0[k] + ll.c * a.x;
                const T arr = A.Kr[k] + lr.c * a.x;
                const size_t jdx = static_cast<size_t>(j) * g.ld + sys;
                const V2<T> uj = u_prev[jdx];
                V2<T> xj;
                if (GM == 0) {
                    xj = uj;
                } else if (GM == 1) {
                    const V2<T> u2 = u_prev2[jdx];
                    xj = mk2<T>(T(2) * uj.x - u2.x, T(2) * uj.y - u2.y);
                } else {
                    xj = x[jdx];
                }
                if (j == row) x0_own = xj;
                br += arr * uj.x - vr * uj.y;
                bi += arr * uj.y + vr * uj.x;
                axr += al * xj.x - vl * xj.y;
                axi += al * xj.y + vl * xj.x;
            }
            const size_t idx = static_cast<size_t>(row) * g.ld + sys;
            const V2<T> rv = mk2<T>(br - axr, bi - axi);
            if (GM != 2) x[idx] = x0_own;
            r[idx] = rv;
            T dr, di;
            diag_at(A, row, ll, dr, di);
            const V2<T> z = cdivT<T>(rv, dr, di);
            p[idx] = z;
            dot_acc<HERM, T>(acc[0], acc[1], rv, z);
            acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
            acc[3] += double(br) * br + double(bi) * bi;
        }
    }
    block_reduce<S, 4>(acc, lds);
    const bool last = publish_finalize<S, 4>(g, chunk, tile, acc, sc, [&](int sy, double* tot) {
        if (sy >= s.n_sys) return;
        const double rr = tot[2], bb = tot[3];
        s.rho[sy] = make_double2(tot[0], tot[1]);
        s.rr[sy] = rr;
        s.bb[sy] = bb;
        s.iters[sy] = 0;
        int a = 1;
        if (!isfinite(rr) || !isfinite(bb)) {
            s.flags[sy] |= 2;
            a = 0;
        } else if (rr <= s.rtol2 * bb) {
            a = 0;
        }
        s.active[sy] = a;
    });
    if (last) recount_tile<S>(tile, s);
}

// Signal: S_s = sum_i w_i x_is in FP64.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_signal(Geom g, const double* __restrict__ w,
                                                   const V2<T>* __restrict__ x,
                                                   double2* __restrict__ out, int32_t n_sys,
                                                   Scratch sc) {
    __shared__ double lds[kWaves * S * 2];
    int chunk, tile;
    block_coords(g, chunk, tile);
    const int sys = tile * S + (threadIdx.x & 63) % S;
    double acc[2] = {0.0, 0.0};
    if (sys < n_sys) {
        const RowIter<S> it(g, chunk);
        for (int row = it.begin; row < it.end; row += it.stride) {
            const V2<T> xv = x[static_cast<size_t>(row) * g.ld + sys];
            acc[0] += w[row] * double(xv.x);
            acc[1] += w[row] * double(xv.y);
        }
    }
    block_reduce<S, 2>(acc, lds);
    publish_finalize<S, 2>(g, chunk, tile, acc, sc, [&](int sy, double* tot) {
        if (sy < n_sys) out[sy] = make_double2(tot[0], tot[1]);
    });
}

// y = (Base + c M_D + i d.V) x with explicit per-system coefficients.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, MatView<T> A, int which,
                                                  const double* __restrict__ cc,
                                                  const double3* __restrict__ dd,
                                                  const V2<T>* __restrict__ x,
                                                  V2<T>* __restrict__ y) {
    int chunk, tile;
    block_coords(g, chunk, tile);
    const int sys = tile * S + (threadIdx.x & 63) % S;
    const T c = static_cast<T>(cc[sys]);
    const double3 d3 = dd[sys];
    const T d0 = static_cast<T>(d3.x), d1 = static_cast<T>(d3.y), d2 = static_cast<T>(d3.z);
    const T* base = which == 0 ? A.K0 : A.Kr;
    const RowIter<S> it(g, chunk);
    for (int row = it.begin; row < it.end; row += it.stride) {
        T yr = 0, yi = 0;
        for (int k = A.row_ptr[row]; k < A.row_ptr[row + 1]; ++k) {
            const V4<T> a = A.aux[k];
            const T ar = base[k] + c * a.x;
            const T ai = d0 * a.y + d1 * a.z + d2 * a.w;
            const V2<T> xv = x[static_cast<size_t>(A.col[k]) * g.ld + sys];
            yr += ar * xv.x - ai * xv.y;
            yi += ar * xv.y + ai * xv.x;
        }
        y[static_cast<size_t>(row) * g.ld + sys] = mk2<T>(yr, yi);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_initial(int64_t n, int32_t ld, int32_t n_sys,
                                                        const double* __restrict__ u0,
                                                        V2<T>* __restrict__ x) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t row = i / ld;
    const int sys = static_cast<int>(i - row * ld);
    x[i] = mk2<T>(sys < n_sys ? static_cast<T>(u0[row]) : T(0), T(0));
}

__global__ void k_sys_params(int32_t n_sys, int32_t ld, const double* __restrict__ b,
                             const double* __restrict__ q, double int_F2,
                             double4* __restrict__ gq, int32_t* __restrict__ bad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ld) return;
    if (s >= n_sys) {
        gq[s] = make_double4(0.0, 1.0, 0.0, 0.0);
        return;
    }
    const double bv = b[s];
    const double qx = q[3 * s], qy = q[3 * s + 1], qz = q[3 * s + 2];
    const double nq = sqrt(qx * qx + qy * qy + qz * qz);
    bool ok = isfinite(bv) && bv >= 0.0 && isfinite(nq);
    if (ok && bv > 0.0 && !(nq > 0.0)) ok = false;
    if (!ok) {
        atomicOr(bad, 1);
        gq[s] = make_double4(0.0, 1.0, 0.0, 0.0);
        return;
    }
    if (bv == 0.0) {
        gq[s] = make_double4(0.0, 1.0, 0.0, 0.0);
    } else {
        gq[s] = make_double4(sqrt(bv / int_F2), qx / nq, qy / nq, qz / nq);
    }
}

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw std::runtime_error(std::string("kernel launch failed (") + what + "): " +
                                 hipGetErrorString(e));
}

inline unsigned grid_of(const Geom& g) {
    return static_cast<unsigned>(g.n_chunks) * static_cast<unsigned>(g.n_tiles);
}

}  // namespace

// ------------------------------------------------------------- launchers

Geom make_geom(int32_t n_rows, int32_t n_sys, int32_t S, int32_t target_blocks) {
    Geom g{};
    g.n_rows = n_rows;
    g.S = S;
    g.n_tiles = (n_sys + S - 1) / S;
    if (g.n_tiles < 1) g.n_tiles = 1;
    g.ld = g.n_tiles * S;
    const int32_t pass = kWaves * (64 / S);
    const int32_t max_chunks = std::max(1, (n_rows + pass - 1) / pass);
    int32_t nc = std::max(1, target_blocks / g.n_tiles);
    nc = std::min(nc, max_chunks);
    int32_t rows = (n_rows + nc - 1) / nc;
    rows = ((rows + pass - 1) / pass) * pass;
    if (rows < pass) rows = pass;
    g.chunk_rows = rows;
    g.n_chunks = std::max(1, (n_rows + rows - 1) / rows);
    return g;
}

#define DMRI_DISPATCH_S(S_, ...)                                             \
    switch (S_) {                                                            \
        case 8: { constexpr int S = 8; __VA_ARGS__; } break;                 \
        case 16: { constexpr int S = 16; __VA_ARGS__; } break;               \
        case 32: { constexpr int S = 32; __VA_ARGS__; } break;               \
        case 64: { constexpr int S = 64; __VA_ARGS__; } break;               \
        default: throw std::runtime_error("unsupported tile width");         \
    }

template <typename T>
void launch_init(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq, Coef lhs,
                 Coef rhs, bool herm, int guess_mode, const V2<T>* u_prev, const V2<T>* u_prev2,
                 V2<T>* x, V2<T>* r, V2<T>* p, SolverState s, Scratch sc) {
    const dim3 grid(grid_of(g)), block(kBlock);
#define DMRI_INIT(H, GMV) \
    k_init<T, S, H, GMV><<<grid, block, 0, st>>>(g, A, gq, lhs, rhs, u_prev, u_prev2, x, r, p, s, sc)
    DMRI_DISPATCH_S(g.S, {
        if (herm) {
            if (guess_mode == 0) DMRI_INIT(true, 0);
            else if (guess_mode == 1) DMRI_INIT(true, 1);
            else DMRI_INIT(true, 2);
        } else {
            if (guess_mode == 0) DMRI_INIT(false, 0);
            else if (guess_mode == 1) DMRI_INIT(false, 1);
            else DMRI_INIT(false, 2);
        }
    });
#undef DMRI_INIT
    check_launch("init");
}

template <typename T>
void launch_spmv_dot(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                     Coef lhs, bool herm, const V2<T>* p, V2<T>* q, SolverState s, Scratch sc) {
    const dim3 grid(grid_of(g)), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        if (herm) k_spmv_dot<T, S, true><<<grid, block, 0, st>>>(g, A, gq, lhs, p, q, s, sc);
        else k_spmv_dot<T, S, false><<<grid, block, 0, st>>>(g, A, gq, lhs, p, q, s, sc);
    });
    check_launch("spmv_dot");
}

template <typename T>
void launch_update(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                   Coef lhs, bool herm, V2<T>* x, V2<T>* r, const V2<T>* p, const V2<T>* q,
                   SolverState s, Scratch sc) {
    const dim3 grid(grid_of(g)), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        if (herm) k_update<T, S, true><<<grid, block, 0, st>>>(g, A, gq, lhs, x, r, p, q, s, sc);
        else k_update<T, S, false><<<grid, block, 0, st>>>(g, A, gq, lhs, x, r, p, q, s, sc);
    });
    check_launch("update");
}

template <typename T>
void launch_pupdate(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                    Coef lhs, const V2<T>* r, V2<T>* p, SolverState s) {
    const dim3 grid(grid_of(g)), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_pupdate<T, S><<<grid, block, 0, st>>>(g, A, gq, lhs, r, p, s); });
    check_launch("pupdate");
}

template <typename T>
void launch_signal(hipStream_t st, const Geom& g, const double* w, const V2<T>* x, double2* out,
                   int32_t n_sys, Scratch sc) {
    const dim3 grid(grid_of(g)), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_signal<T, S><<<grid, block, 0, st>>>(g, w, x, out, n_sys, sc); });
    check_launch("signal");
}

template <typename T>
void launch_apply(hipStream_t st, const Geom& g, const MatView<T>& A, int which, const double* c,
                  const double3* d, const V2<T>* x, V2<T>* y) {
    const dim3 grid(grid_of(g)), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_apply<T, S><<<grid, block, 0, st>>>(g, A, which, c, d, x, y); });
    check_launch("apply");
}

template <typename T>
void launch_set_initial(hipStream_t st, const Geom& g, const double* u0, int32_t n_sys,
                        V2<T>* x) {
    const int64_t n = static_cast<int64_t>(g.n_rows) * g.ld;
    const unsigned blocks = static_cast<unsigned>((n + kBlock - 1) / kBlock);
    k_set_initial<T><<<blocks, kBlock, 0, st>>>(n, g.ld, n_sys, u0, x);
    check_launch("set_initial");
}

void launch_sys_params(hipStream_t st, int32_t n_sys, int32_t ld, const double* b, const double* q,
                       double int_F2, double4* gq, int32_t* bad) {
    const unsigned blocks = static_cast<unsigned>((ld + 255) / 256);
    k_sys_params<<<blocks, 256, 0, st>>>(n_sys, ld, b, q, int_F2, gq, bad);
    check_launch("sys_params");
}

#define DMRI_INST(T)                                                                          \
    template void launch_init<T>(hipStream_t, const Geom&, const MatView<T>&, const double4*,  \
                                 Coef, Coef, bool, int, const V2<T>*, const V2<T>*, V2<T>*,    \
                                 V2<T>*, V2<T>*, SolverState, Scratch);                        \
    template void launch_spmv_dot<T>(hipStream_t, const Geom&, const MatView<T>&,              \
                                     const double4*, Coef, bool, const V2<T>*, V2<T>*,         \
                                     SolverState, Scratch);                                    \
    template void launch_update<T>(hipStream_t, const Geom&, const MatView<T>&,                \
                                   const double4*, Coef, bool, V2<T>*, V2<T>*, const V2<T>*,   \
                                   const V2<T>*, SolverState, Scratch);                        \
    template void launch_pupdate<T>(hipStream_t, const Geom&, const MatView<T>&,               \
                                    const double4*, Coef, const V2<T>*, V2<T>*, SolverState);  \
    template void launch_signal<T>(hipStream_t, const Geom&, const double*, const V2<T>*,      \
                                   double2*, int32_t, Scratch);                                \
    template void launch_apply<T>(hipStream_t, const Geom&, const MatView<T>&, int,            \
                                  const double*, const double3*, const V2<T>*, V2<T>*);        \
    template void launch_set_initial<T>(hipStream_t, const Geom&, const double*, int32_t,      \
                                        V2<T>*);

DMRI_INST(double)
DMRI_INST(float)

}  // namespace dmri
