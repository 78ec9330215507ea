// Device kernels of libdmri for gfx950 (see kernels.hpp for the layouts and
// the XCD-sweep work decomposition).
//
// Inside a wavefront, lane l works on system (tile*S + l % S) and on row
// sub-slot l / S, so one pass of a wavefront covers 64/S rows x S systems:
// for S = 64 every lane reads the same matrix row (uniform loads) and the
// vector gathers are 64 consecutive complex values (1 KiB in FP64); for
// small batches S = 8 keeps all lanes busy with 8 rows at a time.
//
// Reductions (per-system dot products) are FP64 in every precision: lanes
// accumulate their rows, wavefront shuffles and LDS combine a block, each
// block stores one partial per system and item, and a finalize kernel adds
// them in a fixed order. The hot kernels contain no fences and no atomics.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>

namespace dmri {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

template <typename T> using V2 = typename Vec2Of<T>::type;
template <typename T> using V4 = typename Vec4Of<T>::type;

enum FinMode { FIN_ALPHA = 0, FIN_BETA = 1, FIN_INIT = 2, FIN_SIGNAL = 3 };

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
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

template <typename T>
__device__ __forceinline__ V2<T> cdivT(V2<T> a, T dr, T di) {
    const T den = dr * dr + di * di;
    return mk2<T>((a.x * dr + a.y * di) / den, (a.y * dr - a.x * di) / den);
}

// Jacobi diagonal of A_s at a row: dK0 + c dM_D + i d . dV.
template <typename T>
__device__ __forceinline__ void diag_at(const T* __restrict__ dK0, const V4<T>* __restrict__ daux,
                                        int row, const LaneCoef<T>& lc, T& dr, T& di) {
    const V4<T> a = daux[row];
    dr = dK0[row] + lc.c * a.x;
    di = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
}

// Visit this block's rows of one item: block j takes chunks j, j+B, ...
template <int S, typename Body>
__device__ __forceinline__ void sweep_rows(const Geom& g, int part, int j, Body body) {
    constexpr int R = 64 / S;
    const int r0 = part * g.part_rows;
    const int r1 = min(g.n_rows, r0 + g.part_rows);
    int wave = threadIdx.x >> 6;
    if (S == 64) wave = __builtin_amdgcn_readfirstlane(wave);
    const int off = wave * R + (threadIdx.x & 63) / S;
    const int step = g.B * g.chunk_rows;
    for (int c0 = r0 + j * g.chunk_rows; c0 < r1; c0 += step) {
        const int c1 = min(r1, c0 + g.chunk_rows);
        for (int row = c0 + off; row < c1; row += kWaves * R) body(row);
    }
}

// Reduce K doubles over the lanes sharing a system, then over the block,
// and store the block's partial for (item, j). Ends with a barrier.
template <int S, int K>
__device__ __forceinline__ void reduce_store(const Geom& g, Scratch sc, int item, int j,
                                             double (&v)[K], double* lds) {
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
        double* dst = sc.partial + ((static_cast<size_t>(item) * g.B + j) * S + threadIdx.x) * 4;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += lds[(w * S + threadIdx.x) * K + k];
            dst[k] = t;
        }
    }
    __syncthreads();
}

// --------------------------------------------------------------- kernels

// q = A p and sigma = p^H q (or p^T q) per system.
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_spmv_dot(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ K0, const V4<T>* __restrict__ aux, const double4* __restrict__ gq,
    Coef lhs, const V2<T>* __restrict__ p, V2<T>* __restrict__ q, SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * S * 2];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int item = xcd; item < g.n_items; item += 8) {
        const int tile = item / g.n_parts, part = item - tile * g.n_parts;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        const LaneCoef<T> lc(gq[sys], lhs);
        double acc[2] = {0.0, 0.0};
        if (act) {
            sweep_rows<S>(g, part, j, [&](int row) {
                const int kb = row_ptr[row], ke = row_ptr[row + 1];
                T yr = 0, yi = 0;
#pragma unroll 4
                for (int k = kb; k < ke; ++k) {
                    const int jj = col[k];
                    const V4<T> a = aux[k];
                    const T ar = K0[k] + lc.c * a.x;
                    const T ai = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
                    const V2<T> xv = p[static_cast<size_t>(jj) * g.ld + sys];
                    yr += ar * xv.x - ai * xv.y;
                    yi += ar * xv.y + ai * xv.x;
                }
                const size_t idx = static_cast<size_t>(row) * g.ld + sys;
                q[idx] = mk2<T>(yr, yi);
                dot_acc<HERM, T>(acc[0], acc[1], p[idx], mk2<T>(yr, yi));
            });
        }
        reduce_store<S, 2>(g, sc, item, j, acc, lds);
    }
}

// x += alpha p, r -= alpha q, z = D^-1 r; rho' = r^H z (or r^T z), ||r||^2.
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_update(
    Geom g, const T* __restrict__ dK0, const V4<T>* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, V2<T>* __restrict__ x, V2<T>* __restrict__ r,
    const V2<T>* __restrict__ p, const V2<T>* __restrict__ q, SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * S * 3];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int item = xcd; item < g.n_items; item += 8) {
        const int tile = item / g.n_parts, part = item - tile * g.n_parts;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        const LaneCoef<T> lc(gq[sys], lhs);
        const double2 al = act ? s.alpha[sys] : make_double2(0.0, 0.0);
        const T ar = static_cast<T>(al.x), ai = static_cast<T>(al.y);
        double acc[3] = {0.0, 0.0, 0.0};
        if (act) {
            sweep_rows<S>(g, part, j, [&](int row) {
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
                diag_at(dK0, daux, row, lc, dr, di);
                dot_acc<HERM, T>(acc[0], acc[1], rv, cdivT<T>(rv, dr, di));
                acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
            });
        }
        reduce_store<S, 3>(g, sc, item, j, acc, lds);
    }
}

// p = D^-1 r + beta p.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_pupdate(Geom g, const T* __restrict__ dK0,
                                                    const V4<T>* __restrict__ daux,
                                                    const double4* __restrict__ gq, Coef lhs,
                                                    const V2<T>* __restrict__ r,
                                                    V2<T>* __restrict__ p, SolverState s) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int item = xcd; item < g.n_items; item += 8) {
        const int tile = item / g.n_parts, part = item - tile * g.n_parts;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        if (!(sys < s.n_sys && s.active[sys])) continue;
        const LaneCoef<T> lc(gq[sys], lhs);
        const double2 be = s.beta[sys];
        const T br = static_cast<T>(be.x), bi = static_cast<T>(be.y);
        sweep_rows<S>(g, part, j, [&](int row) {
            const size_t idx = static_cast<size_t>(row) * g.ld + sys;
            T dr, di;
            diag_at(dK0, daux, row, lc, dr, di);
            const V2<T> z = cdivT<T>(r[idx], dr, di);
            const V2<T> pv = p[idx];
            p[idx] = mk2<T>(z.x + br * pv.x - bi * pv.y, z.y + br * pv.y + bi * pv.x);
        });
    }
}

// Start of a time step: b = Right(u_prev), x0 = guess, r = b - A x0,
// p = z = D^-1 r; partials rho, ||r||^2, ||b||^2.
template <typename T, int S, bool HERM, int GM>
__global__ __launch_bounds__(kBlock) void k_init(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ K0, const T* __restrict__ Kr, const V4<T>* __restrict__ aux,
    const T* __restrict__ dK0, const V4<T>* __restrict__ daux, const double4* __restrict__ gq,
    Coef lhs, Coef rhs, const V2<T>* __restrict__ u_prev, const V2<T>* __restrict__ u_prev2,
    V2<T>* __restrict__ x, V2<T>* __restrict__ r, V2<T>* __restrict__ p, SolverState s,
    Scratch sc) {
    __shared__ double lds[kWaves * S * 4];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int item = xcd; item < g.n_items; item += 8) {
        const int tile = item / g.n_parts, part = item - tile * g.n_parts;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const bool act = sys < s.n_sys;
        const double4 gg = gq[sys];
        const LaneCoef<T> ll(gg, lhs), lr(gg, rhs);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (act) {
            sweep_rows<S>(g, part, j, [&](int row) {
                const int kb = row_ptr[row], ke = row_ptr[row + 1];
                T br = 0, bi = 0, axr = 0, axi = 0;
                V2<T> x0_own = mk2<T>(0, 0);
#pragma unroll 2
                for (int k = kb; k < ke; ++k) {
                    const int jj = col[k];
                    const V4<T> a = aux[k];
                    const T vl = ll.d0 * a.y + ll.d1 * a.z + ll.d2 * a.w;
                    const T vr = lr.d0 * a.y + lr.d1 * a.z + lr.d2 * a.w;
                    const T al = K0[k] + ll.c * a.x;
                    const T arr = Kr[k] + lr.c * a.x;
                    const size_t jdx = static_cast<size_t>(jj) * g.ld + sys;
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
                    if (jj == row) x0_own = xj;
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
                diag_at(dK0, daux, row, ll, dr, di);
                const V2<T> z = cdivT<T>(rv, dr, di);
                p[idx] = z;
                dot_acc<HERM, T>(acc[0], acc[1], rv, z);
                acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
                acc[3] += double(br) * br + double(bi) * bi;
            });
        }
        reduce_store<S, 4>(g, sc, item, j, acc, lds);
    }
}

// Signal partials: sum_i w_i x_is in FP64.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_signal(Geom g, const double* __restrict__ w,
                                                   const V2<T>* __restrict__ x, int32_t n_sys,
                                                   Scratch sc) {
    __shared__ double lds[kWaves * S * 2];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int item = xcd; item < g.n_items; item += 8) {
        const int tile = item / g.n_parts, part = item - tile * g.n_parts;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        double acc[2] = {0.0, 0.0};
        if (sys < n_sys) {
            sweep_rows<S>(g, part, j, [&](int row) {
                const V2<T> xv = x[static_cast<size_t>(row) * g.ld + sys];
                acc[0] += w[row] * double(xv.x);
                acc[1] += w[row] * double(xv.y);
            });
        }
        reduce_store<S, 2>(g, sc, item, j, acc, lds);
    }
}

// Add a tile's partials in a fixed order and update the per-system scalars.
// One block per tile; thread (grp, s) sums partials grp, grp+G, ... of
// system s, then the groups are combined in order.
template <int S, int K, int MODE>
__global__ __launch_bounds__(kBlock) void k_finalize(Geom g, SolverState s, Scratch sc,
                                                     double2* __restrict__ out, int32_t n_sig) {
    constexpr int G = kBlock / S;
    __shared__ double lds[kBlock * K];
    __shared__ int cnt;
    const int tile = blockIdx.x;
    const int grp = threadIdx.x / S, sl = threadIdx.x % S;
    const int sys = tile * S + sl;
    if (MODE == FIN_ALPHA || MODE == FIN_BETA) {
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) return;
    }
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int nb = g.n_parts * g.B;
    const double* base = sc.partial + static_cast<size_t>(tile) * nb * S * 4;
    for (int i = grp; i < nb; i += G) {
        const double* pp = base + (static_cast<size_t>(i) * S + sl) * 4;
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += pp[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) lds[threadIdx.x * K + k] = acc[k];
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    if (threadIdx.x < S) {
        double tot[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
            for (int gg = 0; gg < G; ++gg) t += lds[(gg * S + sl) * K + k];
            tot[k] = t;
        }
        if (MODE == FIN_SIGNAL) {
            if (sys < n_sig) out[sys] = make_double2(tot[0], tot[1]);
        } else if (MODE == FIN_ALPHA) {
            if (sys < s.n_sys && s.active[sys])
                s.alpha[sys] = cdiv(s.rho[sys], make_double2(tot[0], tot[1]));
        } else if (MODE == FIN_BETA) {
            if (sys < s.n_sys && s.active[sys]) {
                const double2 rho_new = make_double2(tot[0], tot[1]);
                const double rr = tot[2];
                s.rr[sys] = rr;
                const int it_now = s.iters[sys] + 1;
                s.iters[sys] = it_now;
                s.iters_total[sys] += 1;
                bool stop = false;
                if (!isfinite(rr) || !isfinite(rho_new.x) || !isfinite(rho_new.y)) {
                    s.flags[sys] |= 2;
                    stop = true;
                } else if (rr <= s.rtol2 * s.bb[sys]) {
                    stop = true;
                } else if (it_now >= s.max_iter) {
                    s.flags[sys] |= 1;
                    stop = true;
                }
                if (stop) {
                    s.active[sys] = 0;
                } else {
                    s.beta[sys] = cdiv(rho_new, s.rho[sys]);
                    s.rho[sys] = rho_new;
                    atomicAdd(&cnt, 1);
                }
            }
        } else {  // FIN_INIT
            if (sys < s.n_sys) {
                const double rr = tot[2], bb = tot[3];
                s.rho[sys] = make_double2(tot[0], tot[1]);
                s.rr[sys] = rr;
                s.bb[sys] = bb;
                s.iters[sys] = 0;
                int a = 1;
                if (!isfinite(rr) || !isfinite(bb)) {
                    s.flags[sys] |= 2;
                    a = 0;
                } else if (rr <= s.rtol2 * bb) {
                    a = 0;
                }
                s.active[sys] = a;
                if (a) atomicAdd(&cnt, 1);
            }
        }
    }
    __syncthreads();
    if ((MODE == FIN_BETA || MODE == FIN_INIT) && threadIdx.x == 0) s.n_active[tile] = cnt;
}

// y = (Base + c M_D + i d.V) x with explicit per-system coefficients.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_apply(Geom g, MatView<T> A, int which,
                                                  const double* __restrict__ cc,
                                                  const double3* __restrict__ dd,
                                                  const V2<T>* __restrict__ x,
                                                  V2<T>* __restrict__ y) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const T* base = which == 0 ? A.K0 : A.Kr;
    for (int item = xcd; item < g.n_items; item += 8) {
        const int tile = item / g.n_parts, part = item - tile * g.n_parts;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const T c = static_cast<T>(cc[sys]);
        const double3 d3 = dd[sys];
        const T d0 = static_cast<T>(d3.x), d1 = static_cast<T>(d3.y), d2 = static_cast<T>(d3.z);
        sweep_rows<S>(g, part, j, [&](int row) {
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
        });
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

__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
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

inline dim3 grid_of(const Geom& g) { return dim3(8u * static_cast<unsigned>(g.B)); }

template <int MODE, int K>
void launch_fin(hipStream_t st, const Geom& g, SolverState s, Scratch sc, double2* out,
                int32_t n_sig) {
    const dim3 grid(static_cast<unsigned>(g.n_tiles)), block(kBlock);
    switch (g.S) {
        case 8: k_finalize<8, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig); break;
        case 16: k_finalize<16, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig); break;
        case 32: k_finalize<32, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig); break;
        case 64: k_finalize<64, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig); break;
        default: throw std::runtime_error("unsupported tile width");
    }
    check_launch("finalize");
}

}  // namespace

// ------------------------------------------------------------- launchers

Geom make_geom(int32_t n_rows, int32_t n_sys, int32_t S, int32_t blocks_per_xcd,
               int32_t chunk_passes) {
    Geom g{};
    g.n_rows = n_rows;
    g.S = S;
    g.n_tiles = std::max(1, (n_sys + S - 1) / S);
    g.ld = g.n_tiles * S;
    g.n_parts = 8 / std::gcd(g.n_tiles, 8);
    g.n_items = g.n_tiles * g.n_parts;
    g.chunk_rows = kWaves * (64 / S) * std::max(1, chunk_passes);
    int32_t pr = (n_rows + g.n_parts - 1) / g.n_parts;
    pr = ((pr + g.chunk_rows - 1) / g.chunk_rows) * g.chunk_rows;
    g.part_rows = std::max(pr, g.chunk_rows);
    const int32_t chunks = (g.part_rows + g.chunk_rows - 1) / g.chunk_rows;
    g.B = std::max(1, std::min(blocks_per_xcd, chunks));
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
    const dim3 grid = grid_of(g), block(kBlock);
#define DMRI_INIT(H, GMV)                                                                     \
    k_init<T, S, H, GMV><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.Kr, A.aux, A.dK0, \
                                                 A.daux, gq, lhs, rhs, u_prev, u_prev2, x, r, p, \
                                                 s, sc)
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
    launch_fin<FIN_INIT, 4>(st, g, s, sc, nullptr, 0);
}

template <typename T>
void launch_spmv_dot(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                     Coef lhs, bool herm, const V2<T>* p, V2<T>* q, SolverState s, Scratch sc) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        if (herm)
            k_spmv_dot<T, S, true><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.aux, gq,
                                                           lhs, p, q, s, sc);
        else
            k_spmv_dot<T, S, false><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.aux, gq,
                                                            lhs, p, q, s, sc);
    });
    check_launch("spmv_dot");
    launch_fin<FIN_ALPHA, 2>(st, g, s, sc, nullptr, 0);
}

template <typename T>
void launch_update(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                   Coef lhs, bool herm, V2<T>* x, V2<T>* r, const V2<T>* p, const V2<T>* q,
                   SolverState s, Scratch sc) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        if (herm)
            k_update<T, S, true><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, x, r, p, q, s,
                                                         sc);
        else
            k_update<T, S, false><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, x, r, p, q,
                                                          s, sc);
    });
    check_launch("update");
    launch_fin<FIN_BETA, 3>(st, g, s, sc, nullptr, 0);
}

template <typename T>
void launch_pupdate(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                    Coef lhs, const V2<T>* r, V2<T>* p, SolverState s) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        k_pupdate<T, S><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, r, p, s);
    });
    check_launch("pupdate");
}

template <typename T>
void launch_signal(hipStream_t st, const Geom& g, const double* w, const V2<T>* x, double2* out,
                   int32_t n_sys, Scratch sc) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_signal<T, S><<<grid, block, 0, st>>>(g, w, x, n_sys, sc); });
    check_launch("signal");
    launch_fin<FIN_SIGNAL, 2>(st, g, SolverState{}, sc, out, n_sys);
}

template <typename T>
void launch_apply(hipStream_t st, const Geom& g, const MatView<T>& A, int which, const double* c,
                  const double3* d, const V2<T>* x, V2<T>* y) {
    const dim3 grid = grid_of(g), block(kBlock);
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

void launch_zero_i32(hipStream_t st, int32_t* p, int64_t n) {
    if (n <= 0) return;
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    k_zero_i32<<<blocks, 256, 0, st>>>(p, n);
    check_launch("zero");
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
