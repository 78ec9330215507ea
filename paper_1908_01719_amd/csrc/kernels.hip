// Device kernels of libdmri for gfx950 (see kernels.hpp for the layouts and
// the XCD-sweep work decomposition).
//
// Inside a wavefront, lane l works on system (tile*S + l % S) and on row
// sub-slot l / S, so one pass of a wavefront covers 64/S rows x S systems:
// for S = 64 every lane reads the same matrix row (uniform scalar loads) and
// the vector accesses are 64 consecutive complex values (1 KiB in FP64); for
// small batches S = 8 keeps all lanes busy with 8 rows at a time.
//
// Streaming kernels (vector updates) handle kUs row slots per wavefront per
// chunk; out-of-range slots are clamped to a valid row and masked, so every
// load of a chunk is issued before the first use (memory-level parallelism).
//
// Reductions (per-system dot products) are FP64 in every precision: lanes
// accumulate their rows, wavefront shuffles and LDS combine a block, each
// block stores one partial per system and item, and a finalize kernel adds
// them in a fixed order. The hot kernels contain no fences.
#include "kernels.hpp"
#include "mlp.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <string>
#include <type_traits>

namespace dmri {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
#ifndef DMRI_ROW_SLOTS
#define DMRI_ROW_SLOTS 4
#endif
constexpr int kUs = DMRI_ROW_SLOTS;  // row slots per wavefront per chunk
constexpr int kUg = 2;  // row slots per wavefront per queue grab (gather kernels)
constexpr int kLdsRowCap = 32;  // LDS staging: padded entries per row budgeted
constexpr int kPairS = 128;     // systems per tile of the paired-lane FP32 kernels
constexpr int kSpmvRows = 2;    // rows per lane processed together in the LDS SpMV

template <typename T> using V2 = typename Vec2Of<T>::type;
template <typename T> using V4 = typename Vec4Of<T>::type;

// FIN_REFINE: as FIN_INIT for a refinement pass, keeping the step's ||b||^2.
// Flexible CG with a polynomial preconditioner: FIN_CHECK takes the
// convergence decision of FIN_BETA from ||r||^2 alone; FIN_FLEX0 / FIN_FLEX
// read rho' = r^H z and q^H z of the preconditioned residual z and set
// beta = 0 (first direction) or beta = -(q^H z) / (p^H q).
enum FinMode {
    FIN_ALPHA = 0,
    FIN_BETA = 1,
    FIN_INIT = 2,
    FIN_SIGNAL = 3,
    FIN_REFINE = 4,
    FIN_CHECK = 5,
    FIN_FLEX0 = 6,
    FIN_FLEX = 7
};

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Per-lane coefficients of one operator: c on M_D, (d0, d1, d2) on V.
// For anisotropic problems the mass coefficient of a row is c times the
// lane system's q.D_k q of the row's compartment k (cr(row)).
template <typename T>
struct LaneCoef {
    T c, d0, d1, d2;
    const int32_t* comp;
    const double* acs;  // acomp + sys (stride ld)
    int32_t ld;
    __device__ __forceinline__ LaneCoef(const double4 gg, const Coef k, const Geom& g, int sys) {
        const double gf = gg.x * k.F;
        c = static_cast<T>(k.cm * gf * gf);
        const double s = k.cd * gf;
        d0 = static_cast<T>(s * gg.y);
        d1 = static_cast<T>(s * gg.z);
        d2 = static_cast<T>(s * gg.w);
        comp = g.comp;
        acs = g.acomp ? g.acomp + sys : nullptr;
        ld = g.acomp_ld;
    }
    __device__ __forceinline__ T cr(int row) const {
        return comp ? static_cast<T>(static_cast<double>(c) * acs[static_cast<size_t>(comp[row]) * ld])
                    : c;
    }
};

// Store that bypasses cache allocation (the value is not re-read soon), so
// streamed outputs do not evict the gather working set from L2.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_nt(double2* p, double2 v) {
    nt_d2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_d2*>(p));
}
__device__ __forceinline__ void store_nt(float2* p, float2 v) {
    nt_f2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f2*>(p));
}
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt(float4* p, float4 v) {
    nt_f4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<nt_f4*>(p));
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

template <typename T>
__device__ __forceinline__ V2<T> cdivT(V2<T> a, T dr, T di) {
    const T inv = T(1) / (dr * dr + di * di);
    return mk2<T>((a.x * dr + a.y * di) * inv, (a.y * dr - a.x * di) * inv);
}

// Jacobi diagonal of A_s at a row: dK0 + c dM_D + i d . dV.
template <typename T>
__device__ __forceinline__ void diag_at(const T* __restrict__ dK0, const V4<T>* __restrict__ daux,
                                        int row, const LaneCoef<T>& lc, T& dr, T& di) {
    const V4<T> a = daux[row];
    dr = dK0[row] + lc.cr(row) * a.x;
    di = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
}

// Vectors are stored tile-major: [n_tiles][n_rows][S] complex, so the rows of
// one tile are contiguous (S complex values per row) and spread evenly over
// the L2 channels. Element (row, sys) of the tile is at vbase + row * S.
__device__ __forceinline__ size_t vbase(const Geom& g, int tile, int S, int sys) {
    // Several meshes: tile t holds only its mesh's rows, from element
    // mtab[4t + 2] + lo * S on (the base may be below zero; the sum is not).
    if (g.mtab)
        return static_cast<size_t>(g.mtab[4 * tile + 2]) + static_cast<size_t>(sys - tile * S);
    return static_cast<size_t>(tile) * g.n_rows * S + (sys - tile * S);
}

// Rows [r0, r1) of row part `part` of a tile: a slice of the tile's mesh,
// whose parts have their own length (all rows when the batch has one mesh).
__device__ __forceinline__ void part_range(const Geom& g, int tile, int part, int& r0, int& r1) {
    int lo = 0, hi = g.n_rows, pr = g.part_rows;
    if (g.mtab) {
        lo = static_cast<int>(g.mtab[4 * tile]);
        hi = static_cast<int>(g.mtab[4 * tile + 1]);
        pr = static_cast<int>(g.mtab[4 * tile + 3]);
    }
    r0 = lo + part * pr;
    r1 = min(hi, r0 + pr);
}

// Work item kk of a launch: its tile (through the schedule list when the
// launch is restricted to some tiles), its row part, and the slot
// tile * n_parts + part that addresses its partials and queue counter.
struct ItemRef {
    int tile, part, item;
};
__device__ __forceinline__ ItemRef item_ref(const Geom& g, int kk) {
    const int t = kk / g.n_parts, part = kk - t * g.n_parts;
    int tile = t;
    if (g.n_sched) {
        // Uniform select over the list (a dynamic index into the by-value
        // kernel argument would copy it to scratch memory).
#pragma unroll
        for (int i = 0; i < kMaxSched; ++i)
            if (i == t) tile = g.sched[i];
    }
    return {tile, part, tile * g.n_parts + part};
}

__device__ __forceinline__ int wave_id_uniform() {
    return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
}

// Static sweep of a streaming kernel: block j takes chunks j, j+B, ...;
// body(first_slot_row, r1) handles the kUs row slots first + u*kWaves*R.
template <int S, typename Body>
__device__ __forceinline__ void sweep_static(const Geom& g, int tile, int part, int j, Body body) {
    constexpr int R = 64 / S;
    int r0, r1;
    part_range(g, tile, part, r0, r1);
    const int off = wave_id_uniform() * R + (threadIdx.x & 63) / S;
    const int step = g.B * g.chunk_rows;
    for (int c0 = r0 + j * g.chunk_rows; c0 < r1; c0 += step) body(c0 + off, r1);
}

// Row of slot u of a static chunk, clamped into [.., r1).
template <int S>
__device__ __forceinline__ int slot_row(int first, int u, int r1, bool& ok) {
    constexpr int R = 64 / S;
    const int row = first + u * kWaves * R;
    ok = row < r1;
    return ok ? row : r1 - 1;
}

// Next queue position for this wavefront (one atomic per wavefront).
__device__ __forceinline__ int grab(int32_t* ctr) {
    int v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(ctr, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

// Sweep of a gather kernel, body(row) per valid row. Queue mode: each
// wavefront takes grab*kUg*R consecutive rows at a time from the item's
// queue (one atomic per grab). Static mode: block j takes chunks j, j+B, ...
template <int S, typename Body>
__device__ __forceinline__ void sweep_gather(const Geom& g, int tile, int part, int j, int32_t* ctr,
                                             Body body) {
    constexpr int R = 64 / S;
    int r0, r1;
    part_range(g, tile, part, r0, r1);
    if (r1 <= r0) return;
    const int rs = (threadIdx.x & 63) / S;
    if (g.queue) {
        const int per = g.grab * kUg * R;
        const int n = (r1 - r0 + per - 1) / per;
        int c = grab(ctr);
        while (c < n) {
            const int cn = grab(ctr);
            const int base = r0 + c * per + rs;
            for (int m = 0; m < g.grab; ++m) {
#pragma unroll
                for (int u = 0; u < kUg; ++u) {
                    const int row = base + (m * kUg + u) * R;
                    if (row < r1) body(row);
                }
            }
            c = cn;
        }
    } else {
        const int off = wave_id_uniform() * R + rs;
        const int step = g.B * g.chunk_rows;
        for (int c0 = r0 + j * g.chunk_rows; c0 < r1; c0 += step) {
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                const int row = c0 + off + u * kWaves * R;
                if (row < r1) body(row);
            }
        }
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

// One item of q = A p with sigma partial sums (p^H q or p^T q) per lane.
template <typename T, int S, bool HERM>
__device__ __forceinline__ void spmv_item(const Geom& g, int tile, int part, int j, int32_t* ctr, bool act,
                                          size_t tb, const LaneCoef<T>& lc,
                                          const int32_t* __restrict__ row_ptr,
                                          const int32_t* __restrict__ col,
                                          const T* __restrict__ K0, const V4<T>* __restrict__ aux,
                                          const V2<T>* __restrict__ p, V2<T>* __restrict__ q,
                                          double (&acc)[2]) {
    sweep_gather<S>(g, tile, part, j, ctr, [&](int row) {
        if (!act) return;
        const int kb = row_ptr[row], ke = row_ptr[row + 1];
        const T cm = lc.cr(row);
        T yr = 0, yi = 0;
        for (int k0 = kb; k0 < ke; k0 += kRowPad) {
            int jj[kRowPad];
            V2<T> xv[kRowPad];
#pragma unroll
            for (int u = 0; u < kRowPad; ++u) jj[u] = col[k0 + u];
#pragma unroll
            for (int u = 0; u < kRowPad; ++u) xv[u] = p[tb + static_cast<size_t>(jj[u]) * S];
#pragma unroll
            for (int u = 0; u < kRowPad; ++u) {
                const V4<T> a = aux[k0 + u];
                const T ar = K0[k0 + u] + cm * a.x;
                const T ai = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
                yr += ar * xv[u].x - ai * xv[u].y;
                yi += ar * xv[u].y + ai * xv[u].x;
            }
        }
        const size_t idx = tb + static_cast<size_t>(row) * S;
        if (g.nt) store_nt(q + idx, mk2<T>(yr, yi));
        else q[idx] = mk2<T>(yr, yi);
        dot_acc<HERM, T>(acc[0], acc[1], p[idx], mk2<T>(yr, yi));
    });
}

// Accumulate y += (ar + i ai) x with explicit fused multiply-adds.
template <typename T>
__device__ __forceinline__ void cmac(T& yr, T& yi, T ar, T ai, V2<T> x) {
    yr = fma(ar, x.x, yr);
    yr = fma(-ai, x.y, yr);
    yi = fma(ar, x.y, yi);
    yi = fma(ai, x.x, yi);
}

// Gathers from one 64-wide tile go through a buffer resource covering the
// tile: the row offset j * 64 * sizeof(V2) is wavefront-uniform (a scalar
// register) and the lane offset is the same vector register for every
// gather, so a gather costs no vector address arithmetic. Offsets outside
// the resource read as zero.
constexpr int kBufWord3 = 0x00020000;  // raw 32-bit data format (gfx9 family)

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const V2<T>* pt, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<V2<T>*>(pt), 0, static_cast<int>(bytes),
                                             kBufWord3);
}

template <typename T>
__device__ __forceinline__ V2<T> tile_row(__amdgpu_buffer_rsrc_t rs, int j, uint32_t lane_bytes) {
    const uint32_t off = static_cast<uint32_t>(j) * static_cast<uint32_t>(64 * sizeof(V2<T>));
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(V2<T>, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_bytes, off, 0));
    } else {
        return __builtin_bit_cast(V2<T>, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_bytes, off, 0));
    }
}

// Rows of one 64-system tile of a vector read through a buffer resource:
// row j of the tile starts at the wavefront-uniform offset j * stride and
// the lane's element sits lane_bytes further.
struct TileRows {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t lane_bytes;
    uint32_t stride;
};

template <typename V>
__device__ __forceinline__ TileRows tile_rows(const V* base, uint32_t n_rows, uint32_t stride,
                                              uint32_t lane_bytes) {
    TileRows t;
    t.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<V*>(base), 0,
                                             static_cast<int>(n_rows * stride), kBufWord3);
    t.lane_bytes = lane_bytes;
    t.stride = stride;
    return t;
}

template <typename V>
__device__ __forceinline__ V load_row(const TileRows& t, int j) {
    const uint32_t off = static_cast<uint32_t>(j) * t.stride;
    if constexpr (sizeof(V) == 16)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(t.rs, t.lane_bytes, off, 0));
    else
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(t.rs, t.lane_bytes, off, 0));
}

// Rows whose padded length is 16 entries (every interior row of a Kuhn
// mesh): G rows of one wavefront at once, all 16 * G gathers issued before
// the first use. Returns the rows' results in yr/yi.
template <typename T, int G>
__device__ __forceinline__ void spmv16_rows(const int32_t* __restrict__ col,
                                            const T* __restrict__ K0,
                                            const V4<T>* __restrict__ aux,
                                            __amdgpu_buffer_rsrc_t pt, uint32_t lane_bytes,
                                            const int (&kb)[G], const T (&cm)[G],
                                            const LaneCoef<T>& lc, T (&yr)[G], T (&yi)[G]) {
    V2<T> xv[G][16];
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        int jj[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) jj[u] = col[kb[gi] + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) xv[gi][u] = tile_row<T>(pt, jj[u], lane_bytes);
    }
#pragma unroll
    for (int gi = 0; gi < G; ++gi) {
        T r = 0, i = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const V4<T> a = aux[kb[gi] + u];
            const T ar = fma(cm[gi], a.x, K0[kb[gi] + u]);
            const T ai = fma(lc.d2, a.w, fma(lc.d1, a.z, lc.d0 * a.y));
            cmac<T>(r, i, ar, ai, xv[gi][u]);
        }
        yr[gi] = r;
        yi[gi] = i;
    }
}

// One row of any padded length, 8 entries at a time.
template <typename T>
__device__ __forceinline__ void spmv8_row(const int32_t* __restrict__ col,
                                          const T* __restrict__ K0,
                                          const V4<T>* __restrict__ aux,
                                          __amdgpu_buffer_rsrc_t pt, uint32_t lane_bytes,
                                          int kb, int ke, T cm, const LaneCoef<T>& lc, T& yr,
                                          T& yi) {
    yr = 0;
    yi = 0;
    for (int k0 = kb; k0 < ke; k0 += kRowPad) {
        int jj[kRowPad];
        V2<T> xv[kRowPad];
#pragma unroll
        for (int u = 0; u < kRowPad; ++u) jj[u] = col[k0 + u];
#pragma unroll
        for (int u = 0; u < kRowPad; ++u) xv[u] = tile_row<T>(pt, jj[u], lane_bytes);
#pragma unroll
        for (int u = 0; u < kRowPad; ++u) {
            const V4<T> a = aux[k0 + u];
            const T ar = fma(cm, a.x, K0[k0 + u]);
            const T ai = fma(lc.d2, a.w, fma(lc.d1, a.z, lc.d0 * a.y));
            cmac<T>(yr, yi, ar, ai, xv[u]);
        }
    }
}

// SpMV item for 64-system tiles with static chunks: the kUs row slots of a
// wavefront are taken G at a time (G = 2 in FP32, 1 in FP64 for registers).
template <typename T, bool HERM>
__device__ __forceinline__ void spmv_item64(const Geom& g, int part, int j, int tile,
                                            const LaneCoef<T>& lc,
                                            const int32_t* __restrict__ row_ptr,
                                            const int32_t* __restrict__ col,
                                            const T* __restrict__ K0,
                                            const V4<T>* __restrict__ aux,
                                            const V2<T>* __restrict__ p, V2<T>* __restrict__ q,
                                            double (&acc)[2]) {
    constexpr int G = sizeof(T) == 4 ? 2 : 1;
    const int r0 = part * g.part_rows;
    const int r1 = min(g.n_rows, r0 + g.part_rows);
    const int lane = threadIdx.x & 63;
    const uint32_t lane_bytes = static_cast<uint32_t>(lane) * sizeof(V2<T>);
    const size_t tbase = static_cast<size_t>(tile) * g.n_rows * 64;
    const V2<T>* pt = p + tbase;
    V2<T>* qt = q + tbase;
    const __amdgpu_buffer_rsrc_t rs =
        tile_rsrc<T>(pt, static_cast<uint32_t>(g.n_rows) * 64u * sizeof(V2<T>));
    const int off = wave_id_uniform();
    const int step = g.B * g.chunk_rows;
    for (int c0 = r0 + j * g.chunk_rows; c0 < r1; c0 += step) {
#pragma unroll
        for (int u0 = 0; u0 < kUs; u0 += G) {
            int row[G], kb[G], ke[G];
            bool all16 = true, any = false;
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
                row[gi] = c0 + off + (u0 + gi) * kWaves;
                const bool ok = row[gi] < r1;
                any |= ok;
                if (!ok) row[gi] = r1 - 1;  // clamped duplicate, result not stored
                kb[gi] = row_ptr[row[gi]];
                ke[gi] = row_ptr[row[gi] + 1];
                all16 &= (ke[gi] - kb[gi] == 16);
            }
            if (!any) break;
            T yr[G], yi[G], cm[G];
#pragma unroll
            for (int gi = 0; gi < G; ++gi) cm[gi] = lc.cr(row[gi]);
            if (all16) {
                spmv16_rows<T, G>(col, K0, aux, rs, lane_bytes, kb, cm, lc, yr, yi);
            } else {
#pragma unroll
                for (int gi = 0; gi < G; ++gi)
                    spmv8_row<T>(col, K0, aux, rs, lane_bytes, kb[gi], ke[gi], cm[gi], lc, yr[gi],
                                 yi[gi]);
            }
#pragma unroll
            for (int gi = 0; gi < G; ++gi) {
                if (c0 + off + (u0 + gi) * kWaves >= r1) continue;
                const size_t o = static_cast<size_t>(row[gi]) * 64 + lane;
                const V2<T> y = mk2<T>(yr[gi], yi[gi]);
                if (g.nt) store_nt(qt + o, y);
                else qt[o] = y;
                dot_acc<HERM, T>(acc[0], acc[1], pt[o], y);
            }
        }
    }
}

// q = A p and sigma = p^H q (or p^T q) per system.
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_spmv_dot(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ K0, const V4<T>* __restrict__ aux, const double4* __restrict__ gq,
    Coef lhs, const V2<T>* __restrict__ p, V2<T>* __restrict__ q, SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * S * 2];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        const LaneCoef<T> lc(gq[sys], lhs, g, sys);
        double acc[2] = {0.0, 0.0};
        if constexpr (S == 64) {
            if (!g.queue && g.tile_bytes_ok && !g.mtab) {
                if (act)
                    spmv_item64<T, HERM>(g, part, j, tile, lc, row_ptr, col, K0, aux, p, q, acc);
            } else {
                spmv_item<T, S, HERM>(g, tile, part, j, sc.ctr_spmv + item, act, tb, lc, row_ptr, col,
                                      K0, aux, p, q, acc);
            }
        } else {
            spmv_item<T, S, HERM>(g, tile, part, j, sc.ctr_spmv + item, act, tb, lc, row_ptr, col, K0,
                                  aux, p, q, acc);
        }
        reduce_store<S, 2>(g, sc, item, j, acc, lds);
    }
}

// LDS-staged SpMV for wide tiles (S >= 32). Per chunk of rows the block
// copies the chunk's matrix entries (column, K0, {M_D, V}) into LDS with one
// coalesced burst, then every wavefront works on G of its rows at once:
// column indices and values come from LDS (broadcast reads) and the G*kRowPad
// gathers of a batch are issued back to back. Rows with fewer batches than
// the longest row of the group repeat their last batch with a zero mask
// (branch-free). Chunks with more entries than fit fall back to reading the
// matrix from global memory row by row.
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_spmv_lds(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ K0, const V4<T>* __restrict__ aux, const double4* __restrict__ gq,
    Coef lhs, const V2<T>* __restrict__ p, V2<T>* __restrict__ q, SolverState s, Scratch sc) {
    constexpr int R = 64 / S;
    constexpr int CH = kUs * kWaves * R;
    constexpr int MAXE = CH * kLdsRowCap;
    constexpr int G = kSpmvRows;
    __shared__ int32_t s_col[MAXE];
    __shared__ T s_k0[MAXE];
    __shared__ V4<T> s_aux[MAXE];
    __shared__ int32_t s_rp[CH + 1];
    __shared__ double lds[kWaves * S * 2];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        const LaneCoef<T> lc(gq[sys], lhs, g, sys);
        double acc[2] = {0.0, 0.0};
        const int r0 = part * g.part_rows;
        const int r1 = min(g.n_rows, r0 + g.part_rows);
        const int lane_off = wave_id_uniform() * R + (threadIdx.x & 63) / S;
        for (int c0 = r0 + j * CH; c0 < r1; c0 += g.B * CH) {
            const int c1 = min(r1, c0 + CH);
            const int e0 = row_ptr[c0];
            const int ne = row_ptr[c1] - e0;
            const bool staged = ne <= MAXE;
            if (staged) {
                for (int e = threadIdx.x; e < ne; e += kBlock) {
                    s_col[e] = col[e0 + e];
                    s_k0[e] = K0[e0 + e];
                    s_aux[e] = aux[e0 + e];
                }
                for (int i = threadIdx.x; i <= c1 - c0; i += kBlock) s_rp[i] = row_ptr[c0 + i] - e0;
            }
            __syncthreads();
            if (act && staged) {
#pragma unroll
                for (int m = 0; m < kUs / G; ++m) {
                    int rw[G], kb[G], nb[G];
                    bool ok[G];
                    int nbmax = 1;
#pragma unroll
                    for (int gg = 0; gg < G; ++gg) {
                        const int row = c0 + lane_off + (m * G + gg) * kWaves * R;
                        ok[gg] = row < c1;
                        rw[gg] = ok[gg] ? row : c1 - 1;
                        kb[gg] = s_rp[rw[gg] - c0];
                        nb[gg] = (s_rp[rw[gg] - c0 + 1] - kb[gg]) / kRowPad;
                        nbmax = max(nbmax, nb[gg]);
                    }
                    T yr[G], yi[G];
#pragma unroll
                    for (int gg = 0; gg < G; ++gg) yr[gg] = yi[gg] = T(0);
                    for (int b = 0; b < nbmax; ++b) {
                        int jj[G][kRowPad];
                        V2<T> xv[G][kRowPad];
#pragma unroll
                        for (int gg = 0; gg < G; ++gg) {
                            const int base = kb[gg] + kRowPad * min(b, nb[gg] - 1);
#pragma unroll
                            for (int u = 0; u < kRowPad; ++u) jj[gg][u] = s_col[base + u];
                        }
#pragma unroll
                        for (int gg = 0; gg < G; ++gg) {
#pragma unroll
                            for (int u = 0; u < kRowPad; ++u)
                                xv[gg][u] = p[tb + static_cast<size_t>(jj[gg][u]) * S];
                        }
#pragma unroll
                        for (int gg = 0; gg < G; ++gg) {
                            const int base = kb[gg] + kRowPad * min(b, nb[gg] - 1);
                            const T mk = b < nb[gg] ? T(1) : T(0);
                            const T cm = lc.cr(rw[gg]);
#pragma unroll
                            for (int u = 0; u < kRowPad; ++u) {
                                const V4<T> a = s_aux[base + u];
                                const T ar = mk * (s_k0[base + u] + cm * a.x);
                                const T ai = mk * (lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w);
                                yr[gg] += ar * xv[gg][u].x - ai * xv[gg][u].y;
                                yi[gg] += ar * xv[gg][u].y + ai * xv[gg][u].x;
                            }
                        }
                    }
#pragma unroll
                    for (int gg = 0; gg < G; ++gg) {
                        if (!ok[gg]) continue;
                        const size_t idx = tb + static_cast<size_t>(rw[gg]) * S;
                        if (g.nt) store_nt(q + idx, mk2<T>(yr[gg], yi[gg]));
                        else q[idx] = mk2<T>(yr[gg], yi[gg]);
                        dot_acc<HERM, T>(acc[0], acc[1], p[idx], mk2<T>(yr[gg], yi[gg]));
                    }
                }
            } else if (act) {
                for (int u = 0; u < kUs; ++u) {
                    const int row = c0 + lane_off + u * kWaves * R;
                    if (row >= c1) continue;
                    T yr = 0, yi = 0;
                    const T cm = lc.cr(row);
                    for (int k = row_ptr[row]; k < row_ptr[row + 1]; ++k) {
                        const V4<T> a = aux[k];
                        const T ar = K0[k] + cm * a.x;
                        const T ai = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
                        const V2<T> xv = p[tb + static_cast<size_t>(col[k]) * S];
                        yr += ar * xv.x - ai * xv.y;
                        yi += ar * xv.y + ai * xv.x;
                    }
                    const size_t idx = tb + static_cast<size_t>(row) * S;
                    q[idx] = mk2<T>(yr, yi);
                    dot_acc<HERM, T>(acc[0], acc[1], p[idx], mk2<T>(yr, yi));
                }
            }
            __syncthreads();
        }
        reduce_store<S, 2>(g, sc, item, j, acc, lds);
    }
}

// One item of x += alpha p (WITH_X), r -= alpha q, z = D^-1 r with partial
// sums rho' = r^H z (or r^T z) and ||r||^2.
template <typename T, int S, bool HERM, bool WITH_X = true>
__device__ __forceinline__ void update_item(const Geom& g, int tile, int part, int j, size_t tb,
                                            const LaneCoef<T>& lc, T ar, T ai,
                                            const T* __restrict__ dK0,
                                            const V4<T>* __restrict__ daux, V2<T>* __restrict__ x,
                                            V2<T>* __restrict__ r, const V2<T>* __restrict__ p,
                                            const V2<T>* __restrict__ q, double (&acc)[3]) {
    sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
        int row[kUs];
        bool ok[kUs];
        V2<T> pv[kUs], qv[kUs], xv[kUs], rv[kUs];
#pragma unroll
        for (int u = 0; u < kUs; ++u) {
            row[u] = slot_row<S>(first, u, r1, ok[u]);
            const size_t idx = tb + static_cast<size_t>(row[u]) * S;
            if (WITH_X) {
                pv[u] = p[idx];
                xv[u] = x[idx];
            }
            qv[u] = q[idx];
            rv[u] = r[idx];
        }
#pragma unroll
        for (int u = 0; u < kUs; ++u) {
            if (!ok[u]) continue;
            const size_t idx = tb + static_cast<size_t>(row[u]) * S;
            if (WITH_X) {
                xv[u].x += ar * pv[u].x - ai * pv[u].y;
                xv[u].y += ar * pv[u].y + ai * pv[u].x;
                x[idx] = xv[u];
            }
            rv[u].x -= ar * qv[u].x - ai * qv[u].y;
            rv[u].y -= ar * qv[u].y + ai * qv[u].x;
            r[idx] = rv[u];
            T dr, di;
            diag_at(dK0, daux, row[u], lc, dr, di);
            dot_acc<HERM, T>(acc[0], acc[1], rv[u], cdivT<T>(rv[u], dr, di));
            acc[2] += double(rv[u].x) * rv[u].x + double(rv[u].y) * rv[u].y;
        }
    });
}

// r -= alpha q, z = D^-1 r; rho' = r^H z (or r^T z), ||r||^2. (The matching
// x += alpha p is done by the direction update of the same iteration, which
// reads p anyway.)
template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_update(
    Geom g, const T* __restrict__ dK0, const V4<T>* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, V2<T>* __restrict__ x, V2<T>* __restrict__ r,
    const V2<T>* __restrict__ p, const V2<T>* __restrict__ q, SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * S * 3];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        const LaneCoef<T> lc(gq[sys], lhs, g, sys);
        const double2 al = act ? s.alpha[sys] : make_double2(0.0, 0.0);
        double acc[3] = {0.0, 0.0, 0.0};
        if (act)
            update_item<T, S, HERM, false>(g, tile, part, j, tb, lc, static_cast<T>(al.x),
                                           static_cast<T>(al.y), dK0, daux, x, r, p, q, acc);
        reduce_store<S, 3>(g, sc, item, j, acc, lds);
    }
}

// One item of x += alpha p (do_x) and p = D^-1 r + beta p (do_p), per lane.
template <typename T, int S>
__device__ __forceinline__ void pupdate_item(const Geom& g, int tile, int part, int j, size_t tb,
                                             const LaneCoef<T>& lc, T br, T bi, bool do_p,
                                             T ar, T ai, bool do_x,
                                             const T* __restrict__ dK0,
                                             const V4<T>* __restrict__ daux,
                                             const V2<T>* __restrict__ r, V2<T>* __restrict__ p,
                                             V2<T>* __restrict__ x) {
    sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
        int row[kUs];
        bool ok[kUs];
        V2<T> rv[kUs], pv[kUs], xv[kUs];
#pragma unroll
        for (int u = 0; u < kUs; ++u) {
            row[u] = slot_row<S>(first, u, r1, ok[u]);
            const size_t idx = tb + static_cast<size_t>(row[u]) * S;
            pv[u] = p[idx];
            if (do_p) rv[u] = r[idx];
            if (do_x) xv[u] = x[idx];
        }
#pragma unroll
        for (int u = 0; u < kUs; ++u) {
            if (!ok[u]) continue;
            const size_t idx = tb + static_cast<size_t>(row[u]) * S;
            if (do_x)
                x[idx] = mk2<T>(xv[u].x + ar * pv[u].x - ai * pv[u].y,
                                xv[u].y + ar * pv[u].y + ai * pv[u].x);
            if (do_p) {
                T dr, di;
                diag_at(dK0, daux, row[u], lc, dr, di);
                const V2<T> z = cdivT<T>(rv[u], dr, di);
                p[idx] = mk2<T>(z.x + br * pv[u].x - bi * pv[u].y,
                                z.y + br * pv[u].y + bi * pv[u].x);
            }
        }
    });
}

// End of Krylov iteration k: x += alpha p for every system that took part in
// iteration k (its count equals k, including systems that stopped in it),
// then p = D^-1 r + beta p for the systems still active.
template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_pupdate(Geom g, const T* __restrict__ dK0,
                                                    const V4<T>* __restrict__ daux,
                                                    const double4* __restrict__ gq, Coef lhs,
                                                    const V2<T>* __restrict__ r,
                                                    V2<T>* __restrict__ p, V2<T>* __restrict__ x,
                                                    int32_t k_iter, SolverState s) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool real = sys < s.n_sys;
        const bool do_p = real && s.active[sys];
        const bool do_x = real && s.iters[sys] == k_iter;
        if (!(do_p || do_x)) continue;
        const LaneCoef<T> lc(gq[sys], lhs, g, sys);
        const double2 be = do_p ? s.beta[sys] : make_double2(0.0, 0.0);
        const double2 al = s.alpha[sys];
        pupdate_item<T, S>(g, tile, part, j, tb, lc, static_cast<T>(be.x), static_cast<T>(be.y), do_p,
                           static_cast<T>(al.x), static_cast<T>(al.y), do_x, dK0, daux, r, p, x);
    }
}

// ------------------------------ polynomial preconditioner in flexible CG
//
// Chebyshev acceleration of Jacobi on the interval [a, b] of D^-1 A (Saad,
// Iterative Methods for Sparse Linear Systems, Sec. 12.3), m terms from
// y = 0, one launch per term:
//   theta = (b + a)/2, delta = (b - a)/2, sigma = theta/delta, rho_0 = 1/sigma
//   term 0:  d = D^-1 r / theta,  y = d
//   term j:  rho_j = 1 / (2 sigma - rho_{j-1}),
//            d = rho_j rho_{j-1} d + (2 rho_j / delta) D^-1 (r - A y),  y += d
// Neighbouring rows gather y, so a term reads y from one buffer and writes
// y + d to the other; d is updated in place. The last term also forms the
// flexible-CG dot products r^H z and q^H z (z = the new y).

__device__ __forceinline__ void cheb_coef(double2 ab, int j, double& c1, double& c2) {
    const double th = 0.5 * (ab.y + ab.x), de = 0.5 * (ab.y - ab.x);
    if (j == 0) {
        c1 = 0.0;
        c2 = 1.0 / th;
        return;
    }
    const double sg = th / de;
    double rho = 1.0 / sg, prev = rho;
    for (int i = 1; i <= j; ++i) {
        prev = rho;
        rho = 1.0 / (2.0 * sg - prev);
    }
    c1 = rho * prev;
    c2 = 2.0 * rho / de;
}

template <int S, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void k_cheb(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ K0, const double4* __restrict__ aux,
    const double* __restrict__ dK0, const double4* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, const double2* __restrict__ ab, int32_t term,
    const double2* __restrict__ r, const double2* __restrict__ q,
    const double2* __restrict__ y_in, double2* __restrict__ y_out, double2* __restrict__ d,
    SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * S * 4];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        const LaneCoef<double> lc(gq[sys], lhs, g, sys);
        double c1 = 0.0, c2 = 0.0;
        if (act) cheb_coef(ab[sys], term, c1, c2);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        sweep_gather<S>(g, tile, part, j, nullptr, [&](int row) {
            if (!act) return;
            double yr = 0.0, yi = 0.0;
            if (!FIRST) {  // (A y)_row
                const int kb = row_ptr[row], ke = row_ptr[row + 1];
                const double cm = lc.cr(row);
                for (int k0 = kb; k0 < ke; k0 += kRowPad) {
                    int jj[kRowPad];
                    double2 xv[kRowPad];
#pragma unroll
                    for (int u = 0; u < kRowPad; ++u) jj[u] = col[k0 + u];
#pragma unroll
                    for (int u = 0; u < kRowPad; ++u)
                        xv[u] = y_in[tb + static_cast<size_t>(jj[u]) * S];
#pragma unroll
                    for (int u = 0; u < kRowPad; ++u) {
                        const double4 a = aux[k0 + u];
                        const double ar = K0[k0 + u] + cm * a.x;
                        const double ai = lc.d0 * a.y + lc.d1 * a.z + lc.d2 * a.w;
                        yr += ar * xv[u].x - ai * xv[u].y;
                        yi += ar * xv[u].y + ai * xv[u].x;
                    }
                }
            }
            const size_t idx = tb + static_cast<size_t>(row) * S;
            const double2 rv = r[idx];
            double dr, di;
            diag_at(dK0, daux, row, lc, dr, di);
            const double2 w = cdivT<double>(make_double2(rv.x - yr, rv.y - yi), dr, di);
            double2 dn = make_double2(c2 * w.x, c2 * w.y);
            double2 yn = dn;
            if (!FIRST) {
                const double2 dv = d[idx], yv = y_in[idx];
                dn.x = fma(c1, dv.x, dn.x);
                dn.y = fma(c1, dv.y, dn.y);
                yn = make_double2(yv.x + dn.x, yv.y + dn.y);
            }
            if (!LAST) d[idx] = dn;
            y_out[idx] = yn;
            if (LAST) {
                dot_acc<true, double>(acc[0], acc[1], rv, yn);
                dot_acc<true, double>(acc[2], acc[3], q[idx], yn);
            }
        });
        if (LAST) reduce_store<S, 4>(g, sc, item, j, acc, lds);
    }
}

// x += alpha p (systems that took part in iteration k_iter), p = z + beta p
// (systems still active), z read from a vector.
template <int S>
__global__ __launch_bounds__(kBlock) void k_pupdate_z(Geom g, const double2* __restrict__ z,
                                                      double2* __restrict__ p,
                                                      double2* __restrict__ x, int32_t k_iter,
                                                      SolverState s) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool real = sys < s.n_sys;
        const bool do_p = real && s.active[sys];
        const bool do_x = real && k_iter >= 0 && s.iters[sys] == k_iter;
        if (!(do_p || do_x)) continue;
        const double2 be = do_p ? s.beta[sys] : make_double2(0.0, 0.0);
        const double2 al = do_x ? s.alpha[sys] : make_double2(0.0, 0.0);
        sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                bool ok;
                const int row = slot_row<S>(first, u, r1, ok);
                if (!ok) continue;
                const size_t idx = tb + static_cast<size_t>(row) * S;
                const double2 pv = p[idx];
                if (do_x) {
                    const double2 xv = x[idx];
                    x[idx] = make_double2(xv.x + al.x * pv.x - al.y * pv.y,
                                          xv.y + al.x * pv.y + al.y * pv.x);
                }
                if (do_p) {
                    const double2 zv = z[idx];
                    p[idx] = make_double2(zv.x + be.x * pv.x - be.y * pv.y,
                                          zv.y + be.x * pv.y + be.y * pv.x);
                }
            }
        });
    }
}

// Inputs of the interval network for system sys at one step (zero past 7).
__device__ __forceinline__ void pc_features(const double4 gg, const PcScalars ps, float* x) {
    const double gf = fabs(gg.x * ps.F);
    const double k = ps.theta * ps.dt;
    const double qn = sqrt(gg.y * gg.y + gg.z * gg.z + gg.w * gg.w);
    const double iq = qn > 0.0 ? 1.0 / qn : 0.0;
    x[0] = static_cast<float>(log(k * ps.d_max / (ps.h * ps.h)));
    x[1] = static_cast<float>(log1p(k * ps.d_max * gf * gf));
    x[2] = static_cast<float>(log1p(k * ps.d_max * gf / ps.h));
    x[3] = static_cast<float>(log1p(k * ps.kappa / ps.h));
    x[4] = static_cast<float>(fabs(gg.y) * iq);
    x[5] = static_cast<float>(fabs(gg.z) * iq);
    x[6] = static_cast<float>(fabs(gg.w) * iq);
#pragma unroll
    for (int i = 7; i < 16; ++i) x[i] = 0.0f;
}

__global__ void k_pc_features(int32_t ld, const double4* __restrict__ gq, PcScalars ps,
                              float* __restrict__ X) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= ld) return;
    float f[16];
    pc_features(gq[sys], ps, f);
#pragma unroll
    for (int i = 0; i < 16; ++i) X[static_cast<size_t>(sys) * 16 + i] = f[i];
}

__global__ void k_pc_interval(int32_t n_sys, int32_t ld, const float* __restrict__ Y, double a,
                              double b, double2* __restrict__ ab) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= ld) return;
    double lo = a, hi = b;
    if (Y && sys < n_sys) {
        const double y0 = Y[2 * sys], y1 = Y[2 * sys + 1];
        lo = kPcARef;
        hi = kPcBRef;
        if (isfinite(y0) && isfinite(y1)) {
            const double ta = kPcARef * exp(fmin(20.0, fmax(-20.0, y0)));
            const double tb = kPcBRef * exp(fmin(20.0, fmax(-20.0, y1)));
            if (ta * 1.001 < tb) {
                lo = ta;
                hi = tb;
            }
        }
    }
    ab[sys] = make_double2(lo, hi);
}

// Eigenvalues of the Lanczos tridiagonal of a PCG run below x (Sturm count):
// diagonal 1/alpha_0, 1/alpha_k + beta_{k-1}/alpha_{k-1}; squared
// off-diagonal beta_{k-1}/alpha_{k-1}^2.
__device__ int sturm_below(const double2* __restrict__ h, int n, double x) {
    int cnt = 0;
    double qv = 1.0;
    for (int k = 0; k < n; ++k) {
        const double al = h[k].x;
        double dk = 1.0 / al;
        double e2 = 0.0;
        if (k > 0) {
            const double ap = h[k - 1].x, bp = h[k - 1].y;
            dk += bp / ap;
            e2 = bp / (ap * ap);
        }
        qv = dk - x - (k > 0 ? e2 / qv : 0.0);
        if (qv == 0.0) qv = -1e-300;
        if (qv < 0.0) ++cnt;
    }
    return cnt;
}

// One block: systems in order, a block-wide scan of the valid ones gives
// each sample its slot; *count advances by the number written.
__global__ __launch_bounds__(1024) void k_pc_record(int32_t n_sys, const double4* __restrict__ gq,
                                                    PcScalars ps, SolverState s,
                                                    float* __restrict__ X, float* __restrict__ T,
                                                    int64_t* __restrict__ count, int64_t cap) {
    __shared__ int scan[1024];
    __shared__ int64_t base;
    if (threadIdx.x == 0) base = *count;
    __syncthreads();
    for (int c0 = 0; c0 < n_sys; c0 += 1024) {
        const int sys = c0 + static_cast<int>(threadIdx.x);
        bool ok = false;
        double lo = 0.0, hi = 0.0;
        if (sys < n_sys) {
            const int n = s.iters[sys];
            const double2* h = s.ab_hist + static_cast<size_t>(sys) * kRitzMax;
            ok = s.flags[sys] == 0 && n >= 2 && n <= kRitzMax;
            double glo = 1e300, ghi = -1e300;
            for (int k = 0; ok && k < n; ++k) {
                const double al = h[k].x;
                const double bp = k > 0 ? h[k - 1].y : 0.0;
                ok = isfinite(al) && al > 0.0 && isfinite(bp) && bp >= 0.0;
                if (!ok) break;
                // Gershgorin bracket of the tridiagonal
                const double ap = k > 0 ? h[k - 1].x : 1.0;
                const double dk = 1.0 / al + (k > 0 ? bp / ap : 0.0);
                const double el = k > 0 ? sqrt(bp) / ap : 0.0;
                const double er = k + 1 < n ? sqrt(fmax(0.0, h[k].y)) / al : 0.0;
                glo = fmin(glo, dk - el - er);
                ghi = fmax(ghi, dk + el + er);
            }
            if (ok) {
                // smallest: the x with one eigenvalue below; largest: n - 1 below
                double a0 = glo, b0 = ghi;
                for (int it = 0; it < 100; ++it) {
                    const double m = 0.5 * (a0 + b0);
                    if (sturm_below(h, n, m) >= 1) b0 = m; else a0 = m;
                }
                lo = 0.5 * (a0 + b0);
                a0 = glo;
                b0 = ghi;
                for (int it = 0; it < 100; ++it) {
                    const double m = 0.5 * (a0 + b0);
                    if (sturm_below(h, n, m) >= n) b0 = m; else a0 = m;
                }
                hi = 0.5 * (a0 + b0);
                ok = lo > 0.0 && hi >= lo && isfinite(hi);
            }
        }
        scan[threadIdx.x] = ok ? 1 : 0;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int v = threadIdx.x >= static_cast<unsigned>(off) ? scan[threadIdx.x - off] : 0;
            __syncthreads();
            scan[threadIdx.x] += v;
            __syncthreads();
        }
        const int64_t pos = base + scan[threadIdx.x] - 1;
        if (ok && pos < cap) {
            float f[16];
            pc_features(gq[sys], ps, f);
#pragma unroll
            for (int i = 0; i < 16; ++i) X[pos * 16 + i] = f[i];
            T[pos * 2] = static_cast<float>(log(lo / kPcARef));
            T[pos * 2 + 1] = static_cast<float>(log(kPcMargin * hi / kPcBRef));
        }
        __syncthreads();
        if (threadIdx.x == 0) base = base + scan[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base < cap ? base : cap;
}

// ------------------------------------------- paired lanes (FP32, 128 systems)
//
// The FP32 inner solves of wide batches use tiles of 128 systems with two
// systems per lane: systems 2l and 2l + 1 of a tile are the two complex
// halves of the float4 that lane l loads, so a row of a tile is one 1 KiB
// wavefront access of 16-byte lanes. This halves the vector-memory
// instructions per system of the 64-wide layout; those instructions, not
// HBM bandwidth, bound the SpMV gathers. Vector element (row, system s) of
// the paired layout is at ((s / 128) * n_rows + row) * 128 + s % 128
// (complex units); the matrix stays wavefront-uniform.

__device__ __forceinline__ size_t pair_tile(const Geom& g, int tile) {
    return static_cast<size_t>(tile) * g.n_rows * 64;  // lane-element units (float4 or uint2)
}

// Search directions of the paired layout may be stored in BF16 (Geom::dir16):
// a lane's four values (two systems' complex numbers) in 8 bytes, rounded to
// nearest even. The Krylov recurrences use the stored (rounded) direction
// everywhere -- the SpMV's q = A p, x += alpha p, the next p = z + beta p --
// so the residual recurrence stays consistent; only the directions' mutual
// conjugacy is perturbed (BF16 keeps FP32's exponent range: no scaling).
template <bool B16> struct DirOf;
template <> struct DirOf<false> { using type = float4; };
template <> struct DirOf<true> { using type = uint2; };

__device__ __forceinline__ uint32_t bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float4 dir_load(const float4* p, size_t o) { return p[o]; }
__device__ __forceinline__ float4 dir_load(const uint2* p, size_t o) {
    const uint2 w = p[o];
    return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xFFFF0000u),
                       __uint_as_float(w.y << 16), __uint_as_float(w.y & 0xFFFF0000u));
}
__device__ __forceinline__ void dir_store(float4* p, size_t o, float4 v) { p[o] = v; }
__device__ __forceinline__ void dir_store(uint2* p, size_t o, float4 v) {
    p[o] = make_uint2(bf16_bits(v.x) | (bf16_bits(v.y) << 16),
                      bf16_bits(v.z) | (bf16_bits(v.w) << 16));
}

template <int K>
__device__ __forceinline__ void reduce_store_pair(const Geom& g, Scratch sc, int item, int j,
                                                  double (&v)[2][K], double* lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int k = 0; k < K; ++k) lds[(wave * kPairS + 2 * lane + q) * K + k] = v[q][k];
    __syncthreads();
    if (threadIdx.x < kPairS) {
        double* dst =
            sc.partial + ((static_cast<size_t>(item) * g.B + j) * kPairS + threadIdx.x) * 4;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += lds[(w * kPairS + threadIdx.x) * K + k];
            dst[k] = t;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ float2 lo2(float4 v) { return make_float2(v.x, v.y); }
__device__ __forceinline__ float2 hi2(float4 v) { return make_float2(v.z, v.w); }
__device__ __forceinline__ float4 cat4(float2 a, float2 b) { return make_float4(a.x, a.y, b.x, b.y); }

// NB entries of a row from k0 for both systems of the lane.
template <int NB, bool B16>
__device__ __forceinline__ void pair_block(const int32_t* __restrict__ col,
                                           const float* __restrict__ K0,
                                           const float4* __restrict__ aux,
                                           __amdgpu_buffer_rsrc_t rs, uint32_t lane_bytes, int k0,
                                           const LaneCoef<float>& c0, const LaneCoef<float>& c1,
                                           float cm0, float cm1, float& yr0, float& yi0,
                                           float& yr1, float& yi1) {
    float4 xv[NB];
    if constexpr (B16) {
        uint2 w[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const uint32_t off = static_cast<uint32_t>(col[k0 + u]) * (kPairS * 4u);
            w[u] = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_bytes, off, 0));
        }
#pragma unroll
        for (int u = 0; u < NB; ++u)
            xv[u] = make_float4(__uint_as_float(w[u].x << 16), __uint_as_float(w[u].x & 0xFFFF0000u),
                                __uint_as_float(w[u].y << 16), __uint_as_float(w[u].y & 0xFFFF0000u));
    } else {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const uint32_t off = static_cast<uint32_t>(col[k0 + u]) * (kPairS * 8u);
            xv[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_bytes, off, 0));
        }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const float4 a = aux[k0 + u];
        const float k = K0[k0 + u];
        const float ar0 = fma(cm0, a.x, k), ai0 = fma(c0.d2, a.w, fma(c0.d1, a.z, c0.d0 * a.y));
        const float ar1 = fma(cm1, a.x, k), ai1 = fma(c1.d2, a.w, fma(c1.d1, a.z, c1.d0 * a.y));
        cmac<float>(yr0, yi0, ar0, ai0, lo2(xv[u]));
        cmac<float>(yr1, yi1, ar1, ai1, hi2(xv[u]));
    }
}

// The 16 BF16 direction gathers of a 16-entry row, and the row's products
// from them (split so that two rows' gathers can be in flight together).
__device__ __forceinline__ void gather16_b16(const int32_t* __restrict__ col,
                                             __amdgpu_buffer_rsrc_t rs, uint32_t lane_bytes,
                                             int k0, uint2 (&w)[16]) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const uint32_t off = static_cast<uint32_t>(col[k0 + u]) * (kPairS * 4u);
        w[u] = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, lane_bytes, off, 0));
    }
}
__device__ __forceinline__ void fma16_b16(const float* __restrict__ K0,
                                          const float4* __restrict__ aux, int k0,
                                          const LaneCoef<float>& c0, const LaneCoef<float>& c1,
                                          float cm0, float cm1, const uint2 (&w)[16], float& yr0,
                                          float& yi0, float& yr1, float& yi1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const float4 a = aux[k0 + u];
        const float k = K0[k0 + u];
        const float2 x0 = make_float2(__uint_as_float(w[u].x << 16), __uint_as_float(w[u].x & 0xFFFF0000u));
        const float2 x1 = make_float2(__uint_as_float(w[u].y << 16), __uint_as_float(w[u].y & 0xFFFF0000u));
        const float ar0 = fma(cm0, a.x, k), ai0 = fma(c0.d2, a.w, fma(c0.d1, a.z, c0.d0 * a.y));
        const float ar1 = fma(cm1, a.x, k), ai1 = fma(c1.d2, a.w, fma(c1.d1, a.z, c1.d0 * a.y));
        cmac<float>(yr0, yi0, ar0, ai0, x0);
        cmac<float>(yr1, yi1, ar1, ai1, x1);
    }
}

// q = A p and sigma = p^H q (or p^T q) for the paired layout. With R2 = 2 (BF16
// directions) a wavefront takes its rows two at a time: when both have 16
// entries their 32 gathers are issued before either row's products, so two
// rows' dependent chains (row pointer, column indices, gathers) overlap.
template <bool HERM, bool B16, int R2 = 0>
__global__ __launch_bounds__(kBlock) void k_spmv_pair(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const float* __restrict__ K0, const float4* __restrict__ aux, const double4* __restrict__ gq,
    Coef lhs, const typename DirOf<B16>::type* __restrict__ p, float4* __restrict__ q, SolverState s,
    Scratch sc) {
    using DT = typename DirOf<B16>::type;
    __shared__ double lds[kWaves * kPairS * 2];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int lane = threadIdx.x & 63;
    const uint32_t lane_bytes = static_cast<uint32_t>(lane) * static_cast<uint32_t>(sizeof(DT));
    const int off = wave_id_uniform();
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int s0 = tile * kPairS + 2 * lane;
        const bool a0 = s0 < s.n_sys && s.active[s0];
        const bool a1 = s0 + 1 < s.n_sys && s.active[s0 + 1];
        const bool la = a0 || a1;
        if (!__syncthreads_or(la)) continue;
        const LaneCoef<float> c0(gq[s0], lhs, g, s0), c1(gq[s0 + 1], lhs, g, s0 + 1);
        double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        const DT* pt = p + pair_tile(g, tile);
        float4* qt = q + pair_tile(g, tile);
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<DT*>(pt), 0,
            static_cast<int>(static_cast<uint32_t>(g.n_rows) * (64u * sizeof(DT))), kBufWord3);
        const int r0 = part * g.part_rows;
        const int r1 = min(g.n_rows, r0 + g.part_rows);
        const int step = g.B * g.chunk_rows;
        // q row out, and its sigma terms from the lane's own direction row
        auto finish = [&](int row, float yr0, float yi0, float yr1, float yi1) {
            const size_t o = static_cast<size_t>(row) * 64 + lane;
            const float4 y = make_float4(yr0, yi0, yr1, yi1);
            if (g.nt) store_nt(qt + o, y);
            else qt[o] = y;
            const float4 pv = dir_load(pt, o);
            dot_acc<HERM, float>(acc[0][0], acc[0][1], lo2(pv), lo2(y));
            dot_acc<HERM, float>(acc[1][0], acc[1][1], hi2(pv), hi2(y));
        };
        auto one_row = [&](int row, int kb, int ke) {
            const float cm0 = c0.cr(row), cm1 = c1.cr(row);
            float yr0 = 0.f, yi0 = 0.f, yr1 = 0.f, yi1 = 0.f;
            if (ke - kb == 16) {
                pair_block<16, B16>(col, K0, aux, rs, lane_bytes, kb, c0, c1, cm0, cm1, yr0,
                                    yi0, yr1, yi1);
            } else {
                for (int k0 = kb; k0 < ke; k0 += kRowPad)
                    pair_block<kRowPad, B16>(col, K0, aux, rs, lane_bytes, k0, c0, c1, cm0, cm1,
                                             yr0, yi0, yr1, yi1);
            }
            finish(row, yr0, yi0, yr1, yi1);
        };
        for (int c0r = r0 + j * g.chunk_rows; c0r < r1; c0r += step) {
            if constexpr (B16 && R2 == 2) {
                static_assert(kUs % 2 == 0, "rows are taken in pairs");
#pragma unroll
                for (int u = 0; u < kUs; u += 2) {
                    const int ra = c0r + off + u * kWaves, rb = ra + kWaves;
                    if (ra >= r1) break;
                    if (!la) continue;
                    const bool hb = rb < r1;
                    const int kba = row_ptr[ra], kea = row_ptr[ra + 1];
                    const int kbb = hb ? row_ptr[rb] : 0, keb = hb ? row_ptr[rb + 1] : 0;
                    if (hb && kea - kba == 16 && keb - kbb == 16) {
                        uint2 wa[16], wb[16];
                        gather16_b16(col, rs, lane_bytes, kba, wa);
                        gather16_b16(col, rs, lane_bytes, kbb, wb);
                        float ya[4] = {0.f, 0.f, 0.f, 0.f}, yb[4] = {0.f, 0.f, 0.f, 0.f};
                        fma16_b16(K0, aux, kba, c0, c1, c0.cr(ra), c1.cr(ra), wa, ya[0], ya[1],
                                  ya[2], ya[3]);
                        fma16_b16(K0, aux, kbb, c0, c1, c0.cr(rb), c1.cr(rb), wb, yb[0], yb[1],
                                  yb[2], yb[3]);
                        finish(ra, ya[0], ya[1], ya[2], ya[3]);
                        finish(rb, yb[0], yb[1], yb[2], yb[3]);
                    } else {
                        one_row(ra, kba, kea);
                        if (hb) one_row(rb, kbb, keb);
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < kUs; ++u) {
                    const int row = c0r + off + u * kWaves;
                    if (row >= r1) break;
                    // Lanes whose two systems have both converged neither
                    // gather nor store: in a tile that is only partly active,
                    // the cache lines of its converged systems are not fetched.
                    if (!la) continue;
                    one_row(row, row_ptr[row], row_ptr[row + 1]);
                }
            }
        }
        reduce_store_pair<2>(g, sc, item, j, acc, lds);
    }
}

// r -= alpha q, z = D^-1 r; rho' and ||r||^2 partials (paired layout). A
// system that is not active keeps its r (alpha taken as 0).
template <bool HERM>
__global__ __launch_bounds__(kBlock) void k_update_pair(
    Geom g, const float* __restrict__ dK0, const float4* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, float4* __restrict__ r,
    const float4* __restrict__ q, SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * kPairS * 3];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int lane = threadIdx.x & 63;
    const int off = wave_id_uniform();
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int s0 = tile * kPairS + 2 * lane;
        const bool a0 = s0 < s.n_sys && s.active[s0];
        const bool a1 = s0 + 1 < s.n_sys && s.active[s0 + 1];
        if (!__syncthreads_or(a0 || a1)) continue;
        const LaneCoef<float> c0(gq[s0], lhs, g, s0), c1(gq[s0 + 1], lhs, g, s0 + 1);
        const double2 al0 = a0 ? s.alpha[s0] : make_double2(0.0, 0.0);
        const double2 al1 = a1 ? s.alpha[s0 + 1] : make_double2(0.0, 0.0);
        const float ar0 = static_cast<float>(al0.x), ai0 = static_cast<float>(al0.y);
        const float ar1 = static_cast<float>(al1.x), ai1 = static_cast<float>(al1.y);
        double acc[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        float4* rt = r + pair_tile(g, tile);
        const float4* qt = q + pair_tile(g, tile);
        const int r0 = part * g.part_rows;
        const int r1 = min(g.n_rows, r0 + g.part_rows);
        const int step = g.B * g.chunk_rows;
        if (a0 || a1) {
            for (int c0r = r0 + j * g.chunk_rows; c0r < r1; c0r += step) {
                int row[kUs];
                bool ok[kUs];
                float4 rv[kUs], qv[kUs];
#pragma unroll
                for (int u = 0; u < kUs; ++u) {
                    const int rr = c0r + off + u * kWaves;
                    ok[u] = rr < r1;
                    row[u] = ok[u] ? rr : r1 - 1;
                    const size_t o = static_cast<size_t>(row[u]) * 64 + lane;
                    rv[u] = rt[o];
                    qv[u] = qt[o];
                }
#pragma unroll
                for (int u = 0; u < kUs; ++u) {
                    if (!ok[u]) continue;
                    float2 x0 = lo2(rv[u]), x1 = hi2(rv[u]);
                    const float2 q0 = lo2(qv[u]), q1 = hi2(qv[u]);
                    x0 = make_float2(x0.x - (ar0 * q0.x - ai0 * q0.y), x0.y - (ar0 * q0.y + ai0 * q0.x));
                    x1 = make_float2(x1.x - (ar1 * q1.x - ai1 * q1.y), x1.y - (ar1 * q1.y + ai1 * q1.x));
                    rt[static_cast<size_t>(row[u]) * 64 + lane] = cat4(x0, x1);
                    float dr, di;
                    diag_at(dK0, daux, row[u], c0, dr, di);
                    dot_acc<HERM, float>(acc[0][0], acc[0][1], x0, cdivT<float>(x0, dr, di));
                    acc[0][2] += double(x0.x) * x0.x + double(x0.y) * x0.y;
                    diag_at(dK0, daux, row[u], c1, dr, di);
                    dot_acc<HERM, float>(acc[1][0], acc[1][1], x1, cdivT<float>(x1, dr, di));
                    acc[1][2] += double(x1.x) * x1.x + double(x1.y) * x1.y;
                }
            }
        }
        reduce_store_pair<3>(g, sc, item, j, acc, lds);
    }
}

// End of Krylov iteration k_iter in the paired layout: x += alpha p for the
// systems that took part in it, p = D^-1 r + beta p for those still active.
template <bool B16>
__global__ __launch_bounds__(kBlock) void k_pupdate_pair(
    Geom g, const float* __restrict__ dK0, const float4* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, const float4* __restrict__ r,
    typename DirOf<B16>::type* __restrict__ p, float4* __restrict__ x, int32_t k_iter,
    SolverState s) {
    using DT = typename DirOf<B16>::type;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int lane = threadIdx.x & 63;
    const int off = wave_id_uniform();
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int s0 = tile * kPairS + 2 * lane;
        const bool re0 = s0 < s.n_sys, re1 = s0 + 1 < s.n_sys;
        const bool dp0 = re0 && s.active[s0], dp1 = re1 && s.active[s0 + 1];
        const bool dx0 = re0 && s.iters[s0] == k_iter, dx1 = re1 && s.iters[s0 + 1] == k_iter;
        const bool do_p = dp0 || dp1, do_x = dx0 || dx1;
        if (!(do_p || do_x)) continue;
        const LaneCoef<float> c0(gq[s0], lhs, g, s0), c1(gq[s0 + 1], lhs, g, s0 + 1);
        const double2 b0 = dp0 ? s.beta[s0] : make_double2(0.0, 0.0);
        const double2 b1 = dp1 ? s.beta[s0 + 1] : make_double2(0.0, 0.0);
        const double2 al0 = dx0 ? s.alpha[s0] : make_double2(0.0, 0.0);
        const double2 al1 = dx1 ? s.alpha[s0 + 1] : make_double2(0.0, 0.0);
        const float br0 = static_cast<float>(b0.x), bi0 = static_cast<float>(b0.y);
        const float br1 = static_cast<float>(b1.x), bi1 = static_cast<float>(b1.y);
        const float xr0 = static_cast<float>(al0.x), xi0 = static_cast<float>(al0.y);
        const float xr1 = static_cast<float>(al1.x), xi1 = static_cast<float>(al1.y);
        const float4* rt = r + pair_tile(g, tile);
        DT* pt = p + pair_tile(g, tile);
        float4* xt = x + pair_tile(g, tile);
        const int r0 = part * g.part_rows;
        const int r1 = min(g.n_rows, r0 + g.part_rows);
        const int step = g.B * g.chunk_rows;
        for (int c0r = r0 + j * g.chunk_rows; c0r < r1; c0r += step) {
            int row[kUs];
            bool ok[kUs];
            float4 pv[kUs], rv[kUs], xv[kUs];
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                const int rr = c0r + off + u * kWaves;
                ok[u] = rr < r1;
                row[u] = ok[u] ? rr : r1 - 1;
                const size_t o = static_cast<size_t>(row[u]) * 64 + lane;
                pv[u] = dir_load(pt, o);
                if (do_p) rv[u] = rt[o];
                if (do_x) xv[u] = xt[o];
            }
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                if (!ok[u]) continue;
                const size_t o = static_cast<size_t>(row[u]) * 64 + lane;
                const float2 p0 = lo2(pv[u]), p1 = hi2(pv[u]);
                if (do_x) {
                    const float2 x0 = lo2(xv[u]), x1 = hi2(xv[u]);
                    xt[o] = cat4(make_float2(x0.x + xr0 * p0.x - xi0 * p0.y,
                                             x0.y + xr0 * p0.y + xi0 * p0.x),
                                 make_float2(x1.x + xr1 * p1.x - xi1 * p1.y,
                                             x1.y + xr1 * p1.y + xi1 * p1.x));
                }
                if (do_p) {
                    float dr, di;
                    float2 n0 = p0, n1 = p1;
                    if (dp0) {
                        diag_at(dK0, daux, row[u], c0, dr, di);
                        const float2 z = cdivT<float>(lo2(rv[u]), dr, di);
                        n0 = make_float2(z.x + br0 * p0.x - bi0 * p0.y, z.y + br0 * p0.y + bi0 * p0.x);
                    }
                    if (dp1) {
                        diag_at(dK0, daux, row[u], c1, dr, di);
                        const float2 z = cdivT<float>(hi2(rv[u]), dr, di);
                        n1 = make_float2(z.x + br1 * p1.x - bi1 * p1.y, z.y + br1 * p1.y + bi1 * p1.x);
                    }
                    dir_store(pt, o, cat4(n0, n1));
                }
            }
        }
    }
}

// Start of an FP32 inner solve in the paired layout: r = (float) r64 for
// outer-active systems (0 otherwise), dx = 0, p = z = D^-1 r; partials rho,
// ||r||^2, ||r64||^2. r64 is in the 64-wide FP64 layout (n64 rows per tile).
template <bool HERM, bool B16>
__global__ __launch_bounds__(kBlock) void k_inner_start_pair(
    Geom g, const float* __restrict__ dK0, const float4* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, const double2* __restrict__ r64,
    const int32_t* __restrict__ outer_active, float4* __restrict__ r, float4* __restrict__ dx,
    typename DirOf<B16>::type* __restrict__ p, SolverState s, Scratch sc) {
    using DT = typename DirOf<B16>::type;
    __shared__ double lds[kWaves * kPairS * 4];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    const int lane = threadIdx.x & 63;
    const int off = wave_id_uniform();
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int s0 = tile * kPairS + 2 * lane;
        const bool a0 = s0 < s.n_sys && outer_active[s0];
        const bool a1 = s0 + 1 < s.n_sys && outer_active[s0 + 1];
        const LaneCoef<float> c0(gq[s0], lhs, g, s0), c1(gq[s0 + 1], lhs, g, s0 + 1);
        // both systems of the lane sit next to each other in the 64-wide tile
        const size_t b64 = static_cast<size_t>(s0 / 64) * g.n_rows * 64 + (s0 % 64);
        double acc[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
        float4* rt = r + pair_tile(g, tile);
        float4* xt = dx + pair_tile(g, tile);
        DT* pt = p + pair_tile(g, tile);
        const int r0 = part * g.part_rows;
        const int r1 = min(g.n_rows, r0 + g.part_rows);
        const int step = g.B * g.chunk_rows;
        for (int c0r = r0 + j * g.chunk_rows; c0r < r1; c0r += step) {
            int row[kUs];
            bool ok[kUs];
            double2 v0[kUs], v1[kUs];
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                const int rr = c0r + off + u * kWaves;
                ok[u] = rr < r1;
                row[u] = ok[u] ? rr : r1 - 1;
                const size_t o = b64 + static_cast<size_t>(row[u]) * 64;
                v0[u] = a0 ? r64[o] : make_double2(0.0, 0.0);
                v1[u] = a1 ? r64[o + 1] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                if (!ok[u]) continue;
                const size_t o = static_cast<size_t>(row[u]) * 64 + lane;
                const float2 x0 = make_float2(static_cast<float>(v0[u].x), static_cast<float>(v0[u].y));
                const float2 x1 = make_float2(static_cast<float>(v1[u].x), static_cast<float>(v1[u].y));
                float dr, di;
                diag_at(dK0, daux, row[u], c0, dr, di);
                const float2 z0 = cdivT<float>(x0, dr, di);
                diag_at(dK0, daux, row[u], c1, dr, di);
                const float2 z1 = cdivT<float>(x1, dr, di);
                rt[o] = cat4(x0, x1);
                dir_store(pt, o, cat4(z0, z1));
                xt[o] = make_float4(0.f, 0.f, 0.f, 0.f);
                dot_acc<HERM, float>(acc[0][0], acc[0][1], x0, z0);
                dot_acc<HERM, float>(acc[1][0], acc[1][1], x1, z1);
                acc[0][2] += double(x0.x) * x0.x + double(x0.y) * x0.y;
                acc[1][2] += double(x1.x) * x1.x + double(x1.y) * x1.y;
                acc[0][3] += v0[u].x * v0[u].x + v0[u].y * v0[u].y;
                acc[1][3] += v1[u].x * v1[u].x + v1[u].y * v1[u].y;
            }
        }
        reduce_store_pair<4>(g, sc, item, j, acc, lds);
    }
}

// ------------------------------------------------------ persistent solver

constexpr int kMaxPersistSys = 64;
constexpr long kBarrierSpinLimit = 1L << 21;

// Two-level barrier: the blocks of XCD group x (blockIdx % 8 == x) count on
// their own counter (count[32 * (x + 1)], one cache line each), the last of
// each group counts on the global counter count[0], and the last group
// releases everyone by advancing the generation. Every wait is bounded: a
// wait that times out sets *err, and every block that sees *err set returns
// false, so the kernel always terminates.
__device__ __forceinline__ bool grid_sync(GridBarrier b) {
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        ok = 1;
        if (__hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
        } else {
            const uint32_t my =
                __hip_atomic_load(b.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            const uint32_t grp = blockIdx.x & 7;
            const uint32_t in_grp = (gridDim.x - grp + 7) / 8;
            uint32_t* gc = b.count + 32 * (grp + 1);
            bool released = false;
            if (atomicAdd(gc, 1u) == in_grp - 1) {
                __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // The reset must be visible before this group's arrival on the
                // global counter: a block released by the next generation may
                // arrive on gc right after that.
                __threadfence();
                const uint32_t groups = gridDim.x < 8 ? gridDim.x : 8;
                if (atomicAdd(b.count, 1u) == groups - 1) {
                    __hip_atomic_store(b.count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __threadfence();
                    atomicAdd(b.gen, 1u);
                    released = true;
                }
            }
            if (!released) {
                long spins = 0;
                while (__hip_atomic_load(b.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == my) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > kBarrierSpinLimit) {
                        atomicOr(b.err, 1);
                        ok = 0;
                        break;
                    }
                    if ((spins & 1023) == 0 &&
                        __hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        ok = 0;
                        break;
                    }
                }
            }
            __threadfence();
        }
    }
    __syncthreads();
    return ok != 0;
}

// Sum the partials of every system (ld <= 64) in a fixed order; thread t < ld
// receives the totals of system t. Every block computes the same values.
template <int S, int K>
__device__ __forceinline__ void sum_partials(const Geom& g, Scratch sc, double* red,
                                             double (&tot)[K]) {
    const int ld = g.ld;
    const int G = kBlock / ld;
    const int grp = threadIdx.x / ld, sy = threadIdx.x - grp * ld;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    if (grp < G) {
        const int tile = sy / S, sl = sy - tile * S;
        const int nb = g.n_parts * g.B;
        const double* base = sc.partial + static_cast<size_t>(tile) * nb * S * 4;
        for (int i = grp; i < nb; i += G) {
            const double* pp = base + (static_cast<size_t>(i) * S + sl) * 4;
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += pp[k];
        }
        if (grp < G) {
#pragma unroll
            for (int k = 0; k < K; ++k) red[(grp * ld + sy) * K + k] = acc[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < ld) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
            for (int gg = 0; gg < G; ++gg) t += red[(gg * ld + threadIdx.x) * K + k];
            tot[k] = t;
        }
    }
    __syncthreads();
}

template <typename T, int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_krylov_persistent(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ K0, const V4<T>* __restrict__ aux, const T* __restrict__ dK0,
    const V4<T>* __restrict__ daux, const double4* __restrict__ gq, Coef lhs,
    V2<T>* __restrict__ x, V2<T>* __restrict__ r, V2<T>* __restrict__ p, V2<T>* __restrict__ q,
    SolverState s, Scratch sc, GridBarrier bar) {
    __shared__ double2 sh_rho[kMaxPersistSys], sh_alpha[kMaxPersistSys], sh_beta[kMaxPersistSys];
    __shared__ double sh_bb[kMaxPersistSys], sh_rr[kMaxPersistSys];
    __shared__ int sh_act[kMaxPersistSys], sh_it[kMaxPersistSys], sh_flag[kMaxPersistSys];
    __shared__ int sh_any;
    __shared__ double lds[kWaves * S * 3];
    __shared__ double red[kBlock * 3];
    const int ld = g.ld;
    // Separate partial buffers for the two reductions of an iteration: a block
    // may start writing phase-B partials while another still reads phase A's.
    Scratch scA = sc, scB = sc;
    scB.partial = sc.partial + static_cast<size_t>(g.n_items) * g.B * S * 4;
    for (int t = threadIdx.x; t < ld; t += kBlock) {
        const bool real = t < s.n_sys;
        sh_rho[t] = real ? s.rho[t] : make_double2(0.0, 0.0);
        sh_bb[t] = real ? s.bb[t] : 0.0;
        sh_rr[t] = real ? s.rr[t] : 0.0;
        sh_act[t] = real ? s.active[t] : 0;
        sh_it[t] = 0;
        sh_flag[t] = 0;
        sh_alpha[t] = make_double2(0.0, 0.0);
        sh_beta[t] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int it = 0; it <= s.max_iter; ++it) {
        // Phase A: q = A p, sigma partials.
        for (int kk = xcd; kk < g.n_items; kk += 8) {
            const ItemRef ir = item_ref(g, kk);
            const int tile = ir.tile, part = ir.part, item = ir.item;
            const int sys = tile * S + (threadIdx.x & 63) % S;
            const size_t tb = vbase(g, tile, S, sys);
            const bool act = sh_act[sys] != 0;
            if (!__syncthreads_or(act)) continue;
            const LaneCoef<T> lc(gq[sys], lhs, g, sys);
            double acc[2] = {0.0, 0.0};
            spmv_item<T, S, HERM>(g, tile, part, j, nullptr, act, tb, lc, row_ptr, col, K0, aux, p, q,
                                  acc);
            reduce_store<S, 2>(g, scA, item, j, acc, lds);
        }
        if (!grid_sync(bar)) break;
        {
            double tot[2];
            sum_partials<S, 2>(g, scA, red, tot);
            if (threadIdx.x < ld && sh_act[threadIdx.x])
                sh_alpha[threadIdx.x] = cdiv(sh_rho[threadIdx.x], make_double2(tot[0], tot[1]));
            __syncthreads();
        }
        // Phase B: x, r update; rho', ||r||^2 partials.
        for (int kk = xcd; kk < g.n_items; kk += 8) {
            const ItemRef ir = item_ref(g, kk);
            const int tile = ir.tile, part = ir.part, item = ir.item;
            const int sys = tile * S + (threadIdx.x & 63) % S;
            const size_t tb = vbase(g, tile, S, sys);
            const bool act = sh_act[sys] != 0;
            if (!__syncthreads_or(act)) continue;
            const LaneCoef<T> lc(gq[sys], lhs, g, sys);
            const double2 al = sh_alpha[sys];
            double acc[3] = {0.0, 0.0, 0.0};
            if (act)
                update_item<T, S, HERM>(g, tile, part, j, tb, lc, static_cast<T>(al.x),
                                        static_cast<T>(al.y), dK0, daux, x, r, p, q, acc);
            reduce_store<S, 3>(g, scB, item, j, acc, lds);
        }
        if (!grid_sync(bar)) break;
        {
            double tot[3];
            sum_partials<S, 3>(g, scB, red, tot);
            if (threadIdx.x == 0) sh_any = 0;
            __syncthreads();
            if (threadIdx.x < ld && sh_act[threadIdx.x]) {
                const int sy = threadIdx.x;
                const double2 rho_new = make_double2(tot[0], tot[1]);
                const double rr = tot[2];
                sh_rr[sy] = rr;
                sh_it[sy] += 1;
                bool stop = false;
                if (!isfinite(rr) || !isfinite(rho_new.x) || !isfinite(rho_new.y)) {
                    sh_flag[sy] |= 2;
                    stop = true;
                } else if (rr <= s.rtol2 * sh_bb[sy]) {
                    stop = true;
                } else if (sh_it[sy] >= s.max_iter) {
                    sh_flag[sy] |= 1;
                    stop = true;
                }
                if (stop) {
                    sh_act[sy] = 0;
                } else {
                    sh_beta[sy] = cdiv(rho_new, sh_rho[sy]);
                    sh_rho[sy] = rho_new;
                    sh_any = 1;
                }
            }
            __syncthreads();
        }
        if (!sh_any) break;
        // Phase C: p = z + beta p.
        for (int kk = xcd; kk < g.n_items; kk += 8) {
            const ItemRef ir = item_ref(g, kk);
            const int tile = ir.tile, part = ir.part, item = ir.item;
            const int sys = tile * S + (threadIdx.x & 63) % S;
            const size_t tb = vbase(g, tile, S, sys);
            if (!sh_act[sys]) continue;
            const LaneCoef<T> lc(gq[sys], lhs, g, sys);
            const double2 be = sh_beta[sys];
            pupdate_item<T, S>(g, tile, part, j, tb, lc, static_cast<T>(be.x), static_cast<T>(be.y),
                               true, T(0), T(0), false, dK0, daux, r, p, x);
        }
        if (!grid_sync(bar)) break;
    }
    if (blockIdx.x == 0) {
        for (int t = threadIdx.x; t < s.n_sys; t += kBlock) {
            s.rho[t] = sh_rho[t];
            s.rr[t] = sh_rr[t];
            s.active[t] = 0;
            s.iters[t] = sh_it[t];
            s.iters_total[t] += sh_it[t];
            s.flags[t] |= sh_flag[t];
        }
        for (int t = threadIdx.x; t < g.n_tiles; t += kBlock) s.n_active[t] = 0;
    }
}

// Start of a time step (or of an outer refinement pass): b = Right(u_prev),
// x0 = guess, r = b - A x0, p = z = D^-1 r; partials rho, ||r||^2, ||b||^2.
// At a step start (GM 0/1/2) b is also stored to bvec when it is given; a
// refinement pass (GM 3) reads b from bvec instead of recomputing it. GM 4
// is the cheaper refinement pass: r -= A dx (FP64 operator, only the FP32
// correction dx is gathered) and x_out = x + dx; x_out may be x itself,
// since this mode reads x only at the row it writes.
template <typename T, int S, bool HERM, int GM>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(GM == 4 ? 5 : 1))) void k_init(
    Geom g, const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const T* __restrict__ K0, const T* __restrict__ Kr, const V4<T>* __restrict__ aux,
    const T* __restrict__ dK0, const V4<T>* __restrict__ daux, const double4* __restrict__ gq,
    Coef lhs, Coef rhs, const V2<T>* __restrict__ u_prev, const V2<T>* __restrict__ u_prev2,
    V2<T>* x, V2<T>* __restrict__ r, V2<T>* __restrict__ p,
    const float2* __restrict__ dx, V2<T>* x_out, V2<T>* __restrict__ bvec,
    SolverState s, Scratch sc, const int32_t* __restrict__ wmap, const V2<T>* __restrict__ wb) {
    constexpr bool kRhs = GM < 3;  // b formed from u_prev in this launch
    __shared__ double lds[kWaves * S * 4];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys;
        const double4 gg = gq[sys];
        const LaneCoef<T> ll(gg, lhs, g, sys), lr(gg, rhs, g, sys);
        // dx of the refinement passes may be stored in the paired layout.
        const size_t tbx = g.dx_pair ? static_cast<size_t>(sys / kPairS) * g.n_rows * kPairS +
                                           static_cast<size_t>(sys % kPairS)
                                     : tb;
        const size_t sx = g.dx_pair ? kPairS : S;
        // 64-system tiles with static chunks: every row is wavefront-uniform,
        // so the gathers go through buffer resources with uniform row offsets.
        const bool fast = S == 64 && !g.queue && g.tile_bytes_ok && !g.mtab;
        TileRows tu{}, tu2{}, tx{}, tdx{};
        if constexpr (S == 64) {
            if (fast) {
                const uint32_t lane = threadIdx.x & 63;
                const uint32_t nr = static_cast<uint32_t>(g.n_rows);
                const size_t off = static_cast<size_t>(tile) * g.n_rows * 64;
                constexpr uint32_t kRow = 64 * sizeof(V2<T>);
                tu = tile_rows(u_prev + off, nr, kRow, lane * sizeof(V2<T>));
                if (GM == 1) tu2 = tile_rows(u_prev2 + off, nr, kRow, lane * sizeof(V2<T>));
                if (GM == 2 || GM == 3) tx = tile_rows<V2<T>>(x + off, nr, kRow, lane * sizeof(V2<T>));
                if (GM >= 3) {
                    if (g.dx_pair)
                        tdx = tile_rows(dx + static_cast<size_t>(tile / 2) * g.n_rows * kPairS, nr,
                                        kPairS * 8u, ((tile & 1) * 64u + lane) * 8u);
                    else
                        tdx = tile_rows(dx + off, nr, 64u * 8u, lane * 8u);
                }
            }
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        sweep_gather<S>(g, tile, part, j, sc.ctr_init + item, [&](int row) {
            if (!act) return;
            const int kb = row_ptr[row], ke = row_ptr[row + 1];
            const T cml = ll.cr(row), cmr = lr.cr(row);
            T br = 0, bi = 0, axr = 0, axi = 0;
            V2<T> x0_own = mk2<T>(0, 0);
            // NB entries from k0: their column indices, then all their gathers,
            // then the products.
            auto block = [&](auto nb, int k0) {
                constexpr int kB = decltype(nb)::value;
                int jj[kB];
                V2<T> uj[kB], xj[kB];
                float2 dj[kB];  // GM 4: the FP32 correction, widened where it is used
#pragma unroll
                for (int u = 0; u < kB; ++u) jj[u] = col[k0 + u];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    if (fast) {
                        if (kRhs) uj[u] = load_row<V2<T>>(tu, jj[u]);
                        if (GM == 1) {
                            xj[u] = load_row<V2<T>>(tu2, jj[u]);
                        } else if (GM == 2) {
                            xj[u] = load_row<V2<T>>(tx, jj[u]);
                        } else if (GM == 3) {
                            const V2<T> xo = load_row<V2<T>>(tx, jj[u]);
                            const float2 d = load_row<float2>(tdx, jj[u]);
                            xj[u] = mk2<T>(xo.x + static_cast<T>(d.x), xo.y + static_cast<T>(d.y));
                        } else if (GM == 4) {
                            dj[u] = load_row<float2>(tdx, jj[u]);
                        }
                        continue;
                    }
                    const size_t jdx = tb + static_cast<size_t>(jj[u]) * S;
                    if (kRhs) uj[u] = u_prev[jdx];
                    if (GM == 1) {
                        const V2<T> u2 = u_prev2[jdx];
                        xj[u] = mk2<T>(u2.x, u2.y);
                    } else if (GM == 2) {
                        xj[u] = x[jdx];
                    } else if (GM == 3) {
                        const V2<T> xo = x[jdx];
                        const float2 d = dx[tbx + static_cast<size_t>(jj[u]) * sx];
                        xj[u] = mk2<T>(xo.x + static_cast<T>(d.x), xo.y + static_cast<T>(d.y));
                    } else if (GM == 4) {
                        dj[u] = dx[tbx + static_cast<size_t>(jj[u]) * sx];
                    }
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    const int k = k0 + u;
                    if (GM == 0) xj[u] = uj[u];
                    if (GM == 4) xj[u] = mk2<T>(static_cast<T>(dj[u].x), static_cast<T>(dj[u].y));
                    if (GM == 1) xj[u] = mk2<T>(T(2) * uj[u].x - xj[u].x, T(2) * uj[u].y - xj[u].y);
                    const V4<T> a = aux[k];
                    const T vl = ll.d0 * a.y + ll.d1 * a.z + ll.d2 * a.w;
                    const T al = K0[k] + cml * a.x;
                    if (jj[u] == row) x0_own = xj[u];
                    if (kRhs) {
                        const T vr = lr.d0 * a.y + lr.d1 * a.z + lr.d2 * a.w;
                        const T arr = Kr[k] + cmr * a.x;
                        br += arr * uj[u].x - vr * uj[u].y;
                        bi += arr * uj[u].y + vr * uj[u].x;
                    }
                    axr += al * xj[u].x - vl * xj[u].y;
                    axi += al * xj[u].y + vl * xj[u].x;
                }
            };
            constexpr int kB = S == 64 ? kRowPad : kRowPad / 2;
            bool whole = false;
            if constexpr (GM == 4 && S == 64) {
                // The cheap refinement pass gathers only the FP32 correction,
                // so a 16-entry row's 16 gathers fit in flight together.
                if (fast && ke - kb == 2 * kRowPad) {
                    block(std::integral_constant<int, 2 * kRowPad>{}, kb);
                    whole = true;
                }
            }
            if (!whole)
                for (int k0 = kb; k0 < ke; k0 += kB) block(std::integral_constant<int, kB>{}, k0);
            const size_t idx = tb + static_cast<size_t>(row) * S;
            if (kRhs && wmap) {
                // weak pseudo-periodic faces: the lagged partner term
                const int32_t sl = wmap[row];
                if (sl >= 0) {
                    const V2<T> e = wb[static_cast<size_t>(sl) * g.ld + sys];
                    br += e.x;
                    bi += e.y;
                }
            }
            if (GM == 3) {
                const V2<T> bv = bvec[idx];
                br = bv.x;
                bi = bv.y;
            } else if (kRhs && bvec) {
                bvec[idx] = mk2<T>(br, bi);
            }
            V2<T> rv;
            if (GM == 4) {
                const V2<T> r_old = r[idx];
                rv = mk2<T>(r_old.x - axr, r_old.y - axi);
            } else {
                rv = mk2<T>(br - axr, bi - axi);
            }
            r[idx] = rv;
            T dr, di;
            diag_at(dK0, daux, row, ll, dr, di);
            const V2<T> z = cdivT<T>(rv, dr, di);
            if (GM < 3 && p) p[idx] = z;
            dot_acc<HERM, T>(acc[0], acc[1], rv, z);
            acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
            if (GM != 4) acc[3] += double(br) * br + double(bi) * bi;
            // The guess of this row is stored where no other row reads it
            // during this launch: x itself when the gathers read u_prev
            // (GM 0/1), a second buffer when they read x (GM 3).
            if (GM == 0 || GM == 1) x[idx] = x0_own;
            if (GM == 3) x_out[idx] = x0_own;
            if (GM == 4) {
                const V2<T> xo = x[idx];
                x_out[idx] = mk2<T>(xo.x + x0_own.x, xo.y + x0_own.y);
            }
        });
        reduce_store<S, 4>(g, sc, item, j, acc, lds);
    }
}

// Start of the FP32 inner solve: r = (float) r64 for outer-active systems,
// dx = 0 everywhere, p = z = D^-1 r; partials rho, ||r||^2, ||r64||^2.
template <int S, bool HERM>
__global__ __launch_bounds__(kBlock) void k_inner_start(
    Geom g, const float* __restrict__ dK0, const float4* __restrict__ daux,
    const double4* __restrict__ gq, Coef lhs, const double2* __restrict__ r64,
    const int32_t* __restrict__ outer_active, float2* __restrict__ r, float2* __restrict__ dx,
    float2* __restrict__ p, SolverState s, Scratch sc) {
    __shared__ double lds[kWaves * S * 4];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && outer_active[sys];
        const LaneCoef<float> lc(gq[sys], lhs, g, sys);
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
            int row[kUs];
            bool ok[kUs];
            double2 rv64[kUs];
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                row[u] = slot_row<S>(first, u, r1, ok[u]);
                rv64[u] = act ? r64[tb + static_cast<size_t>(row[u]) * S]
                              : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                if (!ok[u]) continue;
                const size_t idx = tb + static_cast<size_t>(row[u]) * S;
                dx[idx] = make_float2(0.0f, 0.0f);
                const float2 rv = make_float2(static_cast<float>(rv64[u].x),
                                              static_cast<float>(rv64[u].y));
                float dr, di;
                diag_at(dK0, daux, row[u], lc, dr, di);
                const float2 z = cdivT<float>(rv, dr, di);
                r[idx] = rv;
                p[idx] = z;
                dot_acc<HERM, float>(acc[0], acc[1], rv, z);
                acc[2] += double(rv.x) * rv.x + double(rv.y) * rv.y;
                acc[3] += rv64[u].x * rv64[u].x + rv64[u].y * rv64[u].y;
            }
        });
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
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        double acc[2] = {0.0, 0.0};
        if (sys < n_sys) {
            sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
#pragma unroll
                for (int u = 0; u < kUs; ++u) {
                    bool ok;
                    const int row = slot_row<S>(first, u, r1, ok);
                    const V2<T> xv = x[tb + static_cast<size_t>(row) * S];
                    const double wv = ok ? w[row] : 0.0;
                    acc[0] += wv * double(xv.x);
                    acc[1] += wv * double(xv.y);
                }
            });
        }
        reduce_store<S, 2>(g, sc, item, j, acc, lds);
    }
}

// Phase-weighted signal partials. For a tetrahedron with vertices x_l (from
// the box centre) and P1 values u_l, the exact integral of u_h exp(-i k.x) is
//   6|e| sum_j u_j E_j,  E_j = exp[z_0, z_1, z_2, z_3, z_j],  z_l = -i k.x_l,
// the divided difference of exp with node z_j repeated (Hermite-Genocchi:
// the barycentric integral of exp(sum lambda_l z_l) is exp[z_0..z_3], and
// weighting by lambda_j is the derivative in z_j). With phi_l = k.x_l minus
// their mean, E_j = exp(-i mean) sum_m (-i)^m H_m^(j) / (m + 4)!, where
// H_m^(j) is the complete homogeneous polynomial of degree m in
// (phi_0..phi_3, phi_j) (real), built degree by degree. Terms are added
// until two in a row fall below 1e-18 of the sum (at most kPhaseTerms).
constexpr int kPhaseTerms = 160;

template <typename T, int S>
__global__ __launch_bounds__(kBlock) void k_signal_phase(Geom gt, int32_t n_rows,
                                                         TetView tv,
                                                         const double4* __restrict__ gq, double F,
                                                         const V2<T>* __restrict__ x,
                                                         int32_t n_sys, Scratch sc) {
    __shared__ double lds[kWaves * S * 2];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < gt.n_items; kk += 8) {
        const ItemRef ir = item_ref(gt, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = static_cast<size_t>(tile) * n_rows * S + (sys - tile * S);
        double acc[2] = {0.0, 0.0};
        if (sys < n_sys) {
            const double4 gg = gq[sys];
            const double kf = gg.x * F;
            const double kx = kf * gg.y, ky = kf * gg.z, kz = kf * gg.w;
            sweep_static<S>(gt, tile, part, j, [&](int first, int r1) {
                for (int u = 0; u < kUs; ++u) {
                    bool ok;
                    const int e = slot_row<S>(first, u, r1, ok);
                    if (!ok) continue;
                    const int4 dv = tv.dof[e], nv = tv.node[e];
                    const int nd[4] = {nv.x, nv.y, nv.z, nv.w};
                    const int dd[4] = {dv.x, dv.y, dv.z, dv.w};
                    double X[4][3], th[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
#pragma unroll
                        for (int a = 0; a < 3; ++a) X[l][a] = tv.xyz[3 * static_cast<size_t>(nd[l]) + a];
                        th[l] = kx * X[l][0] + ky * X[l][1] + kz * X[l][2];
                    }
                    double e1[3], e2[3], e3[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        e1[a] = X[1][a] - X[0][a];
                        e2[a] = X[2][a] - X[0][a];
                        e3[a] = X[3][a] - X[0][a];
                    }
                    const double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) -
                                       e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                                       e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
                    const double w6 = fabs(det);  // 6 |e|
                    const double tm = 0.25 * (th[0] + th[1] + th[2] + th[3]);
                    double ph[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) ph[l] = th[l] - tm;
                    double ur[4], ui[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        const V2<T> v = x[tb + static_cast<size_t>(dd[l]) * S];
                        ur[l] = static_cast<double>(v.x);
                        ui[l] = static_cast<double>(v.y);
                    }
                    // m = 0: every H is 1, 1/4! = 1/24.
                    double inv_f = 1.0 / 24.0;
                    double sr = (ur[0] + ur[1] + ur[2] + ur[3]) * inv_f;
                    double si = (ui[0] + ui[1] + ui[2] + ui[3]) * inv_f;
                    double a0 = 1.0, a1 = 1.0, a2 = 1.0, H = 1.0;
                    double Hj[4] = {1.0, 1.0, 1.0, 1.0};
                    int small = 0;
                    for (int m = 1; m <= kPhaseTerms; ++m) {
                        a0 = ph[0] * a0;
                        a1 = a0 + ph[1] * a1;
                        a2 = a1 + ph[2] * a2;
                        H = a2 + ph[3] * H;
                        double tr = 0.0, ti = 0.0;
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            Hj[l] = H + ph[l] * Hj[l];
                            tr += ur[l] * Hj[l];
                            ti += ui[l] * Hj[l];
                        }
                        inv_f /= (m + 4);
                        tr *= inv_f;
                        ti *= inv_f;
                        switch (m & 3) {  // times (-i)^m
                            case 0: sr += tr; si += ti; break;
                            case 1: sr += ti; si -= tr; break;
                            case 2: sr -= tr; si -= ti; break;
                            default: sr -= ti; si += tr; break;
                        }
                        const double mag = fabs(tr) + fabs(ti);
                        small = (mag <= 1e-18 * (fabs(sr) + fabs(si)) || mag == 0.0) ? small + 1 : 0;
                        if (small >= 2) break;
                    }
                    const double c = cos(tm), sn = sin(tm);  // times exp(-i tm)
                    acc[0] += w6 * (c * sr + sn * si);
                    acc[1] += w6 * (c * si - sn * sr);
                }
            });
        }
        reduce_store<S, 2>(gt, sc, item, j, acc, lds);
    }
}

// Add a tile's partials in a fixed order and update the per-system scalars.
// One block per tile; thread (grp, s) sums partials grp, grp+G, ... of
// system s, then the groups are combined in order. Resets the tile's queue
// counters in `zero_ctr` (items tile*n_parts .. +n_parts-1).
// One wide block per tile: kFinBlock / S thread groups add interleaved block
// partials, then the groups are combined in a fixed order.
constexpr int kFinBlock = 1024;

// First stage of a finalize: block (tile, group) adds group `group` of the
// tile's nb partials (contiguous, in order) and stores the sum at
// stage[tile][group]. Fixed order, so the result is deterministic. Group 0
// also clears the tile's chunk counters (zero_ctr) for the next launch.
constexpr int kStageBlock = 256;
template <int S>
__global__ __launch_bounds__(kStageBlock) void k_fin_stage(Geom g, Scratch sc, int32_t nb,
                                                           int32_t* zero_ctr) {
    int tile = static_cast<int>(blockIdx.x) / kFinGroups;
    const int grp = static_cast<int>(blockIdx.x) % kFinGroups;
    if (g.n_sched) {
        const int t = tile;
#pragma unroll
        for (int i = 0; i < kMaxSched; ++i)
            if (i == t) tile = g.sched[i];
    }
    if (zero_ctr && grp == 0 && static_cast<int>(threadIdx.x) < g.n_parts)
        zero_ctr[tile * g.n_parts + threadIdx.x] = 0;
    const int per = (nb + kFinGroups - 1) / kFinGroups;
    const int i0 = grp * per, i1 = min(nb, i0 + per);
    constexpr int W = S * 4;  // doubles per partial
    const double* base = sc.partial + static_cast<size_t>(tile) * nb * W;
    double* dst = sc.stage + (static_cast<size_t>(tile) * kFinGroups + grp) * W;
    for (int v = threadIdx.x; v < W; v += kStageBlock) {
        double acc = 0.0;
        int i = i0;
        for (; i + 3 < i1; i += 4) {
            const double a0 = base[static_cast<size_t>(i) * W + v];
            const double a1 = base[static_cast<size_t>(i + 1) * W + v];
            const double a2 = base[static_cast<size_t>(i + 2) * W + v];
            const double a3 = base[static_cast<size_t>(i + 3) * W + v];
            acc += a0;
            acc += a1;
            acc += a2;
            acc += a3;
        }
        for (; i < i1; ++i) acc += base[static_cast<size_t>(i) * W + v];
        dst[v] = acc;
    }
}

template <int S, int K, int MODE>
__global__ __launch_bounds__(kFinBlock) void k_finalize(Geom g, SolverState s, Scratch sc,
                                                        double2* __restrict__ out, int32_t n_sig,
                                                        int32_t* __restrict__ zero_ctr) {
    constexpr int G = kFinBlock / S;
    __shared__ double lds[kFinBlock * K];
    __shared__ int cnt;
    int tile = static_cast<int>(blockIdx.x);
    if (g.n_sched) {
        const int t = tile;
#pragma unroll
        for (int i = 0; i < kMaxSched; ++i)
            if (i == t) tile = g.sched[i];
    }
    const int grp = threadIdx.x / S, sl = threadIdx.x % S;
    const int sys = tile * S + sl;
    if (zero_ctr && threadIdx.x < g.n_parts) zero_ctr[tile * g.n_parts + threadIdx.x] = 0;
    constexpr bool kActiveOnly = MODE == FIN_ALPHA || MODE == FIN_BETA || MODE == FIN_CHECK ||
                                 MODE == FIN_FLEX0 || MODE == FIN_FLEX;
    if (kActiveOnly) {
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) return;
    }
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    const int nb = g.n_parts * g.B;
    const double* base = sc.partial + static_cast<size_t>(tile) * nb * S * 4;
    // Partials grp, grp + G, ... in that order; kU loads in flight per batch.
    constexpr int kU = 8;
    int i = grp;
    for (; i + (kU - 1) * G < nb; i += kU * G) {
        double v[kU][K];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const double* pp = base + (static_cast<size_t>(i + u * G) * S + sl) * 4;
#pragma unroll
            for (int k = 0; k < K; ++k) v[u][k] = pp[k];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] += v[u][k];
    }
    for (; i < nb; i += G) {
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
#pragma unroll 4
            for (int gg = 0; gg < G; ++gg) t += lds[(gg * S + sl) * K + k];
            tot[k] = t;
        }
        if (MODE == FIN_SIGNAL) {
            if (sys < n_sig) out[sys] = make_double2(tot[0], tot[1]);
        } else if (MODE == FIN_ALPHA) {
            if (sys < s.n_sys && s.active[sys]) {
                const double2 al = cdiv(s.rho[sys], make_double2(tot[0], tot[1]));
                s.alpha[sys] = al;
                if (s.ab_hist) {
                    const int it = s.iters[sys];
                    if (it < kRitzMax) s.ab_hist[static_cast<size_t>(sys) * kRitzMax + it].x = al.x;
                }
            }
        } else if (MODE == FIN_FLEX0 || MODE == FIN_FLEX) {
            if (sys < s.n_sys && s.active[sys]) {
                const double2 rho_new = make_double2(tot[0], tot[1]);
                const double2 qz = make_double2(tot[2], tot[3]);
                if (!isfinite(rho_new.x) || !isfinite(rho_new.y) || !isfinite(qz.x) ||
                    !isfinite(qz.y)) {
                    s.flags[sys] |= 2;
                    s.active[sys] = 0;
                } else {
                    double2 be = make_double2(0.0, 0.0);
                    if (MODE == FIN_FLEX) {  // -(q^H z) / sigma with sigma = rho / alpha
                        const double2 t = cdiv(cmul(qz, s.alpha[sys]), s.rho[sys]);
                        be = make_double2(-t.x, -t.y);
                    }
                    s.beta[sys] = be;
                    s.rho[sys] = rho_new;
                    atomicAdd(&cnt, 1);
                }
            }
        } else if (MODE == FIN_BETA || MODE == FIN_CHECK) {
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
                } else if (MODE == FIN_CHECK) {
                    atomicAdd(&cnt, 1);
                } else {
                    const double2 be = cdiv(rho_new, s.rho[sys]);
                    s.beta[sys] = be;
                    s.rho[sys] = rho_new;
                    if (s.ab_hist && it_now - 1 < kRitzMax)
                        s.ab_hist[static_cast<size_t>(sys) * kRitzMax + it_now - 1].y = be.x;
                    atomicAdd(&cnt, 1);
                }
            }
        } else {  // FIN_INIT, FIN_REFINE
            if (sys < s.n_sys) {
                const double rr = tot[2];
                const double bb =
                    MODE == FIN_REFINE
                        ? s.bb[sys]
                        : (s.floor_bb ? fmax(tot[3], s.floor_scale * s.floor_bb[sys]) : tot[3]);
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
    if ((MODE == FIN_BETA || MODE == FIN_INIT || MODE == FIN_REFINE || MODE == FIN_CHECK ||
         MODE == FIN_FLEX0 || MODE == FIN_FLEX) &&
        threadIdx.x == 0)
        s.n_active[tile] = cnt;
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
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const T c = static_cast<T>(cc[sys]);
        const double3 d3 = dd[sys];
        const T d0 = static_cast<T>(d3.x), d1 = static_cast<T>(d3.y), d2 = static_cast<T>(d3.z);
        sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
            for (int u = 0; u < kUs; ++u) {
                bool ok;
                const int row = slot_row<S>(first, u, r1, ok);
                if (!ok) continue;
                T yr = 0, yi = 0;
                for (int k = A.row_ptr[row]; k < A.row_ptr[row + 1]; ++k) {
                    const V4<T> a = A.aux[k];
                    const T ar = base[k] + c * a.x;
                    const T ai = d0 * a.y + d1 * a.z + d2 * a.w;
                    const V2<T> xv = x[tb + static_cast<size_t>(A.col[k]) * S];
                    yr += ar * xv.x - ai * xv.y;
                    yi += ar * xv.y + ai * xv.x;
                }
                y[tb + static_cast<size_t>(row) * S] = mk2<T>(yr, yi);
            }
        });
    }
}

// Partner term of the weak pseudo-periodic faces (see launch_weak_rhs):
// one thread per (slot, system), consecutive threads on consecutive systems
// so the u_prev reads of a column are contiguous. FP64 phases and sums.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_weak_rhs(WeakView w, int32_t n_rows, int32_t S,
                                                     int32_t ld, int32_t n_sys,
                                                     const double4* __restrict__ gq, double F,
                                                     double c, const V2<T>* __restrict__ u,
                                                     V2<T>* __restrict__ wb) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= static_cast<int64_t>(w.n_slots) * ld) return;
    const int32_t slot = static_cast<int32_t>(i / ld);
    const int32_t sys = static_cast<int32_t>(i - static_cast<int64_t>(slot) * ld);
    if (sys >= n_sys) {
        wb[i] = mk2<T>(T(0), T(0));
        return;
    }
    const double4 g = gq[sys];
    const double GF = g.x * F;
    double cs[3], sn[3];
    sincos(GF * g.y * w.L[0], &sn[0], &cs[0]);
    sincos(GF * g.z * w.L[1], &sn[1], &cs[1]);
    sincos(GF * g.w * w.L[2], &sn[2], &cs[2]);
    const int32_t tile = sys / S;
    const size_t base = static_cast<size_t>(tile) * n_rows * S + (sys - tile * S);
    double re = 0.0, im = 0.0;
    for (int32_t k = w.ptr[slot]; k < w.ptr[slot + 1]; ++k) {
        const int32_t cd = w.code[k];
        const int32_t a = cd < 3 ? cd : cd - 3;
        const double er = cs[a], ei = cd < 3 ? sn[a] : -sn[a];
        const V2<T> v = u[base + static_cast<size_t>(w.col[k]) * S];
        const double vr = static_cast<double>(v.x), vi = static_cast<double>(v.y);
        const double val = w.val[k];
        re += val * (er * vr - ei * vi);
        im += val * (er * vi + ei * vr);
    }
    wb[i] = mk2<T>(static_cast<T>(c * re), static_cast<T>(c * im));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_initial(int64_t n, int32_t n_rows, int32_t S,
                                                        int32_t n_sys,
                                                        const double* __restrict__ u0,
                                                        V2<T>* __restrict__ x) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t slab = i / S;  // tile * n_rows + row
    const int64_t tile = slab / n_rows;
    const int64_t row = slab - tile * n_rows;
    const int64_t sys = tile * S + (i - slab * S);
    x[i] = mk2<T>(sys < n_sys ? static_cast<T>(u0[row]) : T(0), T(0));
}

// x = sum_k c[k] u_k over all elements (polynomial extrapolation of the
// solution history, or any fixed linear combination of up to kMaxHist
// vectors). Four elements per thread per pass, all loads issued first.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_combine(int64_t n, ExtrapTerms<T> t,
                                                   V2<T>* __restrict__ x) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        V2<T> v[kMaxHist];
#pragma unroll
        for (int k = 0; k < kMaxHist; ++k)
            if (k < t.m) v[k] = t.u[k][i];
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxHist; ++k)
            if (k < t.m) {
                re = fma(t.c[k], static_cast<double>(v[k].x), re);
                im = fma(t.c[k], static_cast<double>(v[k].y), im);
            }
        x[i] = mk2<T>(static_cast<T>(re), static_cast<T>(im));
    }
}

__global__ void k_aniso_params(int32_t n_comp, int32_t ld, const double4* __restrict__ gq,
                               const double* __restrict__ t, double* __restrict__ acomp) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ld) return;
    const double4 g = gq[s];
    const double x = g.y, y = g.z, z = g.w;
    for (int k = 0; k < n_comp; ++k) {
        const double* d = t + 6 * k;
        acomp[static_cast<size_t>(k) * ld + s] = d[0] * x * x + d[1] * y * y + d[2] * z * z +
                                                 2.0 * (d[3] * x * y + d[4] * x * z + d[5] * y * z);
    }
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

// ------------------------------------------------------------ GMRES(m)
//
// Restarted GMRES with right Jacobi preconditioning (A D^-1 y = r0,
// x = x0 + D^-1 V y) for a batch of systems with per-system masks. The
// Krylov basis v_0..v_m lives in `V` (batch-layout vectors); the Hessenberg
// matrix, Givens rotations and the reduced right-hand side per system in
// GmresState (FP64). Orthogonalization is classical Gram-Schmidt applied
// twice (dot pass, subtract pass, again). Kernels of a cycle take a
// SolverState whose `active` is the per-system "still in this cycle" flag.

// v_j = w / hnorm, z = D^-1 v_j for the systems in the cycle.
template <int S>
__global__ __launch_bounds__(kBlock) void k_gm_scale(Geom g, const double* __restrict__ dK0,
                                                     const double4* __restrict__ daux,
                                                     const double4* __restrict__ gq, Coef lhs,
                                                     const double2* __restrict__ w,
                                                     double2* __restrict__ v,
                                                     double2* __restrict__ z, GmresState gm,
                                                     SolverState s) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!act) continue;
        const LaneCoef<double> lc(gq[sys], lhs, g, sys);
        const double inv = 1.0 / gm.hnorm[sys];
        sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
#pragma unroll
            for (int u = 0; u < kUs; ++u) {
                bool ok;
                const int row = slot_row<S>(first, u, r1, ok);
                if (!ok) continue;
                const size_t idx = tb + static_cast<size_t>(row) * S;
                const double2 wv = w[idx];
                const double2 vv = make_double2(wv.x * inv, wv.y * inv);
                v[idx] = vv;
                double dr, di;
                diag_at(dK0, daux, row, lc, dr, di);
                z[idx] = cdivT<double>(vv, dr, di);
            }
        });
    }
}

// Block partials of v_i^H w for i = i0 .. i0+nb-1 (nb <= kGmBatch) into value
// slots 2i, 2i+1 of gm.partial[(item * B + j) * S + lane][kGmVals].
constexpr int kGmBatch = 8;

template <int S>
__global__ __launch_bounds__(kBlock) void k_gm_dots(Geom g, const double2* __restrict__ w,
                                                    GmresBasis V, int i0, int nb, GmresState gm,
                                                    SolverState s) {
    __shared__ double lds[kWaves * S];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        double a[2 * kGmBatch];
#pragma unroll
        for (int c = 0; c < 2 * kGmBatch; ++c) a[c] = 0.0;
        if (act) {
            sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
                for (int u = 0; u < kUs; ++u) {
                    bool ok;
                    const int row = slot_row<S>(first, u, r1, ok);
                    if (!ok) continue;
                    const size_t idx = tb + static_cast<size_t>(row) * S;
                    const double2 wv = w[idx];
#pragma unroll
                    for (int t = 0; t < kGmBatch; ++t) {
                        if (t < nb) {
                            const double2 vv = V.base[static_cast<size_t>(i0 + t) * V.stride + idx];
                            a[2 * t] += vv.x * wv.x + vv.y * wv.y;
                            a[2 * t + 1] += vv.x * wv.y - vv.y * wv.x;
                        }
                    }
                }
            });
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        double* dst = gm.partial + ((static_cast<size_t>(item) * g.B + j) * S) * kGmVals;
#pragma unroll
        for (int c = 0; c < 2 * kGmBatch; ++c) {
            if (c >= 2 * nb) break;
            double t = a[c];
#pragma unroll
            for (int off = S; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
            if (lane < S) lds[wave * S + lane] = t;
            __syncthreads();
            if (threadIdx.x < S) {
                double u = 0.0;
#pragma unroll
                for (int ww = 0; ww < kWaves; ++ww) u += lds[ww * S + threadIdx.x];
                dst[static_cast<size_t>(threadIdx.x) * kGmVals + 2 * i0 + c] = u;
            }
            __syncthreads();
        }
    }
}

// Sum one tile's partials in a fixed order: hout[sys][c] for c < nval.
template <int S>
__global__ __launch_bounds__(kFinBlock) void k_gm_fin(Geom g, int nval, GmresState gm,
                                                      SolverState s) {
    constexpr int G = kFinBlock / S;
    __shared__ double lds[kFinBlock];
    const int tile = static_cast<int>(blockIdx.x);
    const int grp = threadIdx.x / S, sl = threadIdx.x % S;
    const int sys = tile * S + sl;
    const bool act = sys < s.n_sys && s.active[sys];
    if (!__syncthreads_or(act)) return;
    const int nb = g.n_parts * g.B;
    const double* base = gm.partial + static_cast<size_t>(tile) * nb * S * kGmVals;
    for (int c = 0; c < nval; ++c) {
        double acc = 0.0;
        for (int i = grp; i < nb; i += G)
            acc += base[(static_cast<size_t>(i) * S + sl) * kGmVals + c];
        lds[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x < S) {
            double t = 0.0;
            for (int gg = 0; gg < G; ++gg) t += lds[gg * S + sl];
            if (act) gm.hout[static_cast<size_t>(sys) * kGmVals + c] = t;
        }
        __syncthreads();
    }
}

// w -= sum_{i<nv} c_i v_i with c_i from hout (the last dot pass); block
// partials of ||w||^2 in value slot 0.
template <int S>
__global__ __launch_bounds__(kBlock) void k_gm_orth(Geom g, double2* __restrict__ w, GmresBasis V,
                                                    int nv, GmresState gm, SolverState s) {
    __shared__ double lds[kWaves * S];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        double a = 0.0;
        if (act) {
            const double* hs = gm.hout + static_cast<size_t>(sys) * kGmVals;
            sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
                for (int u = 0; u < kUs; ++u) {
                    bool ok;
                    const int row = slot_row<S>(first, u, r1, ok);
                    if (!ok) continue;
                    const size_t idx = tb + static_cast<size_t>(row) * S;
                    double2 wv = w[idx];
                    for (int i = 0; i < nv; ++i) {
                        const double cr = hs[2 * i], ci = hs[2 * i + 1];
                        const double2 vv = V.base[static_cast<size_t>(i) * V.stride + idx];
                        wv.x -= cr * vv.x - ci * vv.y;
                        wv.y -= cr * vv.y + ci * vv.x;
                    }
                    w[idx] = wv;
                    a += wv.x * wv.x + wv.y * wv.y;
                }
            });
        }
#pragma unroll
        for (int off = S; off < 64; off <<= 1) a += __shfl_xor(a, off, 64);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane < S) lds[wave * S + lane] = a;
        __syncthreads();
        if (threadIdx.x < S) {
            double t = 0.0;
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) t += lds[ww * S + threadIdx.x];
            gm.partial[((static_cast<size_t>(item) * g.B + j) * S + threadIdx.x) * kGmVals] = t;
        }
        __syncthreads();
    }
}

// Per system in the cycle: column `col` of H gets the dot pass's
// coefficients (pass 0 sets them, pass 1 adds the re-orthogonalization's).
__global__ void k_gm_addcol(int32_t n_sys, int nv, int col, int pass, GmresState gm) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= n_sys || !gm.cycle[sys]) return;
    const double* hs = gm.hout + static_cast<size_t>(sys) * kGmVals;
    double2* H = gm.H + static_cast<size_t>(sys) * (kGmMax + 1) * kGmMax;
    for (int i = 0; i < nv; ++i) {
        double2& h = H[i * kGmMax + col];
        const double2 c = make_double2(hs[2 * i], hs[2 * i + 1]);
        h = pass == 0 ? c : make_double2(h.x + c.x, h.y + c.y);
    }
}

// Per system in the cycle, with ||w||^2 in hout slot 0:
//  col < 0 (cycle start, w = r): beta = ||r||, g = (beta, 0, ...); a system
//    already within rtol leaves (active and cycle cleared);
//  col >= 0: h_{col+1,col} = ||w||, earlier rotations applied to column col,
//    new rotation, g updated; |g_{col+1}| is the residual norm. Convergence,
//    a non-finite value or max_iter ends the system's solve; the last column
//    (col + 1 = m) or a breakdown (||w|| = 0) ends only the cycle.
__global__ void k_gm_givens(int32_t n_sys, int col, int m, int use_rr, GmresState gm,
                            SolverState s) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= n_sys || !gm.cycle[sys]) return;
    const double nrm2 = use_rr ? s.rr[sys] : gm.hout[static_cast<size_t>(sys) * kGmVals];
    const double nrm = sqrt(fmax(nrm2, 0.0));
    double2* g = gm.g + static_cast<size_t>(sys) * (kGmMax + 1);
    gm.hnorm[sys] = nrm;
    if (col < 0) {
        g[0] = make_double2(nrm, 0.0);
        gm.dim[sys] = 0;
        s.rr[sys] = nrm2;
        if (!isfinite(nrm2)) {
            s.flags[sys] |= 2;
            s.active[sys] = 0;
            gm.cycle[sys] = 0;
        } else if (nrm2 <= s.rtol2 * s.bb[sys]) {
            s.active[sys] = 0;
            gm.cycle[sys] = 0;
        }
        return;
    }
    double2* H = gm.H + static_cast<size_t>(sys) * (kGmMax + 1) * kGmMax;
    double* cs = gm.cs + static_cast<size_t>(sys) * kGmMax;
    double2* sn = gm.sn + static_cast<size_t>(sys) * kGmMax;
    for (int i = 0; i < col; ++i) {
        const double2 a = H[i * kGmMax + col], b = H[(i + 1) * kGmMax + col];
        const double c = cs[i];
        const double2 sv = sn[i];
        // [a; b] -> [c a + s b; -conj(s) a + c b]
        H[i * kGmMax + col] = make_double2(c * a.x + sv.x * b.x - sv.y * b.y,
                                           c * a.y + sv.x * b.y + sv.y * b.x);
        H[(i + 1) * kGmMax + col] = make_double2(-(sv.x * a.x + sv.y * a.y) + c * b.x,
                                                 -(sv.x * a.y - sv.y * a.x) + c * b.y);
    }
    const double2 a = H[col * kGmMax + col];
    const double an = sqrt(a.x * a.x + a.y * a.y);
    const double nu = sqrt(an * an + nrm2);
    double c;
    double2 sv, r;
    if (an == 0.0) {
        c = 0.0;
        sv = make_double2(1.0, 0.0);
        r = make_double2(nrm, 0.0);
    } else {
        // b = nrm (real): s = (a/|a|) b / nu, r = (a/|a|) nu
        c = an / nu;
        const double2 ph = make_double2(a.x / an, a.y / an);
        sv = make_double2(ph.x * nrm / nu, ph.y * nrm / nu);
        r = make_double2(ph.x * nu, ph.y * nu);
    }
    cs[col] = c;
    sn[col] = sv;
    H[col * kGmMax + col] = r;
    const double2 gj = g[col];
    g[col] = make_double2(c * gj.x, c * gj.y);
    g[col + 1] = make_double2(-(sv.x * gj.x + sv.y * gj.y), -(sv.x * gj.y - sv.y * gj.x));
    gm.dim[sys] = col + 1;
    const double2 gn = g[col + 1];
    const double res2 = gn.x * gn.x + gn.y * gn.y;
    s.rr[sys] = res2;
    s.iters[sys] += 1;
    s.iters_total[sys] += 1;
    bool stop = false;
    if (!isfinite(res2) || !isfinite(nrm)) {
        s.flags[sys] |= 2;
        stop = true;
    } else if (res2 <= s.rtol2 * s.bb[sys]) {
        stop = true;
    } else if (s.iters[sys] >= s.max_iter) {
        s.flags[sys] |= 1;
        stop = true;
    }
    if (stop) s.active[sys] = 0;
    if (stop || col + 1 >= m || nrm == 0.0) gm.cycle[sys] = 0;
}

// Per system whose last cycle has columns (dim > 0): y = R^-1 g.
__global__ void k_gm_solve(int32_t n_sys, GmresState gm) {
    const int sys = blockIdx.x * blockDim.x + threadIdx.x;
    if (sys >= n_sys) return;
    const int k = gm.dim[sys];
    const double2* H = gm.H + static_cast<size_t>(sys) * (kGmMax + 1) * kGmMax;
    const double2* g = gm.g + static_cast<size_t>(sys) * (kGmMax + 1);
    double2* y = gm.y + static_cast<size_t>(sys) * kGmMax;
    for (int i = k - 1; i >= 0; --i) {
        double2 t = g[i];
        for (int l = i + 1; l < k; ++l) {
            const double2 h = H[i * kGmMax + l];
            t.x -= h.x * y[l].x - h.y * y[l].y;
            t.y -= h.x * y[l].y + h.y * y[l].x;
        }
        y[i] = cdiv(t, H[i * kGmMax + i]);
    }
}

// x += D^-1 sum_{i<dim} y_i v_i; dim is then cleared.
template <int S>
__global__ __launch_bounds__(kBlock) void k_gm_update(Geom g, const double* __restrict__ dK0,
                                                      const double4* __restrict__ daux,
                                                      const double4* __restrict__ gq, Coef lhs,
                                                      double2* __restrict__ x, GmresBasis V,
                                                      GmresState gm, int32_t n_sys) {
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        if (sys >= n_sys) continue;
        const int k = gm.dim[sys];
        if (k <= 0) continue;
        const LaneCoef<double> lc(gq[sys], lhs, g, sys);
        const double2* y = gm.y + static_cast<size_t>(sys) * kGmMax;
        sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
            for (int u = 0; u < kUs; ++u) {
                bool ok;
                const int row = slot_row<S>(first, u, r1, ok);
                if (!ok) continue;
                const size_t idx = tb + static_cast<size_t>(row) * S;
                double2 t = make_double2(0.0, 0.0);
                for (int i = 0; i < k; ++i) {
                    const double2 vv = V.base[static_cast<size_t>(i) * V.stride + idx];
                    t.x += y[i].x * vv.x - y[i].y * vv.y;
                    t.y += y[i].x * vv.y + y[i].y * vv.x;
                }
                double dr, di;
                diag_at(dK0, daux, row, lc, dr, di);
                const double2 zt = cdivT<double>(t, dr, di);
                const double2 xo = x[idx];
                x[idx] = make_double2(xo.x + zt.x, xo.y + zt.y);
            }
        });
    }
}

// r = b - q (q = A x) for the systems in the cycle; ||r||^2 partials in
// value slot 0.
template <int S>
__global__ __launch_bounds__(kBlock) void k_gm_resid(Geom g, const double2* __restrict__ b,
                                                     const double2* __restrict__ q,
                                                     double2* __restrict__ r, GmresState gm,
                                                     SolverState s) {
    __shared__ double lds[kWaves * S];
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    for (int kk = xcd; kk < g.n_items; kk += 8) {
        const ItemRef ir = item_ref(g, kk);
        const int tile = ir.tile, part = ir.part, item = ir.item;
        const int sys = tile * S + (threadIdx.x & 63) % S;
        const size_t tb = vbase(g, tile, S, sys);
        const bool act = sys < s.n_sys && s.active[sys];
        if (!__syncthreads_or(act)) continue;
        double a = 0.0;
        if (act) {
            sweep_static<S>(g, tile, part, j, [&](int first, int r1) {
#pragma unroll
                for (int u = 0; u < kUs; ++u) {
                    bool ok;
                    const int row = slot_row<S>(first, u, r1, ok);
                    if (!ok) continue;
                    const size_t idx = tb + static_cast<size_t>(row) * S;
                    const double2 bv = b[idx], qv = q[idx];
                    const double2 rv = make_double2(bv.x - qv.x, bv.y - qv.y);
                    r[idx] = rv;
                    a += rv.x * rv.x + rv.y * rv.y;
                }
            });
        }
#pragma unroll
        for (int off = S; off < 64; off <<= 1) a += __shfl_xor(a, off, 64);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane < S) lds[wave * S + lane] = a;
        __syncthreads();
        if (threadIdx.x < S) {
            double t = 0.0;
#pragma unroll
            for (int ww = 0; ww < kWaves; ++ww) t += lds[ww * S + threadIdx.x];
            gm.partial[((static_cast<size_t>(item) * g.B + j) * S + threadIdx.x) * kGmVals] = t;
        }
        __syncthreads();
    }
}

// cycle = active (start of a cycle), dim = 0; n_active[tile] = systems in it.
__global__ void k_gm_cycle_start(Geom g, GmresState gm, SolverState s) {
    const int tile = blockIdx.x;
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int l = threadIdx.x; l < g.S; l += blockDim.x) {
        const int sys = tile * g.S + l;
        const int a = (sys < s.n_sys && s.active[sys]) ? 1 : 0;
        if (sys < g.ld) {
            gm.cycle[sys] = a;
            gm.dim[sys] = 0;
        }
        if (a) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) s.n_active[tile] = cnt;
}

// n_active[tile] = systems still in the cycle (polled by the host).
__global__ void k_gm_count(Geom g, GmresState gm, SolverState s) {
    const int tile = blockIdx.x;
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int l = threadIdx.x; l < g.S; l += blockDim.x) {
        const int sys = tile * g.S + l;
        if (sys < s.n_sys && gm.cycle[sys]) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) s.n_active[tile] = cnt;
}

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw std::runtime_error(std::string("kernel launch failed (") + what + "): " +
                                 hipGetErrorString(e));
}

inline dim3 grid_of(const Geom& g) { return dim3(8u * static_cast<unsigned>(g.B)); }

template <int MODE, int K>
void launch_fin(hipStream_t st, const Geom& g0, SolverState s, Scratch sc, double2* out,
                int32_t n_sig, int32_t* zero_ctr) {
    // With many partials per tile (blocks x row parts) one block per tile
    // would read them all; a first stage spread over kFinGroups blocks per
    // tile adds them in groups, and the finalize adds the group sums.
    Geom g = g0;
    const int32_t nb = g0.n_parts * g0.B;
    if (sc.stage && nb > 2 * kFinGroups) {
        const unsigned nt = static_cast<unsigned>(g0.n_sched ? g0.n_sched : g0.n_tiles);
        const dim3 sgrid(nt * kFinGroups), sblock(kStageBlock);
        switch (g0.S) {
            case 8: k_fin_stage<8><<<sgrid, sblock, 0, st>>>(g0, sc, nb, zero_ctr); break;
            case 16: k_fin_stage<16><<<sgrid, sblock, 0, st>>>(g0, sc, nb, zero_ctr); break;
            case 32: k_fin_stage<32><<<sgrid, sblock, 0, st>>>(g0, sc, nb, zero_ctr); break;
            case 64: k_fin_stage<64><<<sgrid, sblock, 0, st>>>(g0, sc, nb, zero_ctr); break;
            case kPairS: k_fin_stage<kPairS><<<sgrid, sblock, 0, st>>>(g0, sc, nb, zero_ctr); break;
            default: throw std::runtime_error("unsupported tile width");
        }
        check_launch("finalize stage");
        g.n_parts = 1;
        g.B = kFinGroups;
        sc.partial = sc.stage;
        zero_ctr = nullptr;
    }
    const dim3 grid(static_cast<unsigned>(g.n_sched ? g.n_sched : g.n_tiles)), block(kFinBlock);
    switch (g.S) {
        case 8: k_finalize<8, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig, zero_ctr); break;
        case 16: k_finalize<16, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig, zero_ctr); break;
        case 32: k_finalize<32, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig, zero_ctr); break;
        case 64: k_finalize<64, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig, zero_ctr); break;
        case kPairS: k_finalize<kPairS, K, MODE><<<grid, block, 0, st>>>(g, s, sc, out, n_sig, zero_ctr); break;
        default: throw std::runtime_error("unsupported tile width");
    }
    check_launch("finalize");
}

}  // namespace

// ------------------------------------------------------------- launchers

Geom make_geom(int32_t n_rows, int32_t n_sys, int32_t S, int32_t blocks_per_xcd, int32_t queue,
               int32_t grab, bool xcd_split) {
    Geom g{};
    g.queue = queue;
    g.grab = std::max(1, grab);
    g.n_rows = n_rows;
    g.S = S;
    g.n_tiles = std::max(1, (n_sys + S - 1) / S);
    g.ld = g.n_tiles * S;
    // Every tile split into 8 row parts (one per XCD) keeps all XCDs busy
    // when tiles leave the Krylov loop at different times; otherwise tiles
    // are only split as far as needed for a multiple of 8 items.
    g.n_parts = xcd_split ? 8 : 8 / std::gcd(g.n_tiles, 8);
    g.n_items = g.n_tiles * g.n_parts;
    g.chunk_rows = kUs * kWaves * std::max(1, 64 / S);
    int32_t pr = (n_rows + g.n_parts - 1) / g.n_parts;
    pr = ((pr + g.chunk_rows - 1) / g.chunk_rows) * g.chunk_rows;
    g.part_rows = std::max(pr, g.chunk_rows);
    const int32_t chunks = (g.part_rows + g.chunk_rows - 1) / g.chunk_rows;
    g.bpx = std::max(1, blocks_per_xcd);
    g.B = std::max(1, std::min(g.bpx, chunks));
    // Buffer-resource gathers need a tile (FP64, 64 systems) below 2^31 bytes.
    g.tile_bytes_ok = static_cast<int64_t>(n_rows) * 64 * 16 < (int64_t(1) << 31) ? 1 : 0;
    return g;
}

Geom sched_geom(const Geom& g, const int32_t* tiles, int n) {
    if (n <= 0 || n >= g.n_tiles || n > kMaxSched || g.queue || g.mtab) return g;
    Geom s = g;
    s.n_sched = n;
    for (int i = 0; i < n; ++i) {
        if (tiles[i] < 0 || tiles[i] >= g.n_tiles) throw std::runtime_error("schedule: bad tile");
        s.sched[i] = tiles[i];
    }
    s.n_parts = std::max(g.n_parts, 8 / std::gcd(n, 8));
    s.n_items = n * s.n_parts;
    int32_t pr = (g.n_rows + s.n_parts - 1) / s.n_parts;
    pr = ((pr + g.chunk_rows - 1) / g.chunk_rows) * g.chunk_rows;
    s.part_rows = std::max(pr, g.chunk_rows);
    const int32_t chunks = (s.part_rows + g.chunk_rows - 1) / g.chunk_rows;
    s.B = std::max(1, std::min(g.bpx, chunks));
    return s;
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
                 V2<T>* x, V2<T>* r, V2<T>* p, const float2* dx, V2<T>* x_out, V2<T>* bvec,
                 SolverState s, Scratch sc, const int32_t* wmap, const V2<T>* wb) {
    if (guess_mode == 3 && !bvec) throw std::runtime_error("init: refinement needs the stored b");
    if (guess_mode == 4 && !(dx && x_out)) throw std::runtime_error("init: refinement needs dx");
    if (guess_mode == 3 && x_out == x) throw std::runtime_error("init: mode 3 gathers x, x_out must differ");
    if ((wmap == nullptr) != (wb == nullptr)) throw std::runtime_error("init: wmap and wb go together");
    const dim3 grid = grid_of(g), block(kBlock);
#define DMRI_INIT(H, GMV)                                                                     \
    k_init<T, S, H, GMV><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.Kr, A.aux, A.dK0, \
                                                 A.daux, gq, lhs, rhs, u_prev, u_prev2, x, r, p, \
                                                 dx, x_out, bvec, s, sc, wmap, wb)
#define DMRI_INIT_GM(H)                      \
    switch (guess_mode) {                    \
        case 0: DMRI_INIT(H, 0); break;      \
        case 1: DMRI_INIT(H, 1); break;      \
        case 2: DMRI_INIT(H, 2); break;      \
        case 3: DMRI_INIT(H, 3); break;      \
        default: DMRI_INIT(H, 4); break;     \
    }
    DMRI_DISPATCH_S(g.S, {
        if (herm) {
            DMRI_INIT_GM(true)
        } else {
            DMRI_INIT_GM(false)
        }
    });
#undef DMRI_INIT_GM
#undef DMRI_INIT
    check_launch("init");
    if (guess_mode >= 4)
        launch_fin<FIN_REFINE, 4>(st, g, s, sc, nullptr, 0, sc.ctr_init);
    else
        launch_fin<FIN_INIT, 4>(st, g, s, sc, nullptr, 0, sc.ctr_init);
}

void launch_inner_start(hipStream_t st, const Geom& g, const MatView<float>& A, const double4* gq,
                        Coef lhs, bool herm, const double2* r64, const int32_t* outer_active,
                        float2* r, float2* dx, float2* p, SolverState s, Scratch sc) {
    const dim3 grid = grid_of(g), block(kBlock);
    if (g.S == kPairS) {
        auto* r4 = reinterpret_cast<float4*>(r);
        auto* x4 = reinterpret_cast<float4*>(dx);
#define DMRI_ISP(H, B)                                                                        \
    k_inner_start_pair<H, B><<<grid, block, 0, st>>>(                                          \
        g, A.dK0, A.daux, gq, lhs, r64, outer_active, r4, x4,                                 \
        reinterpret_cast<typename DirOf<B>::type*>(p), s, sc)
        if (herm) {
            if (g.dir16) DMRI_ISP(true, true); else DMRI_ISP(true, false);
        } else {
            if (g.dir16) DMRI_ISP(false, true); else DMRI_ISP(false, false);
        }
#undef DMRI_ISP
        check_launch("inner_start");
        launch_fin<FIN_INIT, 4>(st, g, s, sc, nullptr, 0, nullptr);
        return;
    }
    DMRI_DISPATCH_S(g.S, {
        if (herm)
            k_inner_start<S, true><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, r64,
                                                           outer_active, r, dx, p, s, sc);
        else
            k_inner_start<S, false><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, r64,
                                                            outer_active, r, dx, p, s, sc);
    });
    check_launch("inner_start");
    launch_fin<FIN_INIT, 4>(st, g, s, sc, nullptr, 0, nullptr);
}

template <typename T>
void launch_spmv_dot(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                     Coef lhs, bool herm, const V2<T>* p, V2<T>* q, SolverState s, Scratch sc) {
    const dim3 grid = grid_of(g), block(kBlock);
    if (g.S == kPairS) {
        if constexpr (sizeof(T) == 4) {
            auto* q4 = reinterpret_cast<float4*>(q);
#define DMRI_SPP(H, B, R)                                                                     \
    k_spmv_pair<H, B, R><<<grid, block, 0, st>>>(                                              \
        g, A.row_ptr, A.col, A.K0, A.aux, gq, lhs,                                            \
        reinterpret_cast<const typename DirOf<B>::type*>(p), q4, s, sc)
            if (herm) {
                if (g.dir16 && g.rows2 == 2) DMRI_SPP(true, true, 2);
                else if (g.dir16) DMRI_SPP(true, true, 0);
                else DMRI_SPP(true, false, 0);
            } else {
                if (g.dir16 && g.rows2 == 2) DMRI_SPP(false, true, 2);
                else if (g.dir16) DMRI_SPP(false, true, 0);
                else DMRI_SPP(false, false, 0);
            }
#undef DMRI_SPP
            check_launch("spmv_pair");
            launch_fin<FIN_ALPHA, 2>(st, g, s, sc, nullptr, 0, sc.ctr_spmv);
            return;
        } else {
            throw std::runtime_error("paired layout is FP32 only");
        }
    }
    DMRI_DISPATCH_S(g.S, {
        bool done = false;
        if constexpr (S >= 32) {
            if (g.lds) {
                done = true;
                if (herm)
                    k_spmv_lds<T, S, true><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.aux,
                                                               gq, lhs, p, q, s, sc);
                else
                    k_spmv_lds<T, S, false><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0,
                                                                    A.aux, gq, lhs, p, q, s, sc);
            }
        }
        if (!done) {
            if (herm)
                k_spmv_dot<T, S, true><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.aux,
                                                               gq, lhs, p, q, s, sc);
            else
                k_spmv_dot<T, S, false><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.aux,
                                                                gq, lhs, p, q, s, sc);
        }
    });
    check_launch("spmv_dot");
    launch_fin<FIN_ALPHA, 2>(st, g, s, sc, nullptr, 0, sc.ctr_spmv);
}

template <typename T>
void launch_update(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                   Coef lhs, bool herm, V2<T>* x, V2<T>* r, const V2<T>* p, const V2<T>* q,
                   SolverState s, Scratch sc, bool check_only) {
    const dim3 grid = grid_of(g), block(kBlock);
    if (g.S == kPairS) {
        if constexpr (sizeof(T) == 4) {
            auto* r4 = reinterpret_cast<float4*>(r);
            const auto* q4 = reinterpret_cast<const float4*>(q);
            if (herm)
                k_update_pair<true><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, r4, q4, s, sc);
            else
                k_update_pair<false><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, r4, q4, s,
                                                             sc);
            check_launch("update_pair");
            launch_fin<FIN_BETA, 3>(st, g, s, sc, nullptr, 0, nullptr);
            return;
        } else {
            throw std::runtime_error("paired layout is FP32 only");
        }
    }
    DMRI_DISPATCH_S(g.S, {
        if (herm)
            k_update<T, S, true><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, x, r, p, q, s,
                                                         sc);
        else
            k_update<T, S, false><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, x, r, p, q,
                                                          s, sc);
    });
    check_launch("update");
    if (check_only) launch_fin<FIN_CHECK, 3>(st, g, s, sc, nullptr, 0, nullptr);
    else launch_fin<FIN_BETA, 3>(st, g, s, sc, nullptr, 0, nullptr);
}

const double2* launch_cheb(hipStream_t st, const Geom& g, const MatView<double>& A,
                           const double4* gq, Coef lhs, const double2* ab, int m, bool start,
                           const double2* r, const double2* q, double2* const y[2], double2* d,
                           SolverState s, Scratch sc) {
    if (g.queue || g.S == kPairS)
        throw std::runtime_error("polynomial preconditioner: needs static sweeps, 8-64 systems a tile");
    if (m < 1) throw std::runtime_error("polynomial preconditioner: at least one term");
    const dim3 grid = grid_of(g), block(kBlock);
    for (int t = 0; t < m; ++t) {
        const double2* yin = t > 0 ? y[(t - 1) & 1] : nullptr;
        double2* yout = y[t & 1];
        const bool first = t == 0, last = t == m - 1;
#define DMRI_CHEB(F, L)                                                                        \
    k_cheb<S, F, L><<<grid, block, 0, st>>>(g, A.row_ptr, A.col, A.K0, A.aux, A.dK0, A.daux,  \
                                            gq, lhs, ab, t, r, q, yin, yout, d, s, sc)
        DMRI_DISPATCH_S(g.S, {
            if (first && last) DMRI_CHEB(true, true);
            else if (first) DMRI_CHEB(true, false);
            else if (last) DMRI_CHEB(false, true);
            else DMRI_CHEB(false, false);
        });
#undef DMRI_CHEB
        check_launch("cheb");
    }
    if (start) launch_fin<FIN_FLEX0, 4>(st, g, s, sc, nullptr, 0, nullptr);
    else launch_fin<FIN_FLEX, 4>(st, g, s, sc, nullptr, 0, nullptr);
    return y[(m - 1) & 1];
}

void launch_pupdate_z(hipStream_t st, const Geom& g, const double2* z, double2* p, double2* x,
                      int32_t k_iter, SolverState s) {
    if (g.S == kPairS) throw std::runtime_error("pupdate_z: 8-64 systems a tile");
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_pupdate_z<S><<<grid, block, 0, st>>>(g, z, p, x, k_iter, s); });
    check_launch("pupdate_z");
}

void launch_pc_interval(hipStream_t st, int32_t n_sys, int32_t ld, const double4* gq,
                        PcScalars ps, const float* theta, double a, double b, float* X, float* Y,
                        double2* ab) {
    const dim3 grid(static_cast<unsigned>((ld + 255) / 256)), block(256);
    if (theta) {
        k_pc_features<<<grid, block, 0, st>>>(ld, gq, ps, X);
        check_launch("pc_features");
        launch_mlp_forward(st, n_sys, X, theta, Y);
    }
    k_pc_interval<<<grid, block, 0, st>>>(n_sys, ld, theta ? Y : nullptr, a, b, ab);
    check_launch("pc_interval");
}

void launch_pc_record(hipStream_t st, int32_t n_sys, const double4* gq, PcScalars ps,
                      SolverState s, float* X, float* T, int64_t* count, int64_t cap) {
    if (!s.ab_hist) throw std::runtime_error("pc_record: no coefficient history");
    k_pc_record<<<1, 1024, 0, st>>>(n_sys, gq, ps, s, X, T, count, cap);
    check_launch("pc_record");
}

template <typename T>
bool persistent_fits(const Geom& g, bool herm, int n_cu) {
    int per_cu = 0;
    hipError_t e = hipSuccess;
    DMRI_DISPATCH_S(g.S, {
        if (herm)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(&k_krylov_persistent<T, S, true>), kBlock, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(&k_krylov_persistent<T, S, false>), kBlock, 0);
    });
    if (e != hipSuccess) return false;
    return static_cast<int64_t>(per_cu) * n_cu >= static_cast<int64_t>(8) * g.B;
}

template <typename T>
void launch_krylov_persistent(hipStream_t st, const Geom& g, const MatView<T>& A,
                              const double4* gq, Coef lhs, bool herm, V2<T>* x, V2<T>* r,
                              V2<T>* p, V2<T>* q, SolverState s, Scratch sc, GridBarrier bar) {
    if (g.ld > kMaxPersistSys || g.queue)
        throw std::runtime_error("persistent solver needs <= 64 systems and static chunks");
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        if (herm)
            k_krylov_persistent<T, S, true><<<grid, block, 0, st>>>(
                g, A.row_ptr, A.col, A.K0, A.aux, A.dK0, A.daux, gq, lhs, x, r, p, q, s, sc, bar);
        else
            k_krylov_persistent<T, S, false><<<grid, block, 0, st>>>(
                g, A.row_ptr, A.col, A.K0, A.aux, A.dK0, A.daux, gq, lhs, x, r, p, q, s, sc, bar);
    });
    check_launch("krylov_persistent");
}

template <typename T>
void launch_pupdate(hipStream_t st, const Geom& g, const MatView<T>& A, const double4* gq,
                    Coef lhs, const V2<T>* r, V2<T>* p, V2<T>* x, int32_t k_iter, SolverState s) {
    const dim3 grid = grid_of(g), block(kBlock);
    if (g.S == kPairS) {
        if constexpr (sizeof(T) == 4) {
            if (g.dir16)
                k_pupdate_pair<true><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs,
                                                             reinterpret_cast<const float4*>(r),
                                                             reinterpret_cast<uint2*>(p),
                                                             reinterpret_cast<float4*>(x), k_iter, s);
            else
                k_pupdate_pair<false><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs,
                                                              reinterpret_cast<const float4*>(r),
                                                              reinterpret_cast<float4*>(p),
                                                              reinterpret_cast<float4*>(x), k_iter,
                                                              s);
            check_launch("pupdate_pair");
            return;
        } else {
            throw std::runtime_error("paired layout is FP32 only");
        }
    }
    DMRI_DISPATCH_S(g.S, {
        k_pupdate<T, S><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, r, p, x, k_iter, s);
    });
    check_launch("pupdate");
}

template <typename T>
void launch_signal(hipStream_t st, const Geom& g, const double* w, const V2<T>* x, double2* out,
                   int32_t n_sys, Scratch sc) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_signal<T, S><<<grid, block, 0, st>>>(g, w, x, n_sys, sc); });
    check_launch("signal");
    launch_fin<FIN_SIGNAL, 2>(st, g, SolverState{}, sc, out, n_sys, nullptr);
}

template <typename T>
void launch_signal_phase(hipStream_t st, const Geom& g, const Geom& gt, const TetView& tv,
                         const double4* gq, double F, const V2<T>* x, double2* out,
                         int32_t n_sys, Scratch sc) {
    if (gt.S != g.S || gt.n_tiles != g.n_tiles)
        throw std::runtime_error("signal_phase: tet geometry must share the tiles");
    const dim3 grid = grid_of(gt), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        k_signal_phase<T, S><<<grid, block, 0, st>>>(gt, g.n_rows, tv, gq, F, x, n_sys, sc);
    });
    check_launch("signal_phase");
    launch_fin<FIN_SIGNAL, 2>(st, gt, SolverState{}, sc, out, n_sys, nullptr);
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
    if (g.mtab) throw std::runtime_error("set_initial: several-mesh batches fill per tile");
    const int64_t n = static_cast<int64_t>(g.n_rows) * g.ld;
    const unsigned blocks = static_cast<unsigned>((n + kBlock - 1) / kBlock);
    k_set_initial<T><<<blocks, kBlock, 0, st>>>(n, g.n_rows, g.S, n_sys, u0, x);
    check_launch("set_initial");
}

template <typename T>
void launch_set_initial_block(hipStream_t st, int64_t rows, int32_t S, int32_t n_live,
                              const double* u0, V2<T>* x) {
    const int64_t n = rows * S;
    if (n <= 0) return;
    if (rows > INT32_MAX) throw std::runtime_error("set_initial: block too large");
    const unsigned blocks = static_cast<unsigned>((n + kBlock - 1) / kBlock);
    k_set_initial<T><<<blocks, kBlock, 0, st>>>(n, static_cast<int32_t>(rows), S, n_live, u0, x);
    check_launch("set_initial_block");
}

template <typename T>
void launch_weak_rhs(hipStream_t st, const Geom& g, const WeakView& w, const double4* gq,
                     int32_t n_sys, double F, double c, const V2<T>* u_prev, V2<T>* wb) {
    const int64_t n = static_cast<int64_t>(w.n_slots) * g.ld;
    if (n <= 0) return;
    const unsigned blocks = static_cast<unsigned>((n + kBlock - 1) / kBlock);
    k_weak_rhs<T><<<blocks, kBlock, 0, st>>>(w, g.n_rows, g.S, g.ld, n_sys, gq, F, c, u_prev, wb);
    check_launch("weak_rhs");
}
template void launch_weak_rhs<double>(hipStream_t, const Geom&, const WeakView&, const double4*,
                                      int32_t, double, double, const double2*, double2*);
template void launch_weak_rhs<float>(hipStream_t, const Geom&, const WeakView&, const double4*,
                                     int32_t, double, double, const float2*, float2*);

void launch_sys_params(hipStream_t st, int32_t n_sys, int32_t ld, const double* b, const double* q,
                       double int_F2, double4* gq, int32_t* bad) {
    const unsigned blocks = static_cast<unsigned>((ld + 255) / 256);
    k_sys_params<<<blocks, 256, 0, st>>>(n_sys, ld, b, q, int_F2, gq, bad);
    check_launch("sys_params");
}

template <typename T>
void launch_combine(hipStream_t st, const Geom& g, const ExtrapTerms<T>& t, V2<T>* x) {
    if (t.m < 1 || t.m > kMaxHist) throw std::runtime_error("combine: 1..kMaxHist terms");
    const int64_t n = vec_elems(g);
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(8192, (n + kBlock - 1) / kBlock));
    k_combine<T><<<blocks, kBlock, 0, st>>>(n, t, x);
    check_launch("combine");
}
template void launch_combine<double>(hipStream_t, const Geom&, const ExtrapTerms<double>&,
                                     double2*);
template void launch_combine<float>(hipStream_t, const Geom&, const ExtrapTerms<float>&, float2*);

// ------------------------------------------------------ GMRES launchers

namespace {
inline unsigned sys_blocks(int32_t n) { return static_cast<unsigned>((n + 255) / 256); }

void gm_fin(hipStream_t st, const Geom& g, int nval, const GmresState& gm, const SolverState& s) {
    const dim3 grid(static_cast<unsigned>(g.n_tiles)), block(kFinBlock);
    DMRI_DISPATCH_S(g.S, { k_gm_fin<S><<<grid, block, 0, st>>>(g, nval, gm, s); });
    check_launch("gm_fin");
}
}  // namespace

void gmres_cycle_start(hipStream_t st, const Geom& g, const GmresState& gm, const SolverState& s) {
    k_gm_cycle_start<<<dim3(static_cast<unsigned>(g.n_tiles)), dim3(256), 0, st>>>(g, gm, s);
    check_launch("gm_cycle_start");
}

void gmres_count(hipStream_t st, const Geom& g, const GmresState& gm, const SolverState& s) {
    k_gm_count<<<dim3(static_cast<unsigned>(g.n_tiles)), dim3(256), 0, st>>>(g, gm, s);
    check_launch("gm_count");
}

void gmres_scale(hipStream_t st, const Geom& g, const MatView<double>& A, const double4* gq,
                 Coef lhs, const double2* w, double2* v, double2* z, const GmresState& gm,
                 const SolverState& cyc) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        k_gm_scale<S><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, w, v, z, gm, cyc);
    });
    check_launch("gm_scale");
}

void gmres_orthogonalize(hipStream_t st, const Geom& g, double2* w, GmresBasis V, int nv, int col,
                         int32_t n_sys, const GmresState& gm, const SolverState& cyc) {
    const dim3 grid = grid_of(g), block(kBlock);
    for (int pass = 0; pass < 2; ++pass) {
        for (int i0 = 0; i0 < nv; i0 += kGmBatch) {
            const int nb = std::min(kGmBatch, nv - i0);
            DMRI_DISPATCH_S(g.S, {
                k_gm_dots<S><<<grid, block, 0, st>>>(g, w, V, i0, nb, gm, cyc);
            });
            check_launch("gm_dots");
        }
        gm_fin(st, g, 2 * nv, gm, cyc);
        k_gm_addcol<<<sys_blocks(n_sys), 256, 0, st>>>(n_sys, nv, col, pass, gm);
        check_launch("gm_addcol");
        DMRI_DISPATCH_S(g.S, { k_gm_orth<S><<<grid, block, 0, st>>>(g, w, V, nv, gm, cyc); });
        check_launch("gm_orth");
    }
    gm_fin(st, g, 1, gm, cyc);  // ||w||^2 after the second pass
}

void gmres_givens(hipStream_t st, int32_t n_sys, int col, int m, bool use_rr,
                  const GmresState& gm, const SolverState& s) {
    k_gm_givens<<<sys_blocks(n_sys), 256, 0, st>>>(n_sys, col, m, use_rr ? 1 : 0, gm, s);
    check_launch("gm_givens");
}

void gmres_update(hipStream_t st, const Geom& g, const MatView<double>& A, const double4* gq,
                  Coef lhs, double2* x, GmresBasis V, int32_t n_sys, const GmresState& gm) {
    k_gm_solve<<<sys_blocks(n_sys), 256, 0, st>>>(n_sys, gm);
    check_launch("gm_solve");
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, {
        k_gm_update<S><<<grid, block, 0, st>>>(g, A.dK0, A.daux, gq, lhs, x, V, gm, n_sys);
    });
    check_launch("gm_update");
}

void gmres_residual(hipStream_t st, const Geom& g, const double2* b, const double2* q, double2* r,
                    const GmresState& gm, const SolverState& cyc) {
    const dim3 grid = grid_of(g), block(kBlock);
    DMRI_DISPATCH_S(g.S, { k_gm_resid<S><<<grid, block, 0, st>>>(g, b, q, r, gm, cyc); });
    check_launch("gm_resid");
    gm_fin(st, g, 1, gm, cyc);
}

void launch_aniso_params(hipStream_t st, int32_t n_comp, int32_t ld, const double4* gq,
                         const double* tensors, double* acomp) {
    k_aniso_params<<<dim3(static_cast<unsigned>((ld + 255) / 256)), dim3(256), 0, st>>>(
        n_comp, ld, gq, tensors, acomp);
    check_launch("aniso_params");
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
                                 V2<T>*, V2<T>*, const float2*, V2<T>*, V2<T>*, SolverState, \
                                 Scratch, const int32_t*, const V2<T>*);                       \
    template void launch_spmv_dot<T>(hipStream_t, const Geom&, const MatView<T>&,              \
                                     const double4*, Coef, bool, const V2<T>*, V2<T>*,         \
                                     SolverState, Scratch);                                    \
    template void launch_update<T>(hipStream_t, const Geom&, const MatView<T>&,                \
                                   const double4*, Coef, bool, V2<T>*, V2<T>*, const V2<T>*,   \
                                   const V2<T>*, SolverState, Scratch, bool);                  \
    template void launch_pupdate<T>(hipStream_t, const Geom&, const MatView<T>&,               \
                                    const double4*, Coef, const V2<T>*, V2<T>*, V2<T>*,        \
                                    int32_t, SolverState);                                     \
    template void launch_signal<T>(hipStream_t, const Geom&, const double*, const V2<T>*,      \
                                   double2*, int32_t, Scratch);                                \
    template void launch_signal_phase<T>(hipStream_t, const Geom&, const Geom&, const TetView&,\
                                         const double4*, double, const V2<T>*, double2*,       \
                                         int32_t, Scratch);                                    \
    template void launch_apply<T>(hipStream_t, const Geom&, const MatView<T>&, int,            \
                                  const double*, const double3*, const V2<T>*, V2<T>*);        \
    template void launch_set_initial<T>(hipStream_t, const Geom&, const double*, int32_t,      \
                                        V2<T>*);                                               \
    template void launch_set_initial_block<T>(hipStream_t, int64_t, int32_t, int32_t,          \
                                              const double*, V2<T>*);                          \
    template void launch_krylov_persistent<T>(hipStream_t, const Geom&, const MatView<T>&,     \
                                              const double4*, Coef, bool, V2<T>*, V2<T>*,      \
                                              V2<T>*, V2<T>*, SolverState, Scratch,            \
                                              GridBarrier);                                    \
    template bool persistent_fits<T>(const Geom&, bool, int);

DMRI_INST(double)
DMRI_INST(float)

}  // namespace dmri
