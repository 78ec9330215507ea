// Learned initial guess on gfx950: BF16 MFMA dense layers (see mlp.hpp).
//
// Every wavefront owns 64 samples at a time. The three layers are matrix
// products of a [64 samples x K] activation tile in LDS with a weight tile in
// LDS, done with gfx950's v_mfma_f32_32x32x16_bf16 (32x32 output blocks, K in
// steps of 16, FP32 accumulation). Lane l of an MFMA holds A[l % 32][8 (l / 32)
// + t] and B[8 (l / 32) + t][l % 32] (t = 0..7), and accumulator element v of
// lane l is C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]. Biases and ReLU are
// applied when the accumulators are written back to LDS as BF16.
//
// Training keeps per-wavefront gradient sums in registers across its sample
// tiles and writes them once; a reduction kernel adds the wavefronts in a
// fixed order (deterministic), and an Adam kernel updates the FP32 weights.
#include "mlp.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

namespace dmri {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
using bf16 = unsigned short;

constexpr int kBlk = 256;
constexpr int kWavesPerBlock = kBlk / 64;
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kMlpIn * kMlpHid;
constexpr int oW2 = oB1 + kMlpHid;
constexpr int oB2 = oW2 + kMlpHid * kMlpHid;
constexpr int oW3 = oB2 + kMlpHid;
constexpr int oB3 = oW3 + kMlpHid * kMlpOut;
static_assert(oB3 + kMlpOut == kMlpParams, "parameter packing");

// Round to nearest even (finite inputs); non-finite values keep their class.
__device__ inline bf16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return static_cast<bf16>((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<bf16>(u >> 16);
}
__device__ inline float from_bf16(bf16 h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

struct WeightLds {
    bf16 W1[kMlpIn * kMlpHid];
    bf16 W2[kMlpHid * kMlpHid];
    bf16 W3[kMlpHid * 32];  // columns 2..31 zero
    float b1[kMlpHid], b2[kMlpHid], b3[kMlpOut];
};

struct WaveLds {
    bf16 X[64 * 32];   // features in columns 0..15, zeros in 16..31
    bf16 H1[64 * kMlpHid];
    bf16 H2[64 * kMlpHid];
    bf16 dY[64 * 32];  // columns 2..31 zero
    float Y[64 * 2];
};

__device__ void stage_weights(WeightLds& w, const float* __restrict__ theta) {
    for (int i = threadIdx.x; i < kMlpIn * kMlpHid; i += blockDim.x) w.W1[i] = to_bf16(theta[oW1 + i]);
    for (int i = threadIdx.x; i < kMlpHid * kMlpHid; i += blockDim.x) w.W2[i] = to_bf16(theta[oW2 + i]);
    for (int i = threadIdx.x; i < kMlpHid * 32; i += blockDim.x) {
        const int r = i / 32, c = i % 32;
        w.W3[i] = c < kMlpOut ? to_bf16(theta[oW3 + r * kMlpOut + c]) : bf16(0);
    }
    for (int i = threadIdx.x; i < kMlpHid; i += blockDim.x) {
        w.b1[i] = theta[oB1 + i];
        w.b2[i] = theta[oB2 + i];
    }
    if (threadIdx.x < kMlpOut) w.b3[threadIdx.x] = theta[oB3 + threadIdx.x];
    __syncthreads();
}

__device__ inline int lane_id() { return threadIdx.x & 63; }

// Orders the wavefront's LDS writes before its later LDS reads of other
// lanes' elements (the waves of a block run different sample counts, so no
// block barrier is possible inside the sample loops).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__device__ inline int acc_row(int bm, int v) {
    return bm * 32 + 8 * (v >> 2) + 4 * (lane_id() >> 5) + (v & 3);
}
__device__ inline int acc_col(int bn) { return bn * 32 + (lane_id() & 31); }

// acc[bm][bn] += A[bm block rows][K] * B[K][bn block cols]; A(i, k) at
// A[i * a_si + k * a_sk], B(k, j) at B[k * b_sk + j * b_sj] (LDS, BF16).
// K is a multiple of 16.
template <int MB, int NB>
__device__ inline void wave_gemm(const bf16* A, int a_si, int a_sk, const bf16* B, int b_sk,
                                 int b_sj, int K, f32x16_t (&acc)[MB][NB]) {
    const int i = lane_id() & 31, kg = lane_id() >> 5;
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x8_t a[MB], b[NB];
#pragma unroll
        for (int bm = 0; bm < MB; ++bm)
#pragma unroll
            for (int t = 0; t < 8; ++t)
                a[bm][t] = __builtin_bit_cast(
                    __bf16, A[(bm * 32 + i) * a_si + (k0 + 8 * kg + t) * a_sk]);
#pragma unroll
        for (int bn = 0; bn < NB; ++bn)
#pragma unroll
            for (int t = 0; t < 8; ++t)
                b[bn][t] = __builtin_bit_cast(
                    __bf16, B[(k0 + 8 * kg + t) * b_sk + (bn * 32 + i) * b_sj]);
#pragma unroll
        for (int bm = 0; bm < MB; ++bm)
#pragma unroll
            for (int bn = 0; bn < NB; ++bn)
                acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[bm], b[bn], acc[bm][bn],
                                                                      0, 0, 0);
    }
}

template <int MB, int NB>
__device__ inline void zero(f32x16_t (&acc)[MB][NB]) {
#pragma unroll
    for (int bm = 0; bm < MB; ++bm)
#pragma unroll
        for (int bn = 0; bn < NB; ++bn)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[bm][bn][v] = 0.0f;
}

// Forward pass of the wavefront's 64 samples (features already in s.X).
// Leaves H1, H2 (post-ReLU, BF16) and Y (FP32) in LDS.
__device__ void forward_wave(const WeightLds& w, WaveLds& s) {
    wave_sync();
    f32x16_t a[2][2];
    zero(a);
    wave_gemm<2, 2>(s.X, 32, 1, w.W1, kMlpHid, 1, kMlpIn, a);
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = acc_row(bm, v), c = acc_col(bn);
                s.H1[r * kMlpHid + c] = to_bf16(fmaxf(a[bm][bn][v] + w.b1[c], 0.0f));
            }
    wave_sync();
    zero(a);
    wave_gemm<2, 2>(s.H1, kMlpHid, 1, w.W2, kMlpHid, 1, kMlpHid, a);
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = acc_row(bm, v), c = acc_col(bn);
                s.H2[r * kMlpHid + c] = to_bf16(fmaxf(a[bm][bn][v] + w.b2[c], 0.0f));
            }
    wave_sync();
    f32x16_t y[2][1];
    zero(y);
    wave_gemm<2, 1>(s.H2, kMlpHid, 1, w.W3, 32, 1, kMlpHid, y);
    const int c = acc_col(0);
    if (c < kMlpOut) {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int v = 0; v < 16; ++v) s.Y[acc_row(bm, v) * 2 + c] = y[bm][0][v] + w.b3[c];
    }
    wave_sync();
}

__device__ inline void clear_pad(WaveLds& s) {
    const int l = lane_id();
#pragma unroll
    for (int c = kMlpIn; c < 32; ++c) s.X[l * 32 + c] = 0;
#pragma unroll
    for (int c = 0; c < 32; ++c) s.dY[l * 32 + c] = 0;
}

// Features of one element (see mlp.hpp and include/dmri.h): the last four
// changes of the history relative to the newest one, d_k / s with d_k =
// u^{n-1-k} - u^{n-2-k} and s = |d_0| (Re, Im; the first has modulus 1), the
// phase of u^{n-1}, the changes of G F over the last two steps, G F(t^n),
// dt D (G F)^2 at t^n, the position along the gradient, the membrane flag.
// Writes the damped cubic x_dc; returns s (0: no correction, features 0).
__device__ inline double features(float (&f)[kMlpIn], const double2 (&v)[kMlpHist],
                                  const double (&c)[kMlpHist], double4 gg, const MlpStep& ms,
                                  float4 geo, float2 fl, double2& xdc) {
    xdc = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < kMlpHist; ++k) {
        xdc.x += c[k] * v[k].x;
        xdc.y += c[k] * v[k].y;
    }
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) f[k] = 0.0f;
    const double sx = v[0].x - v[1].x, sy = v[0].y - v[1].y;
    const double sc = sqrt(sx * sx + sy * sy);
    const double m = sqrt(v[0].x * v[0].x + v[0].y * v[0].y);
    if (!(sc > 1e-200) || !isfinite(sc) || !(m > 0.0) || !isfinite(m)) return 0.0;
#pragma unroll
    for (int k = 0; k < kMlpHist - 1; ++k) {
        f[2 * k] = static_cast<float>((v[k].x - v[k + 1].x) / sc);
        f[2 * k + 1] = static_cast<float>((v[k].y - v[k + 1].y) / sc);
    }
    const double G = gg.x;
    const double g0 = G * ms.F0, g1 = G * ms.F1, g2 = G * ms.F2;
    f[8] = static_cast<float>(v[0].x / m);
    f[9] = static_cast<float>(v[0].y / m);
    f[10] = static_cast<float>(10.0 * (g0 - g1));
    f[11] = static_cast<float>(10.0 * (g1 - g2));
    f[12] = static_cast<float>(g0);
    f[13] = static_cast<float>(ms.dt * geo.w * g0 * g0);
    f[14] = static_cast<float>(0.1 * (gg.y * geo.x + gg.z * geo.y + gg.w * geo.z));
    f[15] = fl.y;
    return sc;
}

// Element e of a tile-major vector: (tile, row, lane-in-tile).
__device__ inline void decode(const Geom& g, int64_t e, int& row, int& sys) {
    const int64_t slab = e / g.S;
    const int64_t tile = slab / g.n_rows;
    row = static_cast<int>(slab - tile * g.n_rows);
    sys = static_cast<int>(tile * g.S + (e - slab * g.S));
}

__global__ __launch_bounds__(kBlk) void k_mlp_guess(Geom g, const float* __restrict__ theta,
                                                     MlpDofs dofs, const double4* __restrict__ gq,
                                                     MlpStep ms, int32_t n_sys, MlpHist hist,
                                                     double2* __restrict__ x) {
    __shared__ WeightLds w;
    __shared__ WaveLds ws[kWavesPerBlock];
    stage_weights(w, theta);
    WaveLds& s = ws[threadIdx.x >> 6];
    clear_pad(s);
    const int64_t n = static_cast<int64_t>(g.n_rows) * g.ld;
    const int64_t wave0 = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    const int l = lane_id();
    for (int64_t base = wave0 * 64; base < n; base += nwaves * 64) {
        const int64_t e = base + l;
        double2 xdc = make_double2(0.0, 0.0);
        double sc = 0.0;
        float f[kMlpIn];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) f[k] = 0.0f;
        if (e < n) {
            int row = 0, sys = 0;
            decode(g, e, row, sys);
            double2 v[kMlpHist];
#pragma unroll
            for (int k = 0; k < kMlpHist; ++k) v[k] = hist.u[k][e];
            sc = features(f, v, hist.c, gq[sys], ms, dofs.geo[row], dofs.flags[row], xdc);
            if (sys >= n_sys) sc = 0.0;
        }
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) s.X[l * 32 + k] = to_bf16(sc > 0.0 ? f[k] : 0.0f);
        forward_wave(w, s);
        if (e < n) {
            double2 out = xdc;
            if (sc > 0.0) {
                const double cs = sc / kMlpTargetScale;
                out.x += cs * s.Y[l * 2 + 0];
                out.y += cs * s.Y[l * 2 + 1];
                if (!(isfinite(out.x) && isfinite(out.y))) out = xdc;
            }
            x[e] = out;
        }
    }
}

__global__ __launch_bounds__(kBlk) void k_mlp_record(Geom g, MlpDofs dofs,
                                                      const double4* __restrict__ gq, MlpStep ms,
                                                      int32_t n_sys, MlpHist hist,
                                                      const double2* __restrict__ un,
                                                      int64_t stride, int64_t offset, int64_t base,
                                                      int64_t capacity, float* __restrict__ X,
                                                      float* __restrict__ T) {
    const int64_t n = static_cast<int64_t>(g.n_rows) * g.ld;
    const int64_t cnt = (n - offset + stride - 1) / stride;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t pos = base + i;
        if (pos >= capacity) return;
        const int64_t e = offset + i * stride;
        int row, sys;
        decode(g, e, row, sys);
        float f[kMlpIn];
        double2 v[kMlpHist], xdc;
#pragma unroll
        for (int k = 0; k < kMlpHist; ++k) v[k] = hist.u[k][e];
        double sc = features(f, v, hist.c, gq[sys], ms, dofs.geo[row], dofs.flags[row], xdc);
        if (sys >= n_sys) sc = 0.0;
        const double2 c = un[e];
        float t0 = 0.0f, t1 = 0.0f;
        if (sc > 0.0) {
            t0 = static_cast<float>(kMlpTargetScale * (c.x - xdc.x) / sc);
            t1 = static_cast<float>(kMlpTargetScale * (c.y - xdc.y) / sc);
        }
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) X[pos * kMlpIn + k] = sc > 0.0 ? f[k] : 0.0f;
        // Corrections larger than the history's last change are clipped, so a
        // few such samples cannot dominate the squared error.
        T[pos * 2 + 0] = fminf(fmaxf(t0, -kMlpTargetScale), kMlpTargetScale);
        T[pos * 2 + 1] = fminf(fmaxf(t1, -kMlpTargetScale), kMlpTargetScale);
    }
}

__device__ inline void load_samples(WaveLds& s, const float* __restrict__ X, int64_t n,
                                    int64_t base) {
    const int l = lane_id();
    const int64_t e = base + l;
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) s.X[l * 32 + k] = e < n ? to_bf16(X[e * kMlpIn + k]) : bf16(0);
}

__global__ __launch_bounds__(kBlk) void k_mlp_forward(int64_t n, const float* __restrict__ X,
                                                       const float* __restrict__ theta,
                                                       float* __restrict__ Y) {
    __shared__ WeightLds w;
    __shared__ WaveLds ws[kWavesPerBlock];
    stage_weights(w, theta);
    WaveLds& s = ws[threadIdx.x >> 6];
    clear_pad(s);
    const int64_t wave0 = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    const int l = lane_id();
    for (int64_t base = wave0 * 64; base < n; base += nwaves * 64) {
        load_samples(s, X, n, base);
        forward_wave(w, s);
        if (base + l < n) {
            Y[(base + l) * 2 + 0] = s.Y[l * 2 + 0];
            Y[(base + l) * 2 + 1] = s.Y[l * 2 + 1];
        }
    }
}

// Forward + backward over the wavefront's sample tiles; one partial per
// wavefront: [kMlpParams] gradient sums (with the 1/n of the mean) and the
// squared-error sum in slot kMlpParams.
__global__ __launch_bounds__(kBlk) void k_mlp_grad(int64_t n, const float* __restrict__ X,
                                                    const float* __restrict__ T,
                                                    const float* __restrict__ theta,
                                                    float* __restrict__ partial) {
    __shared__ WeightLds w;
    __shared__ WaveLds ws[kWavesPerBlock];
    stage_weights(w, theta);
    WaveLds& s = ws[threadIdx.x >> 6];
    clear_pad(s);
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWavesPerBlock;
    const int l = lane_id();
    const float inv_n = 1.0f / static_cast<float>(n);
    f32x16_t gW1[1][2], gW2[2][2], gW3[2][1];
    zero(gW1);
    zero(gW2);
    zero(gW3);
    float gb1[2] = {0.f, 0.f}, gb2[2] = {0.f, 0.f}, gb3[2] = {0.f, 0.f}, sq = 0.f;
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        load_samples(s, X, n, base);
        forward_wave(w, s);
        const int64_t e = base + l;
        float d0 = 0.f, d1 = 0.f;
        if (e < n) {
            const float r0 = s.Y[l * 2 + 0] - T[e * 2 + 0];
            const float r1 = s.Y[l * 2 + 1] - T[e * 2 + 1];
            sq += r0 * r0 + r1 * r1;
            d0 = 2.0f * r0 * inv_n;
            d1 = 2.0f * r1 * inv_n;
        }
        gb3[0] += d0;
        gb3[1] += d1;
        s.dY[l * 32 + 0] = to_bf16(d0);
        s.dY[l * 32 + 1] = to_bf16(d1);
        wave_sync();
        // dW3 += H2^T dY
        wave_gemm<2, 1>(s.H2, 1, kMlpHid, s.dY, 32, 1, 64, gW3);
        wave_sync();
        // dH2 = dY W3^T, dZ2 = dH2 * (H2 > 0) (in place of H2)
        {
            f32x16_t t[2][2];
            zero(t);
            wave_gemm<2, 2>(s.dY, 32, 1, w.W3, 1, 32, 32, t);
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int r = acc_row(bm, v), c = acc_col(bn);
                        const float h = from_bf16(s.H2[r * kMlpHid + c]);
                        const float dz = h > 0.0f ? t[bm][bn][v] : 0.0f;
                        gb2[bn] += dz;
                        s.H2[r * kMlpHid + c] = to_bf16(dz);
                    }
        }
        wave_sync();
        // dW2 += H1^T dZ2
        wave_gemm<2, 2>(s.H1, 1, kMlpHid, s.H2, kMlpHid, 1, 64, gW2);
        wave_sync();
        // dH1 = dZ2 W2^T, dZ1 = dH1 * (H1 > 0) (in place of H1)
        {
            f32x16_t t[2][2];
            zero(t);
            wave_gemm<2, 2>(s.H2, kMlpHid, 1, w.W2, 1, kMlpHid, kMlpHid, t);
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn)
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int r = acc_row(bm, v), c = acc_col(bn);
                        const float h = from_bf16(s.H1[r * kMlpHid + c]);
                        const float dz = h > 0.0f ? t[bm][bn][v] : 0.0f;
                        gb1[bn] += dz;
                        s.H1[r * kMlpHid + c] = to_bf16(dz);
                    }
        }
        wave_sync();
        // dW1 += X^T dZ1 (rows 16..31 of the 32-row block are the zero padding)
        wave_gemm<1, 2>(s.X, 1, 32, s.H1, kMlpHid, 1, 64, gW1);
        wave_sync();
    }
    float* out = partial + wave * (kMlpParams + 1);
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = acc_row(0, v), c = acc_col(bn);
            if (r < kMlpIn) out[oW1 + r * kMlpHid + c] = gW1[0][bn][v];
        }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                out[oW2 + acc_row(bm, v) * kMlpHid + acc_col(bn)] = gW2[bm][bn][v];
    if (acc_col(0) < kMlpOut) {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                out[oW3 + acc_row(bm, v) * kMlpOut + acc_col(0)] = gW3[bm][0][v];
    }
    // Column sums: lanes l and l ^ 32 hold different rows of the same columns.
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
        gb1[bn] += __shfl_xor(gb1[bn], 32, 64);
        gb2[bn] += __shfl_xor(gb2[bn], 32, 64);
    }
    if (l < 32) {
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            out[oB1 + bn * 32 + l] = gb1[bn];
            out[oB2 + bn * 32 + l] = gb2[bn];
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        gb3[0] += __shfl_xor(gb3[0], off, 64);
        gb3[1] += __shfl_xor(gb3[1], off, 64);
        sq += __shfl_xor(sq, off, 64);
    }
    if (l == 0) {
        out[oB3 + 0] = gb3[0];
        out[oB3 + 1] = gb3[1];
        out[kMlpParams] = sq;
    }
}

// grad[p] = sum over wavefronts (in order) of partial[w][p]; slot kMlpParams
// becomes the mean squared error.
__global__ void k_mlp_reduce(const float* __restrict__ partial, int waves, int64_t n,
                             float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    double t = 0.0;
    for (int wv = 0; wv < waves; ++wv) t += partial[static_cast<size_t>(wv) * (kMlpParams + 1) + p];
    grad[p] = static_cast<float>(p == kMlpParams ? t / static_cast<double>(n) : t);
}

__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float gr = grad[p];
    if (!isfinite(gr)) return;
    const float mm = b1 * m[p] + (1.0f - b1) * gr;
    const float vv = b2 * v[p] + (1.0f - b2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

inline void check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        throw std::runtime_error(std::string("kernel launch failed (") + what + "): " +
                                 hipGetErrorString(e));
}

}  // namespace

void launch_mlp_guess(hipStream_t st, const Geom& g, const float* theta, MlpDofs dofs,
                      const double4* gq, MlpStep ms, int32_t n_sys, const MlpHist& hist,
                      double2* x) {
    const int64_t n = static_cast<int64_t>(g.n_rows) * g.ld;
    const int64_t waves = (n + 63) / 64;
    const unsigned blocks = static_cast<unsigned>(
        std::min<int64_t>(2048, (waves + kWavesPerBlock - 1) / kWavesPerBlock));
    k_mlp_guess<<<blocks, kBlk, 0, st>>>(g, theta, dofs, gq, ms, n_sys, hist, x);
    check("mlp_guess");
}

void launch_mlp_record(hipStream_t st, const Geom& g, MlpDofs dofs, const double4* gq,
                       MlpStep ms, int32_t n_sys, const MlpHist& hist, const double2* un,
                       int64_t stride, int64_t offset, int64_t base, int64_t capacity, float* X,
                       float* T) {
    const int64_t n = static_cast<int64_t>(g.n_rows) * g.ld;
    const int64_t cnt = (n - offset + stride - 1) / stride;
    const unsigned blocks = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>(4096, (cnt + 255) / 256)));
    k_mlp_record<<<blocks, 256, 0, st>>>(g, dofs, gq, ms, n_sys, hist, un, stride, offset, base,
                                         capacity, X, T);
    check("mlp_record");
}

int launch_mlp_grad(hipStream_t st, int64_t n, const float* X, const float* T,
                    const float* theta, float* partial, int partial_waves, float* grad) {
    const int64_t tiles = (n + 63) / 64;
    int waves = static_cast<int>(std::min<int64_t>(partial_waves, tiles));
    waves = std::max(kWavesPerBlock, (waves / kWavesPerBlock) * kWavesPerBlock);
    const unsigned blocks = static_cast<unsigned>(waves / kWavesPerBlock);
    k_mlp_grad<<<blocks, kBlk, 0, st>>>(n, X, T, theta, partial);
    check("mlp_grad");
    k_mlp_reduce<<<(kMlpParams + 1 + 255) / 256, 256, 0, st>>>(partial, waves, n, grad);
    check("mlp_reduce");
    return waves;
}

void launch_mlp_forward(hipStream_t st, int64_t n, const float* X, const float* theta, float* Y) {
    const int64_t tiles = (n + 63) / 64;
    const unsigned blocks = static_cast<unsigned>(
        std::max<int64_t>(1, std::min<int64_t>(2048, (tiles + kWavesPerBlock - 1) / kWavesPerBlock)));
    k_mlp_forward<<<blocks, kBlk, 0, st>>>(n, X, theta, Y);
    check("mlp_forward");
}

void launch_adam(hipStream_t st, float* theta, float* m, float* v, const float* grad, float lr,
                 float beta1, float beta2, float eps, int t) {
    const float c1 = 1.0f - std::pow(beta1, static_cast<float>(t));
    const float c2 = 1.0f - std::pow(beta2, static_cast<float>(t));
    k_adam<<<(kMlpParams + 255) / 256, 256, 0, st>>>(theta, m, v, grad, lr, beta1, beta2, eps, c1,
                                                     c2);
    check("adam");
}

}  // namespace dmri
