// Learned initial guess: a per-sample MLP 16 -> 64 -> 64 -> 2 (ReLU) whose
// output corrects the damped cubic extrapolation x_dc = sum_k c_k u^{n-1-k}
// (k = 0..4, the library's default guess) of the next time step's solution,
// scaled by the local size of the history's last change s = |u^{n-1} -
// u^{n-2}| (a flat history gets no correction). Dense layers run on BF16
// MFMA tiles with FP32 accumulation; parameters are kept in FP32 (packed
// W1[16x64], b1[64], W2[64x64], b2[64], W3[64x2], b3[2] = 5378 floats) and
// trained with Adam by the kernels below. The Krylov solve that follows is
// unchanged, so the network only changes the starting point, never the
// accepted answer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace dmri {

constexpr int kMlpIn = 16;
constexpr int kMlpHid = 64;
constexpr int kMlpOut = 2;
constexpr int kMlpParams = kMlpIn * kMlpHid + kMlpHid + kMlpHid * kMlpHid + kMlpHid +
                           kMlpHid * kMlpOut + kMlpOut;  // 5378
// The network predicts kMlpTargetScale * (u^n - x_dc) / s, recorded targets
// clipped to [-kMlpTargetScale, kMlpTargetScale] (|correction| <= s).
constexpr float kMlpTargetScale = 100.0f;
constexpr int kMlpHist = 5;  // past solutions the features and x_dc use

// History of the step: u[k] = u^{n-1-k} and the damped cubic weights.
struct MlpHist {
    const double2* u[kMlpHist];
    double c[kMlpHist];
};

// Per-step scalars the features need.
struct MlpStep {
    double F0, F1, F2;  // F (or f) at t^n, t^{n-1}, t^{n-2}
    double dt;
};

// Per-DOF geometry for the features: {x, y, z (from the box centre), D} and
// {compartment, membrane flag}.
struct MlpDofs {
    const float4* geo;
    const float2* flags;
};

// x = x_dc + s * MLP / kMlpTargetScale for every element of the tile-major
// vectors; falls back to x_dc where the prediction is not finite.
void launch_mlp_guess(hipStream_t st, const Geom& g, const float* theta, MlpDofs dofs,
                      const double4* gq, MlpStep ms, int32_t n_sys, const MlpHist& hist,
                      double2* x);

// Training samples: every `stride`-th element e (e % stride == offset) of the
// vectors writes features X[base + e / stride] and target T[...] computed
// from the history and the solved u^n = un. Elements beyond capacity are
// dropped.
void launch_mlp_record(hipStream_t st, const Geom& g, MlpDofs dofs, const double4* gq,
                       MlpStep ms, int32_t n_sys, const MlpHist& hist, const double2* un,
                       int64_t stride, int64_t offset, int64_t base, int64_t capacity, float* X,
                       float* T);

// Forward and backward over n samples: per-wave gradient partials into
// `partial` ([n_waves][kMlpParams + 1], last entry = squared-error sum), then
// `grad` = sum over waves / n (deterministic order). Returns n_waves used.
int launch_mlp_grad(hipStream_t st, int64_t n, const float* X, const float* T,
                    const float* theta, float* partial, int partial_waves, float* grad);

// Forward only: Y[n][2].
void launch_mlp_forward(hipStream_t st, int64_t n, const float* X, const float* theta, float* Y);

// Adam step on theta with moments m, v (bias-corrected with step t >= 1).
void launch_adam(hipStream_t st, float* theta, float* m, float* v, const float* grad, float lr,
                 float beta1, float beta2, float eps, int t);

}  // namespace dmri
