// Gather-throughput ceiling of one MI355X, for the SpMV's second roofline.
//
// Every wavefront loads whole 64-lane rows at pseudo-random, wavefront-uniform
// row indices, the access pattern of the batched SpMV (one matrix entry =
// one row of S systems gathered by the wavefront). The buffer is either
// 1 GiB (every load goes to HBM) or 2 MiB (it stays in each XCD's L2), and
// a lane loads 8 bytes (512-byte rows), 16 bytes (1 KB rows) or 16 bytes
// from two half-wave rows. Prints, per case, the time, the cycles per
// wavefront load per CU (at 2.4 GHz) and the bytes moved per second.
//
// Build and run (one GPU):
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         gather_ceiling.hip -o /tmp/gather_ceiling && /tmp/gather_ceiling
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#define CHK(x)                                                                         \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                  \
        }                                                                              \
    } while (0)

// MODE 0: float2 per lane (512-byte rows); 1: float4 per lane (1 KB rows);
// 2: float4 per lane, the two half-waves reading two different 512-byte rows.
// Row indices come from a per-wavefront linear congruential sequence and are
// reduced modulo n_rows, so every load stays inside the buffer.
template <int MODE>
__global__ __launch_bounds__(256) void k_gather(const float4* __restrict__ buf, int n_rows,
                                                int iters, float* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    uint32_t seed = blockIdx.x * 977u + (threadIdx.x >> 6) * 131u + 7u;
    seed = __builtin_amdgcn_readfirstlane(seed);
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            seed = seed * 1664525u + 1013904223u;
            const uint32_t row = (seed >> 8) % static_cast<uint32_t>(n_rows);
            if (MODE == 0) {
                const float2* p = reinterpret_cast<const float2*>(buf) + static_cast<size_t>(row) * 64;
                const float2 v = p[lane];
                acc += v.x + v.y;
            } else if (MODE == 1) {
                const float4 v = buf[static_cast<size_t>(row) * 64 + lane];
                acc += v.x + v.y + v.z + v.w;
            } else {
                const uint32_t row2 = (row * 7u + 3u) % static_cast<uint32_t>(n_rows);
                const uint32_t r = lane < 32 ? row : row2;
                const float4 v = buf[static_cast<size_t>(r) * 32 + (lane & 31)];
                acc += v.x + v.y + v.z + v.w;
            }
        }
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

int main() {
    CHK(hipSetDevice(0));
    int n_cu = 0;
    CHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, 0));
    const size_t big = size_t(1) << 30;
    float4* buf = nullptr;
    CHK(hipMalloc(&buf, big));
    CHK(hipMemset(buf, 0, big));
    const int blocks = n_cu * 8;
    float* out = nullptr;
    CHK(hipMalloc(&out, sizeof(float) * blocks * 256));
    hipEvent_t a, b;
    CHK(hipEventCreate(&a));
    CHK(hipEventCreate(&b));
    const int iters = 200;
    for (int resident = 0; resident < 2; ++resident) {
        for (int mode = 0; mode < 3; ++mode) {
            const size_t row_bytes = mode == 1 ? 1024 : 512;
            const size_t bytes = resident ? (size_t(2) << 20) : big;
            const int n_rows = static_cast<int>(bytes / row_bytes);
            for (int rep = 0; rep < 2; ++rep) {
                CHK(hipEventRecord(a));
                if (mode == 0) k_gather<0><<<blocks, 256>>>(buf, n_rows, iters, out);
                if (mode == 1) k_gather<1><<<blocks, 256>>>(buf, n_rows, iters, out);
                if (mode == 2) k_gather<2><<<blocks, 256>>>(buf, n_rows, iters, out);
                CHK(hipGetLastError());
                CHK(hipEventRecord(b));
                CHK(hipEventSynchronize(b));
                float ms = 0.f;
                CHK(hipEventElapsedTime(&ms, a, b));
                const double loads = static_cast<double>(blocks) * 4 * iters * 16;  // wavefront loads
                const double cycles = ms * 1e-3 * 2.4e9 / (loads / n_cu);
                const double moved = loads * (mode == 0 ? 512.0 : 1024.0);
                if (rep == 1)
                    std::printf("%s rows of %zu B (%s): %.3f ms, %.1f cycles per wavefront load "
                                "per CU, %.2f TB/s\n",
                                resident ? "L2-resident" : "HBM", row_bytes,
                                mode == 0 ? "8 B/lane" : mode == 1 ? "16 B/lane" : "16 B/lane, 2 rows",
                                ms, cycles, moved / (ms * 1e-3) / 1e12);
            }
        }
    }
    CHK(hipFree(buf));
    CHK(hipFree(out));
    return 0;
}
