// Streaming-rate probe: plain device-memory kernels whose measured rates are
// the achievable HBM figures the hot kernels' roofline fractions are read
// against (a read, a write, a copy, and the 2-read : 3-write mix of the
// y-pass kernel).  Not a step of the method.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/sigw.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 8192;    // 32 per CU: enough in flight to saturate HBM

__global__ __launch_bounds__(kThreads) void k_read(const float4* __restrict__ a, size_t n, float* __restrict__ part) {
    float s = 0.0f;
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        const float4 v = a[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    __shared__ float red[kThreads];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kThreads) void k_write(float4* __restrict__ a, size_t n, float v) {
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads)
        a[i] = make_float4(v, v, v, v);
}

__global__ __launch_bounds__(kThreads) void k_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) b[i] = a[i];
}

__global__ __launch_bounds__(kThreads) void k_mix23(const float4* __restrict__ a, const float4* __restrict__ b,
                                                    float4* __restrict__ c, float4* __restrict__ d,
                                                    float4* __restrict__ e, size_t n) {
    for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += size_t(gridDim.x) * kThreads) {
        const float4 x = a[i], y = b[i];
        c[i] = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
        d[i] = make_float4(x.x - y.x, x.y - y.y, x.z - y.z, x.w - y.w);
        e[i] = make_float4(x.x * y.x, x.y * y.y, x.z * y.z, x.w * y.w);
    }
}

}  // namespace

extern "C" sigw_status sigw_stream_probe(int32_t kind, void* buf_dev, size_t bytes, int32_t reps, void* hip_stream,
                                         double* gb_per_s) {
    static const int arrays[4] = {1, 1, 2, 5};
    if (kind < 0 || kind > 3 || !buf_dev || !gb_per_s || reps < 1 || bytes < 16 * size_t(kBlocks) * kThreads ||
        bytes % 16 != 0)
        return SIGW_E_INVALID;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t n = bytes / 16;
    float4* base = static_cast<float4*>(buf_dev);
    float* part = reinterpret_cast<float*>(base + size_t(arrays[kind]) * n);   // read partials after the arrays
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return SIGW_E_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SIGW_E_DEVICE;
    }
    auto launch = [&] {
        switch (kind) {
            case 0: k_read<<<kBlocks, kThreads, 0, s>>>(base, n, part); break;
            case 1: k_write<<<kBlocks, kThreads, 0, s>>>(base, n, 1.0f); break;
            case 2: k_copy<<<kBlocks, kThreads, 0, s>>>(base, base + n, n); break;
            default: k_mix23<<<kBlocks, kThreads, 0, s>>>(base, base + n, base + 2 * n, base + 3 * n, base + 4 * n, n);
        }
    };
    sigw_status st = SIGW_OK;
    float best = 0.0f;
    launch();                                    // warm-up
    for (int r = 0; r < reps && st == SIGW_OK; ++r) {
        float ms = 0.0f;
        if (hipEventRecord(e0, s) != hipSuccess) st = SIGW_E_DEVICE;
        launch();
        if (st == SIGW_OK && (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                              hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = SIGW_E_DEVICE;
        if (st == SIGW_OK && (r == 0 || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == SIGW_OK) *gb_per_s = double(arrays[kind]) * double(bytes) / (double(best) * 1e-3) / 1e9;
    return st;
}
