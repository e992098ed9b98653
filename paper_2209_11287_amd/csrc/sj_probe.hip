// Achievable peaks of the GPU the library runs on: short microbenchmarks of
// the matrix units (the MFMA forms the distance tiles use), the FP64 vector
// ALU and HBM. They are the measured denominators beside the published peaks
// when the distance kernels are placed on their roofline; nothing on the join
// path calls them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sj_internal.h"

namespace sj {
namespace {

typedef double double4_p __attribute__((ext_vector_type(4)));
typedef float float4_p __attribute__((ext_vector_type(4)));
typedef short short8_p __attribute__((ext_vector_type(8)));

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 1024;  // 4096 waves: 4 per SIMD on 256 CUs
constexpr int kChains = 4;          // independent accumulators per wave

enum { PK_F64 = 0, PK_F32 = 1, PK_BF16 = 2, PK_FP8 = 3 };

// Every wave runs kChains independent accumulator chains of one MFMA form, so
// the matrix unit never waits on a result. The operands are lane-dependent
// values near 1 (no overflow over the loop); the sum of the results is
// stored only if it equals a value it cannot take, which keeps the work.
template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma(int iters, float *sink) {
    const int lane = threadIdx.x & 63;
    float s = 0.f;
    if constexpr (KIND == PK_F64) {
        const double a = 1.0 + 0x1p-30 * lane, b = 1.0 - 0x1p-31 * lane;
        double4_p c[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = (double4_p){0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < kChains; ++k) s += (float)(c[k][0] + c[k][3]);
    } else {
        float4_p c[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = (float4_p){0.f, 0.f, 0.f, 0.f};
        if constexpr (KIND == PK_F32) {
            const float a = 1.0f + 0x1p-20f * lane, b = 1.0f - 0x1p-21f * lane;
            for (int i = 0; i < iters; ++i) {
#pragma unroll
                for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[k], 0, 0, 0);
            }
        } else if constexpr (KIND == PK_BF16) {
            // bf16 1.0 = 0x3f80; the low bit varies with the lane
            const short v = (short)(0x3f80 | (lane & 1));
            const short8_p a = (short8_p){v, v, v, v, v, v, v, v};
            const short8_p b = a;
            for (int i = 0; i < iters; ++i) {
#pragma unroll
                for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[k], 0, 0, 0);
            }
        } else {
            // E4M3 1.0 = 0x38 in every byte; the low bit varies with the lane
            const unsigned long long v = 0x3838383838383838ull | (unsigned long long)(lane & 1);
            const long a = (long)v, b = (long)v;
            for (int i = 0; i < iters; ++i) {
#pragma unroll
                for (int k = 0; k < kChains; ++k)
                    c[k] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c[k], 0, 0, 0);
            }
        }
#pragma unroll
        for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][3];
    }
    if (s == -1.0f) sink[blockIdx.x] = s;
}

// FP64 vector FMA: eight independent chains per lane (launched with 16 waves
// per SIMD: fewer leave the FMA latency partly exposed).
constexpr int kValuBlocks = 4096;
__global__ __launch_bounds__(kProbeThreads) void k_probe_valu(int iters, float *sink) {
    const int lane = threadIdx.x & 63;
    const double x = 1.0 - 0x1p-40 * lane, y = 0x1p-30;
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (double)k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = __builtin_fma(a[k], x, y);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += a[k];
    if (s == -1.0) sink[blockIdx.x] = (float)s;
}

// Streaming read: 16-byte non-temporal loads, eight in flight per lane,
// grid-stride (of the forms tried on the chip -- 4 or 8 loads per trip,
// ordinary or non-temporal, grid-stride or a contiguous run per block, 2048
// to 16384 blocks -- the fastest).
typedef unsigned v4u __attribute__((ext_vector_type(4)));
constexpr int kReadBlocks = 8192, kCopyBlocks = 16384;

__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const v4u *__restrict__ src, int64_t n16,
                                                              float *sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned acc = 0;
    for (; i + 7 * stride < n16; i += 8 * stride) {
        v4u v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= v[u].x ^ v[u].w;
    }
    for (; i < n16; i += stride) acc ^= src[i].x;
    if (acc == 0xdeadbeefu) sink[blockIdx.x] = (float)acc;
}

// Streaming copy: 16-byte non-temporal loads and stores, four per trip,
// grid-stride.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                              int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        v4u v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

// Best of `reps` timed launches after one warmup, in ms.
template <class F>
float best_ms(F launch, hipStream_t s, int reps = 3) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SJ_HIP(hipEventCreate(&e0));
    SJ_HIP(hipEventCreate(&e1));
    struct EvGuard {
        hipEvent_t a, b;
        ~EvGuard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    launch();
    SJ_HIP(hipGetLastError());
    float best = 1e30f;
    for (int r = 0; r < reps; ++r) {
        SJ_HIP(hipEventRecord(e0, s));
        launch();
        SJ_HIP(hipGetLastError());
        SJ_HIP(hipEventRecord(e1, s));
        SJ_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SJ_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
    }
    return best;
}

}  // namespace

void probe_peaks(int64_t bytes, sj_peaks &out, hipStream_t s) {
    // the bandwidth buffers come straight from the runtime and go back to
    // it (not to the library's cache); every buffer is released on the way
    // out, also when a launch fails
    struct Bufs {
        hipStream_t s;
        float *sink = nullptr;
        void *big[2] = {nullptr, nullptr};
        ~Bufs() {
            if (big[0] || big[1]) (void)hipStreamSynchronize(s);
            for (void *q : big)
                if (q) (void)hipFree(q);
            if (sink) dev_free(sink, s);
        }
    } bufs{s};
    // one slot per block of the largest grid (written only if a result takes an impossible value)
    float *sink = dev_alloc_n<float>(std::max({kProbeBlocks, kReadBlocks, kCopyBlocks, kValuBlocks}), s);
    bufs.sink = sink;
    const double waves = (double)kProbeBlocks * (kProbeThreads / 64);
    // loop trips per MFMA form: a few ms per launch at the published rates
    const int it64 = 8000, it32 = 16000, it16 = 32000, it8 = 64000, itv = 1 << 13;
    const dim3 grid(kProbeBlocks), block(kProbeThreads);
    auto mfma_tflops = [&](auto kernel, int iters, double flops_per_mfma) {
        const float ms = best_ms([&] { hipLaunchKernelGGL(kernel, grid, block, 0, s, iters, sink); }, s);
        return waves * iters * kChains * flops_per_mfma / (ms * 1e-3) / 1e12;
    };
    out.fp64_mfma_tflops = mfma_tflops(k_probe_mfma<PK_F64>, it64, 16.0 * 16 * 4 * 2);
    out.fp32_mfma_tflops = mfma_tflops(k_probe_mfma<PK_F32>, it32, 16.0 * 16 * 4 * 2);
    out.bf16_mfma_tflops = mfma_tflops(k_probe_mfma<PK_BF16>, it16, 16.0 * 16 * 32 * 2);
    out.fp8_mfma_tflops = mfma_tflops(k_probe_mfma<PK_FP8>, it8, 16.0 * 16 * 32 * 2);
    {
        const float ms =
            best_ms([&] { hipLaunchKernelGGL(k_probe_valu, dim3(kValuBlocks), block, 0, s, itv, sink); }, s);
        out.fp64_valu_tflops = (double)kValuBlocks * kProbeThreads * itv * 8 * 2 / (ms * 1e-3) / 1e12;
    }
    out.hbm_read_gbs = out.hbm_copy_gbs = 0.0;
    if (bytes > 0) {
        const int64_t n16 = bytes / 16;
        const size_t nb = (size_t)n16 * 16;
        SJ_HIP(hipStreamSynchronize(s));
        for (void *&q : bufs.big)
            if (hipMalloc(&q, nb) != hipSuccess) {
                q = nullptr;
                (void)hipGetLastError();
                throw OomError{nb};
            }
        v4u *src = static_cast<v4u *>(bufs.big[0]), *dst = static_cast<v4u *>(bufs.big[1]);
        SJ_HIP(hipMemsetAsync(src, 1, nb, s));
        const float rms =
            best_ms([&] { hipLaunchKernelGGL(k_probe_read, dim3(kReadBlocks), block, 0, s, src, n16, sink); }, s);
        const float cms =
            best_ms([&] { hipLaunchKernelGGL(k_probe_copy, dim3(kCopyBlocks), block, 0, s, src, dst, n16); }, s);
        out.hbm_read_gbs = (double)nb / (rms * 1e-3) / 1e9;
        out.hbm_copy_gbs = 2.0 * (double)nb / (cms * 1e-3) / 1e9;
    }
    SJ_HIP(hipStreamSynchronize(s));
}

}  // namespace sj
