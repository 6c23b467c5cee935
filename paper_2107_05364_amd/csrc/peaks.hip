// Achievable rates of this device, measured with the library's own kernels:
// a streaming read of a device buffer (the bound of the operator passes) and
// register-only MFMA loops of the shapes the batched product uses (the
// bound of its products).  They put the roofline fractions the benchmark
// reports, which are taken against the published peaks, in context.
#include <hip/hip_bf16.h>

#include "common.h"

namespace tmag {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// One workgroup per 64 KiB chunk, as the operator passes read their tiles:
// thread t issues 16 independent 16-byte loads, load j at vector
// chunk * 4096 + 256 j + t (every wave-wide load is 1 KiB in one piece),
// cached or nontemporal.  The sum is stored only if it takes a value the
// zero-filled buffer cannot produce, so that the loads are not removed.
template <bool NT>
__global__ __launch_bounds__(256) void k_read(const v4f* __restrict__ p, float* out) {
    const v4f* q = p + static_cast<int64_t>(blockIdx.x) * 4096 + threadIdx.x;
    v4f v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if constexpr (NT) v[j] = __builtin_nontemporal_load(q + 256 * j);
        else v[j] = q[256 * j];
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) s += v[j].x + v[j].y + v[j].z + v[j].w;
    if (s == 1.0f) out[threadIdx.x] = 1.0f;
}

// One long contiguous stream per workgroup, as the stage kernel reads its
// operator rows: workgroup g reads vectors [g L, (g + 1) L) (L a multiple of
// 2048), eight independent 16-byte loads per thread per round.
template <bool NT>
__global__ __launch_bounds__(256) void k_read_stream(const v4f* __restrict__ p, int64_t L, float* out) {
    const v4f* q = p + static_cast<int64_t>(blockIdx.x) * L + threadIdx.x;
    float s = 0.f;
    for (int64_t i = 0; i < L; i += 256 * 8) {
        v4f v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (NT) v[j] = __builtin_nontemporal_load(q + i + 256 * j);
            else v[j] = q[i + 256 * j];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j].x + v[j].y + v[j].z + v[j].w;
    }
    if (s == 1.0f) out[threadIdx.x] = 1.0f;
}

// Eight (bf16) or four (32x32) independent accumulators per wave.
__global__ __launch_bounds__(256) void k_mfma_bf16_32(int iters, float* out) {
    v8bf a, b;
    for (int e = 0; e < 8; ++e) {
        a[e] = static_cast<__bf16>(1e-3f * threadIdx.x + e);
        b[e] = static_cast<__bf16>(0.5f * e);
    }
    v16f acc[4];
    for (int k = 0; k < 4; ++k)
        for (int e = 0; e < 16; ++e) acc[k][e] = 0.f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[k], 0, 0, 0);
    float s = 0.f;
    for (int k = 0; k < 4; ++k)
        for (int e = 0; e < 16; ++e) s += acc[k][e];
    if (s == 1.0f) out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mfma_f32_16(int iters, float* out) {
    const float a = 1e-3f * threadIdx.x, b = 0.5f;
    v4f acc[8];
    for (int k = 0; k < 8; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[k], 0, 0, 0);
    float s = 0.f;
    for (int k = 0; k < 8; ++k) s += acc[k].x + acc[k].y + acc[k].z + acc[k].w;
    if (s == 1.0f) out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <typename F>
hipError_t best_of(int reps, hipStream_t st, F launch, float* best_ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    *best_ms = 1e30f;
    launch();  // warm-up
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, st);
        launch();
        if (e == hipSuccess) e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < *best_ms) *best_ms = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace
}  // namespace tmag

using namespace tmag;

extern "C" tm_status tm_measure_peaks(int32_t device, int64_t read_bytes, double* read_gbs,
                                      double* mfma_bf16_tflops, double* mfma_fp32_tflops) {
    TM_REQUIRE(read_bytes >= (int64_t(1) << 20) && read_bytes <= (int64_t(16) << 30), TM_EINVAL,
               "tm_measure_peaks: read_bytes must be 1 MiB .. 16 GiB");
    TM_TRY_HIP(hipSetDevice(device));
    const int64_t chunks = read_bytes >> 16;  // 64 KiB chunks, one workgroup each
    const int64_t n4 = chunks * 4096;
    const unsigned grid = 256 * 8;  // MFMA loops: eight workgroups per CU
    void* buf = nullptr;
    float* out = nullptr;
    TM_TRY_HIP(hipMalloc(&buf, n4 * 16));
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&out), grid * 256 * sizeof(float));
    if (e == hipSuccess) e = hipMemset(buf, 0, n4 * 16);
    float ms = 0.f;
    if (e == hipSuccess && read_gbs) {
        // the faster of cached and nontemporal loads
        const v4f* src = static_cast<const v4f*>(buf);
        float ms_nt = 0.f;
        e = best_of(5, nullptr, [&] { k_read<false><<<static_cast<unsigned>(chunks), 256>>>(src, out); }, &ms);
        if (e == hipSuccess)
            e = best_of(5, nullptr, [&] { k_read<true><<<static_cast<unsigned>(chunks), 256>>>(src, out); }, &ms_nt);
        float best = fminf(ms, ms_nt);
        // long streams, 2, 4 and 8 workgroups per CU (each stream a whole
        // number of rounds; sizes that do not divide are not tried)
        for (int wpc : {2, 4, 8}) {
            const int64_t ngrp = 256 * static_cast<int64_t>(wpc);
            if (e != hipSuccess || n4 % (ngrp * 2048) != 0) continue;
            const int64_t L = n4 / ngrp;
            float a = 0.f, b = 0.f;
            e = best_of(5, nullptr, [&] { k_read_stream<false><<<static_cast<unsigned>(ngrp), 256>>>(src, L, out); },
                        &a);
            if (e == hipSuccess)
                e = best_of(5, nullptr,
                            [&] { k_read_stream<true><<<static_cast<unsigned>(ngrp), 256>>>(src, L, out); }, &b);
            if (e == hipSuccess) best = fminf(best, fminf(a, b));
        }
        if (e == hipSuccess) *read_gbs = static_cast<double>(n4) * 16 / (best * 1e-3) / 1e9;
    }
    const int iters = 2000;
    if (e == hipSuccess && mfma_bf16_tflops) {
        e = best_of(3, nullptr, [&] { k_mfma_bf16_32<<<grid, 256>>>(iters, out); }, &ms);
        if (e == hipSuccess)
            *mfma_bf16_tflops = static_cast<double>(grid) * 4 * iters * 4 * (32.0 * 32 * 16 * 2) / (ms * 1e-3) / 1e12;
    }
    if (e == hipSuccess && mfma_fp32_tflops) {
        e = best_of(3, nullptr, [&] { k_mfma_f32_16<<<grid, 256>>>(iters, out); }, &ms);
        if (e == hipSuccess)
            *mfma_fp32_tflops = static_cast<double>(grid) * 4 * iters * 8 * (16.0 * 16 * 4 * 2) / (ms * 1e-3) / 1e12;
    }
    (void)hipFree(buf);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) {
        set_error("tm_measure_peaks: %s", hipGetErrorString(e));
        return TM_EDEVICE;
    }
    return TM_OK;
}
