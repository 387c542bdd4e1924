// Sustained-rate probes of the current device: the dense MFMA rate of each
// precision form and the device-to-device copy bandwidth.  Rooflines are
// quoted against the published peaks; these measured rates sit beside them,
// as the ceiling a kernel can reach at the clock the chip holds under load.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "dloc.h"

namespace {

typedef float rp_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 rp_bf8 __attribute__((ext_vector_type(8)));
typedef int rp_i8 __attribute__((ext_vector_type(8)));

constexpr int RP_THREADS = 256;   // four waves per workgroup

// Each wave runs CH independent MFMA accumulation chains of `iters` steps on
// register operands: no memory traffic, so the launch measures the matrix
// units alone.  `flag` is 0 at run time; the store it guards keeps the chains
// live.
template <int KIND, int RP_CHAINS>
__global__ __launch_bounds__(RP_THREADS) void k_mfma_rate(int iters, int flag, float *sink)
{
    const int t = threadIdx.x;
    rp_f4 acc[RP_CHAINS];
#pragma unroll
    for (int c = 0; c < RP_CHAINS; ++c) acc[c] = rp_f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (KIND == DL_FP32) {
        const float a = 1e-3f * (t & 7), b = 1e-3f * ((t >> 3) & 7);
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < RP_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
    } else if constexpr (KIND == DL_BF16) {
        rp_bf8 a, b;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = (__bf16)(1e-3f * ((t + k) & 7));
            b[k] = (__bf16)(1e-3f * ((t >> 3) + k & 7));
        }
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < RP_CHAINS; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    } else {
        // e4m3 codes 0x30 (0.25) and 0x28 (0.125); unit E8M0 block scales (127)
        rp_i8 a, b;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            a[k] = 0x30303030 ^ ((t & 1) << k);
            b[k] = 0x28282828;
        }
        for (int i = 0; i < iters; ++i)
#pragma unroll
            for (int c = 0; c < RP_CHAINS; ++c)
                acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[c], 0, 0, 0, 0x7F7F7F7F, 0,
                                                                          0x7F7F7F7F);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < RP_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    if (flag) sink[blockIdx.x * RP_THREADS + t] = s;
}

// Grid-stride copy of n 16-byte words.
__global__ __launch_bounds__(RP_THREADS) void k_copy_stride(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                            size_t n)
{
    const size_t stride = (size_t)gridDim.x * RP_THREADS;
    for (size_t i = (size_t)blockIdx.x * RP_THREADS + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Copy of n 16-byte words: each workgroup moves one contiguous chunk of
// RP_COPY_UNROLL * RP_THREADS words, with all its loads issued before its
// stores.
constexpr int RP_COPY_UNROLL = 8;
__global__ __launch_bounds__(RP_THREADS) void k_copy_rate(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          size_t n)
{
    const size_t base = (size_t)blockIdx.x * RP_COPY_UNROLL * RP_THREADS + threadIdx.x;
    uint4 v[RP_COPY_UNROLL];
#pragma unroll
    for (int k = 0; k < RP_COPY_UNROLL; ++k) {
        const size_t i = base + (size_t)k * RP_THREADS;
        if (i < n) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < RP_COPY_UNROLL; ++k) {
        const size_t i = base + (size_t)k * RP_THREADS;
        if (i < n) dst[i] = v[k];
    }
}

}  // namespace

extern "C" int dl_measure_rate(int what, size_t bytes, int reps, double *value)
{
    if (!value || reps <= 0) return DL_ERR_INVALID_ARG;
    if (what < DL_RATE_MFMA_FP32 || what > DL_RATE_HBM_COPY) return DL_ERR_INVALID_ARG;
    if (what == DL_RATE_HBM_COPY && (bytes < 16 || bytes % 16)) return DL_ERR_INVALID_ARG;
    *value = 0.0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return DL_ERR_DEVICE;
    // many short workgroups, so the dispatcher keeps every SIMD busy to the end
    const int blocks = prop.multiProcessorCount * 64;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *a = nullptr, *b = nullptr;
    int rc = DL_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && rc == DL_OK) rc = DL_ERR_DEVICE;
        return rc == DL_OK;
    };
    double best_ms = 0.0;
    if (ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) && ok(hipEventCreate(&e0)) && ok(hipEventCreate(&e1))) {
        if (what == DL_RATE_HBM_COPY) {
            // the best of three copies: the runtime's device-to-device copy, a
            // grid-stride kernel and a chunked kernel with eight loads in flight
            if (ok(hipMalloc(&a, bytes)) && ok(hipMalloc(&b, bytes)) && ok(hipMemsetAsync(a, 0, bytes, s))) {
                const size_t n = bytes / 16;
                const size_t per = (size_t)RP_COPY_UNROLL * RP_THREADS;
                const int grid_chunk = (int)((n + per - 1) / per);
                const int grid_stride = (int)std::min<size_t>((size_t)prop.multiProcessorCount * 16,
                                                              (n + RP_THREADS - 1) / RP_THREADS);
                for (int variant = 0; variant < 3 && rc == DL_OK; ++variant) {
                    best_ms = 0.0;
                    for (int r = 0; r <= reps && rc == DL_OK; ++r) {   // launch 0 warms up
                        ok(hipEventRecord(e0, s));
                        if (variant == 0)
                            ok(hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, s));
                        else if (variant == 1)
                            k_copy_stride<<<grid_stride, RP_THREADS, 0, s>>>((const uint4 *)a, (uint4 *)b, n);
                        else
                            k_copy_rate<<<grid_chunk, RP_THREADS, 0, s>>>((const uint4 *)a, (uint4 *)b, n);
                        ok(hipGetLastError());
                        ok(hipEventRecord(e1, s));
                        float ms = 0.f;
                        if (ok(hipEventSynchronize(e1)) && ok(hipEventElapsedTime(&ms, e0, e1)) && r > 0)
                            best_ms = best_ms == 0.0 ? ms : std::min<double>(best_ms, ms);
                    }
                    if (rc == DL_OK && best_ms > 0.0)
                        *value = std::max(*value, 2.0 * (double)bytes / (best_ms * 1e-3) / 1e9);
                }
            }
        } else {
            // about 8 ms per launch at the published rates (64 workgroups per CU,
            // four of them resident at a time)
            const int iters = what == DL_RATE_MFMA_BF16 ? 5000 : 2500;
            const double flop_mfma = what == DL_RATE_MFMA_FP32 ? 2.0 * 16 * 16 * 4
                                   : what == DL_RATE_MFMA_BF16 ? 2.0 * 16 * 16 * 32
                                                               : 2.0 * 16 * 16 * 128;
            // the best of four and eight independent chains per wave
            if (ok(hipMalloc(&a, (size_t)blocks * RP_THREADS * sizeof(float)))) {
                for (int chains = 4; chains <= 8 && rc == DL_OK; chains += 4) {
                    const int it = iters * 4 / chains;    // the same work either way
                    best_ms = 0.0;
                    for (int r = 0; r <= reps && rc == DL_OK; ++r) {
                        ok(hipEventRecord(e0, s));
                        if (what == DL_RATE_MFMA_FP32)
                            (chains == 4 ? k_mfma_rate<DL_FP32, 4> : k_mfma_rate<DL_FP32, 8>)
                                <<<blocks, RP_THREADS, 0, s>>>(it, 0, (float *)a);
                        else if (what == DL_RATE_MFMA_BF16)
                            (chains == 4 ? k_mfma_rate<DL_BF16, 4> : k_mfma_rate<DL_BF16, 8>)
                                <<<blocks, RP_THREADS, 0, s>>>(it, 0, (float *)a);
                        else
                            (chains == 4 ? k_mfma_rate<DL_FP8, 4> : k_mfma_rate<DL_FP8, 8>)
                                <<<blocks, RP_THREADS, 0, s>>>(it, 0, (float *)a);
                        ok(hipGetLastError());
                        ok(hipEventRecord(e1, s));
                        float ms = 0.f;
                        if (ok(hipEventSynchronize(e1)) && ok(hipEventElapsedTime(&ms, e0, e1)) && r > 0)
                            best_ms = best_ms == 0.0 ? ms : std::min<double>(best_ms, ms);
                    }
                    const double flop = (double)blocks * (RP_THREADS / 64) * it * chains * flop_mfma;
                    if (rc == DL_OK && best_ms > 0.0) *value = std::max(*value, flop / (best_ms * 1e-3) / 1e12);
                }
            }
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (rc != DL_OK) (void)hipGetLastError();
    return rc;
}
