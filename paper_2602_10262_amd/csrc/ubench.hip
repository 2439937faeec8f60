// Matrix-core and LDS microbenchmarks of gfx950 (the counterpart of the
// paper's MFMA characterisation, Sec. 5: FP8 MFMA throughput against the
// number of resident wavefronts, and dependent-issue latency).
//
// MFMA kernels: one workgroup per CU (the dynamic LDS request keeps a second
// one out), `waves` wavefronts per workgroup, each issuing `chains`
// independent accumulator chains of one instruction for `iters` rounds.  With
// chains = 1 every instruction waits for the previous one: the dependent
// issue latency.  Operands are fixed register values (throughput does not
// depend on them).  LDS kernel: every wave reads 16 bytes per lane with
// ds_read_b128 from a conflict-free pattern, `iters` times.
#include <hip/hip_runtime.h>

#include <string>

#include "api_util.hpp"
#include "common.hpp"

namespace fp8k {

namespace {

template <int KIND, int U>
__global__ void __launch_bounds__(1024) mfma_rate(float *sink, int iters, int seed)
{
    v8i a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = seed + (int)threadIdx.x + i;
        b[i] = seed * 3 + i;
    }
    const v4i as = v4i{a[0], a[1], a[2], a[3]};
    float s = 0;
    if constexpr (KIND == 0 || KIND == 2) {
        v4f acc[U];
        for (int u = 0; u < U; ++u) acc[u] = v4f{0, 0, 0, 0};
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (KIND == 0)
                    acc[u] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[u], 0, 0, 0, 0, 0, 0);
                else
                    acc[u] = __builtin_amdgcn_smfmac_f32_16x16x128_fp8_fp8(as, b, acc[u], seed, 0, 0);
            }
        }
        for (int u = 0; u < U; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
    } else {
        v16f acc[U];
        for (int u = 0; u < U; ++u)
            for (int q = 0; q < 16; ++q) acc[u][q] = 0;
        for (int it = 0; it < iters; ++it) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (KIND == 1)
                    acc[u] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc[u], 0, 0, 0, 0, 0, 0);
                else
                    acc[u] = __builtin_amdgcn_smfmac_f32_32x32x64_fp8_fp8(as, b, acc[u], seed, 0, 0);
            }
        }
        for (int u = 0; u < U; ++u)
            for (int q = 0; q < 16; ++q) s += acc[u][q];
    }
    if (s == 1234.5f) sink[threadIdx.x] = s;   // keeps the chains alive; never true for these operands
}

__global__ void __launch_bounds__(1024) lds_rate(float *sink, int iters)
{
    extern __shared__ uint4 lds_buf[];
    // 64 KiB of LDS: lane l of wave w reads 16-byte slot (w * 64 + l + it) % 4096
    const int slots = 4096;
    for (int i = threadIdx.x; i < slots; i += blockDim.x) lds_buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    const int base = threadIdx.x;
    for (int it = 0; it < iters; ++it) {
        const uint4 v = lds_buf[(base + it * 64) & (slots - 1)];
        acc.x ^= v.x; acc.y += v.y; acc.z ^= v.z; acc.w += v.w;
    }
    if (acc.x == 0x12345678u && acc.y == 7u) sink[threadIdx.x] = 1.f;
}

template <int KIND, int U>
hipError_t launch_mfma(int waves, int iters, float *sink, hipStream_t st)
{
    const size_t lds = 96 * 1024;   // more than half the LDS: one workgroup per CU
    hipError_t e = hipFuncSetAttribute((const void *)mfma_rate<KIND, U>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    mfma_rate<KIND, U><<<cus, waves * 64, lds, st>>>(sink, iters, 1);
    return hipGetLastError();
}

}  // namespace

}  // namespace fp8k

using namespace fp8k;

extern "C" {

fp8_status fp8_ubench_mfma(int kind, int waves_per_cu, int chains, int iters, void *stream, double *ms)
{
    if (kind < 0 || kind > 3) return set_error(FP8_ERR_ARG, "kind must be 0..3");
    if (waves_per_cu < 1 || waves_per_cu > 16) return set_error(FP8_ERR_ARG, "waves_per_cu must be 1..16");
    if (chains != 1 && chains != 4 && chains != 8) return set_error(FP8_ERR_ARG, "chains must be 1, 4 or 8");
    if (iters < 1 || !ms) return set_error(FP8_ERR_ARG, "iters >= 1 and ms required");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float *sink = nullptr;
    hipError_t e = hipMalloc(&sink, 1024 * sizeof(float));
    if (e != hipSuccess) return hip_error(e, "sink");
    auto go = [&](int it) -> hipError_t {
#define FP8_UB(K, U) return launch_mfma<K, U>(waves_per_cu, it, sink, st)
        switch (kind * 16 + chains) {
        case 0 * 16 + 1: FP8_UB(0, 1);
        case 0 * 16 + 4: FP8_UB(0, 4);
        case 0 * 16 + 8: FP8_UB(0, 8);
        case 1 * 16 + 1: FP8_UB(1, 1);
        case 1 * 16 + 4: FP8_UB(1, 4);
        case 1 * 16 + 8: FP8_UB(1, 8);
        case 2 * 16 + 1: FP8_UB(2, 1);
        case 2 * 16 + 4: FP8_UB(2, 4);
        case 2 * 16 + 8: FP8_UB(2, 8);
        case 3 * 16 + 1: FP8_UB(3, 1);
        case 3 * 16 + 4: FP8_UB(3, 4);
        default: FP8_UB(3, 8);
        }
#undef FP8_UB
    };
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    e = go(16);   // warm-up (loads the kernel, raises the clock)
    if (e == hipSuccess) (void)hipEventRecord(e0, st);
    if (e == hipSuccess) e = go(iters);
    if (e == hipSuccess) (void)hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) return hip_error(e, "microbenchmark launch");
    *ms = t;
    return FP8_OK;
}

fp8_status fp8_ubench_lds(int waves_per_cu, int iters, void *stream, double *ms)
{
    if (waves_per_cu < 1 || waves_per_cu > 16 || iters < 1 || !ms) return set_error(FP8_ERR_ARG, "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float *sink = nullptr;
    hipError_t e = hipMalloc(&sink, 1024 * sizeof(float));
    if (e != hipSuccess) return hip_error(e, "sink");
    const size_t lds = 64 * 1024;
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    e = hipFuncSetAttribute((const void *)lds_rate, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    if (e == hipSuccess) {
        lds_rate<<<cus, waves_per_cu * 64, lds, st>>>(sink, 16);
        (void)hipEventRecord(e0, st);
        lds_rate<<<cus, waves_per_cu * 64, lds, st>>>(sink, iters);
        (void)hipEventRecord(e1, st);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) (void)hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) return hip_error(e, "LDS microbenchmark launch");
    *ms = t;
    return FP8_OK;
}

}  // extern "C"
