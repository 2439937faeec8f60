// Matrix-core and LDS microbenchmarks of gfx950 (the counterpart of the
// paper's MFMA characterisation, Sec. 5: FP8 MFMA throughput against the
// number of resident wavefronts, and dependent-issue latency).
//
// MFMA kernels: one workgroup per CU (the dynamic LDS request keeps a second
// one out), `waves` wavefronts per workgroup, each issuing `chains`
// independent accumulator chains of one instruction for `iters` rounds.  With
// chains = 1 every instruction waits for the previous one: the dependent
// issue latency.  Operands are fixed register values (throughput does not
// depend on them).  LDS kernels: every wave reads 16 bytes per lane with
// ds_read_b128 (4 with ds_read_b32 for the metadata pattern) `iters` times,
// either from a linear pattern or from the address patterns of the GEMM
// fragment reads, so bank conflicts of those patterns show up in time and in
// the LDS conflict counters.
#include <hip/hip_runtime.h>

#include <string>

#include "api_util.hpp"
#include "common.hpp"
#include "gemm_tile.hpp"

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

// LDS read patterns: 0 linear 16-byte slots; the GEMM fragment reads of one
// 16 x 128 K step, each lane l reading row (l % 16) of a 16-row block at
// chunk positions g = l / 16: 1 dense operand (128-byte rows, chunk 2g, the
// swizzle of the dense tiles), 2 compressed operand (64-byte rows, chunk g,
// its swizzle), 3 the dense B operand of the 2:4 kernels (chunk g + 4, their
// swizzle), 7 the same read on the dense tiles' swizzle (2-way conflicts), 4
// metadata (16-byte rows, a 4-byte word g: ds_read_b32), 5 compressed
// operand without swizzle (row r at r * 64), 6 metadata of two 16-row blocks
// 256 bytes apart in one instruction (ds_read2st64_b32).  Successive
// iterations move to the next 16-row block (mod 256 rows).
template <int P>
__global__ void __launch_bounds__(1024) lds_rate(float *sink, int iters)
{
    extern __shared__ uint4 lds_buf[];
    const int slots = 4096;   // 64 KiB
    for (int i = threadIdx.x; i < slots; i += blockDim.x) lds_buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    const uint8_t *bytes = reinterpret_cast<const uint8_t *>(lds_buf);
    uint4 acc = make_uint4(0, 0, 0, 0);
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, lr = l & 15, lg = l >> 4;
    for (int it = 0; it < iters; ++it) {
        const int r = ((it + w) * 16 + lr) & 255;
        if constexpr (P == 4) {
            const uint32_t v = *reinterpret_cast<const uint32_t *>(bytes + r * 16 + lg * 4);
            acc.x ^= v;
            acc.y += v;
        } else if constexpr (P == 6) {
            // the metadata words of two 16-row blocks at once (256 bytes apart:
            // one ds_read2st64_b32, as the 2:4 GEMM reads them)
            const uint32_t *m = reinterpret_cast<const uint32_t *>(bytes + (r & 127) * 16 + lg * 4);
            const uint32_t v0 = m[0], v1 = m[64];
            acc.x ^= v0;
            acc.y += v1;
        } else {
            int off;
            if constexpr (P == 0) off = ((threadIdx.x + it * 64) & (slots - 1)) * 16;
            else if constexpr (P == 1) off = swz(r, 2 * lg);
            else if constexpr (P == 2) off = swz_sp(r, lg);
            else if constexpr (P == 3) off = swz_b2(r, lg + 4);
            else if constexpr (P == 7) off = swz(r, lg + 4);
            else off = r * 64 + lg * 16;
            const uint4 v = *reinterpret_cast<const uint4 *>(bytes + off);
            acc.x ^= v.x; acc.y += v.y; acc.z ^= v.z; acc.w += v.w;
        }
    }
    // every word of every read feeds the condition, so no part of a read is dead
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x12345678u) sink[threadIdx.x] = 1.f;
}

// Arbitrary per-lane pattern: lane l of every wave reads (or writes) 16 bytes
// at off.v[l] + 2048 * (it % 16) of a 64 KiB buffer (offsets 16-byte aligned
// and below 32 KiB), so any lane grouping or bank mapping can be probed.
struct LaneOffsets {
    int v[64];
};

__global__ void __launch_bounds__(1024) lds_rate_offsets(float *sink, int iters, LaneOffsets off, int write)
{
    extern __shared__ uint4 lds_buf[];
    const int slots = 4096;
    for (int i = threadIdx.x; i < slots; i += blockDim.x) lds_buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    uint8_t *bytes = reinterpret_cast<uint8_t *>(lds_buf);
    const int base = off.v[threadIdx.x & 63];
    uint4 acc = make_uint4(threadIdx.x, 1, 2, 3);
    if (write) {
        // every wave writes its pattern; the values written depend on the
        // iteration so no store is redundant
        for (int it = 0; it < iters; ++it) {
            acc.x += 1u;
            *reinterpret_cast<uint4 *>(bytes + base + 2048 * (it & 15)) = acc;
        }
        __syncthreads();
        acc = *reinterpret_cast<const uint4 *>(bytes + base);
    } else {
        for (int it = 0; it < iters; ++it) {
            const uint4 v = *reinterpret_cast<const uint4 *>(bytes + base + 2048 * (it & 15));
            acc.x ^= v.x; acc.y += v.y; acc.z ^= v.z; acc.w += v.w;
        }
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x12345678u) sink[threadIdx.x] = 1.f;
}

// Engine clock under matrix-core load: every wave of every CU runs the
// 16x16x128 FP8 MFMA throughput loop; wave 0 of block 0 reads the shader
// clock counter (clock64) and the constant-rate wall clock (wall_clock64)
// before and after its loop.
__global__ void __launch_bounds__(1024) mfma_clock(float *sink, unsigned long long *stamps, int iters)
{
    const bool rec = blockIdx.x == 0 && threadIdx.x == 0;
    unsigned long long c0 = 0, w0 = 0;
    if (rec) {
        c0 = clock64();
        w0 = wall_clock64();
    }
    v8i a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (int)threadIdx.x + i;
        b[i] = 3 + i;
    }
    v4f acc[8];
    for (int u = 0; u < 8; ++u) acc[u] = v4f{0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            acc[u] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[u], 0, 0, 0, 0, 0, 0);
    }
    float s = 0;
    for (int u = 0; u < 8; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
    if (s == 1234.5f) sink[threadIdx.x] = s;
    if (rec) {
        stamps[0] = clock64() - c0;
        stamps[1] = wall_clock64() - w0;
    }
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

fp8_status fp8_ubench_lds_pattern(int pattern, int waves_per_cu, int iters, void *stream, double *ms)
{
    if (pattern < 0 || pattern > 7) return set_error(FP8_ERR_ARG, "pattern must be 0..7");
    if (waves_per_cu < 1 || waves_per_cu > 16 || iters < 1 || !ms) return set_error(FP8_ERR_ARG, "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float *sink = nullptr;
    hipError_t e = hipMalloc(&sink, 1024 * sizeof(float));
    if (e != hipSuccess) return hip_error(e, "sink");
    const size_t lds = 64 * 1024;
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void *fn = nullptr;
    switch (pattern) {
    case 0: fn = (const void *)lds_rate<0>; break;
    case 1: fn = (const void *)lds_rate<1>; break;
    case 2: fn = (const void *)lds_rate<2>; break;
    case 3: fn = (const void *)lds_rate<3>; break;
    case 4: fn = (const void *)lds_rate<4>; break;
    case 5: fn = (const void *)lds_rate<5>; break;
    case 6: fn = (const void *)lds_rate<6>; break;
    default: fn = (const void *)lds_rate<7>; break;
    }
    auto go = [&](int it) {
        switch (pattern) {
        case 0: lds_rate<0><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        case 1: lds_rate<1><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        case 2: lds_rate<2><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        case 3: lds_rate<3><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        case 4: lds_rate<4><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        case 5: lds_rate<5><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        case 6: lds_rate<6><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        default: lds_rate<7><<<cus, waves_per_cu * 64, lds, st>>>(sink, it); break;
        }
    };
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    if (e == hipSuccess) {
        go(16);
        (void)hipEventRecord(e0, st);
        go(iters);
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

fp8_status fp8_ubench_lds_offsets(const int *lane_offsets, int write, int waves_per_cu, int iters, void *stream,
                                  double *ms)
{
    if (!lane_offsets || !ms || waves_per_cu < 1 || waves_per_cu > 16 || iters < 1)
        return set_error(FP8_ERR_ARG, "bad arguments");
    LaneOffsets off;
    for (int l = 0; l < 64; ++l) {
        if (lane_offsets[l] < 0 || lane_offsets[l] >= 32768 || lane_offsets[l] % 16)
            return set_error(FP8_ERR_ARG, "lane offsets must be 16-byte aligned and below 32768");
        off.v[l] = lane_offsets[l];
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    float *sink = nullptr;
    hipError_t e = hipMalloc(&sink, 1024 * sizeof(float));
    if (e != hipSuccess) return hip_error(e, "sink");
    const size_t lds = 64 * 1024;
    int cus = 256, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    e = hipFuncSetAttribute((const void *)lds_rate_offsets, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    if (e == hipSuccess) {
        lds_rate_offsets<<<cus, waves_per_cu * 64, lds, st>>>(sink, 16, off, write);
        (void)hipEventRecord(e0, st);
        lds_rate_offsets<<<cus, waves_per_cu * 64, lds, st>>>(sink, iters, off, write);
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

fp8_status fp8_ubench_clock(int iters, void *stream, double *ghz)
{
    if (iters < 1 || !ghz) return set_error(FP8_ERR_ARG, "bad arguments");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int cus = 256, dev = 0, wall_khz = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess || wall_khz <= 0) return set_error(FP8_ERR_UNSUPPORTED, "no wall-clock rate");
    float *sink = nullptr;
    unsigned long long *stamps = nullptr;
    e = hipMalloc(&sink, 1024 * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&stamps, 2 * sizeof(unsigned long long));
    const size_t lds = 96 * 1024;   // one workgroup per CU
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void *)mfma_clock, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    unsigned long long h[2] = {0, 0};
    if (e == hipSuccess) {
        mfma_clock<<<cus, 8 * 64, lds, st>>>(sink, stamps, 64);   // warm-up
        mfma_clock<<<cus, 8 * 64, lds, st>>>(sink, stamps, iters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, stamps, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(sink);
    (void)hipFree(stamps);
    if (e != hipSuccess) return hip_error(e, "clock microbenchmark");
    if (h[1] == 0) return set_error(FP8_ERR_UNSUPPORTED, "wall clock did not advance");
    *ghz = (double)h[0] / ((double)h[1] / (wall_khz * 1e3)) / 1e9;
    return FP8_OK;
}

fp8_status fp8_ubench_lds(int waves_per_cu, int iters, void *stream, double *ms)
{
    return fp8_ubench_lds_pattern(0, waves_per_cu, iters, stream, ms);
}

}  // extern "C"
