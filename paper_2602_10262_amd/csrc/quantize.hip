// amax -> scale -> FP8 codes on gfx950.
//
// Per tensor: three launches on one stream: clear the amax word, a grid-wide
// max of |x| (wave64 shuffles, then one LDS step per workgroup, then one
// global atomic max per workgroup on the FP32 bit pattern, which orders
// non-negative floats and puts NaN above infinity), then the encode pass that
// rebuilds s, d from the amax word in every thread.
// Per row: one workgroup per row does both passes; rows of up to 16384 codes
// (a multiple of 16) stay in registers between them, longer ones are read
// again (then resident in L2).
// Every thread handles 16 consecutive elements of a row: four 128-bit loads,
// one 128-bit store of 16 codes; a ragged row end is done element by element.
#include "common.hpp"
#include "internal.hpp"

namespace fp8k {

constexpr int kQThreads = 256;

__global__ void amax_clear(uint32_t *amax_bits) { *amax_bits = 0u; }

__device__ __forceinline__ uint32_t absbits(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }

__device__ __forceinline__ uint32_t chunk_amax(const float *row, int64_t cols, int64_t c0)
{
    uint32_t m = 0;
    if (c0 + 16 <= cols) {
        const float4 *p = reinterpret_cast<const float4 *>(row + c0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float4 v = p[t];
            uint32_t a = absbits(v.x), b = absbits(v.y), c = absbits(v.z), d = absbits(v.w);
            a = a > b ? a : b;
            c = c > d ? c : d;
            a = a > c ? a : c;
            m = m > a ? m : a;
        }
    } else {
        for (int64_t c = c0; c < cols; ++c) {
            uint32_t a = absbits(row[c]);
            m = m > a ? m : a;
        }
    }
    return m;
}

template <int FMT>
__device__ __forceinline__ void chunk_encode(const float *row, int64_t cols, int64_t c0, float s, uint8_t *qrow)
{
    if (c0 + 16 <= cols) {
        const float4 *p = reinterpret_cast<const float4 *>(row + c0);
        uint32_t w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float4 v = p[t];
            w[t] = encode_fp8<FMT>(v.x * s) | (encode_fp8<FMT>(v.y * s) << 8) |
                   (encode_fp8<FMT>(v.z * s) << 16) | (encode_fp8<FMT>(v.w * s) << 24);
        }
        *reinterpret_cast<uint4 *>(qrow + c0) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
        for (int64_t c = c0; c < cols; ++c) qrow[c] = (uint8_t)encode_fp8<FMT>(row[c] * s);
    }
}

__device__ __forceinline__ uint32_t block_max(uint32_t m, uint32_t *red)
{
    m = wave_max_u32(m);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) red[wave] = m;
    __syncthreads();
    uint32_t r = 0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) r = red[w] > r ? red[w] : r;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kQThreads) amax_tensor(const float *x, int64_t rows, int64_t cols,
                                                         int64_t ldx, uint32_t *amax_bits)
{
    __shared__ uint32_t red[kQThreads / 64];
    const int64_t cpr = (cols + 15) / 16;
    const int64_t total = rows * cpr;
    uint32_t m = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cpr, c0 = (t % cpr) * 16;
        uint32_t a = chunk_amax(x + r * ldx, cols, c0);
        m = m > a ? m : a;
    }
    m = block_max(m, red);
    if (threadIdx.x == 0 && m) atomicMax(amax_bits, m);
}

template <int FMT>
__global__ void __launch_bounds__(kQThreads) quantize_tensor(const float *x, int64_t rows, int64_t cols,
                                                             int64_t ldx, uint8_t *q, int64_t ldq,
                                                             const uint32_t *amax_bits, float *s_out,
                                                             float *d_out)
{
    float s, d;
    scale_from_amax<FMT>(__uint_as_float(*amax_bits), s, d);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *s_out = s;
        *d_out = d;
    }
    const int64_t cpr = (cols + 15) / 16;
    const int64_t total = rows * cpr;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cpr, c0 = (t % cpr) * 16;
        chunk_encode<FMT>(x + r * ldx, cols, c0, s, q + r * ldq);
    }
}

template <int FMT>
__global__ void __launch_bounds__(kQThreads) quantize_rows(const float *x, int64_t rows, int64_t cols,
                                                           int64_t ldx, uint8_t *q, int64_t ldq,
                                                           float *s_out, float *d_out)
{
    __shared__ uint32_t red[kQThreads / 64];
    const int64_t r = blockIdx.x;
    const float *row = x + r * ldx;
    uint32_t m = 0;
    for (int64_t c0 = (int64_t)threadIdx.x * 16; c0 < cols; c0 += (int64_t)blockDim.x * 16) {
        uint32_t a = chunk_amax(row, cols, c0);
        m = m > a ? m : a;
    }
    m = block_max(m, red);
    float s, d;
    scale_from_amax<FMT>(__uint_as_float(m), s, d);
    if (threadIdx.x == 0) {
        s_out[r] = s;
        d_out[r] = d;
    }
    for (int64_t c0 = (int64_t)threadIdx.x * 16; c0 < cols; c0 += (int64_t)blockDim.x * 16)
        chunk_encode<FMT>(row, cols, c0, s, q + r * ldq);
}

// Per row, one read: rows of up to R * 4096 codes (cols % 16 == 0) are held in
// registers (R chunks of 16 per thread, all loads issued up front), so the
// encode pass does not read the row again.  Same amax, scale and codes as
// quantize_rows.
template <int FMT, int R>
__global__ void __launch_bounds__(kQThreads) quantize_rows_reg(const float *x, int64_t cols, int64_t ldx,
                                                               uint8_t *q, int64_t ldq, float *s_out,
                                                               float *d_out)
{
    __shared__ uint32_t red[kQThreads / 64];
    const int64_t r = blockIdx.x;
    const float *row = x + r * ldx;
    float4 v[R][4];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t c0 = ((int64_t)threadIdx.x + k * kQThreads) * 16;
        if (c0 < cols) {
            const float4 *p = reinterpret_cast<const float4 *>(row + c0);
#pragma unroll
            for (int t = 0; t < 4; ++t) v[k][t] = p[t];
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) v[k][t] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t a = absbits(v[k][t].x), b = absbits(v[k][t].y), c = absbits(v[k][t].z), d = absbits(v[k][t].w);
            a = a > b ? a : b;
            c = c > d ? c : d;
            a = a > c ? a : c;
            m = m > a ? m : a;
        }
    m = block_max(m, red);
    float s, d;
    scale_from_amax<FMT>(__uint_as_float(m), s, d);
    if (threadIdx.x == 0) {
        s_out[r] = s;
        d_out[r] = d;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int64_t c0 = ((int64_t)threadIdx.x + k * kQThreads) * 16;
        if (c0 < cols) {
            uint32_t w[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                w[t] = encode_fp8<FMT>(v[k][t].x * s) | (encode_fp8<FMT>(v[k][t].y * s) << 8) |
                       (encode_fp8<FMT>(v[k][t].z * s) << 16) | (encode_fp8<FMT>(v[k][t].w * s) << 24);
            *reinterpret_cast<uint4 *>(q + r * ldq + c0) = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
}

template <int FMT>
static void launch_rows(const float *x, int64_t rows, int64_t cols, int64_t ldx, uint8_t *q, int64_t ldq,
                        float *s, float *d, hipStream_t st)
{
    const dim3 g((unsigned)rows);
    if (cols % 16 == 0 && cols <= 4096)
        quantize_rows_reg<FMT, 1><<<g, kQThreads, 0, st>>>(x, cols, ldx, q, ldq, s, d);
    else if (cols % 16 == 0 && cols <= 8192)
        quantize_rows_reg<FMT, 2><<<g, kQThreads, 0, st>>>(x, cols, ldx, q, ldq, s, d);
    else if (cols % 16 == 0 && cols <= 16384)
        quantize_rows_reg<FMT, 4><<<g, kQThreads, 0, st>>>(x, cols, ldx, q, ldq, s, d);
    else
        quantize_rows<FMT><<<g, kQThreads, 0, st>>>(x, rows, cols, ldx, q, ldq, s, d);
}

// Exhaustive encoder check support: codes of the FP32 bit patterns lo .. lo+n-1.
template <int FMT>
__global__ void encode_bits(uint32_t lo, int64_t n, uint8_t *out)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = (uint8_t)encode_fp8<FMT>(__uint_as_float(lo + (uint32_t)t));
}

static int grid_for(int64_t work_items)
{
    int64_t g = (work_items + kQThreads - 1) / kQThreads;
    if (g > 4096) g = 4096;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_quantize(const float *x, int64_t rows, int64_t cols, int64_t ldx, int fmt, int per_row,
                           uint8_t *q, int64_t ldq, float *s, float *d, void *ws, hipStream_t st)
{
    if (per_row) {
        if (fmt == kE4M3) launch_rows<kE4M3>(x, rows, cols, ldx, q, ldq, s, d, st);
        else launch_rows<kE5M2>(x, rows, cols, ldx, q, ldq, s, d, st);
        return hipGetLastError();
    }
    uint32_t *amax = static_cast<uint32_t *>(ws);
    const int64_t work = rows * ((cols + 15) / 16);
    amax_clear<<<1, 1, 0, st>>>(amax);
    amax_tensor<<<grid_for(work), kQThreads, 0, st>>>(x, rows, cols, ldx, amax);
    if (fmt == kE4M3)
        quantize_tensor<kE4M3><<<grid_for(work), kQThreads, 0, st>>>(x, rows, cols, ldx, q, ldq, amax, s, d);
    else
        quantize_tensor<kE5M2><<<grid_for(work), kQThreads, 0, st>>>(x, rows, cols, ldx, q, ldq, amax, s, d);
    return hipGetLastError();
}

hipError_t launch_amax_tensor(const float *x, int64_t rows, int64_t cols, int64_t ldx, uint32_t *amax_bits,
                              hipStream_t st)
{
    amax_clear<<<1, 1, 0, st>>>(amax_bits);
    amax_tensor<<<grid_for(rows * ((cols + 15) / 16)), kQThreads, 0, st>>>(x, rows, cols, ldx, amax_bits);
    return hipGetLastError();
}

hipError_t launch_encode_bits(int fmt, uint32_t lo, int64_t n, uint8_t *out, hipStream_t st)
{
    if (fmt == kE4M3)
        encode_bits<kE4M3><<<grid_for(n), kQThreads, 0, st>>>(lo, n, out);
    else
        encode_bits<kE5M2><<<grid_for(n), kQThreads, 0, st>>>(lo, n, out);
    return hipGetLastError();
}

}  // namespace fp8k
