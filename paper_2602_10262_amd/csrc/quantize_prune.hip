// Fused quantize + 2:4 prune/compress on gfx950: the encode step of the 2:4
// path in one pass over the FP32 data.  amax -> scale -> FP8 codes exactly as
// in quantize.hip, then the 2:4 survivor choice on the codes while they are
// still in registers, so the dense codes never reach memory (5 bytes per
// element of traffic for quantize-then-prune become 4.75: 4 read, 0.5 values,
// 0.125 metadata, 0.125 mask).  The result equals fp8_quantize followed by
// fp8_sparse24_prune_compress bit for bit.
//
// Work unit: 16 consecutive elements of a row (four groups of four): four
// 128-bit loads, 8 bytes of survivors, 2 bytes of metadata and 2 of mask.  A
// row ending in 8 elements (K % 16 == 8) ends with a half unit.
#include "common.hpp"
#include "internal.hpp"

namespace fp8k {

constexpr int kFThreads = 256;

__device__ __forceinline__ uint32_t abs_bits(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }

// Units of a row: 16 elements each, the last one 8 when K % 16 == 8.
__device__ __forceinline__ int64_t units_of(int64_t K) { return (K + 15) / 16; }

__device__ __forceinline__ void load_unit(const float *row, int64_t K, int64_t c0, float4 (&v)[4])
{
    const float4 *p = reinterpret_cast<const float4 *>(row + c0);
    const bool half = c0 + 16 > K;
    v[0] = p[0];
    v[1] = p[1];
    v[2] = half ? make_float4(0.f, 0.f, 0.f, 0.f) : p[2];
    v[3] = half ? make_float4(0.f, 0.f, 0.f, 0.f) : p[3];
}

__device__ __forceinline__ uint32_t unit_amax(const float4 (&v)[4])
{
    uint32_t m = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint32_t a = abs_bits(v[t].x), b = abs_bits(v[t].y), c = abs_bits(v[t].z), d = abs_bits(v[t].w);
        a = a > b ? a : b;
        c = c > d ? c : d;
        a = a > c ? a : c;
        m = m > a ? m : a;
    }
    return m;
}

// Encodes and prunes one unit and stores its survivors, metadata and mask.
template <int FMT>
__device__ __forceinline__ void encode_prune_store(const float4 (&v)[4], int64_t K, int64_t r, int64_t c0, float s,
                                                   uint8_t *values, uint8_t *meta, uint8_t *mask)
{
    const int ngroups = c0 + 16 <= K ? 4 : 2;
    uint32_t kept[2] = {0, 0}, metaw = 0, maskw = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (g >= ngroups) break;
        const float4 x = v[g];
        const uint32_t w = encode_fp8<FMT>(x.x * s) | (encode_fp8<FMT>(x.y * s) << 8) |
                           (encode_fp8<FMT>(x.z * s) << 16) | (encode_fp8<FMT>(x.w * s) << 24);
        uint32_t vals, keep4;
        const uint32_t nib = prune_group(w, vals, keep4);
        metaw |= nib << (4 * g);
        maskw |= keep4 << (4 * g);
        kept[g / 2] |= vals << (16 * (g % 2));
    }
    uint8_t *vd = values + r * (K / 2) + c0 / 2;
    uint8_t *md = meta + r * (K / 8) + c0 / 8;
    uint8_t *kd = mask ? mask + r * (K / 8) + c0 / 8 : nullptr;
    if (K % 16 == 0) {
        *reinterpret_cast<uint2 *>(vd) = make_uint2(kept[0], kept[1]);
        *reinterpret_cast<uint16_t *>(md) = (uint16_t)metaw;
        if (kd) *reinterpret_cast<uint16_t *>(kd) = (uint16_t)maskw;
    } else {
        for (int b = 0; b < 2 * ngroups; ++b) vd[b] = (uint8_t)(kept[b / 4] >> (8 * (b % 4)));
        for (int b = 0; b < ngroups / 2; ++b) {
            md[b] = (uint8_t)(metaw >> (8 * b));
            if (kd) kd[b] = (uint8_t)(maskw >> (8 * b));
        }
    }
}

__device__ __forceinline__ uint32_t block_max_u32(uint32_t m, uint32_t *red)
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

// Per row, one workgroup per row; rows of up to R * 4096 elements stay in
// registers between the amax and the encode (R units per thread).
template <int FMT, int R>
__global__ void __launch_bounds__(kFThreads) qprune_rows_reg(const float *x, int64_t K, int64_t ldx, uint8_t *values,
                                                             uint8_t *meta, uint8_t *mask, float *s_out, float *d_out)
{
    __shared__ uint32_t red[kFThreads / 64];
    const int64_t r = blockIdx.x;
    const float *row = x + r * ldx;
    const int64_t nu = units_of(K);
    float4 v[R][4];
    uint32_t m = 0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int64_t unit = threadIdx.x + (int64_t)u * kFThreads;
        if (unit < nu) {
            load_unit(row, K, unit * 16, v[u]);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) v[u][t] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const uint32_t a = unit_amax(v[u]);
        m = m > a ? m : a;
    }
    m = block_max_u32(m, red);
    float s, d;
    scale_from_amax<FMT>(__uint_as_float(m), s, d);
    if (threadIdx.x == 0) {
        s_out[r] = s;
        d_out[r] = d;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const int64_t unit = threadIdx.x + (int64_t)u * kFThreads;
        if (unit < nu) encode_prune_store<FMT>(v[u], K, r, unit * 16, s, values, meta, mask);
    }
}

// Per row, longer rows: the amax pass and the encode pass each read the row.
template <int FMT>
__global__ void __launch_bounds__(kFThreads) qprune_rows(const float *x, int64_t K, int64_t ldx, uint8_t *values,
                                                         uint8_t *meta, uint8_t *mask, float *s_out, float *d_out)
{
    __shared__ uint32_t red[kFThreads / 64];
    const int64_t r = blockIdx.x;
    const float *row = x + r * ldx;
    const int64_t nu = units_of(K);
    uint32_t m = 0;
    for (int64_t unit = threadIdx.x; unit < nu; unit += kFThreads) {
        float4 v[4];
        load_unit(row, K, unit * 16, v);
        const uint32_t a = unit_amax(v);
        m = m > a ? m : a;
    }
    m = block_max_u32(m, red);
    float s, d;
    scale_from_amax<FMT>(__uint_as_float(m), s, d);
    if (threadIdx.x == 0) {
        s_out[r] = s;
        d_out[r] = d;
    }
    for (int64_t unit = threadIdx.x; unit < nu; unit += kFThreads) {
        float4 v[4];
        load_unit(row, K, unit * 16, v);
        encode_prune_store<FMT>(v, K, r, unit * 16, s, values, meta, mask);
    }
}

// Per tensor: the scale comes from the amax word a previous launch reduced.
template <int FMT>
__global__ void __launch_bounds__(kFThreads) qprune_tensor(const float *x, int64_t rows, int64_t K, int64_t ldx,
                                                           uint8_t *values, uint8_t *meta, uint8_t *mask,
                                                           const uint32_t *amax_bits, float *s_out, float *d_out)
{
    float s, d;
    scale_from_amax<FMT>(__uint_as_float(*amax_bits), s, d);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *s_out = s;
        *d_out = d;
    }
    const int64_t nu = units_of(K);
    const int64_t total = rows * nu;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / nu, c0 = (t % nu) * 16;
        float4 v[4];
        load_unit(x + r * ldx, K, c0, v);
        encode_prune_store<FMT>(v, K, r, c0, s, values, meta, mask);
    }
}

template <int FMT>
static void launch_qprune_rows(const float *x, int64_t rows, int64_t K, int64_t ldx, uint8_t *values,
                               uint8_t *meta, uint8_t *mask, float *s, float *d, hipStream_t st)
{
    const dim3 g((unsigned)rows);
    if (K <= 4096)
        qprune_rows_reg<FMT, 1><<<g, kFThreads, 0, st>>>(x, K, ldx, values, meta, mask, s, d);
    else if (K <= 8192)
        qprune_rows_reg<FMT, 2><<<g, kFThreads, 0, st>>>(x, K, ldx, values, meta, mask, s, d);
    else if (K <= 16384)
        qprune_rows_reg<FMT, 4><<<g, kFThreads, 0, st>>>(x, K, ldx, values, meta, mask, s, d);
    else
        qprune_rows<FMT><<<g, kFThreads, 0, st>>>(x, K, ldx, values, meta, mask, s, d);
}

hipError_t launch_quantize_prune24(const float *x, int64_t rows, int64_t K, int64_t ldx, int fmt, int per_row,
                                   uint8_t *values, uint8_t *meta, uint8_t *mask, float *s, float *d, void *ws,
                                   hipStream_t st)
{
    if (per_row) {
        if (fmt == kE4M3) launch_qprune_rows<kE4M3>(x, rows, K, ldx, values, meta, mask, s, d, st);
        else launch_qprune_rows<kE5M2>(x, rows, K, ldx, values, meta, mask, s, d, st);
        return hipGetLastError();
    }
    uint32_t *amax = static_cast<uint32_t *>(ws);
    hipError_t e = launch_amax_tensor(x, rows, K, ldx, amax, st);
    if (e != hipSuccess) return e;
    int64_t blocks = (rows * ((K + 15) / 16) + kFThreads - 1) / kFThreads;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    if (fmt == kE4M3)
        qprune_tensor<kE4M3><<<(unsigned)blocks, kFThreads, 0, st>>>(x, rows, K, ldx, values, meta, mask, amax, s, d);
    else
        qprune_tensor<kE5M2><<<(unsigned)blocks, kFThreads, 0, st>>>(x, rows, K, ldx, values, meta, mask, amax, s, d);
    return hipGetLastError();
}

}  // namespace fp8k
