// 2:4 prune + compress and decompress on gfx950: integer-only streaming passes.
//
// One thread per 32 consecutive codes of a row (eight groups of four; two
// such chunks per thread on the row-per-block path when K % 32 == 0): two
// 128-bit loads in, one 128-bit store of the 16 survivors, one 32-bit word of
// metadata (eight nibbles, group 8w+n in bits 4n..4n+3) and one 32-bit word of
// keep-mask out.  Survivor choice per group compares the 7-bit magnitude
// fields (code & 0x7F): the rank of position i counts positions that beat it
// (larger field, or equal field at a lower index); the two with rank < 2 stay.
#include "common.hpp"
#include "internal.hpp"

namespace fp8k {

constexpr int kPThreads = 256;

__global__ void __launch_bounds__(kPThreads) prune24_kernel(const uint8_t *x, int64_t rows, int64_t K,
                                                            int64_t ldx, uint8_t *values, uint8_t *meta,
                                                            uint8_t *mask)
{
    const int64_t cpr = (K + 31) / 32;
    const int64_t total = rows * cpr;
    const bool vec_out = (K % 32) == 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cpr, ch = t % cpr;
        const int64_t k0 = ch * 32;
        const int ngroups = (int)((K - k0) >= 32 ? 8 : (K - k0) / 4);
        const uint8_t *src = x + r * ldx + k0;
        uint32_t w[8];
        if (ngroups == 8) {
            uint4 lo = reinterpret_cast<const uint4 *>(src)[0];
            uint4 hi = reinterpret_cast<const uint4 *>(src)[1];
            w[0] = lo.x; w[1] = lo.y; w[2] = lo.z; w[3] = lo.w;
            w[4] = hi.x; w[5] = hi.y; w[6] = hi.z; w[7] = hi.w;
        } else {
            for (int g = 0; g < 8; ++g) {
                w[g] = 0;
                if (g < ngroups)
                    for (int b = 0; b < 4; ++b) w[g] |= (uint32_t)src[4 * g + b] << (8 * b);
            }
        }
        uint32_t metaw = 0, maskw = 0, v[4] = {0, 0, 0, 0};
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            uint32_t vals, keep4;
            uint32_t nib = prune_group(w[g], vals, keep4);
            metaw |= nib << (4 * g);
            maskw |= keep4 << (4 * g);
            v[g / 2] |= vals << (16 * (g % 2));
        }
        uint8_t *vdst = values + r * (K / 2) + k0 / 2;
        uint8_t *mdst = meta + r * (K / 8) + k0 / 8;
        uint8_t *kdst = mask ? mask + r * (K / 8) + k0 / 8 : nullptr;
        if (vec_out) {
            *reinterpret_cast<uint4 *>(vdst) = make_uint4(v[0], v[1], v[2], v[3]);
            *reinterpret_cast<uint32_t *>(mdst) = metaw;
            if (kdst) *reinterpret_cast<uint32_t *>(kdst) = maskw;
        } else {
            for (int b = 0; b < 2 * ngroups; ++b) vdst[b] = (uint8_t)(v[b / 4] >> (8 * (b % 4)));
            for (int b = 0; b < ngroups / 2; ++b) {
                mdst[b] = (uint8_t)(metaw >> (8 * b));
                if (kdst) kdst[b] = (uint8_t)(maskw >> (8 * b));
            }
        }
    }
}

// Rows of K % 32 == 0 codes, one row per blockIdx.y: thread t of block b takes
// chunks (b * 2 * kPThreads + t) and that + kPThreads of its row (no index
// division; both chunks' loads are issued before any group is pruned).
// Same survivors, metadata and mask as prune24_kernel.
__global__ void __launch_bounds__(kPThreads) prune24_rows_kernel(const uint8_t *x, int64_t K, int64_t ldx,
                                                                 uint8_t *values, uint8_t *meta, uint8_t *mask)
{
    const int64_t r = blockIdx.y;
    const int64_t cpr = K / 32;
    const int64_t c0 = (int64_t)blockIdx.x * (2 * kPThreads) + threadIdx.x;
    uint4 in[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = c0 + h * kPThreads;
        if (ch < cpr) {
            const uint4 *src = reinterpret_cast<const uint4 *>(x + r * ldx + ch * 32);
            in[h][0] = src[0];
            in[h][1] = src[1];
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t ch = c0 + h * kPThreads;
        if (ch >= cpr) continue;
        const uint32_t w[8] = {in[h][0].x, in[h][0].y, in[h][0].z, in[h][0].w,
                               in[h][1].x, in[h][1].y, in[h][1].z, in[h][1].w};
        uint32_t metaw = 0, maskw = 0, v[4] = {0, 0, 0, 0};
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            uint32_t vals, keep4;
            const uint32_t nib = prune_group(w[g], vals, keep4);
            metaw |= nib << (4 * g);
            maskw |= keep4 << (4 * g);
            v[g / 2] |= vals << (16 * (g % 2));
        }
        *reinterpret_cast<uint4 *>(values + r * (K / 2) + ch * 16) = make_uint4(v[0], v[1], v[2], v[3]);
        *reinterpret_cast<uint32_t *>(meta + r * (K / 8) + ch * 4) = metaw;
        if (mask) *reinterpret_cast<uint32_t *>(mask + r * (K / 8) + ch * 4) = maskw;
    }
}

__global__ void __launch_bounds__(kPThreads) decompress24_kernel(const uint8_t *values, const uint8_t *meta,
                                                                 int64_t rows, int64_t K, uint8_t *out,
                                                                 int64_t ldo)
{
    const int64_t cpr = (K + 31) / 32;
    const int64_t total = rows * cpr;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / cpr, ch = t % cpr;
        const int64_t k0 = ch * 32;
        const int ngroups = (int)((K - k0) >= 32 ? 8 : (K - k0) / 4);
        const uint8_t *vsrc = values + r * (K / 2) + k0 / 2;
        const uint8_t *msrc = meta + r * (K / 8) + k0 / 8;
        uint32_t w[8];
        for (int g = 0; g < 8; ++g) {
            w[g] = 0;
            if (g < ngroups) {
                const uint32_t nib = (msrc[g / 2] >> (4 * (g % 2))) & 0xFu;
                const uint32_t i0 = nib & 3u, i1 = nib >> 2;
                w[g] = ((uint32_t)vsrc[2 * g] << (8 * i0)) | ((uint32_t)vsrc[2 * g + 1] << (8 * i1));
            }
        }
        uint8_t *dst = out + r * ldo + k0;
        if (ngroups == 8 && (ldo % 16) == 0) {
            reinterpret_cast<uint4 *>(dst)[0] = make_uint4(w[0], w[1], w[2], w[3]);
            reinterpret_cast<uint4 *>(dst)[1] = make_uint4(w[4], w[5], w[6], w[7]);
        } else {
            for (int b = 0; b < 4 * ngroups; ++b) dst[b] = (uint8_t)(w[b / 4] >> (8 * (b % 4)));
        }
    }
}

static int grid_for(int64_t items)
{
    int64_t g = (items + kPThreads - 1) / kPThreads;
    if (g > 8192) g = 8192;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_prune24(const uint8_t *x, int64_t rows, int64_t K, int64_t ldx, uint8_t *values,
                          uint8_t *meta, uint8_t *mask, hipStream_t st)
{
    if (K % 32 == 0 && rows <= 65535) {
        const int64_t cpr = K / 32;
        const dim3 g((unsigned)((cpr + 2 * kPThreads - 1) / (2 * kPThreads)), (unsigned)rows);
        prune24_rows_kernel<<<g, kPThreads, 0, st>>>(x, K, ldx, values, meta, mask);
    } else {
        prune24_kernel<<<grid_for(rows * ((K + 31) / 32)), kPThreads, 0, st>>>(x, rows, K, ldx, values, meta, mask);
    }
    return hipGetLastError();
}

hipError_t launch_decompress24(const uint8_t *values, const uint8_t *meta, int64_t rows, int64_t K,
                               uint8_t *out, int64_t ldo, hipStream_t st)
{
    decompress24_kernel<<<grid_for(rows * ((K + 31) / 32)), kPThreads, 0, st>>>(values, meta, rows, K, out, ldo);
    return hipGetLastError();
}

}  // namespace fp8k
