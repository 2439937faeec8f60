// Device-side helpers shared by the gfx950 kernels: vector types, the OCP FP8
// encoder, BF16 rounding, wave64 reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fp8k {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kE4M3 = 0;
constexpr int kE5M2 = 1;

__host__ __device__ constexpr float fmax_of(int fmt) { return fmt == kE4M3 ? 448.0f : 57344.0f; }

// FP32 -> OCP FP8, round to nearest even, saturating, NaN -> 0x7F | sign.
// Method: pick the FP8 quantum 2^(e - M) of the binade e of |x| (clamped to
// the subnormal binade), round |x| / quantum to an integer with the FPU's
// round-to-nearest-even, then assemble the code arithmetically: the integer
// y lies in [2^M, 2^(M+1)] for normal values, so ((e + bias - 1) << M) + y
// is the code, a carry out of the mantissa moving into the exponent field.
// In the subnormal binade the same formula gives y itself.
template <int FMT>
__device__ __forceinline__ uint32_t encode_fp8(float x)
{
    constexpr int M = FMT == kE4M3 ? 3 : 2;
    constexpr int BIAS = FMT == kE4M3 ? 7 : 15;
    constexpr uint32_t TOP = FMT == kE4M3 ? 0x7Eu : 0x7Bu;
    constexpr int EMIN = 1 - BIAS;
    const uint32_t bits = __float_as_uint(x);
    const uint32_t sign = (bits >> 24) & 0x80u;
    const uint32_t mag = bits & 0x7FFFFFFFu;
    if (mag > 0x7F800000u) return 0x7Fu | sign;                 // NaN
    const float ax = __uint_as_float(mag);
    if (ax >= fmax_of(FMT)) return TOP | sign;                  // saturate (infinity too)
    int e = (int)(mag >> 23) - 127;                             // FP32 subnormals -> -127
    e = e < EMIN ? EMIN : e;
    const float y = __builtin_rintf(__builtin_ldexpf(ax, M - e));   // exact scaling, RNE
    uint32_t code = ((uint32_t)(e + BIAS - 1) << M) + (uint32_t)y;
    code = code > TOP ? TOP : code;
    return code | sign;
}

// 2:4 survivors of one group of four codes packed in w (byte t = position t):
// the rank of position i counts positions that beat it (larger 7-bit
// magnitude field code & 0x7F, or an equal field at a lower index); the two
// of rank < 2 stay.
// Returns nibble i0 | i1 << 2 and the two survivor codes (v0 at i0, v1 at i1).
__device__ __forceinline__ uint32_t prune_group(uint32_t w, uint32_t &vals, uint32_t &keep4)
{
    uint32_t k[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) k[t] = (w >> (8 * t)) & 0x7Fu;
    uint32_t keep = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int beaten = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j == i) continue;
            beaten += (k[j] > k[i]) || (k[j] == k[i] && j < i);
        }
        keep |= (beaten < 2 ? 1u : 0u) << i;
    }
    // keep has exactly two bits set: lowest is i0, highest is i1
    const uint32_t i0 = (uint32_t)__builtin_ctz(keep);
    const uint32_t i1 = 31u - (uint32_t)__builtin_clz(keep);
    vals = ((w >> (8 * i0)) & 0xFFu) | (((w >> (8 * i1)) & 0xFFu) << 8);
    keep4 = keep;
    return i0 | (i1 << 2);
}

// FP32 -> BF16 bits, round to nearest even, NaN kept quiet.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// FP32 -> FP16 bits, round to nearest even (the hardware conversion),
// overflow to infinity, NaN kept.
__device__ __forceinline__ uint16_t f32_to_f16_rne(float x)
{
    const _Float16 h = (_Float16)x;
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}

// wave64 reductions through cross-lane shuffles
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        uint32_t o = (uint32_t)__shfl_xor((int)v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ double wave_max_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Scale from amax exactly as the host-side definition states: IEEE divisions,
// and 1 / 1 when amax is 0 or not finite or a result is 0 or not finite.
template <int FMT>
__device__ __forceinline__ void scale_from_amax(float amax, float &s, float &d)
{
    s = __fdiv_rn(fmax_of(FMT), amax);
    d = __fdiv_rn(1.0f, s);
    const bool bad = !(amax > 0.0f) || !__builtin_isfinite(amax) || !__builtin_isfinite(s) ||
                     s == 0.0f || !__builtin_isfinite(d);
    if (bad) {
        s = 1.0f;
        d = 1.0f;
    }
}

}  // namespace fp8k
