// Error norms of a GEMM result against FP64 references, on the device.
// FP64 appears here only: the GEMM kernels never touch it.
#include "common.hpp"
#include "internal.hpp"

namespace fp8k {

// out[0] max |c - cref|, out[1] max ratio to the bound, out[2] sum (c - cref)^2,
// out[3] sum cref^2, out[4] number of elements over the bound.  Each
// workgroup reduces its share and then combines with atomics: max of
// non-negative doubles through their bit patterns, sums through FP64 adds.
__global__ void __launch_bounds__(256) validate_kernel(const void *c, int out_bf16, int64_t ldc,
                                                       const double *cref, const double *sabs, int64_t M,
                                                       int64_t N, int64_t K, double *out)
{
    const double u = 1.0 / 16777216.0, ub = 1.0 / 256.0;
    double emax = 0, rmax = 0, se = 0, sr = 0, over = 0;
    const int64_t total = M * N;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / N, j = t % N;
        double v;
        if (out_bf16) {
            uint32_t bits = (uint32_t)reinterpret_cast<const uint16_t *>(c)[i * ldc + j] << 16;
            v = (double)__uint_as_float(bits);
        } else {
            v = (double)reinterpret_cast<const float *>(c)[i * ldc + j];
        }
        const double r = cref[t];
        const double e = fabs(v - r);
        double b = 4.0 * (double)K * u * sabs[t];
        if (out_bf16) b = (1.0 + ub) * b + ub * fabs(r);
        const double ratio = b > 0 ? e / b : (e > 0 ? INFINITY : 0.0);
        emax = e > emax || e != e ? e : emax;
        rmax = ratio > rmax || ratio != ratio ? ratio : rmax;
        se += (v - r) * (v - r);
        sr += r * r;
        over += (e <= b) ? 0.0 : 1.0;
    }
    __shared__ double red[5][4];
    emax = wave_max_f64(emax);
    rmax = wave_max_f64(rmax);
    se = wave_sum_f64(se);
    sr = wave_sum_f64(sr);
    over = wave_sum_f64(over);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) {
        red[0][w] = emax; red[1][w] = rmax; red[2][w] = se; red[3][w] = sr; red[4][w] = over;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 4; ++k) {
            emax = red[0][k] > emax ? red[0][k] : emax;
            rmax = red[1][k] > rmax ? red[1][k] : rmax;
            se += red[2][k]; sr += red[3][k]; over += red[4][k];
        }
        atomicMax(reinterpret_cast<unsigned long long *>(&out[0]), (unsigned long long)__double_as_longlong(emax));
        atomicMax(reinterpret_cast<unsigned long long *>(&out[1]), (unsigned long long)__double_as_longlong(rmax));
        atomicAdd(&out[2], se);
        atomicAdd(&out[3], sr);
        atomicAdd(&out[4], over);
    }
}

__global__ void validate_clear(double *out)
{
    if (threadIdx.x < 5) out[threadIdx.x] = 0.0;
}

hipError_t launch_validate(const void *c, int out_bf16, int64_t ldc, const double *cref, const double *sabs,
                           int64_t M, int64_t N, int64_t K, double *out, hipStream_t st)
{
    validate_clear<<<1, 64, 0, st>>>(out);
    int64_t g = (M * N + 255) / 256;
    if (g > 2048) g = 2048;
    validate_kernel<<<(unsigned)(g < 1 ? 1 : g), 256, 0, st>>>(c, out_bf16, ldc, cref, sabs, M, N, K, out);
    return hipGetLastError();
}

}  // namespace fp8k
