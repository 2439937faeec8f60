// Persistent grouped GEMM kernel over a list of problems of one kind (all
// dense or all 2:4 on the weight side), and its per-tile launcher.
//
// Every problem runs weight-major: the weight (dense N x K rows, or its 2:4
// compressed form) sits in the MFMA A slot and the activations (M x K) in the
// B slot, the result being stored transposed into the row-major M x N output.
// Tile t of the list belongs to the problem whose prefix sum of tiles
// brackets it.  Workgroups (one grid sized to fill every CU) take tiles from
// a device counter with an atomic add until the list is exhausted, which
// every workgroup reaches.  Dense and 2:4 problems have kernels of their own
// so that each kernel carries one tile body.
#pragma once
#include "gemm_launch.hpp"

namespace fp8k {

template <int BM, int BN, int WM, int WN, int OCC, int PF, int FA, int FB, bool SP>
__global__ void __launch_bounds__(WM *WN * 64, OCC)
    grouped_kernel(const GroupEntry *__restrict__ table, int count, int64_t total, unsigned long long *counter)
{
    __shared__ __attribute__((aligned(16))) uint8_t smem[TileSmem<BM, BN, SP, PF>::TOTAL];
    __shared__ long long next;
    for (;;) {
        if (threadIdx.x == 0) next = (long long)atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t t = next;
        __syncthreads();
        if (t >= total) break;
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (table[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        const GemmParams p = table[lo].p;
        const int local = (int)(t - table[lo].tile_begin);
        const int tiles_m = table[lo].tiles_m;
        gemm_tile<BM, BN, WM, WN, FA, FB, SP, true, PF, false>(p, local % tiles_m, local / tiles_m, 0, smem);
    }
}

template <int BM, int BN, int WM, int WN, int OCC, int PF, bool SP>
hipError_t grouped_one(int fa, int fb, const GroupEntry *table, int count, int64_t total,
                       unsigned long long *counter, int grid, hipStream_t st)
{
    dim3 g((unsigned)grid), b(WM * WN * 64);
    switch (fa * 2 + fb) {
    case 0: grouped_kernel<BM, BN, WM, WN, OCC, PF, 0, 0, SP><<<g, b, 0, st>>>(table, count, total, counter); break;
    case 1: grouped_kernel<BM, BN, WM, WN, OCC, PF, 0, 1, SP><<<g, b, 0, st>>>(table, count, total, counter); break;
    case 2: grouped_kernel<BM, BN, WM, WN, OCC, PF, 1, 0, SP><<<g, b, 0, st>>>(table, count, total, counter); break;
    default: grouped_kernel<BM, BN, WM, WN, OCC, PF, 1, 1, SP><<<g, b, 0, st>>>(table, count, total, counter); break;
    }
    return hipGetLastError();
}

// Launcher of table tile T for one kind; instantiated once, in a
// grouped_tiles_*.hip file.
template <int T, bool SP>
hipError_t grouped_launch_tile(int fa, int fb, const GroupEntry *table, int count, int64_t total,
                               unsigned long long *counter, int grid, hipStream_t st);

// Defines the two launchers of table tile i (dense and 2:4 lists).
#define FP8_GROUPED_INSTANTIATE(i)                                                                          \
    template <>                                                                                           \
    hipError_t grouped_launch_tile<i, false>(int fa, int fb, const GroupEntry *table, int count,          \
                                             int64_t total, unsigned long long *counter, int grid,        \
                                             hipStream_t st)                                              \
    {                                                                                                     \
        using C = TileCfg<i>;                                                                             \
        return grouped_one<C::BM, C::BN, C::WM, C::WN, C::OCC, C::PF, false>(fa, fb, table, count, total, \
                                                                             counter, grid, st);          \
    }                                                                                                     \
    template <>                                                                                           \
    hipError_t grouped_launch_tile<i, true>(int fa, int fb, const GroupEntry *table, int count,           \
                                            int64_t total, unsigned long long *counter, int grid,         \
                                            hipStream_t st)                                               \
    {                                                                                                     \
        using C = TileCfg<i>;                                                                             \
        return grouped_one<C::BM, C::BN, C::WM, C::WN, C::OCC, C::PF, true>(fa, fb, table, count, total,  \
                                                                            counter, grid, st);           \
    }

// Tiles the grouped kernels are compiled for (weight-row x token shapes that
// suit transformer mixes; every one has a 2:4 body).  Tile 26 is the 64 x 64
// exact-sum tile that problems with K below kExactBelowK run on.
#define FP8_GROUP_TILES(X) X(0) X(7) X(9) X(12) X(13) X(17) X(19) X(23) X(26)
constexpr int kGroupExactTile = 26;

#define FP8_GROUPED_EXTERN(i)                                                                               \
    template <>                                                                                           \
    hipError_t grouped_launch_tile<i, false>(int, int, const GroupEntry *, int, int64_t, unsigned long long *, \
                                             int, hipStream_t);                                           \
    template <>                                                                                           \
    hipError_t grouped_launch_tile<i, true>(int, int, const GroupEntry *, int, int64_t, unsigned long long *, \
                                            int, hipStream_t);
FP8_GROUP_TILES(FP8_GROUPED_EXTERN)
#undef FP8_GROUPED_EXTERN

}  // namespace fp8k
