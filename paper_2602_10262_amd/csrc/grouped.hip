// Grouped FP8 GEMM: many independent dense and 2:4 problems in one persistent
// launch, the batched form of a transformer-style sequence of FP8 GEMMs.
//
// Every problem runs weight-major: the weight (dense N x K rows, or its 2:4
// compressed form) sits in the MFMA A slot and the activations (M x K) in the
// B slot, the result being stored transposed into the row-major M x N output.
// A tile therefore spans BM weight rows and BN tokens, so one tile shape fits
// the whole mix of token counts and both kinds of problem.
//
// Work list: problems ordered by K, longest first; tile t of the list belongs
// to the problem whose prefix sum of tiles brackets it.  Workgroups (one grid
// sized to fill every CU) take tiles from a device counter with an atomic add
// until the list is exhausted, which every workgroup reaches.  The counter is
// cleared by a one-thread kernel in front of the persistent one, so the pair
// can be captured into a HIP graph and replayed.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "api_util.hpp"
#include "gemm_tile.hpp"

namespace fp8k {

__global__ void grouped_reset(unsigned long long *counter) { *counter = 0ull; }

// Register budget of one workgroup per SIMD set: the kernel carries both the
// dense and the 2:4 tile body, which the plain kernels' occupancy targets do
// not fit (asking for them only makes the compiler spill and reschedule).
template <int BM, int BN, int WM, int WN, int OCC, int PF, int FA, int FB>
__global__ void __launch_bounds__(WM *WN * 64, 1)
    grouped_kernel(const GroupEntry *__restrict__ table, int count, int64_t total, unsigned long long *counter)
{
    constexpr int SMD = TileSmem<BM, BN, false, PF>::TOTAL, SMS = TileSmem<BM, BN, true, PF>::TOTAL;
    __shared__ __attribute__((aligned(16))) uint8_t smem[SMD > SMS ? SMD : SMS];
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
        const int tm = local % tiles_m, tn = local / tiles_m;
        if (table[lo].sparse)
            gemm_tile<BM, BN, WM, WN, FA, FB, true, true, PF, false>(p, tm, tn, 0, smem);
        else
            gemm_tile<BM, BN, WM, WN, FA, FB, false, true, PF, false>(p, tm, tn, 0, smem);
    }
}

template <int BM, int BN, int WM, int WN, int OCC, int PF>
static hipError_t grouped_one(int fa, int fb, const GroupEntry *table, int count, int64_t total, int *counter,
                              int grid, hipStream_t st)
{
    unsigned long long *c = reinterpret_cast<unsigned long long *>(counter);
    grouped_reset<<<1, 1, 0, st>>>(c);
    dim3 g((unsigned)grid), b(WM * WN * 64);
    switch (fa * 2 + fb) {
    case 0: grouped_kernel<BM, BN, WM, WN, OCC, PF, 0, 0><<<g, b, 0, st>>>(table, count, total, c); break;
    case 1: grouped_kernel<BM, BN, WM, WN, OCC, PF, 0, 1><<<g, b, 0, st>>>(table, count, total, c); break;
    case 2: grouped_kernel<BM, BN, WM, WN, OCC, PF, 1, 0><<<g, b, 0, st>>>(table, count, total, c); break;
    default: grouped_kernel<BM, BN, WM, WN, OCC, PF, 1, 1><<<g, b, 0, st>>>(table, count, total, c); break;
    }
    return hipGetLastError();
}

// Tiles the grouped kernel is compiled for (a subset of the tile table: the
// weight-row x token shapes that suit transformer mixes).
#define FP8_GROUP_TILES(X) X(0) X(3) X(7) X(8) X(9) X(12) X(13) X(17) X(19) X(23)

template <int T>
struct TileArgs;
#define FP8_TARGS(i, bm, bn, wm, wn, occ, pf)                                          \
    template <>                                                                        \
    struct TileArgs<i> {                                                               \
        static hipError_t go(int fa, int fb, const GroupEntry *table, int count, int64_t total, \
                             int *counter, int grid, hipStream_t st)                   \
        {                                                                              \
            return grouped_one<bm, bn, wm, wn, occ, pf>(fa, fb, table, count, total, counter, grid, st); \
        }                                                                              \
    };
FP8_TILE_LIST(FP8_TARGS)
#undef FP8_TARGS

bool grouped_tile_supported(int tile)
{
    switch (tile) {
#define FP8_GSUP(i) case i: return true;
        FP8_GROUP_TILES(FP8_GSUP)
#undef FP8_GSUP
    default: return false;
    }
}

hipError_t launch_grouped(int tile, int fa, int fb, const GroupEntry *table, int count, int64_t total_tiles,
                          int *counter, int grid, hipStream_t st)
{
    switch (tile) {
#define FP8_GCASE(i) \
    case i: return TileArgs<i>::go(fa, fb, table, count, total_tiles, counter, grid, st);
        FP8_GROUP_TILES(FP8_GCASE)
#undef FP8_GCASE
    default: return hipErrorInvalidValue;
    }
}

int grouped_max_workgroups(int tile)
{
    switch (tile) {
#define FP8_OCC(i, bm, bn, wm, wn, occ, pf) \
    case i: return occ;
        FP8_TILE_LIST(FP8_OCC)
#undef FP8_OCC
    default: return 1;
    }
}

}  // namespace fp8k

using namespace fp8k;

struct fp8_grouped_plan {
    int tile = 0, fa = 0, fb = 0, count = 0, grid = 0;
    int64_t total_tiles = 0;
    GroupEntry *d_table = nullptr;
    int *d_counter = nullptr;
    int use_graph = 0;
    bool captured = false;
    hipGraphExec_t exec = nullptr;
};

// Dense problem turned weight-major: C^T = W A^T with W = B^T (N x K rows).
static void to_weight_major(Prepared &pr)
{
    GemmParams &p = pr.p;
    std::swap(p.a, p.b);
    std::swap(p.lda, p.ldb);
    std::swap(p.si, p.sj);
    std::swap(p.si_per, p.sj_per);
    std::swap(p.M, p.N);
    std::swap(pr.fa, pr.fb);
    p.trans_out = 1;
}

static int default_group_tile(const std::vector<int64_t> &tokens)
{
    std::vector<int64_t> t = tokens;
    std::sort(t.begin(), t.end());
    const int64_t med = t[t.size() / 2];
    if (med <= 32) return 9;      // 256 weight rows x 32 tokens
    return 19;                    // 256 x 256 on the LDS-DMA pipeline
}

extern "C" {

fp8_status fp8_grouped_plan_create(const fp8_group_problem *problems, int count, int tile, int use_graph,
                                   fp8_grouped_plan **out)
{
    if (!problems || !out || count < 1) return set_error(FP8_ERR_ARG, "null problems/plan or count < 1");
    if (tile >= num_tiles()) return set_error(FP8_ERR_ARG, "tile out of range");
    if (tile >= 0 && !grouped_tile_supported(tile))
        return set_error(FP8_ERR_UNSUPPORTED, "the grouped kernel is not built for tile " + std::to_string(tile));
    std::vector<Prepared> prs((size_t)count);
    std::vector<int64_t> tokens;
    for (int i = 0; i < count; ++i) {
        fp8_status st;
        if (problems[i].is_sparse) {
            st = prepare_sparse(&problems[i].sparse, prs[i]);
            if (st == FP8_OK && problems[i].sparse.side != FP8_SPARSE_B)
                st = set_error(FP8_ERR_UNSUPPORTED, "grouped 2:4 problems take the compressed operand on side B");
            if (st == FP8_OK && problems[i].sparse.g.K % 128)
                st = set_error(FP8_ERR_UNSUPPORTED, "grouped 2:4 problems need K % 128 == 0");
        } else {
            st = prepare_dense(&problems[i].dense, prs[i]);
            if (st == FP8_OK && problems[i].dense.K % 16)
                st = set_error(FP8_ERR_UNSUPPORTED, "grouped dense problems need K % 16 == 0");
            if (st == FP8_OK) to_weight_major(prs[i]);
        }
        if (st != FP8_OK) return set_error(st, "problem " + std::to_string(i) + ": " + fp8_last_error());
        prs[i].p.splits = 1;
        prs[i].p.kchunk = (prs[i].p.K + kBKHost - 1) / kBKHost * kBKHost;
        tokens.push_back(prs[i].p.N);
        if (prs[i].fa != prs[0].fa || prs[i].fb != prs[0].fb)
            return set_error(FP8_ERR_UNSUPPORTED, "all problems of a group must share the operand formats");
    }
    auto *plan = new fp8_grouped_plan();
    plan->tile = tile >= 0 ? tile : default_group_tile(tokens);
    plan->fa = prs[0].fa;
    plan->fb = prs[0].fb;
    plan->count = count;
    plan->use_graph = use_graph;
    const TileDesc &td = tile_desc(plan->tile);
    // longest tiles (largest K) first
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return prs[x].p.K > prs[y].p.K; });
    std::vector<GroupEntry> table((size_t)count);
    int64_t total = 0;
    for (int k = 0; k < count; ++k) {
        const Prepared &pr = prs[order[k]];
        GroupEntry &e = table[k];
        std::memset(&e, 0, sizeof(e));
        e.p = pr.p;
        e.sparse = pr.sparse ? 1 : 0;
        e.tiles_m = (pr.p.M + td.bm - 1) / td.bm;
        e.tiles_n = (pr.p.N + td.bn - 1) / td.bn;
        e.tile_begin = total;
        total += (int64_t)e.tiles_m * e.tiles_n;
    }
    plan->total_tiles = total;
    int cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    plan->grid = (int)std::min<int64_t>(total, (int64_t)cus * grouped_max_workgroups(plan->tile));
    hipError_t e = hipMalloc(&plan->d_table, sizeof(GroupEntry) * (size_t)count);
    if (e == hipSuccess) e = hipMalloc(&plan->d_counter, 64);
    if (e == hipSuccess)
        e = hipMemcpy(plan->d_table, table.data(), sizeof(GroupEntry) * (size_t)count, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        fp8_grouped_plan_destroy(plan);
        return hip_error(e, "grouped plan allocation");
    }
    *out = plan;
    return FP8_OK;
}

fp8_status fp8_grouped_gemm(fp8_grouped_plan *plan, void *stream)
{
    if (!plan) return set_error(FP8_ERR_ARG, "null plan");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!plan->use_graph) {
        hipError_t e = launch_grouped(plan->tile, plan->fa, plan->fb, plan->d_table, plan->count, plan->total_tiles,
                                      plan->d_counter, plan->grid, st);
        return e == hipSuccess ? FP8_OK : hip_error(e, "grouped launch");
    }
    if (!st) return set_error(FP8_ERR_ARG, "graph mode needs a non-null stream");
    if (!plan->captured) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_error(e, "begin capture");
        hipError_t le = launch_grouped(plan->tile, plan->fa, plan->fb, plan->d_table, plan->count, plan->total_tiles,
                                       plan->d_counter, plan->grid, st);
        e = hipStreamEndCapture(st, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_error(le, "grouped launch under capture");
        }
        if (e != hipSuccess) return hip_error(e, "end capture");
        e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_error(e, "graph instantiate");
        plan->captured = true;
    }
    hipError_t e = hipGraphLaunch(plan->exec, st);
    return e == hipSuccess ? FP8_OK : hip_error(e, "graph launch");
}

fp8_status fp8_grouped_plan_info(const fp8_grouped_plan *plan, int *tile, int64_t *num_tiles, int *num_workgroups)
{
    if (!plan) return set_error(FP8_ERR_ARG, "null plan");
    if (tile) *tile = plan->tile;
    if (num_tiles) *num_tiles = plan->total_tiles;
    if (num_workgroups) *num_workgroups = plan->grid;
    return FP8_OK;
}

fp8_status fp8_grouped_plan_destroy(fp8_grouped_plan *plan)
{
    if (!plan) return FP8_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->d_table) (void)hipFree(plan->d_table);
    if (plan->d_counter) (void)hipFree(plan->d_counter);
    delete plan;
    return FP8_OK;
}

}  // extern "C"
