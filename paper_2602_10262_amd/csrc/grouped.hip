// Grouped FP8 GEMM: many independent dense and 2:4 problems run by
// persistent launches, the batched form of a transformer-style sequence of
// FP8 GEMMs.  This file holds the plan (problem tables, tile choice, HIP
// graph) and the launch sequence; the kernels are in grouped_kernel.hpp.
//
// Work lists: dense and 2:4 problems form lists of their own, and so do the
// problems with K below kExactBelowK, which run on the exact-sum tile (FP8
// decoded to BF16) so that their results meet the accuracy bound whatever
// the data; each list is ordered by K, longest first.  A grouped call clears
// the work counters with one small kernel (so that a captured graph holds no
// memset node) and launches each non-empty list's persistent kernel in turn
// on the caller's stream.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "api_util.hpp"
#include "grouped_kernel.hpp"

namespace fp8k {

__global__ void grouped_reset(unsigned long long *counters, int n)
{
    if ((int)threadIdx.x < n) counters[threadIdx.x * 8] = 0ull;
}

bool grouped_tile_supported(int tile)
{
    switch (tile) {
#define FP8_GSUP(i) case i: return true;
        FP8_GROUP_TILES(FP8_GSUP)
#undef FP8_GSUP
    default: return false;
    }
}

static hipError_t launch_list(int tile, bool sparse, int fa, int fb, const GroupEntry *table, int count,
                              int64_t total, unsigned long long *counter, int grid, hipStream_t st)
{
    switch (tile) {
#define FP8_GCASE(i)                                                                              \
    case i:                                                                                       \
        return sparse ? grouped_launch_tile<i, true>(fa, fb, table, count, total, counter, grid, st) \
                      : grouped_launch_tile<i, false>(fa, fb, table, count, total, counter, grid, st);
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

// One work list: a contiguous range of the device table, run with one tile.
struct GroupList {
    int first = 0, count = 0, grid = 0, tile = 0;
    int64_t total_tiles = 0;
};

// List index: bit 0 = 2:4 problems, bit 1 = exact-sum tile (K below kExactBelowK).
constexpr int kGroupLists = 4;

struct fp8_grouped_plan {
    int tile = 0, fa = 0, fb = 0, count = 0;
    GroupList list[kGroupLists];
    GroupEntry *d_table = nullptr;        // the lists' entries, list by list
    unsigned long long *d_counters = nullptr;   // one counter per list, 64 bytes apart
    int use_graph = 0;
    bool captured = false;
    hipGraphExec_t exec = nullptr;
};

static hipError_t run_lists(const fp8_grouped_plan *plan, hipStream_t st)
{
    grouped_reset<<<1, 64, 0, st>>>(plan->d_counters, kGroupLists);
    hipError_t e = hipGetLastError();
    for (int k = 0; k < kGroupLists && e == hipSuccess; ++k) {
        const GroupList &l = plan->list[k];
        if (l.count == 0) continue;
        e = launch_list(l.tile, (k & 1) != 0, plan->fa, plan->fb, plan->d_table + l.first, l.count, l.total_tiles,
                        plan->d_counters + 8 * k, l.grid, st);
    }
    return e;
}

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
    auto list_of = [&](const Prepared &pr) { return (pr.sparse ? 1 : 0) + (pr.p.K < kExactBelowK ? 2 : 0); };
    for (int k = 0; k < kGroupLists; ++k) plan->list[k].tile = (k & 2) ? kGroupExactTile : plan->tile;
    // list by list; inside each, longest (largest K) first
    std::vector<int> order((size_t)count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        if (list_of(prs[x]) != list_of(prs[y])) return list_of(prs[x]) < list_of(prs[y]);
        return prs[x].p.K > prs[y].p.K;
    });
    std::vector<GroupEntry> table((size_t)count);
    int cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    for (int k = 0; k < count; ++k) {
        const Prepared &pr = prs[order[k]];
        GroupList &l = plan->list[list_of(pr)];
        const TileDesc &td = tile_desc(l.tile);
        if (l.count == 0) l.first = k;
        GroupEntry &e = table[k];
        std::memset(&e, 0, sizeof(e));
        e.p = pr.p;
        e.sparse = pr.sparse ? 1 : 0;
        e.tiles_m = (pr.p.M + td.bm - 1) / td.bm;
        e.tiles_n = (pr.p.N + td.bn - 1) / td.bn;
        e.tile_begin = l.total_tiles;
        l.total_tiles += (int64_t)e.tiles_m * e.tiles_n;
        l.count++;
    }
    for (GroupList &l : plan->list)
        l.grid = (int)std::min<int64_t>(l.total_tiles, (int64_t)cus * grouped_max_workgroups(l.tile));
    hipError_t e = hipMalloc(&plan->d_table, sizeof(GroupEntry) * (size_t)count);
    if (e == hipSuccess) e = hipMalloc(&plan->d_counters, 64 * kGroupLists);
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
        hipError_t e = run_lists(plan, st);
        return e == hipSuccess ? FP8_OK : hip_error(e, "grouped launch");
    }
    if (!st) return set_error(FP8_ERR_ARG, "graph mode needs a non-null stream");
    if (!plan->captured) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_error(e, "begin capture");
        hipError_t le = run_lists(plan, st);
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
    int64_t tiles = 0;
    int grid = 0;
    for (const GroupList &l : plan->list) {
        tiles += l.total_tiles;
        grid = std::max(grid, l.grid);
    }
    if (num_tiles) *num_tiles = tiles;
    if (num_workgroups) *num_workgroups = grid;
    return FP8_OK;
}

fp8_status fp8_grouped_plan_destroy(fp8_grouped_plan *plan)
{
    if (!plan) return FP8_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->d_table) (void)hipFree(plan->d_table);
    if (plan->d_counters) (void)hipFree(plan->d_counters);
    delete plan;
    return FP8_OK;
}

fp8_status fp8_grouped_tune(const fp8_group_problem *problems, int count, int iters, void *stream, int *best_tile,
                            double *best_us)
{
    if (!best_tile) return set_error(FP8_ERR_ARG, "null best_tile");
    if (iters < 1) iters = 1;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    static const int kTiles[] = {
#define FP8_GT(i) i,
        FP8_GROUP_TILES(FP8_GT)
#undef FP8_GT
    };
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(FP8_ERR_HIP, "event creation failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(FP8_ERR_HIP, "event creation failed");
    }
    double best = 1e30;
    int bt = -1;
    fp8_status status = FP8_OK;
    for (int tile : kTiles) {
        fp8_grouped_plan *plan = nullptr;
        status = fp8_grouped_plan_create(problems, count, tile, 0, &plan);
        if (status != FP8_OK) break;
        std::vector<float> times;
        for (int i = 0; i < iters + 2 && status == FP8_OK; ++i) {
            (void)hipEventRecord(e0, st);
            status = fp8_grouped_gemm(plan, st);
            (void)hipEventRecord(e1, st);
            if (status != FP8_OK) break;
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (i >= 2) times.push_back(ms);
        }
        (void)hipStreamSynchronize(st);
        fp8_grouped_plan_destroy(plan);
        if (status != FP8_OK) break;
        std::nth_element(times.begin(), times.begin() + times.size() / 2, times.end());
        const double us = 1000.0 * times[times.size() / 2];
        if (us < best) {
            best = us;
            bt = tile;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != FP8_OK) return status;
    *best_tile = bt;
    if (best_us) *best_us = best;
    return FP8_OK;
}

}  // extern "C"
