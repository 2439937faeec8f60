// Autotuner: times every (tile, split-K) candidate for a GEMM with HIP events
// and keeps the fastest in a process-wide cache, keyed on the kernel-view
// shape with M and N rounded up to powers of two, formats, output type,
// scale kinds and the dense / sparse side.  The cache persists as JSON lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "api_util.hpp"

namespace fp8k {

namespace {

using KeyT = std::tuple<int64_t, int64_t, int64_t, int, int, int, int, int, int>;

struct Entry {
    fp8_plan plan;
    double us;
};

std::mutex g_mu;
std::map<KeyT, Entry> g_cache;

int64_t pow2_ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

KeyT make_key(const GemmKey &k)
{
    return KeyT{pow2_ceil(k.mk), pow2_ceil(k.nk), k.kk, k.fa, k.fb, k.out_bf16, k.si_per, k.sj_per, k.sparse};
}

}  // namespace

bool tune_cache_lookup(const GemmKey &k, fp8_plan &out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(make_key(k));
    if (it == g_cache.end()) return false;
    out = it->second.plan;
    return true;
}

void tune_cache_store(const GemmKey &k, const fp8_plan &plan, double us)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[make_key(k)] = Entry{plan, us};
}

static fp8_status tune_prepared(const Prepared &pr, int iters, hipStream_t st, fp8_plan *best, double *best_us)
{
    if (iters < 1) iters = 1;
    std::vector<fp8_plan> cands;
    const int steps = (pr.p.K + kBKHost - 1) / kBKHost;
    for (int t = 0; t < num_tiles(); ++t) {
        const TileDesc &d = tile_desc(t);
        if (pr.sparse && !d.sparse_ok) continue;
        // the accumulation class follows K (exact-sum tiles below kExactBelowK)
        if ((d.exact != 0) != (pr.key.kk < kExactBelowK)) continue;
        const int64_t nb = ((pr.key.mk + d.bm - 1) / d.bm) * ((pr.key.nk + d.bn - 1) / d.bn);
        for (int s : {1, 2, 4, 8, 16, 32}) {
            if (s > steps) break;
            if (s > 1 && nb * s > 8192) break;   // already far more workgroups than the GPU holds
            GemmParams p = pr.p;
            apply_split(p, s);
            if (p.splits != s) continue;
            cands.push_back(fp8_plan{t, s});
        }
    }
    size_t ws_max = 0;
    for (auto &c : cands) ws_max = std::max(ws_max, workspace_bytes(pr, c));
    if (ws_max > ((size_t)8 << 30)) {
        // drop candidates whose partial sums would not fit in 8 GiB
        std::vector<fp8_plan> keep;
        for (auto &c : cands)
            if (workspace_bytes(pr, c) <= ((size_t)8 << 30)) keep.push_back(c);
        cands.swap(keep);
        ws_max = 0;
        for (auto &c : cands) ws_max = std::max(ws_max, workspace_bytes(pr, c));
    }
    void *ws = nullptr;
    if (ws_max) {
        hipError_t e = hipMalloc(&ws, ws_max);
        if (e != hipSuccess) return hip_error(e, "tuning workspace");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best_t = 1e30;
    fp8_plan best_p = cands.empty() ? heuristic_plan(pr.key) : cands[0];
    fp8_status status = FP8_OK;
    std::vector<float> times;
    for (auto &c : cands) {
        fp8_status s = FP8_OK;
        for (int w = 0; w < 2 && s == FP8_OK; ++w) s = run_prepared(pr, c, ws, ws_max, st);
        if (s != FP8_OK) { status = s; break; }
        times.clear();
        for (int i = 0; i < iters; ++i) {
            (void)hipEventRecord(e0, st);
            s = run_prepared(pr, c, ws, ws_max, st);
            (void)hipEventRecord(e1, st);
            if (s != FP8_OK) break;
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            times.push_back(ms);
        }
        if (s != FP8_OK) { status = s; break; }
        std::nth_element(times.begin(), times.begin() + times.size() / 2, times.end());
        const double us = 1000.0 * times[times.size() / 2];
        if (us < best_t) {
            best_t = us;
            best_p = c;
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (ws) (void)hipFree(ws);
    if (status != FP8_OK) return status;
    if (cands.empty()) return set_error(FP8_ERR_UNSUPPORTED, "no tuning candidate");
    tune_cache_store(pr.key, best_p, best_t);
    if (best) *best = best_p;
    if (best_us) *best_us = best_t;
    return FP8_OK;
}

}  // namespace fp8k

using namespace fp8k;

extern "C" {

fp8_status fp8_tune_gemm(const fp8_gemm_args *args, int iters, void *stream, fp8_plan *best, double *best_us)
{
    Prepared pr;
    fp8_status st = prepare_dense(args, pr);
    if (st != FP8_OK) return st;
    return tune_prepared(pr, iters, reinterpret_cast<hipStream_t>(stream), best, best_us);
}

fp8_status fp8_tune_sparse24_gemm(const fp8_sparse24_gemm_args *args, int iters, void *stream, fp8_plan *best,
                                  double *best_us)
{
    Prepared pr;
    fp8_status st = prepare_sparse(args, pr);
    if (st != FP8_OK) return st;
    return tune_prepared(pr, iters, reinterpret_cast<hipStream_t>(stream), best, best_us);
}

fp8_status fp8_tune_cache_save(const char *path)
{
    if (!path) return set_error(FP8_ERR_ARG, "null path");
    FILE *f = std::fopen(path, "w");
    if (!f) return set_error(FP8_ERR_ARG, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_cache) {
        const KeyT &k = kv.first;
        std::fprintf(f,
                     "{\"mk\": %lld, \"nk\": %lld, \"kk\": %lld, \"fa\": %d, \"fb\": %d, \"out_bf16\": %d, "
                     "\"si_per\": %d, \"sj_per\": %d, \"sparse\": %d, \"tile\": %d, \"split_k\": %d, \"us\": %.3f}\n",
                     (long long)std::get<0>(k), (long long)std::get<1>(k), (long long)std::get<2>(k), std::get<3>(k),
                     std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k),
                     kv.second.plan.tile, kv.second.plan.split_k, kv.second.us);
    }
    std::fclose(f);
    return FP8_OK;
}

fp8_status fp8_tune_cache_load(const char *path)
{
    if (!path) return set_error(FP8_ERR_ARG, "null path");
    FILE *f = std::fopen(path, "r");
    if (!f) return set_error(FP8_ERR_ARG, std::string("cannot read ") + path);
    char line[512];
    int n = 0;
    while (std::fgets(line, sizeof line, f)) {
        long long mk, nk, kk;
        int fa, fb, ob, si, sj, sp, tile, split;
        double us;
        if (std::sscanf(line,
                        "{\"mk\": %lld, \"nk\": %lld, \"kk\": %lld, \"fa\": %d, \"fb\": %d, \"out_bf16\": %d, "
                        "\"si_per\": %d, \"sj_per\": %d, \"sparse\": %d, \"tile\": %d, \"split_k\": %d, \"us\": %lf}",
                        &mk, &nk, &kk, &fa, &fb, &ob, &si, &sj, &sp, &tile, &split, &us) != 12)
            continue;
        if (tile < 0 || tile >= num_tiles() || split < 1) continue;
        if (sp && !tile_desc(tile).sparse_ok) continue;
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[KeyT{mk, nk, kk, fa, fb, ob, si, sj, sp}] = Entry{fp8_plan{tile, split}, us};
        ++n;
    }
    std::fclose(f);
    return FP8_OK;
}

void fp8_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
}

}  // extern "C"
