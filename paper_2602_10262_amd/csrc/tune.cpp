// Autotuner: times candidate plans for a GEMM with HIP events and keeps the
// fastest in a process-wide cache; compares the best dense and the best 2:4
// plan of one product and records which wins (the break-even of Sec. 7.1 of
// the paper, per shape); picks the fastest tile of a grouped problem set.
//
// Plan cache key: the kernel-view shape with M and N rounded up to powers of
// two, formats, output type, scale kinds and the dense / sparse side.
// Break-even key: the caller-view M (rounded up to a power of two), N, K,
// the sparse side, formats and output type.  Both persist as JSON lines;
// every line names the device (architecture and product name) and the HIP
// runtime version it was measured with, and lines measured elsewhere are
// skipped when a cache is loaded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "api_util.hpp"

namespace fp8k {

namespace {

using KeyT = std::tuple<int64_t, int64_t, int64_t, int, int, int, int, int, int>;
using BeKeyT = std::tuple<int64_t, int64_t, int64_t, int, int, int, int>;

struct Entry {
    fp8_plan plan;
    double us;
};

std::mutex g_mu;
std::map<KeyT, Entry> g_cache;
std::map<BeKeyT, fp8_breakeven> g_breakeven;

int64_t pow2_ceil(int64_t v)
{
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

KeyT make_key(const GemmKey &k)
{
    return KeyT{pow2_ceil(k.mk), pow2_ceil(k.nk), k.kk, k.fa, k.fb, k.out_type, k.si_per, k.sj_per, k.sparse};
}

BeKeyT make_be_key(int64_t M, int64_t N, int64_t K, int side, int fa, int fb, int out_type)
{
    return BeKeyT{pow2_ceil(M), N, K, side, fa, fb, out_type};
}

// Identity of the current device and runtime: "<arch> <product>" and the HIP
// runtime version ("none" and 0 without a device).
void device_identity(std::string &dev, int &runtime)
{
    dev = "none";
    runtime = 0;
    int d = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&d) != hipSuccess || hipGetDeviceProperties(&prop, d) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    dev = std::string(prop.gcnArchName) + " " + prop.name;
    for (char &c : dev)
        if (c == '"' || c == '\\' || c == '\n') c = '_';
    if (hipRuntimeGetVersion(&runtime) != hipSuccess) runtime = 0;
}

// Flat JSON object reader: "key": number | "string" pairs only.
bool parse_flat_json(const char *line, std::map<std::string, std::string> &kv)
{
    const char *p = std::strchr(line, '{');
    if (!p) return false;
    ++p;
    while (*p) {
        while (*p == ' ' || *p == ',' || *p == '\t') ++p;
        if (*p == '}') return true;
        if (*p != '"') return false;
        const char *ke = std::strchr(p + 1, '"');
        if (!ke) return false;
        std::string key(p + 1, ke);
        p = ke + 1;
        while (*p == ' ' || *p == ':') ++p;
        std::string val;
        if (*p == '"') {
            const char *ve = std::strchr(p + 1, '"');
            if (!ve) return false;
            val.assign(p + 1, ve);
            p = ve + 1;
        } else {
            const char *s = p;
            while (*p && *p != ',' && *p != '}' && *p != ' ') ++p;
            val.assign(s, p);
        }
        kv[key] = val;
    }
    return false;
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

// Median time in microseconds of `iters` calls of fn on st (after two warm-up
// calls).  With `flush`, flush_bytes of it are rewritten before every timed
// call, outside the timed interval, so that operands small enough to stay in
// the 256 MB memory-side cache are read from HBM again, as a stream of
// distinct problems would read them.
template <typename F>
static fp8_status time_median(F &&fn, int iters, hipStream_t st, double *us, void *flush = nullptr,
                              size_t flush_bytes = 0)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(FP8_ERR_HIP, "event creation failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(FP8_ERR_HIP, "event creation failed");
    }
    fp8_status s = FP8_OK;
    for (int w = 0; w < 2 && s == FP8_OK; ++w) s = fn();
    std::vector<float> times;
    for (int i = 0; i < iters && s == FP8_OK; ++i) {
        if (flush && hipMemsetAsync(flush, i & 0xff, flush_bytes, st) != hipSuccess) {
            s = set_error(FP8_ERR_HIP, "cache flush before a timed call failed");
            break;
        }
        (void)hipEventRecord(e0, st);
        s = fn();
        (void)hipEventRecord(e1, st);
        if (s != FP8_OK) break;
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        times.push_back(ms);
    }
    (void)hipStreamSynchronize(st);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != FP8_OK) return s;
    std::nth_element(times.begin(), times.begin() + times.size() / 2, times.end());
    *us = 1000.0 * times[times.size() / 2];
    return FP8_OK;
}

static fp8_status tune_prepared(const Prepared &pr, int iters, hipStream_t st, fp8_plan *best, double *best_us)
{
    if (iters < 1) iters = 1;
    std::vector<fp8_plan> cands;
    const int steps = (pr.p.K + kBKHost - 1) / kBKHost;
    for (int t = 0; t < num_tiles(); ++t) {
        const TileDesc &d = tile_desc(t);
        if (pr.sparse && !d.sparse_ok) continue;
        if (!pr.sparse && !d.dense_ok) continue;
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
    if (cands.empty()) return set_error(FP8_ERR_UNSUPPORTED, "no tuning candidate");
    void *ws = nullptr;
    if (ws_max) {
        hipError_t e = hipMalloc(&ws, ws_max);
        if (e != hipSuccess) return hip_error(e, "tuning workspace");
    }
    // operands that fit in the memory-side cache are flushed from it before
    // every timed call (twice its size is rewritten)
    const size_t operand_bytes = (size_t)pr.key.mk * pr.key.kk + (size_t)pr.key.nk * pr.key.kk;
    const size_t flush_bytes = operand_bytes < ((size_t)512 << 20) ? ((size_t)512 << 20) : 0;
    void *flush = nullptr;
    if (flush_bytes && hipMalloc(&flush, flush_bytes) != hipSuccess) {
        flush = nullptr;             // tune without it
        (void)hipGetLastError();     // and do not leave the failure for a later launch check
    }
    double best_t = 1e30;
    fp8_plan best_p = cands[0];
    fp8_status status = FP8_OK;
    for (auto &c : cands) {
        double us = 0;
        status = time_median([&]() { return run_prepared(pr, c, ws, ws_max, st); }, iters, st, &us, flush,
                             flush ? flush_bytes : 0);
        if (status != FP8_OK) break;
        if (us < best_t) {
            best_t = us;
            best_p = c;
        }
    }
    if (flush) (void)hipFree(flush);
    if (ws) (void)hipFree(ws);
    if (status != FP8_OK) return status;
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

fp8_status fp8_tune_sparse_vs_dense(const fp8_sparse24_gemm_args *sparse, const fp8_gemm_args *dense, int iters,
                                    void *stream, fp8_breakeven *out)
{
    if (!sparse || !dense) return set_error(FP8_ERR_ARG, "null arguments");
    const fp8_gemm_args &g = sparse->g;
    if (g.M != dense->M || g.N != dense->N || g.K != dense->K || g.a_fmt != dense->a_fmt ||
        g.b_fmt != dense->b_fmt || g.c_type != dense->c_type)
        return set_error(FP8_ERR_ARG, "the dense and 2:4 descriptions are not the same product");
    Prepared ps, pd;
    fp8_status st = prepare_sparse(sparse, ps);
    if (st == FP8_OK) st = prepare_dense(dense, pd);
    if (st != FP8_OK) return st;
    fp8_breakeven r{};
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = tune_prepared(pd, iters, s, &r.dense_plan, &r.dense_us);
    if (st == FP8_OK) st = tune_prepared(ps, iters, s, &r.sparse_plan, &r.sparse_us);
    if (st != FP8_OK) return st;
    r.M = g.M; r.N = g.N; r.K = g.K;
    r.side = sparse->side;
    r.a_fmt = g.a_fmt; r.b_fmt = g.b_fmt; r.c_type = g.c_type;
    r.use_sparse = r.sparse_us < r.dense_us ? 1 : 0;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_breakeven[make_be_key(r.M, r.N, r.K, r.side, r.a_fmt, r.b_fmt, r.c_type)] = r;
    }
    if (out) *out = r;
    return FP8_OK;
}

fp8_status fp8_tune_breakeven_lookup(int64_t M, int64_t N, int64_t K, fp8_sparse_side side, fp8_fmt a_fmt,
                                     fp8_fmt b_fmt, fp8_out c_type, fp8_breakeven *out, int *found)
{
    if (!out || !found) return set_error(FP8_ERR_ARG, "null output");
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_breakeven.find(make_be_key(M, N, K, side, a_fmt, b_fmt, c_type));
    *found = it != g_breakeven.end();
    if (*found) *out = it->second;
    return FP8_OK;
}

int fp8_tune_breakeven_count(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_breakeven.size();
}

fp8_status fp8_tune_breakeven_get(int index, fp8_breakeven *out)
{
    if (!out) return set_error(FP8_ERR_ARG, "null output");
    std::lock_guard<std::mutex> lk(g_mu);
    if (index < 0 || index >= (int)g_breakeven.size()) return set_error(FP8_ERR_ARG, "index out of range");
    auto it = g_breakeven.begin();
    std::advance(it, index);
    *out = it->second;
    return FP8_OK;
}

fp8_status fp8_tune_device_key(char *buf, size_t bytes, int *runtime_version)
{
    std::string dev;
    int rt = 0;
    device_identity(dev, rt);
    if (buf && bytes) {
        std::snprintf(buf, bytes, "%s", dev.c_str());
    }
    if (runtime_version) *runtime_version = rt;
    return FP8_OK;
}

fp8_status fp8_tune_cache_save(const char *path)
{
    if (!path) return set_error(FP8_ERR_ARG, "null path");
    std::string dev;
    int rt = 0;
    device_identity(dev, rt);
    FILE *f = std::fopen(path, "w");
    if (!f) return set_error(FP8_ERR_ARG, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_cache) {
        const KeyT &k = kv.first;
        std::fprintf(f,
                     "{\"kind\": \"plan\", \"device\": \"%s\", \"runtime\": %d, \"mk\": %lld, \"nk\": %lld, "
                     "\"kk\": %lld, \"fa\": %d, \"fb\": %d, \"out_type\": %d, \"si_per\": %d, \"sj_per\": %d, "
                     "\"sparse\": %d, \"tile\": %d, \"split_k\": %d, \"us\": %.3f}\n",
                     dev.c_str(), rt, (long long)std::get<0>(k), (long long)std::get<1>(k), (long long)std::get<2>(k),
                     std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), std::get<8>(k),
                     kv.second.plan.tile, kv.second.plan.split_k, kv.second.us);
    }
    for (auto &kv : g_breakeven) {
        const fp8_breakeven &r = kv.second;
        std::fprintf(f,
                     "{\"kind\": \"breakeven\", \"device\": \"%s\", \"runtime\": %d, \"M\": %lld, \"N\": %lld, "
                     "\"K\": %lld, \"side\": %d, \"fa\": %d, \"fb\": %d, \"c_type\": %d, \"dense_us\": %.3f, "
                     "\"sparse_us\": %.3f, \"dense_tile\": %d, \"dense_split\": %d, \"sparse_tile\": %d, "
                     "\"sparse_split\": %d, \"use_sparse\": %d}\n",
                     dev.c_str(), rt, (long long)r.M, (long long)r.N, (long long)r.K, r.side, r.a_fmt, r.b_fmt,
                     r.c_type, r.dense_us, r.sparse_us, r.dense_plan.tile, r.dense_plan.split_k, r.sparse_plan.tile,
                     r.sparse_plan.split_k, r.use_sparse);
    }
    std::fclose(f);
    return FP8_OK;
}

fp8_status fp8_tune_cache_load(const char *path)
{
    if (!path) return set_error(FP8_ERR_ARG, "null path");
    std::string dev;
    int rt = 0;
    device_identity(dev, rt);
    FILE *f = std::fopen(path, "r");
    if (!f) return set_error(FP8_ERR_ARG, std::string("cannot read ") + path);
    char line[1024];
    auto num = [](const std::map<std::string, std::string> &kv, const char *k, bool &ok) -> long long {
        auto it = kv.find(k);
        if (it == kv.end()) {
            ok = false;
            return 0;
        }
        return std::atoll(it->second.c_str());
    };
    auto real = [](const std::map<std::string, std::string> &kv, const char *k, bool &ok) -> double {
        auto it = kv.find(k);
        if (it == kv.end()) {
            ok = false;
            return 0;
        }
        return std::atof(it->second.c_str());
    };
    while (std::fgets(line, sizeof line, f)) {
        std::map<std::string, std::string> kv;
        if (!parse_flat_json(line, kv)) continue;
        // measured on this device and runtime only
        auto d = kv.find("device");
        bool ok = true;
        if (d == kv.end() || d->second != dev || num(kv, "runtime", ok) != rt || !ok) continue;
        const std::string kind = kv.count("kind") ? kv["kind"] : "";
        if (kind == "plan") {
            const KeyT key{num(kv, "mk", ok), num(kv, "nk", ok), num(kv, "kk", ok), (int)num(kv, "fa", ok),
                           (int)num(kv, "fb", ok), (int)num(kv, "out_type", ok), (int)num(kv, "si_per", ok),
                           (int)num(kv, "sj_per", ok), (int)num(kv, "sparse", ok)};
            const int tile = (int)num(kv, "tile", ok), split = (int)num(kv, "split_k", ok);
            const double us = real(kv, "us", ok);
            if (!ok || tile < 0 || tile >= num_tiles() || split < 1) continue;
            const bool sp = std::get<8>(key) != 0;
            if (sp && !tile_desc(tile).sparse_ok) continue;
            if (!sp && !tile_desc(tile).dense_ok) continue;
            std::lock_guard<std::mutex> lk(g_mu);
            g_cache[key] = Entry{fp8_plan{tile, split}, us};
        } else if (kind == "breakeven") {
            fp8_breakeven r{};
            r.M = num(kv, "M", ok); r.N = num(kv, "N", ok); r.K = num(kv, "K", ok);
            r.side = (int)num(kv, "side", ok);
            r.a_fmt = (int)num(kv, "fa", ok); r.b_fmt = (int)num(kv, "fb", ok); r.c_type = (int)num(kv, "c_type", ok);
            r.dense_us = real(kv, "dense_us", ok); r.sparse_us = real(kv, "sparse_us", ok);
            r.dense_plan = fp8_plan{(int)num(kv, "dense_tile", ok), (int)num(kv, "dense_split", ok)};
            r.sparse_plan = fp8_plan{(int)num(kv, "sparse_tile", ok), (int)num(kv, "sparse_split", ok)};
            r.use_sparse = (int)num(kv, "use_sparse", ok);
            if (!ok) continue;
            std::lock_guard<std::mutex> lk(g_mu);
            g_breakeven[make_be_key(r.M, r.N, r.K, r.side, r.a_fmt, r.b_fmt, r.c_type)] = r;
        }
    }
    std::fclose(f);
    return FP8_OK;
}

void fp8_tune_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear();
    g_breakeven.clear();
}

}  // extern "C"
