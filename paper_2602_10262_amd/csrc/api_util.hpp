// Host-side helpers behind the C ABI: error text, argument checks, plan
// choice and the tuning cache.
#pragma once
#include <stdint.h>

#include <string>

#include "../../include/fp8gemm.h"
#include "internal.hpp"

namespace fp8k {

fp8_status set_error(fp8_status st, const std::string &msg);
fp8_status hip_error(hipError_t e, const char *what);
void clear_error();

// Everything that identifies a GEMM for plan choice and for the tuning cache.
struct GemmKey {
    int64_t mk, nk, kk;       // kernel-view dimensions: i count, j count, K
    int fa, fb, out_type, si_per, sj_per, sparse;   // out_type: fp8_out
};

// Kernel-view parameters of a dense or sparse call after argument checking.
struct Prepared {
    GemmParams p;
    int fa, fb;
    bool sparse;
    GemmKey key;
};

fp8_status prepare_dense(const fp8_gemm_args *a, Prepared &out);
fp8_status prepare_sparse(const fp8_sparse24_gemm_args *a, Prepared &out);

// Fills in tile and split_k (explicit plan entries are kept when valid).
fp8_status resolve_plan(const Prepared &pr, const fp8_plan *plan, fp8_plan &res);
size_t workspace_bytes(const Prepared &pr, const fp8_plan &res);
fp8_status run_prepared(Prepared pr, const fp8_plan &res, void *ws, size_t ws_bytes, hipStream_t st);
// Sets splits / kchunk in p for a resolved plan.
void apply_split(GemmParams &p, int split_k);

// Tuning cache (process-wide, thread-safe).
bool tune_cache_lookup(const GemmKey &k, fp8_plan &out);
void tune_cache_store(const GemmKey &k, const fp8_plan &plan, double us);

// Default choice without tuning data.
fp8_plan heuristic_plan(const GemmKey &k);

}  // namespace fp8k
