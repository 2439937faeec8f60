// Mixed-precision GEMM sequences and their co-scheduling on streams (the
// mixed-precision workload of Sec. 8.3 and the scheduling guidance of
// Sec. 9.2: co-schedule kernels of similar wavefront needs, co-locate
// memory-bound FP8 work with compute-bound FP32 work).
//
// A chain is a sequence of GEMM stages Y_s = X_s W_s^T of width M, each in
// its own precision (FP32, FP16, BF16 or FP8).  Stage s writes its result
// directly in the input type of stage s + 1 (the GEMM epilogue converts);
// an FP8 stage takes FP32 input and quantizes it per row (E4M3) before its
// GEMM.  Several independent chains share the weights and run under one of
// three schedules:
//   SERIAL     one stream, chain after chain;
//   IN_PHASE   chain c on stream c % S, every stream starting at once, so
//              the stages that run together have the same precision;
//   STAGGERED  as IN_PHASE, but stream k starts when stream k - 1 has
//              finished its first stage, so neighbouring streams run
//              different precisions side by side.
// Every stage is bracketed by events on its stream: its time is the span in
// which its kernels ran, contention included.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "api_util.hpp"

namespace fp8k {

struct ChainBuffers {
    std::vector<void *> x;        // input of stage s (type of stage s; FP8 stage: FP32)
    void *y = nullptr;            // output of the last stage (FP32)
    uint8_t *q = nullptr;         // FP8 codes of an FP8 stage's input (largest M x K)
    float *qs = nullptr, *qd = nullptr;   // its per-row scales and descales
    void *ws = nullptr;           // split-K workspace of the FP8 GEMMs
    size_t ws_bytes = 0;
};

}  // namespace fp8k

struct fp8_chain {
    std::vector<fp8_chain_stage> stages;
    std::vector<int64_t> kdim;    // K of stage s
    int64_t M = 0;
    int n_chains = 0;
    std::vector<fp8k::ChainBuffers> buf;
    float *ones = nullptr;        // unit scales of the non-FP8 stages
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> ev;   // [chain][stage][begin, end]
    hipEvent_t start = nullptr;
    std::vector<hipEvent_t> stream_end;
    std::vector<hipEvent_t> first_done;   // per stream: end of its first stage
};

namespace fp8k {

static int elem_bytes(int prec) { return prec == FP8_STAGE_F32 || prec == FP8_STAGE_FP8 ? 4 : 2; }

static fp8_out out_for(int next_prec)
{
    switch (next_prec) {
    case FP8_STAGE_F16: return FP8_OUT_F16;
    case FP8_STAGE_BF16: return FP8_OUT_BF16;
    default: return FP8_OUT_F32;   // FP32 stage, FP8 stage (quantizes FP32) or the chain's output
    }
}

static void free_chain(fp8_chain *c)
{
    for (auto &b : c->buf) {
        for (void *p : b.x) (void)hipFree(p);
        (void)hipFree(b.y);
        (void)hipFree(b.q);
        (void)hipFree(b.qs);
        (void)hipFree(b.qd);
        (void)hipFree(b.ws);
    }
    (void)hipFree(c->ones);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->stream_end) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->first_done) (void)hipEventDestroy(e);
    if (c->start) (void)hipEventDestroy(c->start);
    for (hipStream_t s : c->streams) (void)hipStreamDestroy(s);
    delete c;
}

static fp8_gemm_args fp8_stage_args(const fp8_chain *c, int ch, int s, void *out)
{
    const ChainBuffers &b = c->buf[ch];
    const fp8_chain_stage &st = c->stages[s];
    fp8_gemm_args g;
    std::memset(&g, 0, sizeof(g));
    g.M = c->M; g.N = st.N; g.K = c->kdim[s];
    g.a = b.q; g.a_fmt = FP8_E4M3; g.lda = c->kdim[s];
    g.b = static_cast<const uint8_t *>(st.w); g.b_fmt = FP8_E4M3; g.ldb = c->kdim[s];
    g.a_descale = b.qd; g.a_kind = FP8_SCALE_ROW;
    g.b_descale = st.w_scale ? st.w_scale : c->ones; g.b_kind = st.w_scale ? FP8_SCALE_ROW : FP8_SCALE_TENSOR;
    g.c = out;
    g.c_type = out_for(s + 1 < (int)c->stages.size() ? c->stages[s + 1].precision : FP8_STAGE_F32);
    g.ldc = st.N;
    return g;
}

// Enqueues stage s of chain ch on stream st (bracketed by its events).
static fp8_status run_stage(fp8_chain *c, int ch, int s, hipStream_t st)
{
    ChainBuffers &b = c->buf[ch];
    const fp8_chain_stage &sg = c->stages[s];
    const int last = s + 1 == (int)c->stages.size();
    void *out = last ? b.y : b.x[s + 1];
    hipEvent_t *e = &c->ev[((size_t)ch * c->stages.size() + s) * 2];
    (void)hipEventRecord(e[0], st);
    fp8_status r;
    if (sg.precision == FP8_STAGE_FP8) {
        r = fp8_quantize(static_cast<const float *>(b.x[s]), c->M, c->kdim[s], c->kdim[s], FP8_E4M3, FP8_SCALE_ROW,
                         b.q, c->kdim[s], b.qs, b.qd, nullptr, 0, st);
        if (r != FP8_OK) return r;
        fp8_gemm_args g = fp8_stage_args(c, ch, s, out);
        r = fp8_gemm(&g, nullptr, b.ws, b.ws_bytes, st);
    } else {
        fp8_hp_gemm_args g;
        std::memset(&g, 0, sizeof(g));
        g.M = c->M; g.N = sg.N; g.K = c->kdim[s];
        g.a = b.x[s]; g.lda = c->kdim[s];
        g.b = sg.w; g.ldb = c->kdim[s];
        g.ab_type = sg.precision == FP8_STAGE_F32 ? FP8_HP_F32 : (sg.precision == FP8_STAGE_F16 ? FP8_HP_F16 : FP8_HP_BF16);
        g.a_scale = c->ones; g.a_kind = FP8_SCALE_TENSOR;
        g.b_scale = sg.w_scale ? sg.w_scale : c->ones; g.b_kind = sg.w_scale ? FP8_SCALE_ROW : FP8_SCALE_TENSOR;
        g.c = out;
        g.c_type = out_for(last ? FP8_STAGE_F32 : c->stages[s + 1].precision);
        g.ldc = sg.N;
        r = fp8_hp_gemm(&g, st);
    }
    if (r != FP8_OK) return r;
    (void)hipEventRecord(e[1], st);
    return FP8_OK;
}

}  // namespace fp8k

using namespace fp8k;

extern "C" {

fp8_status fp8_chain_create(const fp8_chain_stage *stages, int n_stages, int64_t M, int64_t in_width, int n_chains,
                            int max_streams, fp8_chain **out)
{
    if (!stages || !out || n_stages < 1 || n_stages > 16) return set_error(FP8_ERR_ARG, "1..16 stages required");
    if (M < 1 || in_width < 1 || n_chains < 1 || n_chains > 64) return set_error(FP8_ERR_SHAPE, "bad M, width or chain count");
    if (max_streams < 1 || max_streams > 8) return set_error(FP8_ERR_ARG, "max_streams must be 1..8");
    int64_t k = in_width;
    for (int s = 0; s < n_stages; ++s) {
        const fp8_chain_stage &sg = stages[s];
        if (sg.precision < FP8_STAGE_F32 || sg.precision > FP8_STAGE_FP8) return set_error(FP8_ERR_ARG, "unknown stage precision");
        if (sg.N < 1 || !sg.w) return set_error(FP8_ERR_ARG, "stage needs N >= 1 and a weight");
        // 16-byte row strides for every operand of the stage
        if ((k * elem_bytes(sg.precision)) % 16 || (sg.precision == FP8_STAGE_FP8 && k % 16))
            return set_error(FP8_ERR_ALIGN, "stage widths must give 16-byte rows");
        k = sg.N;
    }
    fp8_chain *c = new fp8_chain();
    c->stages.assign(stages, stages + n_stages);
    c->M = M;
    c->n_chains = n_chains;
    k = in_width;
    for (int s = 0; s < n_stages; ++s) {
        c->kdim.push_back(k);
        k = stages[s].N;
    }
    auto fail = [&](hipError_t e, const char *what) {
        free_chain(c);
        return hip_error(e, what);
    };
    hipError_t e = hipMalloc(&c->ones, 16);
    if (e != hipSuccess) return fail(e, "chain scales");
    const float one[4] = {1.f, 1.f, 1.f, 1.f};
    e = hipMemcpy(c->ones, one, sizeof(one), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(e, "chain scales");
    int64_t max_fp8_k = 0;
    for (int s = 0; s < n_stages; ++s)
        if (stages[s].precision == FP8_STAGE_FP8) max_fp8_k = std::max(max_fp8_k, c->kdim[s]);
    c->buf.resize(n_chains);
    for (int ch = 0; ch < n_chains; ++ch) {
        ChainBuffers &b = c->buf[ch];
        for (int s = 0; s < n_stages; ++s) {
            void *p = nullptr;
            e = hipMalloc(&p, (size_t)M * c->kdim[s] * elem_bytes(stages[s].precision));
            if (e != hipSuccess) return fail(e, "chain activations");
            b.x.push_back(p);
        }
        e = hipMalloc(&b.y, (size_t)M * stages[n_stages - 1].N * 4);
        if (e != hipSuccess) return fail(e, "chain output");
        if (max_fp8_k > 0) {
            if ((e = hipMalloc(&b.q, (size_t)M * max_fp8_k)) != hipSuccess ||
                (e = hipMalloc(&b.qs, (size_t)M * 4)) != hipSuccess || (e = hipMalloc(&b.qd, (size_t)M * 4)) != hipSuccess)
                return fail(e, "chain FP8 staging");
            size_t need = 0;
            for (int s = 0; s < n_stages; ++s) {
                if (stages[s].precision != FP8_STAGE_FP8) continue;
                fp8_gemm_args g = fp8_stage_args(c, ch, s, b.x[0]);
                size_t bytes = 0;
                fp8_status r = fp8_gemm_workspace_size(&g, nullptr, &bytes);
                if (r != FP8_OK) {
                    free_chain(c);
                    return r;
                }
                need = std::max(need, bytes);
            }
            if (need > 0) {
                if ((e = hipMalloc(&b.ws, need)) != hipSuccess) return fail(e, "chain workspace");
                b.ws_bytes = need;
            }
        }
    }
    c->streams.resize(max_streams);
    c->stream_end.resize(max_streams);
    c->first_done.resize(max_streams);
    for (int i = 0; i < max_streams; ++i) {
        if ((e = hipStreamCreateWithFlags(&c->streams[i], hipStreamNonBlocking)) != hipSuccess) return fail(e, "chain streams");
        if ((e = hipEventCreate(&c->stream_end[i])) != hipSuccess || (e = hipEventCreate(&c->first_done[i])) != hipSuccess)
            return fail(e, "chain events");
    }
    c->ev.resize((size_t)n_chains * n_stages * 2);
    for (auto &ev : c->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) return fail(e, "chain events");
    if ((e = hipEventCreate(&c->start)) != hipSuccess) return fail(e, "chain events");
    *out = c;
    return FP8_OK;
}

fp8_status fp8_chain_buffer(fp8_chain *c, int chain, int stage, void **ptr, int64_t *ld)
{
    if (!c || !ptr) return set_error(FP8_ERR_ARG, "null argument");
    if (chain < 0 || chain >= c->n_chains || stage < 0 || stage > (int)c->stages.size())
        return set_error(FP8_ERR_ARG, "chain or stage out of range");
    if (stage == (int)c->stages.size()) {
        *ptr = c->buf[chain].y;
        if (ld) *ld = c->stages.back().N;
    } else {
        *ptr = c->buf[chain].x[stage];
        if (ld) *ld = c->kdim[stage];
    }
    return FP8_OK;
}

fp8_status fp8_chain_run(fp8_chain *c, int mode, int n_streams, fp8_chain_stats *stats)
{
    if (!c) return set_error(FP8_ERR_ARG, "null chain");
    if (mode < FP8_CHAIN_SERIAL || mode > FP8_CHAIN_STAGGERED) return set_error(FP8_ERR_ARG, "unknown schedule");
    if (n_streams < 1 || n_streams > (int)c->streams.size()) return set_error(FP8_ERR_ARG, "n_streams out of range");
    const int S = mode == FP8_CHAIN_SERIAL ? 1 : n_streams;
    const int ns = (int)c->stages.size();
    hipError_t e = hipDeviceSynchronize();   // the caller's inputs are complete
    if (e != hipSuccess) return hip_error(e, "chain start");
    (void)hipEventRecord(c->start, c->streams[0]);
    for (int k = 1; k < S; ++k) (void)hipStreamWaitEvent(c->streams[k], c->start, 0);
    // chains of stream k, in order
    std::vector<std::vector<int>> per(S);
    for (int ch = 0; ch < c->n_chains; ++ch) per[ch % S].push_back(ch);
    // issue stage by stage across streams so the queues fill evenly
    std::vector<size_t> pos(S, 0);
    std::vector<int> stage_of(S, 0);
    bool more = true;
    bool first_recorded[8] = {false, false, false, false, false, false, false, false};
    while (more) {
        more = false;
        for (int k = 0; k < S; ++k) {
            if (pos[k] >= per[k].size()) continue;
            more = true;
            const int ch = per[k][pos[k]];
            const int s = stage_of[k];
            if (mode == FP8_CHAIN_STAGGERED && k > 0 && pos[k] == 0 && s == 0)
                (void)hipStreamWaitEvent(c->streams[k], c->first_done[k - 1], 0);
            fp8_status r = run_stage(c, ch, s, c->streams[k]);
            if (r != FP8_OK) {
                (void)hipDeviceSynchronize();
                return r;
            }
            if (!first_recorded[k]) {
                (void)hipEventRecord(c->first_done[k], c->streams[k]);
                first_recorded[k] = true;
            }
            if (++stage_of[k] == ns) {
                stage_of[k] = 0;
                ++pos[k];
            }
        }
    }
    for (int k = 0; k < S; ++k) (void)hipEventRecord(c->stream_end[k], c->streams[k]);
    for (int k = 0; k < S; ++k)
        if ((e = hipEventSynchronize(c->stream_end[k])) != hipSuccess) return hip_error(e, "chain run");
    if (!stats) return FP8_OK;
    std::memset(stats, 0, sizeof(*stats));
    float mk = 0;
    for (int k = 0; k < S; ++k) {
        float t = 0;
        (void)hipEventElapsedTime(&t, c->start, c->stream_end[k]);
        mk = std::max(mk, t);
    }
    stats->makespan_ms = mk;
    double sum[4] = {0, 0, 0, 0}, sq[4] = {0, 0, 0, 0}, flops = 0;
    for (int ch = 0; ch < c->n_chains; ++ch)
        for (int s = 0; s < ns; ++s) {
            float t = 0;
            hipEvent_t *ev = &c->ev[((size_t)ch * ns + s) * 2];
            (void)hipEventElapsedTime(&t, ev[0], ev[1]);
            const int p = c->stages[s].precision;
            sum[p] += t;
            sq[p] += (double)t * t;
            stats->stage_count[p] += 1;
            flops += 2.0 * (double)c->M * (double)c->stages[s].N * (double)c->kdim[s];
        }
    for (int p = 0; p < 4; ++p) {
        const int n = stats->stage_count[p];
        if (n == 0) continue;
        const double mean = sum[p] / n;
        stats->stage_ms_mean[p] = mean;
        const double var = std::max(0.0, sq[p] / n - mean * mean);
        stats->stage_ms_cv[p] = mean > 0 ? std::sqrt(var) / mean : 0.0;
    }
    stats->tflops = mk > 0 ? flops / (mk * 1e-3) / 1e12 : 0.0;
    return FP8_OK;
}

fp8_status fp8_chain_stage_ms(fp8_chain *c, int chain, int stage, double *ms)
{
    if (!c || !ms || chain < 0 || chain >= c->n_chains || stage < 0 || stage >= (int)c->stages.size())
        return set_error(FP8_ERR_ARG, "bad arguments");
    float t = 0;
    hipEvent_t *ev = &c->ev[((size_t)chain * c->stages.size() + stage) * 2];
    hipError_t e = hipEventElapsedTime(&t, ev[0], ev[1]);
    if (e != hipSuccess) return hip_error(e, "stage time");
    *ms = t;
    return FP8_OK;
}

fp8_status fp8_chain_destroy(fp8_chain *c)
{
    if (!c) return FP8_OK;
    (void)hipDeviceSynchronize();
    free_chain(c);
    return FP8_OK;
}

}  // extern "C"
