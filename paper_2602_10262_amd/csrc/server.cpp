// Serving runtime: a request loop that admits FP8 GEMM requests by device
// memory budget and runs them concurrently on several HIP streams (the
// single-GPU form of the paper's concurrent-stream execution, Sec. 6 and
// Sec. 8.2), with latency percentiles, throughput and per-stream fairness.
//
// Threads: any number of client threads call submit/poll/wait; one scheduler
// thread owns every HIP call.  Its loop retires finished requests (event
// query), then admits pending requests in arrival order while (a) their
// arrival time has passed, (b) fewer than max_inflight are running and (c)
// their transient memory fits in the arena; each admitted request is
// launched on the stream with the fewest requests in flight.  Requests that
// arrive while others run are admitted as soon as memory and a slot free up.
//
// A request quantizes its FP32 activations per row (per token) into arena
// memory and multiplies them with a registered weight (dense, or 2:4 on the
// weight side) into the caller's output.  Its kernel plan depends only on its
// own shape, so its result is the same alone and in any mix.
//
// The executor is an interface: the HIP executor above, or a simulated one
// (virtual durations, no device) used to test the scheduler on a CPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_util.hpp"

namespace fp8k {

namespace {

using Clock = std::chrono::steady_clock;

struct Weight {
    const uint8_t *w = nullptr, *meta = nullptr;
    const float *descale = nullptr;
    int64_t N = 0, K = 0;
    int fmt = 0;
    bool sparse = false;
};

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
public:
    void reset(size_t size) { size_ = size; free_.clear(); free_[0] = size; }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    size_t size_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Job {
    uint64_t ticket = 0;
    fp8_request req{};
    double arrival = 0;       // server clock, seconds
    double admitted = 0;
    size_t bytes = 0, off = 0;
    int stream = -1;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double sim_done = 0;      // simulated executor: completion time
    double flops = 0;
    bool queued = false;      // device work was enqueued (retire through ev1 even on failure)
    fp8_status fail = FP8_OK; // failure to report when such a job retires
};

struct TicketState {
    fp8_status status = FP8_ERR_PENDING;
    double latency_ms = 0;
};

}  // namespace

class Executor {
public:
    virtual ~Executor() = default;
    virtual fp8_status start(Job &job, const Weight &w, uint8_t *arena_base, int stream) = 0;
    virtual bool finished(Job &job, double now) = 0;
    // GPU execution time of a finished job in milliseconds (per-stream accounting)
    virtual double exec_ms(Job &job) = 0;
    virtual void release(Job &job) = 0;
};

class HipExecutor : public Executor {
public:
    explicit HipExecutor(const std::vector<hipStream_t> &s) : streams_(s) {}
    ~HipExecutor() override
    {
        for (auto e : pool_) (void)hipEventDestroy(e);
    }
    fp8_status start(Job &job, const Weight &w, uint8_t *arena, int stream) override
    {
        hipStream_t st = streams_[stream];
        const int64_t M = job.req.M, K = w.K;
        const int64_t ldq = (K + 15) / 16 * 16;
        uint8_t *q = arena + job.off;
        float *s = reinterpret_cast<float *>(q + align(M * ldq));
        float *d = s + align_f(M);
        void *ws = reinterpret_cast<uint8_t *>(d + align_f(M));
        const size_t ws_bytes = job.bytes - (size_t)((uint8_t *)ws - q);
        // Every argument is checked before anything is enqueued: the GEMM's
        // own validation runs through its workspace query on the final
        // arguments, so a request that cannot run leaves no work behind.
        fp8_gemm_args g{};
        g.M = M; g.N = w.N; g.K = K;
        g.a_fmt = job.req.x_fmt; g.b_fmt = (fp8_fmt)w.fmt;
        g.a_descale = d; g.a_kind = FP8_SCALE_ROW;
        g.b_descale = w.descale; g.b_kind = FP8_SCALE_ROW;
        g.c = job.req.c; g.c_type = job.req.c_type; g.ldc = w.N;
        fp8_sparse24_gemm_args sa{};
        size_t need = 0;
        fp8_status r;
        if (w.sparse) {
            sa.g = g;
            sa.g.a = q; sa.g.lda = ldq;
            sa.side = FP8_SPARSE_B;
            sa.values = w.w; sa.meta = w.meta;
            r = fp8_sparse24_gemm_workspace_size(&sa, nullptr, &need);
        } else {
            g.a = q; g.lda = ldq;
            g.b = w.w; g.ldb = w.K;
            r = fp8_gemm_workspace_size(&g, nullptr, &need);
        }
        if (r != FP8_OK) return r;
        if (need > ws_bytes) return set_error(FP8_ERR_ARG, "request workspace exceeds its arena range");
        if (!job.req.x || (reinterpret_cast<uintptr_t>(job.req.x) & 15) || (K % 4))
            return set_error(FP8_ERR_ALIGN, "activations must be 16-byte aligned with K % 4 == 0");
        job.ev0 = take();
        job.ev1 = take();
        if (!job.ev0 || !job.ev1) return set_error(FP8_ERR_HIP, "event creation failed");
        (void)hipEventRecord(job.ev0, st);
        job.queued = true;
        r = fp8_quantize(job.req.x, M, K, K, job.req.x_fmt, FP8_SCALE_ROW, q, ldq, s, d, nullptr, 0, st);
        if (r == FP8_OK) r = w.sparse ? fp8_sparse24_gemm(&sa, nullptr, ws, ws_bytes, st)
                                      : fp8_gemm(&g, nullptr, ws, ws_bytes, st);
        // The completion event is recorded whatever happened above, so a job
        // whose later launch failed is retired (and its arena range reused)
        // only after the work already queued for it has finished.
        hipError_t e = hipEventRecord(job.ev1, st);
        if (r != FP8_OK) return set_error(r, std::string("request launch failed after queueing: ") + fp8_last_error());
        return e == hipSuccess ? FP8_OK : hip_error(e, "event record");
    }
    bool finished(Job &job, double) override { return hipEventQuery(job.ev1) == hipSuccess; }
    double exec_ms(Job &job) override
    {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, job.ev0, job.ev1);
        return ms;
    }
    void release(Job &job) override
    {
        if (job.ev0) pool_.push_back(job.ev0);
        if (job.ev1) pool_.push_back(job.ev1);
        job.ev0 = job.ev1 = nullptr;
    }
    static int64_t align(int64_t b) { return (b + 255) / 256 * 256; }
    static int64_t align_f(int64_t n) { return (n + 63) / 64 * 64; }

private:
    hipEvent_t take()
    {
        if (!pool_.empty()) {
            hipEvent_t e = pool_.back();
            pool_.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    std::vector<hipStream_t> streams_;
    std::vector<hipEvent_t> pool_;
};

// Test double: a job occupies its stream for launch_us + flops / rate; jobs
// on one stream run one after another; nothing touches a device.
class SimExecutor : public Executor {
public:
    SimExecutor(int nstreams, double gflops_per_ms, double launch_us)
        : busy_until_((size_t)nstreams, 0.0), rate_(gflops_per_ms), launch_us_(launch_us)
    {
    }
    fp8_status start(Job &job, const Weight &, uint8_t *, int stream) override
    {
        const double begin = std::max(job.admitted, busy_until_[stream]);
        const double dur = launch_us_ * 1e-6 + job.flops / (rate_ * 1e9) * 1e-3;
        job.sim_done = begin + dur;
        busy_until_[stream] = job.sim_done;
        exec_[job.ticket] = dur * 1e3;
        return FP8_OK;
    }
    bool finished(Job &job, double now) override { return now >= job.sim_done; }
    double exec_ms(Job &job) override { return exec_[job.ticket]; }
    void release(Job &job) override { exec_.erase(job.ticket); }

private:
    std::vector<double> busy_until_;
    double rate_, launch_us_;
    std::unordered_map<uint64_t, double> exec_;
};

}  // namespace fp8k

using namespace fp8k;

struct fp8_server {
    fp8_server_config cfg{};
    bool simulated = false;
    int device = 0;
    std::vector<hipStream_t> streams;
    std::unique_ptr<Executor> exec;
    uint8_t *arena_base = nullptr;
    Arena arena;
    std::vector<Weight> weights;

    std::mutex mu;
    std::condition_variable cv_done, cv_work;
    std::deque<Job> pending;
    std::vector<Job> inflight;
    std::unordered_map<uint64_t, TicketState> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread thread;
    Clock::time_point t0;

    // statistics since the last reset
    std::vector<double> latencies_ms;
    std::vector<double> stream_ms;
    double flops = 0, first_arrival = -1, last_done = 0;
    uint64_t done = 0, failed = 0, rejected = 0, peak_inflight = 0;
    size_t peak_bytes = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

size_t job_bytes(const fp8_server *s, const fp8_request &r, const Weight &w)
{
    const int64_t M = r.M, K = w.K;
    const int64_t ldq = (K + 15) / 16 * 16;
    size_t bytes = (size_t)HipExecutor::align(M * ldq) + 2 * sizeof(float) * (size_t)HipExecutor::align_f(M);
    if (!s->simulated) {
        // split-K workspace of the plan the GEMM will pick for this shape
        fp8_gemm_args g{};
        g.M = M; g.N = w.N; g.K = K;
        g.a_fmt = r.x_fmt; g.b_fmt = (fp8_fmt)w.fmt;
        g.a = reinterpret_cast<const uint8_t *>(256); g.lda = ldq;
        g.b = reinterpret_cast<const uint8_t *>(256); g.ldb = ldq;
        g.a_descale = reinterpret_cast<const float *>(256); g.a_kind = FP8_SCALE_ROW;
        g.b_descale = reinterpret_cast<const float *>(256); g.b_kind = FP8_SCALE_ROW;
        g.c = reinterpret_cast<void *>(256); g.c_type = r.c_type; g.ldc = w.N;
        size_t ws = 0;
        if (w.sparse) {
            fp8_sparse24_gemm_args sa{};
            sa.g = g;
            sa.side = FP8_SPARSE_B;
            sa.values = reinterpret_cast<const uint8_t *>(256);
            sa.meta = reinterpret_cast<const uint8_t *>(256);
            (void)fp8_sparse24_gemm_workspace_size(&sa, nullptr, &ws);
        } else {
            (void)fp8_gemm_workspace_size(&g, nullptr, &ws);
        }
        bytes += ws;
    }
    return (bytes + 255) & ~size_t(255);
}

void scheduler(fp8_server *s)
{
    if (!s->simulated) (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        const double now = s->now();
        bool progress = false;
        // retire
        for (size_t i = 0; i < s->inflight.size();) {
            Job &j = s->inflight[i];
            if (s->exec->finished(j, now)) {
                const double t_done = s->simulated ? j.sim_done : now;
                TicketState &ts = s->tickets[j.ticket];
                if (j.fail != FP8_OK) {
                    // a launch failed after part of the job was queued: its
                    // arena range is reused only now that the queued work is done
                    ts.status = j.fail;
                    s->failed++;
                    s->exec->release(j);
                    s->arena.release(j.off, j.bytes);
                    s->inflight[i] = s->inflight.back();
                    s->inflight.pop_back();
                    progress = true;
                    continue;
                }
                ts.status = FP8_OK;
                ts.latency_ms = (t_done - j.arrival) * 1e3;
                s->latencies_ms.push_back(ts.latency_ms);
                s->stream_ms[(size_t)j.stream] += s->exec->exec_ms(j);
                s->flops += j.flops;
                s->last_done = std::max(s->last_done, t_done);
                s->done++;
                s->exec->release(j);
                s->arena.release(j.off, j.bytes);
                s->inflight[i] = s->inflight.back();
                s->inflight.pop_back();
                progress = true;
            } else {
                ++i;
            }
        }
        if (progress) s->cv_done.notify_all();
        // admit in arrival order
        const size_t max_inflight = (size_t)s->cfg.max_inflight;
        while (!s->pending.empty() && s->inflight.size() < max_inflight) {
            Job &j = s->pending.front();
            if (j.arrival > now) break;
            size_t off = 0;
            if (!s->arena.alloc(j.bytes, off)) break;
            j.off = off;
            j.admitted = now;
            std::vector<int> load(s->streams.size() ? s->streams.size() : (size_t)s->cfg.num_streams, 0);
            for (auto &f : s->inflight) load[(size_t)f.stream]++;
            j.stream = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            const Weight &w = s->weights[(size_t)j.req.weight_id];
            fp8_status st = s->exec->start(j, w, s->arena_base, j.stream);
            if (st != FP8_OK && j.queued) {
                j.fail = st;
                s->inflight.push_back(j);
                s->pending.pop_front();
                progress = true;
                continue;
            }
            if (st != FP8_OK) {
                s->exec->release(j);
                s->arena.release(j.off, j.bytes);
                s->tickets[j.ticket].status = st;
                s->failed++;
                s->pending.pop_front();
                s->cv_done.notify_all();
                continue;
            }
            s->inflight.push_back(j);
            s->pending.pop_front();
            s->peak_inflight = std::max<uint64_t>(s->peak_inflight, s->inflight.size());
            s->peak_bytes = std::max(s->peak_bytes, s->arena.used());
            progress = true;
        }
        if (s->stop && s->pending.empty() && s->inflight.empty()) break;
        if (!progress) {
            // sleep until the next arrival, a submit, or a short poll interval
            double wait_s = 50e-6;
            if (s->inflight.empty() && !s->pending.empty()) {
                wait_s = std::max(0.0, std::min(0.01, s->pending.front().arrival - now));
            } else if (s->inflight.empty() && s->pending.empty()) {
                wait_s = 0.01;
            }
            if (wait_s > 0) s->cv_work.wait_for(lk, std::chrono::duration<double>(wait_s));
        }
    }
}

fp8_status create_common(const fp8_server_config *cfg, bool simulated, double rate, double launch_us,
                         fp8_server **out)
{
    if (!cfg || !out) return set_error(FP8_ERR_ARG, "null config or server");
    if (cfg->num_streams < 1 || cfg->num_streams > 16) return set_error(FP8_ERR_ARG, "num_streams must be 1..16");
    if (cfg->hbm_budget_bytes < 4096) return set_error(FP8_ERR_ARG, "hbm_budget_bytes too small");
    auto *s = new fp8_server();
    s->cfg = *cfg;
    if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 4 * cfg->num_streams;
    s->simulated = simulated;
    s->stream_ms.assign((size_t)cfg->num_streams, 0.0);
    s->arena.reset(cfg->hbm_budget_bytes);
    if (simulated) {
        s->exec.reset(new SimExecutor(cfg->num_streams, rate, launch_us));
    } else {
        (void)hipGetDevice(&s->device);
        hipError_t e = hipMalloc(&s->arena_base, cfg->hbm_budget_bytes);
        if (e != hipSuccess) {
            delete s;
            return hip_error(e, "server arena");
        }
        for (int i = 0; i < cfg->num_streams; ++i) {
            hipStream_t st = nullptr;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (e != hipSuccess) {
                for (auto x : s->streams) (void)hipStreamDestroy(x);
                (void)hipFree(s->arena_base);
                delete s;
                return hip_error(e, "server stream");
            }
            s->streams.push_back(st);
        }
        s->exec.reset(new HipExecutor(s->streams));
    }
    s->t0 = Clock::now();
    s->thread = std::thread(scheduler, s);
    *out = s;
    return FP8_OK;
}

double percentile(std::vector<double> v, double p)
{
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    size_t rank = (size_t)std::ceil(p * (double)v.size());
    if (rank < 1) rank = 1;
    return v[rank - 1];
}

}  // namespace

extern "C" {

fp8_status fp8_server_create(const fp8_server_config *cfg, fp8_server **srv)
{
    return create_common(cfg, false, 0, 0, srv);
}

fp8_status fp8_server_create_simulated(const fp8_server_config *cfg, double gflop_per_ms, double launch_us,
                                       fp8_server **srv)
{
    if (!(gflop_per_ms > 0) || launch_us < 0) return set_error(FP8_ERR_ARG, "bad simulated rates");
    return create_common(cfg, true, gflop_per_ms, launch_us, srv);
}

fp8_status fp8_server_register_weight(fp8_server *s, const uint8_t *w, const uint8_t *meta, const float *w_descale,
                                      int64_t N, int64_t K, fp8_fmt fmt, int *weight_id)
{
    if (!s || !weight_id) return set_error(FP8_ERR_ARG, "null server or id");
    if (N < 1 || K < 1) return set_error(FP8_ERR_SHAPE, "N, K must be >= 1");
    if (fmt != FP8_E4M3 && fmt != FP8_E5M2) return set_error(FP8_ERR_ARG, "unknown format");
    if (!s->simulated && (!w || !w_descale)) return set_error(FP8_ERR_ARG, "null weight or descale");
    // Weights the request path could never run are refused here, before any
    // request queues work for them: a dense weight is read as N rows of K
    // codes (leading dimension K, so K % 16 == 0), a 2:4 weight needs whole
    // metadata bytes (K % 8 == 0); both need 16-byte aligned buffers.
    if (meta && K % 8) return set_error(FP8_ERR_SHAPE, "2:4 weight needs K % 8 == 0");
    if (!meta && K % 16) return set_error(FP8_ERR_SHAPE, "dense weight needs K % 16 == 0");
    auto misaligned = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) != 0; };
    if (misaligned(w) || misaligned(meta)) return set_error(FP8_ERR_ALIGN, "weight buffers must be 16-byte aligned");
    std::lock_guard<std::mutex> lk(s->mu);
    Weight x;
    x.w = w; x.meta = meta; x.descale = w_descale; x.N = N; x.K = K; x.fmt = fmt; x.sparse = meta != nullptr;
    s->weights.push_back(x);
    *weight_id = (int)s->weights.size() - 1;
    return FP8_OK;
}

fp8_status fp8_server_submit(fp8_server *s, const fp8_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) return set_error(FP8_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(FP8_ERR_CLOSED, "server is shutting down");
    if (req->weight_id < 0 || req->weight_id >= (int)s->weights.size()) return set_error(FP8_ERR_ARG, "unknown weight");
    if (req->M < 1) return set_error(FP8_ERR_SHAPE, "M must be >= 1");
    if (req->x_fmt != FP8_E4M3 && req->x_fmt != FP8_E5M2) return set_error(FP8_ERR_ARG, "unknown format");
    if (!s->simulated && (!req->x || !req->c)) return set_error(FP8_ERR_ARG, "null x or c");
    const Weight &w = s->weights[(size_t)req->weight_id];
    Job j;
    j.req = *req;
    j.bytes = job_bytes(s, *req, w);
    j.flops = 2.0 * (double)req->M * (double)w.N * (double)w.K;
    if (j.bytes > s->arena.size()) {
        s->rejected++;
        return set_error(FP8_ERR_BUDGET, "request needs more memory than the whole budget");
    }
    j.ticket = s->next_ticket++;
    j.arrival = req->arrival_time_s >= 0 ? req->arrival_time_s : s->now();
    if (s->first_arrival < 0 || j.arrival < s->first_arrival) s->first_arrival = j.arrival;
    s->tickets[j.ticket] = TicketState{};
    // keep pending in arrival order (submitters may interleave)
    auto it = s->pending.end();
    while (it != s->pending.begin() && std::prev(it)->arrival > j.arrival) --it;
    s->pending.insert(it, j);
    *ticket = j.ticket;
    s->cv_work.notify_one();
    return FP8_OK;
}

fp8_status fp8_server_poll(fp8_server *s, uint64_t ticket)
{
    if (!s) return set_error(FP8_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return set_error(FP8_ERR_ARG, "unknown ticket");
    return it->second.status;
}

fp8_status fp8_server_wait(fp8_server *s, uint64_t ticket, int64_t timeout_us)
{
    if (!s) return set_error(FP8_ERR_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return set_error(FP8_ERR_ARG, "unknown ticket");
    auto ready = [&] { return s->tickets[ticket].status != FP8_ERR_PENDING; };
    if (timeout_us < 0) s->cv_done.wait(lk, ready);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
        return set_error(FP8_ERR_TIMEOUT, "wait timed out");
    return s->tickets[ticket].status;
}

fp8_status fp8_server_latency(fp8_server *s, uint64_t ticket, double *ms)
{
    if (!s || !ms) return set_error(FP8_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return set_error(FP8_ERR_ARG, "unknown ticket");
    if (it->second.status != FP8_OK) return it->second.status;
    *ms = it->second.latency_ms;
    return FP8_OK;
}

fp8_status fp8_server_drain(fp8_server *s)
{
    if (!s) return set_error(FP8_ERR_ARG, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_work.notify_one();
    s->cv_done.wait(lk, [&] { return s->pending.empty() && s->inflight.empty(); });
    return FP8_OK;
}

fp8_status fp8_server_stats_get(fp8_server *s, fp8_server_stats *st)
{
    if (!s || !st) return set_error(FP8_ERR_ARG, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    fp8_server_stats r{};
    r.p50_ms = percentile(s->latencies_ms, 0.50);
    r.p99_ms = percentile(s->latencies_ms, 0.99);
    if (!s->latencies_ms.empty()) {
        double sum = 0;
        for (double v : s->latencies_ms) sum += v;
        r.mean_ms = sum / (double)s->latencies_ms.size();
        r.max_ms = *std::max_element(s->latencies_ms.begin(), s->latencies_ms.end());
    }
    r.span_s = s->first_arrival >= 0 ? s->last_done - s->first_arrival : 0;
    r.tflops = r.span_s > 0 ? s->flops / r.span_s / 1e12 : 0;
    const std::vector<double> &t = s->stream_ms;
    double mean = 0, mx = 0, mn = 1e300;
    for (double v : t) {
        mean += v;
        mx = std::max(mx, v);
        mn = std::min(mn, v);
    }
    mean /= (double)t.size();
    double var = 0;
    for (double v : t) var += (v - mean) * (v - mean);
    var /= (double)t.size();
    r.stream_cv = mean > 0 ? std::sqrt(var) / mean : 0;
    r.fairness_range = mean > 0 ? 1.0 - (mx - mn) / mean : 1.0;
    r.fairness_minmax = mx > 0 ? mn / mx : 1.0;
    r.done = s->done;
    r.failed = s->failed;
    r.rejected = s->rejected;
    r.peak_inflight = s->peak_inflight;
    r.peak_bytes = s->peak_bytes;
    *st = r;
    return FP8_OK;
}

fp8_status fp8_server_reset_stats(fp8_server *s)
{
    if (!s) return set_error(FP8_ERR_ARG, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->latencies_ms.clear();
    std::fill(s->stream_ms.begin(), s->stream_ms.end(), 0.0);
    s->flops = 0;
    s->first_arrival = -1;
    s->last_done = 0;
    s->done = s->failed = s->rejected = s->peak_inflight = 0;
    s->peak_bytes = 0;
    return FP8_OK;
}

double fp8_server_now(fp8_server *s) { return s ? s->now() : 0.0; }

fp8_status fp8_server_destroy(fp8_server *s)
{
    if (!s) return FP8_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_one();
    }
    if (s->thread.joinable()) s->thread.join();
    s->exec.reset();
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
    return FP8_OK;
}

}  // extern "C"
