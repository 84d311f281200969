// Extraction server: continuous batching of extraction requests on one GPU.
//
// Requests are queued in arrival order. A scheduler thread admits them in that
// order while the predicted device memory of the admitted, unfinished jobs
// stays within the budget (the complex size is unknown up front; the
// prediction only gates admission). Admitted small networks are gathered into
// the next tick of the batched persistent kernel: ticks run back to back, and
// whatever arrived while one ran joins the next. Admitted large networks run on
// the per-step path in worker threads, each on its own stream, so their kernels
// overlap with the ticks and with each other; so does a small network that
// would be alone in its tick while a worker is free (at low load the per-step
// path answers it sooner). Every result is the complex pcx_extract returns for
// the same request.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>

#include "batch.h"
#include "host.h"

using namespace pcx;

namespace {

using Clock = std::chrono::steady_clock;

struct BatchHolder {
    pcx_batch *bt = nullptr;
    ~BatchHolder() { pcx_batch_free(bt); }
};

struct Job {
    uint64_t id = 0;
    const pcx_mlp *mlp = nullptr;
    std::vector<double> lo, hi;
    Clock::time_point t_submit, t_admit, t_done;
    double pred_bytes = 0;
    bool small = false;
    int status = PCX_PENDING;  // PCX_PENDING until done, then PCX_OK or an error
    std::string err;
    pcx_complex *cx = nullptr;
    std::shared_ptr<BatchHolder> batch;
    int bidx = -1;
    int64_t V = 0, E = 0, splits = 0;
    int D = 0, Wd = 0;  // row sizes of the result (Wd counts the output word with include_output)
};

}  // namespace

struct pcx_server {
    pcx_server_opts opts{};
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<Job *> pending;    // not yet admitted, arrival order
    std::deque<Job *> large_q;    // admitted large jobs waiting for a worker
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    double mem_in_use = 0;
    int running_large = 0, running_ticks = 0;
    int64_t inflight = 0;  // admitted, not finished
    std::vector<double> latencies_ms, queue_ms;
    Clock::time_point t_first{}, t_last{};
    bool any = false;
    int64_t done_splits = 0, done_vertices = 0, ticks = 0, tick_jobs = 0;
    std::thread sched;
    std::vector<std::thread> workers;
    hipStream_t tick_stream = nullptr;
    std::vector<hipStream_t> worker_streams;
    int device = 0;
};

namespace {

void finish(pcx_server *s, Job *j) {
    // caller holds s->mu
    j->t_done = Clock::now();
    s->mem_in_use -= j->pred_bytes;
    s->inflight--;
    if (j->status == PCX_OK) {
        s->latencies_ms.push_back(std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count());
        s->queue_ms.push_back(std::chrono::duration<double, std::milli>(j->t_admit - j->t_submit).count());
        s->done_splits += j->splits;
        s->done_vertices += j->V;
    }
    if (!s->any || j->t_done > s->t_last) s->t_last = j->t_done;
    s->cv_done.notify_all();
    s->cv_sched.notify_all();
}

void worker_loop(pcx_server *s, int w) {
    (void)hipSetDevice(s->device);
    for (;;) {
        Job *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_sched.wait(lk, [&] { return s->stop || !s->large_q.empty(); });
            if (s->large_q.empty()) return;  // stop requested and nothing left
            j = s->large_q.front();
            s->large_q.pop_front();
            s->running_large++;
        }
        pcx_opts o{};
        o.include_output = s->opts.include_output;
        o.stream = s->worker_streams[w];
        pcx_complex *cx = nullptr;
        // no graph capture in the server: it sees few repeats, and its threads run concurrently
        const int rc = extract_ordinary(j->mlp, j->lo.data(), j->hi.data(), &o, &cx, kShortcutTiny);
        std::string err = rc ? pcx_last_error() : "";
        std::lock_guard<std::mutex> lk(s->mu);
        s->running_large--;
        j->status = rc;
        j->err = err;
        j->cx = cx;
        if (cx) {
            j->V = cx->V;
            j->E = cx->E;
            j->splits = cx->total_splits;
            j->D = cx->D;
            j->Wd = cx->Wd;
        }
        finish(s, j);
    }
}

void sched_loop(pcx_server *s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<Job *> tick;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_sched.wait(lk, [&] { return s->stop || !s->pending.empty(); });
            if (s->stop && s->pending.empty()) return;
            // admit in arrival order while the predicted memory fits
            while (!s->pending.empty()) {
                Job *j = s->pending.front();
                const bool idle = s->inflight == 0;  // always admit onto an idle GPU
                if (!idle && s->mem_in_use + j->pred_bytes > (double)s->opts.mem_budget) break;
                // a small request that would be alone in its tick while a worker is
                // free: the per-step path answers it sooner than one workgroup does
                if (j->small && tick.empty() && s->pending.size() == 1 &&
                    s->running_large + (int)s->large_q.size() < s->opts.large_workers)
                    j->small = false;
                s->pending.pop_front();
                j->t_admit = Clock::now();
                s->mem_in_use += j->pred_bytes;
                s->inflight++;
                if (j->small && (int)tick.size() < s->opts.max_batch) {
                    tick.push_back(j);
                } else if (j->small) {
                    // tick full: leave it for the next tick
                    s->mem_in_use -= j->pred_bytes;
                    s->inflight--;
                    s->pending.push_front(j);
                    break;
                } else {
                    s->large_q.push_back(j);
                    s->cv_sched.notify_all();
                }
            }
            if (!tick.empty()) s->running_ticks++;
        }
        if (tick.empty()) {
            // nothing admissible now: wait for memory to free up or new arrivals
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        // one tick of the persistent batched kernel over the admitted small jobs
        std::vector<const pcx_mlp *> mlps;
        std::vector<double> lo, hi;
        for (Job *j : tick) {
            mlps.push_back(j->mlp);
            lo.insert(lo.end(), j->lo.begin(), j->lo.end());
            hi.insert(hi.end(), j->hi.begin(), j->hi.end());
        }
        pcx_opts o{};
        o.include_output = s->opts.include_output;
        o.stream = s->tick_stream;
        pcx_batch *bt = nullptr;
        const int rc = pcx_extract_batch((int)tick.size(), mlps.data(), lo.data(), hi.data(), &o, &bt);
        std::string err = rc ? pcx_last_error() : "";
        auto holder = std::make_shared<BatchHolder>();
        holder->bt = bt;
        std::lock_guard<std::mutex> lk(s->mu);
        s->running_ticks--;
        s->ticks++;
        s->tick_jobs += (int64_t)tick.size();
        for (size_t k = 0; k < tick.size(); ++k) {
            Job *j = tick[k];
            if (rc) {
                j->status = rc;
                j->err = err;
            } else {
                pcx_info inf;
                const int r2 = pcx_batch_info(bt, (int)k, &inf);
                j->status = r2;
                if (r2 == PCX_OK) {
                    j->batch = holder;
                    j->bidx = (int)k;
                    j->V = inf.V;
                    j->E = inf.E;
                    j->splits = inf.total_splits;
                    j->D = inf.D;
                    j->Wd = inf.Wd;
                } else {
                    j->err = pcx_last_error();
                }
            }
            finish(s, j);
        }
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

extern "C" {

int pcx_server_create(const pcx_server_opts *opts, pcx_server **out) {
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    auto *s = new pcx_server();
    if (opts) s->opts = *opts;
    if (s->opts.mem_budget == 0) s->opts.mem_budget = 64ull << 30;
    if (s->opts.max_batch <= 0) s->opts.max_batch = 4096;
    if (s->opts.large_workers <= 0) s->opts.large_workers = 6;
    if (s->opts.small_vertices <= 0) s->opts.small_vertices = 65536;
    (void)hipGetDevice(&s->device);
    if (hipStreamCreateWithFlags(&s->tick_stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return fail(PCX_ERR_DEVICE, "hipStreamCreate failed");
    }
    s->worker_streams.resize(s->opts.large_workers);
    for (auto &st : s->worker_streams)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            pcx_server_destroy(s);
            return fail(PCX_ERR_DEVICE, "hipStreamCreate failed");
        }
    s->sched = std::thread(sched_loop, s);
    for (int w = 0; w < s->opts.large_workers; ++w) s->workers.emplace_back(worker_loop, s, w);
    *out = s;
    return PCX_OK;
}

int pcx_server_submit(pcx_server *s, const pcx_mlp *mlp, const double *lo, const double *hi, uint64_t *ticket) {
    if (!s || !mlp || !lo || !hi || !ticket) return fail(PCX_ERR_INVALID, "NULL argument");
    const int D = mlp->D;
    for (int j = 0; j < D; ++j)
        if (!(lo[j] < hi[j])) return fail(PCX_ERR_INVALID, "box must have lo < hi in every coordinate");
    auto job = std::make_unique<Job>();
    job->mlp = mlp;
    job->lo.assign(lo, lo + D);
    job->hi.assign(hi, hi + D);
    job->t_submit = Clock::now();
    const int nsub = s->opts.include_output ? mlp->L : mlp->L - 1;
    int N = 0, Wd = 1, ZS = 1;
    bool fits = D <= kBatchMaxD && mlp->L <= kBatchMaxLayers;
    for (int l = 1; l <= nsub; ++l) {
        N += mlp->widths[l];
        Wd += (mlp->widths[l] + 31) / 32;
        ZS = std::max(ZS, mlp->widths[l]);
        if (mlp->widths[l] > kMaxWidth) fits = false;
    }
    job->D = D;
    job->Wd = Wd;
    const double pv = predict_vertices(D, N);
    job->small = fits && Wd <= kBatchMaxWords && pv <= (double)s->opts.small_vertices;
    // rows (coordinates, signs, pre-activations) and ~(D+1) edges per vertex
    job->pred_bytes = pv * (8.0 * (D + Wd + ZS) + 16.0 * (D + 1));
    std::lock_guard<std::mutex> lk(s->mu);
    job->id = s->next_id++;
    *ticket = job->id;
    if (!s->any) {
        s->t_first = job->t_submit;
        s->any = true;
    }
    s->pending.push_back(job.get());
    s->jobs[job->id] = std::move(job);
    s->cv_sched.notify_all();
    return PCX_OK;
}

static int fill_result(Job *j, pcx_server_result *r) {
    std::memset(r, 0, sizeof *r);
    r->status = j->status;
    r->V = j->V;
    r->E = j->E;
    r->total_splits = j->splits;
    r->batched = j->small ? 1 : 0;
    r->D = j->D;
    r->Wd = j->Wd;
    if (j->status != PCX_PENDING) {
        r->latency_ms = std::chrono::duration<double, std::milli>(j->t_done - j->t_submit).count();
        r->queue_ms = std::chrono::duration<double, std::milli>(j->t_admit - j->t_submit).count();
    }
    return j->status == PCX_PENDING ? PCX_PENDING : PCX_OK;
}

int pcx_server_poll(pcx_server *s, uint64_t ticket, pcx_server_result *r) {
    if (!s || !r) return fail(PCX_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(PCX_ERR_INVALID, "unknown ticket");
    return fill_result(it->second.get(), r);
}

int pcx_server_wait(pcx_server *s, uint64_t ticket, pcx_server_result *r) {
    if (!s || !r) return fail(PCX_ERR_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return fail(PCX_ERR_INVALID, "unknown ticket");
    Job *j = it->second.get();
    s->cv_done.wait(lk, [&] { return j->status != PCX_PENDING; });
    return fill_result(j, r);
}

int pcx_server_copy(pcx_server *s, uint64_t ticket, double *coords, uint64_t *signs, int32_t *edges) {
    if (!s) return fail(PCX_ERR_INVALID, "NULL argument");
    Job *j;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(PCX_ERR_INVALID, "unknown ticket");
        j = it->second.get();
        if (j->status == PCX_PENDING) return PCX_PENDING;
        if (j->status != PCX_OK) return fail(j->status, j->err);
    }
    if (j->cx) return pcx_complex_copy(j->cx, coords, signs, edges);
    return pcx_batch_copy(j->batch->bt, j->bidx, coords, signs, edges);
}

int pcx_server_release(pcx_server *s, uint64_t ticket) {
    if (!s) return fail(PCX_ERR_INVALID, "NULL argument");
    std::unique_ptr<Job> j;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->jobs.find(ticket);
        if (it == s->jobs.end()) return fail(PCX_ERR_INVALID, "unknown ticket");
        if (it->second->status == PCX_PENDING) return fail(PCX_ERR_INVALID, "job still running");
        j = std::move(it->second);
        s->jobs.erase(it);
    }
    pcx_complex_free(j->cx);
    return PCX_OK;
}

int pcx_server_stats(pcx_server *s, pcx_server_summary *st) {
    if (!s || !st) return fail(PCX_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(st, 0, sizeof *st);
    st->completed = (int64_t)s->latencies_ms.size();
    st->p50_ms = percentile(s->latencies_ms, 0.50);
    st->p99_ms = percentile(s->latencies_ms, 0.99);
    st->mean_ms = 0;
    for (double x : s->latencies_ms) st->mean_ms += x;
    if (!s->latencies_ms.empty()) st->mean_ms /= s->latencies_ms.size();
    st->p50_queue_ms = percentile(s->queue_ms, 0.50);
    st->p99_queue_ms = percentile(s->queue_ms, 0.99);
    const double span = s->any ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    st->span_s = span;
    st->jobs_per_s = span > 0 ? st->completed / span : 0.0;
    st->splits_per_s = span > 0 ? s->done_splits / span : 0.0;
    st->vertices_per_s = span > 0 ? s->done_vertices / span : 0.0;
    st->ticks = s->ticks;
    st->mean_tick_jobs = s->ticks ? (double)s->tick_jobs / s->ticks : 0.0;
    return PCX_OK;
}

void pcx_server_destroy(pcx_server *s) {
    if (!s) return;
    {
        // drain: every submitted job finishes before the threads stop
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] {
            for (auto &kv : s->jobs)
                if (kv.second->status == PCX_PENDING) return false;
            return true;
        });
        s->stop = true;
        s->cv_sched.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    for (auto &t : s->workers)
        if (t.joinable()) t.join();
    for (auto &kv : s->jobs) pcx_complex_free(kv.second->cx);
    s->jobs.clear();
    if (s->tick_stream) (void)hipStreamDestroy(s->tick_stream);
    for (auto st : s->worker_streams)
        if (st) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
