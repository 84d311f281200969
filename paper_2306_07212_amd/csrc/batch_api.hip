// C ABI of the batched extraction (one persistent launch for many networks).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "batch.h"
#include "host.h"

using namespace pcx;

struct pcx_batch {
    int n = 0;
    std::vector<int> D, Wd, M, nsteps;
    std::vector<BatchResult> res;
    std::vector<pcx_complex *> fallback;  // networks extracted on the per-step path
    double *oX = nullptr;
    uint64_t *oSG = nullptr;
    int2 *oE = nullptr;
    double time_ms = 0.0, kernel_ms = 0.0;
    int workgroups = 0, wg_per_cu = 0, n_fallback = 0;
    int sched = 0;                            // schedule bits of the launch (kSched*)
    std::vector<int> sig;                     // size signature of the batched networks
    std::vector<std::vector<int64_t>> steps;  // per-step counters of each batched network (kStepsNow)
    StepRec *rec_dev = nullptr;               // the same, still on the device (kStepsLater)
    std::vector<size_t> rec_off;              //   network i's first record
    std::vector<int> nsub, ZS;
    std::vector<std::vector<uint64_t>> valid;
};

namespace {

// the autotuner's choices: batch size signature -> (workgroups per CU, schedule bits)
std::mutex g_tune_mu;
std::map<std::vector<int>, std::pair<int, int>> g_tuned;

// size signature of a batch: the sorted (subdivided neurons, D) of its batched networks
std::vector<int> signature(const std::vector<int> &nsteps, const std::vector<int> &D, const std::vector<int> &idx) {
    std::vector<int> sig;
    for (int i : idx) sig.push_back(nsteps[i] * 16 + D[i]);
    std::sort(sig.begin(), sig.end());
    return sig;
}

// This thread's pinned staging buffer of at least `bytes` bytes, kept for its
// later calls (every caller synchronizes its stream before it returns, so no
// copy through the old buffer is pending when it grows). Like the thread's
// other pinned buffers and events it is never released: the runtime may be
// gone at thread exit.
int staging(size_t bytes, char *&out) {
    thread_local char *buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        std::shared_lock<std::shared_mutex> gate(capture_gate());
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        const size_t nc = std::max<size_t>(bytes, 64 << 10);
        if (hipHostMalloc((void **)&buf, nc, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            buf = nullptr;
            return fail(PCX_ERR_OOM, "pinned staging buffer");
        }
        cap = nc;
    }
    out = buf;
    return PCX_OK;
}

// this thread's pair of timing events on the current device (created once)
int launch_events(hipEvent_t &a, hipEvent_t &b) {
    thread_local std::map<int, std::pair<hipEvent_t, hipEvent_t>> ev;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    auto it = ev.find(dev);
    if (it == ev.end()) {
        std::shared_lock<std::shared_mutex> gate(capture_gate());
        hipEvent_t x = nullptr, y = nullptr;
        HIPCHK(hipEventCreate(&x));
        HIPCHK(hipEventCreate(&y));
        it = ev.emplace(dev, std::make_pair(x, y)).first;
    }
    a = it->second.first;
    b = it->second.second;
    return PCX_OK;
}

size_t align16(size_t x) { return (x + 15) / 16 * 16; }

}  // namespace

namespace {

// The batched extraction. steps: kStepsNow copies every batched network's
// per-step counters to the host at once (the batch of one behind small
// pcx_extract calls); kStepsLater keeps them on the device for
// pcx_batch_steps to copy one network's on request; kStepsNone logs nothing.
enum { kStepsNone = 0, kStepsNow = 1, kStepsLater = 2 };
int batch_run(int32_t n, const pcx_mlp *const *mlps, const double *lo, const double *hi, const pcx_opts *opts,
              int steps_mode, pcx_batch **out, int force_sched = -1) {
    const bool keep_steps = steps_mode != kStepsNone;
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 0 || (n > 0 && (!mlps || !lo || !hi))) return fail(PCX_ERR_INVALID, "NULL argument");
    pcx_opts o{};
    if (opts) o = *opts;
    if (o.prune || o.record_tape) return fail(PCX_ERR_INVALID, "batched extraction supports neither prune nor record_tape");
    hipStream_t st = (hipStream_t)o.stream;
    auto t_start = std::chrono::steady_clock::now();
    auto *bt = new pcx_batch();
    bt->n = n;
    bt->res.assign(n, BatchResult{});
    bt->fallback.assign(n, nullptr);
    bt->D.resize(n);
    bt->Wd.resize(n);
    bt->M.resize(n);
    bt->nsteps.resize(n);
    bt->nsub.resize(n);
    bt->ZS.resize(n);
    bt->valid.resize(n);
    bt->steps.resize(n);
    std::vector<BatchNet> nets(n);
    std::vector<double> pred(n);
    std::vector<int> batched, direct;
    size_t box_off = 0;
    int maxD = 1, maxWd = 1, maxZS = 1;
    double predV = 0;
    for (int i = 0; i < n; ++i) {
        const pcx_mlp *m = mlps[i];
        if (!m) {
            pcx_batch_free(bt);
            return fail(PCX_ERR_INVALID, "NULL network");
        }
        const int D = m->D, L = m->L, nsub = o.include_output ? L : L - 1;
        for (int j = 0; j < D; ++j)
            if (!(lo[box_off + j] < hi[box_off + j])) {
                pcx_batch_free(bt);
                return fail(PCX_ERR_INVALID, "box must have lo < hi in every coordinate");
            }
        int Wd = 1, M = 2 * D, N = 0, ZS = 1;
        bool fits = D <= kBatchMaxD && L <= kBatchMaxLayers;
        for (int l = 1; l <= nsub; ++l) {
            if (m->widths[l] > kMaxWidth) fits = false;
            Wd += (m->widths[l] + 31) / 32;
            M += m->widths[l];
            N += m->widths[l];
            ZS = std::max(ZS, m->widths[l]);
        }
        if (Wd > kBatchMaxWords) fits = false;
        bt->D[i] = D;
        bt->Wd[i] = Wd;
        bt->M[i] = M;
        bt->nsteps[i] = N;
        bt->nsub[i] = nsub;
        bt->ZS[i] = ZS;
        if (steps_mode == kStepsNow) {
            std::vector<uint64_t> v(Wd, 0);
            for (int e = 0; e < 2 * D; ++e) v[0] |= 1ull << (2 * e);
            int w0 = 1;
            for (int l = 1; l <= nsub; ++l) {
                for (int c = 0; c < m->widths[l]; ++c) v[w0 + (c >> 5)] |= 1ull << (2 * (c & 31));
                w0 += (m->widths[l] + 31) / 32;
            }
            bt->valid[i] = v;
        }
        pred[i] = predict_vertices(D, N);
        if (pred[i] > 65536.0) fits = false;  // larger networks use the per-step path
        if (fits) {
            BatchNet &bn = nets[i];
            std::memset(&bn, 0, sizeof bn);
            for (int l = 0; l < L; ++l) {
                bn.Wt[l] = m->Wt[l];
                bn.b[l] = m->b[l];
            }
            for (int l = 0; l <= L; ++l) bn.widths[l] = m->widths[l];
            bn.L = L;
            bn.nsub = nsub;
            bn.D = D;
            for (int j = 0; j < D; ++j) {
                bn.lo[j] = lo[box_off + j];
                bn.hi[j] = hi[box_off + j];
            }
            batched.push_back(i);
            maxD = std::max(maxD, D);
            maxWd = std::max(maxWd, Wd);
            maxZS = std::max(maxZS, ZS);
            predV = std::max(predV, pred[i]);
        } else {
            direct.push_back(i);
        }
        box_off += D;
    }
    // largest predicted work first (the queue of the persistent kernel)
    std::sort(batched.begin(), batched.end(), [&](int a, int b) {
        return pred[a] * bt->nsteps[a] > pred[b] * bt->nsteps[b] || (pred[a] * bt->nsteps[a] == pred[b] * bt->nsteps[b] && a < b);
    });
    int rc = PCX_OK;
    Arena ar;
    ar.cap = o.max_bytes;
    float kms = 0.f;
    StepRec *rec_dev = nullptr;
    size_t rec_tot = 0;
    std::vector<size_t> rec_off(n, 0);
    size_t in_bytes = 0, out_bytes = 0, res_bytes = 0;
    char *in_dev = nullptr, *out_dev = nullptr;
    if (!batched.empty()) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // per-workgroup arena from the largest batched network
        const int P = 2 * (maxD - 1) > 0 ? 2 * (maxD - 1) : 1;
        size_t vcap = (size_t)(predV * 1.25) + 64;
        size_t vbytes = vcap * 8 * (size_t)(maxD + maxWd + maxZS);
        vbytes = (vbytes + 255) / 256 * 256;
        int ecap = (int)(((size_t)vcap * (maxD + 1) + 15) / 16 * 16);
        int kcap = (int)std::max<size_t>(1024, (size_t)P * std::max<size_t>(256, vcap / 12));
        uint32_t tcap = 256;
        while ((uint64_t)tcap < 2ull * (uint64_t)kcap && tcap < (1u << 31)) tcap <<= 1;
        size_t abytes = batch_arena_bytes(vbytes, ecap, kcap, tcap);
        abytes = (abytes + 255) / 256 * 256;
        // workgroups per CU and schedule: from the autotuner's cache, else 2 and the default
        const std::vector<int> sig = signature(bt->nsteps, bt->D, batched);
        bt->sig = sig;
        int wpc = 2, sched = kSchedDefault;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(sig);
            if (it != g_tuned.end()) {
                wpc = it->second.first;
                sched = it->second.second;
            }
        }
        if (o.batch_wg_per_cu > 0) wpc = o.batch_wg_per_cu;
        if (force_sched < 0) {
            // test hook: one schedule for every launch (0 .. kSchedCount-1)
            const char *v = getenv("PCX_BATCH_SCHED");
            if (v && *v) force_sched = std::max(0, std::min(kSchedCount - 1, atoi(v)));
        }
        if (force_sched >= 0) sched = force_sched;
        bt->sched = sched;
        int grid = std::min<int>((int)batched.size(), cus * wpc);
        // output pool from the predictions (overflowing networks fall back)
        double sv = 0, ssg = 0, se = 0;
        for (int i : batched) {
            const double v = std::min(pred[i], (double)vcap);
            sv += v * bt->D[i];
            ssg += v * bt->Wd[i];
            se += v * (bt->D[i] + 1);
        }
        const unsigned long long capV = (unsigned long long)(sv * 1.1) + 1024, capSG = (unsigned long long)(ssg * 1.1) + 1024,
                                 capE = (unsigned long long)(se * 1.1) + 1024;
        void *p;
        BatchArgs A{};
        if ((rc = ar.alloc(&p, (size_t)grid * abytes))) goto fail_out;
        A.arena = (char *)p;
        if ((rc = ar.alloc(&p, capV * sizeof(double)))) goto fail_out;
        bt->oX = (double *)p;
        ar.forget(p);  // owned by the batch from here on
        if ((rc = ar.alloc(&p, capSG * sizeof(uint64_t)))) goto fail_out;
        bt->oSG = (uint64_t *)p;
        ar.forget(p);  // owned by the batch from here on
        if ((rc = ar.alloc(&p, capE * sizeof(int2)))) goto fail_out;
        bt->oE = (int2 *)p;
        ar.forget(p);  // owned by the batch from here on
        // the inputs in one block (the pool counters, zero; the order; the network
        // descriptors) and the outputs in one block (the results, and the step
        // log with kStepsNow), each moved by one copy through pinned memory
        in_bytes = 8 * sizeof(unsigned long long) + align16(batched.size() * sizeof(int)) + (size_t)n * sizeof(BatchNet);
        if ((rc = ar.alloc(&p, in_bytes))) goto fail_out;
        in_dev = (char *)p;
        A.pool = (unsigned long long *)in_dev;
        A.ticket = (int *)(A.pool + 4);
        A.order = (const int *)(in_dev + 8 * sizeof(unsigned long long));
        A.nets = (const BatchNet *)(in_dev + 8 * sizeof(unsigned long long) + align16(batched.size() * sizeof(int)));
        res_bytes = align16((size_t)n * sizeof(BatchResult));
        {
            size_t tot = 0;
            if (keep_steps)
                for (int i : batched) tot += (size_t)bt->nsteps[i];
            out_bytes = res_bytes + (steps_mode == kStepsNow ? std::max<size_t>(tot, 1) * sizeof(StepRec) : 0);
        }
        if ((rc = ar.alloc(&p, out_bytes))) goto fail_out;
        out_dev = (char *)p;
        A.res = (BatchResult *)out_dev;
        if (keep_steps) {
            size_t tot = 0;
            for (int i : batched) tot += (size_t)bt->nsteps[i];
            if (steps_mode == kStepsLater) {
                // kept by the batch (returned to the pool by pcx_batch_free)
                size_t got = 0;
                rec_dev = (StepRec *)pool().get(std::max<size_t>(tot, 1) * sizeof(StepRec), &got, ~(size_t)0);
                if (!rec_dev) {
                    rc = fail(PCX_ERR_OOM, "step log of the batch");
                    goto fail_out;
                }
                bt->rec_dev = rec_dev;
            } else {
                rec_dev = (StepRec *)(out_dev + res_bytes);
            }
            size_t off = 0;
            for (int i : batched) {
                nets[i].rec = rec_dev + off;
                rec_off[i] = off;
                off += (size_t)bt->nsteps[i];
            }
            rec_tot = tot;
            if (steps_mode == kStepsLater) bt->rec_off = rec_off;
        }
        A.n = (int)batched.size();
        A.arena_bytes = abytes;
        A.vbytes = vbytes;
        A.ecap = ecap;
        A.kcap = kcap;
        A.tcap = tcap;
        A.oX = bt->oX;
        A.oSG = bt->oSG;
        A.oE = bt->oE;
        A.capV = capV;
        A.capSG = capSG;
        A.capE = capE;
        {
            // (PCX_DEBUG_HASH_BITS: as in pcx_extract, collisions on purpose for tests)
            const char *v = getenv("PCX_DEBUG_HASH_BITS");
            const int hb = v ? atoi(v) : 64;
            A.hbits = hb >= 1 && hb < 64 ? hb : 64;
            A.verify = o.verify_pairs ? 1 : 0;
        }
        {
            char *stg = nullptr;
            if ((rc = staging(std::max(in_bytes, out_bytes), stg))) goto fail_out;
            std::memset(stg, 0, 8 * sizeof(unsigned long long));
            std::memcpy(stg + 8 * sizeof(unsigned long long), batched.data(), batched.size() * sizeof(int));
            std::memcpy(stg + 8 * sizeof(unsigned long long) + align16(batched.size() * sizeof(int)), nets.data(),
                        (size_t)n * sizeof(BatchNet));
            HIPCHK(hipMemcpyAsync(in_dev, stg, in_bytes, hipMemcpyHostToDevice, st));
            hipEvent_t e0, e1;
            if ((rc = launch_events(e0, e1))) goto fail_out;
            HIPCHK(hipEventRecord(e0, st));
            launch_batch(A, grid, sched, st);
            HIPCHK(hipGetLastError());
            HIPCHK(hipEventRecord(e1, st));
            // (stream order: the input copy out of the staging buffer is done before this one lands there)
            HIPCHK(hipMemcpyAsync(stg, out_dev, out_bytes, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            std::memcpy(bt->res.data(), stg, (size_t)n * sizeof(BatchResult));
            std::vector<StepRec> rec(steps_mode == kStepsNow ? rec_tot : 0);
            if (!rec.empty()) std::memcpy(rec.data(), stg + res_bytes, rec_tot * sizeof(StepRec));
            for (int i : batched) {
                if (steps_mode != kStepsNow || bt->res[i].status != BATCH_OK) continue;
                auto &sv = bt->steps[i];
                sv.resize((size_t)bt->nsteps[i] * 4);
                for (int k = 0; k < bt->nsteps[i]; ++k) {
                    const StepRec &q = rec[rec_off[i] + k];
                    sv[(size_t)k * 4 + 0] = q.V0;
                    sv[(size_t)k * 4 + 1] = q.E0;
                    sv[(size_t)k * 4 + 2] = q.S;
                    sv[(size_t)k * 4 + 3] = 2 * ((int64_t)q.E1 - q.E0 - q.S);
                }
            }
            HIPCHK(hipEventElapsedTime(&kms, e0, e1));
        }
        bt->workgroups = grid;
        bt->wg_per_cu = wpc;
        for (int i : batched) {
            const int s = bt->res[i].status;
            if (s == BATCH_OVERFLOW || s == BATCH_POOL || s == BATCH_RETRY) direct.push_back(i);
            else if (s == BATCH_INTERNAL) {
                rc = fail(PCX_ERR_DEVICE, "internal error in the batched kernel");
                goto fail_out;
            }
        }
    }
    bt->kernel_ms = kms;
    // networks that do not fit the batched kernel: the per-step path
    box_off = 0;
    {
        std::vector<size_t> offs(n);
        for (int i = 0; i < n; ++i) {
            offs[i] = box_off;
            box_off += bt->D[i];
        }
        pcx_opts od = o;
        for (int i : direct) {
            pcx_complex *cx = nullptr;
            int r = extract_ordinary(mlps[i], lo + offs[i], hi + offs[i], &od, &cx);
            BatchResult &br = bt->res[i];
            std::memset(&br, 0, sizeof br);
            if (r == PCX_ERR_DEGENERATE) {
                br.status = BATCH_DEGENERATE;
                continue;
            }
            if (r != PCX_OK) {
                rc = r;
                goto fail_out;
            }
            bt->fallback[i] = cx;
            br.status = BATCH_OK;
            br.V = (int)cx->V;
            br.E = (int)cx->E;
            br.Wd = cx->Wd;
            br.splits = cx->total_splits;
            br.pairs = cx->total_pairs;
            bt->n_fallback++;
        }
    }
    bt->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    *out = bt;
    return PCX_OK;
fail_out:
    pcx_batch_free(bt);
    return rc;
}

}  // namespace

extern "C" int pcx_extract_batch(int32_t n, const pcx_mlp *const *mlps, const double *lo, const double *hi,
                                 const pcx_opts *opts, pcx_batch **out) {
    return batch_run(n, mlps, lo, hi, opts, kStepsLater, out);
}

namespace pcx {

// A small network's pcx_extract as a batch of one: one launch of the batched
// kernel (one workgroup runs every step) instead of several launches per
// neuron step. The complex, its numbering and its per-step counters are those
// of the per-step path (the same device functions in the same order).
int tiny_extract(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts &o, pcx_complex **out) {
    *out = nullptr;
    pcx_batch *bt = nullptr;
    const pcx_mlp *const one[1] = {mlp};
    int rc = batch_run(1, one, lo, hi, &o, kStepsNow, &bt);
    if (rc) return rc;
    const BatchResult &r = bt->res[0];
    if (r.status == BATCH_DEGENERATE) {
        pcx_batch_free(bt);
        return fail(PCX_ERR_DEGENERATE, "input is not generic");
    }
    if (bt->fallback[0]) {  // too large for the kernel's arena: the per-step path ran
        *out = bt->fallback[0];
        bt->fallback[0] = nullptr;
        pcx_batch_free(bt);
        return PCX_OK;
    }
    auto *cx = new pcx_complex();
    cx->D = bt->D[0];
    cx->M = bt->M[0];
    cx->Wd = bt->Wd[0];
    cx->n_steps = bt->nsteps[0];
    cx->V = r.V;
    cx->E = r.E;
    cx->valid = bt->valid[0];
    // the output pools hold this network alone, from offset 0: they become its arrays
    cx->X = bt->oX;
    cx->SG = bt->oSG;
    cx->EDG = bt->oE;
    bt->oX = nullptr;
    bt->oSG = nullptr;
    bt->oE = nullptr;
    cx->steps = bt->steps[0];
    cx->total_splits = r.splits;
    cx->total_pairs = r.pairs;
    cx->time_ms = bt->kernel_ms;
    cx->ZS = bt->ZS[0];
    cx->nsub = bt->nsub[0];
    pcx_batch_free(bt);
    *out = cx;
    return PCX_OK;
}

}  // namespace pcx

extern "C" {

int pcx_batch_info(const pcx_batch *bt, int32_t i, pcx_info *info) {
    if (!bt || !info || i < 0 || i >= bt->n) return fail(PCX_ERR_INVALID, "bad argument");
    const BatchResult &r = bt->res[i];
    if (r.status == BATCH_DEGENERATE) return fail(PCX_ERR_DEGENERATE, "network is not generic");
    std::memset(info, 0, sizeof *info);
    info->V = r.V;
    info->E = r.E;
    info->D = bt->D[i];
    info->M = bt->M[i];
    info->Wd = bt->Wd[i];
    info->n_steps = bt->nsteps[i];
    info->total_splits = r.splits;
    info->total_pairs = r.pairs;
    return PCX_OK;
}

int pcx_batch_copy(const pcx_batch *bt, int32_t i, double *coords, uint64_t *signs, int32_t *edges) {
    if (!bt || i < 0 || i >= bt->n) return fail(PCX_ERR_INVALID, "bad argument");
    const BatchResult &r = bt->res[i];
    if (r.status == BATCH_DEGENERATE) return fail(PCX_ERR_DEGENERATE, "network is not generic");
    if (bt->fallback[i]) return pcx_complex_copy(bt->fallback[i], coords, signs, edges);
    const int D = bt->D[i];
    int rc;
    if (coords &&
        (rc = copy_sync(coords, bt->oX + (size_t)r.offV, (size_t)r.V * D * sizeof(double), hipMemcpyDeviceToHost)))
        return rc;
    if (signs &&
        (rc = copy_sync(signs, bt->oSG + r.offSG, (size_t)r.V * r.Wd * sizeof(uint64_t), hipMemcpyDeviceToHost)))
        return rc;
    if (edges && (rc = copy_sync(edges, bt->oE + r.offE, (size_t)r.E * sizeof(int2), hipMemcpyDeviceToHost)))
        return rc;
    return PCX_OK;
}

int pcx_batch_steps(const pcx_batch *bt, int32_t i, int64_t *steps) {
    if (!bt || !steps || i < 0 || i >= bt->n) return fail(PCX_ERR_INVALID, "bad argument");
    const BatchResult &r = bt->res[i];
    if (r.status == BATCH_DEGENERATE) return fail(PCX_ERR_DEGENERATE, "network is not generic");
    if (bt->fallback[i]) return pcx_complex_steps(bt->fallback[i], steps);
    if (!bt->steps[i].empty()) {
        std::memcpy(steps, bt->steps[i].data(), bt->steps[i].size() * sizeof(int64_t));
        return PCX_OK;
    }
    if (!bt->rec_dev) return fail(PCX_ERR_INVALID, "the batch kept no step log");
    // this network's records, from the device
    const int ns = bt->nsteps[i];
    std::vector<StepRec> rec(ns);
    int rc;
    if ((rc = copy_sync(rec.data(), bt->rec_dev + bt->rec_off[i], (size_t)ns * sizeof(StepRec), hipMemcpyDeviceToHost)))
        return rc;
    for (int k = 0; k < ns; ++k) {
        steps[(size_t)k * 4 + 0] = rec[k].V0;
        steps[(size_t)k * 4 + 1] = rec[k].E0;
        steps[(size_t)k * 4 + 2] = rec[k].S;
        steps[(size_t)k * 4 + 3] = 2 * ((int64_t)rec[k].E1 - rec[k].E0 - rec[k].S);
    }
    return PCX_OK;
}

int pcx_batch_summary(const pcx_batch *bt, pcx_batch_stats *s) {
    if (!bt || !s) return fail(PCX_ERR_INVALID, "NULL argument");
    std::memset(s, 0, sizeof *s);
    s->n = bt->n;
    for (int i = 0; i < bt->n; ++i) {
        const BatchResult &r = bt->res[i];
        if (r.status == BATCH_DEGENERATE) {
            s->degenerate++;
            continue;
        }
        s->total_V += r.V;
        s->total_E += r.E;
        s->total_splits += r.splits;
    }
    s->fallbacks = bt->n_fallback;
    s->workgroups = bt->workgroups;
    s->wg_per_cu = bt->wg_per_cu;
    s->split_lanes = sched_split_lanes(bt->sched);
    s->select_items = (bt->sched & kSchedSelect8) ? 8 : 16;
    s->kernel_ms = bt->kernel_ms;
    s->time_ms = bt->time_ms;
    return PCX_OK;
}

void pcx_batch_free(pcx_batch *bt) {
    if (!bt) return;
    pool().put(bt->oX);
    pool().put(bt->oSG);
    pool().put(bt->oE);
    pool().put(bt->rec_dev);
    for (auto *c : bt->fallback) pcx_complex_free(c);
    delete bt;
}

int pcx_batch_tune(int32_t n, const pcx_mlp *const *mlps, const double *lo, const double *hi, const pcx_opts *opts,
                   pcx_batch_tuning *result) {
    // time the batch's launch under each schedule at two workgroups per CU,
    // then each occupancy under the best schedule (best of two launches each)
    std::vector<int> sig;
    auto measure = [&](int wpc, int sched, double *ms) -> int {
        *ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            pcx_opts o{};
            if (opts) o = *opts;
            o.batch_wg_per_cu = wpc;
            pcx_batch *bt = nullptr;
            int rc = batch_run(n, mlps, lo, hi, &o, kStepsNone, &bt, sched);
            if (rc) return rc;
            *ms = std::min(*ms, bt->kernel_ms);
            sig = bt->sig;
            pcx_batch_free(bt);
        }
        return PCX_OK;
    };
    int rc, best_sched = kSchedDefault, best_wpc = 2, tried = 0;
    double ms_default = 0, best = 1e300, ms;
    for (int i = 0; i < kSchedCount; ++i) {
        // the default first, then the others in order
        const int sc = i == 0 ? kSchedDefault : (i <= kSchedDefault ? i - 1 : i);
        if ((rc = measure(2, sc, &ms))) return rc;
        ++tried;
        if (i == 0) ms_default = ms;
        if (ms < best) {
            best = ms;
            best_sched = sc;
        }
    }
    for (int w : {1, 4}) {
        if ((rc = measure(w, best_sched, &ms))) return rc;
        ++tried;
        if (ms < best) {
            best = ms;
            best_wpc = w;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[sig] = {best_wpc, best_sched};
    }
    if (result) {
        result->wg_per_cu = best_wpc;
        result->split_lanes = sched_split_lanes(best_sched);
        result->select_items = (best_sched & kSchedSelect8) ? 8 : 16;
        result->candidates = tried;
        result->ms_default = ms_default;
        result->ms_best = best;
    }
    return PCX_OK;
}

}  // extern "C"
