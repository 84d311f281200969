// Repeated extractions of one network as a replayed HIP graph.
//
// Edge subdivision is deterministic: the same network on the same box gives the
// same counts at every neuron step (Sec. 4.2 fixes the work; this library's
// compactions and pairings are ordered). After a network's first extraction the
// library keeps its per-step log; the next extraction with the same box and
// options captures the whole kernel sequence -- every layer's evaluation and
// first-crossing scan, every step's compaction, split and pairing, with launch
// shapes taken from the log -- into a graph with storage of its own, sized
// exactly from the log, and later ones replay it: one launch, no host reads
// between the steps. A replay is accepted only if no flag is raised and its
// step log equals the recorded one; otherwise the graph is dropped and the
// extraction runs on the ordinary path. The complex is copied out of the
// graph's storage into arrays of its own, so the graph can run again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <shared_mutex>

#include "host.h"

namespace pcx {

namespace {
constexpr uint64_t kGraphMaxBytes = uint64_t(1) << 29;     // storage one cached graph may hold (512 MiB)
constexpr uint64_t kGraphBudget = uint64_t(1) << 32;       // storage all cached graphs may hold (4 GiB)
constexpr int kGraphBusy = -1000;  // build() could not have the capture gate: try again at a later request
std::atomic<uint64_t> g_graph_bytes{0};
}

struct GraphLog {
    std::vector<double> lo, hi;
    int include_output = 0;
    int seen = 1;                // ordinary extractions with this key (a graph is built at the third request)
    std::vector<int64_t> steps;  // [n_steps][4]: V, E before the step, splits, 2-face key slots
    int64_t V = 0, E = 0, Ebound = 0, Smax = 0;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> blocks;  // storage (pool blocks)
    Bufs b{};
    uint64_t bytes = 0;
    std::vector<uint64_t> valid;
    int D = 0, Wd = 0, ZS = 0, M = 0, nsub = 0, n_steps = 0;
    ~GraphEntry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (void *p : blocks) pool().put(p);
        g_graph_bytes -= bytes;
    }
};

struct GraphCache {
    std::mutex mu;
    std::unique_ptr<GraphLog> log;
    std::unique_ptr<GraphEntry> entry;
};

GraphCache *graph_cache_new() { return new GraphCache(); }
void graph_cache_free(GraphCache *c) { delete c; }

namespace {

bool eligible(const pcx_opts &o) {
    const char *off = getenv("PCX_NO_GRAPH");
    if (off && off[0] == '1') return false;
    return o.pairing == PCX_PAIR_HASH && !o.prune && !o.record_tape && o.timing == 0 && o.max_bytes == 0 &&
           !o.verify_pairs;
}

bool same_key(const GraphLog &g, int D, const double *lo, const double *hi, int incl) {
    if (g.include_output != incl || (int)g.lo.size() != D) return false;
    for (int j = 0; j < D; ++j)
        if (g.lo[j] != lo[j] || g.hi[j] != hi[j]) return false;
    return true;
}

// storage of the graph and the capture of the whole extraction on stream cs
int build(const pcx_mlp *mlp, const GraphLog &lg, GraphEntry &ge, hipStream_t cs) {
    const int D = mlp->D, nsub = lg.include_output ? mlp->L : mlp->L - 1;
    std::vector<int> lw(nsub + 1), step0(nsub + 1);
    lw[0] = 1;
    step0[0] = 0;
    int ZS = 1;
    for (int l = 0; l < nsub; ++l) {
        const int N = mlp->widths[l + 1];
        lw[l + 1] = lw[l] + (N + 31) / 32;
        step0[l + 1] = step0[l] + N;
        ZS = std::max(ZS, N);
    }
    const int Wd = lw[nsub], n_steps = step0[nsub], P = D >= 2 ? 2 * (D - 1) : 0;
    if ((int64_t)lg.steps.size() != (int64_t)n_steps * 4 || n_steps == 0) return fail(PCX_ERR_INVALID, "graph log");
    const size_t Vcap = (size_t)lg.V, Ecap = (size_t)std::max(lg.Ebound, lg.E);
    const size_t Kcap = std::max<size_t>(1, (size_t)P * (size_t)lg.Smax);
    size_t Tcap = 256;
    while (Tcap < 2 * Kcap) Tcap <<= 1;
    const uint64_t bytes = Vcap * 8ull * (D + Wd + ZS + 8) + Ecap * (8ull + 1 + 4 + 16) + Kcap * 12ull +
                           Tcap * 16ull + (uint64_t)n_steps * sizeof(StepRec) + kNextBlocks * 4ull;
    if (bytes > kGraphMaxBytes) return fail(PCX_ERR_CAPACITY, "graph storage above its cap");
    if (g_graph_bytes.fetch_add(bytes) + bytes > kGraphBudget) {
        g_graph_bytes -= bytes;
        return fail(PCX_ERR_CAPACITY, "cached graphs hold their whole budget");
    }
    ge.bytes = bytes;  // (returned to the budget when the entry goes)
    auto take = [&](size_t n) -> void * {
        size_t got = 0;
        void *p = pool().get(std::max<size_t>(n, 256), &got, ~(size_t)0);
        if (p) ge.blocks.push_back(p);
        return p;
    };
    Bufs &b = ge.b;
    b.X = (double *)take(Vcap * D * 8);
    b.SG = (uint64_t *)take(Vcap * Wd * 8);
    b.Z = (double *)take(Vcap * ZS * 8);
    b.LW = (uint64_t *)take(Vcap * 64);
    b.EDG = (int2 *)take(Ecap * 8);
    b.NX8 = (uint8_t *)take(Ecap);
    b.SPLX = (int *)take(Ecap * 4);
    b.SPLE = (int4 *)take(Ecap * 16);
    b.PINFO = (uint32_t *)take(Kcap * 4);
    b.PART = (uint64_t *)take(Kcap * 8);
    unsigned long long *HT[2] = {(unsigned long long *)take(Tcap * 8), (unsigned long long *)take(Tcap * 8)};
    b.CTR = (int *)take(CTR_COUNT * 4);
    b.SELCNT = (int *)take(kNextBlocks * 4);
    b.REC = (StepRec *)take((size_t)n_steps * sizeof(StepRec));
    uint64_t *valid = (uint64_t *)take(Wd * 8);
    double *dbox = (double *)take(2 * D * 8);
    b.VALID = valid;
    for (void *p : ge.blocks)
        if (!p) return fail(PCX_ERR_OOM, "graph storage");
    ge.valid.assign(Wd, 0);
    for (int e = 0; e < 2 * D; ++e) ge.valid[0] |= 1ull << (2 * e);
    for (int l = 0; l < nsub; ++l)
        for (int c = 0; c < mlp->widths[l + 1]; ++c) ge.valid[lw[l] + (c >> 5)] |= 1ull << (2 * (c & 31));
    std::vector<double> box(2 * D);
    for (int j = 0; j < D; ++j) {
        box[j] = lg.lo[j];
        box[D + j] = lg.hi[j];
    }
    // constant for every replay: copied once, outside the graph
    HIPCHK(hipMemcpyAsync(valid, ge.valid.data(), Wd * 8, hipMemcpyHostToDevice, cs));
    HIPCHK(hipMemcpyAsync(dbox, box.data(), 2 * D * 8, hipMemcpyHostToDevice, cs));
    HIPCHK(hipStreamSynchronize(cs));

    // no allocation or free of this library on another thread during the capture
    std::unique_lock<std::shared_mutex> gate(capture_gate(), std::try_to_lock);
    if (!gate.owns_lock()) return kGraphBusy;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int V0 = 1 << D, E0 = D << (D - 1);
    launch_ctr_init(b.CTR, V0, E0, cs);
    launch_fill64(b.PART, Kcap, 0ull, cs);
    launch_fill64(reinterpret_cast<uint64_t *>(HT[0]), Tcap, 0ull, cs);
    launch_fill64(reinterpret_cast<uint64_t *>(HT[1]), Tcap, 0ull, cs);
    launch_init_box(b, D, Wd, dbox, dbox + D, cs);
    for (int l = 0; l < nsub; ++l) {
        const int N = mlp->widths[l + 1], K = mlp->widths[l];
        const int64_t *sl = &lg.steps[(size_t)step0[l] * 4];
        const int Vl = (int)sl[0], El = (int)sl[1];
        if (l == 0) launch_gemm(b, ZS, b.X, D, 0, Vl, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], cs);
        else launch_gemm(b, ZS, b.Z, ZS, 1, Vl, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], cs);
        for (int j = 0; j < N; ++j) {
            const int s = step0[l] + j, par = s & 1;
            const int64_t *st4 = &lg.steps[(size_t)s * 4];
            StepGeom g{};
            g.D = D;
            g.Wd = Wd;
            g.ZS = ZS;
            g.Nl = N;
            g.lw0 = lw[l];
            g.lw1 = lw[l + 1];
            g.j = j;
            g.wn = lw[l] + (j >> 5);
            g.bn = 2 * (j & 31);
            g.P = P;
            g.zlo = l == nsub - 1 ? j + 1 : 0;
            g.pair_mode = PAIR_HASH;
            g.HT = HT[par];
            g.HTo = HT[par ^ 1];
            g.step = s;
            g.par = par;
            g.nx8 = 1;
            g.hkeep = ~0ull;
            g.fbits = 64;
            g.Vcap = (int)Vcap;
            g.Ecap = (int)Ecap;
            g.Kcap = (int)Kcap;
            if (j == 0) {
                launch_next_all(b, Vl, Wd, lw[l], lw[l + 1], El, par, s, cs);
                launch_gather(b, El, par, s, cs);
            } else {
                launch_select(b, (uint16_t)j, par, s, select_grid(st4[1]), cs);
            }
            launch_split(b, g, split_blocks((int)st4[2], N), cs);
            launch_hash_pair(b, g, pair_grid(st4[2] * P), cs);
        }
    }
    const hipError_t le = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    gate.unlock();
    if (le != hipSuccess || ce != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();  // a failed capture leaves no error behind for this thread's later calls
        return fail(PCX_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
    }
    ge.graph = graph;
    HIPCHK(hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0));
    ge.D = D;
    ge.Wd = Wd;
    ge.ZS = ZS;
    ge.M = 2 * D + n_steps;
    ge.nsub = nsub;
    ge.n_steps = n_steps;
    return PCX_OK;
}

// one replay on stream st; *ok = the replay reproduced the log
int replay(const GraphLog &lg, GraphEntry &ge, hipStream_t st, hipEvent_t t0, hipEvent_t t1, int *pinned, bool *ok,
           float *ms) {
    *ok = false;
    HIPCHK(hipEventRecord(t0, st));
    HIPCHK(hipGraphLaunch(ge.exec, st));
    HIPCHK(hipEventRecord(t1, st));
    std::vector<StepRec> rec(ge.n_steps);
    HIPCHK(hipMemcpyAsync(pinned, ge.b.CTR, CTR_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(rec.data(), ge.b.REC, rec.size() * sizeof(StepRec), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipEventElapsedTime(ms, t0, t1));
    if (pinned[CTR_FLAGS] || pinned[CTR_PFLAGS]) return PCX_OK;
    const int par = ge.n_steps & 1;
    if (pinned[CTR_V + par] != lg.V || pinned[CTR_E + par] != lg.E) return PCX_OK;
    for (int s = 0; s < ge.n_steps; ++s) {
        const int64_t *st4 = &lg.steps[(size_t)s * 4];
        if (rec[s].V0 != st4[0] || rec[s].E0 != st4[1] || rec[s].S != st4[2] ||
            2 * ((int64_t)rec[s].E1 - rec[s].E0 - rec[s].S) != st4[3])
            return PCX_OK;
    }
    *ok = true;
    return PCX_OK;
}

}  // namespace

int graph_try(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts &o, hipStream_t st,
              hipStream_t cs, hipEvent_t t0, hipEvent_t t1, int *pinned, pcx_complex **out) {
    *out = nullptr;
    if (!eligible(o) || !mlp->gcache) return kGraphDeclined;
    GraphCache &gc = *mlp->gcache;
    std::unique_lock<std::mutex> lk(gc.mu, std::try_to_lock);
    if (!lk.owns_lock()) return kGraphDeclined;  // another thread uses this network's graph
    const int D = mlp->D;
    if (!gc.log || !same_key(*gc.log, D, lo, hi, o.include_output)) return kGraphDeclined;
    int rc;
    if (!gc.entry) {
        // a network requested once or twice runs on the ordinary path; the third request builds
        if (gc.log->seen < 2) return kGraphDeclined;
        auto ge = std::make_unique<GraphEntry>();
        if ((rc = build(mlp, *gc.log, *ge, cs))) {
            if (rc != kGraphBusy) gc.log.reset();  // not this network again
            return kGraphDeclined;
        }
        gc.entry = std::move(ge);
    }
    GraphEntry &ge = *gc.entry;
    const GraphLog &lg = *gc.log;
    bool ok = false;
    float ms = 0.f;
    if ((rc = replay(lg, ge, st, t0, t1, pinned, &ok, &ms))) return rc;
    if (!ok) {
        gc.entry.reset();
        gc.log.reset();
        return kGraphDeclined;
    }
    // the complex gets arrays of its own
    size_t got = 0;
    double *X = (double *)pool().get((size_t)lg.V * D * 8, &got, ~(size_t)0);
    uint64_t *SG = (uint64_t *)pool().get((size_t)lg.V * ge.Wd * 8, &got, ~(size_t)0);
    int2 *EDG = (int2 *)pool().get((size_t)lg.E * 8, &got, ~(size_t)0);
    if (!X || !SG || !EDG) {
        pool().put(X);
        pool().put(SG);
        pool().put(EDG);
        return fail(PCX_ERR_OOM, "complex storage");
    }
    HIPCHK(hipMemcpyAsync(X, ge.b.X, (size_t)lg.V * D * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(SG, ge.b.SG, (size_t)lg.V * ge.Wd * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(EDG, ge.b.EDG, (size_t)lg.E * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    auto *cx = new pcx_complex();
    cx->valid = ge.valid;
    cx->D = D;
    cx->M = ge.M;
    cx->Wd = ge.Wd;
    cx->n_steps = ge.n_steps;
    cx->V = lg.V;
    cx->E = lg.E;
    cx->X = X;
    cx->SG = SG;
    cx->EDG = EDG;
    cx->steps = lg.steps;
    for (int s = 0; s < ge.n_steps; ++s) {
        cx->total_splits += lg.steps[(size_t)s * 4 + 2];
        cx->total_pairs += lg.steps[(size_t)s * 4 + 3] / 2;
    }
    cx->peak = ge.bytes;
    cx->time_ms = ms;
    cx->ZS = ge.ZS;
    cx->nsub = ge.nsub;
    cx->from_graph = 1;
    *out = cx;
    return PCX_OK;
}

void graph_record(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts &o, const pcx_complex *cx,
                  int64_t Ebound, int64_t Smax) {
    if (!eligible(o) || !mlp->gcache || cx->n_steps == 0) return;
    GraphCache &gc = *mlp->gcache;
    std::unique_lock<std::mutex> lk(gc.mu, std::try_to_lock);
    if (!lk.owns_lock()) return;
    if (gc.log && same_key(*gc.log, mlp->D, lo, hi, o.include_output)) {
        ++gc.log->seen;  // (the log itself is the same: the extraction is deterministic)
        return;
    }
    auto lg = std::make_unique<GraphLog>();
    lg->lo.assign(lo, lo + mlp->D);
    lg->hi.assign(hi, hi + mlp->D);
    lg->include_output = o.include_output;
    lg->steps = cx->steps;
    lg->V = cx->V;
    lg->E = cx->E;
    lg->Ebound = Ebound;
    lg->Smax = Smax;
    gc.entry.reset();
    gc.log = std::move(lg);
}

}  // namespace pcx
