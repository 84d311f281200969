// Host side of libpcx.so: the C ABI of include/pcx.h and the orchestration of
// edge subdivision (Berzins 2023, Sec. 4.2) on one GPU. Weights are copied to
// the device once per network; an extraction keeps every array on the device.
// With hash pairing the kernels of a neuron step take their counts from device
// counters, so the host queues steps ahead and reads the counters only every
// few steps (to grow the storage ahead of the complex) and at layer starts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <map>
#include <mutex>
#include <unordered_map>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "host.h"

namespace pcx {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

Pool &pool() {
    static Pool *p = new Pool();  // never destroyed: the runtime may be gone at exit
    return *p;
}

std::shared_mutex &capture_gate() {
    static std::shared_mutex g;
    return g;
}

int copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
    if (!bytes) return PCX_OK;
    thread_local std::unordered_map<int, hipStream_t> *streams = new std::unordered_map<int, hipStream_t>();
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipStream_t &s = (*streams)[dev];
    if (!s) {
        std::shared_lock<std::shared_mutex> gate(capture_gate());
        HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    }
    HIPCHK(hipMemcpyAsync(dst, src, bytes, kind, s));
    HIPCHK(hipStreamSynchronize(s));
    return PCX_OK;
}

}  // namespace pcx

using namespace pcx;

namespace {

struct EventPool {
    std::vector<hipEvent_t> free_, all_;
    struct Pending { hipEvent_t a, b; int fam; };
    std::vector<Pending> pend;
    hipEvent_t get() {
        if (free_.empty()) {
            hipEvent_t e;
            // timing only: no system-scope fence, which would write back the
            // caches between the kernels it separates
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            all_.push_back(e);
            return e;
        }
        hipEvent_t e = free_.back();
        free_.pop_back();
        return e;
    }
    ~EventPool() {
        for (auto e : all_) (void)hipEventDestroy(e);
    }
};

// Pinned counter buffers and events of one thread on one device, kept for the
// thread's later extractions: creating them costs more than a small
// extraction does. (Never released: the runtime may be gone at thread exit.)
struct HostRes {
    int *pinned = nullptr;  // [3][CTR_COUNT]: counters after a drain, two snapshots
    hipEvent_t snap[2] = {nullptr, nullptr}, t0 = nullptr, t1 = nullptr;
    hipStream_t cap = nullptr;  // stream on which graphs are captured
    bool busy = false;
};

int host_res(HostRes *&out) {
    thread_local std::unordered_map<int, HostRes *> *per_dev = new std::unordered_map<int, HostRes *>();
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HostRes *&r = (*per_dev)[dev];
    if (!r) {
        std::shared_lock<std::shared_mutex> gate(capture_gate());
        auto *n = new HostRes();
        HIPCHK(hipHostMalloc((void **)&n->pinned, 3 * CTR_COUNT * sizeof(int), hipHostMallocDefault));
        for (int i = 0; i < 2; ++i) HIPCHK(hipEventCreateWithFlags(&n->snap[i], hipEventDisableTiming));
        HIPCHK(hipEventCreate(&n->t0));
        HIPCHK(hipEventCreate(&n->t1));
        HIPCHK(hipStreamCreateWithFlags(&n->cap, hipStreamNonBlocking));
        r = n;
    }
    if (r->busy) return fail(PCX_ERR_DEVICE, "internal error: nested extraction on one thread");
    out = r;
    return PCX_OK;
}

struct Extraction {
    const pcx_mlp *mlp;
    hipStream_t st;
    int timing_mask = 0;
    Arena arena;
    Bufs b{};
    size_t Vcap = 0, Ecap = 0, Scap = 0, Kcap = 0, Hcap = 0, Xcap = 0;
    int pair_mode = PAIR_HASH;
    unsigned long long *HT[2] = {nullptr, nullptr};  // 2-face hash tables, alternating by step
    size_t Tcap = 0;                                 // words per table
    bool tape = false;
    bool prune = false;
    int D = 0, Wd = 0, ZS = 0, P = 0;
    int *hctr = nullptr;     // pinned: the counters after a drain
    int *hsnap[2] = {};      // pinned: counter snapshots taken ahead of the host
    hipEvent_t evsnap[2] = {};
    int snap_at[2] = {-1, -1};  // step before which each pending snapshot was taken
    int snap_next = 0;
    bool tables_reset = false;  // the hash tables were reallocated (zeroed)
    EventPool ev;
    double ktime[PCX_K_COUNT] = {};
    int64_t klaunch[PCX_K_COUNT] = {};

    HostRes *res = nullptr;  // borrowed: the thread's pinned counters and events

    ~Extraction() {
        if (res) res->busy = false;
    }
    int attach_host() {
        int rc;
        if ((rc = host_res(res))) return rc;
        res->busy = true;
        hctr = res->pinned;
        hsnap[0] = res->pinned + CTR_COUNT;
        hsnap[1] = res->pinned + 2 * CTR_COUNT;
        evsnap[0] = res->snap[0];
        evsnap[1] = res->snap[1];
        return PCX_OK;
    }

    // every enqueued kernel done; hctr = the device counters
    int drain() {
        HIPCHK(hipMemcpyAsync(hctr, b.CTR, CTR_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        snap_at[0] = snap_at[1] = -1;
        return collect();
    }
    // set one device counter (between drains: nothing else is in flight)
    int put_ctr(int idx, int v) {
        hctr[idx] = v;
        HIPCHK(hipMemcpyAsync(b.CTR + idx, hctr + idx, sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return PCX_OK;
    }

    int mark(int fam, bool start) {
        if (!(timing_mask & (1 << fam))) return PCX_OK;
        hipEvent_t e = ev.get();
        if (!e) return fail(PCX_ERR_DEVICE, "hipEventCreate failed");
        HIPCHK(hipEventRecord(e, st));
        if (start) {
            ev.pend.push_back({e, nullptr, fam});
        } else {
            ev.pend.back().b = e;
        }
        return PCX_OK;
    }
    // the two events of one timed launch that records them itself (its start
    // and end, with no packets between it and its neighbours), or nulls
    int launch_events(int fam, hipEvent_t &a, hipEvent_t &e) {
        a = e = nullptr;
        if (!(timing_mask & (1 << fam))) return PCX_OK;
        a = ev.get();
        e = ev.get();
        if (!a || !e) return fail(PCX_ERR_DEVICE, "hipEventCreate failed");
        ev.pend.push_back({a, e, fam});
        return PCX_OK;
    }
    int collect() {  // after a stream synchronisation
        for (auto &p : ev.pend) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
            ktime[p.fam] += ms;
            klaunch[p.fam] += 1;
            ev.free_.push_back(p.a);
            ev.free_.push_back(p.b);
        }
        ev.pend.clear();
        return PCX_OK;
    }

    // grow an array whose first `used` elements must survive
    template <class T>
    int grow_keep(T *&p, size_t &cap, size_t need, size_t used, size_t per) {
        if (need <= cap) return PCX_OK;
        size_t nc = std::max(need, cap + cap / 2);
        void *q;
        int rc = arena.alloc(&q, nc * per * sizeof(T));
        if (rc) return rc;
        if (p && used) HIPCHK(hipMemcpyAsync(q, p, used * per * sizeof(T), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        arena.release(p);
        p = (T *)q;
        cap = nc;
        return PCX_OK;
    }
    template <class T>
    int grow_scratch(T *&p, size_t cap, size_t nc) {  // contents need not survive
        if (p) HIPCHK(hipStreamSynchronize(st));
        arena.release(p);
        void *q;
        int rc = arena.alloc(&q, nc * sizeof(T));
        if (rc) return rc;
        p = (T *)q;
        (void)cap;
        return PCX_OK;
    }

    int ensure_vertices(size_t need, size_t used) {
        if (need <= Vcap) return PCX_OK;
        size_t c0 = Vcap, c1 = Vcap, c2 = Vcap;
        int rc;
        if ((rc = grow_keep(b.X, c0, need, used, (size_t)D))) return rc;
        if ((rc = grow_keep(b.SG, c1, need, used, (size_t)Wd))) return rc;
        if ((rc = grow_keep(b.Z, c2, need, used, (size_t)ZS))) return rc;
        if (tape) {
            size_t c3 = Vcap;
            if ((rc = grow_keep(b.PQ, c3, need, used, 1))) return rc;
            c2 = std::min(c2, c3);
        }
        Vcap = std::min(c0, std::min(c1, c2));
        return PCX_OK;
    }
    // spl_used: split ids already written by this step's compaction (kept)
    int ensure_edges(size_t need, size_t used, size_t spl_used) {
        if (need <= Ecap) return PCX_OK;
        size_t c0 = Ecap, c1 = Ecap;
        int rc;
        if ((rc = grow_keep(b.EDG, c0, need, used, 1))) return rc;
        if ((rc = grow_keep(b.NX8, c1, need, used, 1))) return rc;
        Ecap = std::min(c0, c1);
        if ((rc = grow_scratch(b.SPLX, Ecap, Ecap))) return rc;  // chunk match lists: edge capacity
        // the compaction writes up to E split ids before the host learns S,
        // so the split list always has the edge capacity
        if (Ecap > Scap) {
            size_t c2 = Scap;
            if ((rc = grow_keep(b.SPLE, c2, Ecap, spl_used, 1))) return rc;
            Scap = c2;
        }
        return PCX_OK;
    }
    int ensure_hist(size_t K) {
        size_t h = (size_t)kSortBins * ((K + kSortTile - 1) / kSortTile + 1);
        if (h > Hcap) {
            size_t nc = std::max(h, Hcap * 2);
            int rc;
            if ((rc = grow_scratch(b.HIST, Hcap, nc))) return rc;
            Hcap = nc;
        }
        return PCX_OK;
    }
    int ensure_step(size_t S, size_t K) {
        int rc;
        if (S > Scap) return fail(PCX_ERR_DEVICE, "split list smaller than the split count");
        if (K > Kcap) {
            size_t nc = std::max(K, Kcap * 2);
            if (pair_mode == PAIR_SORT) {
                if ((rc = grow_scratch(b.K32a, Kcap, nc))) return rc;
                if ((rc = grow_scratch(b.K32b, Kcap, nc))) return rc;
                if ((rc = grow_scratch(b.VALa, Kcap, nc))) return rc;
                if ((rc = grow_scratch(b.VALb, Kcap, nc))) return rc;
                if ((rc = grow_scratch(b.FULL, Kcap, nc))) return rc;
            }
            if ((rc = grow_scratch(b.PINFO, Kcap, nc))) return rc;
            // partner records start untagged (no step has written them)
            if ((rc = grow_scratch(b.PART, Kcap, nc))) return rc;
            launch_fill64(b.PART, nc, 0ull, st);
            Kcap = nc;
            Xcap = 0;  // the exact pass's keys follow the key capacity
        }
        if (pair_mode == PAIR_HASH) {
            size_t tc = 256;
            while (tc < 2 * Kcap) tc <<= 1;
            if (tc > Tcap) {
                for (int t = 0; t < 2; ++t) {
                    if ((rc = grow_scratch(HT[t], Tcap, tc))) return rc;
                    launch_fill64(reinterpret_cast<uint64_t *>(HT[t]), tc, 0ull, st);
                }
                Tcap = tc;
                tables_reset = true;
            }
            return PCX_OK;
        }
        return ensure_hist(K);
    }
    // the exact pass of a step with K key slots (K <= Kcap)
    int ensure_exact(size_t K) {
        int rc;
        if (Xcap < Kcap) {
            if ((rc = grow_scratch(b.K64a, Xcap, Kcap))) return rc;
            if ((rc = grow_scratch(b.K64b, Xcap, Kcap))) return rc;
            if (pair_mode == PAIR_HASH) {
                if ((rc = grow_scratch(b.VALa, Xcap, Kcap))) return rc;
                if ((rc = grow_scratch(b.VALb, Xcap, Kcap))) return rc;
            }
            Xcap = Kcap;
        }
        return ensure_hist(K);
    }
};

// Pruning (Sec. 5.4.2): the signs of the neurons of the later layers (the
// output included) at every current vertex, written into their sign words by
// the evaluation, in chunks of rows through two scratch buffers.
int future_signs(Extraction &x, const pcx_mlp *mlp, int l, int nsub, int64_t V, const std::vector<int> &lw) {
    if (l + 1 >= nsub || V == 0) return PCX_OK;
    const int ZS = x.ZS, Wd = x.Wd;
    const int64_t chunk = std::min<int64_t>(V, 1 << 20);
    void *q[2];
    int rc;
    if ((rc = x.arena.alloc(&q[0], (size_t)chunk * ZS * sizeof(double)))) return rc;
    if ((rc = x.arena.alloc(&q[1], (size_t)chunk * ZS * sizeof(double)))) return rc;
    for (int64_t c0 = 0; c0 < V; c0 += chunk) {
        const int n = (int)std::min(chunk, V - c0);
        const double *src = x.b.Z + (size_t)c0 * ZS;
        for (int m = l + 1; m < nsub; ++m) {
            Bufs bb = x.b;
            bb.LW = nullptr;
            bb.Z = (double *)q[m & 1];
            bb.SG = x.b.SG + (size_t)c0 * Wd;
            launch_gemm(bb, ZS, src, ZS, 1, n, mlp->widths[m], mlp->widths[m + 1], mlp->Wt[m], mlp->b[m], Wd, lw[m],
                        x.st);
            src = bb.Z;
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(x.st));
    x.arena.release(q[0]);
    x.arena.release(q[1]);
    return PCX_OK;
}

// Drop the edges whose vertices agree on every sign word from lwf on, then the
// vertices left without an edge; survivors keep their order. V, E are the
// exact counts (after a drain); the new ones go to the counters of parity par.
int prune_now(Extraction &x, int64_t &V, int64_t &E, int lwf, int par) {
    if (V == 0) return PCX_OK;
    hipStream_t st = x.st;
    void *pm, *pmap, *pe, *px, *ps, *pz;
    int rc;
    if ((rc = x.arena.alloc(&pm, (size_t)V))) return rc;
    if ((rc = x.arena.alloc(&pmap, (size_t)V * sizeof(int)))) return rc;
    if ((rc = x.arena.alloc(&pe, x.Ecap * sizeof(int2)))) return rc;
    HIPCHK(hipMemsetAsync(pm, 0, (size_t)V, st));
    launch_prune_edges(x.b, (int)V, (int)E, x.Wd, lwf, (int2 *)pe, (uint8_t *)pm, par, st);
    launch_prune_vertices(x.b, (int)V, (const uint8_t *)pm, (int *)pmap, par, st);
    HIPCHK(hipGetLastError());
    if ((rc = x.drain())) return rc;
    if (x.hctr[CTR_FLAGS]) return degenerate_message(x.hctr[CTR_FLAGS]);
    const int64_t Vn = x.hctr[CTR_V + par], En = x.hctr[CTR_E + par];
    if ((rc = x.arena.alloc(&px, x.Vcap * (size_t)x.D * sizeof(double)))) return rc;
    if ((rc = x.arena.alloc(&ps, x.Vcap * (size_t)x.Wd * sizeof(uint64_t)))) return rc;
    if ((rc = x.arena.alloc(&pz, x.Vcap * (size_t)x.ZS * sizeof(double)))) return rc;
    launch_move_rows(x.b, (const uint8_t *)pm, (const int *)pmap, (int)V, x.D, x.Wd, x.ZS, (double *)px,
                     (uint64_t *)ps, (double *)pz, (int2 *)pe, (int)En, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    x.arena.release(x.b.X);
    x.arena.release(x.b.SG);
    x.arena.release(x.b.Z);
    x.arena.release(x.b.EDG);
    x.arena.release(pm);
    x.arena.release(pmap);
    x.b.X = (double *)px;
    x.b.SG = (uint64_t *)ps;
    x.b.Z = (double *)pz;
    x.b.EDG = (int2 *)pe;
    V = Vn;
    E = En;
    return PCX_OK;
}

}  // namespace

namespace pcx {
int degenerate_message(int flags) {
    std::string m = "input is not generic:";
    if (flags & FLAG_ZERO_SIGN) m += " a vertex lies on a hyperplane;";
    if (flags & FLAG_CONFLICT) m += " sign conflict on an edge;";
    if (flags & FLAG_ZERO_COUNT) m += " a splitting edge without D-1 zeros;";
    if (flags & FLAG_RUN) m += " a 2-face not met by exactly two splitting edges;";
    if (flags & FLAG_VERIFY) m += " 2-face hashes equal but sign-vectors differ;";
    if (flags & FLAG_BOUNDS) return fail(PCX_ERR_DEVICE, "internal error: a kernel saw an index out of range");
    return fail(PCX_ERR_DEGENERATE, m);
}
}  // namespace pcx

extern "C" {

const char *pcx_last_error(void) { return g_err.c_str(); }

int pcx_mlp_create(int32_t n_layers, const int32_t *widths, const double *const *W, const double *const *b,
                   pcx_mlp **out) {
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n_layers < 1 || !widths || !W || !b) return fail(PCX_ERR_INVALID, "bad network description");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1) return fail(PCX_ERR_INVALID, "every width must be >= 1");
    if (widths[0] > 16) return fail(PCX_ERR_INVALID, "input dimension D must be 1..16");
    pcx_mlp *m = new pcx_mlp();
    m->gcache = graph_cache_new();
    m->L = n_layers;
    m->D = widths[0];
    m->widths.assign(widths, widths + n_layers + 1);
    std::vector<double> tmp;
    for (int l = 0; l < n_layers; ++l) {
        const int nin = widths[l], nout = widths[l + 1];
        if (!W[l] || !b[l]) {
            pcx_mlp_free(m);
            return fail(PCX_ERR_INVALID, "NULL weight or bias pointer");
        }
        tmp.resize((size_t)nin * nout);
        for (int i = 0; i < nout; ++i)
            for (int k = 0; k < nin; ++k) tmp[(size_t)k * nout + i] = W[l][(size_t)i * nin + k];
        double *dw = nullptr, *db = nullptr, *dr = nullptr;
        bool ok;
        {
            std::shared_lock<std::shared_mutex> gate(capture_gate());
            ok = hipMalloc((void **)&dw, tmp.size() * sizeof(double)) == hipSuccess &&
                 hipMalloc((void **)&db, (size_t)nout * sizeof(double)) == hipSuccess &&
                 hipMalloc((void **)&dr, tmp.size() * sizeof(double)) == hipSuccess;
            if (!ok) (void)hipGetLastError();
        }
        // (pcx_mlp_free takes the gate itself: it is not held here)
        if (dw) m->Wt.push_back(dw);
        if (db) m->b.push_back(db);
        if (dr) m->Wr.push_back(dr);
        if (!ok) {
            pcx_mlp_free(m);
            return fail(PCX_ERR_OOM, "hipMalloc for weights failed");
        }
        if (copy_sync(dw, tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice) ||
            copy_sync(dr, W[l], tmp.size() * sizeof(double), hipMemcpyHostToDevice) ||
            copy_sync(db, b[l], (size_t)nout * sizeof(double), hipMemcpyHostToDevice)) {
            pcx_mlp_free(m);
            return fail(PCX_ERR_DEVICE, "copying weights to the device failed");
        }
    }
    *out = m;
    return PCX_OK;
}

void pcx_mlp_free(pcx_mlp *m) {
    if (!m) return;
    graph_cache_free(m->gcache);
    std::shared_lock<std::shared_mutex> gate(capture_gate());
    for (auto p : m->Wt) (void)hipFree(p);
    for (auto p : m->Wr) (void)hipFree(p);
    for (auto p : m->b) (void)hipFree(p);
    delete m;
}

}  // extern "C"

namespace {

// The domain of Sec. 4.1: m half-spaces (the first m sign entries, all in word
// 0) and its 1-skeleton. The box is generated on the device from lo / hi; any
// other domain brings its vertices (coordinates and word 0) and edges.
struct Domain {
    int m = 0;
    const double *lo = nullptr, *hi = nullptr;  // the box
    std::vector<double> X0;                     // [nv][D]
    std::vector<uint64_t> W0;                   // [nv] word 0 of each vertex
    std::vector<int2> E0;                       // [ne]
};

// Small networks go to the batched kernel as a batch of one: one launch
// instead of several per neuron step, the same complex (PCX_NO_TINY=1 in the
// environment turns it off). Up to which predicted vertex count, by input
// dimension: where one workgroup stops being faster than the per-step kernels
// (measured crossovers near 10,000 actual vertices for D = 2 and 2,800 for
// D = 3; for D >= 4 the per-step kernels were faster at nearly every size tried).
double tiny_vertices(int D) { return D <= 2 ? 15000.0 : D == 3 ? 3500.0 : 0.0; }
bool tiny_eligible(const pcx_mlp *mlp, const pcx_opts &o, int nsub) {
    const char *off = getenv("PCX_NO_TINY");
    if (off && off[0] == '1') return false;
    if (o.pairing != PCX_PAIR_HASH || o.prune || o.record_tape || o.timing || o.max_bytes) return false;
    if (mlp->D > kBatchMaxD || mlp->L > kBatchMaxLayers) return false;
    int N = 0, Wd = 1;
    for (int l = 1; l <= nsub; ++l) {
        if (mlp->widths[l] > kMaxWidth) return false;
        N += mlp->widths[l];
        Wd += (mlp->widths[l] + 31) / 32;
    }
    double limit = tiny_vertices(mlp->D);
    if (const char *v = getenv("PCX_TINY_VERTICES")) limit = atof(v);
    return Wd <= kBatchMaxWords && N > 0 && predict_vertices(mlp->D, N) <= limit;
}

int extract_impl(const pcx_mlp *mlp, const Domain &dom, const pcx_opts *opts, pcx_complex **out,
                 int shortcuts = 0) {
    pcx_opts o{};
    if (opts) o = *opts;
    const int D = mlp->D, L = mlp->L;
    const int nsub = o.include_output ? L : L - 1;
    if ((shortcuts & kShortcutTiny) && dom.lo && tiny_eligible(mlp, o, nsub))
        return tiny_extract(mlp, dom.lo, dom.hi, o, out);
    std::vector<int> lw(nsub + 1);
    lw[0] = 1;
    int M = dom.m, ZS = 1, n_steps = 0;
    for (int l = 0; l < nsub; ++l) {
        const int N = mlp->widths[l + 1];
        if (N > kMaxWidth) return fail(PCX_ERR_INVALID, "subdivided layers wider than 256 are not supported");
        if (N >= (int)kNone) return fail(PCX_ERR_INVALID, "layer too wide");
        lw[l + 1] = lw[l] + (N + 31) / 32;
        M += N;
        ZS = std::max(ZS, N);
        n_steps += N;
    }
    const int Wd = lw[nsub];

    Extraction x;
    x.mlp = mlp;
    x.st = (hipStream_t)o.stream;
    x.timing_mask = o.timing;
    x.arena.cap = o.max_bytes;
    x.D = D;
    x.Wd = Wd;
    x.ZS = ZS;
    x.P = D >= 2 ? 2 * (D - 1) : 0;
    if (o.pairing != PCX_PAIR_HASH && o.pairing != PCX_PAIR_SORT) return fail(PCX_ERR_INVALID, "unknown pairing");
    x.pair_mode = o.pairing == PCX_PAIR_SORT ? PAIR_SORT : PAIR_HASH;
    x.tape = o.record_tape != 0;
    x.prune = o.prune != 0;
    if (x.prune && !o.include_output) return fail(PCX_ERR_INVALID, "pruning needs include_output (the level set)");
    if (x.prune && x.tape) return fail(PCX_ERR_INVALID, "pruning and record_tape cannot be combined");
    std::vector<double *> tapeZ;
    hipStream_t st = x.st;
    int rc;

    // host-side tables
    std::vector<uint64_t> valid(Wd, 0);
    for (int e = 0; e < dom.m; ++e) valid[0] |= 1ull << (2 * e);
    for (int l = 0; l < nsub; ++l)
        for (int c = 0; c < mlp->widths[l + 1]; ++c) valid[lw[l] + (c >> 5)] |= 1ull << (2 * (c & 31));

    const bool box = dom.lo != nullptr;
    const size_t V0 = box ? (size_t)1 << D : dom.W0.size(), E0 = box ? (size_t)D << (D - 1) : dom.E0.size();
    if ((rc = x.attach_host())) return rc;
    if ((shortcuts & kShortcutGraph) && dom.lo) {
        // a repeat of the network's last extraction: its captured graph
        rc = graph_try(mlp, dom.lo, dom.hi, o, st, x.res->cap, x.res->t0, x.res->t1, x.res->pinned, out);
        if (rc != kGraphDeclined) return rc;
    }
    {
        void *p;
        if ((rc = x.arena.alloc(&p, CTR_COUNT * sizeof(int)))) return rc;
        x.b.CTR = (int *)p;
        if ((rc = x.arena.alloc(&p, Wd * sizeof(uint64_t)))) return rc;
        x.b.VALID = (const uint64_t *)p;
        HIPCHK(hipMemcpyAsync(p, valid.data(), Wd * sizeof(uint64_t), hipMemcpyHostToDevice, st));
        if ((rc = x.arena.alloc(&p, (size_t)kNextBlocks * sizeof(int)))) return rc;
        x.b.SELCNT = (int *)p;
    }
    double *dbox = nullptr;
    if (box) {
        void *p;
        if ((rc = x.arena.alloc(&p, 2 * D * sizeof(double)))) return rc;
        dbox = (double *)p;
        HIPCHK(hipMemcpyAsync(dbox, dom.lo, D * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(dbox + D, dom.hi, D * sizeof(double), hipMemcpyHostToDevice, st));
    }
    // Initial storage: the sizes this network reached before, else (a first
    // extraction) the fitted vertex predictor with half again as margin, as
    // long as that stays small (about E = D V edges and D V / N splits per
    // step); growth and redone steps cover the rest.
    // (PCX_SMALL_START=1 starts from the minimum instead: a test hook for the
    // growth path)
    const char *small_env = getenv("PCX_SMALL_START");
    const bool small_start = small_env && small_env[0] == '1';
    // (PCX_FULL_GRIDS=1 launches every step's compaction, split and pairing with
    // their largest grids, the launch shape of the big steps of large complexes:
    // a test hook that runs a complex the oracle can check through that shape)
    const char *fg_env = getenv("PCX_FULL_GRIDS");
    const bool full_grids = fg_env && fg_env[0] == '1';
    // (PCX_DEBUG_HASH_BITS=b keeps only b bits of every 2-face hash, and
    // PCX_DEBUG_EXACT_BITS=b of the exact pass's sort keys: collisions on
    // purpose, test hooks for the exact pass and its grouping)
    auto env_bits = [](const char *name) {
        const char *v = getenv(name);
        const int b = v ? atoi(v) : 64;
        return b >= 1 && b < 64 ? b : 64;
    };
    const int hbits = env_bits("PCX_DEBUG_HASH_BITS"), fbits = env_bits("PCX_DEBUG_EXACT_BITS");
    size_t Vinit = std::max<size_t>({V0, 1024, small_start ? 0 : (size_t)mlp->hintV.load()});
    size_t Einit = std::max<size_t>({E0, 4096, small_start ? 0 : (size_t)mlp->hintE.load()});
    size_t Sinit = small_start ? 0 : (size_t)mlp->hintS.load();
    if (!small_start && mlp->hintV.load() == 0 && n_steps > 0) {
        const double pv = 1.5 * predict_vertices(D, n_steps);
        const double per_v = 8.0 * (D + Wd + ZS) + (double)std::max(1, D) * (8 + 1 + 16 + 4);
        // (within a quarter of a byte cap, so a cap that fits the complex is never hit by the margin)
        if (pv * per_v <= 4.0e9 && (o.max_bytes == 0 || 4.0 * pv * per_v <= (double)o.max_bytes)) {
            Vinit = std::max(Vinit, (size_t)pv);
            Einit = std::max(Einit, (size_t)(pv * std::max(1, D)));
            Sinit = std::max(Sinit, (size_t)(2.0 * pv * std::max(1, D) / n_steps) + 256);
        }
    }
    if ((rc = x.ensure_vertices(Vinit, 0))) return rc;
    if ((rc = x.ensure_edges(Einit, 0, 0))) return rc;
    {
        int h[CTR_COUNT] = {0};
        h[CTR_V] = (int)V0;
        h[CTR_E] = (int)E0;
        h[CTR_FAIL] = 0x7fffffff;
        h[CTR_PFAIL] = 0x7fffffff;
        std::memcpy(x.hctr, h, sizeof h);
        HIPCHK(hipMemcpyAsync(x.b.CTR, x.hctr, sizeof h, hipMemcpyHostToDevice, st));
    }

    hipEvent_t t0 = x.res->t0, t1 = x.res->t1;
    HIPCHK(hipEventRecord(t0, st));
    std::vector<uint64_t> rows0;
    if (box) {
        launch_init_box(x.b, D, Wd, dbox, dbox + D, st);
    } else {
        rows0.assign(V0 * (size_t)Wd, 0ull);
        for (size_t v = 0; v < V0; ++v) rows0[v * Wd] = dom.W0[v];
        HIPCHK(hipMemcpyAsync(x.b.X, dom.X0.data(), V0 * D * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(x.b.SG, rows0.data(), rows0.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(x.b.EDG, dom.E0.data(), E0 * sizeof(int2), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));  // the host vectors are not kept
    }
    HIPCHK(hipGetLastError());

    std::vector<int64_t> steps((size_t)n_steps * 4, 0);
    std::vector<int> step0(nsub + 1, 0);
    for (int l = 0; l < nsub; ++l) step0[l + 1] = step0[l] + mlp->widths[l + 1];
    if (n_steps > 0) {
        void *p;
        if ((rc = x.arena.alloc(&p, (size_t)n_steps * sizeof(StepRec)))) return rc;
        x.b.REC = (StepRec *)p;
    }
    // Hash pairing runs ahead of the host: every count a kernel needs is on the
    // device, and the host looks at the counters every kAhead steps (a
    // snapshot taken kAhead steps earlier, so the queue never runs dry). A step
    // that finds the storage too small writes nothing, every later kernel
    // returns at once, and the host grows the storage (geometrically, from the
    // exact counts) and redoes that step. The storage starts at the sizes of
    // the network's earlier extractions, so a repeated extraction never grows.
    // Sort pairing sizes its radix sort on the host and reads the counters at
    // every step.
    const bool lagged = x.pair_mode == PAIR_HASH;
    constexpr int kAhead = 8;
    const int64_t Shint = std::min<int64_t>((int64_t)Sinit, (int64_t)x.Scap);
    if ((rc = x.ensure_step((size_t)Shint, (size_t)Shint * x.P))) return rc;
    x.tables_reset = false;  // new tables are zero, and so are the counters
    int64_t V = (int64_t)V0, E = (int64_t)E0;
    int64_t Sgrid = 64;  // split count the split launch is shaped for (any count is covered)
    int64_t Eseen = 0;   // latest edge count the host has seen (a lower bound: shapes the compaction)
    int64_t prevE = -1, prevS = 0;  // sort pairing: the host's own step log
    bool pairs_logged = false;      //   the previous step's pair count was taken at a layer start
    const char *verbose_env = getenv("PCX_VERBOSE");
    const bool verbose = verbose_env && verbose_env[0] == '1';
    int redone = 0;

    // grow the storage for `ahead` more steps of up to Sx splits each from the
    // exact counts Vx, Ex (after a drain); spl_used: split ids the current
    // step's compaction already wrote (kept)
    auto grow_for = [&](int64_t Vx, int64_t Ex, int64_t Sx, int ahead, size_t spl_used = 0) -> int {
        int r;
        const int64_t Vneed = Vx + (int64_t)ahead * Sx, Eneed = Ex + (int64_t)ahead * Sx * std::max(1, D);
        if (Vneed >= INT32_MAX || Eneed >= INT32_MAX)
            return fail(PCX_ERR_CAPACITY, "complex exceeds 2^31 vertices or edges");
        if ((r = x.ensure_vertices((size_t)Vneed, (size_t)Vx))) return r;
        if ((r = x.ensure_edges((size_t)Eneed, (size_t)Ex, spl_used))) return r;
        if ((r = x.ensure_step((size_t)Sx, (size_t)Sx * x.P))) return r;
        if (x.tables_reset) {
            x.tables_reset = false;
            if ((r = x.put_ctr(CTR_TUSED, 0)) || (r = x.put_ctr(CTR_TUSED + 1, 0))) return r;
        }
        return PCX_OK;
    };
    // the geometry of neuron j of subdivided layer l (global step s)
    auto geom = [&](int l, int j) {
        const int s = step0[l] + j, par = s & 1;
        StepGeom g{};
        g.D = D;
        g.Wd = Wd;
        g.ZS = ZS;
        g.Nl = mlp->widths[l + 1];
        g.lw0 = lw[l];
        g.lw1 = lw[l + 1];
        g.j = j;
        g.wn = lw[l] + (j >> 5);
        g.bn = 2 * (j & 31);
        g.P = x.P;
        // in the last subdivided layer nothing reads the processed columns again
        g.zlo = (l == nsub - 1 && !x.tape) ? j + 1 : 0;
        g.pair_mode = x.pair_mode;
        g.hmask = 0;
        g.HT = x.HT[par];
        g.HTo = x.HT[par ^ 1];
        g.step = s;
        g.par = par;
        g.nx8 = 1;
        g.hkeep = hbits < 64 ? (1ull << hbits) - 1ull : ~0ull;
        g.fbits = fbits;
        g.verify = o.verify_pairs ? 1 : 0;
        g.Vcap = (int)std::min<size_t>(x.Vcap, INT32_MAX);
        g.Ecap = (int)std::min<size_t>(x.Ecap, INT32_MAX);
        g.Kcap = (int)std::min<size_t>(x.Kcap, INT32_MAX);
        return g;
    };
    auto layer_of = [&](int s) { return (int)(std::upper_bound(step0.begin(), step0.end(), s) - step0.begin()) - 1; };
    int exact_steps = 0;
    // after a drain, act on the device flags. A step that found the storage too
    // small is redone from its compaction once the storage fits it (next = that
    // step). A step whose pairing failed has its pairing redone by the exact
    // pass, and work resumes after it (next = the following step; fresh: that
    // step starts a layer not yet begun, or is the end). next = -1: nothing to do.
    auto recover = [&](int &next, bool &fresh) -> int {
        next = -1;
        fresh = false;
        const int flags = x.hctr[CTR_FLAGS], pflags = x.hctr[CTR_PFLAGS];
        if (!flags && !pflags) return PCX_OK;
        if (flags & ~FLAG_CAPACITY) return degenerate_message((flags & ~FLAG_CAPACITY) | pflags);
        int r;
        if (flags) {
            // (a step that found the storage too small wrote nothing, and no later step ran)
            const int f = x.hctr[CTR_FAIL];
            if (f < 0 || f >= n_steps) return fail(PCX_ERR_DEVICE, "internal error: bad failing step");
            const int64_t Sf = x.hctr[CTR_S], Vf = x.hctr[CTR_V + (f & 1)], Ef = x.hctr[CTR_E + (f & 1)];
            V = Vf;  // a redone first step of a layer rescans the edges from these counts
            E = Ef;
            // exactly what step f needs: each array that is short grows by half
            if ((r = grow_for(Vf, Ef, Sf, 1))) return r;
            if ((r = x.put_ctr(CTR_FAIL, 0x7fffffff)) || (r = x.put_ctr(CTR_FLAGS, 0))) return r;
            next = f;
            ++redone;
            return PCX_OK;
        }
        if (pflags & ~kPairFlags) return fail(PCX_ERR_DEVICE, "internal error: unknown pairing flag");
        // the pairing of step pf failed; its split is complete and no later step ran
        const int pf = x.hctr[CTR_PFAIL];
        if (pf < 0 || pf >= n_steps) return fail(PCX_ERR_DEVICE, "internal error: bad failing pairing step");
        const int lf = layer_of(pf);
        StepGeom g = geom(lf, pf - step0[lf]);
        const int64_t nslots = (int64_t)x.hctr[CTR_S] * x.P;
        if (nslots > (int64_t)x.Kcap) return fail(PCX_ERR_DEVICE, "internal error: key slots beyond the storage");
        if ((r = x.put_ctr(CTR_PFLAGS, 0)) || (r = x.put_ctr(CTR_PFAIL, 0x7fffffff))) return r;
        if ((r = x.ensure_exact((size_t)nslots))) return r;
        const int grid = full_grids ? kSelBlocks : pair_grid(nslots);
        launch_exact_pair(x.b, g, (int)nslots, grid, st);
        HIPCHK(hipGetLastError());
        if ((r = x.drain())) return r;
        if (x.hctr[CTR_FLAGS] || x.hctr[CTR_PFLAGS])
            return degenerate_message(x.hctr[CTR_FLAGS] | x.hctr[CTR_PFLAGS]);
        ++exact_steps;
        if (verbose) {
            fprintf(stderr, "[pcx] step %d paired by the exact pass (flags %d)\n", pf, pflags);
            fflush(stderr);
        }
        next = pf + 1;
        fresh = next == n_steps || next == step0[layer_of(next)];
        return PCX_OK;
    };

    int l = 0, j = 0;
    bool started = false;
    while (true) {
        if (!started) {
            // layer start (or the end): every enqueued step is done
            if ((rc = x.drain())) return rc;
            int f;
            bool fresh;
            if ((rc = recover(f, fresh))) return rc;
            if (f >= 0) {
                if (fresh) {
                    // resume at the start of a layer (or the end): this layer start again
                    l = f >= n_steps ? nsub : layer_of(f);
                    continue;
                }
                // the step to continue from belongs to the layer just finished
                l = layer_of(f);
                j = f - step0[l];
                started = true;
                continue;
            }
            // the previous layer's word copies are no longer read
            if (x.b.LW) {
                x.arena.release(x.b.LW);
                x.b.LW = nullptr;
            }
            if (l == nsub) break;
            const int par0 = step0[l] & 1;
            V = x.hctr[CTR_V + par0];
            E = x.hctr[CTR_E + par0];
            Eseen = 0;
            // launch shape from the previous step's count until this layer's own largest is known
            const int64_t Slast = step0[l] > 0 ? x.hctr[CTR_S] : 0;
            Sgrid = Slast + Slast / 4 + 64;
            if (lagged && (rc = x.put_ctr(CTR_SMAX, 0))) return rc;
            if (!lagged && step0[l] > 0) {
                // before pruning can change the edge count
                steps[(size_t)(step0[l] - 1) * 4 + 3] = 2 * (E - prevE - prevS);
                pairs_logged = true;
            }
            const int N = mlp->widths[l + 1], K = mlp->widths[l];
            if (verbose) {
                fprintf(stderr, "[pcx] layer %d start: V=%lld E=%lld device bytes=%llu peak=%llu\n", l + 1,
                        (long long)V, (long long)E, (unsigned long long)x.arena.cur,
                        (unsigned long long)x.arena.peak);
                fflush(stderr);
            }
            // the evaluation also keeps the layer's sign words in 64-byte rows for the
            // layer-start scan (not with pruning, which renumbers the vertices after it)
            if (!x.prune) {
                void *q;
                if ((rc = x.arena.alloc(&q, (size_t)std::max<int64_t>(V, 1) * 8 * sizeof(uint64_t)))) return rc;
                x.b.LW = (uint64_t *)q;
            }
            // step 1 for the whole layer: pre-activations at every vertex
            if ((rc = x.mark(PCX_K_GEMM, true))) return rc;
            if (l == 0) {
                launch_gemm(x.b, ZS, x.b.X, D, 0, (int)V, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], st);
            } else if (x.tape) {
                // keep the previous layer's rows: evaluate into a fresh buffer
                double *prev = x.b.Z;
                void *q;
                if ((rc = x.arena.alloc(&q, x.Vcap * (size_t)ZS * sizeof(double)))) return rc;
                tapeZ.push_back(prev);
                x.b.Z = (double *)q;
                launch_gemm(x.b, ZS, prev, ZS, 1, (int)V, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], st);
            } else {
                launch_gemm(x.b, ZS, x.b.Z, ZS, 1, (int)V, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], st);
            }
            if ((rc = x.mark(PCX_K_GEMM, false))) return rc;
            if (x.prune) {
                if ((rc = x.mark(PCX_K_GEMM, true))) return rc;
                if ((rc = future_signs(x, mlp, l, nsub, V, lw))) return rc;
                if ((rc = x.mark(PCX_K_GEMM, false))) return rc;
                if ((rc = x.mark(PCX_K_NEXT, true))) return rc;
                if ((rc = prune_now(x, V, E, lw[l], par0))) return rc;
                if ((rc = x.mark(PCX_K_NEXT, false))) return rc;
            }
            started = true;
            j = 0;
        }
        const int N = mlp->widths[l + 1];
        if (j == N) {
            ++l;
            started = false;
            continue;
        }
        const int s = step0[l] + j, par = s & 1;
        int blocks;
        if (lagged) {
            if (j % kAhead == 0) {
                // snapshot before this step; read the one taken kAhead steps ago
                const int slot = x.snap_next, other = slot ^ 1;
                HIPCHK(hipMemcpyAsync(x.hsnap[slot], x.b.CTR, CTR_COUNT * sizeof(int), hipMemcpyDeviceToHost, st));
                HIPCHK(hipEventRecord(x.evsnap[slot], st));
                x.snap_at[slot] = s;
                x.snap_next = other;
                if (x.snap_at[other] >= 0) {
                    HIPCHK(hipEventSynchronize(x.evsnap[other]));
                    const int *c = x.hsnap[other];
                    x.snap_at[other] = -1;
                    Sgrid = std::max<int64_t>(Sgrid, c[CTR_SMAX] + c[CTR_SMAX] / 4 + 64);
                    Eseen = std::max<int64_t>({Eseen, c[CTR_E], c[CTR_E + 1]});
                    if (c[CTR_FLAGS] || c[CTR_PFLAGS]) {
                        // stop running ahead: exact counts, then redo, resume or report
                        if ((rc = x.drain())) return rc;
                        int f;
                        bool fresh;
                        if ((rc = recover(f, fresh))) return rc;
                        if (f >= 0) {
                            if (fresh || f < step0[l] || f > s)
                                return fail(PCX_ERR_DEVICE, "internal error: bad failing step");
                            j = f - step0[l];
                            continue;
                        }
                    }
                }
            }
            blocks = split_blocks(full_grids ? INT32_MAX : (int)std::min<int64_t>(Sgrid, INT32_MAX), N);
        }
        StepGeom g = geom(l, j);
        if (j == 0) {
            // the layer's first crossings; its scan is also the first pass of this step's compaction
            if ((rc = x.mark(PCX_K_NEXT, true))) return rc;
            launch_next_all(x.b, (int)V, Wd, lw[l], lw[l + 1], (int)E, par, s, st);
            if ((rc = x.mark(PCX_K_NEXT, false))) return rc;
            if ((rc = x.mark(PCX_K_SELECT, true))) return rc;
            launch_gather(x.b, (int)E, par, s, st);
        } else {
            if ((rc = x.mark(PCX_K_SELECT, true))) return rc;
            launch_select(x.b, (uint16_t)j, par, s,
                          full_grids ? kSelBlocks : select_grid(lagged ? std::max(Eseen, E) : E), st);
        }
        if ((rc = x.mark(PCX_K_SELECT, false))) return rc;
        HIPCHK(hipGetLastError());
        int64_t S = 0;
        if (!lagged) {
            if ((rc = x.drain())) return rc;
            int f;
            bool fresh;
            if ((rc = recover(f, fresh))) return rc;
            if (f >= 0) {
                // the previous step's pairing was redone: this step's compaction again
                if (fresh || f < step0[l] || f > s) return fail(PCX_ERR_DEVICE, "internal error: bad failing step");
                j = f - step0[l];
                continue;
            }
            S = x.hctr[CTR_S];
            E = x.hctr[CTR_E + par];
            V = x.hctr[CTR_V + par];
            if (s > 0 && !pairs_logged) steps[(size_t)(s - 1) * 4 + 3] = 2 * (E - prevE - prevS);
            pairs_logged = false;
            steps[(size_t)s * 4 + 0] = V;
            steps[(size_t)s * 4 + 1] = E;
            steps[(size_t)s * 4 + 2] = S;
            prevE = E;
            prevS = S;
            if ((rc = grow_for(V, E, S, 1, (size_t)S))) return rc;
            blocks = split_blocks(full_grids ? INT32_MAX : (int)S, N);
            g = geom(l, j);  // capacities may have grown
        }
        const int pgrid = full_grids ? kSelBlocks : pair_grid(lagged ? Sgrid * x.P : S * x.P);
        hipEvent_t es, ee;
        if ((rc = x.launch_events(PCX_K_SPLIT, es, ee))) return rc;
        launch_split(x.b, g, blocks, st, es, ee);
        HIPCHK(hipGetLastError());
        if (lagged) {
            if ((rc = x.mark(PCX_K_PAIR, true))) return rc;
            launch_hash_pair(x.b, g, pgrid, st);
            if ((rc = x.mark(PCX_K_PAIR, false))) return rc;
            HIPCHK(hipGetLastError());
        } else if (S * x.P > 0) {
            if ((rc = x.mark(PCX_K_SORT, true))) return rc;
            const uint32_t *skeys = nullptr, *svals = nullptr;
            launch_sort(x.b, (int)(S * x.P), st, &skeys, &svals);
            if ((rc = x.mark(PCX_K_SORT, false))) return rc;
            HIPCHK(hipGetLastError());
            if ((rc = x.mark(PCX_K_PAIR, true))) return rc;
            launch_pair(x.b, g, (int)V, (int)(E + S), (int)(S * x.P), skeys, svals, st);
            if ((rc = x.mark(PCX_K_PAIR, false))) return rc;
            HIPCHK(hipGetLastError());
        } else {
            if ((rc = x.put_ctr(CTR_E + (par ^ 1), (int)(E + S)))) return rc;
        }
        ++j;
    }
    HIPCHK(hipEventRecord(t1, st));
    if ((rc = x.drain())) return rc;
    if (x.hctr[CTR_FLAGS] || x.hctr[CTR_PFLAGS]) return degenerate_message(x.hctr[CTR_FLAGS] | x.hctr[CTR_PFLAGS]);
    V = x.hctr[CTR_V + (n_steps & 1)];
    E = x.hctr[CTR_E + (n_steps & 1)];
    int64_t total_splits = 0, Smax = 0;
    if (lagged && n_steps > 0) {
        std::vector<StepRec> rec(n_steps);
        HIPCHK(hipMemcpyAsync(rec.data(), x.b.REC, n_steps * sizeof(StepRec), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int t = 0; t < n_steps; ++t) {
            steps[(size_t)t * 4 + 0] = rec[t].V0;
            steps[(size_t)t * 4 + 1] = rec[t].E0;
            steps[(size_t)t * 4 + 2] = rec[t].S;
            steps[(size_t)t * 4 + 3] = 2 * ((int64_t)rec[t].E1 - rec[t].E0 - rec[t].S);
        }
    } else if (n_steps > 0 && !pairs_logged) {
        steps[(size_t)(n_steps - 1) * 4 + 3] = 2 * (E - prevE - prevS);
    }
    int64_t Ebound = E;  // the most edges any step's storage check asked for
    for (int t = 0; t < n_steps; ++t) {
        const int64_t St = steps[(size_t)t * 4 + 2];
        total_splits += St;
        Smax = std::max<int64_t>(Smax, St);
        Ebound = std::max<int64_t>(Ebound, steps[(size_t)t * 4 + 1] + St * std::max(1, D));
    }
    if (verbose) {
        fprintf(stderr, "[pcx] done: V=%lld E=%lld steps redone after growing the storage: %d, paired by the exact "
                "pass: %d\n", (long long)V, (long long)E, redone, exact_steps);
        fflush(stderr);
    }
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t0, t1));

    pcx_complex *cx = new pcx_complex();
    cx->valid = valid;
    cx->pruned = x.prune;
    cx->D = D;
    cx->M = M;
    cx->Wd = Wd;
    cx->n_steps = n_steps;
    cx->V = V;
    cx->E = E;
    cx->X = x.b.X;
    cx->SG = x.b.SG;
    cx->EDG = x.b.EDG;
    x.arena.forget(x.b.X);
    x.arena.forget(x.b.SG);
    x.arena.forget(x.b.EDG);
    if (x.tape) {
        tapeZ.push_back(x.b.Z);
        for (double *z : tapeZ) x.arena.forget(z);
        x.arena.forget(x.b.PQ);
        cx->taped = true;
        cx->PQ = x.b.PQ;
        cx->Zl = tapeZ;
        int s0 = 0;
        for (int l = 0; l < nsub; ++l) {
            cx->layer_step0.push_back(s0);
            s0 += mlp->widths[l + 1];
        }
    }
    cx->ZS = ZS;
    cx->nsub = nsub;
    cx->steps = std::move(steps);
    cx->total_splits = total_splits;
    int64_t pairs = 0;
    for (int s = 0; s < n_steps; ++s) pairs += cx->steps[(size_t)s * 4 + 3] / 2;
    cx->total_pairs = pairs;
    cx->exact_steps = exact_steps;
    cx->peak = x.arena.peak;
    cx->time_ms = ms;
    for (int k = 0; k < PCX_K_COUNT; ++k) {
        cx->ktime[k] = x.ktime[k];
        cx->klaunch[k] = x.klaunch[k];
    }
    auto *m = const_cast<pcx_mlp *>(mlp);
    m->hintV.store(std::max<int64_t>(m->hintV.load(), V));
    m->hintE.store(std::max<int64_t>(m->hintE.load(), Ebound));
    m->hintS.store(std::max<int64_t>(m->hintS.load(), Smax));
    if ((shortcuts & kShortcutGraph) && dom.lo) graph_record(mlp, dom.lo, dom.hi, o, cx, Ebound, Smax);
    *out = cx;
    return PCX_OK;
}

}  // namespace

namespace pcx {
int extract_ordinary(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts *opts, pcx_complex **out,
                     int shortcuts) {
    Domain dom;
    dom.m = 2 * mlp->D;
    dom.lo = lo;
    dom.hi = hi;
    return extract_impl(mlp, dom, opts, out, shortcuts);
}

}  // namespace pcx

extern "C" {

int pcx_extract(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts *opts, pcx_complex **out) {
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!mlp || !lo || !hi) return fail(PCX_ERR_INVALID, "NULL argument");
    for (int j = 0; j < mlp->D; ++j)
        if (!(lo[j] < hi[j])) return fail(PCX_ERR_INVALID, "box must have lo < hi in every coordinate");
    Domain dom;
    dom.m = 2 * mlp->D;
    dom.lo = lo;
    dom.hi = hi;
    return extract_impl(mlp, dom, opts, out, kShortcutTiny | kShortcutGraph);
}

int pcx_extract_simplex(const pcx_mlp *mlp, const double *corners, const pcx_opts *opts, pcx_complex **out) {
    if (!out) return fail(PCX_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (!mlp || !corners) return fail(PCX_ERR_INVALID, "NULL argument");
    const int D = mlp->D;
    // affinely independent corners: the (D+1) x (D+1) matrix of rows (P_i, 1) is regular
    std::vector<double> T((size_t)(D + 1) * (D + 1));
    double scale = 0.0;
    for (int i = 0; i <= D; ++i) {
        for (int k = 0; k < D; ++k) {
            const double v = corners[(size_t)i * D + k];
            if (!std::isfinite(v)) return fail(PCX_ERR_INVALID, "simplex corners must be finite");
            T[(size_t)i * (D + 1) + k] = v;
            scale = std::max(scale, std::fabs(v));
        }
        T[(size_t)i * (D + 1) + D] = 1.0;
    }
    double det = 1.0;
    for (int c = 0; c <= D; ++c) {
        int piv = c;
        for (int r = c + 1; r <= D; ++r)
            if (std::fabs(T[(size_t)r * (D + 1) + c]) > std::fabs(T[(size_t)piv * (D + 1) + c])) piv = r;
        const double p = T[(size_t)piv * (D + 1) + c];
        if (std::fabs(p) <= 1e-12 * std::max(1.0, scale)) return fail(PCX_ERR_INVALID, "simplex corners are affinely dependent");
        if (piv != c)
            for (int k = 0; k <= D; ++k) std::swap(T[(size_t)c * (D + 1) + k], T[(size_t)piv * (D + 1) + k]);
        det *= p;
        for (int r = c + 1; r <= D; ++r) {
            const double f = T[(size_t)r * (D + 1) + c] / p;
            for (int k = c; k <= D; ++k) T[(size_t)r * (D + 1) + k] -= f * T[(size_t)c * (D + 1) + k];
        }
    }
    (void)det;
    Domain dom;
    dom.m = D + 1;
    dom.X0.assign(corners, corners + (size_t)(D + 1) * D);
    dom.W0.resize(D + 1);
    for (int i = 0; i <= D; ++i) dom.W0[i] = 1ull << (2 * i);  // + at its own barycentric entry, 0 at the others
    for (int i = 0; i <= D; ++i)
        for (int j = i + 1; j <= D; ++j) dom.E0.push_back(make_int2(i, j));
    return extract_impl(mlp, dom, opts, out);
}

int pcx_complex_info(const pcx_complex *cx, pcx_info *info) {
    if (!cx || !info) return fail(PCX_ERR_INVALID, "NULL argument");
    info->V = cx->V;
    info->E = cx->E;
    info->D = cx->D;
    info->M = cx->M;
    info->Wd = cx->Wd;
    info->n_steps = cx->n_steps;
    info->total_splits = cx->total_splits;
    info->total_pairs = cx->total_pairs;
    info->peak_bytes = cx->peak;
    info->time_ms = cx->time_ms;
    info->exact_steps = cx->exact_steps;
    info->from_graph = cx->from_graph;
    return PCX_OK;
}

int pcx_complex_steps(const pcx_complex *cx, int64_t *steps) {
    if (!cx || !steps) return fail(PCX_ERR_INVALID, "NULL argument");
    std::memcpy(steps, cx->steps.data(), cx->steps.size() * sizeof(int64_t));
    return PCX_OK;
}

int pcx_complex_copy(const pcx_complex *cx, double *coords, uint64_t *signs, int32_t *edges) {
    if (!cx) return fail(PCX_ERR_INVALID, "NULL complex");
    int rc;
    if (coords && (rc = copy_sync(coords, cx->X, (size_t)cx->V * cx->D * sizeof(double), hipMemcpyDeviceToHost)))
        return rc;
    if (signs && (rc = copy_sync(signs, cx->SG, (size_t)cx->V * cx->Wd * sizeof(uint64_t), hipMemcpyDeviceToHost)))
        return rc;
    if (edges && (rc = copy_sync(edges, cx->EDG, (size_t)cx->E * 2 * sizeof(int32_t), hipMemcpyDeviceToHost)))
        return rc;
    return PCX_OK;
}

int pcx_complex_device(const pcx_complex *cx, void **coords, void **signs, void **edges) {
    if (!cx) return fail(PCX_ERR_INVALID, "NULL complex");
    if (coords) *coords = cx->X;
    if (signs) *signs = cx->SG;
    if (edges) *edges = cx->EDG;
    return PCX_OK;
}

int pcx_complex_kernel_time(const pcx_complex *cx, int32_t family, double *ms, int64_t *launches) {
    if (!cx || family < 0 || family >= PCX_K_COUNT) return fail(PCX_ERR_INVALID, "bad argument");
    if (ms) *ms = cx->ktime[family];
    if (launches) *launches = cx->klaunch[family];
    return PCX_OK;
}

void pcx_complex_free(pcx_complex *cx) {
    if (!cx) return;
    pool().put(cx->X);
    pool().put(cx->SG);
    pool().put(cx->EDG);
    pool().put(cx->PQ);
    for (double *z : cx->Zl) pool().put(z);
    delete cx;
}

int pcx_complex_copy_device(const pcx_complex *cx, double *coords, uint64_t *signs, int32_t *edges, void *stream) {
    if (!cx) return fail(PCX_ERR_INVALID, "NULL complex");
    hipStream_t st = (hipStream_t)stream;
    if (coords)
        HIPCHK(hipMemcpyAsync(coords, cx->X, (size_t)cx->V * cx->D * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (signs)
        HIPCHK(hipMemcpyAsync(signs, cx->SG, (size_t)cx->V * cx->Wd * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    if (edges)
        HIPCHK(hipMemcpyAsync(edges, cx->EDG, (size_t)cx->E * 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return PCX_OK;
}

}  // extern "C"

namespace {
template <typename T>
int backward_impl(const pcx_mlp *mlp, const pcx_complex *cx, const double *grad, double *const *gW, double *const *gb,
                  hipStream_t st) {
    const int D = cx->D, ZS = cx->ZS, nsub = cx->nsub;
    Arena ar;
    int rc;
    void *p;
    int *dflag;
    if ((rc = ar.alloc(&p, sizeof(int)))) return rc;
    dflag = (int *)p;
    HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int), st));
    if ((rc = ar.alloc(&p, (size_t)cx->V * D * sizeof(T)))) return rc;
    T *gx = (T *)p;
    if ((rc = ar.alloc(&p, (size_t)cx->V * ZS * sizeof(T)))) return rc;
    T *gz = (T *)p;
    bwd_init<T>(grad, gx, (size_t)cx->V * D, gz, (size_t)cx->V * ZS, st);
    // every parent's children in increasing order: one sort of (parent, child, side) records
    const int Vb = cx->n_steps > 0 ? (int)cx->steps[0] : (int)cx->V;
    const int nrec = 2 * (int)(cx->V - Vb);
    Bufs sb{};
    int *pos = nullptr;
    double *tt = nullptr;
    T *gtt = nullptr;
    const uint64_t *skey = nullptr;
    if (nrec > 0) {
        if ((rc = ar.alloc(&p, (size_t)nrec * sizeof(uint64_t)))) return rc;
        sb.K64a = (uint64_t *)p;
        if ((rc = ar.alloc(&p, (size_t)nrec * sizeof(uint64_t)))) return rc;
        sb.K64b = (uint64_t *)p;
        if ((rc = ar.alloc(&p, (size_t)nrec * sizeof(uint32_t)))) return rc;
        sb.VALa = (uint32_t *)p;
        if ((rc = ar.alloc(&p, (size_t)nrec * sizeof(uint32_t)))) return rc;
        sb.VALb = (uint32_t *)p;
        if ((rc = ar.alloc(&p, (size_t)kSortBins * ((nrec + kSortTile - 1) / kSortTile + 1) * sizeof(uint32_t))))
            return rc;
        sb.HIST = (uint32_t *)p;
        if ((rc = ar.alloc(&p, (size_t)nrec * sizeof(int)))) return rc;
        pos = (int *)p;
        if ((rc = ar.alloc(&p, (size_t)cx->V * sizeof(double)))) return rc;
        tt = (double *)p;
        if ((rc = ar.alloc(&p, (size_t)cx->V * sizeof(T)))) return rc;
        gtt = (T *)p;
        bwd_records(cx->PQ, Vb, (int)cx->V, sb.K64a, dflag, st);
        const uint32_t *svals = nullptr;
        launch_sort64(sb, nrec, st, &skey, &svals);
        bwd_pos(svals, nrec, pos, st);
        HIPCHK(hipGetLastError());
    }
    // layers that were not subdivided do not move any vertex
    for (int l = nsub; l < mlp->L; ++l) {
        HIPCHK(hipMemsetAsync(gW[l], 0, (size_t)mlp->widths[l + 1] * mlp->widths[l] * sizeof(double), st));
        HIPCHK(hipMemsetAsync(gb[l], 0, (size_t)mlp->widths[l + 1] * sizeof(double), st));
    }
    for (int l = nsub - 1; l >= 0; --l) {
        const int N = mlp->widths[l + 1], K = mlp->widths[l];
        const int s0 = cx->layer_step0[l];
        for (int j = N - 1; j >= 0; --j) {
            const int64_t *st4 = &cx->steps[(size_t)(s0 + j) * 4];
            bwd_step<T>(cx->X, cx->Zl[l], cx->PQ, gx, gz, D, N, ZS, j, Vb, (int)st4[0], (int)st4[2], skey, nrec, pos,
                        tt, gtt, dflag, st);
        }
        HIPCHK(hipGetLastError());
        const int Vs = (int)cx->steps[(size_t)s0 * 4];
        const int chunks = std::max(1, std::min(256, Vs / 2048));
        if ((rc = ar.alloc(&p, (size_t)chunks * N * (K + 1) * sizeof(double)))) return rc;
        double *part = (double *)p;
        T *gzp = nullptr;
        if (l > 0) {
            if ((rc = ar.alloc(&p, (size_t)Vs * ZS * sizeof(T)))) return rc;
            gzp = (T *)p;
        }
        const double *hin = l == 0 ? cx->X : cx->Zl[l - 1];
        bwd_layer<T>(gz, ZS, hin, l == 0 ? D : ZS, l > 0 ? 1 : 0, Vs, N, K, mlp->Wr[l], part, chunks, gW[l], gb[l],
                     gzp, ZS, st);
        HIPCHK(hipGetLastError());
        if (gzp) {
            HIPCHK(hipStreamSynchronize(st));
            ar.release(gz);
            gz = gzp;
        }
    }
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hflag) return fail(PCX_ERR_DEVICE, "internal error: tape index out of range");
    return PCX_OK;
}
}  // namespace

extern "C" {

int pcx_backward(const pcx_mlp *mlp, const pcx_complex *cx, const double *grad_coords, double *const *gW,
                 double *const *gb, int32_t precision, void *stream) {
    if (!mlp || !cx || !grad_coords || !gW || !gb) return fail(PCX_ERR_INVALID, "NULL argument");
    if (!cx->taped) return fail(PCX_ERR_INVALID, "complex was extracted without record_tape");
    if (cx->D != mlp->D || cx->nsub > mlp->L) return fail(PCX_ERR_INVALID, "complex does not belong to this network");
    for (int l = 0; l < mlp->L; ++l)
        if (!gW[l] || !gb[l]) return fail(PCX_ERR_INVALID, "NULL gradient buffer");
    hipStream_t st = (hipStream_t)stream;
    if (precision == PCX_F64) return backward_impl<double>(mlp, cx, grad_coords, gW, gb, st);
    if (precision == PCX_F32) return backward_impl<float>(mlp, cx, grad_coords, gW, gb, st);
    return fail(PCX_ERR_INVALID, "precision must be PCX_F64 or PCX_F32");
}

void pcx_cache_trim(void) { pool().trim(); }

}  // extern "C"
