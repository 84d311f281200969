// Host-side helpers shared by the C ABI sources of libpcx.so (api.hip,
// batch_api.hip): error reporting, the handle structs, the device block cache
// and per-extraction arenas.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "pcx.h"

namespace pcx {
// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string &msg);
// The error for device failure flags (FLAG_*): PCX_ERR_DEGENERATE with what
// was found, or PCX_ERR_DEVICE for an internal index error.
int degenerate_message(int flags);

// Predicted vertex count of the complex of a random-initialised network with N
// subdivided neurons on a box in R^D: 0.6 N^D / ((D-1)! 2^(D-2)) (fitted on
// the seeded workloads: about 0.4-0.55 N^2 for D = 2 and 0.08-0.09 N^3 for
// D = 3). It only sizes buffers, orders queues and gates admission.
inline double predict_vertices(int D, int N) {
    double f = 1.0;
    for (int k = 2; k < D; ++k) f *= 2.0 * k;
    const double nd = D >= 2 ? 0.6 * std::pow((double)N, D) / f : (double)N;
    return nd + std::pow(2.0, D) + 4.0 * N;
}
}  // namespace pcx

#define HIPCHK(x)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) return pcx::fail(PCX_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace pcx {
struct GraphCache;
GraphCache *graph_cache_new();
void graph_cache_free(GraphCache *c);
}  // namespace pcx

struct pcx_mlp {
    int L = 0, D = 0;
    std::vector<int> widths;
    std::vector<double *> Wt;  // device, layer l: [N_{l-1}][N_l] (transposed for coalesced GEMM reads)
    std::vector<double *> Wr;  // device, layer l: [N_l][N_{l-1}] as given (backward pass)
    std::vector<double *> b;   // device, [N_l]
    std::atomic<int64_t> hintV{0}, hintE{0}, hintS{0};  // sizes seen by earlier extractions (capacity hints)
    pcx::GraphCache *gcache = nullptr;  // the last extraction's step log and its captured graph (graph.hip)
};

struct pcx_complex {
    int D = 0, M = 0, Wd = 0, n_steps = 0;
    int64_t V = 0, E = 0;
    std::vector<uint64_t> valid;  // [Wd] 01 at every entry in use
    bool pruned = false;          // extracted with pcx_opts.prune: a sub-complex, not the whole domain
    double *X = nullptr;
    uint64_t *SG = nullptr;
    int2 *EDG = nullptr;
    std::vector<int64_t> steps;
    int64_t total_splits = 0, total_pairs = 0;
    int exact_steps = 0;          // steps whose pairing the exact pass redid
    int from_graph = 0;           // 1: replayed from the network's captured graph
    uint64_t peak = 0;
    double time_ms = 0.0;
    double ktime[PCX_K_COUNT] = {};
    int64_t klaunch[PCX_K_COUNT] = {};
    // tape (record_tape): parents of each new vertex, each subdivided layer's
    // pre-activation rows at its end (stride ZS), and the first step of each layer
    bool taped = false;
    int ZS = 0, nsub = 0;
    int2 *PQ = nullptr;
    std::vector<double *> Zl;
    std::vector<int> layer_step0;
};


namespace pcx {
// A graph capture (graph.hip) on one thread must not overlap this library's
// device allocations and frees on other threads: those take this gate shared,
// a capture takes it exclusively (and is skipped when it cannot have it).
std::shared_mutex &capture_gate();
// Blocking copy through this thread's own non-blocking stream: the library
// puts no work on the legacy default stream, which a capture elsewhere in the
// process would make an error.
int copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);

// Device blocks released by finished extractions are kept for reuse, per
// device and size class, so that repeated extractions of large complexes do
// not pay for hipMalloc / hipFree of tens of GB each time. pcx_cache_trim()
// returns them to the runtime; a failed hipMalloc trims and retries once.
struct Pool {
    std::mutex m;
    std::map<std::pair<int, size_t>, std::vector<void *>> cached;  // (device, bytes) -> blocks
    std::unordered_map<void *, std::pair<int, size_t>> owned;       // every block handed out
    uint64_t cached_bytes = 0;

    static size_t size_class(size_t bytes) {
        const size_t g = bytes >= (size_t(1) << 20) ? (size_t(1) << 20) : 256;
        return (bytes + g - 1) / g * g;
    }
    // limit: largest block the caller may take (a cached block can be bigger than asked)
    void *get(size_t bytes, size_t *got, size_t limit) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        const size_t sz = size_class(bytes);
        *got = sz;
        {
            // best fit among cached blocks of this device no larger than 1.6x the request
            std::lock_guard<std::mutex> lk(m);
            auto it = cached.lower_bound({dev, sz});
            const size_t fit = std::min(limit, sz + sz / 2 + sz / 10);
            for (; it != cached.end() && it->first.first == dev && it->first.second <= fit; ++it) {
                if (it->second.empty()) continue;
                void *p = it->second.back();
                it->second.pop_back();
                cached_bytes -= it->first.second;
                *got = it->first.second;
                return p;
            }
        }
        void *p = nullptr;
        {
            std::shared_lock<std::shared_mutex> gate(capture_gate());
            if (hipMalloc(&p, sz) != hipSuccess) {
                (void)hipGetLastError();
                trim_gated();
                if (hipMalloc(&p, sz) != hipSuccess) {
                    (void)hipGetLastError();
                    return nullptr;
                }
            }
        }
        std::lock_guard<std::mutex> lk(m);
        owned[p] = {dev, sz};
        return p;
    }
    void put(void *p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(m);
        auto it = owned.find(p);
        if (it == owned.end()) return;
        auto &v = cached[it->second];
        if (std::find(v.begin(), v.end(), p) != v.end()) return;  // already returned
        v.push_back(p);
        cached_bytes += it->second.second;
    }
    void trim() {
        std::shared_lock<std::shared_mutex> gate(capture_gate());
        trim_gated();
    }
    void trim_gated() {
        std::lock_guard<std::mutex> lk(m);
        int cur = 0;
        (void)hipGetDevice(&cur);
        for (auto &kv : cached) {
            if (kv.first.first != cur) continue;
            for (void *p : kv.second) {
                (void)hipFree(p);
                owned.erase(p);
                cached_bytes -= kv.first.second;
            }
            kv.second.clear();
        }
    }
};

Pool &pool();

// Device memory of one extraction, with a byte cap and peak accounting.
struct Arena {
    uint64_t cap = 0, cur = 0, peak = 0;
    std::vector<std::pair<void *, size_t>> live;
    int alloc(void **p, size_t bytes) {
        *p = nullptr;
        if (bytes == 0) bytes = 256;
        const size_t sz = Pool::size_class(bytes);
        if (cap && cur + sz > cap)
            return fail(PCX_ERR_CAPACITY, "extraction needs more device memory than max_bytes allows");
        size_t got = 0;
        *p = pool().get(bytes, &got, cap ? (size_t)(cap - cur) : ~(size_t)0);
        if (!*p) return fail(PCX_ERR_OOM, "hipMalloc of " + std::to_string(sz) + " bytes failed");
        live.push_back({*p, got});
        cur += got;
        peak = std::max(peak, cur);
        return PCX_OK;
    }
    void release(void *p) {
        if (!p) return;
        for (size_t i = 0; i < live.size(); ++i)
            if (live[i].first == p) {
                cur -= live[i].second;
                live.erase(live.begin() + i);
                pool().put(p);
                return;
            }
    }
    void forget(void *p) {  // ownership moves out (to a pcx_complex)
        for (size_t i = 0; i < live.size(); ++i)
            if (live[i].first == p) {
                live.erase(live.begin() + i);
                return;
            }
    }
    ~Arena() {
        for (auto &a : live) pool().put(a.first);
    }
};

// Repeated extractions as a replayed graph (graph.hip). graph_try serves the
// extraction from the network's cached graph when its step log matches the
// request (same box and options), building the graph on first use; it returns
// kGraphDeclined when the ordinary path must run. graph_record keeps the step
// log of a finished ordinary extraction for the next request.
constexpr int kGraphDeclined = 1000;
// pcx_extract without the batch-of-one path for small networks (what a batch's
// own fallback runs), and that path (batch_api.hip)
// pcx_extract's box extraction; shortcuts: which of a small network's batch of
// one (kShortcutTiny) and a repeated network's graph (kShortcutGraph) may serve it
enum { kShortcutTiny = 1, kShortcutGraph = 2 };
int extract_ordinary(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts *opts, pcx_complex **out,
                     int shortcuts = 0);
int tiny_extract(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts &o, pcx_complex **out);
int graph_try(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts &o, hipStream_t st,
              hipStream_t cs, hipEvent_t t0, hipEvent_t t1, int *pinned, pcx_complex **out);
void graph_record(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts &o, const pcx_complex *cx,
                  int64_t Ebound, int64_t Smax);
}  // namespace pcx
