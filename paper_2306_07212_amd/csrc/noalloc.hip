// pcx_extract_into: the extraction of pcx_extract for callers that cannot
// allocate device memory. The complex goes into caller-allocated device
// buffers; every other array the kernels use (pre-activations, first
// crossings, split lists, 2-face key slots and tables, counters, the step log
// and the exact pass's sort buffers) is carved from `scratch`, a file-scope
// device array of kScratchBytes that each GPU holds from the library's load
// until the process ends. No device or pinned memory is allocated, and no HIP
// event or stream is created: counters come back by plain copies into host
// stack memory, at layer starts and every kAhead steps. The steps and kernels
// are those of pcx_extract (Sec. 4.2, every neuron in layer order), so the
// result is the same complex with the same numbering. Calls that overlap on one
// GPU share its scratch and race: callers serialize them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>

#include "host.h"

namespace pcx {
namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per GPU
constexpr int kFixedMaxLayers = 32;                  // subdivided layers this entry point takes
constexpr int kFixedMaxWords = 128;                  // sign words per vertex row
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// The scratch's device address on each GPU (its own copy of the array), taken
// once per device with that device current. Host code uses only these
// addresses: the array's name is a host-side stand-in, not a device address.
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

int scratch_base(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PCX_ERR_INVALID, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PCX_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return PCX_OK;
}

// bump allocation inside the scratch (256-byte aligned pieces)
struct Carve {
    char *base = nullptr;
    size_t used = 0;
    template <class T>
    T *take(size_t n) {
        T *p = reinterpret_cast<T *>(base ? base + used : nullptr);
        used += (std::max<size_t>(n * sizeof(T), 1) + 255) / 256 * 256;
        return p;
    }
};

size_t pow2_at_least(size_t n) {
    size_t t = 256;
    while (t < n) t <<= 1;
    return t;
}

}  // namespace
}  // namespace pcx

using namespace pcx;

extern "C" int pcx_extract_into(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts *opts,
                                double *coords, uint64_t *signs, int32_t *edges, int64_t max_vertices,
                                int64_t max_edges, pcx_info *info, int64_t *steps_out) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!mlp || !lo || !hi || !coords || !signs || !edges || !info) return fail(PCX_ERR_INVALID, "NULL argument");
    pcx_opts o{};
    if (opts) o = *opts;
    if (o.prune || o.record_tape) return fail(PCX_ERR_INVALID, "pcx_extract_into supports neither prune nor record_tape");
    if (o.pairing != PCX_PAIR_HASH) return fail(PCX_ERR_INVALID, "pcx_extract_into pairs with the hash table only");
    const int D = mlp->D, L = mlp->L;
    for (int j = 0; j < D; ++j)
        if (!(lo[j] < hi[j])) return fail(PCX_ERR_INVALID, "box must have lo < hi in every coordinate");
    const int nsub = o.include_output ? L : L - 1;
    if (nsub > kFixedMaxLayers) return fail(PCX_ERR_INVALID, "pcx_extract_into takes at most 32 subdivided layers");
    int lw[kFixedMaxLayers + 1], step0[kFixedMaxLayers + 1];
    lw[0] = 1;
    step0[0] = 0;
    int ZS = 1;
    for (int l = 0; l < nsub; ++l) {
        const int N = mlp->widths[l + 1];
        if (N > kMaxWidth) return fail(PCX_ERR_INVALID, "subdivided layers wider than 256 are not supported");
        lw[l + 1] = lw[l] + (N + 31) / 32;
        step0[l + 1] = step0[l] + N;
        ZS = std::max(ZS, N);
    }
    const int Wd = lw[nsub], n_steps = step0[nsub];
    if (Wd > kFixedMaxWords) return fail(PCX_ERR_INVALID, "sign rows longer than 128 words are not supported here");
    const int P = D >= 2 ? 2 * (D - 1) : 0;
    const int64_t V0 = int64_t(1) << D, E0 = int64_t(D) << (D - 1);
    if (max_vertices < V0 || max_edges < E0 || max_vertices >= INT32_MAX || max_edges >= INT32_MAX)
        return fail(PCX_ERR_CAPACITY, "max_vertices / max_edges below the box skeleton or beyond 2^31 - 1");
    const size_t Vcap = (size_t)max_vertices, Ecap = (size_t)max_edges;
    // a step splits at most min(Vcap, Ecap) edges: that many splits' key slots
    const size_t Scap = std::min(Vcap, Ecap), Kcap = std::max<size_t>(1, (size_t)P * Scap);
    const size_t Tcap = pow2_at_least(2 * Kcap);  // (huge maxima fail the scratch check below)

    // the scratch layout for these maxima (first with a null base, to size it)
    Bufs b{};
    unsigned long long *HT[2] = {nullptr, nullptr};
    auto layout = [&](Carve &c) {
        b.CTR = c.take<int>(CTR_COUNT);
        b.VALID = c.take<uint64_t>(Wd);
        b.SELCNT = c.take<int>(kNextBlocks);
        b.REC = c.take<StepRec>(std::max(1, n_steps));
        b.Z = c.take<double>(Vcap * ZS);
        b.LW = c.take<uint64_t>(Vcap * 8);
        b.NX8 = c.take<uint8_t>(Ecap);
        b.SPLX = c.take<int>(Ecap);
        b.SPLE = c.take<int4>(Ecap);
        b.PINFO = c.take<uint32_t>(Kcap);
        b.PART = c.take<uint64_t>(Kcap);
        HT[0] = c.take<unsigned long long>(Tcap);
        HT[1] = c.take<unsigned long long>(Tcap);
        b.K64a = c.take<uint64_t>(Kcap);
        b.K64b = c.take<uint64_t>(Kcap);
        b.VALa = c.take<uint32_t>(Kcap);
        b.VALb = c.take<uint32_t>(Kcap);
        b.HIST = c.take<uint32_t>((size_t)kSortBins * ((Kcap + kSortTile - 1) / kSortTile + 1));
        return c.take<double>(2 * D);  // the box
    };
    Carve sizing;
    layout(sizing);
    if (sizing.used > kScratchBytes)
        return fail(PCX_ERR_CAPACITY, "pcx_extract_into needs " + std::to_string(sizing.used) +
                                          " bytes of scratch for these maxima; it has " +
                                          std::to_string(kScratchBytes));
    void *base = nullptr;
    int rc;
    if ((rc = scratch_base(&base))) return rc;
    Carve c;
    c.base = (char *)base;
    double *dbox = layout(c);
    b.X = coords;
    b.SG = signs;
    b.EDG = (int2 *)edges;
    b.PQ = nullptr;
    hipStream_t st = (hipStream_t)o.stream;

    // the scratch keeps the previous call's contents: what must start at zero is cleared here
    int hc[CTR_COUNT] = {0};
    hc[CTR_V] = (int)V0;
    hc[CTR_E] = (int)E0;
    hc[CTR_FAIL] = 0x7fffffff;
    hc[CTR_PFAIL] = 0x7fffffff;
    uint64_t valid[kFixedMaxWords] = {0};
    for (int e = 0; e < 2 * D; ++e) valid[0] |= 1ull << (2 * e);
    for (int l = 0; l < nsub; ++l)
        for (int col = 0; col < mlp->widths[l + 1]; ++col) valid[lw[l] + (col >> 5)] |= 1ull << (2 * (col & 31));
    double box[32];
    for (int j = 0; j < D; ++j) {
        box[j] = lo[j];
        box[D + j] = hi[j];
    }
    HIPCHK(hipMemcpyAsync(b.CTR, hc, sizeof hc, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync((void *)b.VALID, valid, Wd * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dbox, box, 2 * D * sizeof(double), hipMemcpyHostToDevice, st));
    launch_fill64(b.PART, Kcap, 0ull, st);
    launch_fill64(reinterpret_cast<uint64_t *>(HT[0]), Tcap, 0ull, st);
    launch_fill64(reinterpret_cast<uint64_t *>(HT[1]), Tcap, 0ull, st);
    launch_init_box(b, D, Wd, dbox, dbox + D, st);
    HIPCHK(hipGetLastError());

    // counters into host stack memory: every queued kernel done
    int ctr[CTR_COUNT];
    auto drain = [&]() -> int {
        HIPCHK(hipMemcpyAsync(ctr, b.CTR, sizeof ctr, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return PCX_OK;
    };
    auto put = [&](int idx, int v) -> int {
        HIPCHK(hipMemcpyAsync(b.CTR + idx, &v, sizeof v, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
        return PCX_OK;
    };
    auto layer_of = [&](int s) { return (int)(std::upper_bound(step0, step0 + nsub + 1, s) - step0) - 1; };
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
        g.verify = o.verify_pairs ? 1 : 0;
        g.Vcap = (int)Vcap;
        g.Ecap = (int)Ecap;
        g.Kcap = (int)std::min<size_t>(Kcap, INT32_MAX);
        return g;
    };
    // after a drain: storage too small is an error here (nothing can grow); a
    // failed pairing is redone by the exact pass and work resumes after it
    int exact_steps = 0;
    auto recover = [&](int &next) -> int {
        next = -1;
        const int flags = ctr[CTR_FLAGS], pflags = ctr[CTR_PFLAGS];
        if (!flags && !pflags) return PCX_OK;
        if (flags == FLAG_CAPACITY)
            return fail(PCX_ERR_CAPACITY, "the complex exceeds max_vertices or max_edges (pcx_extract_into cannot grow)");
        if (flags) return degenerate_message(flags | pflags);
        if (pflags & ~kPairFlags) return fail(PCX_ERR_DEVICE, "internal error: unknown pairing flag");
        const int pf = ctr[CTR_PFAIL];
        if (pf < 0 || pf >= n_steps) return fail(PCX_ERR_DEVICE, "internal error: bad failing pairing step");
        const int lf = layer_of(pf);
        const int64_t nslots = (int64_t)ctr[CTR_S] * P;
        if (nslots > (int64_t)Kcap) return fail(PCX_ERR_DEVICE, "internal error: key slots beyond the storage");
        int r;
        if ((r = put(CTR_PFLAGS, 0)) || (r = put(CTR_PFAIL, 0x7fffffff))) return r;
        launch_exact_pair(b, geom(lf, pf - step0[lf]), (int)nslots, pair_grid(nslots), st);
        HIPCHK(hipGetLastError());
        if ((r = drain())) return r;
        if (ctr[CTR_FLAGS] || ctr[CTR_PFLAGS]) return degenerate_message(ctr[CTR_FLAGS] | ctr[CTR_PFLAGS]);
        ++exact_steps;
        next = pf + 1;
        return PCX_OK;
    };

    constexpr int kAhead = 8;
    int64_t V = V0, E = E0, Sgrid = 64;
    int l = 0, j = 0;
    bool started = false;
    while (true) {
        if (!started) {
            if ((rc = drain())) return rc;
            int f;
            if ((rc = recover(f))) return rc;
            if (f >= 0) {
                // resume after the step the exact pass paired (at a layer start: that layer start again)
                l = f >= n_steps ? nsub : layer_of(f);
                j = f - step0[std::min(l, nsub)];
                started = j > 0;
                continue;
            }
            if (l == nsub) break;
            const int par0 = step0[l] & 1;
            V = ctr[CTR_V + par0];
            E = ctr[CTR_E + par0];
            const int64_t Slast = step0[l] > 0 ? ctr[CTR_S] : 0;
            Sgrid = Slast + Slast / 4 + 64;
            if ((rc = put(CTR_SMAX, 0))) return rc;
            const int N = mlp->widths[l + 1], K = mlp->widths[l];
            if (l == 0) launch_gemm(b, ZS, b.X, D, 0, (int)V, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], st);
            else launch_gemm(b, ZS, b.Z, ZS, 1, (int)V, K, N, mlp->Wt[l], mlp->b[l], Wd, lw[l], st);
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
        if (j > 0 && j % kAhead == 0) {
            if ((rc = drain())) return rc;
            int f;
            if ((rc = recover(f))) return rc;
            if (f >= 0) {
                if (f < step0[l] || f > s) return fail(PCX_ERR_DEVICE, "internal error: bad failing step");
                j = f - step0[l];
                continue;
            }
            Sgrid = std::max<int64_t>(Sgrid, ctr[CTR_SMAX] + ctr[CTR_SMAX] / 4 + 64);
            E = std::max<int64_t>(E, std::max(ctr[CTR_E], ctr[CTR_E + 1]));
        }
        StepGeom g = geom(l, j);
        if (j == 0) {
            launch_next_all(b, (int)V, Wd, lw[l], lw[l + 1], (int)E, par, s, st);
            launch_gather(b, (int)E, par, s, st);
        } else {
            launch_select(b, (uint16_t)j, par, s, select_grid(E), st);
        }
        launch_split(b, g, split_blocks((int)std::min<int64_t>(Sgrid, INT32_MAX), N), st);
        launch_hash_pair(b, g, pair_grid(Sgrid * P), st);
        HIPCHK(hipGetLastError());
        ++j;
    }
    if ((rc = drain())) return rc;
    if (ctr[CTR_FLAGS] || ctr[CTR_PFLAGS]) return degenerate_message(ctr[CTR_FLAGS] | ctr[CTR_PFLAGS]);
    // the step log, a few records at a time into stack memory
    int64_t total_splits = 0, total_pairs = 0;
    StepRec rec[256];
    for (int s0 = 0; s0 < n_steps; s0 += 256) {
        const int n = std::min(256, n_steps - s0);
        HIPCHK(hipMemcpyAsync(rec, b.REC + s0, n * sizeof(StepRec), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int k = 0; k < n; ++k) {
            const int64_t K2 = 2 * ((int64_t)rec[k].E1 - rec[k].E0 - rec[k].S);
            total_splits += rec[k].S;
            total_pairs += K2 / 2;
            if (steps_out) {
                int64_t *o4 = steps_out + (size_t)(s0 + k) * 4;
                o4[0] = rec[k].V0;
                o4[1] = rec[k].E0;
                o4[2] = rec[k].S;
                o4[3] = K2;
            }
        }
    }
    std::memset(info, 0, sizeof *info);
    info->V = ctr[CTR_V + (n_steps & 1)];
    info->E = ctr[CTR_E + (n_steps & 1)];
    info->D = D;
    info->M = 2 * D + n_steps;
    info->Wd = Wd;
    info->n_steps = n_steps;
    info->total_splits = total_splits;
    info->total_pairs = total_pairs;
    info->peak_bytes = sizing.used;
    info->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    info->exact_steps = exact_steps;
    return PCX_OK;
}
