// Device kernels of libpcx.so: edge subdivision (Berzins 2023, Sec. 4.2) on
// gfx950. One neuron step is: compaction of the splitting edges (step 3),
// interpolation + split + 2-face keys (steps 4-5), radix sort of the keys and
// pairing into intersecting edges (step 5). Each layer starts with the
// pre-activation evaluation (step 1) and a scan that records, per edge, the
// first neuron of the layer whose sign differs at its endpoints (steps 2-3).
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

#include "device.h"
#include "internal.h"

namespace pcx {

// A per-step kernel of global step `step` does nothing while a hard failure is
// flagged or an earlier step's pairing failed (the host redoes that pairing
// exactly, then queues the later steps again). A step's own pairing failure
// does not stop its split, which the exact pass needs whole.
__device__ __forceinline__ bool step_blocked(const int *ctr, int step) {
    return ctr[CTR_FLAGS] != 0 || ctr[CTR_PFAIL] < step;
}

// --------------------------------------------------------- step 0: the box

// 2^D corners (bit j of the corner id picks hi_j) and D 2^(D-1) edges between
// corners at Hamming distance one. Box entries: 2j is x_j - lo_j (zero at
// lo_j), 2j+1 is hi_j - x_j (zero at hi_j).
__global__ void k_init_box(Bufs b, int D, int Wd, const double *__restrict__ lo, const double *__restrict__ hi) {
    const int nc = 1 << D;
    const int ne = D << (D - 1);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc + ne; i += gridDim.x * blockDim.x) {
        if (i < nc) {
            uint64_t w0 = 0;
            for (int j = 0; j < D; ++j) {
                const int up = (i >> j) & 1;
                b.X[(size_t)i * D + j] = up ? hi[j] : lo[j];
                w0 |= (uint64_t)(up ? 1 : 0) << (4 * j);      // entry 2j:   + unless at lo
                w0 |= (uint64_t)(up ? 0 : 1) << (4 * j + 2);  // entry 2j+1: + unless at hi
            }
            b.SG[(size_t)i * Wd] = w0;
            for (int w = 1; w < Wd; ++w) b.SG[(size_t)i * Wd + w] = 0;
        } else {
            const int e = i - nc;
            const int j = e >> (D - 1);
            const int r = e & ((1 << (D - 1)) - 1);
            const int c = ((r >> j) << (j + 1)) | (r & ((1 << j) - 1));
            b.EDG[e] = make_int2(c, c | (1 << j));
        }
    }
}

void launch_init_box(const Bufs &b, int D, int Wd, const double *lo, const double *hi, hipStream_t st) {
    const int n = (1 << D) + (D << (D - 1));
    const int grid = (n + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_init_box, dim3(grid), dim3(kThreads), 0, st, b, D, Wd, lo, hi);
}

// ------------------------------------------------- step 1: pre-activations
//
// Z[v] = W h(v) + b with h(v) = ReLU(in[v]) (or in[v] itself for the first
// layer). A workgroup owns kGemmRows vertex rows and all N <= 256 outputs, so
// with in == Z the evaluation runs in place: every read of the workgroup's
// rows happens before its first write. Thread (tv, tc) holds 4 rows x 8
// columns {tc, tc+32, ..., tc+224}; this lane order makes the LDS reads of W
// conflict-free and builds each 32-entry sign word from two wave ballots. The
// epilogue writes the layer's sign entries (Sec. 3.4: the sign of the
// pre-activation) into the layer's own words of each row.
__global__ __launch_bounds__(kThreads) void k_gemm(Bufs b, int ZS, const double *in, int in_stride, int relu,
                                                    int V, int K, int N, const double *__restrict__ Wt,
                                                    const double *__restrict__ bias, int Wd, int lw0) {
    __shared__ double hs[kGemmRows][kGemmK + 1];
    __shared__ double ws[kGemmK][kMaxWidth];
    gemm_tile(b, ZS, in, in_stride, relu, V, K, N, Wt, bias, Wd, lw0, blockIdx.x * kGemmRows, hs, ws);
}

// The same evaluation for a narrow layer (N <= kGemvMaxN outputs, e.g. the
// output neuron): one vertex per thread, 512 rows per workgroup, the rows
// staged through LDS in chunks of kGemvK (64-byte row pieces: small chunks,
// 18 KB of LDS per workgroup, keep many workgroups' loads in flight),
// and the same sequential fma chain over k per output as gemm_tile, so every
// evaluation kernel rounds alike. Weights are read at uniform addresses. In
// place as above: a thread reads its whole row before it writes it.
constexpr int kGemvMaxN = 8, kGemvRows = 512, kGemvK = 8;
__global__ __launch_bounds__(kGemvRows) void k_gemv(Bufs b, int ZS, const double *in, int in_stride, int relu, int V,
                                                     int K, int N, const double *__restrict__ Wt,
                                                     const double *__restrict__ bias, int Wd, int lw0) {
    __shared__ double hs[kGemvRows][kGemvK + 1];
    const int t = threadIdx.x;
    const int v0 = blockIdx.x * kGemvRows, v = v0 + t;
    double acc[kGemvMaxN];
#pragma unroll
    for (int n = 0; n < kGemvMaxN; ++n) acc[n] = 0.0;
    for (int k0 = 0; k0 < K; k0 += kGemvK) {
        __syncthreads();  // the previous chunk has been read
#pragma unroll
        for (int i = 0; i < kGemvK; ++i) {
            // element idx of the chunk: row idx / kGemvK, column idx % kGemvK
            const int idx = t + kGemvRows * i, r = idx / kGemvK, k = idx % kGemvK;
            double h = 0.0;
            if (v0 + r < V && k0 + k < K) {
                h = in[(size_t)(v0 + r) * in_stride + k0 + k];
                if (relu) h = h > 0.0 ? h : 0.0;
            }
            hs[r][k] = h;
        }
        __syncthreads();
        const int kc = min(kGemvK, K - k0);
        for (int kk = 0; kk < kc; ++kk) {
            const double h = hs[t][kk];
#pragma unroll
            for (int n = 0; n < kGemvMaxN; ++n)
                if (n < N) acc[n] = fma(h, Wt[(size_t)(k0 + kk) * N + n], acc[n]);
        }
    }
    if (v >= V) return;
    uint32_t pos = 0, neg = 0;
    int zero = 0;
#pragma unroll
    for (int n = 0; n < kGemvMaxN; ++n) {
        if (n < N) {
            const double z = acc[n] + bias[n];
            b.Z[(size_t)v * ZS + n] = z;
            zero |= (z == 0.0);
            pos |= (uint32_t)(z > 0.0) << n;
            neg |= (uint32_t)(z < 0.0) << n;
        }
    }
    const uint64_t cw = codes_of(pos, neg);
    b.SG[(size_t)v * Wd + lw0] = cw;
    if (b.LW) b.LW[(size_t)v * 8] = cw;
    if (zero) raise_flag(b.CTR, FLAG_ZERO_SIGN);
}

// The same evaluation on the matrix cores, for wide layers (N > 128, K >= 16).
// Wave w owns columns [64 (w%4), +64) of the row band w/4 as RT x 4 tiles of
// the FP64 16x16x4 MFMA (lane l of a tile holds rows l/16 + 4i, column l%16,
// i = 0..3). A chain of these MFMAs rounds exactly like the sequential fma
// chain of k_gemm, so both kernels give identical bits. K advances in chunks
// of MK staged through LDS (h k-major, W^T row-major); the next chunk's global
// loads are in flight while the current chunk's MFMAs run, and with DB the LDS
// is double-buffered (one barrier per chunk). In place as above: a workgroup
// reads all its rows before the epilogue writes them. Launched with 8 waves
// of 2 x 4 tiles (64 rows per workgroup, 4 waves per SIMD), MK = 8.
constexpr int kMPad = 2;
typedef double dbl4 __attribute__((ext_vector_type(4)));

// RT: 16-row tiles per wave; WAVES: waves per workgroup, 4 per 64-row band of
// column blocks (wave w: columns [64 (w%4), +64), row band w/4).
template <int MK, int RT, int WAVES, int MINW, bool DB, int PF>
__global__ __launch_bounds__(64 * WAVES, MINW) void k_gemm_mfma(Bufs b, int ZS, const double *in, int in_stride,
                                                                int relu, int V, int K, int N,
                                                                const double *__restrict__ Wt,
                                                                const double *__restrict__ bias, int Wd, int lw0) {
    constexpr int T = 64 * WAVES;
    constexpr int ROWS = (WAVES / 4) * RT * 16;
    constexpr int APT = ROWS * MK / T;  // h values staged per thread
    constexpr int WPT = MK * kMaxWidth / T;  // W^T values staged per thread
    static_assert(APT >= 1 && MK % APT == 0 && WPT >= 1, "staging map");
    constexpr int NB = DB ? 2 : 1;
    __shared__ double as[NB][MK][ROWS + kMPad];
    __shared__ double ws[NB][MK][kMaxWidth + kMPad];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int v0 = blockIdx.x * ROWS;
    // staging map: h row t / (MK/APT), k offsets APT (t % (MK/APT)) .. +APT-1;
    // W^T rows WPT (t / 256) .. +WPT-1, column t % 256
    const int ar = t / (MK / APT), ak = (t % (MK / APT)) * APT;
    const int wc = t % kMaxWidth, wk = (t / kMaxWidth) * WPT;
    const bool arow = v0 + ar < V;
    const double *arow_p = in + (size_t)(v0 + ar) * in_stride;
    double pa[PF][APT], pw[PF][WPT];  // PF chunks of staged loads in flight
    auto fetch = [&](int k0, int slot) {
#pragma unroll
        for (int i = 0; i < APT; ++i) {
            double h = 0.0;
            if (arow && k0 + ak + i < K) {
                h = arow_p[k0 + ak + i];
                if (relu) h = h > 0.0 ? h : 0.0;
            }
            pa[slot][i] = h;
        }
#pragma unroll
        for (int i = 0; i < WPT; ++i)
            pw[slot][i] = (k0 + wk + i < K && wc < N) ? Wt[(size_t)(k0 + wk + i) * N + wc] : 0.0;
    };
    dbl4 acc[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = dbl4{0.0, 0.0, 0.0, 0.0};
    const int col0 = (w & 3) * 64;
    const int rb = (w >> 2) * RT * 16;
    const bool wave_live = col0 < N;
    double bv[4];  // this lane's bias values, loaded before the main loop
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
        const int col = col0 + ct * 16 + (l & 15);
        bv[ct] = col < N ? bias[col] : 0.0;
    }
    auto put = [&](int buf, int slot) {
#pragma unroll
        for (int i = 0; i < APT; ++i) as[buf][ak + i][ar] = pa[slot][i];
#pragma unroll
        for (int i = 0; i < WPT; ++i) ws[buf][wk + i][wc] = pw[slot][i];
    };
    auto compute = [&](int buf) {
        if (!wave_live) return;
        __builtin_amdgcn_s_setprio(1);  // MFMA issue ahead of the other waves' staging
#pragma unroll
        for (int kk = 0; kk < MK; kk += 4) {
            double af[RT], bf[4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) af[rt] = as[buf][kk + (l >> 4)][rb + rt * 16 + (l & 15)];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) bf[ct] = ws[buf][kk + (l >> 4)][col0 + ct * 16 + (l & 15)];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < 4; ++ct)
                    acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[rt], bf[ct], acc[rt][ct], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
    };
#pragma unroll
    for (int p = 0; p < PF; ++p)
        if (p * MK < K) fetch(p * MK, p);
    if (DB) {
        // one barrier per chunk: compute from one buffer while the next chunk is stored into the other
        put(0, 0);
        __syncthreads();
        int c = 0;
        for (int k0 = 0; k0 < K; k0 += MK, ++c) {
            const bool more = k0 + MK < K;
            if (k0 + PF * MK < K) fetch(k0 + PF * MK, c % PF);
            compute(c & 1);
            if (more) put((c & 1) ^ 1, (c + 1) % PF);
            __syncthreads();
        }
    } else {
        int c = 0;
        for (int k0 = 0; k0 < K; k0 += MK, ++c) {
            __syncthreads();
            put(0, c % PF);
            __syncthreads();
            if (k0 + PF * MK < K) fetch(k0 + PF * MK, c % PF);
            compute(0);
        }
    }
    if (!wave_live) return;
    // epilogue: bias, store, and the layer's sign words (two per wave: columns
    // col0..col0+31 and col0+32..col0+63, each from two tiles' ballots)
    const int nwords = (N + 31) >> 5;
    const int q = l >> 4;
    int zero = 0;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = v0 + rb + rt * 16 + q + 4 * i;
            uint64_t pb[4], nb[4];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const int col = col0 + ct * 16 + (l & 15);
                const bool ok = v < V && col < N;
                double z = 0.0;
                if (ok) {
                    z = acc[rt][ct][i] + bv[ct];
                    b.Z[(size_t)v * ZS + col] = z;
                    zero |= (z == 0.0);
                }
                pb[ct] = __ballot(ok && z > 0.0);
                nb[ct] = __ballot(ok && z < 0.0);
            }
            // lane 16q + p writes word p (p = 0, 1) of this row
            const int p = l & 15;
            if (p < 2 && v < V) {
                const int word = (col0 >> 5) + p;
                if (word < nwords) {
                    const int sh = 16 * q;
                    const uint32_t pos = (uint32_t)((pb[2 * p] >> sh) & 0xFFFFu) |
                                         ((uint32_t)((pb[2 * p + 1] >> sh) & 0xFFFFu) << 16);
                    const uint32_t neg = (uint32_t)((nb[2 * p] >> sh) & 0xFFFFu) |
                                         ((uint32_t)((nb[2 * p + 1] >> sh) & 0xFFFFu) << 16);
                    const uint64_t cw = codes_of(pos, neg);
                    b.SG[(size_t)v * Wd + lw0 + word] = cw;
                    if (b.LW) b.LW[(size_t)v * 8 + word] = cw;
                }
            }
        }
    }
    if (zero) raise_flag(b.CTR, FLAG_ZERO_SIGN);
}

void launch_gemm(const Bufs &b, int ZS, const double *in, int in_stride, int relu, int V, int K, int N,
                 const double *Wt, const double *bias, int Wd, int lw0, hipStream_t st) {
    if (V <= 0) return;
    if (N > 128 && N <= kMaxWidth && K >= 16) {
        const int grid = (V + 63) / 64;
        hipLaunchKernelGGL((k_gemm_mfma<8, 2, 8, 4, false, 1>), dim3(grid), dim3(512), 0, st, b, ZS, in, in_stride, relu, V, K, N, Wt,
                           bias, Wd, lw0);
        return;
    }
    if (N <= kGemvMaxN) {
        hipLaunchKernelGGL(k_gemv, dim3((V + kGemvRows - 1) / kGemvRows), dim3(kGemvRows), 0, st, b, ZS, in, in_stride,
                           relu, V, K, N, Wt, bias, Wd, lw0);
        return;
    }
    const int grid = (V + kGemmRows - 1) / kGemmRows;
    hipLaunchKernelGGL(k_gemm, dim3(grid), dim3(kThreads), 0, st, b, ZS, in, in_stride, relu, V, K, N, Wt, bias,
                       Wd, lw0);
}

// ---------------------------------------------- step 3: splitting edges
//
// Ordered stream compaction of {e : NX8[e] == target}. The edge array is cut
// into one contiguous chunk per workgroup (up to kSelBlocks; fewer for small
// steps). The first kernel reads its chunk once and writes the matching ids in
// order (wave ballot / prefix sum inside each tile) to the chunk's own range of
// SPLX, with the chunk's count; the second moves each chunk's matches to their
// offset in SPLE, the sum of the counts before it, with their endpoints (work
// proportional to the matches, not to the edges). No
// workgroup ever waits on another, so the scan runs at streaming speed on all
// XCDs and reads each next-crossing once per step.
__device__ __forceinline__ void sel_chunk(int E, int &c0, int &c1) {
    const int per = ((E + (int)gridDim.x - 1) / (int)gridDim.x + kScanItems - 1) / kScanItems * kScanItems;
    c0 = min(E, (int)blockIdx.x * per);
    c1 = min(E, c0 + per);
}

__global__ __launch_bounds__(kThreads) void k_sel_local(Bufs b, uint16_t target, int par, int step) {
    __shared__ int s_w[kThreads / 64];
    if (step_blocked(b.CTR, step)) return;  // an earlier step failed: the host redoes or reports it
    const int E = b.CTR[CTR_E + par];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int c0, c1;
    sel_chunk(E, c0, c1);
    int run = c0;
    // the next tile's bytes are loaded before this tile's scan, so that their
    // latency hides behind it (raw words carried, compared at the next round)
    int nbase = c0 + t * kScanItems;
    uint4 ra = make_uint4(0, 0, 0, 0), rc = ra;
    if (nbase + kScanItems <= c1) load32b(b.NX8, nbase, ra, rc);
    for (int tb = c0; tb < c1; tb += kScanTile) {
        const int base = nbase;
        uint32_t hit = base < c1 ? match32b_raw(b.NX8, base, c1, (uint8_t)target, ra, rc) : 0u;
        nbase = base + kScanTile;
        if (nbase + kScanItems <= c1) load32b(b.NX8, nbase, ra, rc);
        const int cnt = __popc(hit);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        __syncthreads();  // s_w reuse
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        int wave_off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const int ws = s_w[w];
            if (w < wave) wave_off += ws;
            total += ws;
        }
        int pos = run + wave_off + incl - cnt;
        while (hit) {
            const int i = __builtin_ctz(hit);
            hit &= hit - 1;
            b.SPLX[pos++] = base + i;
        }
        run += total;
    }
    if (t == 0) b.SELCNT[blockIdx.x] = run - c0;
}

__global__ __launch_bounds__(kThreads) void k_sel_gather(Bufs b, int par, int step) {
    __shared__ int s_w[kThreads / 64];
    __shared__ int s_base;
    if (step_blocked(b.CTR, step)) return;
    const int E = b.CTR[CTR_E + par];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int c0, c1;
    sel_chunk(E, c0, c1);
    // the first round of entries is loaded while the chunk's offset is summed
    const int n = b.SELCNT[blockIdx.x];
    int e0 = 0;
    int2 ab0 = make_int2(0, 0);
    if (t < n) {
        e0 = b.SPLX[c0 + t];
        ab0 = b.EDG[e0];
    }
    int pre = 0;
    for (int i = t; i < (int)blockIdx.x; i += kThreads) pre += b.SELCNT[i];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if (lane == 0) s_w[wave] = pre;
    __syncthreads();
    if (t == 0) {
        int x = 0;
        for (int w = 0; w < kThreads / 64; ++w) x += s_w[w];
        s_base = x;
        if (blockIdx.x == gridDim.x - 1) b.CTR[CTR_S] = x + b.SELCNT[blockIdx.x];
    }
    __syncthreads();
    // each entry carries its edge's endpoints, so the split starts from them
    // without another dependent load
    const int base = s_base;
    if (t < n) b.SPLE[base + t] = make_int4(e0, ab0.x, ab0.y, 0);
    for (int i = t + kThreads; i < n; i += kThreads) {
        const int e = b.SPLX[c0 + i];
        const int2 ab = b.EDG[e];
        b.SPLE[base + i] = make_int4(e, ab.x, ab.y, 0);
    }
}

static int clamp_grid(int64_t g) { return (int)std::min<int64_t>(kSelBlocks, std::max<int64_t>(32, g)); }
int select_grid(int64_t edges) { return clamp_grid((edges + 2047) / 2048); }
int pair_grid(int64_t slots) { return clamp_grid((slots + 255) / 256); }

// both kernels chunk the edges by the grid they are launched with: the same one
void launch_select(const Bufs &b, uint16_t target, int par, int step, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_sel_local, dim3(grid), dim3(kThreads), 0, st, b, target, par, step);
    hipLaunchKernelGGL(k_sel_gather, dim3(grid), dim3(kThreads), 0, st, b, par, step);
}

// ------------------------------------ steps 2-3 at a layer start, per edge
//
// For every edge, the first neuron of the layer at which its endpoints carry
// different signs (both are nonzero there: every vertex has all of this
// layer's entries set by the evaluation above). Edges with no such neuron
// never split in this layer. Each workgroup takes one contiguous chunk of the
// edges (one edge per thread per tile) and also writes the edges whose first
// crossing is the layer's neuron 0, in edge order, to its chunk's range of
// SPLX: the first pass of that step's compaction (byte 0 stands for both
// "none" and neuron 0, which no later step looks up).
__global__ __launch_bounds__(kThreads) void k_next_all(Bufs b, int V, int Wd, int lw0, int lw1, int par, int step) {
    __shared__ int s_w[kThreads / 64];
    if (step_blocked(b.CTR, step)) return;
    const int E = b.CTR[CTR_E + par];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    int c0, c1;
    sel_chunk(E, c0, c1);
    int run = c0;
    for (int tb = c0; tb < c1; tb += kThreads) {
        const int e = tb + t;
        int col = kNoCol;
        if (e < c1) {
            const int2 ab = b.EDG[e];
            if ((unsigned)ab.x >= (unsigned)V || (unsigned)ab.y >= (unsigned)V) {
                raise_flag(b.CTR, FLAG_BOUNDS);
            } else if (b.LW) {
                // the layer's words from their 64-byte copies: four aligned 16-byte loads per endpoint
                const uint4 *ra = reinterpret_cast<const uint4 *>(b.LW + (size_t)ab.x * 8);
                const uint4 *rb = reinterpret_cast<const uint4 *>(b.LW + (size_t)ab.y * 8);
                uint4 qa[4], qb[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    qa[i] = ra[i];
                    qb[i] = rb[i];
                }
                const int nw = lw1 - lw0;
#pragma unroll
                for (int i = 3; i >= 0; --i) {
                    const uint64_t x1 = (((uint64_t)(qa[i].w ^ qb[i].w)) << 32) | (qa[i].z ^ qb[i].z);
                    const uint64_t x0 = (((uint64_t)(qa[i].y ^ qb[i].y)) << 32) | (qa[i].x ^ qb[i].x);
                    if (2 * i + 1 < nw && x1) col = first_col(x1, lw0 + 2 * i + 1, lw0);
                    if (2 * i < nw && x0) col = first_col(x0, lw0 + 2 * i, lw0);
                }
            } else {
                const uint64_t *ra = b.SG + (size_t)ab.x * Wd;
                const uint64_t *rb = b.SG + (size_t)ab.y * Wd;
                for (int w = lw0; w < lw1 && col == kNoCol; ++w) col = first_col(ra[w] ^ rb[w], w, lw0);
            }
            b.NX8[e] = (col == kNoCol || col == 0) ? 0 : (uint8_t)col;
        }
        const bool hit = col == 0;
        const uint64_t m = __ballot(hit);
        __syncthreads();  // s_w reuse
        if (lane == 0) s_w[wave] = __popcll(m);
        __syncthreads();
        int wave_off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const int ws = s_w[w];
            if (w < wave) wave_off += ws;
            total += ws;
        }
        if (hit) b.SPLX[run + wave_off + __popcll(m & below)] = e;
        run += total;
    }
    if (t == 0) b.SELCNT[blockIdx.x] = run - c0;
}

// chunks of the layer-start scan: about 4096 edges each, up to kNextBlocks
static int next_blocks(int E) {
    int g = (E + 4095) / 4096;
    return g < 1 ? 1 : (g > kNextBlocks ? kNextBlocks : g);
}

void launch_next_all(const Bufs &b, int V, int Wd, int lw0, int lw1, int E, int par, int step, hipStream_t st) {
    hipLaunchKernelGGL(k_next_all, dim3(next_blocks(E)), dim3(kThreads), 0, st, b, V, Wd, lw0, lw1, par, step);
}

void launch_gather(const Bufs &b, int E, int par, int step, hipStream_t st) {
    hipLaunchKernelGGL(k_sel_gather, dim3(next_blocks(E)), dim3(kThreads), 0, st, b, par, step);
}

// -------------------------------------------- steps 4-5a: split and keys
//
// One group of G lanes per splitting edge (p, q), p = V+ and q = V-:
//   t = z_p / (z_p - z_q), x0 = x_p + t (x_q - x_p)            (Sec. 4.2.1)
// and the same interpolation for every pre-activation of the layer (each is
// affine along the edge, since all earlier layers are already subdivided), with
// the current neuron set to exactly 0. The sign row of x0 is the join of the
// endpoints' rows before this neuron, 0 at it, and the signs of the
// interpolated pre-activations after it. The edge slot becomes (a, x0) and
// (x0, b) is appended; each half records its next crossing in the layer.
// The splitting edge's sign-vector over earlier entries has D-1 zeros; each is
// perturbed to + and - (box zeros only to +, Sec. 4.1) to give the parent
// 2-faces, hashed as the sum of per-word hashes (Sec. 4.2.2).
//
// Every load of a split (both endpoint rows of pre-activations, signs and
// coordinates) is issued before any arithmetic or store, so a wave keeps
// ~NC+3 independent memory requests in flight per split. Lane c of chunk k
// holds column k*G + c; the sign words of the layer are built from the chunk
// ballots, parked in LDS for the lane that owns each word.

// hash-table words for n key slots (at most n / 2 faces): a power of two, at
// least 2n, so the table is at most a quarter full
__device__ __forceinline__ uint32_t table_size(int n) {
    uint32_t t = 256;
    while (t < 2u * (uint32_t)n) t <<= 1;
    return t;
}

template <int G, int NC>
__global__ __launch_bounds__(kThreads, 5) void k_split(Bufs b, StepGeom g) {
    if (step_blocked(b.CTR, g.step)) return;
    const int V0 = b.CTR[CTR_V + g.par], E0 = b.CTR[CTR_E + g.par], S = b.CTR[CTR_S];
    // every later kernel of the step writes within these bounds
    if ((int64_t)V0 + S > g.Vcap || (int64_t)E0 + (int64_t)S * g.D > g.Ecap || (int64_t)S * g.P > g.Kcap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            atomicMin(&b.CTR[CTR_FAIL], g.step);
            atomicOr(&b.CTR[CTR_FLAGS], FLAG_CAPACITY);
        }
        return;
    }
    const int nslots = S * g.P;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        b.CTR[CTR_V + (g.par ^ 1)] = V0 + S;
        // more key slots than a table word can name: the exact pass pairs this step
        if (g.pair_mode == PAIR_HASH && (uint32_t)nslots > kMaxHashSlots) raise_pair_flag(b.CTR, FLAG_BIGSTEP, g.step);
    }
    if (g.pair_mode == PAIR_HASH) {
        g.hmask = (uint32_t)nslots <= kMaxHashSlots ? table_size(nslots) - 1u : 0u;
        g.sbits = slot_bits(nslots);
    }
    constexpr int groups = kThreads / G;
    // new vertices' rows streamed past the caches for layers wider than 128 neurons
    constexpr bool kStream = G * NC > 128;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int half = (threadIdx.x & 63) / G;
    for (int s = blockIdx.x * groups + grp; s < S; s += gridDim.x * groups) {
        const int4 q = b.SPLE[s];
        const int2 ab = make_int2(q.y, q.z);
        if (!split_entry_ok(b, q.x, E0) || !split_edge_ok(ab, V0)) {
            if (lane == 0) raise_flag(b.CTR, FLAG_BOUNDS);
            continue;
        }
        split_core<G, NC, kStream>(b, g, V0, E0, s, q.x, ab, lane, half, nslots);
    }
}

// two splits per wave (32-lane groups; layers of up to 128 neurons take four,
// in 16-lane groups): the per-split bookkeeping on the sign words runs once
// for all groups of the wave. (The grid is sized for 32-lane groups; the
// launch cuts it to one residency wave, split_resident below.)
int split_blocks(int S_hint, int Nl) {
    (void)Nl;
    const int groups = kThreads / 32;
    int grid = (S_hint + groups - 1) / groups;
    return grid < 1 ? 1 : (grid > 16384 ? 16384 : grid);
}

// Workgroups of k_split<G, NC> that the device holds at once (one residency
// wave), per device, from the occupancy of the compiled kernel; 0 if unknown.
// A split grid is cut to one such wave and the grid-stride loop takes the
// rest: on the 768-neuron network (five workgroups per CU, 1280 in all) one
// wave took 57.1-57.8 us per split launch, 0.8 wave 60.2-60.6, 1.2 waves 65-66,
// two waves 57.6, and one workgroup per eight splits (up to ~12.5K) 59.0-59.7.
template <int G, int NC>
static int split_resident() {
    constexpr int kDevs = 64;
    static std::atomic<int> cache[kDevs];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (dev < 0 || dev >= kDevs) return 0;
    int r = cache[dev].load(std::memory_order_relaxed);
    if (r) return r;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_split<G, NC>, kThreads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
        cus < 1) {
        // (the launch then keeps its grid; the error must not be reported by
        // the caller's check of the launch)
        (void)hipGetLastError();
        return 0;
    }
    r = per_cu * cus;
    cache[dev].store(r, std::memory_order_relaxed);
    return r;
}

// untimed: the plain launch (also what a captured graph records); timed: the
// launch records its own start and end events
template <int G, int NC>
static void launch_split_as(const Bufs &b, const StepGeom &g, int blocks, hipStream_t st, hipEvent_t t0,
                            hipEvent_t t1) {
    const int wave = split_resident<G, NC>();
    if (wave > 0 && blocks > wave) blocks = wave;
    if (!t0 && !t1)
        hipLaunchKernelGGL((k_split<G, NC>), dim3(blocks), dim3(kThreads), 0, st, b, g);
    else
        hipExtLaunchKernelGGL((k_split<G, NC>), dim3(blocks), dim3(kThreads), 0, st, t0, t1, 0, b, g);
}

void launch_split(const Bufs &b, const StepGeom &g, int blocks, hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
    // a group builds each of a split's 2-face keys in a lane of its own: 16-lane
    // groups only while 2(D - 1) <= 16
    const bool narrow = g.P <= 16;
    if (g.Nl <= 32) {
        if (narrow) launch_split_as<16, 2>(b, g, blocks, st, t0, t1);
        else launch_split_as<32, 1>(b, g, blocks, st, t0, t1);
    } else if (g.Nl <= 64) {
        if (narrow) launch_split_as<16, 4>(b, g, blocks, st, t0, t1);
        else launch_split_as<32, 2>(b, g, blocks, st, t0, t1);
    } else if (g.Nl <= 128) {
        if (narrow) launch_split_as<16, 8>(b, g, blocks, st, t0, t1);
        else launch_split_as<32, 4>(b, g, blocks, st, t0, t1);
    } else {
        launch_split_as<32, 8>(b, g, blocks, st, t0, t1);
    }
}

// ---------------------------------------------------- step 5b: radix sort
//
// Stable LSD radix sort of (key, slot) pairs, 8-bit digits, kSortPasses passes
// over the low 24 bits (keys are 24-bit slices of the 2-face hash, all-ones
// excluded; the sentinel of an unused slot sorts last).
// Per pass: tile histograms, an exclusive scan over the tiles of each digit
// (one workgroup per digit), and a stable scatter that adds the totals of the
// smaller digits and ranks equal digits inside a tile by wave ballots.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_sort_hist(const K *__restrict__ keys, int n, int shift,
                                                         uint32_t *__restrict__ hist, int ntiles) {
    __shared__ uint32_t h[kSortBins];
    const int t = threadIdx.x, tile = blockIdx.x;
    h[t] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = tile * kSortTile + i * kThreads + t;
        if (idx < n) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    hist[(size_t)t * ntiles + tile] = h[t];
}

// per digit d (one workgroup each): exclusive scan of hist[d][0..ntiles) in
// place, and the digit's total in hist[kSortBins * ntiles + d] (the scatter
// adds the totals of the smaller digits itself)
__global__ __launch_bounds__(kThreads) void k_sort_scan(uint32_t *hist, int ntiles) {
    __shared__ uint32_t wsum[kThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, d = blockIdx.x;
    uint32_t *h = hist + (size_t)d * ntiles;
    uint32_t carry = 0;
    for (int base = 0; base < ntiles; base += 4 * kThreads) {
        const int i0 = base + 4 * t;
        uint32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = i0 + k < ntiles ? h[i0 + k] : 0u;
        const uint32_t tsum = x[0] + x[1] + x[2] + x[3];
        uint32_t incl = tsum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        uint32_t woff = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const uint32_t v = wsum[w];
            if (w < wave) woff += v;
            total += v;
        }
        uint32_t run = carry + woff + incl - tsum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < ntiles) h[i0 + k] = run;
            run += x[k];
        }
        carry += total;
        __syncthreads();
    }
    if (t == 0) hist[(size_t)kSortBins * ntiles + d] = carry;
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_sort_scatter(const K *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin,
                                                            K *__restrict__ kout, uint32_t *__restrict__ vout,
                                                            int n, int shift, const uint32_t *__restrict__ hist,
                                                            int ntiles) {
    __shared__ uint32_t base[kSortBins];
    __shared__ uint32_t wcnt[kThreads / 64][kSortBins];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, tile = blockIdx.x;
    static_assert(kSortBins == kThreads, "one digit per thread");
    // digit t starts after the keys of all smaller digits: exclusive scan of the totals
    const uint32_t tot = hist[(size_t)kSortBins * ntiles + t];
    uint32_t incl = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wcnt[0][wave] = incl;
    __syncthreads();
    uint32_t woff = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w)
        if (w < wave) woff += wcnt[0][w];
    base[t] = woff + incl - tot + hist[(size_t)t * ntiles + tile];
    __syncthreads();  // wcnt[0] read by every wave before it is cleared
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = tile * kSortTile + i * kThreads + t;
        const bool valid = idx < n;
        const K k = valid ? kin[idx] : (K)0;
        const uint32_t v = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
        const uint32_t d = (uint32_t)(k >> shift) & 0xFFu;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            m &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const int rank = __popcll(m & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(m);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            add += wcnt[w][t];
            wcnt[w][t] = 0;
        }
        base[t] += add;
        __syncthreads();
    }
}

// passes of 8 bits over the low 8 * passes key bits; the first pass takes the
// slot ids as values
template <typename K>
static void sort_passes(K *ka, K *kb, uint32_t *va, uint32_t *vb, uint32_t *hist, int n, int passes, hipStream_t st,
                        const K **keys, const uint32_t **vals) {
    const int ntiles = (n + kSortTile - 1) / kSortTile;
    for (int pass = 0; n > 0 && pass < passes; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist<K>, dim3(ntiles), dim3(kThreads), 0, st, ka, n, shift, hist, ntiles);
        hipLaunchKernelGGL(k_sort_scan, dim3(kSortBins), dim3(kThreads), 0, st, hist, ntiles);
        hipLaunchKernelGGL(k_sort_scatter<K>, dim3(ntiles), dim3(kThreads), 0, st, ka, pass == 0 ? nullptr : va, kb,
                           vb, n, shift, hist, ntiles);
        K *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    *keys = ka;
    *vals = va;
}

void launch_sort(const Bufs &b, int n, hipStream_t st, const uint32_t **keys, const uint32_t **vals) {
    sort_passes<uint32_t>(b.K32a, b.K32b, b.VALa, b.VALb, b.HIST, n, kSortPasses, st, keys, vals);
}

// all 64 key bits (eight passes): the exact pass's sort
void launch_sort64(const Bufs &b, int n, hipStream_t st, const uint64_t **keys, const uint32_t **vals) {
    sort_passes<uint64_t>(b.K64a, b.K64b, b.VALa, b.VALb, b.HIST, n, 8, st, keys, vals);
}

// ------------------------------------------- step 5c: pair and connect
//
// In the sorted key array every run of equal keys has even length (each
// splitting 2-face is met by exactly two splitting edges, Sec. 4.2.2), so the
// run starting at sorted position i owns output edges i/2, i/2+1, ... A run of
// two is the common case; a longer run (two faces whose 24-bit keys collide)
// is grouped by the full 64-bit hash. Every pair is verified by comparing the
// two perturbed sign-vectors word by word. The new edge joins the two new
// vertices; its sign is the face's with 0 at the current neuron (Sec. 4.2.2).
__global__ __launch_bounds__(kThreads) void k_pair(Bufs b, StepGeom g, int V0, int E1, int nslots,
                                                    const uint32_t *__restrict__ KS, const uint32_t *__restrict__ VS) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += gridDim.x * blockDim.x) {
        const uint32_t k = KS[i];
        // valid keys (< 2^24 - 1) sort before the sentinels: the last valid one fixes the edge count
        if (k == kSentinel) {
            if (i == 0) b.CTR[CTR_E + (g.par ^ 1)] = E1;
            continue;
        }
        if (i + 1 == nslots || KS[i + 1] == kSentinel) b.CTR[CTR_E + (g.par ^ 1)] = E1 + (i + 1) / 2;
        if (i > 0 && KS[i - 1] == k) continue;  // not the start of a run
        int j = i + 1;
        while (j < nslots && KS[j] == k) ++j;
        const int len = j - i;
        if (len == 2) {
            emit_pair(b, g, V0, nslots, (int)VS[i], (int)VS[i + 1], (size_t)E1 + i / 2);
            continue;
        }
        if ((len & 1) || len > 32) {
            raise_pair_flag(b.CTR, FLAG_RUN, g.step);
            continue;
        }
        uint32_t used = 0;
        int np = 0;
        for (int u = 0; u < len; ++u) {
            if (used & (1u << u)) continue;
            const uint32_t su = VS[i + u];
            if (su >= (uint32_t)nslots) {
                raise_flag(b.CTR, FLAG_BOUNDS);
                break;
            }
            const uint64_t hu = b.FULL[su];
            int w = u + 1;
            while (w < len && ((used & (1u << w)) || VS[i + w] >= (uint32_t)nslots || b.FULL[VS[i + w]] != hu)) ++w;
            if (w == len) {
                raise_pair_flag(b.CTR, FLAG_RUN, g.step);
                break;
            }
            used |= (1u << u) | (1u << w);
            emit_pair(b, g, V0, nslots, (int)VS[i + u], (int)VS[i + w], (size_t)E1 + i / 2 + np++);
        }
    }
}

void launch_pair(const Bufs &b, const StepGeom &g, int V0, int E1, int nslots, const uint32_t *keys,
                 const uint32_t *vals, hipStream_t st) {
    int grid = (nslots + kThreads - 1) / kThreads;
    grid = grid < 1 ? 1 : (grid > 8192 ? 8192 : grid);
    hipLaunchKernelGGL(k_pair, dim3(grid), dim3(kThreads), 0, st, b, g, V0, E1, nslots, keys, vals);
}

// ---------------------------------- step 5c with the hash table
//
// The split recorded every pair as it found it (the second arrival at a
// 2-face). Two passes over the key slots emit the pairs in the order of their
// owner slots (the smaller slot of a pair): the first counts the owners of each
// workgroup's chunk of slots from the slots' own records; the second adds the
// counts of the chunks before its own, ranks the owners inside the chunk by
// wave ballots, and checks every slot: a fresh record must be mutual, and a
// valid slot must have one (a failure sends the step to the exact pass). The
// edge list is therefore the same on every run and whatever the launch shapes.
__device__ __forceinline__ void pair_chunk(int n, int &c0, int &c1) {
    const int per = ((n + (int)gridDim.x - 1) / (int)gridDim.x + kPairItems - 1) / kPairItems * kPairItems;
    c0 = min(n, (int)blockIdx.x * per);
    c1 = min(n, c0 + per);
}

// Pass 1: owners of each chunk (SELCNT), from one coalesced read of the
// records (a slot whose fresh record names a larger slot). It also empties the
// previous step's table, which no kernel reads any more, for the next step.
__global__ __launch_bounds__(kThreads) void k_hpair_count(Bufs b, StepGeom g) {
    __shared__ int s_w[kThreads / 64];
    // this step's split must not have failed its pairing (else the exact pass redoes it)
    if (b.CTR[CTR_FLAGS] || b.CTR[CTR_PFAIL] <= g.step) return;
    const int S = b.CTR[CTR_S], nslots = S * g.P;
    int c0, c1;
    pair_chunk(nslots, c0, c1);
    if (g.HTo) {
        const uint32_t clear_n = (uint32_t)b.CTR[CTR_TUSED + (g.par ^ 1)];
        for (uint32_t i = blockIdx.x * kThreads + threadIdx.x; i < clear_n; i += gridDim.x * kThreads) g.HTo[i] = 0ull;
    }
    int cnt = 0;
    for (int u = c0 + (int)threadIdx.x; u < c1; u += kThreads) cnt += slot_partner(b, g, u, nslots) > u;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
        b.SELCNT[blockIdx.x] = t;
    }
}

// Pass 2: every slot's record checked; owners in slot order append their
// intersecting edges.
__global__ __launch_bounds__(kThreads) void k_hpair_emit(Bufs b, StepGeom g) {
    __shared__ int s_w[kThreads / 64];
    __shared__ int s_base;
    if (b.CTR[CTR_FLAGS] || b.CTR[CTR_PFAIL] <= g.step) return;
    const int S = b.CTR[CTR_S], nslots = S * g.P;
    const int V0 = b.CTR[CTR_V + g.par], E0 = b.CTR[CTR_E + g.par], E1 = E0 + S;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int c0, c1;
    pair_chunk(nslots, c0, c1);
    // one slot per thread: an owner's edge is a chain of dependent row loads,
    // so owners are spread over as many threads as possible. A slot's record,
    // its partner's, and its row words from the neuron on (where an owner's
    // first-crossing search starts) are loaded together.
    int partner = -1;
    uint64_t pre[4];
    auto load_slot = [&](int u) {
        partner = -1;
#pragma unroll
        for (int i = 0; i < 4; ++i) pre[i] = 0ull;
        if (u >= c1) return;
        const uint64_t *Ra = b.SG + (size_t)(V0 + u / g.P) * g.Wd;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (g.wn + i < g.lw1) pre[i] = Ra[g.wn + i];
        partner = slot_partner(b, g, u, nslots);
        // a fresh record must be returned by the partner's; a valid slot must have one
        if (partner >= 0 ? slot_partner(b, g, partner, nslots) != u : b.PINFO[u] != kNoInfo)
            raise_pair_flag(b.CTR, FLAG_RUN, g.step);
    };
    load_slot(c0 + t);  // in flight while the chunk's offset is summed
    int pre_cnt = 0;
    for (int i = t; i < (int)blockIdx.x; i += kThreads) pre_cnt += b.SELCNT[i];
    for (int o = 32; o > 0; o >>= 1) pre_cnt += __shfl_xor(pre_cnt, o, 64);
    if (lane == 0) s_w[wave] = pre_cnt;
    __syncthreads();
    if (t == 0) {
        int x = 0;
        for (int w = 0; w < kThreads / 64; ++w) x += s_w[w];
        s_base = x;
        if (blockIdx.x == gridDim.x - 1) {
            // the next step's counts, and this step's log entry
            const int En = E1 + x + b.SELCNT[blockIdx.x];
            b.CTR[CTR_E + (g.par ^ 1)] = En;
            if (g.HT) b.CTR[CTR_TUSED + g.par] = (uint32_t)nslots <= kMaxHashSlots ? (int)table_size(nslots) : 0;
            if (S > b.CTR[CTR_SMAX]) b.CTR[CTR_SMAX] = S;
            if (b.REC) b.REC[g.step] = StepRec{V0, E0, S, En};
        }
    }
    __syncthreads();
    int run = s_base;
    for (int tb = c0; tb < c1; tb += kThreads) {
        const int u = tb + t;
        if (tb != c0) load_slot(u);
        const bool own = partner > u;
        const uint64_t m = __ballot(own);
        __syncthreads();  // s_w of the previous round has been read
        if (lane == 0) s_w[wave] = __popcll(m);
        __syncthreads();
        int wave_off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const int ws = s_w[w];
            if (w < wave) wave_off += ws;
            total += ws;
        }
        if (own) {
            const int pos = run + wave_off + __popcll(m & ((1ull << lane) - 1ull));
            emit_pair(b, g, V0, nslots, u, partner, (size_t)E1 + pos, false, g.verify != 0, pre);
        }
        run += total;
    }
}

void launch_hash_pair(const Bufs &b, const StepGeom &g, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_hpair_count, dim3(grid), dim3(kThreads), 0, st, b, g);
    hipLaunchKernelGGL(k_hpair_emit, dim3(grid), dim3(kThreads), 0, st, b, g);
}

// ------------------------------------- step 5c, the exact pass of a step
//
// After a pairing failure (a 2-face word reached three times, a valid slot
// left without a partner, equal hashes of different faces, or a step too big
// for the table) the step's pairing is redone without trusting any hash: each
// valid key slot's 2-face sign-vector is rebuilt from its new vertex's row
// (entries before the neuron, one zero perturbed: Sec. 4.1), the slots are
// sorted by a second, independent 64-bit hash of it, and inside each run of
// equal hashes the slots are grouped by comparing the sign-vectors word by
// word. Every group must have exactly two slots (Sec. 4.2.2); anything else is
// a true degeneracy of the input. The pairs are recorded as the table path
// records them, so the emission (and the edge order) is the same.

__device__ __forceinline__ uint64_t face_word(const uint64_t *R, uint32_t info, int w, int wn, int bn) {
    uint64_t f = R[w] & lt_mask(w, wn, bn);
    if (w == (int)(info >> 8)) f |= ((info & 1u) ? 2ull : 1ull) << ((info >> 1) & 63u);
    return f;
}

__global__ __launch_bounds__(kThreads) void k_exact_keys(Bufs b, StepGeom g, int nslots) {
    const int V0 = b.CTR[CTR_V + g.par];
    for (int u = blockIdx.x * kThreads + threadIdx.x; u < nslots; u += gridDim.x * kThreads) {
        const uint32_t info = b.PINFO[u];
        uint64_t k = ~0ull;  // unused slots sort last
        if (info != kNoInfo) {
            const uint64_t *R = b.SG + (size_t)(V0 + u / g.P) * g.Wd;
            uint64_t h = 0x243f6a8885a308d3ull;
            for (int w = 0; w <= g.wn; ++w) h = mix64(h ^ face_word(R, info, w, g.wn, g.bn)) + (uint64_t)(w + 1);
            if (g.fbits < 64) h &= (1ull << g.fbits) - 1ull;  // (collisions on purpose: a test of the grouping)
            k = h == ~0ull ? h - 1 : h;
        }
        b.K64a[u] = k;
        b.VALa[u] = (uint32_t)u;
    }
}

__device__ __forceinline__ bool same_face(const Bufs &b, const StepGeom &g, int V0, uint32_t ua, uint32_t ub) {
    const uint64_t *Ra = b.SG + (size_t)(V0 + ua / g.P) * g.Wd, *Rb = b.SG + (size_t)(V0 + ub / g.P) * g.Wd;
    const uint32_t ia = b.PINFO[ua], ib = b.PINFO[ub];
    uint64_t diff = 0;
    for (int w = 0; w <= g.wn; ++w) diff |= face_word(Ra, ia, w, g.wn, g.bn) ^ face_word(Rb, ib, w, g.wn, g.bn);
    return diff == 0;
}

constexpr int kExactRun = 64;  // longest run of equal 64-bit hashes the grouping takes

__global__ __launch_bounds__(kThreads) void k_exact_group(Bufs b, StepGeom g, int nslots,
                                                           const uint64_t *__restrict__ KS,
                                                           const uint32_t *__restrict__ VS) {
    const int V0 = b.CTR[CTR_V + g.par];
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < nslots; i += gridDim.x * kThreads) {
        const uint64_t k = KS[i];
        if (k == ~0ull) continue;                  // unused slots (sorted last)
        if (i > 0 && KS[i - 1] == k) continue;     // not the start of a run
        int j = i + 1;
        while (j < nslots && KS[j] == k && j - i <= kExactRun) ++j;
        const int len = j - i;
        if (len > kExactRun) {
            raise_flag(b.CTR, FLAG_RUN);  // more than kExactRun slots on one hash: not generic
            continue;
        }
        uint64_t used = 0;
        for (int a = 0; a < len; ++a) {
            if (used >> a & 1ull) continue;
            const uint32_t ua = VS[i + a];
            int mate = -1, same = 0;
            for (int c = a + 1; c < len; ++c) {
                if (used >> c & 1ull) continue;
                if (same_face(b, g, V0, ua, VS[i + c])) {
                    if (mate < 0) mate = c;
                    ++same;
                }
            }
            if (same != 1) {
                raise_flag(b.CTR, FLAG_RUN);  // a 2-face not met by exactly two splitting edges
                break;
            }
            used |= (1ull << a) | (1ull << mate);
            record_pair(b, g, ua, VS[i + mate], nslots);
        }
    }
}

// the counters at the start of an extraction (a kernel, so that a captured graph can set them)
__global__ void k_ctr_init(int *ctr, int V0, int E0) {
    const int i = threadIdx.x;
    if (i < CTR_COUNT)
        ctr[i] = i == CTR_V ? V0 : i == CTR_E ? E0 : (i == CTR_FAIL || i == CTR_PFAIL) ? 0x7fffffff : 0;
}

void launch_ctr_init(int *ctr, int V0, int E0, hipStream_t st) {
    hipLaunchKernelGGL(k_ctr_init, dim3(1), dim3(64), 0, st, ctr, V0, E0);
}

__global__ __launch_bounds__(kThreads) void k_fill64(uint64_t *p, size_t n, uint64_t v) {
    for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads) p[i] = v;
}

void launch_fill64(uint64_t *p, size_t n, uint64_t v, hipStream_t st) {
    if (n == 0) return;
    const int grid = (int)std::min<size_t>(4096, (n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_fill64, dim3(grid), dim3(kThreads), 0, st, p, n, v);
}

void launch_exact_pair(const Bufs &b, const StepGeom &g, int nslots, int grid, hipStream_t st) {
    if (nslots > 0) {
        const int kg = std::min(8192, (nslots + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_exact_keys, dim3(kg), dim3(kThreads), 0, st, b, g, nslots);
        const uint64_t *keys = nullptr;
        const uint32_t *vals = nullptr;
        launch_sort64(b, nslots, st, &keys, &vals);
        hipLaunchKernelGGL(k_exact_group, dim3(kg), dim3(kThreads), 0, st, b, g, nslots, keys, vals);
    }
    launch_hash_pair(b, g, grid, st);
}

}  // namespace pcx
