// Batched edge subdivision: many independent networks in one persistent
// launch. Each workgroup takes the next network from a ticket counter
// (networks are queued largest first), runs the whole extraction for it
// (Sec. 4.2 steps 0-5, every neuron of every subdivided layer) in a private
// arena of global memory with workgroup barriers between the phases, copies
// the finished complex into a shared output pool, and takes the next one.
//
// The per-edge, per-split and per-pair work uses the same device functions
// as the per-step kernels, in the same order, so every network's complex is
// bit-identical to what pcx_extract returns for it (same vertex and edge
// numbering too). A network that does not fit the arena or the pool is
// reported back and extracted by the host on the per-step path.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.h"
#include "device.h"

namespace pcx {

// Ordered compaction of {e < E : NXT[e] == target} by the whole workgroup,
// SI edges per thread per round (SI = 16 or 8: a schedule choice).
template <int SI>
__device__ __forceinline__ uint32_t match_si(const uint16_t *__restrict__ nxt, int base, int E, uint16_t target) {
    if (SI == 16) return match16(nxt, base, E, target);
    uint32_t hit = 0;
    if (base + SI <= E) {
        const uint4 a = *reinterpret_cast<const uint4 *>(nxt + base);
        const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if ((uint16_t)(w[i] & 0xFFFFu) == target) hit |= 1u << (2 * i);
            if ((uint16_t)(w[i] >> 16) == target) hit |= 1u << (2 * i + 1);
        }
    } else {
        for (int i = 0; i < SI; ++i)
            if (base + i < E && nxt[base + i] == target) hit |= 1u << i;
    }
    return hit;
}

template <int SI>
__device__ int block_select(const Bufs &b, int E, uint16_t target, int *s_w) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int run = 0;
    for (int tb = 0; tb < E; tb += kThreads * SI) {
        const int base = tb + t * SI;
        uint32_t hit = base < E ? match_si<SI>(b.NXT, base, E, target) : 0u;
        const int cnt = __popc(hit);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
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
            b.SPL[pos++] = base + i;
        }
        run += total;
        __syncthreads();
    }
    return run;
}

// Hash pairing by the whole workgroup: the split recorded the pairs; owners
// (smaller key slot) emit them in slot order.
__device__ int block_pair(const Bufs &b, const StepGeom &g, int V0, int E1, int nslots, int *s_w) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int run = 0;
    for (int tb = 0; tb < nslots; tb += kThreads * kPairItems) {
        const int base = tb + t * kPairItems;
        int partner[kPairItems];
        uint32_t own = 0;
#pragma unroll
        for (int i = 0; i < kPairItems; ++i)
            if (base + i < nslots && slot_owner(b, g, base + i, nslots, partner[i])) own |= 1u << i;
        const int cnt = __popc(own);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
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
#pragma unroll
        for (int i = 0; i < kPairItems; ++i)
            if (own & (1u << i))
                emit_pair(b, g, V0, nslots, base + i, partner[i], (size_t)E1 + pos++, false, g.verify != 0);
        run += total;
        __syncthreads();
    }
    return run;
}

template <int G, int NC>
__device__ __forceinline__ void block_split(const Bufs &b, const StepGeom &g, int V0, int E0, int S) {
    constexpr int groups = kThreads / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G, half = (threadIdx.x & 63) / G;
    for (int s = grp; s < S; s += groups) split_one<G, NC>(b, g, V0, E0, s, lane, half, S * g.P);
}

// One network, whole, by the workgroup. Schedule (chosen per size bucket by
// the autotuner): SI edges per thread in each step's compaction, GS lanes per
// splitting edge.
template <int SI, int GS>
__device__ void run_net(const BatchArgs &A, const BatchNet &net, int ni, Bufs &b, GemmLds *gl, int *s_w,
                        int *s_misc) {
    const int t = threadIdx.x;
    const int D = net.D, nsub = net.nsub;
    int lw[kBatchMaxLayers + 1];
    lw[0] = 1;
    int ZS = 1;
    for (int l = 0; l < nsub; ++l) {
        lw[l + 1] = lw[l] + (net.widths[l + 1] + 31) / 32;
        ZS = max(ZS, net.widths[l + 1]);
    }
    const int Wd = lw[nsub];
    const int P = D >= 2 ? 2 * (D - 1) : 0;
    // carve the arena for this network's row sizes
    char *base = A.arena + (size_t)blockIdx.x * A.arena_bytes;
    const size_t per_v = 8ull * (D + Wd + ZS);
    const int Vcap = (int)min((size_t)0x7fffffff, A.vbytes / per_v);
    const int Ecap = A.ecap, Kcap = A.kcap;
    b.X = (double *)base;
    b.SG = (uint64_t *)(base + (size_t)Vcap * 8 * D);
    b.Z = (double *)(base + (size_t)Vcap * 8 * (D + Wd));
    char *eb = base + A.vbytes;
    b.EDG = (int2 *)eb;
    b.NXT = (uint16_t *)(eb + (size_t)Ecap * 8);
    b.SPL = (int *)(eb + (size_t)Ecap * 10);
    char *kb = eb + (size_t)Ecap * 16;
    b.PART = (uint64_t *)kb;
    b.PINFO = (uint32_t *)(kb + (size_t)Kcap * 8);
    b.FULL = nullptr;
    unsigned long long *table = (unsigned long long *)(kb + (size_t)Kcap * 12 + 256 - ((size_t)Kcap * 12) % 256);
    uint64_t *valid = (uint64_t *)((char *)table + (size_t)A.tcap * sizeof(unsigned long long));
    b.CTR = (int *)(valid + kBatchMaxWords);
    b.VALID = valid;
    b.PQ = nullptr;

    int status = BATCH_OK;
    const int V0 = 1 << D, E0 = D << (D - 1);
    if (V0 > Vcap || E0 > Ecap || Wd > kBatchMaxWords) status = BATCH_OVERFLOW;
    if (status == BATCH_OK) {
        for (int w = t; w < Wd; w += kThreads) {
            uint64_t v = 0;
            if (w == 0)
                for (int e = 0; e < 2 * D; ++e) v |= 1ull << (2 * e);
            for (int l = 0; l < nsub; ++l)
                if (w >= lw[l] && w < lw[l + 1]) {
                    const int c0 = (w - lw[l]) * 32, n = min(32, net.widths[l + 1] - c0);
                    for (int c = 0; c < n; ++c) v |= 1ull << (2 * c);
                }
            valid[w] = v;
        }
        if (t < CTR_COUNT) b.CTR[t] = t == CTR_PFAIL ? 0x7fffffff : 0;
        // partner records of an earlier network in this arena: untagged again
        for (int i = t; i < Kcap; i += kThreads) b.PART[i] = 0ull;
        // step 0: the box
        for (int i = t; i < V0 + E0; i += kThreads) {
            if (i < V0) {
                uint64_t w0 = 0;
                for (int j = 0; j < D; ++j) {
                    const int up = (i >> j) & 1;
                    b.X[(size_t)i * D + j] = up ? net.hi[j] : net.lo[j];
                    w0 |= (uint64_t)(up ? 1 : 0) << (4 * j);
                    w0 |= (uint64_t)(up ? 0 : 1) << (4 * j + 2);
                }
                b.SG[(size_t)i * Wd] = w0;
                for (int w = 1; w < Wd; ++w) b.SG[(size_t)i * Wd + w] = 0;
            } else {
                const int e = i - V0;
                const int j = e >> (D - 1);
                const int r = e & ((1 << (D - 1)) - 1);
                const int c = ((r >> j) << (j + 1)) | (r & ((1 << j) - 1));
                b.EDG[e] = make_int2(c, c | (1 << j));
            }
        }
        __syncthreads();
    }
    int V = V0, E = E0;
    long long splits = 0, pairs = 0;
    int step = 0;  // neuron steps of this network so far (tags its partner records)
    for (int l = 0; l < nsub && status == BATCH_OK; ++l) {
        const int N = net.widths[l + 1], K = net.widths[l];
        // step 1 for the layer, in place, one 32-row tile at a time
        for (int v0 = 0; v0 < V; v0 += kGemmRows)
            gemm_tile(b, ZS, l == 0 ? b.X : b.Z, l == 0 ? D : ZS, l > 0, V, K, N, net.Wt[l], net.b[l], Wd, lw[l], v0,
                      gl->hs, gl->ws);
        __syncthreads();
        for (int e = t; e < E; e += kThreads) {
            const int2 ab = b.EDG[e];
            const uint64_t *ra = b.SG + (size_t)ab.x * Wd, *rb = b.SG + (size_t)ab.y * Wd;
            int col = kNoCol;
            for (int w = lw[l]; w < lw[l + 1] && col == kNoCol; ++w) col = first_col(ra[w] ^ rb[w], w, lw[l]);
            b.NXT[e] = col == kNoCol ? kNone : (uint16_t)col;
        }
        if (t == 0) s_misc[0] = __hip_atomic_load(&b.CTR[CTR_FLAGS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (s_misc[0]) {  // a vertex on one of this layer's hyperplanes
            status = (s_misc[0] & FLAG_BOUNDS) ? BATCH_INTERNAL : BATCH_DEGENERATE;
            __syncthreads();
            break;
        }
        for (int j = 0; j < N; ++j, ++step) {
            const int S = block_select<SI>(b, E, (uint16_t)j, s_w);
            if (S == 0) {
                if (t == 0 && net.rec) net.rec[step] = StepRec{V, E, 0, E};
                continue;
            }
            if (V + S > Vcap || E + S * D > Ecap || S * P > Kcap) {
                status = BATCH_OVERFLOW;
                break;
            }
            uint32_t tsz = 256;  // (S * P <= Kcap: the doubling ends)
            while (tsz < 2u * (uint32_t)(S * P)) tsz <<= 1;
            if (tsz > A.tcap) {
                status = BATCH_OVERFLOW;
                break;
            }
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
            g.pair_mode = PAIR_HASH;
            g.HT = table;
            g.hmask = tsz - 1;
            g.sbits = kSlotBits;  // (a network's steps have far fewer key slots than 2^24)
            g.zlo = 0;
            g.nx8 = 0;
            g.step = step;
            g.par = 0;
            g.hkeep = A.hbits < 64 ? (1ull << A.hbits) - 1ull : ~0ull;
            g.fbits = 64;
            g.verify = A.verify;
            if (P > 0) {
                for (uint32_t i = t; i < tsz; i += kThreads) table[i] = 0ull;
                __syncthreads();
            }
            if (GS == 32) {
                if (N <= 32) block_split<32, 1>(b, g, V, E, S);
                else if (N <= 64) block_split<32, 2>(b, g, V, E, S);
                else if (N <= 128) block_split<32, 4>(b, g, V, E, S);
                else block_split<32, 8>(b, g, V, E, S);
            } else {
                if (N <= 64) block_split<64, 1>(b, g, V, E, S);
                else if (N <= 128) block_split<64, 2>(b, g, V, E, S);
                else block_split<64, 4>(b, g, V, E, S);
            }
            __syncthreads();
            // the pairing reads partner records other waves of this workgroup stored: past the L1
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            int np = 0;
            if (P > 0) np = block_pair(b, g, V, E + S, S * P, s_w);
            if (t == 0 && net.rec) net.rec[step] = StepRec{V, E, S, E + S + np};
            V += S;
            E += S + np;
            splits += S;
            pairs += np;
            if (t == 0) {
                s_misc[0] = __hip_atomic_load(&b.CTR[CTR_FLAGS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_misc[1] = __hip_atomic_load(&b.CTR[CTR_PFLAGS], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            const int flags = s_misc[0], pflags = s_misc[1];
            __syncthreads();
            if (flags) {
                status = (flags & FLAG_BOUNDS) ? BATCH_INTERNAL : BATCH_DEGENERATE;
                break;
            }
            if (pflags) {
                // a hash collision or a face not met twice: the per-step path decides exactly
                status = BATCH_RETRY;
                break;
            }
        }
    }
    // hand the complex over to the pool
    if (t == 0) {
        long long ov = -1, osg = -1, oe = -1;
        if (status == BATCH_OK) {
            ov = (long long)atomicAdd(&A.pool[0], (unsigned long long)V * D);  // doubles: D differs per network
            osg = (long long)atomicAdd(&A.pool[1], (unsigned long long)V * Wd);
            oe = (long long)atomicAdd(&A.pool[2], (unsigned long long)E);
            if ((unsigned long long)ov + (unsigned long long)V * D > A.capV || (unsigned long long)osg + (unsigned long long)V * Wd > A.capSG ||
                (unsigned long long)oe + E > A.capE)
                status = BATCH_POOL;
        }
        BatchResult r;
        r.status = status;
        r.V = V;
        r.E = E;
        r.Wd = Wd;
        r.offV = ov;
        r.offSG = osg;
        r.offE = oe;
        r.splits = splits;
        r.pairs = pairs;
        A.res[ni] = r;
        s_misc[1] = status;
        s_misc[2] = (int)ov;
        s_misc[3] = (int)osg;
        s_misc[4] = (int)oe;
        s_misc[5] = (int)(ov >> 31);
    }
    __syncthreads();
    if (s_misc[1] == BATCH_OK) {
        const size_t ov = (size_t)A.res[ni].offV, osg = (size_t)A.res[ni].offSG, oe = (size_t)A.res[ni].offE;
        for (size_t i = t; i < (size_t)V * D; i += kThreads) A.oX[ov + i] = b.X[i];
        for (size_t i = t; i < (size_t)V * Wd; i += kThreads) A.oSG[osg + i] = b.SG[i];
        for (size_t i = t; i < (size_t)E; i += kThreads) A.oE[oe + i] = b.EDG[i];
    }
    __syncthreads();
}

// the persistent kernel for one schedule (SI, GS) of the whole batch
template <int SI, int GS>
__global__ __launch_bounds__(kThreads) void k_batch(BatchArgs A) {
    __shared__ GemmLds gl;
    __shared__ int s_w[kThreads / 64];
    __shared__ int s_misc[8];
    __shared__ int s_net;
    Bufs b{};
    for (;;) {
        if (threadIdx.x == 0) s_net = atomicAdd(A.ticket, 1);
        __syncthreads();
        const int k = s_net;
        __syncthreads();
        if (k >= A.n) break;
        const int ni = A.order[k];
        run_net<SI, GS>(A, A.nets[ni], ni, b, &gl, s_w, s_misc);
    }
}

void launch_batch(const BatchArgs &A, int grid, int sched, hipStream_t st) {
    switch (sched) {
        case kSchedSelect8: hipLaunchKernelGGL((k_batch<8, 32>), dim3(grid), dim3(kThreads), 0, st, A); break;
        case kSchedSplit64: hipLaunchKernelGGL((k_batch<16, 64>), dim3(grid), dim3(kThreads), 0, st, A); break;
        case kSchedSelect8 | kSchedSplit64:
            hipLaunchKernelGGL((k_batch<8, 64>), dim3(grid), dim3(kThreads), 0, st, A);
            break;
        default: hipLaunchKernelGGL((k_batch<16, 32>), dim3(grid), dim3(kThreads), 0, st, A); break;
    }
}

}  // namespace pcx
