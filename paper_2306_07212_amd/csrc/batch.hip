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
        // each entry carries its edge's endpoints, so a split starts with one load
        while (hit) {
            const int i = __builtin_ctz(hit);
            hit &= hit - 1;
            const int2 ab = b.EDG[base + i];
            b.SPLE[pos++] = make_int4(base + i, ab.x, ab.y, 0);
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

// Step 1 (Sec. 4.2) for one layer of at most 64 neurons, by the whole
// workgroup on the matrix cores: each wave takes strips of 16 vertex rows and
// computes all 16 CT >= N columns of a strip with FP64 16x16x4 MFMAs (A lane l:
// row l%16, k l/16; B lane l: k l/16, column l%16; result lane l, value i:
// row l/16 + 4i, column l%16), its inputs and the weights read straight from
// memory (no LDS, no barrier: a wave reads every input of its rows before it
// writes them, so the evaluation can be in place). A chain of these MFMAs
// rounds as the sequential FMA chain over k from zero does (the padding of k
// adds a zero, which leaves any sum other than -0 unchanged, and a sum started
// at +0 becomes -0 only if a product underflows), and then + bias: the values
// are those of every other evaluation kernel, bit for bit.
typedef double dbl4 __attribute__((ext_vector_type(4)));

// (Not inlined, and given plain pointers rather than the workgroup's Bufs, so
// that its registers and the Bufs stay out of the split's register allocation.)
// (The pointers are taken as global memory, so that the loads are global
// loads whose completion is counted in order, and every operand load is made
// unconditional, from a clamped in-bounds address, with the value selected
// after it: the loads of a round are all in flight together.)
typedef const __attribute__((address_space(1))) double gcdouble;
typedef const __attribute__((address_space(1))) uint64_t gcuint64;
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) uint64_t guint64;

template <int CT>
__device__ __noinline__ void eval_mfma(double *Zo_, uint64_t *SGo_, uint64_t *LWo_, int *ctr, int ZS,
                                       const double *in_, int in_stride, int relu, int V, int K, int N,
                                       const double *Wt_, const double *bias_, int Wd, int lw0) {
    gdouble *Zo = (gdouble *)Zo_;
    guint64 *SGo = (guint64 *)SGo_, *LWo = (guint64 *)LWo_;
    gcuint64 *in = (gcuint64 *)in_, *Wt = (gcuint64 *)Wt_;
    gcdouble *bias = (gcdouble *)bias_;
    const int l = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = l & 15, q = l >> 4;
    double bv[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) bv[ct] = ct * 16 + r < N ? bias[ct * 16 + r] : 0.0;
    int zero = 0;
    for (int v0 = wave * 16; v0 < V; v0 += 16 * (kThreads / 64)) {
        const bool arow = v0 + r < V;
        gcuint64 *hp = in + (size_t)(arow ? v0 + r : 0) * in_stride;
        dbl4 acc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) acc[ct] = dbl4{0.0, 0.0, 0.0, 0.0};
        // four k-steps of 4 per round, each with its own operand registers: a
        // step's operands for the next round are loaded right after its MFMAs
        // issue, three steps ahead of their use, as raw bits from clamped
        // in-bounds addresses; the zeros past K (weights) and the ReLU are
        // applied when the step is used, so no load waits on a condition
        uint64_t ar[4], br[4][CT];
        auto load = [&](int k0, uint64_t &a, uint64_t *bw) {
            const int k = k0 + q, kc = k < K ? k : K - 1;
            a = hp[kc];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = ct * 16 + r;
                bw[ct] = Wt[(size_t)kc * N + (col < N ? col : N - 1)];
            }
        };
#pragma unroll
        for (int st = 0; st < 4; ++st) load(4 * st, ar[st], br[st]);
        // (every round is whole: a step past K has zero weights, adding a zero
        // to the sum)
        for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bool kin = k0 + 4 * st + q < K;
                const double h = __builtin_bit_cast(double, ar[st]);
                const double af = relu ? (h > 0.0 ? h : 0.0) : h;
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    const uint64_t m = (kin && ct * 16 + r < N) ? ~0ull : 0ull;
                    const double bf = __builtin_bit_cast(double, br[st][ct] & m);
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc[ct], 0, 0, 0);
                }
                load(k0 + 16 + 4 * st, ar[st], br[st]);
                // (keeps the loads here, in flight, rather than moved next to their use)
                asm volatile("" ::: "memory");
            }
        }
        // bias, store, and the layer's sign words (word p from tiles 2p and 2p+1)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int v = v0 + q + 4 * i;
            uint64_t pb[CT], nb[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int col = ct * 16 + r;
                const bool ok = v < V && col < N;
                double z = 0.0;
                if (ok) {
                    z = acc[ct][i] + bv[ct];
                    Zo[(size_t)v * ZS + col] = z;
                    zero |= (z == 0.0);
                }
                pb[ct] = __ballot(ok && z > 0.0);
                nb[ct] = __ballot(ok && z < 0.0);
            }
            const int sh = 16 * q;
#pragma unroll
            for (int p = 0; p < (CT + 1) / 2; ++p) {
                if (r == p && v < V) {
                    uint32_t pos = (uint32_t)((pb[2 * p] >> sh) & 0xFFFFu);
                    uint32_t neg = (uint32_t)((nb[2 * p] >> sh) & 0xFFFFu);
                    if (2 * p + 1 < CT) {
                        pos |= (uint32_t)((pb[2 * p + 1] >> sh) & 0xFFFFu) << 16;
                        neg |= (uint32_t)((nb[2 * p + 1] >> sh) & 0xFFFFu) << 16;
                    }
                    const uint64_t cw = codes_of(pos, neg);
                    SGo[(size_t)v * Wd + lw0 + p] = cw;
                    if (LWo) LWo[(size_t)v * 8 + p] = cw;
                }
            }
        }
    }
    if (zero) raise_flag(ctr, FLAG_ZERO_SIGN);
}

template <int G, int NC>
__device__ __forceinline__ void block_split(const Bufs &b, const StepGeom &g, int V0, int E0, int S) {
    constexpr int groups = kThreads / G;
    const int lane = threadIdx.x % G, grp = threadIdx.x / G, half = (threadIdx.x & 63) / G;
    for (int s = grp; s < S; s += groups) {
        const int4 q = b.SPLE[s];
        const int2 ab = make_int2(q.y, q.z);
        if (split_entry_ok(b, q.x, E0) && split_edge_ok(ab, V0))
            split_core<G, NC, false>(b, g, V0, E0, s, q.x, ab, lane, half, S * g.P);
        else if (lane == 0)
            raise_flag(b.CTR, FLAG_BOUNDS);
    }
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
    b.SPL = nullptr;
    b.SPLE = (int4 *)(eb + (size_t)Ecap * 16);
    char *kb = eb + (size_t)Ecap * 32;
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
        // step 1 for the layer, in place: layers of up to 64 neurons on the
        // matrix cores, wider ones one 32-row tile at a time
        {
            const double *in = l == 0 ? b.X : b.Z;
            const int ins = l == 0 ? D : ZS;
            if (N <= 16) eval_mfma<1>(b.Z, b.SG, b.LW, b.CTR, ZS, in, ins, l > 0, V, K, N, net.Wt[l], net.b[l], Wd, lw[l]);
            else if (N <= 32) eval_mfma<2>(b.Z, b.SG, b.LW, b.CTR, ZS, in, ins, l > 0, V, K, N, net.Wt[l], net.b[l], Wd, lw[l]);
            else if (N <= 48) eval_mfma<3>(b.Z, b.SG, b.LW, b.CTR, ZS, in, ins, l > 0, V, K, N, net.Wt[l], net.b[l], Wd, lw[l]);
            else if (N <= 64) eval_mfma<4>(b.Z, b.SG, b.LW, b.CTR, ZS, in, ins, l > 0, V, K, N, net.Wt[l], net.b[l], Wd, lw[l]);
            else
                for (int v0 = 0; v0 < V; v0 += kGemmRows)
                    gemm_tile(b, ZS, in, ins, l > 0, V, K, N, net.Wt[l], net.b[l], Wd, lw[l], v0, gl->hs, gl->ws);
        }
        __syncthreads();
        // each edge's first crossing in the layer: four edges per thread at a
        // time, their endpoints' first two words of the layer loaded together
        {
            const int w0 = lw[l], nw = lw[l + 1] - lw[l];
            for (int e0 = t; e0 < E; e0 += 4 * kThreads) {
                int2 ab[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = e0 + i * kThreads;
                    ab[i] = e < E ? b.EDG[e] : make_int2(0, 0);
                }
                uint64_t x0[4], x1[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint64_t *ra = b.SG + (size_t)ab[i].x * Wd + w0, *rb = b.SG + (size_t)ab[i].y * Wd + w0;
                    x0[i] = ra[0] ^ rb[0];
                    x1[i] = nw > 1 ? ra[1] ^ rb[1] : 0ull;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = e0 + i * kThreads;
                    if (e >= E) continue;
                    int col = first_col(x0[i], w0, w0);
                    if (col == kNoCol && nw > 1) col = first_col(x1[i], w0 + 1, w0);
                    if (col == kNoCol && nw > 2) {
                        const uint64_t *ra = b.SG + (size_t)ab[i].x * Wd, *rb = b.SG + (size_t)ab[i].y * Wd;
                        for (int w = w0 + 2; w < w0 + nw && col == kNoCol; ++w) col = first_col(ra[w] ^ rb[w], w, w0);
                    }
                    b.NXT[e] = col == kNoCol ? kNone : (uint16_t)col;
                }
            }
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
            if (GS == 16) {
                if (N <= 32) block_split<16, 2>(b, g, V, E, S);
                else if (N <= 64) block_split<16, 4>(b, g, V, E, S);
                else if (N <= 128) block_split<16, 8>(b, g, V, E, S);
                else block_split<32, 8>(b, g, V, E, S);
            } else if (GS == 32) {
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
__global__ __launch_bounds__(kThreads, 2) void k_batch(BatchArgs A) {
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
        case kSchedSplit16: hipLaunchKernelGGL((k_batch<16, 16>), dim3(grid), dim3(kThreads), 0, st, A); break;
        case kSchedSelect8 | kSchedSplit16:
            hipLaunchKernelGGL((k_batch<8, 16>), dim3(grid), dim3(kThreads), 0, st, A);
            break;
        default: hipLaunchKernelGGL((k_batch<16, 32>), dim3(grid), dim3(kThreads), 0, st, A); break;
    }
}

}  // namespace pcx
