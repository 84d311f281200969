// Device kernels of libpcx.so: edge subdivision (Berzins 2023, Sec. 4.2) on
// gfx950. One neuron step is: compaction of the splitting edges (step 3),
// interpolation + split + 2-face keys (steps 4-5), radix sort of the keys and
// pairing into intersecting edges (step 5). Each layer starts with the
// pre-activation evaluation (step 1) and a scan that records, per edge, the
// first neuron of the layer whose sign differs at its endpoints (steps 2-3).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace pcx {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    // 64-bit finaliser (splitmix64 constants, Steele et al. 2014)
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

// Hash of one sign-row word at position w; a row hashes to the sum over words,
// so a single perturbed entry changes the hash in O(1).
__device__ __forceinline__ uint64_t word_hash(int w, uint64_t v) {
    return mix64(v + (uint64_t)(w + 1) * 0x9e3779b97f4a7c15ull);
}

// spread the 32 bits of x to the even bit positions of a 64-bit word
__device__ __forceinline__ uint64_t part1by1(uint32_t x) {
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// 2-bit codes of 32 entries from their positive / negative masks
__device__ __forceinline__ uint64_t codes_of(uint32_t pos, uint32_t neg) {
    return part1by1(pos) | (part1by1(neg) << 1);
}

// entries strictly before entry n = (wn, bn) inside word w
__device__ __forceinline__ uint64_t lt_mask(int w, int wn, int bn) {
    if (w < wn) return ~0ull;
    if (w > wn) return 0ull;
    return bn == 0 ? 0ull : ((1ull << bn) - 1ull);
}

// entries strictly after entry n inside this layer's words
__device__ __forceinline__ uint64_t gt_mask(int w, int wn, int bn, int lw1) {
    if (w < wn || w >= lw1) return 0ull;
    if (w > wn) return ~0ull;
    return bn + 2 >= 64 ? 0ull : ~((1ull << (bn + 2)) - 1ull);
}

constexpr int kNoCol = 0x7fffffff;

__device__ __forceinline__ int first_col(uint64_t x, int w, int lw0) {
    if (!x) return kNoCol;
    return (w - lw0) * 32 + (__builtin_ctzll(x) >> 1);
}

__device__ __forceinline__ void raise_flag(int *ctr, int f) { atomicOr(&ctr[CTR_FLAGS], f); }

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}
template <int G>
__device__ __forceinline__ int group_min(int v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, G));
    return v;
}
template <int G>
__device__ __forceinline__ int group_or(int v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v |= __shfl_xor(v, o, G);
    return v;
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
    const int t = threadIdx.x;
    const int tc = t & 31, tv = t >> 5;
    const int v0 = blockIdx.x * kGemmRows;
    double acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[i][c] = 0.0;

    for (int k0 = 0; k0 < K; k0 += kGemmK) {
        for (int idx = t; idx < kGemmRows * kGemmK; idx += kThreads) {
            const int r = idx / kGemmK, k = idx % kGemmK;
            const int v = v0 + r;
            double h = 0.0;
            if (v < V && k0 + k < K) {
                h = in[(size_t)v * in_stride + k0 + k];
                if (relu) h = h > 0.0 ? h : 0.0;
            }
            hs[r][k] = h;
        }
        for (int idx = t; idx < kGemmK * kMaxWidth; idx += kThreads) {
            const int k = idx / kMaxWidth, c = idx % kMaxWidth;
            ws[k][c] = (k0 + k < K && c < N) ? Wt[(size_t)(k0 + k) * N + c] : 0.0;
        }
        __syncthreads();
        const int kc = min(kGemmK, K - k0);
        for (int kk = 0; kk < kc; ++kk) {
            double h[4], w[8];
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = hs[tv * 4 + i][kk];
#pragma unroll
            for (int c = 0; c < 8; ++c) w[c] = ws[kk][tc + 32 * c];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[i][c] += h[i] * w[c];
        }
        __syncthreads();
    }
    const int half = (t >> 5) & 1;  // which 32-lane half of the wave holds this vertex group
    const int nwords = (N + 31) >> 5;
    int zero = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int v = v0 + tv * 4 + i;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int col = tc + 32 * c;
            const bool ok = v < V && col < N;
            double z = 0.0;
            if (ok) {
                z = acc[i][c] + bias[col];
                b.Z[(size_t)v * ZS + col] = z;
                zero |= (z == 0.0);
            }
            const uint64_t pb = __ballot(ok && z > 0.0);
            const uint64_t nb = __ballot(ok && z < 0.0);
            if (tc == 0 && v < V && c < nwords)
                b.SG[(size_t)v * Wd + lw0 + c] = codes_of((uint32_t)(pb >> (32 * half)), (uint32_t)(nb >> (32 * half)));
        }
    }
    if (zero) raise_flag(b.CTR, FLAG_ZERO_SIGN);
}

void launch_gemm(const Bufs &b, int ZS, const double *in, int in_stride, int relu, int V, int K, int N,
                 const double *Wt, const double *bias, int Wd, int lw0, hipStream_t st) {
    if (V <= 0) return;
    const int grid = (V + kGemmRows - 1) / kGemmRows;
    hipLaunchKernelGGL(k_gemm, dim3(grid), dim3(kThreads), 0, st, b, ZS, in, in_stride, relu, V, K, N, Wt, bias,
                       Wd, lw0);
}

// ------------------------------------ steps 2-3 at a layer start, per edge
//
// For every edge, the first neuron of the layer at which its endpoints carry
// different signs (both are nonzero there: every vertex has all of this
// layer's entries set by the evaluation above). Edges with no such neuron
// never split in this layer.
__global__ __launch_bounds__(kThreads) void k_next_all(Bufs b, int V, int Wd, int lw0, int lw1) {
    const int E = b.CTR[CTR_E];
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x) {
        const int2 ab = b.EDG[e];
        if ((unsigned)ab.x >= (unsigned)V || (unsigned)ab.y >= (unsigned)V) {
            raise_flag(b.CTR, FLAG_BOUNDS);
            b.NXT[e] = kNone;
            continue;
        }
        const uint64_t *ra = b.SG + (size_t)ab.x * Wd;
        const uint64_t *rb = b.SG + (size_t)ab.y * Wd;
        int col = kNoCol;
        for (int w = lw0; w < lw1 && col == kNoCol; ++w) col = first_col(ra[w] ^ rb[w], w, lw0);
        b.NXT[e] = col == kNoCol ? kNone : (uint16_t)col;
    }
}

void launch_next_all(const Bufs &b, int V, int Wd, int lw0, int lw1, int Ehint, hipStream_t st) {
    int grid = (Ehint + kThreads - 1) / kThreads;
    grid = grid < 1 ? 1 : (grid > 8192 ? 8192 : grid);
    hipLaunchKernelGGL(k_next_all, dim3(grid), dim3(kThreads), 0, st, b, V, Wd, lw0, lw1);
}

// ---------------------------------------------- step 3: splitting edges
//
// Ordered stream compaction of {e : NXT[e] == target}. The edge array is cut
// into kSelBlocks contiguous chunks, one per workgroup. The first kernel counts
// the matches of each chunk; the second re-reads its chunk, takes its offset
// as the sum of the counts of the chunks before it, and writes the matching
// ids in order (wave ballot / prefix sum inside each tile). No workgroup ever
// waits on another, so the scan runs at streaming speed on all XCDs.
__device__ __forceinline__ uint32_t match16(const uint16_t *__restrict__ nxt, int base, int E, uint16_t target) {
    uint32_t hit = 0;
    if (base + kSelItems <= E) {
        const uint4 *p = reinterpret_cast<const uint4 *>(nxt + base);
        const uint4 a = p[0], c = p[1];
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if ((uint16_t)(w[i] & 0xFFFFu) == target) hit |= 1u << (2 * i);
            if ((uint16_t)(w[i] >> 16) == target) hit |= 1u << (2 * i + 1);
        }
    } else {
        for (int i = 0; i < kSelItems; ++i)
            if (base + i < E && nxt[base + i] == target) hit |= 1u << i;
    }
    return hit;
}

__device__ __forceinline__ void sel_chunk(int E, int &c0, int &c1) {
    const int per = ((E + (int)gridDim.x - 1) / (int)gridDim.x + kSelItems - 1) / kSelItems * kSelItems;
    c0 = min(E, (int)blockIdx.x * per);
    c1 = min(E, c0 + per);
}

__global__ __launch_bounds__(kThreads) void k_sel_count(Bufs b, uint16_t target) {
    __shared__ int s_w[kThreads / 64];
    const int E = b.CTR[CTR_E];
    int c0, c1;
    sel_chunk(E, c0, c1);
    int cnt = 0;
    for (int base = c0 + threadIdx.x * kSelItems; base < c1; base += kSelTile)
        cnt += __popc(match16(b.NXT, base, c1, target));
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
        b.SELCNT[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_sel_scatter(Bufs b, uint16_t target) {
    __shared__ int s_w[kThreads / 64];
    __shared__ int s_base;
    const int E = b.CTR[CTR_E];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int c0, c1;
    sel_chunk(E, c0, c1);
    // offset of this chunk: sum of the counts of the chunks before it
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
    int run = s_base;
    for (int tb = c0; tb < c1; tb += kSelTile) {
        const int base = tb + t * kSelItems;
        uint32_t hit = base < c1 ? match16(b.NXT, base, c1, target) : 0u;
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
            b.SPL[pos++] = base + i;
        }
        run += total;
    }
}

void launch_select(const Bufs &b, uint16_t target, hipStream_t st) {
    hipLaunchKernelGGL(k_sel_count, dim3(kSelBlocks), dim3(kThreads), 0, st, b, target);
    hipLaunchKernelGGL(k_sel_scatter, dim3(kSelBlocks), dim3(kThreads), 0, st, b, target);
}

// ----------------------------------------------- 2-face hash table (f1)
//
// Open addressing with linear probing on the full 64-bit key. The first
// splitting edge to reach a 2-face claims the slot with a 64-bit CAS and
// records its key slot in `a`; the second finds the key and records itself in
// `b`. A third arrival means the 2-face is not met by exactly two splitting
// edges (Sec. 4.2.2) and raises FLAG_RUN.
__device__ __forceinline__ void hash_insert(HEntry *T, uint32_t mask, uint64_t H, uint32_t u, int *ctr) {
    uint32_t h = (uint32_t)H & mask;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const unsigned long long prev = atomicCAS(&T[h].key, 0ull, (unsigned long long)H);
        if (prev == 0ull) {
            T[h].a = u + 1;
            return;
        }
        if (prev == (unsigned long long)H) {
            if (atomicCAS(&T[h].b, 0u, u + 1) != 0u) raise_flag(ctr, FLAG_RUN);
            return;
        }
        h = (h + 1) & mask;
    }
    raise_flag(ctr, FLAG_BOUNDS);  // table full: cannot happen at load factor <= 1/2
}

__device__ __forceinline__ int hash_find(const HEntry *T, uint32_t mask, uint64_t H) {
    uint32_t h = (uint32_t)H & mask;
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        const unsigned long long k = T[h].key;
        if (k == (unsigned long long)H) return (int)h;
        if (k == 0ull) return -1;
        h = (h + 1) & mask;
    }
    return -1;
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
// holds column k*G + c; the sign words of the layer come straight from the
// chunk ballots (no LDS).
template <int G, int NC>
__global__ __launch_bounds__(kThreads) void k_split(Bufs b, StepGeom g, int V0, int E0, int S) {
    constexpr int groups = kThreads / G;
    constexpr int wpc = G / 32;  // sign words per chunk
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int half = (threadIdx.x & 63) / G;  // G == 32: which half of the wave
    const int D = g.D, Wd = g.Wd, ZS = g.ZS, j = g.j, N = g.Nl;
    const int nw = g.lw1 - g.lw0;
    for (int s = blockIdx.x * groups + grp; s < S; s += gridDim.x * groups) {
        const int e = b.SPL[s];
        if ((unsigned)e >= (unsigned)E0) {
            if (lane == 0) raise_flag(b.CTR, FLAG_BOUNDS);
            continue;
        }
        const int2 ab = b.EDG[e];
        if ((unsigned)ab.x >= (unsigned)V0 || (unsigned)ab.y >= (unsigned)V0) {
            if (lane == 0) raise_flag(b.CTR, FLAG_BOUNDS);
            continue;
        }
        const double *Za = b.Z + (size_t)ab.x * ZS, *Zb = b.Z + (size_t)ab.y * ZS;
        const uint64_t *Ra = b.SG + (size_t)ab.x * Wd, *Rb = b.SG + (size_t)ab.y * Wd;
        // ---- loads
        const double za = Za[j], zb = Zb[j];
        double A[NC], B[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int c = k * G + lane;
            A[k] = c < N ? Za[c] : 0.0;
            B[k] = c < N ? Zb[c] : 0.0;
        }
        const uint64_t wa0 = lane < Wd ? Ra[lane] : 0ull, wb0 = lane < Wd ? Rb[lane] : 0ull;
        const double xa = lane < D ? b.X[(size_t)ab.x * D + lane] : 0.0;
        const double xb = lane < D ? b.X[(size_t)ab.y * D + lane] : 0.0;
        // ---- interpolation
        const bool apos = za > 0.0;
        const double zp = apos ? za : zb, zq = apos ? zb : za;
        const double tt = zp / (zp - zq);
        const size_t x0 = (size_t)V0 + s;
        int bad = 0;
        double Zx[NC];
        uint64_t pb[NC], nb[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int c = k * G + lane;
            const bool in = c < N;
            const double p = apos ? A[k] : B[k], q = apos ? B[k] : A[k];
            const double z = (c == j) ? 0.0 : p + tt * (q - p);
            if (in && c > j && z == 0.0) bad |= FLAG_ZERO_SIGN;
            Zx[k] = z;
            pb[k] = __ballot(in && z > 0.0);
            nb[k] = __ballot(in && z < 0.0);
        }
        const double xp = apos ? xa : xb, xq = apos ? xb : xa;
        const double x0c = xp + tt * (xq - xp);
        // ---- sign row of x0, hash of the edge's sign-vector, zeros, next crossings
        uint64_t hsum = 0, rx0 = 0, f0 = 0;
        int nz = 0, nkeys = 0, da = kNoCol, db = kNoCol;
        for (int w = lane, it = 0; w < Wd; w += G, ++it) {
            const uint64_t wa = it == 0 ? wa0 : Ra[w], wb = it == 0 ? wb0 : Rb[w];
            const uint64_t lt = lt_mask(w, g.wn, g.bn), gt = gt_mask(w, g.wn, g.bn, g.lw1);
            const uint64_t f = (wa | wb) & lt;
            if (f & (f >> 1) & 0x5555555555555555ull) bad |= FLAG_CONFLICT;
            uint64_t cw = 0;
            const int u = w - g.lw0;
            if (u >= 0 && u < nw) {
                const int ku = u / wpc, sh = 32 * (wpc == 2 ? (u & 1) : half);
                uint64_t P = 0, Q = 0;
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    if (k == ku) {
                        P = pb[k];
                        Q = nb[k];
                    }
                cw = codes_of((uint32_t)(P >> sh), (uint32_t)(Q >> sh));
            }
            const uint64_t rx = f | (cw & gt);
            if (it == 0) {
                rx0 = rx;
                f0 = f;
            } else {
                b.SG[x0 * Wd + w] = rx;
            }
            if (w <= g.wn) hsum += word_hash(w, f);
            const uint64_t zm = ~(f | (f >> 1)) & b.VALID[w] & lt;
            const int zc = __popcll(zm);
            nz += zc;
            nkeys += (w == 0) ? zc : 2 * zc;  // box entries all live in word 0
            da = min(da, first_col((wa ^ rx) & gt, w, g.lw0));
            db = min(db, first_col((rx ^ wb) & gt, w, g.lw0));
        }
        hsum = group_sum<G>(hsum);
        nz = group_sum<G>(nz);
        const int ktot = group_sum<G>(nkeys);
        da = group_min<G>(da);
        db = group_min<G>(db);
        bad = group_or<G>(bad);
        // ---- stores
        if (lane < D) b.X[x0 * D + lane] = x0c;
        double *Zo = b.Z + x0 * ZS;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const int c = k * G + lane;
            if (c < N) Zo[c] = Zx[k];
        }
        if (lane < Wd) b.SG[x0 * Wd + lane] = rx0;
        if (lane == 0) {
            if (nz != D - 1 || ktot > g.P) bad |= FLAG_ZERO_COUNT;
            if (bad) raise_flag(b.CTR, bad);
            b.EDG[e] = make_int2(ab.x, (int)x0);
            b.EDG[E0 + s] = make_int2((int)x0, ab.y);
            b.NXT[e] = da == kNoCol ? kNone : (uint16_t)da;
            b.NXT[E0 + s] = db == kNoCol ? kNone : (uint16_t)db;
            if (b.PQ) b.PQ[x0] = apos ? ab : make_int2(ab.y, ab.x);
        }
        if (g.P > 0) {
            // exclusive prefix of key counts over the group's lanes
            int incl = nkeys;
#pragma unroll
            for (int o = 1; o < G; o <<= 1) {
                const int y = __shfl_up(incl, o, G);
                if (lane >= o) incl += y;
            }
            int r = incl - nkeys;
            const size_t sbase = (size_t)s * g.P;
            for (int w = lane, it = 0; w < Wd && nkeys; w += G, ++it) {
                const uint64_t lt = lt_mask(w, g.wn, g.bn);
                const uint64_t f = it == 0 ? f0 : ((Ra[w] | Rb[w]) & lt);
                uint64_t zm = ~(f | (f >> 1)) & b.VALID[w] & lt;
                if (!zm) continue;
                const uint64_t hw = word_hash(w, f);
                while (zm) {
                    const int bit = __builtin_ctzll(zm);
                    zm &= zm - 1;
                    for (int minus = 0; minus < (w == 0 ? 1 : 2); ++minus) {
                        const uint64_t h = hsum - hw + word_hash(w, f | ((minus ? 2ull : 1ull) << bit));
                        if (r < g.P) {
                            const size_t slot = sbase + r;
                            b.PINFO[slot] = ((uint32_t)w << 8) | ((uint32_t)bit << 1) | (uint32_t)minus;
                            if (g.pair_mode == PAIR_SORT) {
                                b.K32a[slot] = (uint32_t)(h >> 33);
                                b.FULL[slot] = h;
                            } else {
                                const uint64_t hk = h | (1ull << 63);  // never 0 (= empty)
                                b.FULL[slot] = hk;
                                hash_insert(g.HT, g.hmask, hk, (uint32_t)slot, b.CTR);
                            }
                        }
                        ++r;
                    }
                }
            }
            for (int rr = ktot + lane; rr < g.P; rr += G) {
                if (g.pair_mode == PAIR_SORT) b.K32a[sbase + rr] = kSentinel;
                else b.FULL[sbase + rr] = 0ull;
            }
        }
    }
}

void launch_split(const Bufs &b, const StepGeom &g, int V0, int E0, int S, hipStream_t st) {
    if (S <= 0) return;
    const int G = g.Nl > 32 ? 64 : 32;
    const int groups = kThreads / G;
    int grid = (S + groups - 1) / groups;
    grid = grid > 16384 ? 16384 : grid;
    if (G == 32)
        hipLaunchKernelGGL((k_split<32, 1>), dim3(grid), dim3(kThreads), 0, st, b, g, V0, E0, S);
    else if (g.Nl <= 64)
        hipLaunchKernelGGL((k_split<64, 1>), dim3(grid), dim3(kThreads), 0, st, b, g, V0, E0, S);
    else if (g.Nl <= 128)
        hipLaunchKernelGGL((k_split<64, 2>), dim3(grid), dim3(kThreads), 0, st, b, g, V0, E0, S);
    else
        hipLaunchKernelGGL((k_split<64, 4>), dim3(grid), dim3(kThreads), 0, st, b, g, V0, E0, S);
}

// ---------------------------------------------------- step 5b: radix sort
//
// Stable LSD radix sort of (32-bit key, slot) pairs, 8-bit digits, 4 passes.
// Per pass: tile histograms, one exclusive scan over [digit][tile], and a
// stable scatter that ranks equal digits inside a tile by wave ballots.
__global__ __launch_bounds__(kThreads) void k_sort_hist(const uint32_t *__restrict__ keys, int n, int shift,
                                                         uint32_t *__restrict__ hist, int ntiles) {
    __shared__ uint32_t h[kSortBins];
    const int t = threadIdx.x, tile = blockIdx.x;
    h[t] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = tile * kSortTile + i * kThreads + t;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(size_t)t * ntiles + tile] = h[t];
}

// exclusive scan of the [digit][tile] histogram in place: one workgroup of
// 1024 threads, 4 consecutive counters per thread, coalesced 16-byte accesses
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *hist, int len) {
    __shared__ uint32_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < len; base += 4096) {
        const int i0 = base + 4 * t;
        uint32_t x[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) x[k] = i0 + k < len ? hist[i0 + k] : 0u;
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
        for (int w = 0; w < 16; ++w) {
            const uint32_t v = wsum[w];
            if (w < wave) woff += v;
            total += v;
        }
        uint32_t run = carry + woff + incl - tsum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < len) hist[i0 + k] = run;
            run += x[k];
        }
        carry += total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(const uint32_t *__restrict__ kin,
                                                            const uint32_t *__restrict__ vin,
                                                            uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                            int n, int shift, const uint32_t *__restrict__ hist,
                                                            int ntiles) {
    __shared__ uint32_t base[kSortBins];
    __shared__ uint32_t wcnt[kThreads / 64][kSortBins];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, tile = blockIdx.x;
    base[t] = hist[(size_t)t * ntiles + tile];
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = 0; i < kSortItems; ++i) {
        const int idx = tile * kSortTile + i * kThreads + t;
        const bool valid = idx < n;
        const uint32_t k = valid ? kin[idx] : 0u;
        const uint32_t v = valid ? (vin ? vin[idx] : (uint32_t)idx) : 0u;
        const uint32_t d = (k >> shift) & 0xFF;
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

void launch_sort(const Bufs &b, int n, hipStream_t st) {
    if (n <= 0) return;
    const int ntiles = (n + kSortTile - 1) / kSortTile;
    uint32_t *ka = b.K32a, *kb = b.K32b, *va = b.VALa, *vb = b.VALb;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(kThreads), 0, st, ka, n, shift, b.HIST, ntiles);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, b.HIST, kSortBins * ntiles);
        hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(kThreads), 0, st, ka, pass == 0 ? nullptr : va, kb, vb,
                           n, shift, b.HIST, ntiles);
        uint32_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    // four passes: the result is back in K32a / VALa
}

// ------------------------------------------- step 5c: pair and connect
//
// In the sorted key array every run of equal keys has even length (each
// splitting 2-face is met by exactly two splitting edges, Sec. 4.2.2), so the
// run starting at sorted position i owns output edges i/2, i/2+1, ... A run of
// two is the common case; a longer run (two faces whose 31-bit keys collide)
// is grouped by the full 64-bit hash. Every pair is verified by comparing the
// two perturbed sign-vectors word by word. The new edge joins the two new
// vertices; its sign is the face's with 0 at the current neuron (Sec. 4.2.2).
__device__ void emit_pair(const Bufs &b, const StepGeom &g, int V0, int nslots, int sa, int sb, size_t out) {
    if ((unsigned)sa >= (unsigned)nslots || (unsigned)sb >= (unsigned)nslots) {
        raise_flag(b.CTR, FLAG_BOUNDS);
        return;
    }
    const int xa = V0 + sa / g.P, xb = V0 + sb / g.P;
    const uint32_t pa = b.PINFO[sa], pb = b.PINFO[sb];
    const int wa = (int)(pa >> 8), wb = (int)(pb >> 8);
    const uint64_t ca = ((pa & 1u) ? 2ull : 1ull) << ((pa >> 1) & 63u);
    const uint64_t cb = ((pb & 1u) ? 2ull : 1ull) << ((pb >> 1) & 63u);
    const uint64_t *Ra = b.SG + (size_t)xa * g.Wd, *Rb = b.SG + (size_t)xb * g.Wd;
    bool same = b.FULL[sa] == b.FULL[sb];
    for (int w = 0; w <= g.wn && same; ++w) {
        const uint64_t lt = lt_mask(w, g.wn, g.bn);
        const uint64_t fa = (Ra[w] & lt) | (w == wa ? ca : 0ull);
        const uint64_t fb = (Rb[w] & lt) | (w == wb ? cb : 0ull);
        same = fa == fb;
    }
    if (!same) raise_flag(b.CTR, FLAG_VERIFY);
    int col = kNoCol;
    for (int w = g.wn; w < g.lw1 && col == kNoCol; ++w)
        col = first_col((Ra[w] ^ Rb[w]) & gt_mask(w, g.wn, g.bn, g.lw1), w, g.lw0);
    b.EDG[out] = make_int2(xa, xb);
    b.NXT[out] = col == kNoCol ? kNone : (uint16_t)col;
}

__global__ __launch_bounds__(kThreads) void k_pair(Bufs b, StepGeom g, int V0, int E1, int nslots) {
    const uint32_t *KS = b.K32a;
    const uint32_t *VS = b.VALa;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += gridDim.x * blockDim.x) {
        const uint32_t k = KS[i];
        // valid keys (< 2^31) sort before the sentinels: the last valid one fixes the edge count
        if (k == kSentinel) {
            if (i == 0) b.CTR[CTR_E] = E1;
            continue;
        }
        if (i + 1 == nslots || KS[i + 1] == kSentinel) b.CTR[CTR_E] = E1 + (i + 1) / 2;
        if (i > 0 && KS[i - 1] == k) continue;  // not the start of a run
        int j = i + 1;
        while (j < nslots && KS[j] == k) ++j;
        const int len = j - i;
        if (len == 2) {
            emit_pair(b, g, V0, nslots, (int)VS[i], (int)VS[i + 1], (size_t)E1 + i / 2);
            continue;
        }
        if ((len & 1) || len > 32) {
            raise_flag(b.CTR, FLAG_RUN);
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
                raise_flag(b.CTR, FLAG_RUN);
                break;
            }
            used |= (1u << u) | (1u << w);
            emit_pair(b, g, V0, nslots, (int)VS[i + u], (int)VS[i + w], (size_t)E1 + i / 2 + np++);
        }
    }
}

void launch_pair(const Bufs &b, const StepGeom &g, int V0, int E1, int nslots, hipStream_t st) {
    int grid = (nslots + kThreads - 1) / kThreads;
    grid = grid < 1 ? 1 : (grid > 8192 ? 8192 : grid);
    hipLaunchKernelGGL(k_pair, dim3(grid), dim3(kThreads), 0, st, b, g, V0, E1, nslots);
}

// ---------------------------------- step 5c with the hash table (f1)
//
// Every valid key slot u finds its 2-face entry; the smaller of the two slots
// owns the pair. Owners are emitted in slot order (chunk counts, then an
// ordered scatter, as in the compaction), so the edge list is deterministic.
__device__ __forceinline__ bool hash_owner(const Bufs &b, const StepGeom &g, int u, int nslots, int &partner) {
    const uint64_t H = b.FULL[u];
    if (H == 0ull) return false;
    const int h = hash_find(g.HT, g.hmask, H);
    if (h < 0) {
        raise_flag(b.CTR, FLAG_BOUNDS);
        return false;
    }
    const uint32_t a = g.HT[h].a, c = g.HT[h].b;
    if (c == 0u || a == 0u) {
        raise_flag(b.CTR, FLAG_RUN);
        return false;
    }
    const uint32_t p = (a - 1 == (uint32_t)u) ? c - 1 : a - 1;
    if (p >= (uint32_t)nslots) {
        raise_flag(b.CTR, FLAG_BOUNDS);
        return false;
    }
    partner = (int)p;
    return (uint32_t)u < p;
}

__device__ __forceinline__ void pair_chunk(int n, int &c0, int &c1) {
    const int per = ((n + (int)gridDim.x - 1) / (int)gridDim.x + kPairItems - 1) / kPairItems * kPairItems;
    c0 = min(n, (int)blockIdx.x * per);
    c1 = min(n, c0 + per);
}

__global__ __launch_bounds__(kThreads) void k_hpair_count(Bufs b, StepGeom g, int nslots) {
    __shared__ int s_w[kThreads / 64];
    int c0, c1;
    pair_chunk(nslots, c0, c1);
    int cnt = 0;
    for (int base = c0 + threadIdx.x * kPairItems; base < c1; base += kThreads * kPairItems)
        for (int i = 0; i < kPairItems; ++i) {
            int partner;
            if (base + i < c1 && hash_owner(b, g, base + i, nslots, partner)) ++cnt;
        }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
        b.SELCNT[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_hpair_emit(Bufs b, StepGeom g, int V0, int E1, int nslots,
                                                          HEntry *clear_t, uint32_t clear_n) {
    __shared__ int s_w[kThreads / 64];
    __shared__ int s_base;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    // the table of the previous step is no longer read: make it empty again
    for (uint32_t i = blockIdx.x * kThreads + t; i < clear_n; i += gridDim.x * kThreads) {
        HEntry z;
        z.key = 0ull;
        z.a = 0u;
        z.b = 0u;
        clear_t[i] = z;
    }
    int c0, c1;
    pair_chunk(nslots, c0, c1);
    int pre = 0;
    for (int i = t; i < (int)blockIdx.x; i += kThreads) pre += b.SELCNT[i];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if (lane == 0) s_w[wave] = pre;
    __syncthreads();
    if (t == 0) {
        int x = 0;
        for (int w = 0; w < kThreads / 64; ++w) x += s_w[w];
        s_base = x;
        if (blockIdx.x == gridDim.x - 1) b.CTR[CTR_E] = E1 + x + b.SELCNT[blockIdx.x];
    }
    __syncthreads();
    int run = s_base;
    for (int tb = c0; tb < c1; tb += kThreads * kPairItems) {
        const int base = tb + t * kPairItems;
        int partner[kPairItems];
        uint32_t own = 0;
#pragma unroll
        for (int i = 0; i < kPairItems; ++i)
            if (base + i < c1 && hash_owner(b, g, base + i, nslots, partner[i])) own |= 1u << i;
        const int cnt = __popc(own);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        __syncthreads();
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
            if (own & (1u << i)) emit_pair(b, g, V0, nslots, base + i, partner[i], (size_t)E1 + pos++);
        run += total;
    }
}

void launch_hash_pair(const Bufs &b, const StepGeom &g, int V0, int E1, int nslots, HEntry *clear_t,
                      uint32_t clear_n, hipStream_t st) {
    hipLaunchKernelGGL(k_hpair_count, dim3(kSelBlocks), dim3(kThreads), 0, st, b, g, nslots);
    hipLaunchKernelGGL(k_hpair_emit, dim3(kSelBlocks), dim3(kThreads), 0, st, b, g, V0, E1, nslots, clear_t,
                       clear_n);
}

}  // namespace pcx
