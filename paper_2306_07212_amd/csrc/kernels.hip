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
// Ordered stream compaction of {e : NXT[e] == target} with a wave ballot /
// prefix inside each tile and decoupled look-back between tiles (tiles are
// taken from a ticket counter, so every predecessor of a waiting tile is
// resident and will publish). Status words carry an epoch so that they never
// need clearing: epoch << 34 | flag << 32 | count, flag 1 = tile aggregate,
// 2 = inclusive prefix.
__device__ __forceinline__ uint64_t sel_pack(uint32_t epoch, uint32_t flag, uint32_t v) {
    return ((uint64_t)epoch << 34) | ((uint64_t)flag << 32) | v;
}

__global__ __launch_bounds__(kThreads) void k_select(Bufs b, uint16_t target, uint32_t epoch) {
    __shared__ int s_tile, s_prefix;
    __shared__ int s_wsum[kThreads / 64];
    const int E = b.CTR[CTR_E];
    const int ntiles = (E + kSelTile - 1) / kSelTile;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int *tickets = b.TICKETS + epoch;
    if (blockIdx.x == 0 && t == 0) b.CTR[CTR_KVALID] = 0;  // counted by the split that follows
    if (ntiles == 0) {
        if (blockIdx.x == 0 && t == 0) b.CTR[CTR_S] = 0;
        return;
    }
    for (;;) {
        if (t == 0) s_tile = atomicAdd(tickets, 1);
        __syncthreads();
        const int tile = s_tile;
        if (tile >= ntiles) break;
        const int base = tile * kSelTile + t * kSelItems;
        uint32_t hit = 0;  // bit i set: edge base+i splits now
#pragma unroll
        for (int i = 0; i < kSelItems; ++i) {
            const int e = base + i;
            if (e < E && b.NXT[e] == target) hit |= 1u << i;
        }
        const int cnt = __popc(hit);
        // wave inclusive scan
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        int wave_off = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            const int ws = s_wsum[w];
            if (w < wave) wave_off += ws;
            total += ws;
        }
        if (t == 0) {
            uint64_t *st = b.SELST;
            int prefix = 0;
            if (tile == 0) {
                __hip_atomic_store(&st[0], sel_pack(epoch, 2, (uint32_t)total), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            } else {
                __hip_atomic_store(&st[tile], sel_pack(epoch, 1, (uint32_t)total), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
                int p = tile - 1;
                for (;;) {
                    const uint64_t s = __hip_atomic_load(&st[p], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t ep = (uint32_t)(s >> 34), fl = (uint32_t)(s >> 32) & 3u;
                    if (ep != epoch || fl == 0) continue;  // predecessor not published yet
                    prefix += (int)(uint32_t)s;
                    if (fl == 2) break;
                    --p;
                }
                __hip_atomic_store(&st[tile], sel_pack(epoch, 2, (uint32_t)(prefix + total)), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            s_prefix = prefix;
            if (tile == ntiles - 1) b.CTR[CTR_S] = prefix + total;
        }
        __syncthreads();
        int pos = s_prefix + wave_off + incl - cnt;
        while (hit) {
            const int i = __builtin_ctz(hit);
            hit &= hit - 1;
            b.SPL[pos++] = base + i;
        }
        __syncthreads();  // s_tile / s_wsum reuse
    }
}

void launch_select(const Bufs &b, uint16_t target, uint32_t epoch, int Emax, hipStream_t st) {
    int tiles = (Emax + kSelTile - 1) / kSelTile;
    int grid = tiles < 1 ? 1 : (tiles > 2048 ? 2048 : tiles);
    hipLaunchKernelGGL(k_select, dim3(grid), dim3(kThreads), 0, st, b, target, epoch);
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
template <int G>
__global__ __launch_bounds__(kThreads) void k_split(Bufs b, StepGeom g, int V0, int E0, int S) {
    extern __shared__ uint64_t lds_codes[];  // [groups][nw]
    constexpr int groups = kThreads / G;
    const int nw = g.lw1 - g.lw0;
    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int half = (threadIdx.x & 63) / G;  // group within the wave (G = 32: 0 or 1)
    uint64_t *codes = lds_codes + (size_t)grp * nw;
    const int D = g.D, Wd = g.Wd, ZS = g.ZS, j = g.j;
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
        const double za = b.Z[(size_t)ab.x * ZS + j], zb = b.Z[(size_t)ab.y * ZS + j];
        const bool apos = za > 0.0;
        const int p = apos ? ab.x : ab.y, q = apos ? ab.y : ab.x;
        const double zp = apos ? za : zb, zq = apos ? zb : za;
        const double tt = zp / (zp - zq);
        const size_t x0 = (size_t)V0 + s;
        for (int d = lane; d < D; d += G) {
            const double xp = b.X[(size_t)p * D + d], xq = b.X[(size_t)q * D + d];
            b.X[x0 * D + d] = xp + tt * (xq - xp);
        }
        int bad = 0;
        const double *Zp = b.Z + (size_t)p * ZS, *Zq = b.Z + (size_t)q * ZS;
        double *Zx = b.Z + x0 * ZS;
        for (int c0 = 0; c0 < g.Nl; c0 += G) {
            const int c = c0 + lane;
            const bool in = c < g.Nl;
            double z = 0.0;
            if (in) {
                const double a = Zp[c], bq = Zq[c];
                z = (c == j) ? 0.0 : a + tt * (bq - a);
                Zx[c] = z;
                if (c > j && z == 0.0) bad |= FLAG_ZERO_SIGN;
            }
            const uint64_t pb = __ballot(in && z > 0.0);
            const uint64_t nb = __ballot(in && z < 0.0);
            if (G == 64) {
                if (lane == 0) codes[c0 >> 5] = codes_of((uint32_t)pb, (uint32_t)nb);
                if (lane == 1 && (c0 >> 5) + 1 < nw) codes[(c0 >> 5) + 1] = codes_of((uint32_t)(pb >> 32), (uint32_t)(nb >> 32));
            } else {
                if (lane == 0) codes[c0 >> 5] = codes_of((uint32_t)(pb >> (32 * half)), (uint32_t)(nb >> (32 * half)));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // sign row of x0, hash of the edge's sign-vector, zeros, next crossings
        uint64_t hsum = 0;
        int nz = 0, nkeys = 0;
        int da = kNoCol, db = kNoCol;
        const uint64_t *Rp = b.SG + (size_t)p * Wd, *Rq = b.SG + (size_t)q * Wd;
        uint64_t *Rx = b.SG + x0 * Wd;
        for (int w = lane; w < Wd; w += G) {
            const uint64_t rp = Rp[w], rq = Rq[w];
            const uint64_t lt = lt_mask(w, g.wn, g.bn), gt = gt_mask(w, g.wn, g.bn, g.lw1);
            const uint64_t f = (rp | rq) & lt;
            if (f & (f >> 1) & 0x5555555555555555ull) bad |= FLAG_CONFLICT;
            const uint64_t cw = (w >= g.lw0 && w < g.lw1) ? codes[w - g.lw0] : 0ull;
            const uint64_t rx = f | (cw & gt);
            Rx[w] = rx;
            if (w <= g.wn) hsum += word_hash(w, f);
            const uint64_t zm = ~(f | (f >> 1)) & b.VALID[w] & lt;
            const int zc = __popcll(zm);
            nz += zc;
            nkeys += (w == 0) ? zc : 2 * zc;  // box entries all live in word 0
            const uint64_t ra = apos ? rp : rq, rb = apos ? rq : rp;
            da = min(da, first_col((ra ^ rx) & gt, w, g.lw0));
            db = min(db, first_col((rx ^ rb) & gt, w, g.lw0));
        }
        hsum = group_sum<G>(hsum);
        nz = group_sum<G>(nz);
        const int ktot = group_sum<G>(nkeys);
        da = group_min<G>(da);
        db = group_min<G>(db);
        bad = group_or<G>(bad);
        if (lane == 0) {
            if (nz != D - 1) bad |= FLAG_ZERO_COUNT;
            if (bad) raise_flag(b.CTR, bad);
            b.EDG[e] = make_int2(ab.x, (int)x0);
            b.EDG[E0 + s] = make_int2((int)x0, ab.y);
            b.NXT[e] = da == kNoCol ? kNone : (uint16_t)da;
            b.NXT[E0 + s] = db == kNoCol ? kNone : (uint16_t)db;
            if (ktot) atomicAdd(&b.CTR[CTR_KVALID], ktot);
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
            for (int w = lane; w < Wd && nkeys; w += G) {
                const uint64_t rp = Rp[w], rq = Rq[w];
                const uint64_t lt = lt_mask(w, g.wn, g.bn);
                const uint64_t f = (rp | rq) & lt;
                uint64_t zm = ~(f | (f >> 1)) & b.VALID[w] & lt;
                const uint64_t hw = word_hash(w, f);
                while (zm) {
                    const int bit = __builtin_ctzll(zm);
                    zm &= zm - 1;
                    for (int minus = 0; minus < (w == 0 ? 1 : 2); ++minus) {
                        const uint64_t f2 = f | ((minus ? 2ull : 1ull) << bit);
                        const uint64_t h = hsum - hw + word_hash(w, f2);
                        const size_t slot = sbase + r++;
                        if (r <= g.P) {
                            b.K32a[slot] = (uint32_t)(h >> 33);
                            b.FULL[slot] = h;
                            b.PINFO[slot] = ((uint32_t)w << 8) | ((uint32_t)bit << 1) | (uint32_t)minus;
                        }
                    }
                }
            }
            for (int rr = ktot + lane; rr < g.P; rr += G) b.K32a[sbase + rr] = kSentinel;
            if (ktot > g.P && lane == 0) raise_flag(b.CTR, FLAG_ZERO_COUNT);
        }
    }
}

void launch_split(const Bufs &b, const StepGeom &g, int V0, int E0, int S, hipStream_t st) {
    if (S <= 0) return;
    const int G = g.Nl > 32 ? 64 : 32;
    const int groups = kThreads / G;
    int grid = (S + groups - 1) / groups;
    grid = grid > 16384 ? 16384 : grid;
    const size_t lds = (size_t)groups * (g.lw1 - g.lw0) * sizeof(uint64_t);
    if (G == 64)
        hipLaunchKernelGGL(k_split<64>, dim3(grid), dim3(kThreads), lds, st, b, g, V0, E0, S);
    else
        hipLaunchKernelGGL(k_split<32>, dim3(grid), dim3(kThreads), lds, st, b, g, V0, E0, S);
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

__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *hist, int len) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int chunk = (len + 1023) / 1024;
    const int b0 = t * chunk, b1 = min(len, b0 + chunk);
    uint32_t s = 0;
    for (int i = b0; i < b1; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t y = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int i = b0; i < b1; ++i) {
        const uint32_t x = hist[i];
        hist[i] = run;
        run += x;
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
    if (blockIdx.x == 0 && threadIdx.x == 0) b.CTR[CTR_E] = E1 + b.CTR[CTR_KVALID] / 2;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += gridDim.x * blockDim.x) {
        const uint32_t k = KS[i];
        if (k == kSentinel) continue;
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

}  // namespace pcx
