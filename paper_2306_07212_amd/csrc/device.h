// Device functions shared by the per-step kernels (kernels.hip) and the
// persistent batched kernel (batch.hip) of libpcx.so. Both paths run the same
// arithmetic in the same order, so a network gives bit-identical results on
// either.
#pragma once
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

// spread the 16 low bits of x to the even bit positions of a 32-bit word
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// 2-bit codes of 32 entries from their positive / negative masks (entry i at
// bits 2i, 2i+1: 01 positive, 10 negative, 00 zero)
__device__ __forceinline__ uint64_t codes_of(uint32_t pos, uint32_t neg) {
    const uint32_t lo = spread16(pos) | (spread16(neg) << 1);
    const uint32_t hi = spread16(pos >> 16) | (spread16(neg >> 16) << 1);
    return ((uint64_t)hi << 32) | lo;
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

// bits 0..3: which bytes of v equal the byte t4 repeats (exact: no borrow
// between bytes, since the top bit of each byte is handled apart)
__device__ __forceinline__ uint32_t eq_bytes4(uint32_t v, uint32_t t4) {
    const uint32_t x = v ^ t4;
    const uint32_t nz = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // top bit set in every nonzero byte
    const uint32_t z = ~nz & 0x80808080u;
    return ((z >> 7) * 0x00204081u) >> 21 & 0xFu;  // gather the four top bits
}

__device__ __forceinline__ void load32b(const uint8_t *__restrict__ nx, int base, uint4 &a, uint4 &c) {
    a = *reinterpret_cast<const uint4 *>(nx + base);
    c = *reinterpret_cast<const uint4 *>(nx + base + 16);
}

// bit i: edge base + i has first crossing `target` (kScanItems one-byte
// entries): from the words load32b fetched for a whole group, else (the
// chunk's last, partial group) from the bytes one by one
__device__ __forceinline__ uint32_t match32b_raw(const uint8_t *__restrict__ nx, int base, int E, uint8_t target,
                                                 uint4 a, uint4 c) {
    uint32_t hit = 0;
    if (base + kScanItems <= E) {
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
        const uint32_t t4 = 0x01010101u * target;
#pragma unroll
        for (int i = 0; i < 8; ++i) hit |= eq_bytes4(w[i], t4) << (4 * i);
    } else {
        for (int i = 0; i < kScanItems; ++i)
            if (base + i < E && nx[base + i] == target) hit |= 1u << i;
    }
    return hit;
}

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

// ----------------------------------------------- 2-face hash table
//
// Open addressing with linear probing, one 64-bit word per splitting 2-face
// (layout in internal.h). The first splitting edge to reach a face claims an
// empty word with a CAS that publishes its key and its slot together; the
// second finds the key in the value its own CAS returns, takes the partner's
// slot from it and records the pair at once: each of the two slots gets a
// record naming the other, tagged with the step. The pairing then checks that
// every valid slot's record is fresh and mutual. A face met once leaves its
// slot without a fresh record; a word reached three or more times leaves a
// record its partner does not return (a slot names one partner only) -- and
// two different faces whose keys are equal (the hash bits beside the slot
// field, at most 39) and whose probe chains meet put four arrivals on one
// word, so for a generic input no wrong pair gets through. Each of these sends
// the step to the exact pass. With verify_pairs the emission also compares the
// two perturbed sign rows, which catches two faces each met once (a non-generic
// input) with equal keys.

// pairing failures: recorded with their step (the exact pass redoes that step)
__device__ __forceinline__ void raise_pair_flag(int *ctr, int f, int step) {
    atomicOr(&ctr[CTR_PFLAGS], f);
    atomicMin(&ctr[CTR_PFAIL], step);
}

// the pair (u, p) of one 2-face: each slot's record names the other
__device__ __forceinline__ void record_pair(const Bufs &b, const StepGeom &g, uint32_t u, uint32_t p, int nslots) {
    if (p >= (uint32_t)nslots || p == u) {
        raise_flag(b.CTR, FLAG_BOUNDS);
        return;
    }
    const uint64_t tag = (uint64_t)(uint32_t)(g.step + 1) << 32;
    b.PART[u] = tag | (uint64_t)(p + 1);
    b.PART[p] = tag | (uint64_t)(u + 1);
}

__device__ __forceinline__ void hash_insert(const Bufs &b, const StepGeom &g, uint64_t H, uint32_t u, int nslots) {
    const int sb = g.sbits;  // (the key: the hash bits above 25 that fit beside the slot)
    const unsigned long long key = (H >> 25) & ((1ull << (64 - sb)) - 1ull);
    const unsigned long long mine = (key << sb) | (unsigned long long)(u + 1);
    uint32_t h = (uint32_t)H & g.hmask;
    for (uint32_t probe = 0; probe <= g.hmask; ++probe) {
        const unsigned long long old = atomicCAS(&g.HT[h], 0ull, mine);
        if (old == 0ull) return;  // first arrival: the second records the pair
        if ((old >> sb) == key) {
            record_pair(b, g, u, (uint32_t)(old & ((1ull << sb) - 1ull)) - 1u, nslots);
            return;
        }
        h = (h + 1) & g.hmask;
    }
    raise_flag(b.CTR, FLAG_BOUNDS);  // table full: cannot happen at load factor <= 1/2
}

// partner of valid key slot u from its record (-1: no fresh record)
__device__ __forceinline__ int slot_partner(const Bufs &b, const StepGeom &g, int u, int nslots) {
    const uint64_t r = b.PART[u];
    const uint32_t p1 = (uint32_t)r;
    if ((uint32_t)(r >> 32) != (uint32_t)(g.step + 1) || p1 == 0u || p1 - 1u >= (uint32_t)nslots) return -1;
    return (int)(p1 - 1u);
}

// Key slot u at the pairing's check: true if u owns a pair (the smaller slot
// of a mutual pair of fresh records). A valid slot without a fresh mutual
// record is a pairing failure of the step.
__device__ __forceinline__ bool slot_owner(const Bufs &b, const StepGeom &g, int u, int nslots, int &partner) {
    if (b.PINFO[u] == kNoInfo) return false;
    const int p = slot_partner(b, g, u, nslots);
    if (p < 0 || slot_partner(b, g, p, nslots) != u) {
        raise_pair_flag(b.CTR, FLAG_RUN, g.step);
        return false;
    }
    partner = p;
    return u < p;
}

// Appends the intersecting edge between the new vertices of key slots sa, sb
// (the same 2-face). check_rows: first verify that their perturbed sign rows
// agree on every entry before the current neuron; check_hash: also compare the
// stored 64-bit hashes (the hash table already matched them exactly). preA:
// words wn .. wn+3 of sa's row, when the caller has loaded them already.
__device__ __forceinline__ void emit_pair(const Bufs &b, const StepGeom &g, int V0, int nslots, int sa, int sb,
                                          size_t out, bool check_hash = true, bool check_rows = true,
                                          const uint64_t *preA = nullptr) {
    if ((unsigned)sa >= (unsigned)nslots || (unsigned)sb >= (unsigned)nslots) {
        raise_flag(b.CTR, FLAG_BOUNDS);
        return;
    }
    const int xa = V0 + sa / g.P, xb = V0 + sb / g.P;
    const uint64_t *Ra = b.SG + (size_t)xa * g.Wd, *Rb = b.SG + (size_t)xb * g.Wd;
    uint64_t diff = check_hash ? (b.FULL[sa] ^ b.FULL[sb]) : 0ull;
    if (check_rows) {
        const uint32_t pa = b.PINFO[sa], pb = b.PINFO[sb];
        const int wa = (int)(pa >> 8), wb = (int)(pb >> 8);
        const uint64_t ca = ((pa & 1u) ? 2ull : 1ull) << ((pa >> 1) & 63u);
        const uint64_t cb = ((pb & 1u) ? 2ull : 1ull) << ((pb >> 1) & 63u);
        // no early exit: the row loads of all words are independent and pipeline
#pragma unroll 8
        for (int w = 0; w <= g.wn; ++w) {
            const uint64_t lt = lt_mask(w, g.wn, g.bn);
            const uint64_t fa = (Ra[w] & lt) | (w == wa ? ca : 0ull);
            const uint64_t fb = (Rb[w] & lt) | (w == wb ? cb : 0ull);
            diff |= fa ^ fb;
        }
    }
    if (diff) raise_pair_flag(b.CTR, FLAG_VERIFY, g.step);
    // first crossing after the neuron: four words per round, loaded together
    int col = kNoCol;
    for (int w0 = g.wn; w0 < g.lw1 && col == kNoCol; w0 += 4) {
        uint64_t x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int w = w0 + i;
            const uint64_t a = preA && w0 == g.wn ? preA[i] : (w < g.lw1 ? Ra[w] : 0ull);
            x[i] = w < g.lw1 ? (a ^ Rb[w]) & gt_mask(w, g.wn, g.bn, g.lw1) : 0ull;
        }
#pragma unroll
        for (int i = 3; i >= 0; --i)
            if (x[i]) col = first_col(x[i], w0 + i, g.lw0);
    }
    b.EDG[out] = make_int2(xa, xb);
    if (g.nx8)
        b.NX8[out] = col == kNoCol ? 0 : (uint8_t)col;  // col > j >= 0
    else
        b.NXT[out] = col == kNoCol ? kNone : (uint16_t)col;
}

// One tile of kGemmRows vertex rows x all N <= 256 outputs (see k_gemm). The
// whole workgroup calls it; hs / ws are its LDS staging arrays. Products are
// accumulated with explicit FMAs in k order, so every caller rounds alike.
__device__ __forceinline__ void gemm_tile(const Bufs &b, int ZS, const double *in, int in_stride, int relu, int V,
                                          int K, int N, const double *__restrict__ Wt,
                                          const double *__restrict__ bias, int Wd, int lw0, int v0,
                                          double (*hs)[kGemmK + 1], double (*ws)[kMaxWidth]) {
    const int t = threadIdx.x;
    const int tc = t & 31, tv = t >> 5;
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
                for (int c = 0; c < 8; ++c) acc[i][c] = fma(h[i], w[c], acc[i][c]);
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
            if (tc == 0 && v < V && c < nwords) {
                const uint64_t cw = codes_of((uint32_t)(pb >> (32 * half)), (uint32_t)(nb >> (32 * half)));
                b.SG[(size_t)v * Wd + lw0 + c] = cw;
                if (b.LW) b.LW[(size_t)v * 8 + c] = cw;
            }
        }
    }
    if (zero) raise_flag(b.CTR, FLAG_ZERO_SIGN);
}

// LDS staging of one evaluation tile (gemm_tile)
struct GemmLds {
    double hs[kGemmRows][kGemmK + 1];
    double ws[kGemmK][kMaxWidth];
};

// -------------------------------------------- steps 4-5a: split and keys
// The work of one splitting edge s for a group of G lanes (G = 16, 32 or 64;
// lane = 0..G-1; half = which G-lane part of the wave the group is).
// stores of a split's new vertex (its pre-activation row, sign row and
// coordinates): NT streams them past the caches. The per-step split takes it
// for layers wider than 128 neurons, whose rows are read back only by the next
// layer's evaluation, a launch after the whole layer has been split (3.5% off
// the split on 256-wide layers); narrower layers' rows can still sit in the
// caches by then (streaming them measured 1% slower on 64-wide layers), and
// the batched kernel evaluates its rows soon after, in the same launch.
template <bool NT, typename T>
__device__ __forceinline__ void vstore(T *p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// split_core: the split of edge e = ab (already read and bounds-checked)
template <int G, int NC, bool NT>
__device__ __forceinline__ void split_core(const Bufs &b, const StepGeom &g, int V0, int E0, int s, int e, int2 ab,
                                           int lane, int half, int nslots) {
    const int D = g.D, Wd = g.Wd, ZS = g.ZS;
    // every 2-face key of the split is built by a lane of the group (callers
    // choose G >= 2(D - 1)); anything else is refused as an internal error
    if (g.P > G) {
        if (lane == 0) raise_flag(b.CTR, FLAG_BOUNDS);
        return;
    }
    // the per-column predicates below (c < N, c vs j, c >= zlo) are cheap to
    // recompute; an empty asm makes their bounds opaque per split so that they
    // are not hoisted out of the caller's loop into dozens of live lane masks
    // (uniform values: readfirstlane keeps them in scalar registers in every caller)
    int j = __builtin_amdgcn_readfirstlane(g.j), N = __builtin_amdgcn_readfirstlane(g.Nl),
        zlo = __builtin_amdgcn_readfirstlane(g.zlo);
    asm volatile("" : "+s"(j), "+s"(N), "+s"(zlo));
    const int nw = g.lw1 - g.lw0;
    const double *Za = b.Z + (size_t)ab.x * ZS, *Zb = b.Z + (size_t)ab.y * ZS;
    const uint64_t *Ra = b.SG + (size_t)ab.x * Wd, *Rb = b.SG + (size_t)ab.y * Wd;
    // ---- loads
    const double za = Za[j], zb = Zb[j];
    double A[NC], B[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int c = k * G + lane;
        const bool live = c < N && c >= zlo;
        A[k] = live ? Za[c] : 0.0;
        B[k] = live ? Zb[c] : 0.0;
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
    double *Zo = b.Z + x0 * ZS;
    // the chunk ballots of x0's pre-activations (which columns are +, which -),
    // parked in LDS for the lane that owns the corresponding sign word below.
    // Lanes outside [zlo, N) hold A = B = 0, so their z is exactly 0 and they
    // add no bit to either ballot. Column j is interpolated like the others:
    // every use of its ballot bits below is masked to the entries after j, and
    // its stored value is overwritten by an exact 0.
    __shared__ uint64_t s_bal[kThreads / 64][kMaxWidth / 32][2];
    static_assert(G == 64 ? NC <= kMaxWidth / 64 : NC <= kMaxWidth / 32, "chunk ballots exceed the LDS slots");
    static_assert(G != 16 || NC % 2 == 0, "16-lane groups take whole 32-column words");
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const int c = k * G + lane;
        const double p = apos ? A[k] : B[k], q = apos ? B[k] : A[k];
        const double z = p + tt * (q - p);
        if (c < N && c >= zlo) vstore<NT>(&Zo[c], z);
        const uint64_t pbk = __ballot(z > 0.0), nbk = __ballot(z < 0.0);
        if ((threadIdx.x & 63) == 0) {
            s_bal[wv][k][0] = pbk;
            s_bal[wv][k][1] = nbk;
        }
    }
    if (lane == (j & (G - 1)) && j >= zlo) Zo[j] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double xp = apos ? xa : xb, xq = apos ? xb : xa;
    const double x0c = xp + tt * (xq - xp);
    // ---- sign row of x0, hash of the edge's sign-vector, zeros, next crossings.
    // The loop runs uniformly over the group; lane c of iteration it owns word
    // it*G + c. Zero entries are few (D-1), so their counts travel by ballot:
    // every zero of the edge's sign-vector gives the 2-faces of step 5 (one for
    // a box entry, two for a neuron, in word, bit, sign order), and key r is
    // built by lane r, which here learns the word that holds it.
    const uint64_t gmask = G == 64 ? ~0ull : (1ull << G) - 1ull;
    const int gshift = G * half;
    uint64_t hsum = 0, rx0 = 0;
    uint64_t kf = 0, kz = 0;  // for key `lane`: the edge's sign word and its zeros there
    int kw = -1, kli = 0;     //                 that word's index, the key's rank inside the word
    int nz = 0, ktot = 0, da = kNoCol, db = kNoCol;
    for (int it = 0; it * G < Wd; ++it) {
        const int w = it * G + lane;
        const bool live = w < Wd;
        uint64_t wa = 0, wb = 0;
        if (live) {
            wa = it == 0 ? wa0 : Ra[w];
            wb = it == 0 ? wb0 : Rb[w];
        }
        const uint64_t lt = live ? lt_mask(w, g.wn, g.bn) : 0ull;
        const uint64_t gt = live ? gt_mask(w, g.wn, g.bn, g.lw1) : 0ull;
        const uint64_t f = (wa | wb) & lt;
        if (f & (f >> 1) & 0x5555555555555555ull) bad |= FLAG_CONFLICT;
        const uint64_t vw = live ? b.VALID[w] : 0ull;
        const int u = w - g.lw0;
        uint64_t cw = 0;
        if (live && u >= 0 && u < nw) {
            if (G == 16) {
                // word u = chunks 2u and 2u+1: this group's 16 bits of each ballot
                const int sh = 16 * half;
                const uint32_t pw = (uint32_t)((s_bal[wv][2 * u][0] >> sh) & 0xFFFFu) |
                                    ((uint32_t)((s_bal[wv][2 * u + 1][0] >> sh) & 0xFFFFu) << 16);
                const uint32_t nw2 = (uint32_t)((s_bal[wv][2 * u][1] >> sh) & 0xFFFFu) |
                                     ((uint32_t)((s_bal[wv][2 * u + 1][1] >> sh) & 0xFFFFu) << 16);
                cw = codes_of(pw, nw2);
            } else {
                // word u = chunk u / (G/32); inside the chunk's 64-bit ballot, this group's 32 columns
                const int ku = G == 64 ? (u >> 1) : u, sh = G == 64 ? 32 * (u & 1) : 32 * half;
                cw = codes_of((uint32_t)(s_bal[wv][ku][0] >> sh), (uint32_t)(s_bal[wv][ku][1] >> sh));
            }
            // an exact zero at a later neuron of the layer: x0 lies on two hyperplanes
            if (~(cw | (cw >> 1)) & vw & gt) bad |= FLAG_ZERO_SIGN;
        }
        const uint64_t rx = f | (cw & gt);
        if (it == 0) rx0 = rx;
        else if (live) vstore<NT>(&b.SG[x0 * Wd + w], rx);
        if (live && w <= g.wn) hsum += word_hash(w, f);
        const uint64_t zm = ~(f | (f >> 1)) & vw & lt;
        const int zc = __popcll(zm);
        uint64_t has = (__ballot(zc != 0) >> gshift) & gmask;
        int srcl = lane;
        bool mine = false;
        while (has) {
            const int sl = __builtin_ctzll(has);
            has &= has - 1;
            const int c = __shfl(zc, sl, G);
            const int keys = (it == 0 && sl == 0) ? c : 2 * c;  // box entries all live in word 0
            if (lane >= ktot && lane < ktot + keys) {
                srcl = sl;
                kli = lane - ktot;
                mine = true;
            }
            nz += c;
            ktot += keys;
        }
        const uint64_t fz = __shfl(f, srcl, G), zz = __shfl(zm, srcl, G);
        if (mine) {
            kf = fz;
            kz = zz;
            kw = it * G + srcl;
        }
        // the first crossing after j: columns grow with the word, so it sits in the first lane that has one
        const int cda = first_col((wa ^ rx) & gt, w, g.lw0), cdb = first_col((rx ^ wb) & gt, w, g.lw0);
        if (da == kNoCol) {
            const uint64_t m = (__ballot(cda != kNoCol) >> gshift) & gmask;
            if (m) da = __shfl(cda, __builtin_ctzll(m), G);
        }
        if (db == kNoCol) {
            const uint64_t m = (__ballot(cdb != kNoCol) >> gshift) & gmask;
            if (m) db = __shfl(cdb, __builtin_ctzll(m), G);
        }
    }
    hsum = group_sum<G>(hsum);
    if ((__ballot(bad != 0) >> gshift) & gmask) bad = group_or<G>(bad);
    // ---- stores
    {
        // (the lane's store addresses are rebuilt per split rather than kept
        // live across the split loop, where they would take more registers)
        int xl = lane;
        asm volatile("" : "+v"(xl));
        if (xl < D) vstore<NT>(&b.X[x0 * D + xl], x0c);
        if (xl < Wd) vstore<NT>(&b.SG[x0 * Wd + xl], rx0);
    }
    if (lane == 0) {
        if (nz != D - 1 || ktot > g.P) bad |= FLAG_ZERO_COUNT;
        if (bad) raise_flag(b.CTR, bad);
        b.EDG[e] = make_int2(ab.x, (int)x0);
        b.EDG[E0 + s] = make_int2((int)x0, ab.y);
        if (g.nx8) {  // crossings after j >= 0: 1..255
            b.NX8[e] = da == kNoCol ? 0 : (uint8_t)da;
            b.NX8[E0 + s] = db == kNoCol ? 0 : (uint8_t)db;
        } else {
            b.NXT[e] = da == kNoCol ? kNone : (uint16_t)da;
            b.NXT[E0 + s] = db == kNoCol ? kNone : (uint16_t)db;
        }
        if (b.PQ) b.PQ[x0] = apos ? ab : make_int2(ab.y, ab.x);
    }
    if (g.P > 0) {
        const size_t sbase = (size_t)s * g.P;
        if (lane < ktot && lane < g.P && kw >= 0) {
            // the key's zero: bit rank kli (box word) or kli/2 with sign kli%2 (neuron words)
            const int minus = kw == 0 ? 0 : (kli & 1);
            uint64_t z = kz;
            for (int k = kw == 0 ? kli : (kli >> 1); k > 0; --k) z &= z - 1;
            const int bit = __builtin_ctzll(z);
            // (hkeep drops hash bits only to test the exact pass: collisions on purpose)
            const uint64_t myh = (hsum - word_hash(kw, kf) + word_hash(kw, kf | ((minus ? 2ull : 1ull) << bit))) & g.hkeep;
            const size_t slot = sbase + lane;
            b.PINFO[slot] = ((uint32_t)kw << 8) | ((uint32_t)bit << 1) | (uint32_t)minus;
            if (g.pair_mode == PAIR_SORT) {
                // 24 bits for three 8-bit radix passes; all-ones is the sentinel's
                const uint32_t k24 = (uint32_t)(myh >> 40);
                b.K32a[slot] = k24 < 0xFFFFFFu ? k24 : 0xFFFFFEu;
                b.FULL[slot] = myh;
            } else if (g.hmask != 0u) {  // (0: more key slots than the table names; the exact pass pairs the step)
                hash_insert(b, g, myh, (uint32_t)slot, nslots);
            }
        }
        for (int rr = ktot + lane; rr < g.P; rr += G) {
            b.PINFO[sbase + rr] = kNoInfo;
            if (g.pair_mode == PAIR_SORT) b.K32a[sbase + rr] = kSentinel;
        }
    }
}

// checks of a split-list entry and its edge (out of range: flag, no work)
__device__ __forceinline__ bool split_entry_ok(const Bufs &b, int e, int E0) { return (unsigned)e < (unsigned)E0; }
__device__ __forceinline__ bool split_edge_ok(int2 ab, int V0) {
    return (unsigned)ab.x < (unsigned)V0 && (unsigned)ab.y < (unsigned)V0;
}

}  // namespace pcx
