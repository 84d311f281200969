// Higher cells of an extracted complex by repeated perturbation (Berzins 2023,
// Sec. 4.1): the parents of a k-cell are found by perturbing each zero of its
// sign-vector to + and to - (zeros of the domain's half-spaces, all in word 0,
// only to +), and every (k+1)-cell is a parent of some k-cell. Starting from
// the edges (an edge's sign-vector is the join of its vertices', Sec. 3.5) this
// gives the 2-faces, then the 3-cells, ..., up to the regions.
//
// A k-cell is named by one edge below it and the signs given to that edge's
// D-1 zeros (2 bits each, in entry order: 00 still zero, 01 +, 10 -), so a cell
// costs 8 bytes and its sign row is rebuilt from the edge's two vertex rows.
// Distinct cells are told apart by a 128-bit hash of the sign-vector (two
// independent 64-bit sums of per-word hashes); an open-addressing table keeps
// one representative per cell, and a cell met with equal first halves but
// different second halves raises FLAG_VERIFY.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "compact.h"
#include "device.h"
#include "host.h"
#include "internal.h"
#include "pcx.h"

namespace pcx {

namespace {

// second, independent per-word hash (murmur3 finaliser constants)
__device__ __forceinline__ uint64_t word_check(int w, uint64_t v) {
    uint64_t x = v ^ ((uint64_t)(w + 1) * 0xd1b54a32d192ed03ull);
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

struct CellTable {
    unsigned long long *key, *chk;
    int2 *org;  // (edge, codes) of the representative
    uint32_t mask;
};

__device__ __forceinline__ void cell_insert(const CellTable &T, uint64_t K, uint64_t C, int edge, uint32_t code,
                                            int *ctr) {
    uint32_t h = (uint32_t)K & T.mask;
    for (uint32_t probe = 0; probe <= T.mask; ++probe) {
        const unsigned long long prev = atomicCAS(&T.key[h], 0ull, (unsigned long long)K);
        if (prev == 0ull || prev == (unsigned long long)K) {
            if (prev == 0ull) T.org[h] = make_int2(edge, (int)code);
            const unsigned long long pc = atomicCAS(&T.chk[h], 0ull, (unsigned long long)C);
            if (pc != 0ull && pc != (unsigned long long)C) raise_flag(ctr, FLAG_VERIFY);
            return;
        }
        h = (h + 1) & T.mask;
    }
    raise_flag(ctr, FLAG_BOUNDS);  // full: cannot happen at load factor <= 1/2
}

// The sign row of cell (edge, code) in the lanes of one wave: word it*64+lane
// for it = 0.. (uniform loop). Calls visit(it, w, live, row_word, zeros_all,
// remaining_zeros, rank_of_first_zero) per iteration.
template <class F>
__device__ __forceinline__ void cell_row(const uint64_t *SG, const uint64_t *VALID, int Wd, int2 ab, uint32_t code,
                                         int lane, F visit) {
    int rank = 0;  // zeros of the edge before this iteration's words
    for (int it = 0; it * 64 < Wd; ++it) {
        const int w = it * 64 + lane;
        const bool live = w < Wd;
        uint64_t r = live ? (SG[(size_t)ab.x * Wd + w] | SG[(size_t)ab.y * Wd + w]) : 0ull;
        const uint64_t zm = live ? (~(r | (r >> 1)) & VALID[w]) : 0ull;
        const int zc = __popcll(zm);
        int mybase = 0;
        uint64_t has = __ballot(zc != 0);
        while (has) {
            const int sl = __builtin_ctzll(has);
            has &= has - 1;
            if (lane == sl) mybase = rank;
            rank += __shfl(zc, sl, 64);
        }
        uint64_t rem = 0, z = zm;
        for (int k = 0; z; ++k) {
            const int p = __builtin_ctzll(z);
            z &= z - 1;
            const uint32_t cc = (code >> (2 * (mybase + k))) & 3u;
            if (cc) r |= (uint64_t)cc << p;
            else rem |= 1ull << p;
        }
        visit(it, w, live, r, zm, rem, mybase);
    }
}

// One wave per k-cell: every parent (k+1)-cell goes into the table.
__global__ __launch_bounds__(kThreads) void k_cell_parents(const int2 *cells, int n, const int2 *EDG,
                                                          const uint64_t *SG, const uint64_t *VALID, int Wd, int V,
                                                          CellTable T, int *ctr) {
    const int lane = threadIdx.x & 63;
    const int waves = (gridDim.x * kThreads) >> 6;
    for (int c = (blockIdx.x * kThreads + threadIdx.x) >> 6; c < n; c += waves) {
        const int2 ec = cells ? cells[c] : make_int2(c, 0);
        const int2 ab = EDG[ec.x];
        if ((unsigned)ab.x >= (unsigned)V || (unsigned)ab.y >= (unsigned)V) {
            if (lane == 0) raise_flag(ctr, FLAG_BOUNDS);
            continue;
        }
        uint64_t hsum = 0, csum = 0;
        // candidate `lane`: its word, that word of the cell row, its remaining zeros, all zeros, zero rank base
        uint64_t kf = 0, kz = 0, ka = 0;
        int kw = -1, kli = 0, kbase = 0, ktot = 0;
        cell_row(SG, VALID, Wd, ab, (uint32_t)ec.y, lane,
                 [&](int it, int w, bool live, uint64_t r, uint64_t zm, uint64_t rem, int mybase) {
                     if (live) {
                         hsum += word_hash(w, r);
                         csum += word_check(w, r);
                     }
                     const int rc = __popcll(rem);
                     uint64_t has = __ballot(rc != 0);
                     int srcl = lane;
                     bool mine = false;
                     while (has) {
                         const int sl = __builtin_ctzll(has);
                         has &= has - 1;
                         const int c2 = __shfl(rc, sl, 64);
                         const int keys = (it == 0 && sl == 0) ? c2 : 2 * c2;  // domain zeros only to +
                         if (lane >= ktot && lane < ktot + keys) {
                             srcl = sl;
                             kli = lane - ktot;
                             mine = true;
                         }
                         ktot += keys;
                     }
                     const uint64_t f = __shfl(r, srcl, 64), rz = __shfl(rem, srcl, 64), az = __shfl(zm, srcl, 64);
                     const int b0 = __shfl(mybase, srcl, 64);
                     if (mine) {
                         kf = f;
                         kz = rz;
                         ka = az;
                         kbase = b0;
                         kw = it * 64 + srcl;
                     }
                 });
        for (int o = 32; o > 0; o >>= 1) {
            hsum += __shfl_xor(hsum, o, 64);
            csum += __shfl_xor(csum, o, 64);
        }
        if (lane < ktot && kw >= 0) {
            const uint64_t sg = (kw == 0 || (kli & 1) == 0) ? 1ull : 2ull;
            uint64_t z = kz;
            for (int k = kw == 0 ? kli : (kli >> 1); k > 0; --k) z &= z - 1;
            const int p = __builtin_ctzll(z);
            const int gi = kbase + __popcll(ka & ((1ull << p) - 1ull));  // rank among the edge's zeros
            const uint64_t fp = kf | (sg << p);
            const uint64_t K = (hsum - word_hash(kw, kf) + word_hash(kw, fp)) | (1ull << 63);
            const uint64_t C = (csum - word_check(kw, kf) + word_check(kw, fp)) | 1ull;
            cell_insert(T, K, C, ec.x, (uint32_t)ec.y | ((uint32_t)sg << (2 * gi)), ctr);
        }
    }
}

struct Occupied {
    const unsigned long long *key;
    __device__ bool operator()(int h) const { return key[h] != 0ull; }
};
struct TakeOrigin {
    const unsigned long long *key;
    const int2 *org;
    int2 *out;
    unsigned long long *out_key;
    __device__ void operator()(int h, int pos) const {
        out[pos] = org[h];
        if (out_key) out_key[pos] = key[h];
    }
};

// sign rows of the given cells (every zero of their edge coded)
__global__ __launch_bounds__(kThreads) void k_cell_rows(const int2 *cells, int n, const int2 *EDG, const uint64_t *SG,
                                                       const uint64_t *VALID, int Wd, uint64_t *out) {
    const int lane = threadIdx.x & 63;
    const int waves = (gridDim.x * kThreads) >> 6;
    for (int c = (blockIdx.x * kThreads + threadIdx.x) >> 6; c < n; c += waves) {
        const int2 ec = cells[c];
        const int2 ab = EDG[ec.x];
        cell_row(SG, VALID, Wd, ab, (uint32_t)ec.y, lane,
                 [&](int, int w, bool live, uint64_t r, uint64_t, uint64_t, int) {
                     if (live) out[(size_t)c * Wd + w] = r;
                 });
    }
}

int grid_for(int64_t waves) { return (int)std::max<int64_t>(1, std::min<int64_t>(65536, (waves + 3) / 4)); }

// Runs the levels; counts[k] = number of k-cells, k = 0..D. With regions != null
// the D-cells' (edge, codes) and keys are left in *regions / *rkeys (device,
// owned by the arena).
int cells_run(const pcx_complex *cx, hipStream_t st, std::vector<int64_t> &counts, Arena &ar, int2 **regions,
              unsigned long long **rkeys, int64_t *nreg) {
    const int D = cx->D, Wd = cx->Wd;
    if (cx->pruned) return fail(PCX_ERR_INVALID, "cells need the whole complex: this one was pruned");
    counts.assign(D + 1, 0);
    counts[0] = cx->V;
    counts[1] = cx->E;
    void *p;
    int rc;
    if ((rc = ar.alloc(&p, CTR_COUNT * sizeof(int)))) return rc;
    int *ctr = (int *)p;
    HIPCHK(hipMemsetAsync(ctr, 0, CTR_COUNT * sizeof(int), st));
    if ((rc = ar.alloc(&p, Wd * sizeof(uint64_t)))) return rc;
    uint64_t *valid = (uint64_t *)p;
    HIPCHK(hipMemcpyAsync(valid, cx->valid.data(), Wd * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    if ((rc = ar.alloc(&p, kChunks * sizeof(int)))) return rc;
    int *cnt = (int *)p;
    int hctr[CTR_COUNT];
    int2 *level = nullptr;  // null: the edges themselves
    int64_t n = cx->E;
    unsigned long long *lkeys = nullptr;
    for (int k = 1; k < D && n > 0; ++k) {
        const int64_t cand = n * 2 * (D - k);
        size_t tsz = 256;
        while ((double)tsz < 2.0 * (double)cand / (double)(k + 2)) tsz <<= 1;
        if (tsz > ((size_t)1 << 30)) return fail(PCX_ERR_CAPACITY, "too many cells for one table (more than 2^29)");
        CellTable T;
        if ((rc = ar.alloc(&p, tsz * sizeof(unsigned long long)))) return rc;
        T.key = (unsigned long long *)p;
        if ((rc = ar.alloc(&p, tsz * sizeof(unsigned long long)))) return rc;
        T.chk = (unsigned long long *)p;
        if ((rc = ar.alloc(&p, tsz * sizeof(int2)))) return rc;
        T.org = (int2 *)p;
        T.mask = (uint32_t)(tsz - 1);
        HIPCHK(hipMemsetAsync(T.key, 0, tsz * sizeof(unsigned long long), st));
        HIPCHK(hipMemsetAsync(T.chk, 0, tsz * sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_cell_parents, dim3(grid_for(n)), dim3(kThreads), 0, st, level, (int)n, cx->EDG, cx->SG,
                           valid, Wd, (int)cx->V, T, ctr);
        HIPCHK(hipGetLastError());
        // the (k+1)-cells, in table order
        hipLaunchKernelGGL(k_ccount<Occupied>, dim3(kChunks), dim3(kThreads), 0, st, Occupied{T.key}, (int)tsz, cnt);
        HIPCHK(hipMemcpyAsync(hctr, ctr, sizeof hctr, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hctr[CTR_FLAGS] & FLAG_BOUNDS) return fail(PCX_ERR_DEVICE, "internal error: cell table overflow or index out of range");
        if (hctr[CTR_FLAGS] & FLAG_VERIFY) return fail(PCX_ERR_DEVICE, "two cells share a 64-bit hash (retry is not possible)");
        std::vector<int> hc(kChunks);
        HIPCHK(hipMemcpyAsync(hc.data(), cnt, kChunks * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const int64_t nn = std::accumulate(hc.begin(), hc.end(), (int64_t)0);
        counts[k + 1] = nn;
        int2 *next = nullptr;
        unsigned long long *nkeys = nullptr;
        if (nn > 0) {
            if ((rc = ar.alloc(&p, nn * sizeof(int2)))) return rc;
            next = (int2 *)p;
            if (k + 1 == D && regions) {
                if ((rc = ar.alloc(&p, nn * sizeof(unsigned long long)))) return rc;
                nkeys = (unsigned long long *)p;
            }
            hipLaunchKernelGGL((k_cscatter<Occupied, TakeOrigin>), dim3(kChunks), dim3(kThreads), 0, st,
                               Occupied{T.key}, TakeOrigin{T.key, T.org, next, nkeys}, (int)tsz, (const int *)cnt,
                               ctr + CTR_V);
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(st));
        ar.release(T.key);
        ar.release(T.chk);
        ar.release(T.org);
        if (level) ar.release(level);
        if (lkeys) ar.release(lkeys);
        level = next;
        lkeys = nkeys;
        n = nn;
    }
    if (regions) {
        *regions = level;
        *rkeys = lkeys;
        *nreg = D == 1 ? cx->E : n;
    }
    return PCX_OK;
}

}  // namespace
}  // namespace pcx

using namespace pcx;

extern "C" {

int pcx_cell_counts(const pcx_complex *cx, int64_t *counts, void *stream) {
    if (!cx || !counts) return fail(PCX_ERR_INVALID, "NULL argument");
    Arena ar;
    std::vector<int64_t> c;
    int rc = cells_run(cx, (hipStream_t)stream, c, ar, nullptr, nullptr, nullptr);
    if (rc) return rc;
    std::copy(c.begin(), c.end(), counts);
    return PCX_OK;
}

int pcx_regions(const pcx_complex *cx, uint64_t *rows, int64_t *n, void *stream) {
    if (!cx || !n) return fail(PCX_ERR_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const int D = cx->D, Wd = cx->Wd;
    Arena ar;
    std::vector<int64_t> c;
    int2 *reg = nullptr;
    unsigned long long *keys = nullptr;
    int64_t nr = 0;
    int rc = cells_run(cx, st, c, ar, &reg, &keys, &nr);
    if (rc) return rc;
    *n = nr;
    if (!rows || nr == 0) return PCX_OK;
    void *p;
    if ((rc = ar.alloc(&p, (size_t)nr * Wd * sizeof(uint64_t)))) return rc;
    uint64_t *drows = (uint64_t *)p;
    if ((rc = ar.alloc(&p, Wd * sizeof(uint64_t)))) return rc;
    uint64_t *valid = (uint64_t *)p;
    HIPCHK(hipMemcpyAsync(valid, cx->valid.data(), Wd * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    if (D == 1) {
        // the regions are the edges: their rows are the joins of their vertices
        if ((rc = ar.alloc(&p, (size_t)nr * sizeof(int2)))) return rc;
        std::vector<int2> idc(nr);
        for (int64_t i = 0; i < nr; ++i) idc[i] = make_int2((int)i, 0);
        HIPCHK(hipMemcpyAsync(p, idc.data(), nr * sizeof(int2), hipMemcpyHostToDevice, st));
        reg = (int2 *)p;
        HIPCHK(hipStreamSynchronize(st));
    }
    hipLaunchKernelGGL(k_cell_rows, dim3(grid_for(nr)), dim3(kThreads), 0, st, reg, (int)nr, cx->EDG, cx->SG, valid, Wd,
                       drows);
    HIPCHK(hipGetLastError());
    std::vector<uint64_t> h((size_t)nr * Wd);
    HIPCHK(hipMemcpyAsync(h.data(), drows, h.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // deterministic order: lexicographic by sign row (words from the first)
    std::vector<int64_t> ord(nr);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
        return std::lexicographical_compare(h.begin() + a * Wd, h.begin() + (a + 1) * Wd, h.begin() + b * Wd,
                                            h.begin() + (b + 1) * Wd);
    });
    for (int64_t i = 0; i < nr; ++i) std::copy(h.begin() + ord[i] * Wd, h.begin() + (ord[i] + 1) * Wd, rows + i * Wd);
    (void)keys;
    return PCX_OK;
}

}  // extern "C"
