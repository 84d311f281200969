// Ordered stream compaction (per-chunk counts, then an ordered scatter):
// survivors keep their index order, so the result does not depend on
// scheduling. Used by the pruning and the cell reconstruction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace pcx {

constexpr int kChunks = 1024;

__device__ __forceinline__ void chunk_of(int n, int &c0, int &c1) {
    const int per = (n + kChunks - 1) / kChunks;
    c0 = min(n, (int)blockIdx.x * per);
    c1 = min(n, c0 + per);
}

// Pred: bool operator()(int i) const; counts per chunk into cnt[blockIdx.x]
template <class Pred>
__global__ __launch_bounds__(kThreads) void k_ccount(Pred pred, int n, int *cnt) {
    __shared__ int s_w[kThreads / 64];
    int c0, c1;
    chunk_of(n, c0, c1);
    int c = 0;
    for (int i = c0 + (int)threadIdx.x; i < c1; i += kThreads) c += pred(i) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += s_w[w];
        cnt[blockIdx.x] = t;
    }
}

// survivors of chunk b go to [sum of counts before b, ...) in index order;
// the last chunk writes the total to *total
template <class Pred, class Emit>
__global__ __launch_bounds__(kThreads) void k_cscatter(Pred pred, Emit emit, int n, const int *cnt, int *total) {
    __shared__ int s_w[kThreads / 64];
    __shared__ int s_base;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    int c0, c1;
    chunk_of(n, c0, c1);
    int pre = 0;
    for (int i = t; i < (int)blockIdx.x; i += kThreads) pre += cnt[i];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if (lane == 0) s_w[wave] = pre;
    __syncthreads();
    if (t == 0) {
        int x = 0;
        for (int w = 0; w < kThreads / 64; ++w) x += s_w[w];
        s_base = x;
        if (blockIdx.x == gridDim.x - 1) *total = x + cnt[blockIdx.x];
    }
    __syncthreads();
    int run = s_base;
    for (int tb = c0; tb < c1; tb += kThreads) {
        const int i = tb + t;
        const bool keep = i < c1 && pred(i);
        const uint64_t bal = __ballot(keep);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        __syncthreads();  // s_w reuse
        if (lane == 0) s_w[wave] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) {
            if (w < wave) off += s_w[w];
            tot += s_w[w];
        }
        if (keep) emit(i, run + off + below);
        run += tot;
    }
}


}  // namespace pcx
