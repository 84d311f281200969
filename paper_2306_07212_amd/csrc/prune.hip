// Pruning during subdivision (Berzins 2023, Sec. 5.4.2) for level-set
// extraction. Before a layer is subdivided, every current vertex carries the
// signs of every neuron still to come (this layer, the later ones and the
// output: the evaluation writes them into their sign words). An edge whose two
// vertices agree on all of them is never split again and never meets the
// output's zero level set, so it is dropped; vertices left without an edge go
// with it. Both compactions keep the survivors' order (per-chunk counts, then
// an ordered scatter), so the result is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "compact.h"
#include "device.h"
#include "internal.h"

namespace pcx {

namespace {

// edges whose endpoints differ in a sign word of a neuron still to come
struct EdgeKeep {
    const int2 *E;
    const uint64_t *SG;
    int Wd, lwf, V;
    int *CTR;
    __device__ bool operator()(int e) const {
        const int2 ab = E[e];
        if ((unsigned)ab.x >= (unsigned)V || (unsigned)ab.y >= (unsigned)V) {
            raise_flag(CTR, FLAG_BOUNDS);
            return false;
        }
        const uint64_t *ra = SG + (size_t)ab.x * Wd, *rb = SG + (size_t)ab.y * Wd;
        uint64_t d = 0;
        for (int w = lwf; w < Wd; ++w) d |= ra[w] ^ rb[w];
        return d != 0;
    }
};
struct EdgeEmit {
    const int2 *E;
    int2 *out;
    uint8_t *mark;
    __device__ void operator()(int e, int pos) const {
        const int2 ab = E[e];
        out[pos] = ab;
        mark[ab.x] = 1;
        mark[ab.y] = 1;
    }
};
struct Marked {
    const uint8_t *m;
    __device__ bool operator()(int v) const { return m[v] != 0; }
};
struct MapEmit {
    int *map;
    __device__ void operator()(int v, int pos) const { map[v] = pos; }
};

// one wave per surviving vertex: coordinates, sign row and carried
// pre-activations move to the vertex's new index
__global__ __launch_bounds__(kThreads) void k_move_rows(const uint8_t *mark, const int *map, int V, int D, int Wd,
                                                        int ZS, const double *X, const uint64_t *SG, const double *Z,
                                                        double *X2, uint64_t *SG2, double *Z2) {
    const int lane = threadIdx.x & 63;
    for (int v = (blockIdx.x * kThreads + threadIdx.x) >> 6; v < V; v += (gridDim.x * kThreads) >> 6) {
        if (!mark[v]) continue;
        const size_t u = (size_t)map[v];
        for (int k = lane; k < D; k += 64) X2[u * D + k] = X[(size_t)v * D + k];
        for (int k = lane; k < Wd; k += 64) SG2[u * Wd + k] = SG[(size_t)v * Wd + k];
        for (int k = lane; k < ZS; k += 64) Z2[u * ZS + k] = Z[(size_t)v * ZS + k];
    }
}

__global__ __launch_bounds__(kThreads) void k_remap_edges(int2 *E, int n, const int *map) {
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) {
        const int2 ab = E[e];
        E[e] = make_int2(map[ab.x], map[ab.y]);
    }
}

}  // namespace

void launch_prune_edges(const Bufs &b, int V, int E, int Wd, int lwf, int2 *out, uint8_t *mark, int par,
                        hipStream_t st) {
    EdgeKeep keep{b.EDG, b.SG, Wd, lwf, V, b.CTR};
    hipLaunchKernelGGL(k_ccount<EdgeKeep>, dim3(kChunks), dim3(kThreads), 0, st, keep, E, b.SELCNT);
    hipLaunchKernelGGL((k_cscatter<EdgeKeep, EdgeEmit>), dim3(kChunks), dim3(kThreads), 0, st, keep,
                       EdgeEmit{b.EDG, out, mark}, E, (const int *)b.SELCNT, b.CTR + CTR_E + par);
}

void launch_prune_vertices(const Bufs &b, int V, const uint8_t *mark, int *map, int par, hipStream_t st) {
    Marked m{mark};
    hipLaunchKernelGGL(k_ccount<Marked>, dim3(kChunks), dim3(kThreads), 0, st, m, V, b.SELCNT);
    hipLaunchKernelGGL((k_cscatter<Marked, MapEmit>), dim3(kChunks), dim3(kThreads), 0, st, m, MapEmit{map}, V,
                       (const int *)b.SELCNT, b.CTR + CTR_V + par);
}

void launch_move_rows(const Bufs &b, const uint8_t *mark, const int *map, int V, int D, int Wd, int ZS, double *X2,
                      uint64_t *SG2, double *Z2, int2 *E2, int Enew, hipStream_t st) {
    if (V > 0) {
        const int grid = std::min(16384, (V + 3) / 4);
        hipLaunchKernelGGL(k_move_rows, dim3(grid), dim3(kThreads), 0, st, mark, map, V, D, Wd, ZS, b.X, b.SG, b.Z, X2,
                           SG2, Z2);
    }
    if (Enew > 0) {
        const int grid = std::min(16384, (Enew + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_remap_edges, dim3(grid), dim3(kThreads), 0, st, E2, Enew, map);
    }
}

}  // namespace pcx
