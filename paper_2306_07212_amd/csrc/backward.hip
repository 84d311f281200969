// Backward pass of edge subdivision: gradients of a loss on the vertex
// coordinates with respect to the weights and biases (the differentiability
// used in Sec. 5.3 of Berzins 2023).
//
// The forward pass computed every value along a graph that is recorded in the
// tape: the box corners' pre-activations by the layer evaluation
//   Z^(l)[v] = W^(l) h(v) + b^(l),  h(v) = ReLU(Z^(l-1)[v])  (x_v for l = 1),
// and each new vertex x0 of step (l, j) from its splitting edge (p, q), p = V+:
//   t = z_p / (z_p - z_q),  x0 = x_p + t (x_q - x_p),
//   Z(x0)[c] = Z_p[c] + t (Z_q[c] - Z_p[c])  (c != j),   Z(x0)[j] = 0.
// Reverse mode walks it back: steps in reverse order (children before their
// parents), then each layer start. Within one step the new vertices are
// independent; each parent then sums the contributions of its children of the
// step itself, in increasing child order (no atomics: the gradients are the
// same bits on every run). Every parent's children come from one sort of
// (parent, child) records per backward call. T is the arithmetic type of the
// gradients (double, or float for the throughput mode); the recorded values
// are FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "internal.h"

namespace pcx {

template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_init(const double *__restrict__ grad, T *__restrict__ gx, size_t n,
                                                        T *__restrict__ gz, size_t nz) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        gx[i] = (T)grad[i];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nz; i += (size_t)gridDim.x * blockDim.x)
        gz[i] = (T)0;
}

// Records of the creation graph, one per (new vertex, parent): key = parent
// << 32 | child << 1 | side (side 0: the child's V+ parent, 1: its V- parent),
// record index 2 (child - Vb) + side. Sorted, they list each parent's
// children in increasing order.
__global__ __launch_bounds__(kThreads) void k_bwd_records(const int2 *__restrict__ PQ, int Vb, int V,
                                                           uint64_t *__restrict__ keys, int *flag) {
    for (int x0 = Vb + blockIdx.x * kThreads + threadIdx.x; x0 < V; x0 += gridDim.x * kThreads) {
        const int2 pq = PQ[x0];
        if ((unsigned)pq.x >= (unsigned)x0 || (unsigned)pq.y >= (unsigned)x0) atomicOr(flag, 1);
        const uint64_t c2 = (uint64_t)(uint32_t)x0 << 1;
        keys[2 * (size_t)(x0 - Vb)] = ((uint64_t)(uint32_t)pq.x << 32) | c2;
        keys[2 * (size_t)(x0 - Vb) + 1] = ((uint64_t)(uint32_t)pq.y << 32) | c2 | 1u;
    }
}

// position of every record in the sorted order
__global__ __launch_bounds__(kThreads) void k_bwd_pos(const uint32_t *__restrict__ vals, int n, int *__restrict__ pos) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) pos[vals[i]] = i;
}

// One wave per new vertex of the step: t of its splitting edge and dL/dt,
// from its coordinates and every carried pre-activation but the current one
// (lanes over columns, a fixed reduction order).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_child(const double *__restrict__ X, const double *__restrict__ Zs,
                                                         const int2 *__restrict__ PQ, const T *__restrict__ gx,
                                                         const T *__restrict__ gz, int D, int N, int ZS, int j, int V0,
                                                         int S, double *__restrict__ tt, T *__restrict__ gtt) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    const int nwv = gridDim.x * (kThreads / 64);
    for (int s = wv; s < S; s += nwv) {
        const int x0 = V0 + s;
        const int2 pq = PQ[x0];
        const size_t p = pq.x, q = pq.y;
        const double zp = Zs[p * ZS + j], zq = Zs[q * ZS + j];
        const double t = zp / (zp - zq);
        T gt = 0;
        for (int d = lane; d < D; d += 64) gt += gx[(size_t)x0 * D + d] * (T)(X[q * D + d] - X[p * D + d]);
        for (int c = lane; c < N; c += 64) {
            if (c == j) continue;
            gt += gz[(size_t)x0 * ZS + c] * (T)(Zs[q * ZS + c] - Zs[p * ZS + c]);
        }
        for (int o = 32; o > 0; o >>= 1) gt += __shfl_xor(gt, o, 64);
        if (lane == 0) {
            tt[x0] = t;
            gtt[x0] = gt;
        }
    }
}

// One wave per (new vertex, side) record of the step. The record that comes
// first among its parent's children of this step sums, in child order, every
// such child's contribution to the parent:
//   dL/dx_p += (1 - t) dL/dx0,  dL/dZ_p[c] += (1 - t) dL/dZ0[c]  (c != j),
//   dL/dz_p += dL/dt * dt/dz_p  with dt/dz_p = -z_q / (z_p - z_q)^2
// (and with t, dt/dz_q = z_p / (z_p - z_q)^2 for the V- parent q).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_parent(const double *__restrict__ Zs, const int2 *__restrict__ PQ,
                                                          T *__restrict__ gx, T *__restrict__ gz, int D, int N, int ZS,
                                                          int j, int Vb, int V0, int S,
                                                          const uint64_t *__restrict__ skey, int nrec,
                                                          const int *__restrict__ pos, const double *__restrict__ tt,
                                                          const T *__restrict__ gtt, int *flag) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    const int nwv = gridDim.x * (kThreads / 64);
    for (int r = wv; r < 2 * S; r += nwv) {
        const int rec = 2 * (V0 - Vb) + r;
        const int i = pos[rec];
        if ((unsigned)i >= (unsigned)nrec) {
            if (lane == 0) atomicOr(flag, 1);
            continue;
        }
        const uint64_t k = skey[i];
        const uint32_t P = (uint32_t)(k >> 32);
        // a child of P in this step comes before: it is that one's work
        if (i > 0 && (uint32_t)(skey[i - 1] >> 32) == P && (int)((uint32_t)skey[i - 1] >> 1) >= V0) continue;
        for (int e = i; e < nrec; ++e) {
            const uint64_t ke = skey[e];
            const int c = (int)((uint32_t)ke >> 1);
            if ((uint32_t)(ke >> 32) != P || c >= V0 + S) break;
            const int side = (int)(ke & 1u);
            const int2 pq = PQ[c];
            const double zp = Zs[(size_t)pq.x * ZS + j], zq = Zs[(size_t)pq.y * ZS + j];
            const double t = tt[c], den = zp - zq;
            const double inv = 1.0 / (den * den);
            const T coef = side ? (T)t : (T)(1.0 - t);
            for (int d = lane; d < D; d += 64) gx[(size_t)P * D + d] += coef * gx[(size_t)c * D + d];
            for (int col = lane; col < N; col += 64) {
                if (col == j) continue;
                gz[(size_t)P * ZS + col] += coef * gz[(size_t)c * ZS + col];
            }
            if (lane == 0) gz[(size_t)P * ZS + j] += gtt[c] * (T)(side ? zp * inv : -zq * inv);
        }
    }
}

// Partial sums of the weight and bias gradients over one chunk of vertices:
// part[chunk][c][k] = sum_v gz[v][c] h[v][k], h = ReLU of the previous layer's
// pre-activations (the coordinates for layer 1), and k == K is the bias
// (h = 1). A workgroup takes a 64 x 64 tile of the (c, k) entries and its
// chunk, stages 32 vertices' gz and h values of the tile through LDS at a time,
// and each thread accumulates 4 x 4 entries. Every entry sums its chunk's
// vertices in order, one fused multiply-add each, and k_bwd_wreduce adds the
// chunks in order: the gradients are the same bits on every run.
constexpr int kWgTile = 64, kWgRows = 32;
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_wgrad_tiled(const T *__restrict__ gz, int ZS,
                                                         const double *__restrict__ hin, int hstride, int relu, int Vs,
                                                         int N, int K, int tiles_k, double *__restrict__ part) {
    __shared__ T gs[kWgRows][kWgTile + 1];
    __shared__ T hs[kWgRows][kWgTile + 1];
    const int t = threadIdx.x, tc = t & 15, tk = t >> 4;
    const int c0 = (blockIdx.x / tiles_k) * kWgTile, k0 = (blockIdx.x % tiles_k) * kWgTile;
    const int chunk = (Vs + gridDim.y - 1) / gridDim.y;
    const int v0 = blockIdx.y * chunk, v1 = min(Vs, v0 + chunk);
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    for (int vb = v0; vb < v1; vb += kWgRows) {
        const int nv = min(kWgRows, v1 - vb);
        for (int idx = t; idx < kWgRows * kWgTile; idx += 256) {
            const int r = idx / kWgTile, q = idx % kWgTile;
            const int v = vb + r, c = c0 + q, k = k0 + q;
            T g = 0, h = 0;
            if (r < nv) {
                if (c < N) g = gz[(size_t)v * ZS + c];
                if (k < K) {
                    double x = hin[(size_t)v * hstride + k];
                    if (relu) x = x > 0.0 ? x : 0.0;
                    h = (T)x;
                } else if (k == K) {
                    h = 1;
                }
            }
            gs[r][q] = g;
            hs[r][q] = h;
        }
        __syncthreads();
        for (int r = 0; r < nv; ++r) {
            T a[4], bb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = gs[r][tc + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bb[j] = hs[r][tk + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fma(a[i], bb[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int c = c0 + tc + 16 * i;
        if (c >= N) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + tk + 16 * j;
            if (k <= K) part[(size_t)blockIdx.y * N * (K + 1) + (size_t)c * (K + 1) + k] = (double)acc[i][j];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_bwd_wreduce(const double *__restrict__ part, int chunks, int N, int K,
                                                           double *__restrict__ gW, double *__restrict__ gb) {
    const int entry = blockIdx.x * kThreads + threadIdx.x;
    if (entry >= N * (K + 1)) return;
    double s = 0.0;
    for (int y = 0; y < chunks; ++y) s += part[(size_t)y * N * (K + 1) + entry];
    const int c = entry / (K + 1), k = entry % (K + 1);
    if (k == K) gb[c] = s;
    else gW[(size_t)c * K + k] = s;
}

// gz_prev[v][k] = (sum_c W[c][k] gz[v][c]) * [Z_prev[v][k] > 0] for the
// vertices present at the layer start. A workgroup takes 64 vertices x 64
// columns k, stages 32 neurons c of gz and W at a time through LDS, and each
// thread accumulates 4 x 4 entries, summing over c in order.
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_prev(const T *__restrict__ gz, int ZS, const double *__restrict__ W,
                                                  const double *__restrict__ Zprev, int ZSp, int Vs, int N, int K,
                                                  T *__restrict__ gzp) {
    __shared__ T gs[kWgTile][kWgRows + 1];
    __shared__ T ws[kWgRows][kWgTile + 1];
    const int t = threadIdx.x, tv = t & 15, tk = t >> 4;
    const int v0 = blockIdx.x * kWgTile, k0 = blockIdx.y * kWgTile;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0;
    for (int cb = 0; cb < N; cb += kWgRows) {
        const int nc = min(kWgRows, N - cb);
        for (int idx = t; idx < kWgTile * kWgRows; idx += 256) {
            const int r = idx / kWgRows, q = idx % kWgRows;  // gz: vertex r, neuron q
            const int v = v0 + r;
            gs[r][q] = (v < Vs && q < nc) ? gz[(size_t)v * ZS + cb + q] : (T)0;
            const int cr = idx / kWgTile, kq = idx % kWgTile;  // W: neuron cr, column kq
            ws[cr][kq] = (cr < nc && k0 + kq < K) ? (T)W[(size_t)(cb + cr) * K + k0 + kq] : (T)0;
        }
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
            T a[4], bb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = gs[tv + 16 * i][c];
#pragma unroll
            for (int j = 0; j < 4; ++j) bb[j] = ws[c][tk + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fma(bb[j], a[i], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int v = v0 + tv + 16 * i;
        if (v >= Vs) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + tk + 16 * j;
            if (k < K) gzp[(size_t)v * ZSp + k] = Zprev[(size_t)v * ZSp + k] > 0.0 ? acc[i][j] : (T)0;
        }
    }
}

// ------------------------------------------------------------- launchers

template <typename T>
void bwd_init(const double *grad, T *gx, size_t n, T *gz, size_t nz, hipStream_t st) {
    hipLaunchKernelGGL(k_bwd_init<T>, dim3(1024), dim3(kThreads), 0, st, grad, gx, n, gz, nz);
}
void bwd_records(const int2 *PQ, int Vb, int V, uint64_t *keys, int *flag, hipStream_t st) {
    if (V <= Vb) return;
    const int grid = std::min(8192, (V - Vb + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_bwd_records, dim3(grid), dim3(kThreads), 0, st, PQ, Vb, V, keys, flag);
}
void bwd_pos(const uint32_t *vals, int n, int *pos, hipStream_t st) {
    if (n <= 0) return;
    const int grid = std::min(8192, (n + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_bwd_pos, dim3(grid), dim3(kThreads), 0, st, vals, n, pos);
}
template <typename T>
void bwd_step(const double *X, const double *Zs, const int2 *PQ, T *gx, T *gz, int D, int N, int ZS, int j, int Vb,
              int V0, int S, const uint64_t *skey, int nrec, const int *pos, double *tt, T *gtt, int *flag,
              hipStream_t st) {
    if (S <= 0) return;
    int grid = (S + 3) / 4;
    grid = grid > 8192 ? 8192 : grid;
    hipLaunchKernelGGL(k_bwd_child<T>, dim3(grid), dim3(kThreads), 0, st, X, Zs, PQ, gx, gz, D, N, ZS, j, V0, S, tt,
                       gtt);
    grid = (2 * S + 3) / 4;
    grid = grid > 8192 ? 8192 : grid;
    hipLaunchKernelGGL(k_bwd_parent<T>, dim3(grid), dim3(kThreads), 0, st, Zs, PQ, gx, gz, D, N, ZS, j, Vb, V0, S, skey,
                       nrec, pos, tt, gtt, flag);
}
template <typename T>
void bwd_layer(const T *gz, int ZS, const double *hin, int hstride, int relu, int Vs, int N, int K, const double *W,
               double *part, int chunks, double *gW, double *gb, T *gzp, int ZSp, hipStream_t st) {
    const int entries = N * (K + 1);
    const int gx = (entries + kThreads - 1) / kThreads;
    const int tiles_c = (N + kWgTile - 1) / kWgTile, tiles_k = (K + 1 + kWgTile - 1) / kWgTile;
    hipLaunchKernelGGL(k_bwd_wgrad_tiled<T>, dim3(tiles_c * tiles_k, chunks), dim3(256), 0, st, gz, ZS, hin, hstride,
                       relu, Vs, N, K, tiles_k, part);
    hipLaunchKernelGGL(k_bwd_wreduce, dim3(gx), dim3(kThreads), 0, st, part, chunks, N, K, gW, gb);
    if (gzp && Vs > 0) {
        const dim3 grid((Vs + kWgTile - 1) / kWgTile, (K + kWgTile - 1) / kWgTile);
        hipLaunchKernelGGL(k_bwd_prev<T>, grid, dim3(256), 0, st, gz, ZS, W, hin, hstride, Vs, N, K, gzp);
    }
}

template void bwd_init<double>(const double *, double *, size_t, double *, size_t, hipStream_t);
template void bwd_init<float>(const double *, float *, size_t, float *, size_t, hipStream_t);
template void bwd_step<double>(const double *, const double *, const int2 *, double *, double *, int, int, int, int, int,
                               int, int, const uint64_t *, int, const int *, double *, double *, int *, hipStream_t);
template void bwd_step<float>(const double *, const double *, const int2 *, float *, float *, int, int, int, int, int,
                              int, int, const uint64_t *, int, const int *, double *, float *, int *, hipStream_t);
template void bwd_layer<double>(const double *, int, const double *, int, int, int, int, int, const double *, double *,
                                int, double *, double *, double *, int, hipStream_t);
template void bwd_layer<float>(const float *, int, const double *, int, int, int, int, int, const double *, double *,
                               int, double *, double *, float *, int, hipStream_t);

}  // namespace pcx
