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
// independent; their contributions to the (older) parents are summed with
// atomic adds. T is the arithmetic type of the gradients (double, or float
// for the throughput mode); the recorded values are FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// One wave per new vertex of the step; lanes over the layer's columns.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_step(const double *__restrict__ X, const double *__restrict__ Zs,
                                                        const int2 *__restrict__ PQ, T *__restrict__ gx,
                                                        T *__restrict__ gz, int D, int N, int ZS, int j, int V0, int S,
                                                        int *flag) {
    const int lane = threadIdx.x & 63;
    const int wv = (blockIdx.x * kThreads + threadIdx.x) >> 6;
    const int nwv = gridDim.x * (kThreads / 64);
    for (int s = wv; s < S; s += nwv) {
        const int x0 = V0 + s;
        const int2 pq = PQ[x0];
        if ((unsigned)pq.x >= (unsigned)V0 || (unsigned)pq.y >= (unsigned)V0) {
            if (lane == 0) atomicOr(flag, 1);
            continue;
        }
        const size_t p = pq.x, q = pq.y;
        const double zp = Zs[p * ZS + j], zq = Zs[q * ZS + j];
        const double den = zp - zq;
        const double t = zp / den;
        const T tt = (T)t, omt = (T)(1.0 - t);
        // dL/dt from the coordinates and from every carried pre-activation but the current one
        T gt = 0;
        for (int d = lane; d < D; d += 64) {
            const T g0 = gx[(size_t)x0 * D + d];
            gt += g0 * (T)(X[q * D + d] - X[p * D + d]);
            atomicAdd(&gx[p * D + d], omt * g0);
            atomicAdd(&gx[q * D + d], tt * g0);
        }
        for (int c = lane; c < N; c += 64) {
            if (c == j) continue;
            const T g0 = gz[(size_t)x0 * ZS + c];
            if (g0 == (T)0) continue;
            gt += g0 * (T)(Zs[q * ZS + c] - Zs[p * ZS + c]);
            atomicAdd(&gz[p * ZS + c], omt * g0);
            atomicAdd(&gz[q * ZS + c], tt * g0);
        }
        for (int o = 32; o > 0; o >>= 1) gt += __shfl_xor(gt, o, 64);
        if (lane == 0 && gt != (T)0) {
            // t = z_p / (z_p - z_q): dt/dz_p = -z_q / den^2, dt/dz_q = z_p / den^2
            const double inv = 1.0 / (den * den);
            atomicAdd(&gz[p * ZS + j], gt * (T)(-zq * inv));
            atomicAdd(&gz[q * ZS + j], gt * (T)(zp * inv));
        }
    }
}

// Partial sums of dW[c][k] = sum_v gz[v][c] h[v][k] and db[c] = sum_v gz[v][c]
// over a chunk of the vertices present at the layer start (blockIdx.y).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_wgrad(const T *__restrict__ gz, int ZS, const double *__restrict__ hin,
                                                         int hstride, int relu, int Vs, int N, int K,
                                                         double *__restrict__ part) {
    const int entry = blockIdx.x * kThreads + threadIdx.x;  // c * (K + 1) + k, k == K is the bias
    const int c = entry / (K + 1), k = entry % (K + 1);
    const int chunk = (Vs + gridDim.y - 1) / gridDim.y;
    const int v0 = blockIdx.y * chunk, v1 = min(Vs, v0 + chunk);
    if (c >= N) return;
    T acc = 0;
    for (int v = v0; v < v1; ++v) {
        const T g = gz[(size_t)v * ZS + c];
        if (k == K) {
            acc += g;
        } else {
            double h = hin[(size_t)v * hstride + k];
            if (relu) h = h > 0.0 ? h : 0.0;
            acc += g * (T)h;
        }
    }
    part[(size_t)blockIdx.y * N * (K + 1) + entry] = (double)acc;
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
// vertices present at the layer start.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bwd_prev(const T *__restrict__ gz, int ZS, const double *__restrict__ W,
                                                        const double *__restrict__ Zprev, int ZSp, int Vs, int N, int K,
                                                        T *__restrict__ gzp) {
    for (size_t i = blockIdx.x * (size_t)kThreads + threadIdx.x; i < (size_t)Vs * K;
         i += (size_t)gridDim.x * kThreads) {
        const size_t v = i / K;
        const int k = (int)(i % K);
        T acc = 0;
        if (Zprev[v * ZSp + k] > 0.0)
            for (int c = 0; c < N; ++c) acc += (T)W[(size_t)c * K + k] * gz[v * ZS + c];
        gzp[v * ZSp + k] = acc;
    }
}

// ------------------------------------------------------------- launchers

template <typename T>
void bwd_init(const double *grad, T *gx, size_t n, T *gz, size_t nz, hipStream_t st) {
    hipLaunchKernelGGL(k_bwd_init<T>, dim3(1024), dim3(kThreads), 0, st, grad, gx, n, gz, nz);
}
template <typename T>
void bwd_step(const double *X, const double *Zs, const int2 *PQ, T *gx, T *gz, int D, int N, int ZS, int j, int V0,
              int S, int *flag, hipStream_t st) {
    if (S <= 0) return;
    int grid = (S + 3) / 4;
    grid = grid > 8192 ? 8192 : grid;
    hipLaunchKernelGGL(k_bwd_step<T>, dim3(grid), dim3(kThreads), 0, st, X, Zs, PQ, gx, gz, D, N, ZS, j, V0, S, flag);
}
template <typename T>
void bwd_layer(const T *gz, int ZS, const double *hin, int hstride, int relu, int Vs, int N, int K, const double *W,
               double *part, int chunks, double *gW, double *gb, T *gzp, int ZSp, hipStream_t st) {
    const int entries = N * (K + 1);
    const int gx = (entries + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_bwd_wgrad<T>, dim3(gx, chunks), dim3(kThreads), 0, st, gz, ZS, hin, hstride, relu, Vs, N, K,
                       part);
    hipLaunchKernelGGL(k_bwd_wreduce, dim3(gx), dim3(kThreads), 0, st, part, chunks, N, K, gW, gb);
    if (gzp) {
        int grid = (int)std::min<size_t>(8192, ((size_t)Vs * K + kThreads - 1) / kThreads);
        grid = grid < 1 ? 1 : grid;
        hipLaunchKernelGGL(k_bwd_prev<T>, dim3(grid), dim3(kThreads), 0, st, gz, ZS, W, hin, hstride, Vs, N, K, gzp);
    }
}

template void bwd_init<double>(const double *, double *, size_t, double *, size_t, hipStream_t);
template void bwd_init<float>(const double *, float *, size_t, float *, size_t, hipStream_t);
template void bwd_step<double>(const double *, const double *, const int2 *, double *, double *, int, int, int, int, int,
                               int, int *, hipStream_t);
template void bwd_step<float>(const double *, const double *, const int2 *, float *, float *, int, int, int, int, int,
                              int, int *, hipStream_t);
template void bwd_layer<double>(const double *, int, const double *, int, int, int, int, int, const double *, double *,
                                int, double *, double *, double *, int, hipStream_t);
template void bwd_layer<float>(const float *, int, const double *, int, int, int, int, int, const double *, double *,
                               int, double *, double *, float *, int, hipStream_t);

}  // namespace pcx
