/*
 * sanitize_main.c -- TEST INFRASTRUCTURE ONLY: a stand-alone driver that runs
 * the oracle's entry points (box and simplex extraction with and without the
 * output level set and pruning, one and several threads, the forward pass and
 * the vertex solve) on networks read from a file, so that the oracle can be
 * built with the compiler's address and undefined-behaviour sanitizers and
 * exercised outside Python. Exit status 0: every call succeeded and agreed
 * across thread counts.
 *
 * Input file (little-endian): int32 count; per network: int32 L, int32
 * widths[L + 1], then for each layer W [N_l][N_{l-1}] and b [N_l] as float64.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int D, L;
    const int *widths;
    const double *const *W;
    const double *const *b;
} pcxo_net;
typedef struct pcxo_result pcxo_result;

void pcxo_set_threads(int n);
pcxo_result *pcxo_extract(const pcxo_net *net, const double *lo, const double *hi, int include_output, int prune,
                          int mutation);
pcxo_result *pcxo_extract_simplex(const pcxo_net *net, const double *corners, int include_output, int prune,
                                  int mutation);
void pcxo_free(pcxo_result *r);
int pcxo_status(const pcxo_result *r);
const char *pcxo_message(const pcxo_result *r);
long pcxo_V(const pcxo_result *r);
long pcxo_E(const pcxo_result *r);
int pcxo_M(const pcxo_result *r);
int pcxo_n_steps(const pcxo_result *r);
void pcxo_copy(const pcxo_result *r, double *X, int8_t *S, int32_t *edges, long *steps);
int pcxo_forward(const pcxo_net *net, const double *x, double *z_all);
int pcxo_vertex_solve(const pcxo_net *net, int include_output, const double *lo, const double *hi,
                      const int8_t *sigma, double *x_out);

static int read_exact(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

/* runs one extraction; returns a checksum of its arrays, or -1 on failure */
static double run(const pcxo_net *net, int simplex, int incl, int prune, int threads, long *V_out) {
    const int D = net->D;
    double lo[16], hi[16], corners[17 * 16];
    for (int j = 0; j < D; ++j) { lo[j] = -1.0; hi[j] = 1.0; }
    for (int i = 0; i <= D; ++i)
        for (int j = 0; j < D; ++j) corners[i * D + j] = (i > 0 && j == i - 1) ? 2.0 : -1.0;
    pcxo_set_threads(threads);
    pcxo_result *r = simplex ? pcxo_extract_simplex(net, corners, incl, prune, 0) : pcxo_extract(net, lo, hi, incl, prune, 0);
    pcxo_set_threads(1);
    if (!r) return -1.0;
    if (pcxo_status(r) != 0) {
        fprintf(stderr, "extraction failed: %s\n", pcxo_message(r));
        pcxo_free(r);
        return -1.0;
    }
    const long V = pcxo_V(r), E = pcxo_E(r);
    const int M = pcxo_M(r), ns = pcxo_n_steps(r);
    double *X = malloc(sizeof(double) * (size_t)(V ? V : 1) * D);
    int8_t *S = malloc((size_t)(V ? V : 1) * M);
    int32_t *Ed = malloc(sizeof(int32_t) * (size_t)(E ? E : 1) * 2);
    long *st = malloc(sizeof(long) * (size_t)(ns ? ns : 1) * 4);
    pcxo_copy(r, X, S, Ed, st);
    double sum = 0.0;
    for (long i = 0; i < V * D; ++i) sum += X[i] * (double)((i % 7) + 1);
    for (long i = 0; i < V * M; ++i) sum += S[i] * (double)((i % 5) + 1);
    for (long i = 0; i < 2 * E; ++i) sum += Ed[i];
    /* every vertex solved back from its sign-vector (the box, without the output) */
    if (!simplex && !incl && !prune) {
        double x[16];
        for (long v = 0; v < V; v += 1 + V / 64)
            if (pcxo_vertex_solve(net, 0, lo, hi, S + v * M, x) != 0) sum = -1e300;
    }
    double *z = malloc(sizeof(double) * 4096);
    for (long v = 0; v < V; v += 1 + V / 64) pcxo_forward(net, X + v * D, z);
    free(z);
    *V_out = V;
    free(X); free(S); free(Ed); free(st);
    pcxo_free(r);
    return sum;
}

int main(int argc, char **argv) {
    if (argc != 2) { fprintf(stderr, "usage: %s nets.bin\n", argv[0]); return 2; }
    FILE *f = fopen(argv[1], "rb");
    if (!f) { perror("open"); return 2; }
    int32_t count = 0;
    if (!read_exact(f, &count, 4)) return 2;
    int bad = 0;
    for (int n = 0; n < count; ++n) {
        int32_t L = 0;
        if (!read_exact(f, &L, 4) || L < 1 || L > 16) return 2;
        int widths[17];
        for (int l = 0; l <= L; ++l) {
            int32_t w;
            if (!read_exact(f, &w, 4) || w < 1 || w > 4096) return 2;
            widths[l] = w;
        }
        double *W[16], *b[16];
        for (int l = 0; l < L; ++l) {
            const size_t nw = (size_t)widths[l + 1] * widths[l];
            W[l] = malloc(sizeof(double) * nw);
            b[l] = malloc(sizeof(double) * (size_t)widths[l + 1]);
            if (!read_exact(f, W[l], sizeof(double) * nw) || !read_exact(f, b[l], sizeof(double) * widths[l + 1])) return 2;
        }
        pcxo_net net = {widths[0], L, widths, (const double *const *)W, (const double *const *)b};
        const int cases[][3] = {{0, 0, 0}, {0, 1, 0}, {0, 1, 1}, {1, 0, 0}, {1, 1, 1}};
        for (size_t c = 0; c < sizeof cases / sizeof cases[0]; ++c) {
            long V1 = 0, V4 = 0;
            const double s1 = run(&net, cases[c][0], cases[c][1], cases[c][2], 1, &V1);
            const double s4 = run(&net, cases[c][0], cases[c][1], cases[c][2], 4, &V4);
            if (s1 == -1.0 || s1 != s4 || V1 != V4) {
                fprintf(stderr, "network %d case %zu: %g vs %g\n", n, c, s1, s4);
                bad = 1;
            } else {
                printf("network %d case %zu: V=%ld\n", n, c, V1);
            }
        }
        for (int l = 0; l < L; ++l) { free(W[l]); free(b[l]); }
    }
    fclose(f);
    return bad;
}
