/*
 * pcx_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of edge subdivision
 * (Berzins, "Polyhedral Complex Extraction from ReLU Networks using Edge
 * Subdivision", ICML 2023). It exists to check the GPU library: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or helper with the GPU path.
 *
 * Conventions (readings of the paper where it is silent or garbled):
 *  - Layers follow Sec. 3.4: x^(l) = ReLU(W^(l) x^(l-1) + b^(l)), with W^(l)
 *    stored row-major as [N_l][N_{l-1}] (z = W x + b).
 *  - Sign of a neuron at x is sgn(z) (Sec. 3.4): + iff z > 0.
 *  - The domain is a bounded polyhedron given as m half-spaces (Sec. 4.1): the
 *    box [lo, hi]^D (m = 2D; entry 2j is x_j - lo_j >= 0, entry 2j+1 is
 *    hi_j - x_j >= 0) or a simplex (m = D + 1; entry i is the barycentric
 *    coordinate of corner i). They are the first m entries of every
 *    sign-vector; interior cells are + there.
 *  - Then one entry per subdivided neuron, layer by layer in index order.
 *    Hidden neurons are always subdivided; the output layer only when
 *    include_output is set (zero level set of the output, Sec. 5.4).
 *  - Sign entries are stored as int8: +1, 0, -1.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -fPIC -shared (no FMA
 * contraction). pcxo_set_threads(n) spreads the per-vertex loops (the forward
 * pass at the layer start, the evaluation of a neuron at every vertex, the new
 * vertices of a step) over n threads; each vertex's arithmetic is the same
 * sequential expression whatever the thread count, so the result is too. The
 * default is one thread.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static int g_threads = 1;

void pcxo_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

#define PCXO_OK 0
#define PCXO_ERR_INVALID (-1)
#define PCXO_ERR_OOM (-2)
#define PCXO_ERR_DEGENERATE (-3)
#define PCXO_ERR_SINGULAR (-6)

typedef struct {
    int D;              /* input dimension */
    int L;              /* number of affine layers (hidden + output) */
    const int *widths;  /* L+1 entries: D, N_1, ..., N_L */
    const double *const *W; /* W[l-1] is [N_l][N_{l-1}] row-major */
    const double *const *b; /* b[l-1] is [N_l] */
} pcxo_net;

typedef struct {
    int status;
    char msg[256];
    int D, M, n_steps;
    long V, E;
    double *X;      /* [V][D] */
    int8_t *S;      /* [V][M] */
    int32_t *edges; /* [E][2] */
    long *steps;    /* [n_steps][4]: V_n, E_n, S_n (splitting edges), K_n (2-face records) */
    double min_margin; /* smallest |z| over all sign decisions at old vertices */
} pcxo_result;

/* ------------------------------------------------------------------ utils */

static void *xrealloc(void *p, size_t n) {
    void *q = realloc(p, n ? n : 1);
    return q;
}

static int n_sub_layers(const pcxo_net *net, int include_output) {
    return include_output ? net->L : net->L - 1;
}

static int entry_count_m(const pcxo_net *net, int m, int include_output) {
    int M = m;
    for (int l = 1; l <= n_sub_layers(net, include_output); ++l) M += net->widths[l];
    return M;
}

static int entry_count(const pcxo_net *net, int include_output) {
    int M = 2 * net->D;
    for (int l = 1; l <= n_sub_layers(net, include_output); ++l) M += net->widths[l];
    return M;
}

/* Sec. 3.4: the plain forward pass. Writes every layer's pre-activation
 * (layers 1..L, concatenated) into z_all. ReLU between layers, none after L. */
int pcxo_forward(const pcxo_net *net, const double *x, double *z_all) {
    int maxw = 0;
    for (int l = 0; l <= net->L; ++l) if (net->widths[l] > maxw) maxw = net->widths[l];
    double *h = (double *)malloc(sizeof(double) * maxw);
    double *hn = (double *)malloc(sizeof(double) * maxw);
    if (!h || !hn) { free(h); free(hn); return PCXO_ERR_OOM; }
    for (int k = 0; k < net->D; ++k) h[k] = x[k];
    long off = 0;
    for (int l = 1; l <= net->L; ++l) {
        int nin = net->widths[l - 1], nout = net->widths[l];
        const double *W = net->W[l - 1], *b = net->b[l - 1];
        for (int i = 0; i < nout; ++i) {
            double acc = 0.0;
            for (int k = 0; k < nin; ++k) acc += W[(long)i * nin + k] * h[k];
            double z = acc + b[i];
            z_all[off + i] = z;
            hn[i] = z > 0.0 ? z : 0.0;
        }
        off += nout;
        double *t = h; h = hn; hn = t;
    }
    free(h); free(hn);
    return PCXO_OK;
}

/* Post-activation output of layer `upto` (0 = the input itself) at x.
 * `t1`, `t2` must each hold the widest layer; `out` holds widths[upto] values. */
static void hidden_at(const pcxo_net *net, const double *x, int upto, double *out, double *t1, double *t2) {
    int D = net->D;
    double *h = t1, *hn = t2;
    for (int k = 0; k < D; ++k) h[k] = x[k];
    for (int l = 1; l <= upto; ++l) {
        int nin = net->widths[l - 1], nout = net->widths[l];
        const double *W = net->W[l - 1], *b = net->b[l - 1];
        for (int i = 0; i < nout; ++i) {
            double acc = 0.0;
            for (int k = 0; k < nin; ++k) acc += W[(long)i * nin + k] * h[k];
            double z = acc + b[i];
            hn[i] = z > 0.0 ? z : 0.0;
        }
        double *t = h; h = hn; hn = t;
    }
    memcpy(out, h, sizeof(double) * (size_t)net->widths[upto]);
}

/* Join of two sign entries in the intersection poset (Sec. 3.5): the closest
 * common ascendant. Equal signs stay, 0 joins with s to s, + and - conflict. */
static int join_sign(int a, int b, int *conflict) {
    if (a == b) return a;
    if (a == 0) return b;
    if (b == 0) return a;
    *conflict = 1;
    return 0;
}

/* ---------------------------------------------------- stable merge sort */

typedef struct {
    const int8_t *keys; /* [K][len] */
    int len;
} face_ctx;

static int face_cmp(const face_ctx *c, int32_t a, int32_t b) {
    return memcmp(c->keys + (long)a * c->len, c->keys + (long)b * c->len, (size_t)c->len);
}

static void merge_sort(int32_t *idx, int32_t *tmp, long n, const face_ctx *c) {
    if (n < 2) return;
    long h = n / 2;
    merge_sort(idx, tmp, h, c);
    merge_sort(idx + h, tmp, n - h, c);
    long i = 0, j = h, k = 0;
    while (i < h && j < n) {
        if (face_cmp(c, idx[j], idx[i]) < 0) tmp[k++] = idx[j++];
        else tmp[k++] = idx[i++];
    }
    while (i < h) tmp[k++] = idx[i++];
    while (j < n) tmp[k++] = idx[j++];
    memcpy(idx, tmp, sizeof(int32_t) * (size_t)n);
}

/* ------------------------------------------------------------- extract */

static void fail(pcxo_result *r, int code, const char *msg) {
    r->status = code;
    snprintf(r->msg, sizeof r->msg, "%s", msg);
}

/* Pruning during subdivision (Sec. 5.4.2), applied before each subdivided
 * layer l: the sign of every neuron still to come (layers l..L, the output
 * included) is taken at every current vertex by the forward pass; an edge
 * whose two vertices agree on all of them can never split again nor meet the
 * output's zero level set, so it is dropped, and so are vertices left without
 * edges. Survivors keep their relative order. Only meaningful for the level
 * set, so it requires include_output. Returns the new vertex count. */
static long prune_complex(const pcxo_net *net, int l, int mutation, double *X, int8_t *S, int M,
                          int32_t *Ed, long V, long *E_io, int *status) {
    const int D = net->D;
    int total = 0, first = 0;
    for (int m = 1; m <= net->L; ++m) {
        if (m < l) first += net->widths[m];
        total += net->widths[m];
    }
    int last = total;                         /* future neurons: [first, last) of the forward pass */
    if (mutation == 6) last = first + net->widths[l];  /* planted mistake: current layer only */
    const int nf = last - first;
    int8_t *fs = (int8_t *)malloc((size_t)(V ? V : 1) * (size_t)(nf ? nf : 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)total);
    long *map = (long *)malloc(sizeof(long) * (size_t)(V ? V : 1));
    if (!fs || !z || !map) { free(fs); free(z); free(map); *status = PCXO_ERR_OOM; return V; }
    for (long v = 0; v < V; ++v) {
        if (pcxo_forward(net, X + v * D, z) != PCXO_OK) { *status = PCXO_ERR_OOM; break; }
        for (int k = 0; k < nf; ++k) {
            double zk = z[first + k];
            fs[v * nf + k] = (int8_t)(zk > 0.0 ? 1 : (zk < 0.0 ? -1 : 0));
        }
        map[v] = -1;
    }
    long E = *E_io, ne = 0;
    for (long e = 0; e < E && *status == PCXO_OK; ++e) {
        int32_t a = Ed[2 * e], b = Ed[2 * e + 1];
        if (memcmp(fs + (long)a * nf, fs + (long)b * nf, (size_t)nf) == 0) continue;
        Ed[2 * ne] = a; Ed[2 * ne + 1] = b; ++ne;
        map[a] = 0; map[b] = 0;
    }
    long nv = 0;
    for (long v = 0; v < V; ++v) {
        if (map[v] < 0) continue;
        if (nv != v) {
            memmove(X + nv * D, X + v * D, sizeof(double) * (size_t)D);
            memmove(S + nv * M, S + v * M, (size_t)M);
        }
        map[v] = nv++;
    }
    for (long e = 0; e < ne; ++e) { Ed[2 * e] = (int32_t)map[Ed[2 * e]]; Ed[2 * e + 1] = (int32_t)map[Ed[2 * e + 1]]; }
    *E_io = ne;
    free(fs); free(z); free(map);
    return nv;
}

/* mutation (test-only planted mistakes; 0 = none):
 *   1: perturb neuron zeros only toward + (drops half of the parent 2-faces)
 *   2: interpolate with the wrong weight, x0 = x_p + (1-t)(x_q - x_p)
 *   3: forget to append the intersecting edges of step 5
 *   4: new vertices inherit the sign of V+ instead of the join
 *   5: step 1 reads the bias of the neighbouring neuron (an index slip)
 *   6: pruning compares only the current layer's neurons */
/* The domain (Sec. 4.1) is given by m half-spaces, the first m entries of every
 * sign-vector, and by its 1-skeleton: nv vertices X0 [nv][D] with their domain
 * entries S0 [nv][m] (+1 or 0) and ne edges E0 [ne][2]. */
static pcxo_result *extract_core(const pcxo_net *net, int m, long nv, const double *X0, const int8_t *S0, long ne,
                                 const int32_t *E0, int include_output, int prune, int mutation) {
    pcxo_result *r = (pcxo_result *)calloc(1, sizeof(pcxo_result));
    if (!r) return NULL;
    const int D = net->D;
    if (D < 1 || D > 20 || net->L < 1 || net->widths[0] != D) { fail(r, PCXO_ERR_INVALID, "bad widths"); return r; }
    if (prune && !include_output) { fail(r, PCXO_ERR_INVALID, "pruning needs the output level set"); return r; }
    const int nsub = n_sub_layers(net, include_output);
    const int M = entry_count_m(net, m, include_output);
    r->D = D; r->M = M;
    int maxw = D;
    for (int l = 0; l <= net->L; ++l) if (net->widths[l] > maxw) maxw = net->widths[l];
    int nsteps = 0;
    for (int l = 1; l <= nsub; ++l) nsteps += net->widths[l];
    r->n_steps = nsteps;
    r->steps = (long *)calloc((size_t)nsteps * 4 + 1, sizeof(long));
    r->min_margin = INFINITY;

    /* Step 0 (Sec. 4.2.1): the 1-skeleton of the domain */
    long V = nv, E = ne;
    long capV = V < 1024 ? 1024 : V, capE = E < 1024 ? 1024 : E;
    double *X = (double *)malloc(sizeof(double) * (size_t)capV * D);
    int8_t *S = (int8_t *)calloc((size_t)capV * M, 1);
    int32_t *Ed = (int32_t *)malloc(sizeof(int32_t) * (size_t)capE * 2);
    if (!X || !S || !Ed) { free(X); free(S); free(Ed); fail(r, PCXO_ERR_OOM, "oom"); return r; }
    memcpy(X, X0, sizeof(double) * (size_t)V * D);
    for (long v = 0; v < V; ++v) memcpy(S + v * M, S0 + v * m, (size_t)m);
    memcpy(Ed, E0, sizeof(int32_t) * (size_t)E * 2);

    double *Hm = NULL;   /* memoised h^(l-1)(v) for the layer being subdivided */
    const int nth = g_threads;
    /* forward-pass scratch: two rows of the widest layer per thread */
    double *tmp = (double *)malloc(sizeof(double) * (size_t)maxw * 2 * (size_t)nth);
    if (!tmp) { free(X); free(S); free(Ed); fail(r, PCXO_ERR_OOM, "oom"); return r; }
    double *tmp2 = NULL;
    double *zv = NULL;   /* pre-activation of the current neuron at each vertex */
    long capZ = 0;
    int32_t *spl = NULL; long capSpl = 0;
    int8_t *fkeys = NULL; int32_t *fvert = NULL; int32_t *fidx = NULL, *ftmp = NULL; long capF = 0; size_t capFB = 0;
    int status = PCXO_OK;
    const char *why = "";
    int step = 0;
    int entry_base = m;

    for (int l = 1; l <= nsub && status == PCXO_OK; ++l) {
        const int nin = net->widths[l - 1], nl = net->widths[l];
        const double *W = net->W[l - 1], *b = net->b[l - 1];
        if (prune) {
            V = prune_complex(net, l, mutation, X, S, M, Ed, V, &E, &status);
            if (status != PCXO_OK) { why = "oom"; break; }
        }
        /* memoise h^(l-1) at every current vertex by the forward pass from coordinates */
        free(Hm);
        long capH = capV;
        Hm = (double *)malloc(sizeof(double) * (size_t)capH * nin);
        if (!Hm) { status = PCXO_ERR_OOM; why = "oom"; break; }
#pragma omp parallel for num_threads(nth) schedule(static)
        for (long v = 0; v < V; ++v) {
            double *t1 = tmp + (size_t)maxw * 2 * (size_t)omp_get_thread_num();
            hidden_at(net, X + v * D, l - 1, Hm + v * nin, t1, t1 + maxw);
        }

        for (int i = 0; i < nl && status == PCXO_OK; ++i, ++step) {
            const int n = entry_base + i; /* entry of this neuron in the sign-vector */
            r->steps[4 * step + 0] = V;
            r->steps[4 * step + 1] = E;
            /* Steps 1-2: evaluate the pre-activation at every vertex, take its sign.
             * Genericity (Sec. 3.2, 3.4, 4.2.1): no old vertex lies on H. */
            if (capZ < V) { free(zv); capZ = capV; zv = (double *)malloc(sizeof(double) * (size_t)capZ); }
            int zero_hit = 0;
            double margin = r->min_margin;
#pragma omp parallel for num_threads(nth) schedule(static) reduction(min : margin) reduction(| : zero_hit)
            for (long v = 0; v < V; ++v) {
                double acc = 0.0;
                const double *h = Hm + v * nin;
                for (int k = 0; k < nin; ++k) acc += W[(long)i * nin + k] * h[k];
                double z = acc + b[mutation == 5 ? (i + 1) % nl : i];
                zv[v] = z;
                if (z == 0.0) { zero_hit = 1; continue; }
                if (fabs(z) < margin) margin = fabs(z);
                S[v * M + n] = z > 0.0 ? 1 : -1;
            }
            r->min_margin = margin;
            if (zero_hit) { status = PCXO_ERR_DEGENERATE; why = "vertex on a hyperplane (non-generic)"; break; }
            /* Step 3: splitting edges have endpoints of opposite sign, listed in
             * edge order (each thread takes one contiguous range of the edges,
             * counts its matches, then writes them after those of the ranges
             * before it) */
            long ns = 0;
            long cnt[nth + 1];
#pragma omp parallel num_threads(nth)
            {
                const int t = omp_get_thread_num(), nt = omp_get_num_threads();
                const long e0 = E * t / nt, e1 = E * (t + 1) / nt;
                long c = 0;
                for (long e = e0; e < e1; ++e)
                    c += S[(long)Ed[2 * e] * M + n] != S[(long)Ed[2 * e + 1] * M + n];
                cnt[t + 1] = c;
#pragma omp barrier
#pragma omp single
                {
                    cnt[0] = 0;
                    for (int k = 0; k < nt; ++k) cnt[k + 1] += cnt[k];
                    ns = cnt[nt];
                    if (ns > capSpl) {
                        capSpl = ns + ns / 2 + 1024;
                        spl = (int32_t *)xrealloc(spl, sizeof(int32_t) * (size_t)capSpl);
                    }
                }
                if (spl) {
                    long pos = cnt[t];
                    for (long e = e0; e < e1; ++e)
                        if (S[(long)Ed[2 * e] * M + n] != S[(long)Ed[2 * e + 1] * M + n]) spl[pos++] = (int32_t)e;
                }
            }
            if (ns > 0 && !spl) { status = PCXO_ERR_OOM; why = "oom"; break; }
            r->steps[4 * step + 2] = ns;
            /* grow vertex / edge storage */
            if (V + ns > capV) {
                long nc = capV; while (nc < V + ns) nc *= 2;
                X = (double *)xrealloc(X, sizeof(double) * (size_t)nc * D);
                S = (int8_t *)xrealloc(S, (size_t)nc * M);
                Hm = (double *)xrealloc(Hm, sizeof(double) * (size_t)nc * nin);
                if (!X || !S || !Hm) { status = PCXO_ERR_OOM; why = "oom"; break; }
                memset(S + (size_t)capV * M, 0, (size_t)(nc - capV) * M);
                capV = nc;
            }
            long maxE = E + ns + (long)(D > 1 ? D - 1 : 0) * ns;
            if (maxE > capE) {
                long nc = capE; while (nc < maxE) nc *= 2;
                Ed = (int32_t *)xrealloc(Ed, sizeof(int32_t) * (size_t)nc * 2);
                if (!Ed) { status = PCXO_ERR_OOM; why = "oom"; break; }
                capE = nc;
            }
            /* Step 4: the new vertex on each splitting edge, by linear interpolation
             * of V+ and V- weighted by their pre-activations; it takes sign 0 at H
             * and inherits the rest (join of the endpoints). The edge is replaced by
             * E+ and E-. */
            const long V0 = V, E0 = E;
            int conflict_hit = 0;
#pragma omp parallel for num_threads(nth) schedule(static) reduction(| : conflict_hit)
            for (long s = 0; s < ns; ++s) {
                long e = spl[s];
                int32_t a = Ed[2 * e], bq = Ed[2 * e + 1];
                int32_t p = zv[a] > 0.0 ? a : bq;   /* V+ */
                int32_t q = zv[a] > 0.0 ? bq : a;   /* V- */
                double zp = zv[p], zq = zv[q];
                double t = zp / (zp - zq);
                if (mutation == 2) t = 1.0 - t;
                long x0 = V0 + s;
                for (int j = 0; j < D; ++j) {
                    double xp = X[(long)p * D + j], xq = X[(long)q * D + j];
                    X[x0 * D + j] = xp + t * (xq - xp);
                }
                int conflict = 0;
                for (int k = 0; k < n; ++k) {
                    int sp = S[(long)p * M + k], sq = S[(long)q * M + k];
                    S[x0 * M + k] = (int8_t)(mutation == 4 ? sp : join_sign(sp, sq, &conflict));
                }
                S[x0 * M + n] = 0;
                for (int k = n + 1; k < M; ++k) S[x0 * M + k] = 0; /* set when those neurons are processed */
                if (conflict) { conflict_hit = 1; continue; }
                double *t1 = tmp + (size_t)maxw * 2 * (size_t)omp_get_thread_num();
                hidden_at(net, X + x0 * D, l - 1, Hm + x0 * nin, t1, t1 + maxw);
                Ed[2 * e] = a; Ed[2 * e + 1] = (int32_t)x0;          /* one half keeps the slot */
                Ed[2 * (E0 + s)] = (int32_t)x0; Ed[2 * (E0 + s) + 1] = bq; /* the other is appended */
            }
            if (conflict_hit) { status = PCXO_ERR_DEGENERATE; why = "sign conflict on an edge"; break; }
            V = V0 + ns; E = E0 + ns;
            /* Step 5 (Sec. 4.2.2): perturb each splitting edge to its parent 2-faces
             * (Sec. 4.1: every zero to + and -, boundary zeros only to +). Each
             * splitting 2-face comes up exactly twice; pair the two new vertices. */
            long nf = 0;
            long maxf = (long)2 * (D > 1 ? D - 1 : 0) * ns;
            if (maxf > capF) {
                capF = maxf;
                fvert = (int32_t *)xrealloc(fvert, sizeof(int32_t) * (size_t)capF);
                fidx = (int32_t *)xrealloc(fidx, sizeof(int32_t) * (size_t)capF);
                ftmp = (int32_t *)xrealloc(ftmp, sizeof(int32_t) * (size_t)capF);
                if (!fvert || !fidx || !ftmp) { status = PCXO_ERR_OOM; why = "oom"; break; }
            }
            if ((size_t)maxf * (size_t)n > capFB) {
                capFB = (size_t)maxf * (size_t)n;
                fkeys = (int8_t *)xrealloc(fkeys, capFB);
                if (!fkeys) { status = PCXO_ERR_OOM; why = "oom"; break; }
            }
            for (long s = 0; s < ns && status == PCXO_OK; ++s) {
                long x0 = V0 + s;
                /* sign-vector of the splitting edge over the entries before n is the
                 * new vertex's inherited part */
                const int8_t *se = S + x0 * M;
                int zeros = 0;
                for (int k = 0; k < n; ++k) if (se[k] == 0) ++zeros;
                if (zeros != D - 1) { status = PCXO_ERR_DEGENERATE; why = "edge without D-1 zeros"; break; }
                for (int k = 0; k < n; ++k) {
                    if (se[k] != 0) continue;
                    int box = k < m;  /* domain entries are perturbed only to + */
                    for (int sg = 1; sg >= -1; sg -= 2) {
                        if (box && sg < 0) continue;
                        if (mutation == 1 && sg < 0) continue;
                        int8_t *key = fkeys + nf * n;
                        memcpy(key, se, (size_t)n);
                        key[k] = (int8_t)sg;
                        fvert[nf] = (int32_t)x0;
                        fidx[nf] = (int32_t)nf;
                        ++nf;
                    }
                }
            }
            if (status != PCXO_OK) break;
            r->steps[4 * step + 3] = nf;
            if (nf > 0) {
                face_ctx c = { fkeys, n };
                merge_sort(fidx, ftmp, nf, &c);
                long k = 0;
                while (k < nf) {
                    long j = k + 1;
                    while (j < nf && face_cmp(&c, fidx[j], fidx[k]) == 0) ++j;
                    if (j - k != 2) {
                        status = PCXO_ERR_DEGENERATE; why = "2-face not shared by exactly two splitting edges"; break;
                    }
                    if (mutation != 3) {
                        Ed[2 * E] = fvert[fidx[k]];
                        Ed[2 * E + 1] = fvert[fidx[k + 1]];
                        ++E;
                    }
                    k = j;
                }
            }
        }
        entry_base += nl;
    }

    free(Hm); free(tmp); free(tmp2); free(zv); free(spl); free(fkeys); free(fvert); free(fidx); free(ftmp);
    r->V = V; r->E = E; r->X = X; r->S = S; r->edges = Ed;
    if (status != PCXO_OK) fail(r, status, why);
    r->n_steps = step < nsteps ? step : nsteps;
    return r;
}

/* The box [lo, hi]^D: entry 2j is x_j - lo_j >= 0, entry 2j+1 is hi_j - x_j >= 0.
 * Corner c has x_j = hi_j if bit j of c is set, else lo_j; corners at Hamming
 * distance one share an edge. */
pcxo_result *pcxo_extract(const pcxo_net *net, const double *lo, const double *hi,
                          int include_output, int prune, int mutation) {
    const int D = net->D;
    if (D < 1 || D > 20) {
        pcxo_result *r = (pcxo_result *)calloc(1, sizeof(pcxo_result));
        if (r) fail(r, PCXO_ERR_INVALID, "bad widths");
        return r;
    }
    for (int j = 0; j < D; ++j)
        if (!(lo[j] < hi[j])) {
            pcxo_result *r = (pcxo_result *)calloc(1, sizeof(pcxo_result));
            if (r) fail(r, PCXO_ERR_INVALID, "empty box");
            return r;
        }
    const long nv = 1L << D, ne = (long)D << (D - 1);
    const int m = 2 * D;
    double *X0 = (double *)malloc(sizeof(double) * (size_t)nv * D);
    int8_t *S0 = (int8_t *)malloc((size_t)nv * m);
    int32_t *E0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne * 2);
    pcxo_result *r = NULL;
    if (X0 && S0 && E0) {
        for (long c = 0; c < nv; ++c)
            for (int j = 0; j < D; ++j) {
                int up = (int)((c >> j) & 1);
                X0[c * D + j] = up ? hi[j] : lo[j];
                S0[c * m + 2 * j] = up ? 1 : 0;     /* x_j - lo_j */
                S0[c * m + 2 * j + 1] = up ? 0 : 1; /* hi_j - x_j */
            }
        long e = 0;
        for (int j = 0; j < D; ++j)
            for (long c = 0; c < nv; ++c)
                if (!((c >> j) & 1)) { E0[2 * e] = (int32_t)c; E0[2 * e + 1] = (int32_t)(c | (1L << j)); ++e; }
        r = extract_core(net, m, nv, X0, S0, ne, E0, include_output, prune, mutation);
    }
    free(X0); free(S0); free(E0);
    return r;
}

/* The simplex with corners P_0..P_D (rows of `corners`, affinely independent):
 * entry i is the barycentric coordinate of x for P_i, >= 0 inside (the facet
 * opposite P_i is its zero set). Corner i is + at entry i and 0 at the D
 * others; every pair of corners shares an edge, in order (0,1), (0,2), ...,
 * (D-1,D). */
pcxo_result *pcxo_extract_simplex(const pcxo_net *net, const double *corners, int include_output, int prune,
                                  int mutation) {
    const int D = net->D;
    if (D < 1 || D > 20) {
        pcxo_result *r = (pcxo_result *)calloc(1, sizeof(pcxo_result));
        if (r) fail(r, PCXO_ERR_INVALID, "bad widths");
        return r;
    }
    const long nv = D + 1, ne = (long)D * (D + 1) / 2;
    const int m = D + 1;
    int8_t *S0 = (int8_t *)calloc((size_t)nv * m, 1);
    int32_t *E0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)ne * 2);
    pcxo_result *r = NULL;
    if (S0 && E0) {
        for (long i = 0; i < nv; ++i) S0[i * m + i] = 1;
        long e = 0;
        for (int i = 0; i < nv; ++i)
            for (int j = i + 1; j < nv; ++j) { E0[2 * e] = i; E0[2 * e + 1] = j; ++e; }
        r = extract_core(net, m, nv, corners, S0, ne, E0, include_output, prune, mutation);
    }
    free(S0); free(E0);
    return r;
}

void pcxo_free(pcxo_result *r) {
    if (!r) return;
    free(r->X); free(r->S); free(r->edges); free(r->steps); free(r);
}

/* --------------------------------------------- vertex from its sign-vector
 *
 * A vertex is the transversal intersection of the D (folded) hyperplanes at
 * its zero entries (Sec. 3.3: a k-cell has D-k zeros). With the activation
 * pattern read off the sign-vector (zeros taken as inactive; either side gives
 * the same point, since the pre-activation is continuous across a fold), each
 * zero entry is an affine equation in x; solve the D x D system by Gaussian
 * elimination with partial pivoting. */
int pcxo_vertex_solve(const pcxo_net *net, int include_output, const double *lo, const double *hi,
                      const int8_t *sigma, double *x_out) {
    const int D = net->D;
    const int M = entry_count(net, include_output);
    const int nsub = n_sub_layers(net, include_output);
    int maxw = D;
    for (int l = 0; l <= net->L; ++l) if (net->widths[l] > maxw) maxw = net->widths[l];
    double *A = (double *)calloc((size_t)D * (D + 1), sizeof(double));
    /* affine maps of the current layer input: G [width][D], c [width] */
    double *G = (double *)calloc((size_t)maxw * D, sizeof(double));
    double *c = (double *)calloc((size_t)maxw, sizeof(double));
    double *Gn = (double *)calloc((size_t)maxw * D, sizeof(double));
    double *cn = (double *)calloc((size_t)maxw, sizeof(double));
    int rows = 0, status = PCXO_OK;
    if (!A || !G || !c || !Gn || !cn) { status = PCXO_ERR_OOM; goto done; }
    for (int j = 0; j < D; ++j) {
        if (sigma[2 * j] == 0 && rows < D) { A[rows * (D + 1) + j] = 1.0; A[rows * (D + 1) + D] = lo[j]; ++rows; }
        else if (sigma[2 * j] == 0) { status = PCXO_ERR_INVALID; goto done; }
        if (sigma[2 * j + 1] == 0 && rows < D) { A[rows * (D + 1) + j] = 1.0; A[rows * (D + 1) + D] = hi[j]; ++rows; }
        else if (sigma[2 * j + 1] == 0) { status = PCXO_ERR_INVALID; goto done; }
    }
    for (int j = 0; j < D; ++j) { G[j * D + j] = 1.0; c[j] = 0.0; }
    int base = 2 * D;
    for (int l = 1; l <= nsub; ++l) {
        int nin = net->widths[l - 1], nl = net->widths[l];
        const double *W = net->W[l - 1], *b = net->b[l - 1];
        for (int i = 0; i < nl; ++i) {
            for (int d = 0; d < D; ++d) {
                double acc = 0.0;
                for (int k = 0; k < nin; ++k) acc += W[(long)i * nin + k] * G[k * D + d];
                Gn[i * D + d] = acc;
            }
            double acc = 0.0;
            for (int k = 0; k < nin; ++k) acc += W[(long)i * nin + k] * c[k];
            cn[i] = acc + b[i];
            int s = sigma[base + i];
            if (s == 0) {
                if (rows >= D) { status = PCXO_ERR_INVALID; goto done; }
                for (int d = 0; d < D; ++d) A[rows * (D + 1) + d] = Gn[i * D + d];
                A[rows * (D + 1) + D] = -cn[i];
                ++rows;
            }
            if (s <= 0) { for (int d = 0; d < D; ++d) Gn[i * D + d] = 0.0; cn[i] = 0.0; }
        }
        double *t = G; G = Gn; Gn = t;
        t = c; c = cn; cn = t;
        base += nl;
    }
    if (base != M || rows != D) { status = PCXO_ERR_INVALID; goto done; }
    for (int col = 0; col < D; ++col) {
        int piv = col;
        for (int rr = col + 1; rr < D; ++rr)
            if (fabs(A[rr * (D + 1) + col]) > fabs(A[piv * (D + 1) + col])) piv = rr;
        if (A[piv * (D + 1) + col] == 0.0) { status = PCXO_ERR_SINGULAR; goto done; }
        if (piv != col)
            for (int k = 0; k <= D; ++k) { double t = A[col * (D + 1) + k]; A[col * (D + 1) + k] = A[piv * (D + 1) + k]; A[piv * (D + 1) + k] = t; }
        for (int rr = col + 1; rr < D; ++rr) {
            double f = A[rr * (D + 1) + col] / A[col * (D + 1) + col];
            for (int k = col; k <= D; ++k) A[rr * (D + 1) + k] -= f * A[col * (D + 1) + k];
        }
    }
    for (int rr = D - 1; rr >= 0; --rr) {
        double acc = A[rr * (D + 1) + D];
        for (int k = rr + 1; k < D; ++k) acc -= A[rr * (D + 1) + k] * x_out[k];
        x_out[rr] = acc / A[rr * (D + 1) + rr];
    }
done:
    free(A); free(G); free(c); free(Gn); free(cn);
    return status;
}

/* ---------------------------------------------- accessors for ctypes */
int pcxo_status(const pcxo_result *r) { return r->status; }
const char *pcxo_message(const pcxo_result *r) { return r->msg; }
long pcxo_V(const pcxo_result *r) { return r->V; }
long pcxo_E(const pcxo_result *r) { return r->E; }
int pcxo_M(const pcxo_result *r) { return r->M; }
int pcxo_n_steps(const pcxo_result *r) { return r->n_steps; }
double pcxo_min_margin(const pcxo_result *r) { return r->min_margin; }
void pcxo_copy(const pcxo_result *r, double *X, int8_t *S, int32_t *edges, long *steps) {
    if (X) memcpy(X, r->X, sizeof(double) * (size_t)r->V * r->D);
    if (S) memcpy(S, r->S, (size_t)r->V * r->M);
    if (edges) memcpy(edges, r->edges, sizeof(int32_t) * (size_t)r->E * 2);
    if (steps) memcpy(steps, r->steps, sizeof(long) * (size_t)r->n_steps * 4);
}
