/*
 * pcx.h -- C ABI of the MI355X (gfx950) edge-subdivision library libpcx.so.
 *
 * Polyhedral complex extraction from ReLU networks by edge subdivision
 * (Berzins, ICML 2023). A continuous piecewise-affine ReLU MLP (Sec. 3.4:
 * x^(l) = ReLU(W^(l) x^(l-1) + b^(l))) and an input box in R^D go in; the
 * 1-skeleton of the polyhedral complex its folded hyperplanes induce on the
 * box comes out: vertex coordinates, packed sign-vectors (Sec. 3.3) and an edge
 * list. Every neuron of every hidden layer is processed in layer order with
 * the five steps of Sec. 4.2 (evaluate, sign, find splitting edges,
 * interpolate and split, connect new vertices sharing a 2-face).
 *
 * Conventions shared by every call
 *  - All floating point is IEEE binary64.
 *  - W^(l) is row-major [N_l][N_{l-1}] (z = W x + b); b^(l) is [N_l].
 *  - widths = {D, N_1, ..., N_{L-1}, N_L}; layers 1..L-1 are hidden (ReLU),
 *    layer L is the output. Hidden neurons are always subdivided; output
 *    neurons only with pcx_opts.include_output (their zero level set).
 *  - Sign-vector entries (Sec. 4.1): the 2D box half-spaces first, entry 2j
 *    is x_j - lo_j >= 0 and entry 2j+1 is hi_j - x_j >= 0 (interior cells are
 *    + there), then the subdivided neurons layer by layer in index order.
 *  - Sign-vector packing: 2 bits per entry, code 00 = 0, 01 = +, 10 = -
 *    (11 never occurs), so the join of two cells (Sec. 3.5) is a bitwise OR.
 *    A row is Wd uint64 words. Word 0 holds the box entries (entry e at bits
 *    2e, so D <= 16). Each subdivided layer starts on a fresh word: neuron i
 *    of subdivided layer l sits in word lw_l + (i >> 5), bits 2(i & 31),
 *    where lw_1 = 1 and lw_{l+1} = lw_l + ceil(N_l / 32). Unused bits are 0.
 *  - Errors: every int-returning call returns PCX_OK (0) or a negative code;
 *    pcx_last_error() gives a message for the calling thread. Inputs are
 *    copied during the call; no call keeps a caller pointer. Handles are owned
 *    by the library and released with the matching *_free call.
 *  - Device pointers are HIP device pointers on the current device.
 */
#ifndef PCX_H
#define PCX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCX_OK 0
#define PCX_PENDING 1
#define PCX_ERR_INVALID (-1)    /* bad argument: widths, box (lo >= hi), D outside 1..16, NULL */
#define PCX_ERR_OOM (-2)        /* device or host allocation failed */
#define PCX_ERR_DEGENERATE (-3) /* input not generic (Sec. 3.2, 3.4): a vertex on a hyperplane,
                                   or a splitting 2-face not met by exactly two splitting edges */
#define PCX_ERR_DEVICE (-4)     /* a HIP runtime call failed */
#define PCX_ERR_CAPACITY (-5)   /* result would exceed pcx_opts.max_bytes */

#define PCX_PAIR_HASH 0 /* open-addressing table on 64-bit 2-face hashes, linear time */
#define PCX_PAIR_SORT 1 /* LSD radix sort of 24-bit slices of the 2-face keys (the paper's sort, Sec. 5.1) */

typedef struct pcx_mlp pcx_mlp;
typedef struct pcx_complex pcx_complex;

/* Options of one extraction. A zeroed struct (or NULL) gives the defaults. */
typedef struct {
    int32_t include_output; /* 1: subdivide the output neurons too (zero level set, Sec. 5.4) */
    int32_t timing;         /* bit f set: time kernel family f (PCX_K_*) with HIP events on the stream */
    int32_t pairing;        /* step 5 grouping of 2-face keys: PCX_PAIR_HASH (default) or PCX_PAIR_SORT */
    int32_t record_tape;    /* 1: keep what pcx_backward needs (parents of new vertices, every layer's
                               pre-activations); costs V * N_l doubles per subdivided layer */
    uint64_t max_bytes;     /* cap on device bytes the extraction may hold; 0 = no cap */
    void *stream;           /* hipStream_t to run on; NULL = the default stream */
    int32_t batch_wg_per_cu;/* pcx_extract_batch: workgroups per compute unit; 0 = tuned / default */
    int32_t prune;          /* 1 (needs include_output; pcx_extract only, not with record_tape): pruning
                               during subdivision for level-set extraction (Sec. 5.4.2). Before each
                               subdivided layer, edges whose two vertices agree in sign on every neuron
                               still to come (the output included) are dropped, then vertices left
                               without edges; survivors keep their order. The result holds the whole
                               output level set and the cells pruning could not exclude; the per-step
                               counters show the pruned sizes at each layer start. */
    int32_t verify_pairs;   /* 1: with hash pairing, also compare the two perturbed sign rows of every
                               pair word by word (Sec. 4.2.2's exact grouping, checked row by row).
                               Without it a pair is exact for every generic input all the same: a
                               table entry reached by two different 2-faces gets four arrivals,
                               which the mutual-record check always catches (the step then goes
                               to the exact pass). The comparison only adds the detection of two
                               2-faces each met once (a non-generic input) whose hashes collide.
                               Sort pairing always compares rows. */
} pcx_opts;

/* Summary of an extracted complex. */
typedef struct {
    int64_t V;              /* vertices */
    int64_t E;              /* edges */
    int32_t D;              /* input dimension */
    int32_t M;              /* sign-vector entries: 2D + subdivided neurons */
    int32_t Wd;             /* uint64 words per packed sign-vector row */
    int32_t n_steps;        /* subdivided neurons (one step each) */
    int64_t total_splits;   /* sum over steps of splitting edges (= new vertices) */
    int64_t total_pairs;    /* sum over steps of intersecting edges (step 5) */
    uint64_t peak_bytes;    /* device bytes held at the peak of the extraction */
    double time_ms;         /* device time of the extraction (HIP events, weights resident) */
    int32_t exact_steps;    /* steps whose 2-face pairing was redone by the exact pass (a hash
                               collision, or a step with more than 2^29 - 2 key slots); the result
                               is the same complex either way */
    int32_t from_graph;     /* 1: a repeat of the network's last extraction (same box and options),
                               replayed from its captured HIP graph (the same complex) */
} pcx_info;

const char *pcx_last_error(void);

/* Copy a ReLU MLP to the device. widths has n_layers+1 entries (D first);
 * W[l] points to N_{l+1} x N_l doubles (row-major), b[l] to N_{l+1} doubles,
 * for l = 0 .. n_layers-1 (host pointers). Sec. 3.4 defines the network. */
int pcx_mlp_create(int32_t n_layers, const int32_t *widths, const double *const *W,
                   const double *const *b, pcx_mlp **out);
void pcx_mlp_free(pcx_mlp *mlp);

/* Edge subdivision of the box [lo, hi] (D host doubles each, lo < hi) by every
 * subdivided neuron of mlp, in layer order (Sec. 4.2); a subdivided layer may
 * have at most 256 neurons (else PCX_ERR_INVALID). On success *out owns
 * the complex on the device. On error *out is NULL. Work is queued on
 * opts->stream; the call returns when the complex is complete. A network keeps
 * the step log of its last extraction (hash pairing, no prune, tape, timing or
 * byte cap); its third request with the same box and options captures the
 * whole kernel sequence in a HIP graph (storage of its own, up to 512 MiB per
 * network and 4 GiB over all networks, held until pcx_mlp_free) and later ones
 * replay it (PCX_NO_GRAPH=1 in the environment turns this off). A replay whose
 * steps differ from the log is discarded and the ordinary path runs. A capture
 * waits for no other call: while another thread of the process is inside a
 * device allocation or free of this library it is skipped until a later
 * request. A network whose predicted complex is small (at most 15000 vertices
 * for D <= 2, 3500 for D = 3; never for D >= 4) runs as a batch of one instead
 * (one launch of the batched kernel, the same complex; PCX_NO_TINY=1 turns
 * this off, PCX_TINY_VERTICES sets the threshold for every D). */
int pcx_extract(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts *opts,
                pcx_complex **out);

/* The same on the simplex with corners P_0..P_D: `corners` holds (D+1) x D host
 * doubles, row i = P_i, affinely independent (else PCX_ERR_INVALID). The
 * domain is given by m = D + 1 half-spaces (Sec. 4.1; the simplex domain is the
 * paper's remedy for the 2^D corners of the hypercube, Sec. 5.2): sign entry i
 * is the barycentric coordinate of P_i, + inside, 0 on the facet opposite P_i.
 * These D + 1 entries take word 0 (entry i at bits 2i); the layers follow as
 * for the box. Initial skeleton: corner i is vertex i, edges (i, j) for i < j in
 * lexicographic order. Vertices on a facet lie on it up to rounding (their
 * zero entries are exact in the sign-vector). Every option of pcx_extract
 * applies (pruning, tape, pairing). */
int pcx_extract_simplex(const pcx_mlp *mlp, const double *corners, const pcx_opts *opts, pcx_complex **out);

/* Higher cells by repeated perturbation (Sec. 4.1): the parents of a k-cell come
 * from perturbing each zero of its sign-vector to + and - (domain zeros only to
 * +), starting from the edges (sign-vector of an edge = join of its vertices',
 * Sec. 3.5). counts (host, D + 1 entries) receives the f-vector: counts[k] =
 * number of k-cells, counts[0] = V, counts[1] = E, counts[D] = regions. For a
 * complex on a ball-shaped domain the alternating sum is 1 (Euler). Distinct
 * cells are told apart by a 128-bit hash of their sign-vector; two cells with
 * equal first 64 bits but different second halves give PCX_ERR_DEVICE. Runs on
 * `stream` and returns when done; temporary device memory is released. A
 * complex extracted with pcx_opts.prune is a sub-complex: PCX_ERR_INVALID. */
int pcx_cell_counts(const pcx_complex *cx, int64_t *counts, void *stream);

/* Sign-vectors of all regions (D-cells), packed like the vertex rows (Wd words
 * each, host memory), sorted lexicographically by word. *n receives the count;
 * with rows == NULL only the count is computed. */
int pcx_regions(const pcx_complex *cx, uint64_t *rows, int64_t *n, void *stream);

int pcx_complex_info(const pcx_complex *cx, pcx_info *info);

/* Per-step counters, n_steps rows of 4 int64 (host buffer): vertices and
 * edges before the step, splitting edges, and 2-face records (Sec. 4.2.2). */
int pcx_complex_steps(const pcx_complex *cx, int64_t *steps);

/* Copy the complex to caller-allocated host buffers (any may be NULL):
 * coords V*D doubles, signs V*Wd uint64 (packing above), edges E*2 int32. */
int pcx_complex_copy(const pcx_complex *cx, double *coords, uint64_t *signs, int32_t *edges);

/* The same copy into caller-allocated device buffers (any may be NULL), e.g.
 * the storage of framework tensors; ordered on `stream` (NULL = default). */
int pcx_complex_copy_device(const pcx_complex *cx, double *coords, uint64_t *signs, int32_t *edges, void *stream);

/* Borrowed device pointers to the same three arrays, valid until
 * pcx_complex_free. Any out-pointer may be NULL. */
int pcx_complex_device(const pcx_complex *cx, void **coords, void **signs, void **edges);

/* Kernel-family device time in milliseconds accumulated during an extraction
 * run with bit `family` of opts.timing set: family is one of the PCX_K_* values below;
 * *launches receives the number of launches timed. PCX_K_SPLIT launches record
 * their own start and end events (kernel time only); the other families are
 * timed between event markers around their launches. Each timed launch adds a
 * few microseconds of stream time. */
#define PCX_K_GEMM 0     /* per-layer pre-activation evaluation (step 1) */
#define PCX_K_NEXT 1     /* per-layer first-crossing scan of every edge (steps 2-3) */
#define PCX_K_SELECT 2   /* per-step splitting-edge compaction (step 3) */
#define PCX_K_SPLIT 3    /* per-step interpolation, split, 2-face keys (steps 4-5) */
#define PCX_K_SORT 4     /* per-step radix sort of 2-face keys (step 5, PCX_PAIR_SORT) */
#define PCX_K_PAIR 5     /* per-step pairing into intersecting edges (step 5; with PCX_PAIR_HASH the
                            table inserts run inside PCX_K_SPLIT) */
#define PCX_K_COUNT 6
#define PCX_K_ALL ((1 << PCX_K_COUNT) - 1)
int pcx_complex_kernel_time(const pcx_complex *cx, int32_t family, double *ms, int64_t *launches);

void pcx_complex_free(pcx_complex *cx);

/* ---- Batched extraction: many networks in one persistent launch ----------
 * Each network is extracted exactly as pcx_extract would (same vertex and edge
 * numbering, bit-identical values); a workgroup runs one network at a time
 * from a largest-first queue. Networks that exceed the batched kernel's limits
 * (D > 8, more than 8 layers, a layer wider than 256, or a predicted complex
 * above 65536 vertices), or its per-workgroup arena, and networks whose
 * 2-face pairing failed inside the kernel (a hash collision: the per-step path
 * has the exact pass) are extracted on the per-step path inside the same call.
 * mlps[i] and the boxes lo/hi (the D_i
 * coordinates of network i, concatenated over i; host memory) are read during
 * the call. opts->include_output applies to every network. */
typedef struct pcx_batch pcx_batch;
typedef struct {
    int64_t n, total_V, total_E, total_splits;
    int32_t fallbacks;      /* networks extracted on the per-step path */
    int32_t degenerate;     /* networks rejected as non-generic */
    int32_t workgroups, wg_per_cu;
    double kernel_ms;       /* device time of the persistent launch */
    double time_ms;         /* host wall time of the whole call */
    int32_t split_lanes;    /* schedule of the launch: lanes per splitting edge (16, 32 or 64;
                             * 16 applies to layers of up to 128 neurons, 32 to wider ones) */
    int32_t select_items;   /*   and edges per thread in each step's compaction (16 or 8) */
} pcx_batch_stats;
int pcx_extract_batch(int32_t n, const pcx_mlp *const *mlps, const double *lo, const double *hi,
                      const pcx_opts *opts, pcx_batch **out);
/* Per-network info / copy; PCX_ERR_DEGENERATE for a non-generic network. */
int pcx_batch_info(const pcx_batch *bt, int32_t i, pcx_info *info);
int pcx_batch_copy(const pcx_batch *bt, int32_t i, double *coords, uint64_t *signs, int32_t *edges);
/* Per-step counters of network i (as pcx_complex_steps: n_steps rows of 4 int64, host);
 * they stay on the device until asked for. */
int pcx_batch_steps(const pcx_batch *bt, int32_t i, int64_t *steps);
int pcx_batch_summary(const pcx_batch *bt, pcx_batch_stats *stats);
void pcx_batch_free(pcx_batch *bt);
/* Autotuner: times the batch's persistent launch under each of six schedules
 * (lanes per splitting edge 16, 32 or 64; edges per thread in each step's
 * compaction 16 or 8) at 2 workgroups per compute unit, then 1 and 4 workgroups per compute
 * unit under the best schedule (best of two launches each), and keeps the
 * fastest for batches with the same size signature (the sorted subdivided-
 * neuron counts and input dimensions of the batched networks); later
 * pcx_extract_batch calls of that signature use it (batch_wg_per_cu > 0 still
 * overrides the occupancy). result (may be NULL) receives the choice. */
typedef struct {
    int32_t wg_per_cu, split_lanes, select_items;
    int32_t candidates;     /* launches configurations timed */
    double ms_default;      /* kernel time with the default schedule: 2 per CU, 16 lanes, 16 edges */
    double ms_best;         /* kernel time with the chosen one */
} pcx_batch_tuning;
int pcx_batch_tune(int32_t n, const pcx_mlp *const *mlps, const double *lo, const double *hi,
                   const pcx_opts *opts, pcx_batch_tuning *result);

/* ---- Extraction server: continuous batching of requests -------------------
 * Requests are queued in arrival order and admitted in that order while the
 * predicted device memory of admitted, unfinished jobs fits mem_budget (a job
 * is always admitted onto an idle GPU). Small networks (predicted complex of
 * at most small_vertices vertices) are gathered into back-to-back ticks of the
 * batched kernel; whatever arrives during a tick joins the next one. Larger
 * networks run on the per-step path in large_workers threads, each on its own
 * stream, overlapping with the ticks; so does a small network that would be
 * alone in its tick while a worker is free. A result is exactly the complex
 * pcx_extract returns for the same request. The server keeps the pcx_mlp
 * handle of a request until that request is released: the caller must not
 * free it before. Latency = completion - submission (host steady clock). */
typedef struct pcx_server pcx_server;
typedef struct {
    uint64_t mem_budget;    /* bytes of predicted device memory in flight; 0 = 64 GiB */
    int32_t max_batch;      /* jobs per tick; 0 = 4096 */
    int32_t large_workers;  /* concurrent per-step extractions; 0 = 6 */
    int32_t include_output; /* as pcx_opts.include_output, for every request */
    int32_t small_vertices; /* batched-kernel threshold on the predicted vertex count; 0 = 65536 */
} pcx_server_opts;
typedef struct {
    int32_t status;         /* PCX_PENDING, PCX_OK or the error of the request */
    int32_t batched;        /* 1: ran in a batched tick, 0: on the per-step path */
    int64_t V, E, total_splits;
    double latency_ms, queue_ms;  /* submission to completion / to admission */
    int32_t D, Wd;          /* row sizes of the result: pcx_server_copy writes V*D doubles,
                               V*Wd sign words (output word included with include_output), E*2 ints */
} pcx_server_result;
typedef struct {
    int64_t completed;
    double p50_ms, p99_ms, mean_ms, p50_queue_ms, p99_queue_ms;
    double span_s;          /* first submission to last completion */
    double jobs_per_s, splits_per_s, vertices_per_s;
    int64_t ticks;
    double mean_tick_jobs;
} pcx_server_summary;
int pcx_server_create(const pcx_server_opts *opts, pcx_server **out);
int pcx_server_submit(pcx_server *s, const pcx_mlp *mlp, const double *lo, const double *hi, uint64_t *ticket);
/* PCX_PENDING while the request runs; PCX_OK once *r holds its outcome. */
int pcx_server_poll(pcx_server *s, uint64_t ticket, pcx_server_result *r);
int pcx_server_wait(pcx_server *s, uint64_t ticket, pcx_server_result *r);
/* Copy a finished request's complex to host buffers (as pcx_complex_copy). */
int pcx_server_copy(pcx_server *s, uint64_t ticket, double *coords, uint64_t *signs, int32_t *edges);
/* Free a finished request's result (and drop the server's use of its mlp). */
int pcx_server_release(pcx_server *s, uint64_t ticket);
int pcx_server_stats(pcx_server *s, pcx_server_summary *stats);
/* Waits for every submitted request, then stops the server's threads. */
void pcx_server_destroy(pcx_server *s);

/* For callers that cannot allocate device memory (code under HIP graph capture
 * elsewhere in the process, tight serving loops, harnesses that forbid
 * hipMalloc): the extraction of pcx_extract, written into caller-allocated
 * device buffers. Every other array the kernels use comes from a static device
 * scratch of 256 MiB that each GPU the library runs on holds until the process
 * ends; no device or pinned memory is allocated and no HIP event or stream is
 * created. coords: max_vertices * D doubles; signs: max_vertices * Wd words
 * (packing above); edges: max_edges * 2 int32 (all device memory). On success
 * *info (host) receives the summary (peak_bytes = scratch bytes used, time_ms =
 * host wall time) and steps (host, n_steps rows of 4 int64 as in
 * pcx_complex_steps; may be NULL) the per-step counters; the first V rows of
 * coords / signs and E rows of edges hold the complex, equal to what
 * pcx_extract returns (same numbering). Errors: PCX_ERR_CAPACITY when the
 * complex exceeds max_vertices or max_edges (nothing can grow), or when the
 * scratch these maxima need exceeds 256 MiB (the message gives the bytes);
 * PCX_ERR_INVALID for prune, record_tape, sort pairing, more than 32
 * subdivided layers or 128 sign words. The scratch keeps the last call's
 * contents: calls that overlap on one GPU race, so callers serialize them. */
int pcx_extract_into(const pcx_mlp *mlp, const double *lo, const double *hi, const pcx_opts *opts, double *coords,
                     uint64_t *signs, int32_t *edges, int64_t max_vertices, int64_t max_edges, pcx_info *info,
                     int64_t *steps);

/* Gradient of a loss L(coordinates) with respect to every weight and bias,
 * through the vertex positions (Sec. 5.3: a loss on the extracted complex is
 * optimised through its vertices). cx must come from pcx_extract of the same
 * mlp with opts.record_tape = 1. grad_coords: device, V*D doubles, dL/dx for
 * every vertex in the complex's order. gW[l], gb[l]: device buffers of
 * N_{l+1} x N_l and N_{l+1} doubles for l = 0 .. n_layers-1, overwritten
 * (layers whose neurons were not subdivided get zeros). precision selects the
 * arithmetic of the reverse pass: PCX_F64 or PCX_F32 (results still FP64).
 * Each new vertex x0 = x_p + t (x_q - x_p), t = z_p / (z_p - z_q) of its
 * splitting edge (Sec. 4.2.1) is differentiated exactly as the forward pass
 * computed it; every vertex sums its children's contributions in child order
 * (no atomics), so the gradients are bit-identical from run to run. The call
 * returns when the gradients are complete. */
#define PCX_F64 0
#define PCX_F32 1
int pcx_backward(const pcx_mlp *mlp, const pcx_complex *cx, const double *grad_coords, double *const *gW,
                 double *const *gb, int32_t precision, void *stream);

/* Device blocks of finished extractions (scratch and freed complexes) are kept
 * by the library for reuse by later extractions on the same device. This call
 * returns every cached block of the current device to the HIP runtime. A
 * failed allocation also trims the cache and retries once. */
void pcx_cache_trim(void);

#ifdef __cplusplus
}
#endif
#endif /* PCX_H */
