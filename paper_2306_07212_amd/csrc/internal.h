// Internal declarations shared by the kernels and the host orchestrator of
// libpcx.so. Not part of the public ABI (include/pcx.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcx {

constexpr int kThreads = 256;            // every kernel uses 256-thread workgroups (4 waves)
constexpr int kSelItems = 16;            // edges per thread in the compaction scan
constexpr int kSelTile = kThreads * kSelItems;
constexpr int kScanItems = 32;           // one-byte first crossings per thread in the per-step compaction
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kSelBlocks = 1024;         // largest grid of the per-step compaction and hash pairing
constexpr int kNextBlocks = 8192;        // most chunks of the layer-start scan (its compaction included)
constexpr int kSortItems = 8;            // keys per thread in a radix-sort tile
constexpr int kSortTile = kThreads * kSortItems;
constexpr int kSortBins = 256;           // 8-bit digits
constexpr int kSortPasses = 3;           // over the low 24 key bits: valid keys < 2^24 - 1, the sentinel's all set
constexpr uint32_t kSentinel = 0xFFFFFFFFu;  // key of an unused 2-face slot (valid keys < 2^24 - 1)
constexpr uint16_t kNone = 0xFFFF;       // "no further crossing in this layer"
constexpr int kGemmRows = 32;            // vertices per GEMM workgroup
constexpr int kGemmK = 16;               // K-chunk staged in LDS
constexpr int kMaxWidth = 256;           // widest layer the in-place GEMM handles

// device counters (int32 slots of one small array). The vertex and edge counts
// and the table fill come in two slots, by the parity of the neuron step: step
// s reads slot s & 1 and its last kernels write slot (s + 1) & 1, so no kernel
// overwrites a count that another workgroup of the same launch still reads.
enum {
    CTR_S = 0,       // splitting edges of the current step (the compaction's result)
    CTR_KVALID = 1,  // valid 2-face keys (sort pairing)
    CTR_FLAGS = 3,   // FLAG_* bits; every per-step kernel returns at once while any is set
    CTR_FAIL = 4,    // first step that found the storage too small (FLAG_CAPACITY)
    CTR_SMAX = 5,    // largest split count so far in the layer (shapes the split launches)
    CTR_PFLAGS = 6,  // pairing failures (FLAG_RUN, FLAG_VERIFY, FLAG_BIGSTEP): the host redoes that
                     // step's pairing exactly; only a failure of the exact pass is an error
    CTR_PFAIL = 7,   // first step whose pairing failed (INT_MAX: none); kernels of later steps return
                     // at once, so the failed step's own split always completes
    CTR_V = 8,       // [2] vertex count at the start of a step
    CTR_E = 10,      // [2] edge count at the start of a step
    CTR_TUSED = 12,  // [2] hash-table entries a step used (cleared by the next step)
    CTR_COUNT = 16
};

// degeneracy / failure flags (bitwise)
enum : int {
    FLAG_ZERO_SIGN = 1,   // a pre-activation exactly 0 at a vertex where the neuron is not zero by construction
    FLAG_CONFLICT = 2,    // +/- conflict in the join of a splitting edge's endpoints
    FLAG_ZERO_COUNT = 4,  // splitting edge without exactly D-1 zeros
    FLAG_RUN = 8,         // a 2-face key met by other than exactly two splitting edges
    FLAG_VERIFY = 16,     // equal hashes but different exact 2-face sign-vectors
    FLAG_BOUNDS = 32,     // an index outside the live arrays (internal error; the access is skipped)
    FLAG_CAPACITY = 64,   // a step needs more storage than allocated: nothing written, the host grows and redoes it
    FLAG_BIGSTEP = 128,   // a step with more 2-face key slots than a table word can name (exact pass instead)
};
constexpr int kPairFlags = FLAG_RUN | FLAG_VERIFY | FLAG_BIGSTEP;

// One 64-bit word of the 2-face hash table per splitting 2-face; 0 = empty.
// The first splitting edge to reach a face claims a word with one CAS that
// publishes its key and its key slot together: bits 63..24 = 40 bits of the
// face hash, bits 23..0 = 1 + the key slot. The second arrival finds its
// partner's slot in the value its own CAS returns.
constexpr int kSlotBits = 24;                              // narrowest slot field of a table word
constexpr uint32_t kMaxHashSlots = (1u << 29) - 2;         // key slots a step may have on the table path
// Width of the slot field of a step's table words (the key takes the other
// bits): at least kSlotBits, and enough to name n slots plus the empty value.
__host__ __device__ inline int slot_bits(int n) {
    int b = kSlotBits;
    while ((1ll << b) < (long long)n + 2) ++b;
    return b;
}
// Partner record of a key slot, written by the second arrival at its 2-face
// (or by the exact pass) for both slots of the pair: high 32 bits = 1 + the
// step that wrote it, low 32 bits = 1 + the other slot. The pair's owner is
// its smaller slot.
constexpr uint32_t kNoInfo = 0xFFFFFFFFu;  // PINFO of an unused key slot
constexpr int kPairItems = 4;  // hash pairing: chunk granularity of the passes, key slots per thread in the batched kernel

enum { PAIR_HASH = 0, PAIR_SORT = 1 };

// Geometry of one neuron step (layer l, neuron j of that layer).
struct StepGeom {
    int D, Wd, ZS;   // input dim, words per sign row, pre-activation row stride
    int Nl;          // width of the layer being subdivided
    int lw0, lw1;    // first word of this layer's entries, first word of the next layer
    int j;           // neuron within the layer
    int wn, bn;      // word and bit offset of this neuron's entry
    int P;           // 2-face key slots per split: 2(D-1)
    int zlo;         // first pre-activation column carried to new vertices: 0, or j + 1 in the
                     // last subdivided layer (no later evaluation reads the processed columns)
    int pair_mode;   // PAIR_HASH or PAIR_SORT
    uint32_t hmask;  // hash table words - 1 (PAIR_HASH); the per-step kernels derive it from the split count
    unsigned long long *HT;   // this step's hash table (PAIR_HASH)
    unsigned long long *HTo;  // the previous step's table, cleared by this step's pairing
    int step, par;   // global neuron step and its parity (selects the CTR_V / CTR_E / CTR_TUSED slot)
    int nx8;         // 1: first crossings go to NX8 (per-step path); 0: to NXT (batched kernel)
    int Vcap, Ecap, Kcap;  // storage the step may fill (else FLAG_CAPACITY)
    uint64_t hkeep;  // mask of the 2-face hash bits kept (all; fewer only to test the exact pass)
    int fbits;       // bits of the exact pass's sort key kept (64; fewer only to test its grouping)
    int verify;      // 1: also compare the two perturbed sign rows of every hash-table pair word by word
    int sbits;       // slot field width of this step's table words (slot_bits of its key slots)
};

// Log of one neuron step, written by its last kernel: counts at its start, its
// split count, and the edge count after it.
struct StepRec {
    int V0, E0, S, E1;
};

struct Bufs {
    double *X;        // [Vcap][D]
    uint64_t *SG;     // [Vcap][Wd]
    double *Z;        // [Vcap][ZS]
    int2 *EDG;        // [Ecap]
    uint16_t *NXT;    // [Ecap] first crossing in the layer, kNone if none (batched kernel)
    uint8_t *NX8;     // [Ecap] the same on the per-step path: 1..255, 0 = none (the layer's first
                      // neuron is never looked up: its splitting edges come from the layer-start scan)
    int *SPL;         // [Scap] split list (batched kernel)
    int4 *SPLE;       // [Scap] split list: (edge, its two endpoints, 0)
    int *SPLX;        // [Ecap] per-chunk match lists of the compaction (chunk c at its own edge range)
    uint32_t *K32a, *K32b, *VALa, *VALb;  // [Kcap] radix-sort ping-pong
    uint64_t *FULL;   // [Kcap] full 64-bit 2-face hash by slot (sort pairing)
    uint32_t *PINFO;  // [Kcap] perturbed entry of the slot: word << 8 | bit << 1 | minus; kNoInfo if unused
    uint64_t *PART;   // [Kcap] partner record of each key slot (hash pairing and the exact pass)
    uint64_t *K64a, *K64b;  // [Kcap] exact pass: 64-bit sort keys (ping-pong; VALa / VALb carry the slots)
    uint32_t *HIST;   // [256 * tiles]
    int *SELCNT;      // [kNextBlocks] per-chunk match counts of the compaction (also the pairing passes)
    int *CTR;         // [CTR_COUNT]
    const uint64_t *VALID;  // [Wd] 01-pattern at every valid entry
    int2 *PQ;         // [Vcap] (V+, V-) parents of each new vertex, when the tape is recorded (else null)
    StepRec *REC;     // [n_steps] per-step log (per-step path only; null in the batched kernel)
    uint64_t *LW;     // [V][8] the evaluated layer's sign words again, in 64-byte rows, for the
                      // layer-start scan (written by the evaluation when set; else null)
};

// launchers (kernels.hip)
void launch_init_box(const Bufs &b, int D, int Wd, const double *lo, const double *hi, hipStream_t st);
void launch_gemm(const Bufs &b, int ZS, const double *in, int in_stride, int relu, int V, int K, int N,
                 const double *Wt, const double *bias, int Wd, int lw0, hipStream_t st);
// first crossing of every edge in the layer (NX8; the edge count comes from
// CTR_E[par]), and the ordered compaction of the edges that cross the layer's
// first neuron (the first pass of that step's split list: SPLX, SELCNT)
// (every per-step kernel takes its global step: it returns at once while a hard
// failure is flagged or a pairing failure of an earlier step is recorded)
void launch_next_all(const Bufs &b, int V, int Wd, int lw0, int lw1, int E, int par, int step, hipStream_t st);
// the compaction's second pass alone, after launch_next_all over the same E edges
void launch_gather(const Bufs &b, int E, int par, int step, hipStream_t st);
// splitting edges of neuron `target` from the CTR_E[par] edges: SPL, CTR_S
void launch_select(const Bufs &b, uint16_t target, int par, int step, int grid, hipStream_t st);
// grids (<= kSelBlocks) of the per-step compaction and hash pairing for an
// expected edge count / key-slot count: small steps take fewer workgroups
int select_grid(int64_t edges);
int pair_grid(int64_t slots);
// V0, E0 and S come from the device counters of step g.step; `blocks` only
// shapes the launch (the kernel strides over any S). The split also writes the
// next step's vertex count.
// t0 / t1: events the launch records at the kernel's start and end (null: none)
void launch_split(const Bufs &b, const StepGeom &g, int blocks, hipStream_t st, hipEvent_t t0 = nullptr,
                  hipEvent_t t1 = nullptr);
int split_blocks(int S_hint, int Nl);
// pruning during subdivision (prune.hip): kept edges -> out (count in CTR_E[par]), their endpoints marked;
// then marked vertices numbered in order (count in CTR_V[par]); then rows moved and edges renumbered
void launch_prune_edges(const Bufs &b, int V, int E, int Wd, int lwf, int2 *out, uint8_t *mark, int par,
                        hipStream_t st);
void launch_prune_vertices(const Bufs &b, int V, const uint8_t *mark, int *map, int par, hipStream_t st);
void launch_move_rows(const Bufs &b, const uint8_t *mark, const int *map, int V, int D, int Wd, int ZS, double *X2,
                      uint64_t *SG2, double *Z2, int2 *E2, int Enew, hipStream_t st);
// result: *keys / *vals (K32a/VALa or K32b/VALb, by the pass count)
void launch_sort(const Bufs &b, int n, hipStream_t st, const uint32_t **keys, const uint32_t **vals);
// the same over 64-bit keys K64a / K64b, all bits (the exact pass)
void launch_sort64(const Bufs &b, int n, hipStream_t st, const uint64_t **keys, const uint32_t **vals);
// sort pairing (host-known counts): edges from E1 on, the edge count after the step into CTR_E[par ^ 1]
void launch_pair(const Bufs &b, const StepGeom &g, int V0, int E1, int nslots, const uint32_t *keys,
                 const uint32_t *vals, hipStream_t st);
// hash pairing (the split recorded the pairs): a check and count pass over the
// key slots, then the ordered emit, all counts from the device; the emit also
// clears the previous step's table (g.HTo), writes the next step's edge count
// and the step's log entry
void launch_hash_pair(const Bufs &b, const StepGeom &g, int grid, hipStream_t st);
// the exact pass of one step's pairing (after a pairing failure): every valid
// key slot's 2-face sign-vector is rebuilt from its new vertex's row, sorted by
// a 64-bit hash, and grouped by exact comparison of the rows; the pairs are
// recorded as the table path records them and emitted by launch_hash_pair
// with the same grid. It needs K64a/K64b, VALa/VALb and HIST for nslots keys.
void launch_exact_pair(const Bufs &b, const StepGeom &g, int nslots, int grid, hipStream_t st);
// fill n 64-bit words with v (a kernel, so that no memset node enters a captured graph)
void launch_fill64(uint64_t *p, size_t n, uint64_t v, hipStream_t st);
// the device counters at the start of an extraction from V0 vertices and E0 edges
void launch_ctr_init(int *ctr, int V0, int E0, hipStream_t st);

// backward (backward.hip)
template <typename T>
void bwd_init(const double *grad, T *gx, size_t n, T *gz, size_t nz, hipStream_t st);
// the creation graph's (parent, child, side) records of the new vertices Vb .. V-1, unsorted
void bwd_records(const int2 *PQ, int Vb, int V, uint64_t *keys, int *flag, hipStream_t st);
// pos[vals[i]] = i: where each record sits after the sort
void bwd_pos(const uint32_t *vals, int n, int *pos, hipStream_t st);
// one step in reverse: each child's t and dL/dt, then each parent sums its children (in order)
template <typename T>
void bwd_step(const double *X, const double *Zs, const int2 *PQ, T *gx, T *gz, int D, int N, int ZS, int j, int Vb,
              int V0, int S, const uint64_t *skey, int nrec, const int *pos, double *tt, T *gtt, int *flag,
              hipStream_t st);
template <typename T>
void bwd_layer(const T *gz, int ZS, const double *hin, int hstride, int relu, int Vs, int N, int K, const double *W,
               double *part, int chunks, double *gW, double *gb, T *gzp, int ZSp, hipStream_t st);

}  // namespace pcx
