// Descriptors of the persistent batched kernel (batch.hip) and its host side.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace pcx {

constexpr int kBatchMaxLayers = 8;  // affine layers per network in a batch
constexpr int kBatchMaxD = 8;       // input dimension in a batch
constexpr int kBatchMaxWords = 64;  // sign-row words per vertex in a batch

// BATCH_RETRY: the 2-face pairing failed in the batched kernel (a hash
// collision, or a degenerate face); the per-step path, whose exact pass tells
// the two apart, extracts the network instead
enum { BATCH_OK = 0, BATCH_OVERFLOW = 1, BATCH_POOL = 2, BATCH_DEGENERATE = 3, BATCH_INTERNAL = 4, BATCH_RETRY = 5 };

struct BatchNet {
    const double *Wt[kBatchMaxLayers];  // transposed weights, [N_{l-1}][N_l]
    const double *b[kBatchMaxLayers];
    int widths[kBatchMaxLayers + 1];
    int L, nsub, D;
    double lo[kBatchMaxD], hi[kBatchMaxD];
    StepRec *rec;  // per-step log of this network (null: not kept)
};

// schedule bits of a batched launch (0: 16 edges per thread in each step's
// compaction, 32 lanes per splitting edge; kSchedSplit16: 16 lanes per
// splitting edge in layers of up to 128 neurons). The schedules are the values
// 0 .. kSchedCount-1 (kSchedSplit64 and kSchedSplit16 exclude each other).
enum { kSchedSelect8 = 1, kSchedSplit64 = 2, kSchedSplit16 = 4, kSchedCount = 6 };
// the schedule of an untuned batch: 16 edges per thread, 16 lanes per split
constexpr int kSchedDefault = kSchedSplit16;
inline int sched_split_lanes(int sched) { return (sched & kSchedSplit64) ? 64 : (sched & kSchedSplit16) ? 16 : 32; }

struct BatchResult {
    int status, V, E, Wd;
    long long offV, offSG, offE;  // offsets into the output pool: doubles, sign words, edges
    long long splits, pairs;
};

struct BatchArgs {
    const BatchNet *nets;
    int n;
    const int *order;  // processing order (largest predicted network first)
    int *ticket;
    char *arena;       // one arena per workgroup
    size_t arena_bytes, vbytes;  // per workgroup; vbytes = vertex region
    int ecap, kcap;    // edges, 2-face key slots per workgroup
    uint32_t tcap;     // hash-table entries per workgroup
    double *oX;
    uint64_t *oSG;
    int2 *oE;
    unsigned long long *pool;  // used: [0] coordinate doubles, [1] sign words, [2] edges
    unsigned long long capV, capSG, capE;
    BatchResult *res;
    int hbits;         // bits of the 2-face hash kept (64; fewer only in tests)
    int verify;        // 1: compare the perturbed sign rows of every pair (pcx_opts.verify_pairs)
};

// bytes of one workgroup arena: vertex region + edges (10 B, and a 16-byte
// split-list entry per possible split: 32 B with alignment) + key slots
// (partner record 8 B, perturbed entry 4 B) + table (8 B words) + valid words
// + counters
inline size_t batch_arena_bytes(size_t vbytes, int ecap, int kcap, uint32_t tcap) {
    size_t k = (size_t)kcap * 12;
    k += 256 - k % 256;
    return vbytes + (size_t)ecap * 32 + k + (size_t)tcap * sizeof(unsigned long long) + kBatchMaxWords * 8 + 256;
}

void launch_batch(const BatchArgs &A, int grid, int sched, hipStream_t st);

}  // namespace pcx
