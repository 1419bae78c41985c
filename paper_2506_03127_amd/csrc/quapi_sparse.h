// Host/device interface of the hash-table merge (masks whose merge positions
// are not a contiguous run 0..L-1): argument block and launcher.
#pragma once

#include "quapi_host.h"

namespace quapi_dev {

// Groups are full histories of one or two 64-bit words (point j at bits
// [BP*j, BP*j+BP) of the number, the newest point lowest) in no particular
// order, merged through an open-addressing hash table keyed on the gathered
// merge positions.
constexpr int kSparseThreads = 256;
constexpr unsigned long long kMinTable = 1024;   // smallest table a step uses (slots)

// The stored groups of a step sit in kSegs segments of seg_cap groups each, one
// counter per segment: a workgroup of the merge writes to segment
// blockIdx.x % kSegs, so that the counter updates that place merged groups are
// spread over kSegs addresses (updates to one address serialise).  A step
// reads its input as one sequence, segment after segment.
constexpr int kSegs = 64;
constexpr int kSegStride = 64;                   // counters 256 bytes apart

__host__ __device__ inline int seg_counter(int parity, int s) { return (parity * kSegs + s) * kSegStride; }

// Partition merge (QUAPI_MERGE_PARTITION): in place of the table, the merged
// slots of each expand pass are appended to partitions chosen by the hash of
// their key (one counter increment per slot), and a second kernel merges each
// partition in an LDS table and writes its groups.  A step uses about one
// partition per kPartLoad children of its input, each holding at most
// kPartCap entries.
constexpr unsigned int kPartCap = 768;
constexpr unsigned int kPartLoad = 512;
constexpr int kPartLds = 1024;                   // LDS table slots of the partition merge

// One hash-table slot.  key holds the merge key plus one, so that an all-zero
// slot is free.  best is the largest "representative word" of the key's
// children: in the packed form the quantised |w|^2 above the complement of the
// child's points at the other positions (the largest word is then the largest
// quantised |w|^2 and, among those, the smallest history); otherwise the
// quantised |w|^2 alone, with the history settled by a second pass.
struct __align__(32) SpSlot {
    unsigned long long key;
    unsigned long long best;
    double wr, wi;                  // sum of the key's child weights
};

// One entry of a partition: the merge key and the representative word (packed
// form: the word itself; unpacked form: the key, the other points and the
// quantised |w|^2 >> qbits side by side as one 128-bit number where they fit,
// else the key and the quantised |w|^2, the other points in an array of their
// own), and the weight sum.
struct __align__(32) PartRec {
    unsigned long long x, y;
    double wr, wi;
};

struct SparseArgs {
    const uint64_t* h_in;           // [kSegs * seg_cap * hw] stored groups (state at t-1)
    const double2* w_in;            // FP64 form: amplitudes
    uint64_t* h_out;                // [kSegs * seg_cap * hw] groups after step t
    double2* w_out;
    const float2* wf_in;            // FP32 precision form: (ln|w|, arg w)
    float2* wf_out;
    int hw;                         // 64-bit words per history (1 or 2)
    unsigned int* count;            // [seg_counter(2, 0)] stored groups per segment, by parity of the time step
    unsigned long long seg_cap;     // groups per segment
    SpSlot* slot;                   // [tsize] the table, all zero between steps
    unsigned long long tsize;       // allocated slots (a power of two >= kMinTable)
    unsigned long long* tN;         // [tsize] unpacked form: smallest other points at the best q, ~0 when free
    unsigned int* cslot;            // [cap * P] unpacked form: table slot of each child, ~0u if filtered
    unsigned long long* cN;         // [cap * P] unpacked form: its points at the other positions
    unsigned long long* cq;         // [cap * P] unpacked form: its quantised |w|^2
    long long cap;                  // group capacity (all segments together)
    int P, K, t;
    double theta2;
    int qbits;                      // low bits of |w|^2 cleared by the quantisation
    int packed;                     // 1: representative word packs the other positions
    const double* tables;
    const double* coef;
    int nq;                         // merge positions, most significant first
    int nn;                         // the other positions, oldest (most significant) first
    int qpos[kMaxK];
    int npos[kMaxK];
    unsigned long long cmask;       // key bits of the merge positions q with q+1 also one (table windows)
    int part;                       // 1: partition merge in place of the table
    unsigned int n_part_max;        // partitions allocated (a power of two)
    unsigned int* pcount;           // [n_part_max] entries appended this step, zero between steps
    PartRec* prec;                  // [n_part_max * kPartCap] the entries
    unsigned long long* pother;     // ... unpacked form, when pfit is 0: smallest other points at the best |w|^2
    int pfit;                       // unpacked form: key, other points and quantised |w|^2 fill one 128-bit number
    double* partials;               // [partial_stride(P)][grid] per expand workgroup
    int grid;
    int grid_merge;                 // workgroups of the partition merge (resident at once)
    double2* rho_hist;
    StepStatsDev* stats_hist;
    unsigned int* error;
};


// expand, resolve, compact, reduce (partition merge: expand, merge, reduce);
// records after_expand (a hipEvent_t, may be null) on the stream between expand
// and the rest
int launch_sparse_step(const SparseArgs& a, void* stream, void* after_expand);

// workgroups of the partition merge resident at once on n_cu compute units, a
// multiple of kSegs (at least kSegs)
int sparse_merge_grid(int P, int hw, bool f32, int n_cu);

}  // namespace quapi_dev
