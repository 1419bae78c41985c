// Host/device interface of the direct-mapped store (two-level systems, merge
// positions 0..L-1 with a short key): argument blocks and launchers.
#pragma once

#include "quapi_host.h"

namespace quapi_dev {

// Every key of the L merge positions owns a slot: slot = key, the points read
// as a base-P number with point 0 most significant, so slots are in key order.
// A slot holds the rest of the representative's history (points L..K-1, point
// L lowest) and the group amplitude; a bitmap (one 64-bit word per 64 slots)
// says which slots hold a group.
//
// The parents whose children merge (same points 0..L-2) are the P slots
// [P j, P j + P) of segment j, and the merged child of segment j by pair p has
// the fixed slot p * Q + j, Q = P^(L-1): an output position never depends on
// other groups, so chunks of parents need no offsets from one another.  The
// planner between steps turns the bitmap into chunks of equal size: the list
// of nonempty bitmap words with the number of groups before each, and the
// word holding each chunk's first group.
constexpr int kDenseThreads = 256;             // threads per chunk = parents loaded per chunk
constexpr int kDenseMinL = 6;                  // 4^L slots; short keys take the bucketed store
constexpr int kDenseMaxL = 12;                 // 4^12 slots: 64 planner regions
constexpr int kDensePlanThreads = 256;
constexpr int kDensePlanPer = 16;              // bitmap words per planner thread
constexpr int kDenseRegion = kDensePlanThreads * kDensePlanPer;   // words per planner workgroup
constexpr int kDenseMaxRegions = 64;           // the planner's regions, all resident at once

struct DensePlan {
    unsigned int n_groups;      // groups stored (input of the planned step)
    unsigned int n_chunks;
    unsigned int pad;
    unsigned int n_nonempty;    // nonempty bitmap words
};

struct DenseArgs {
    const unsigned long long* bits_in;   // [S/64] slots holding a group (state at t-1)
    const unsigned long long* tail_in;   // [S]
    const double2* w_in;                 // [S]
    unsigned long long* bits_out;        // [S/64] cleared by the planner, set here
    unsigned long long* tail_out;
    double2* w_out;
    const unsigned int* nz_word;         // [n_nonempty] nonempty words of bits_in, in order ...
    const unsigned int* nz_prefix;       // ... the groups before each ...
    const unsigned long long* nz_bits;   // ... and the word itself
    const unsigned int* desc;            // [n_chunks] rank of the word holding the chunk's first group
    const DensePlan* plan;
    double* partials;                    // [partial_stride(4)][grid] each workgroup's sums
    int max_chunks;
    const double* tables;                // TableLayout
    const double* coef;                  // this step's coefficients: cre, cim, dre, dim [4][K+1]
    int L, K, t;
    double theta2;
    unsigned long long qmask;
    unsigned int* error;
};

struct DensePlanArgs {
    const unsigned long long* bits;      // [n_words] the stored groups
    unsigned long long* bits_next;       // [n_words] cleared for the planned step's output
    long long n_words;
    unsigned int* nz_word;
    unsigned int* nz_prefix;
    unsigned long long* nz_bits;
    unsigned int* desc;
    DensePlan* plan;                     // plan of the step to plan
    const DensePlan* plan_prev;          // plan of the step just done (for its counters)
    int max_chunks;
    int reduce_t;                        // step whose partials to reduce, 0: none
    const double* partials;              // [partial_stride(4)][n_parts]
    int n_parts;                         // workgroups of the step kernel
    unsigned long long* agg;             // [kDenseMaxRegions] region totals, tagged with the epoch
    unsigned int epoch;                  // this launch's tag (nonzero in its low 24 bits)
    double2* rho_hist;
    StepStatsDev* stats_hist;
    unsigned int* error;
};

int dense_chunk_heads();
int launch_dense_step(const DenseArgs& a, int grid, void* stream);
int launch_dense_plan(const DensePlanArgs& a, void* stream);
int dense_step_grid(int n_cu);            // persistent workgroups resident at once

}  // namespace quapi_dev
