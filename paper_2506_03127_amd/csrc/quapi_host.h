// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "host_math.h"

namespace quapi_dev {

constexpr int kThreads = 256;      // threads per tile = parents loaded per tile
constexpr int kMaxP = 16;          // pairs per point (M <= 4)
constexpr int kMaxK = 64;          // memory length bound (history words)

// Stored group list: the key space is cut into P^D buckets by the top D
// points of the merge key (point 0 most significant); bucket b holds count[b]
// groups sorted by key at [b * cap, b * cap + count[b]).  A group is its key
// (points 0..L-1, point 0 in the top bits), the rest of the representative's
// history (points L..K-1, point L in the low bits) and the group amplitude.
struct GroupBuf {
    uint64_t* key;
    uint64_t* tail;
    double2* w;
};

// Per-chunk partial sums, partial_stride(P) doubles: rho(t) re/im for the P
// pairs, dropped |w|, survivors.  The planner that follows a step reduces
// them in chunk order.
constexpr int partial_stride(int P) { return 2 * P + 2; }

struct StepStatsDev {
    unsigned long long n_groups, n_children, n_survivors, n_stored;
    double dropped_abs;
    double pad;
};

// Plan of one step, written by the planner.
struct Plan {
    unsigned int n_groups;     // groups stored (input of the planned step)
    unsigned int n_chunks;     // chunks of the planned step
    unsigned int pad;
    unsigned int n_nonempty;   // nonempty buckets
};

// Chunk c covers the global group indices [c*C, (c+1)*C) with C =
// chunk_heads(P) (segment heads; it also reads the P-1 groups after them).
// desc[c] is the index, in the list of nonempty buckets, of the bucket that
// holds group c*C.

// Batched form: n_inst instances (bath parameter points) share one store; the
// buckets of instance j are [j*P^D, (j+1)*P^D).  Each instance's groups start
// at a multiple of the chunk size in the global group order, so that a chunk
// never holds two instances, and an entry kNoBucket closes each instance in
// the nonempty-bucket list (its prefix is the instance's end).
constexpr unsigned int kNoBucket = 0xffffffffu;

struct StepArgs {
    GroupBuf in, out;
    unsigned int* out_count;        // [n_inst * P^D] output bucket sizes (zeroed by the planner)
    const unsigned int* nz_bucket;  // [n_nonempty] nonempty input buckets, in key order (kNoBucket: an instance's end)
    const unsigned int* nz_prefix;  // [n_nonempty] their first global group index
    const unsigned int* desc;       // [n_chunks]
    const Plan* plan;               // this step's plan
    long long cap;                  // capacity of one bucket
    int P, L, K, t;
    int n_super;                    // P^(D-1), per instance
    int n_inst;                     // instances (1 unless batched)
    int chunk_run;                  // consecutive chunks a workgroup takes in turn (1: round-robin)
    unsigned int epoch;             // step number of the context, tags the look-back words
    double theta2;
    unsigned long long qmask;       // keep-mask of the |w|^2 bit pattern
    const double* tables;           // device tables, see TableLayout
    const double* coef;             // this step's coefficients: cre, cim, dre, dim [n_inst][4][K+1]
    const double* k4_batch;         // [n_inst][P*P] complex K4 per instance (batched form with one H_S
                                    // per instance), or null: the K4 of tables for all
    const double* inst_tabs;        // batched form: [n_inst][instance_table_doubles()] subset tables and
                                    // end-point factors of this step's coefficients, or null: rebuilt
    unsigned long long* chain;      // [P * max_chunks] look-back words, one per chunk and pair
    int max_chunks;
    double* partials;               // [partial_stride(P)][max_chunks], component-major
    unsigned int* error;            // (failing step << 4) | code, 0 if none
};

struct PlanArgs {
    const unsigned int* counts;     // [n_buckets] bucket sizes of the stored groups
    unsigned int* counts_next;      // [n_buckets] output bucket sizes of the planned step: zeroed here
    unsigned int* nz_bucket;        // [n_buckets + n_inst]
    unsigned int* nz_prefix;        // [n_buckets + n_inst]
    unsigned int* desc;             // [max_chunks]
    Plan* plan;                     // plan of the step to plan
    const Plan* plan_prev;          // plan of the step just done (for its counters)
    long long n_buckets;
    int max_chunks;
    int P;
    int reduce_t;                   // step whose partials to reduce, 0: none
    const double* partials;
    double2* rho_hist;              // [history][n_inst][P]
    StepStatsDev* stats_hist;       // [history][n_inst]
    const unsigned int* error;
    // batched form
    int n_inst;
    int inst_buckets;               // P^D, at most the buckets one planner workgroup takes
    unsigned long long* totals;     // [n_inst] (groups << 32) | nonempty buckets of the stored groups
    unsigned int* inst_next;        // [n_inst][2] first chunk and groups of each instance, planned step
    const unsigned int* inst_prev;  // [n_inst][2] the same for the step just done
};

// Device table layout (doubles): K4 re/im [2*P*P], ds[P], ss[P], eta [2*3*(K+1)]
struct TableLayout {
    static constexpr size_t k4(int) { return 0; }
    static constexpr size_t ds(int P) { return 2 * (size_t)P * P; }
    static constexpr size_t ss(int P) { return ds(P) + P; }
    static constexpr size_t eta(int P) { return ss(P) + P; }
    static constexpr size_t total(int P, int K) { return eta(P) + 6 * (size_t)(K + 1); }
};

enum : unsigned int { kErrNone = 0, kErrOverflow = 1, kErrSpin = 2 };

int launch_step(const StepArgs& a, int grid, void* stream);   // returns hipError_t
int launch_plan(const PlanArgs& a, void* stream);
int launch_plan_batch(const PlanArgs& a, void* stream);   // two kernels: totals and reduce, then lists
int plan_batch_max_buckets();                            // P^D of one instance at most
size_t instance_table_doubles();                         // per instance, of instance_tables
int launch_instance_tables(const StepArgs& a, double* out, void* stream);   // one workgroup per instance
int chunk_heads(int P);
int plan_max_buckets();              // bucket count the planner is built for
int step_grid(int P, int n_cu, int per_cu, bool batch);   // persistent workgroups that are co-resident

}  // namespace quapi_dev
