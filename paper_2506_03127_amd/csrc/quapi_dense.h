// Host/device interface of the direct-mapped store (two-level systems, merge
// positions 0..L-1 with a short key): argument blocks and launchers.
#pragma once

#include "quapi_host.h"

namespace quapi_dev {

// Every key of the L merge positions owns a slot: slot = key, the points read
// as a base-4 number with point 0 most significant, so slots are in key order.
// A slot holds a 32-byte record -- the group amplitude and the rest of the
// representative's history (points L..K-1, point L lowest) -- and an occupancy
// byte in an array of its own: the slot holds a group after step t when its
// byte is dense_tag(t) (other values are left by earlier steps; the planner
// clears a buffer every kDenseClearPeriod launches, so no old tag comes back).
//
// Segment j is the four slots [4 j, 4 j + 4): the parents whose children merge
// (same points 0..L-2, Sec. 3.1.2).  The merged child of segment j by pair p
// has the fixed slot p * Q + j, Q = 4^(L-1), so an output position never
// depends on other groups.  Between steps the planner lists the nonempty
// segments by how many groups they hold (lists 0..3 for 1..4 groups; entry
// (j << 4) | the segment's four occupancy bits); a step takes 64 segments of
// one list per wave, one segment per lane, so every lane of a wave extends the
// same number of parents.
constexpr int kDenseThreads = 256;             // step workgroup: four independent waves
constexpr int kDenseMinL = 6;                  // 4^L slots; short keys take the bucketed store
constexpr int kDenseMaxL = 12;
constexpr int kDenseChunk = 64;                // segments per chunk (one wave)
constexpr int kDensePlanThreads = 256;
constexpr int kDensePlanIters = 1;             // 16-byte loads (four segments) per planner thread
constexpr int kDenseRegion = kDensePlanThreads * kDensePlanIters * 4;   // segments per planner workgroup
constexpr int kDenseMaxRegions = (1 << (2 * (kDenseMaxL - 1))) / kDenseRegion;

// Occupancy tag of the groups after step t.  A buffer holds the tags of every
// other step since its last clear; tags repeat after 255 steps, so a stale byte
// could match only 510 steps on.  The planner clears the buffer the planned step
// writes when that step is 0 or 1 modulo kDenseClearPeriod: each buffer at least
// every kDenseClearPeriod steps.
constexpr int kDenseClearPeriod = 128;
__host__ __device__ inline unsigned int dense_tag(int t) { return 1u + (unsigned int)(t % 255); }
inline int dense_clear_due(int t_done) { return (t_done + 1) % kDenseClearPeriod < 2 ? 1 : 0; }

struct alignas(32) DenseRec {
    double2 w;                   // group amplitude
    unsigned long long tail;     // points L..K-1 of the representative, point L lowest
    unsigned long long pad;
};

// the FP32 precision form's record: the amplitude as FP32 (ln|w|, arg w)
struct alignas(16) DenseRec32 {
    float lw, aw;
    unsigned long long tail;
};

// Lag-sum tables of one coefficient set: per table 64 entries of (A, B, Ac, Bc),
// the sums over the table's points of (cre ds, cim ss, dre ds, dim ss), then
// exp(-D^2 Re c_0) and exp(-D^2 Re delta_0); tables 0.. cover the segment's
// key points 0..L-2 two at a time (the first point the high digit), the
// rest the tail points L..K-1 two at a time (the first point the low digit).
int dense_tab_count(int L, int K);
size_t dense_tabset_doubles(int L, int K);   // one set, padded to 32 bytes

struct DensePlan {
    unsigned int n_seg[4];      // nonempty segments holding 1, 2, 3, 4 groups
    unsigned int n_groups;      // groups stored (input of the planned step)
    unsigned int n_chunks;      // chunks of 64 segments: list 3 first, then 2, 1, 0
    unsigned int pad[2];
};

struct DenseArgs {
    const unsigned int* seg;             // [4][S/4] the planner's lists
    const DenseRec* rec_in;              // [S] the stored groups (FP64 form)
    DenseRec* rec_out;                   // [S] the step's merged children (FP64 form)
    const DenseRec32* rec32_in;          // the same in the FP32 precision form
    DenseRec32* rec32_out;
    int f32;                             // 1: the FP32 precision form
    unsigned char* flag_out;             // [S] set to dense_tag(t) at the step's merged children
    const DensePlan* plan;
    double* partials;                    // [partial_stride(4)][grid] each workgroup's sums
    const double* tables;                // TableLayout
    const double* coef;                  // this step's coefficients: cre, cim, dre, dim [4][K+1]
    const double* tabset;                // this step's lag-sum tables (dense_tabset_doubles)
    long long n_segs;                    // S/4
    int L, K, t;                         // (the kernel takes its tag from t)
    double theta2;
    unsigned long long qmask;
    unsigned int* error;
};

struct DensePlanArgs {
    const unsigned int* flags;           // [S/4] occupancy of the stored groups, a byte per slot
    unsigned int* flags_spent;           // [S/4] occupancy buffer the planned step writes
    int clear_spent;                     // 1: clear flags_spent first (dense_clear_due(reduce_t))
    unsigned int* seg;                   // [4][S/4] lists for the planned step
    long long n_segs;                    // S/4
    DensePlan* plan;                     // plan of the step to plan
    const DensePlan* plan_prev;          // plan of the step just done (for its counters)
    int reduce_t;                        // step whose partials to reduce, 0: none
    const double* partials;              // [partial_stride(4)][n_parts]
    int n_parts;                         // workgroups of the step kernel
    unsigned long long* agg;             // [kDenseMaxRegions] region counts, tagged with the epoch
    unsigned int epoch;                  // this launch's tag, 1..4095
    double2* rho_hist;
    StepStatsDev* stats_hist;
    unsigned int* error;
};

int dense_lds_bytes(int L, int K, bool f32);   // dynamic LDS of the step kernel (lag-sum tables)
// the lag-sum table sets of coefficient sets 0..n_sets-1 (coef: [n_sets][4][K+1],
// tables: TableLayout) into out [n_sets][dense_tabset_doubles]
int launch_dense_tables(const double* coef, const double* tables, int L, int K, int n_sets, double* out,
                        void* stream);
int launch_dense_step(const DenseArgs& a, int grid, int lds_bytes, void* stream);
int launch_dense_plan(const DensePlanArgs& a, void* stream);
int dense_step_grid(int n_cu, int lds_bytes, bool f32);   // persistent workgroups resident at once
int dense_max_chunks(long long n_segs);

}  // namespace quapi_dev
