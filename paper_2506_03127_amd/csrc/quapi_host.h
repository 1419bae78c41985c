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

// Stored group list: P runs ("classes"), one per value of the newest point.
// Run c holds count[c] groups sorted by key; its arrays start at c * cap.
struct GroupBuf {
    uint64_t* key;     // merge key: points 0..L-1, point 0 in the top bits
    uint64_t* tail;    // points L..K-1, point L in the low bits
    double2* w;        // group amplitude
};

// Per-tile partial sums, reduced in tile order by the last tile to finish.
struct TilePartial {
    double2 rho[kMaxP];
    double dropped;
    unsigned long long n_surv;
};

struct StepStatsDev {
    unsigned long long n_groups, n_children, n_survivors, n_stored;
    double dropped_abs;
    double pad;
};

struct StepArgs {
    GroupBuf in, out;
    const unsigned int* in_count;   // [P]
    unsigned int* out_count;        // [P]
    long long cap;                  // capacity of one run
    int P, L, K, t;
    unsigned int epoch;             // monotonically increasing step number of the context
    int bits;                       // bits per point
    int max_tiles;
    double theta2;
    unsigned long long qmask;       // keep-mask of the |w|^2 bit pattern
    const double* tables;           // device tables, see TableLayout
    unsigned int* counters;         // [4]: tile counter x2, done counter x2 (indexed by epoch parity)
    unsigned long long* status;     // [P * max_tiles] look-back words
    TilePartial* partials;          // [max_tiles]
    double2* rho_out;               // rho(t): P values
    StepStatsDev* stats_out;        // counters of step t
    unsigned int* error;            // [2]: code, step
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
int max_tiles_for(int P, long long cap);
int tile_heads(int P);

}  // namespace quapi_dev
