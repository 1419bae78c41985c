// One time step of the MACGIC-iQUAPI path propagation on gfx950 (wave64):
// a one-workgroup planner kernel and a persistent step kernel.
//
// State between steps: the groups the next step extends.  A group is a merge
// key (points 0..L-1 of its history, point 0 most significant), the rest of
// the representative's history (points L..K-1) and the group amplitude.  The
// merge positions are 0..L-1: L = E-1 for pre-merging on the reduced mask
// {mask[i]-1} of a contiguous mask {0..E-1} (Sec. 3.1), L = E for
// post-merging on the mask (Sec. 2.1).  Groups live in P^D buckets indexed
// by the top D points of the key, sorted by key inside a bucket.
//
// Where the children go: a child of group g by pair p has key (p, points
// 0..L-2 of g).  For a super-bucket sigma (top D-1 points) the parents in the
// P buckets (sigma, x) produce exactly the children of the P buckets
// (p, sigma), and the children that merge -- same p, parents agreeing on
// points 0..L-2 -- come from consecutive parents inside one super-bucket
// (they differ only in point L-1, the lowest digit of the sorted order).  So
// output positions are local to a super-bucket: no global scan is needed.
//
// Planner (between steps): scans the bucket sizes, lists the nonempty
// buckets with their first global group index and, for each chunk of C
// consecutive groups of the global key order, the bucket holding its first
// group.  It also zeroes the next bucket sizes and reduces the finished
// step's per-chunk sums of rho(t) and counters in chunk order
// (deterministic).
//
// Step: a co-resident grid of persistent workgroups takes chunks round-robin
// and fetches each chunk's parents one chunk ahead.  A chunk extends each
// parent by every pair (eq. SysP propagator element times the influence
// factor of eq. inf_fun), drops children below theta (Sec. 2.1), merges each
// segment of consecutive parents per p (sum of weights; representative of
// largest quantised |w|^2, ties to the smaller history read from the oldest
// point; Sec. 3.1.2), ranks the merged groups per output bucket with wave
// ballots and a block scan segmented by super-bucket, and writes them.
// rho(t) collects the survivors with the end-point correction of the final
// point (Sec. 3.2.1).  A super-bucket cut by a chunk boundary continues at
// offsets found by a decoupled look-back: each chunk publishes the totals of
// its last super-bucket run at once -- inclusive when they do not depend on
// the chunks before it, its own otherwise, inclusive later.

#include <hip/hip_runtime.h>

#include "quapi_host.h"
#include "quapi_device.h"

namespace quapi_dev {

namespace {

constexpr int kWaves = kThreads / 64;
constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
// nonempty-bucket entries cached per chunk: the groups around it lie in at most
// kThreads + 2 buckets, plus the ends of up to two instances in the batched form
constexpr int kWin = kThreads + 6;
constexpr int kTabPts = 2;            // points per subset-sum table (two-level systems)
constexpr int kTabEntries = 16;       // 4^2
constexpr int kMaxTabs = 16;
constexpr int kInstTabs = kMaxTabs * kTabEntries * 4 + 2;   // doubles per instance of instance_tables
constexpr unsigned int kSpinLimit = 1u << 22;
constexpr unsigned long long kAgg = 1ull << 32;   // look-back word: own totals only
constexpr unsigned long long kInc = 2ull << 32;   // look-back word: inclusive totals

// ------------------------------------------------------------------ planner
// Workgroup w < n_regions plans the buckets [w*kRegion, (w+1)*kRegion)
// (thread i owns kPlanPer consecutive ones) and finds the groups and
// nonempty buckets before its region by summing the bucket sizes there with
// coalesced loads; the last workgroup reduces the finished step's per-chunk
// sums.  All of them run side by side.
constexpr int kPlanPer = 4;
constexpr int kRegion = kPlanThreads * kPlanPer;

__device__ inline unsigned long long pack_sizes(unsigned int a0, unsigned int a1, unsigned int a2,
                                                unsigned int a3) {
    // (groups << 32) | nonempty buckets
    const unsigned int nz = (a0 != 0u) + (a1 != 0u) + (a2 != 0u) + (a3 != 0u);
    return ((unsigned long long)(a0 + a1 + a2 + a3) << 32) | nz;
}

template <int P>
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const PlanArgs a) {
    constexpr int S = partial_stride(P);
    constexpr unsigned int C = kThreads - (P - 1);
    __shared__ unsigned long long wsum[kPlanWaves];
    __shared__ unsigned long long wpre[kPlanWaves];
    __shared__ double wred[kPlanWaves][S];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const long long NB = a.n_buckets;
    const int n_regions = (int)((NB + kRegion - 1) / kRegion);
    const int w = (int)blockIdx.x;

    if (w == n_regions) {
        // ---- counters and rho(t) of the step just finished, summed in chunk order
        if (a.reduce_t <= 0) return;
        const unsigned int nc = a.plan_prev->n_chunks;
        const unsigned int err = error_word(a.error);
        if (err != 0u && (int)(err >> 4) <= a.reduce_t) return;   // that step failed: keep nothing
        double acc[S];
#pragma unroll
        for (int k = 0; k < S; ++k) acc[k] = 0.0;
#pragma unroll 2
        for (unsigned int c = i; c < nc; c += kPlanThreads)
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] += a.partials[(size_t)k * a.max_chunks + c];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) wred[wave][k] = v;
        }
        __syncthreads();
        if (i < S) {
            double v = 0.0;
            for (int q = 0; q < kPlanWaves; ++q) v += wred[q][i];
            wred[0][i] = v;
        }
        __syncthreads();
        if (i == 0) {
            const unsigned long long ng = a.plan_prev->n_groups;
#pragma unroll
            for (int p = 0; p < P; ++p)
                a.rho_hist[(size_t)a.reduce_t * P + p] = make_double2(wred[0][2 * p], wred[0][2 * p + 1]);
            StepStatsDev* st = a.stats_hist + a.reduce_t;   // n_stored comes from the last region
            st->n_groups = ng;
            st->n_children = ng * (unsigned long long)P;
            st->n_survivors = (unsigned long long)wred[0][2 * P + 1];
            st->dropped_abs = wred[0][2 * P];
            st->pad = 0.0;
        }
        return;
    }

    // a failed step leaves the stored groups of the step before it in place: the
    // lists, the plan and the bucket sizes (counts_next holds the last complete
    // state's sizes after a failure) stay as they are
    if (error_word(a.error) != 0u) return;

    // ---- this thread's bucket sizes and, in the same batch, those before the region
    const long long b_lo = (long long)w * kRegion + (long long)i * kPlanPer;
    unsigned int cnt[kPlanPer];
    if (b_lo + kPlanPer <= NB) {
        const uint4 v = *reinterpret_cast<const uint4*>(a.counts + b_lo);
        cnt[0] = v.x; cnt[1] = v.y; cnt[2] = v.z; cnt[3] = v.w;
    } else {
#pragma unroll
        for (int k = 0; k < kPlanPer; ++k) cnt[k] = b_lo + k < NB ? a.counts[b_lo + k] : 0u;
    }
    unsigned long long before = 0;                     // this thread's share of the earlier regions
#pragma unroll 8
    for (int r = 0; r < w; ++r) {
        const uint4 v = *reinterpret_cast<const uint4*>(a.counts + (long long)r * kRegion + (long long)i * kPlanPer);
        before += pack_sizes(v.x, v.y, v.z, v.w);
    }

    // ---- block sums: exclusive scan of this region, plus the earlier regions' total
    const unsigned long long mine = pack_sizes(cnt[0], cnt[1], cnt[2], cnt[3]);
    unsigned long long incl = mine, bsum = before;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long v = __shfl_up(incl, off, 64);
        if ((int)lane >= off) incl += v;
    }
    for (int off = 32; off > 0; off >>= 1) bsum += __shfl_xor(bsum, off, 64);
    if (lane == 63) wsum[wave] = incl;
    if (lane == 0) wpre[wave] = bsum;
    __syncthreads();
    unsigned long long base = incl - mine, region = 0;
    for (int q = 0; q < kPlanWaves; ++q) {
        if (q < wave) base += wsum[q];
        base += wpre[q];
        region += wsum[q] + wpre[q];
    }

    // ---- nonempty buckets; each chunk's first group lies in the one of rank desc[c]
    unsigned int run = (unsigned int)(base >> 32), rank = (unsigned int)base;
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) {
        const unsigned int n = cnt[k];
        if (n == 0u) continue;
        a.nz_bucket[rank] = (unsigned int)(b_lo + k);
        a.nz_prefix[rank] = run;
        for (unsigned int c = (run + C - 1) / C; c * C < run + n; ++c)
            if ((int)c < a.max_chunks) a.desc[c] = rank;
        ++rank;
        run += n;
    }

    // ---- zero the next step's bucket sizes
    if (b_lo + kPlanPer <= NB) {
        *reinterpret_cast<uint4*>(a.counts_next + b_lo) = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (long long b = b_lo; b < NB; ++b) a.counts_next[b] = 0u;
    }

    // ---- the last region knows the totals
    if (w == n_regions - 1 && i == 0) {
        const unsigned int N = (unsigned int)(region >> 32);
        if (a.reduce_t > 0) a.stats_hist[a.reduce_t].n_stored = N;
        Plan pl;
        pl.n_groups = N;
        pl.n_chunks = (N + C - 1) / C;
        pl.pad = 0u;
        pl.n_nonempty = (unsigned int)region;
        *a.plan = pl;
    }
}

// ------------------------------------------------------------------ batched planner
// Instance j owns the buckets [j*IB, (j+1)*IB), IB = P^D <= kRegion; one
// workgroup plans one instance.  Its groups start at chunk
// sum_{r<j} ceil(n_r / C) of the global order, and its nonempty buckets at rank
// sum_{r<j} (nz_r + 1): each instance's list ends with an entry kNoBucket whose
// prefix is the instance's end, so that the positions up to the next chunk
// boundary hold no group.  Two kernels: (1) each instance's totals, and the
// reduction of the finished step per instance; (2) the lists.

// thread i's kPlanPer buckets of instance w (zero past the instance)
__device__ inline void batch_counts(const PlanArgs& a, int w, int i, unsigned int cnt[kPlanPer]) {
    const long long lo = (long long)w * a.inst_buckets + (long long)i * kPlanPer;
    const long long hi = (long long)(w + 1) * a.inst_buckets;
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) cnt[k] = lo + k < hi ? a.counts[lo + k] : 0u;
}

template <int P>
__global__ __launch_bounds__(kPlanThreads) void plan_batch_totals(const PlanArgs a) {
    constexpr int S = partial_stride(P);
    constexpr unsigned int C = kThreads - (P - 1);
    __shared__ unsigned long long wsum[kPlanWaves];
    __shared__ double wred[kPlanWaves][S];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const int B = a.n_inst;
    const int w = (int)blockIdx.x;

    if (w >= B) {
        // ---- counters and rho(t) of instance w - B in the step just finished, in chunk
        //      order from the instance's first chunk (the order a lone instance has)
        const int j = w - B;
        if (a.reduce_t <= 0) return;
        const unsigned int err = error_word(a.error);
        if (err != 0u && (int)(err >> 4) <= a.reduce_t) return;
        const unsigned int c0 = a.inst_prev[2 * j], ng = a.inst_prev[2 * j + 1];
        const unsigned int nc = (ng + C - 1) / C;
        double acc[S];
#pragma unroll
        for (int k = 0; k < S; ++k) acc[k] = 0.0;
#pragma unroll 2
        for (unsigned int c = i; c < nc; c += kPlanThreads)
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] += a.partials[(size_t)k * a.max_chunks + c0 + c];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) wred[wave][k] = v;
        }
        __syncthreads();
        if (i < S) {
            double v = 0.0;
            for (int q = 0; q < kPlanWaves; ++q) v += wred[q][i];
            wred[0][i] = v;
        }
        __syncthreads();
        if (i == 0) {
            const size_t h = (size_t)a.reduce_t * B + j;
#pragma unroll
            for (int p = 0; p < P; ++p) a.rho_hist[h * P + p] = make_double2(wred[0][2 * p], wred[0][2 * p + 1]);
            StepStatsDev* st = a.stats_hist + h;          // n_stored comes from the lists kernel
            st->n_groups = ng;
            st->n_children = (unsigned long long)ng * (unsigned long long)P;
            st->n_survivors = (unsigned long long)wred[0][2 * P + 1];
            st->dropped_abs = wred[0][2 * P];
            st->pad = 0.0;
        }
        return;
    }

    // ---- instance w's totals
    unsigned int cnt[kPlanPer];
    batch_counts(a, w, i, cnt);
    unsigned long long v = pack_sizes(cnt[0], cnt[1], cnt[2], cnt[3]);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[wave] = v;
    __syncthreads();
    if (i == 0) {
        unsigned long long t = 0;
        for (int q = 0; q < kPlanWaves; ++q) t += wsum[q];
        a.totals[w] = t;
    }
}

template <int P>
__global__ __launch_bounds__(kPlanThreads) void plan_batch_lists(const PlanArgs a) {
    constexpr unsigned int C = kThreads - (P - 1);
    __shared__ unsigned long long wsum[kPlanWaves];
    __shared__ unsigned long long wpre[kPlanWaves];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const int B = a.n_inst;
    const int w = (int)blockIdx.x;
    if (error_word(a.error) != 0u) return;       // keep the last complete state (see plan_kernel)

    // ---- where instance w starts: chunks and list entries of the instances before it
    unsigned long long before = 0;                     // (chunks << 32) | list entries
    for (int r = i; r < w; r += kPlanThreads) {
        const unsigned long long tr = a.totals[r];
        const unsigned int n = (unsigned int)(tr >> 32), nz = (unsigned int)tr;
        before += ((unsigned long long)((n + C - 1) / C) << 32) + nz + 1u;
    }
    for (int off = 32; off > 0; off >>= 1) before += __shfl_xor(before, off, 64);

    // ---- this instance's buckets: exclusive scan of (groups, nonempty)
    unsigned int cnt[kPlanPer];
    batch_counts(a, w, i, cnt);
    const unsigned long long mine = pack_sizes(cnt[0], cnt[1], cnt[2], cnt[3]);
    unsigned long long incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long x = __shfl_up(incl, off, 64);
        if ((int)lane >= off) incl += x;
    }
    if (lane == 63) wsum[wave] = incl;
    if (lane == 0) wpre[wave] = before;
    __syncthreads();
    unsigned long long base = incl - mine, total = 0, pre = 0;
    for (int q = 0; q < kPlanWaves; ++q) {
        if (q < wave) base += wsum[q];
        total += wsum[q];
        pre += wpre[q];
    }
    const unsigned int g_start = (unsigned int)(pre >> 32) * C;    // first global group index
    const unsigned int r_start = (unsigned int)pre;                // first list entry
    const unsigned int n_w = (unsigned int)(total >> 32), nz_w = (unsigned int)total;

    // ---- nonempty buckets; each chunk's first group lies in the one of rank desc[c]
    unsigned int run = g_start + (unsigned int)(base >> 32), rank = r_start + (unsigned int)base;
    const long long b_lo = (long long)w * a.inst_buckets + (long long)i * kPlanPer;
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k) {
        const unsigned int n = cnt[k];
        if (n == 0u) continue;
        a.nz_bucket[rank] = (unsigned int)(b_lo + k);
        a.nz_prefix[rank] = run;
        for (unsigned int c = (run + C - 1) / C; c * C < run + n; ++c)
            if ((int)c < a.max_chunks) a.desc[c] = rank;
        ++rank;
        run += n;
    }

    // ---- zero the next step's bucket sizes of this instance
    const long long hi = (long long)(w + 1) * a.inst_buckets;
#pragma unroll
    for (int k = 0; k < kPlanPer; ++k)
        if (b_lo + k < hi) a.counts_next[b_lo + k] = 0u;

    if (i == 0) {
        // the entry that closes the instance, its extent, and the groups stored
        a.nz_bucket[r_start + nz_w] = kNoBucket;
        a.nz_prefix[r_start + nz_w] = g_start + n_w;
        a.inst_next[2 * w] = g_start / C;
        a.inst_next[2 * w + 1] = n_w;
        if (a.reduce_t > 0) a.stats_hist[(size_t)a.reduce_t * B + w].n_stored = n_w;
        if (w == B - 1) {
            Plan pl;
            pl.n_groups = g_start + n_w;
            pl.n_chunks = (g_start + n_w + C - 1) / C;
            pl.pad = 0u;
            pl.n_nonempty = r_start + nz_w + 1u;
            *a.plan = pl;
        }
    }
}

// ------------------------------------------------------------------ step
template <int P>
struct Lds {
    double k4re[P * P], k4im[P * P];
    double ds[P], ss[P];
    double cre[kMaxK + 1], cim[kMaxK + 1], dre[kMaxK + 1], dim[kMaxK + 1];   // this step's coefficients
    double tab[P == 4 ? kMaxTabs : 1][P == 4 ? kTabEntries : 1][4];         // subset sums (two levels)
    double2 cw[P][kThreads];               // child weights
    unsigned long long ctail[kThreads];    // child history tails
    unsigned int surv[kThreads];           // bit p: child p survives
    unsigned int win_b[kWin];              // nonempty buckets of the next chunk ...
    unsigned int win_p[kWin];              // ... and their first global group index
    unsigned long long hmask[kWaves];      // segment heads, one word per wave
    unsigned long long vmask[kWaves];      // loaded parents
    unsigned long long omask[P][kWaves];   // merged groups written, per pair
    unsigned int ocount[P][kWaves];        // their popcounts
    int wstart[kWaves];                    // last super-bucket run start in each wave
    unsigned int base[P];                  // offsets of the first run when it continues
    double wrho[kWaves][4][P == 4 ? 8 : 2 * P];   // rho sums per wave and row of 16 lanes (two levels)
    double wdrop[kWaves];
    unsigned int wsurv[kWaves];
    unsigned int sig0, prev_sig;           // super-bucket of the first parent and of the group before
    unsigned int chunk_inst;               // instance of the chunk fetched last (batched form)
    double e0, f0;
};

// One thread's parent of a chunk.  Lane 0 of each wave also holds the group
// before it (pkey, psig) and lane 63 the super-bucket of the group after it.
struct Parent {
    unsigned long long key, tail, pkey;
    double2 w;
    unsigned int sig, psig, nsig;         // 0xffffffff: none
};

// Window of nonempty buckets around a chunk: entries [rb, rb + kWin) of the
// list, rb one before the bucket of the chunk's first group.  Thread i holds
// entries i and kThreads + i (i < kWin - kThreads) until they are written to the LDS.
struct WinRegs {
    unsigned int b0, p0, b1, p1;
};

__device__ inline WinRegs load_window(const StepArgs& a, unsigned int first_rank, unsigned int n_nz,
                                      unsigned int N, int i) {
    const unsigned int rb = first_rank > 0u ? first_rank - 1u : 0u;
    WinRegs w;
    const unsigned int k0 = rb + (unsigned int)i, k1 = rb + kThreads + (unsigned int)i;
    w.b0 = k0 < n_nz ? a.nz_bucket[k0] : 0u;
    w.p0 = k0 < n_nz ? a.nz_prefix[k0] : N;
    w.b1 = (i < kWin - kThreads && k1 < n_nz) ? a.nz_bucket[k1] : 0u;
    w.p1 = (i < kWin - kThreads && k1 < n_nz) ? a.nz_prefix[k1] : N;
    return w;
}

// largest k with win_p[k] <= g; the window holds groups g0-1 .. g0+kThreads of its chunk
template <int P>
__device__ inline int window_search(const Lds<P>& s, unsigned int g) {
    int lo = 0, hi = kWin - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s.win_p[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

template <int P, int C, bool BATCH>
__device__ inline Parent fetch_parent(const StepArgs& a, const Lds<P>& s, unsigned int c, unsigned int N,
                                      unsigned int nrec, int i, unsigned int lane) {
    Parent r;
    r.key = ~0ull;
    r.tail = 0ull;
    r.pkey = ~0ull;
    r.w = make_double2(0.0, 0.0);
    r.sig = 0xffffffffu;
    r.psig = 0xffffffffu;
    r.nsig = 0xffffffffu;
    const unsigned int g = c * (unsigned int)C + (unsigned int)i;
    const int k = g < N ? window_search(s, g) : 0;
    // a position past an instance's end (batched form) holds no group
    if (g < N && (!BATCH || s.win_b[k] != kNoBucket)) {
        const unsigned int b = s.win_b[k];
        const unsigned int o = b * (unsigned int)a.cap + (g - s.win_p[k]);   // the store has < 2^31 records
        if (o < nrec) {
            r.key = a.in.key[o];
            r.tail = a.in.tail[o];
            r.w = a.in.w[o];
            r.sig = b / P;
        } else {
            raise_error(a.error, a.t, kErrOverflow);
        }
        // lane 0: the group before; lane 63: the group after.  Each lies in the
        // bucket of g or in the nonempty bucket next to it in the list.
        if (lane == 0u && g > 0u) {
            const int kn = (g - 1u >= s.win_p[k] || k == 0) ? k : k - 1;
            const unsigned int bn = s.win_b[kn];
            if (!BATCH || (bn != kNoBucket && g - 1u >= s.win_p[kn])) {
                const unsigned int op = bn * (unsigned int)a.cap + (g - 1u - s.win_p[kn]);
                if (op < nrec) {
                    r.pkey = a.in.key[op];
                    r.psig = bn / P;
                }
            }
        }
        if (lane == 63u && g + 1u < N) {
            const int kn = (k + 1 < kWin && g + 1u >= s.win_p[k + 1]) ? k + 1 : k;
            r.nsig = (BATCH && s.win_b[kn] == kNoBucket) ? 0xffffffffu : s.win_b[kn] / P;
        }
    }
    return r;
}

template <int P>
__device__ inline void store_window(Lds<P>& s, const WinRegs& w, int i) {
    s.win_b[i] = w.b0;
    s.win_p[i] = w.p0;
    if (i < kWin - kThreads) {
        s.win_b[kThreads + i] = w.b1;
        s.win_p[kThreads + i] = w.p1;
    }
}

// number of merged groups of pair p before position j of the chunk (0 <= j <= kThreads)
template <int P>
__device__ inline unsigned int excl_at(const Lds<P>& s, int p, int j) {
    const int wj = j >> 6;
    unsigned int e = 0u;
    for (int w = 0; w < wj && w < kWaves; ++w) e += s.ocount[p][w];
    if (wj < kWaves) e += (unsigned int)__popcll(s.omask[p][wj] & ((1ull << (j & 63)) - 1ull));
    return e;
}

__device__ inline unsigned long long shfl_up1_u64(unsigned long long v) {
    return (unsigned long long)__shfl_up((long long)v, 1, 64);
}

// One instance's coefficients of this step into the LDS.
template <int P>
__device__ inline void load_coefficients(Lds<P>& s, const double* coef, int K, int i) {
    for (int k = i; k < 4 * (K + 1); k += kThreads) {
        const int r = k / (K + 1), d = k - r * (K + 1);
        double* dst = r == 0 ? s.cre : r == 1 ? s.cim : r == 2 ? s.dre : s.dim;
        dst[d] = coef[k];
    }
}

// Subset-sum tables of the coefficients in the LDS (two levels):
// tab[q][v] = sum over the points of table q of coefficient(lag) * (ds, ss)(point).
template <int P, int BP>
__device__ inline void build_tables(Lds<P>& s, int K, int L, int nk, int nt, bool use_tabs, int i) {
    constexpr unsigned long long DM = (1ull << BP) - 1;
    if constexpr (P == 4) {
        if (use_tabs) {
            for (int idx = i; idx < (nk + nt) * kTabEntries; idx += kThreads) {
                const int q = idx / kTabEntries, v = idx - q * kTabEntries;
                const bool in_key = q < nk;
                const int st = in_key ? kTabPts * q : L + kTabPts * (q - nk);
                const int len = in_key ? min(kTabPts, L - st) : min(kTabPts, K - st);
                double A = 0, B = 0, Ac = 0, Bc = 0;
                if (v < (1 << (BP * len))) {
                    for (int m = 0; m < len; ++m) {
                        const int sh = in_key ? BP * (len - 1 - m) : BP * m;
                        const int x = (v >> sh) & (int)DM;
                        const int d = st + m + 1;                     // lag of that point
                        A += s.cre[d] * s.ds[x];
                        B += s.cim[d] * s.ss[x];
                        Ac += s.dre[d] * s.ds[x];
                        Bc += s.dim[d] * s.ss[x];
                    }
                }
                s.tab[q][v][0] = A;
                s.tab[q][v][1] = B;
                s.tab[q][v][2] = Ac;
                s.tab[q][v][3] = Bc;
            }
        }
        if (i == 0) {
            const double D = s.ds[1];
            s.e0 = exp(-D * D * s.cre[0]);
            s.f0 = exp(-D * D * s.dre[0]);
        }
    }
}

// Each instance's subset tables and end-point factors of one coefficient set,
// built by the code the step kernel builds them with (so bit for bit the same),
// for the batched form's chunks to copy instead of rebuilding:
// out[inst][kInstTabs]: tab[q][v][4] for q < kMaxTabs, then e0, f0.
template <int P, int BP>
__global__ __launch_bounds__(kThreads) void instance_tables(const StepArgs a, double* out) {
    __shared__ Lds<P> s;
    const int i = threadIdx.x;
    const unsigned int inst = blockIdx.x;
    const int K = a.K, L = a.L;
    if (i < P) {
        s.ds[i] = a.tables[TableLayout::ds(P) + i];
        s.ss[i] = a.tables[TableLayout::ss(P) + i];
    }
    load_coefficients(s, a.coef + (size_t)inst * 4 * (K + 1), K, i);
    __syncthreads();
    const int nk = (L + kTabPts - 1) / kTabPts, nt = (K - L + kTabPts - 1) / kTabPts;
    build_tables<P, BP>(s, K, L, nk, nt, (P == 4) && (nk + nt <= kMaxTabs), i);
    __syncthreads();
    double* o = out + (size_t)inst * kInstTabs;
    if constexpr (P == 4) {
        const double* t = &s.tab[0][0][0];
        for (int idx = i; idx < (nk + nt) * kTabEntries * 4; idx += kThreads) o[idx] = t[idx];
        if (i == 0) {
            o[kMaxTabs * kTabEntries * 4] = s.e0;
            o[kMaxTabs * kTabEntries * 4 + 1] = s.f0;
        }
    }
}

// BATCH: the batched form (several instances; chunks reload the coefficients of
// their instance, and positions past an instance's end hold no group)
template <int P, int BP, bool BATCH>
__global__ __launch_bounds__(kThreads, P == 4 ? 4 : 1) void step_kernel(const StepArgs a) {
    constexpr int C = kThreads - (P - 1);              // segment heads per chunk
    constexpr int S = partial_stride(P);
    constexpr unsigned long long DM = (1ull << BP) - 1;
    __shared__ Lds<P> s;
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();

    if (error_word(a.error) != 0u) return;             // an earlier step failed: leave the state alone
    const unsigned int N = a.plan->n_groups;
    const unsigned int n_chunks = a.plan->n_chunks;
    const unsigned int n_nz = a.plan->n_nonempty;
    const unsigned int G = gridDim.x;
    // chunks in runs of R consecutive ones: workgroup w takes runs w, w+G, w+2G, ...
    // (R = 1: plain round-robin).  Every workgroup takes its chunks in increasing
    // order, so the look-back, which waits only on earlier chunks, always ends.
    // (runs are used by the batched form, whose workgroups then change instance less often)
    const unsigned int R = (BATCH && a.chunk_run > 0) ? (unsigned int)a.chunk_run : 1u;
    auto succ = [&](unsigned int x, unsigned int k) -> unsigned int {   // the k-th chunk after x
        if constexpr (!BATCH) {
            return x + k * G;
        } else {
            for (unsigned int j = 0; j < k; ++j) x = (x % R == R - 1u) ? x + (G - 1u) * R + 1u : x + 1u;
            return x;
        }
    };
    unsigned int c = blockIdx.x * R;
    if (c >= n_chunks) return;

    // ---- the first chunk's window and the next one's, in flight during the set-up
    const unsigned int nrec = (unsigned int)((long long)a.n_super * P * a.cap * a.n_inst);
    WinRegs wr = load_window(a, a.desc[c], n_nz, N, i);
    WinRegs wn = {0u, 0u, 0u, 0u};
    if (succ(c, 1) < n_chunks) wn = load_window(a, a.desc[succ(c, 1)], n_nz, N, i);
    unsigned int d_after = (succ(c, 2) < n_chunks) ? a.desc[succ(c, 2)] : 0u;

    // ---- tables and coefficients of this step
    const int K = a.K, L = a.L, t = a.t;
    for (int k = i; k < P * P; k += kThreads) {
        s.k4re[k] = a.tables[2 * k];
        s.k4im[k] = a.tables[2 * k + 1];
    }
    if (i < P) {
        s.ds[i] = a.tables[TableLayout::ds(P) + i];
        s.ss[i] = a.tables[TableLayout::ss(P) + i];
    }
    load_coefficients(s, a.coef, K, i);              // instance 0; a chunk of another reloads
    unsigned int loaded = 0u;
    const int nk = (L + kTabPts - 1) / kTabPts, nt = (K - L + kTabPts - 1) / kTabPts;
    const bool use_tabs = (P == 4) && (nk + nt <= kMaxTabs);
    store_window(s, wr, i);
    __syncthreads();
    Parent cur = fetch_parent<P, C, BATCH>(a, s, c, N, nrec, i, lane);
    // a chunk's first group is always one; its instance picks the coefficients
    if (BATCH && i == 0) s.chunk_inst = cur.sig == 0xffffffffu ? 0u : cur.sig / (unsigned int)a.n_super;
    build_tables<P, BP>(s, K, L, nk, nt, use_tabs, i);

    const int dmax = t < K ? t : K;
    const int tail_pts = K - L;
    const unsigned long long tail_mask =
        tail_pts <= 0 ? 0ull : (tail_pts * BP >= 64 ? ~0ull : ((1ull << (tail_pts * BP)) - 1));
    const int top_shift = BP * (L - 1);
    const unsigned long long etag = (unsigned long long)(a.epoch & 0x3fffffffu);
    const unsigned long long ep = etag << 34;
    const unsigned long long lane_le = (lane == 63u) ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0..lane

    for (;;) {
        // ---- fetch the next chunk's parents now; they arrive while this chunk computes
        const unsigned int c1 = succ(c, 1);
        const bool has_next = c1 < n_chunks;
        Parent nxt = cur;
        __syncthreads();                                   // the chunk before is done with the LDS
        // this chunk's instance: its coefficients and tables unless they are in the LDS
        unsigned int ob_base = 0u;                         // output bucket offset of the instance
        if constexpr (BATCH) {
            const unsigned int inst = s.chunk_inst;
            if (inst != loaded) {
                if (a.k4_batch)
                    for (int k = i; k < P * P; k += kThreads) {
                        s.k4re[k] = a.k4_batch[2 * ((size_t)inst * P * P + k)];
                        s.k4im[k] = a.k4_batch[2 * ((size_t)inst * P * P + k) + 1];
                    }
                load_coefficients(s, a.coef + (size_t)inst * 4 * (K + 1), K, i);
                if (P == 4 && use_tabs && a.inst_tabs) {
                    // the instance's tables as instance_tables built them
                    const double* src = a.inst_tabs + (size_t)inst * kInstTabs;
                    double* t = &s.tab[0][0][0];
                    for (int idx = i; idx < (nk + nt) * kTabEntries * 4; idx += kThreads) t[idx] = src[idx];
                    if (i == 0) {
                        s.e0 = src[kMaxTabs * kTabEntries * 4];
                        s.f0 = src[kMaxTabs * kTabEntries * 4 + 1];
                    }
                } else {
                    __syncthreads();
                    build_tables<P, BP>(s, K, L, nk, nt, use_tabs, i);
                }
                loaded = inst;
            }
            ob_base = inst * (unsigned int)(P - 1) * (unsigned int)a.n_super;
        }
        if (has_next) {
            store_window(s, wn, i);
            __syncthreads();                               // (also publishes the tables)
            nxt = fetch_parent<P, C, BATCH>(a, s, c1, N, nrec, i, lane);
            if (BATCH && i == 0) s.chunk_inst = nxt.sig == 0xffffffffu ? 0u : nxt.sig / (unsigned int)a.n_super;
            const unsigned int c2 = succ(c1, 1), c3 = succ(c2, 1);
            if (c2 < n_chunks) wn = load_window(a, d_after, n_nz, N, i);
            d_after = (c3 < n_chunks) ? a.desc[c3] : 0u;
        }

        // ---- this chunk: groups [g0, g0 + nsz) loaded, segment heads [g0, g0 + H) owned;
        //      for all but the last chunk H = C and positions >= H lie in the last wave
        const unsigned int g0 = c * (unsigned int)C;
        const int H = (int)min((unsigned int)C, N - g0);
        const bool valid = cur.sig != 0xffffffffu;
        const unsigned long long key = cur.key, tail = cur.tail;
        const double2 W = cur.w;
        const unsigned int my_sig = cur.sig;
        // neighbours: inside the wave by shuffles, across waves from the fetch
        const unsigned long long up_key = shfl_up1_u64(key);
        const unsigned int up_sig = (unsigned int)__shfl_up((int)my_sig, 1, 64);
        const unsigned int dn_sig = (unsigned int)__shfl_down((int)my_sig, 1, 64);
        const unsigned long long pk = lane == 0u ? cur.pkey : up_key;
        const unsigned int psg = lane == 0u ? cur.psig : up_sig;
        const unsigned int nsg = lane == 63u ? cur.nsig : dn_sig;
        // (parents with equal points 0..L-2 share the super-bucket; across
        // instances of the batched form they do not)
        const bool head = valid && (g0 + i == 0u || (key >> BP) != (pk >> BP) || (BATCH && my_sig != psg));
        const bool rstart = valid && (i == 0 || my_sig != psg);
        const unsigned long long hm = __ballot(head), vm = __ballot(valid), rsm = __ballot(rstart);
        if (lane == 0u) {
            s.hmask[wave] = hm;
            s.vmask[wave] = vm;
            s.wstart[wave] = rsm ? wave * 64 + 63 - __builtin_clzll(rsm) : -1;
        }
        if (i == 0) {
            s.sig0 = my_sig;
            s.prev_sig = cur.psig;
        }
        __syncthreads();

        // a parent belongs to this chunk when its segment head does
        bool owned = false;
        if (valid) {
            if (i < H) {
                const int lo = (int)lane - (P - 1);
                const unsigned long long span = lo >= 0 ? (lane_le & ~((1ull << lo) - 1ull)) : lane_le;
                owned = (hm & span) != 0ull;
                if (!owned && lo < 0 && wave > 0) owned = (s.hmask[wave - 1] >> (64 + lo)) != 0ull;
            } else {
                const int hl = H - wave * 64;              // H lies in this wave (see above)
                owned = (hm & lane_le & ~((1ull << hl) - 1ull)) == 0ull;
            }
        }
        // segment length of a head: up to the next head or the end of the loaded parents
        const bool is_head = (i < H) && head;
        int len = 0;
        if (is_head) {
            const unsigned long long stop_lo = hm | ~vm;
            const unsigned long long stop_hi = wave + 1 < kWaves ? (s.hmask[wave + 1] | ~s.vmask[wave + 1]) : ~0ull;
            const unsigned long long after = lane == 63u ? stop_hi : ((stop_lo >> (lane + 1)) | (stop_hi << (63 - lane)));
            len = 1 + (after ? __builtin_ctzll(after) : 64);
            if (len > P) len = P;
        }
        // start of this parent's super-bucket run inside the chunk
        int start;
        {
            const unsigned long long m = rsm & lane_le;
            if (m) {
                start = wave * 64 + 63 - __builtin_clzll(m);
            } else {
                start = 0;
                for (int w = wave - 1; w >= 0; --w)
                    if (s.wstart[w] >= 0) { start = s.wstart[w]; break; }
            }
        }

        // ---- extend: influence sums of the parent over lags 1..dmax
        double rho_re[P], rho_im[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { rho_re[p] = 0.0; rho_im[p] = 0.0; }
        double dropped = 0.0;
        unsigned int surv_bits = 0;
        unsigned long long ctail = 0;
        if (owned) {
            double A = 0.0, B = 0.0, Ac = 0.0, Bc = 0.0;
            if (use_tabs) {
                for (int q = 0; q < nk; ++q) {
                    const int st = kTabPts * q, ln = min(kTabPts, L - st);
                    const int v = (int)((key >> (BP * (L - st - ln))) & ((1ull << (BP * ln)) - 1));
                    A += s.tab[q][v][0];
                    B += s.tab[q][v][1];
                    Ac += s.tab[q][v][2];
                    Bc += s.tab[q][v][3];
                }
                for (int q = nk; q < nk + nt; ++q) {
                    const int st = L + kTabPts * (q - nk), ln = min(kTabPts, K - st);
                    const int v = (int)((tail >> (BP * (st - L))) & ((1ull << (BP * ln)) - 1));
                    A += s.tab[q][v][0];
                    B += s.tab[q][v][1];
                    Ac += s.tab[q][v][2];
                    Bc += s.tab[q][v][3];
                }
            } else {
                for (int d = 1; d <= dmax; ++d) {
                    const int pos = d - 1;
                    const unsigned int x = pos < L ? (unsigned int)((key >> (BP * (L - 1 - pos))) & DM)
                                                   : (unsigned int)((tail >> (BP * (pos - L))) & DM);
                    const double dsx = s.ds[x], ssx = s.ss[x];
                    A = __builtin_fma(s.cre[d], dsx, A);
                    B = __builtin_fma(s.cim[d], ssx, B);
                    Ac = __builtin_fma(s.dre[d], dsx, Ac);
                    Bc = __builtin_fma(s.dim[d], ssx, Bc);
                }
            }
            const int h0 = (int)(key >> top_shift);
            ctail = ((tail << BP) | (key & DM)) & tail_mask;
            // influence factor e[p] of the new point and end-point correction f[p]
            double er[P], ei[P], fr[P], fi[P];
            if constexpr (P == 4) {
                // two levels: pairs (0,1) and (1,0) have ds = +D, -D and equal ss, so
                // their exponents are mirror images and share one exp and one sincos
                const double D = s.ds[1], Sg = s.ss[1];
                const double x = D * A, y = D * __builtin_fma(s.cim[0], Sg, B);
                const double xc = D * Ac, yc = D * __builtin_fma(s.dim[0], Sg, Bc);
                const double ex = exp_fast(x), exc = exp_fast(xc);
                const double iex = recip(ex), iexc = recip(exc);
                double sy, cy, syc, cyc;
                sincos_fast(y, &sy, &cy);
                sincos_fast(yc, &syc, &cyc);
                const double e0 = s.e0, f0 = s.f0;    // exp(-D^2 Re c_0), exp(-D^2 Re delta_0)
                er[0] = 1.0; ei[0] = 0.0; fr[0] = 1.0; fi[0] = 0.0;
                er[3] = 1.0; ei[3] = 0.0; fr[3] = 1.0; fi[3] = 0.0;
                er[1] = e0 * iex * cy;  ei[1] = -(e0 * iex * sy);
                er[2] = e0 * ex * cy;   ei[2] = e0 * ex * sy;
                fr[1] = f0 * iexc * cyc; fi[1] = -(f0 * iexc * syc);
                fr[2] = f0 * exc * cyc;  fi[2] = f0 * exc * syc;
            } else {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const double dsp = s.ds[p], ssp = s.ss[p];
                    er[p] = 1.0; ei[p] = 0.0; fr[p] = 1.0; fi[p] = 0.0;
                    if (dsp != 0.0) {
                        const double e = exp_fast(-dsp * (s.cre[0] * dsp + A));
                        double sn, cs2;
                        sincos_fast(-dsp * (s.cim[0] * ssp + B), &sn, &cs2);
                        er[p] = e * cs2;
                        ei[p] = e * sn;
                        const double f = exp_fast(-dsp * (s.dre[0] * dsp + Ac));
                        double fs, fc;
                        sincos_fast(-dsp * (s.dim[0] * ssp + Bc), &fs, &fc);
                        fr[p] = f * fc;
                        fi[p] = f * fs;
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double k4r = s.k4re[p * P + h0], k4i = s.k4im[p * P + h0];
                const double br = W.x * k4r - W.y * k4i;
                const double bi = W.x * k4i + W.y * k4r;
                const double wr2 = br * er[p] - bi * ei[p];
                const double wi2 = br * ei[p] + bi * er[p];
                const double n2 = norm2_nocontract(wr2, wi2);
                const bool keep = (a.theta2 == 0.0) || !(n2 < a.theta2);
                if (keep) {
                    surv_bits |= 1u << p;
                    rho_re[p] = wr2 * fr[p] - wi2 * fi[p];
                    rho_im[p] = wr2 * fi[p] + wi2 * fr[p];
                } else {
                    dropped += sqrt(n2);
                }
                s.cw[p][i] = make_double2(wr2, wi2);
            }
        }
        s.surv[i] = surv_bits;
        s.ctail[i] = ctail;

        // ---- partial sums of rho, dropped weight and survivor count
        if constexpr (P == 4) {
            const double v[8] = {rho_re[0], rho_im[0], rho_re[1], rho_im[1],
                                 rho_re[2], rho_im[2], rho_re[3], rho_im[3]};
            double x0, x1;
            row_sums8(v, lane, x0, x1);
            if ((lane & 15u) >= 12u) {
                const unsigned int r = lane & 3u;
                const int k = 4 * (int)(r & 1u) + 2 * (int)(r >> 1);
                s.wrho[wave][lane >> 4][k] = x0;
                s.wrho[wave][lane >> 4][k + 1] = x1;
            }
        } else {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double r = wave_sum(rho_re[p]), m = wave_sum(rho_im[p]);
                if (lane == 0u) {
                    s.wrho[wave][0][2 * p] = r;
                    s.wrho[wave][0][2 * p + 1] = m;
                }
            }
        }
        {
            const double dsum = wave_sum(dropped);
            unsigned int ns = 0u;
#pragma unroll
            for (int p = 0; p < P; ++p) ns += (unsigned int)__popcll(__ballot((surv_bits >> p) & 1u));
            if (lane == 0u) { s.wdrop[wave] = dsum; s.wsurv[wave] = ns; }
        }
        __syncthreads();

        // ---- which pairs of each segment keep a merged group (any member survives)
        bool ov[P];
        unsigned int msurv[P];
        unsigned long long mtail[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {                      // members of the segment (clamped reads)
            const int j = min(i + m, kThreads - 1);
            msurv[m] = m < len ? s.surv[j] : 0u;
            mtail[m] = s.ctail[j];
        }
        {
            unsigned int anyp = 0u;
#pragma unroll
            for (int m = 0; m < P; ++m) anyp |= msurv[m];
#pragma unroll
            for (int p = 0; p < P; ++p) ov[p] = (anyp >> p) & 1u;
        }

        // ---- ranks: per pair, wave ballots; block offsets from the per-wave counts
        unsigned int lrank[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const unsigned long long bal = __ballot(ov[p]);
            lrank[p] = rank_below(bal);
            if (lane == 0u) {
                s.omask[p][wave] = bal;
                s.ocount[p][wave] = (unsigned int)__popcll(bal);
            }
        }
        if (i < S) {                                       // this chunk's partial sums
            double v = 0.0;
            if (i < 2 * P) {
                for (int w = 0; w < kWaves; ++w)
                    for (int r = 0; r < (P == 4 ? 4 : 1); ++r) v += s.wrho[w][r][i];
            } else if (i == 2 * P) {
                for (int w = 0; w < kWaves; ++w) v += s.wdrop[w];
            } else {
                unsigned int ns = 0u;
                for (int w = 0; w < kWaves; ++w) ns += s.wsurv[w];
                v = (double)ns;
            }
            a.partials[(size_t)i * a.max_chunks + c] = v;
        }
        __syncthreads();
        unsigned int my_excl[P], run_base[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            unsigned int e = lrank[p];
            for (int w = 0; w < wave; ++w) e += s.ocount[p][w];
            my_excl[p] = e;
            run_base[p] = excl_at(s, p, start);
        }

        // ---- publish the totals of the last run for the chunk after this one: inclusive
        //      now unless the last run is the continued first run
        const bool first_cont = g0 > 0u && s.prev_sig == s.sig0;
        const bool next_cont = (!BATCH || valid) && (i == H - 1) && (c + 1 < n_chunks) && nsg == my_sig;
        const bool from_prev = (start == 0) && first_cont;
        unsigned long long* const slot_c = a.chain + c;
        if (next_cont) {
#pragma unroll
            for (int p = 0; p < P; ++p)
                st_relaxed(slot_c + (size_t)p * a.max_chunks,
                           ep | (from_prev ? kAgg : kInc) | (my_excl[p] + (ov[p] ? 1u : 0u) - run_base[p]));
        }

        // ---- merge each segment per pair: sum of the surviving weights and the
        //      representative (while the word published above travels)
        double2 ow[P];
        unsigned long long otail[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double2 mw[P];
#pragma unroll
            for (int m = 0; m < P; ++m) mw[m] = s.cw[p][min(i + m, kThreads - 1)];
            bool any = false;
            double sr = 0.0, si = 0.0;
            unsigned long long bq = 0, bt = 0;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                if (!((msurv[m] >> p) & 1u)) continue;
                const double2 w = mw[m];
                sr += w.x;
                si += w.y;
                const unsigned long long q =
                    (unsigned long long)__double_as_longlong(norm2_nocontract(w.x, w.y)) & a.qmask;
                if (!any || q > bq || (q == bq && mtail[m] < bt)) { bq = q; bt = mtail[m]; }
                any = true;
            }
            ow[p] = make_double2(sr, si);
            otail[p] = bt;
        }

        // ---- look-back: the first run continues a super-bucket cut by the chunk boundary
        if (first_cont) {
            if (wave == 0 && (int)lane < P) {
                const unsigned long long* row = a.chain + (size_t)lane * a.max_chunks;
                unsigned int sum = 0u, slot = c - 1u, spins = 0u;
                for (;;) {
                    const unsigned long long v = ld_relaxed(row + slot);
                    if ((v >> 34) != etag) {
                        if (++spins > kSpinLimit) { raise_error(a.error, t, kErrSpin); break; }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    sum += (unsigned int)v;
                    if (v & kInc) break;
                    if (slot == 0u) { raise_error(a.error, t, kErrSpin); break; }
                    --slot;
                }
                s.base[lane] = sum;
            }
            __syncthreads();
            if (next_cont && from_prev) {
#pragma unroll
                for (int p = 0; p < P; ++p)
                    st_relaxed(slot_c + (size_t)p * a.max_chunks,
                               ep | kInc | (my_excl[p] + (ov[p] ? 1u : 0u) - run_base[p] + s.base[p]));
            }
        }

        // ---- write merged groups to the output buckets (p, sigma)
        const unsigned int n_out_buckets = (unsigned int)a.n_inst * (unsigned int)P * (unsigned int)a.n_super;
        if (is_head) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!ov[p]) continue;
                const unsigned int idx = my_excl[p] - run_base[p] + (from_prev ? s.base[p] : 0u);
                if (idx >= (unsigned int)a.cap) {
                    raise_error(a.error, t, kErrOverflow);
                    continue;
                }
                const unsigned int ob = (unsigned int)p * (unsigned int)a.n_super + my_sig + ob_base;
                if (BATCH && ob >= n_out_buckets) {              // a head outside its chunk's instance
                    raise_error(a.error, t, kErrSpin);
                    continue;
                }
                const unsigned int o = ob * (unsigned int)a.cap + idx;
                a.out.key[o] = ((unsigned long long)p << top_shift) | (key >> BP);
                a.out.tail[o] = otail[p];
                a.out.w[o] = ow[p];
            }
        }
        // bucket sizes: the last parent of each run that ends in this chunk records the totals
        if ((!BATCH || valid) && i < H && ((i == H - 1) ? !next_cont : (nsg != my_sig))) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const unsigned int tot = my_excl[p] + (ov[p] ? 1u : 0u) - run_base[p] +
                                         (from_prev ? s.base[p] : 0u);
                const unsigned int ob = (unsigned int)p * (unsigned int)a.n_super + my_sig + ob_base;
                if (tot && (!BATCH || ob < n_out_buckets))
                    a.out_count[ob] = tot > (unsigned int)a.cap ? (unsigned int)a.cap : tot;
            }
        }
        if (!has_next) break;
        cur = nxt;
        c = c1;
    }
}

}  // namespace

int chunk_heads(int P) { return kThreads - (P - 1); }

int plan_max_buckets() { return 64 * kRegion; }

int step_grid(int P, int n_cu, int per_cu, bool batch) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (P == 4 && !batch) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<4, 2, false>, kThreads, 0);
    if (P == 4 && batch) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<4, 2, true>, kThreads, 0);
    if (P == 9 && !batch) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<9, 4, false>, kThreads, 0);
    if (P == 9 && batch) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, step_kernel<9, 4, true>, kThreads, 0);
    if (e != hipSuccess || nb < 1) return 0;
    // the look-back waits on other workgroups: every workgroup of the grid must be resident
    return (per_cu > 0 ? (per_cu < nb ? per_cu : nb) : nb) * n_cu;
}

int launch_step(const StepArgs& a, int grid, void* stream) {

    hipStream_t st = (hipStream_t)stream;
    const bool batch = a.n_inst > 1;
    switch (a.P) {
        case 4:
            if (batch) hipLaunchKernelGGL((step_kernel<4, 2, true>), dim3(grid), dim3(kThreads), 0, st, a);
            else hipLaunchKernelGGL((step_kernel<4, 2, false>), dim3(grid), dim3(kThreads), 0, st, a);
            break;
        case 9:
            if (batch) hipLaunchKernelGGL((step_kernel<9, 4, true>), dim3(grid), dim3(kThreads), 0, st, a);
            else hipLaunchKernelGGL((step_kernel<9, 4, false>), dim3(grid), dim3(kThreads), 0, st, a);
            break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int plan_batch_max_buckets() { return kRegion; }

size_t instance_table_doubles() { return kInstTabs; }

int launch_instance_tables(const StepArgs& a, double* out, void* stream) {
    if (a.P != 4) return (int)hipSuccess;    // the tables serve two-level systems
    hipLaunchKernelGGL((instance_tables<4, 2>), dim3(a.n_inst), dim3(kThreads), 0, (hipStream_t)stream, a, out);
    return (int)hipGetLastError();
}

int launch_plan_batch(const PlanArgs& a, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int B = a.n_inst;
    switch (a.P) {
        case 4:
            hipLaunchKernelGGL((plan_batch_totals<4>), dim3(2 * B), dim3(kPlanThreads), 0, st, a);
            hipLaunchKernelGGL((plan_batch_lists<4>), dim3(B), dim3(kPlanThreads), 0, st, a);
            break;
        case 9:
            hipLaunchKernelGGL((plan_batch_totals<9>), dim3(2 * B), dim3(kPlanThreads), 0, st, a);
            hipLaunchKernelGGL((plan_batch_lists<9>), dim3(B), dim3(kPlanThreads), 0, st, a);
            break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_plan(const PlanArgs& a, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int grid = (int)((a.n_buckets + kRegion - 1) / kRegion) + 1;
    switch (a.P) {
        case 4: hipLaunchKernelGGL((plan_kernel<4>), dim3(grid), dim3(kPlanThreads), 0, st, a); break;
        case 9: hipLaunchKernelGGL((plan_kernel<9>), dim3(grid), dim3(kPlanThreads), 0, st, a); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace quapi_dev
