// One time step of the MACGIC-iQUAPI path propagation on the direct-mapped
// store (two-level systems, merge positions 0..L-1): a planner and a step
// kernel per step.
//
// The store has a slot for every key of the merge positions (slot = key, point
// 0 most significant) and a bitmap of the slots that hold a group, so the
// groups in slot order are the groups sorted by key.  The parents whose
// children merge -- those agreeing on points 0..L-2 (Sec. 3.1.2) -- are
// consecutive in that order, and the merged child of a segment by pair p has
// the fixed slot (p, points 0..L-2 of the parents): writing it needs no offset
// from any other chunk.
//
// Planner (between steps): scans the popcounts of the bitmap words, lists the
// nonempty words with the groups before each (and the word itself), and, for
// each chunk of C consecutive groups, the word holding its first group; it
// clears the next step's output bitmap and reduces the finished step's
// per-workgroup sums of rho(t) and counters in workgroup order (deterministic).
//
// Step: persistent workgroups take chunks round-robin and fetch each chunk's
// parents one chunk ahead (a parent's slot is the rank of its bit in its
// word).  A chunk extends each parent by every pair (propagator element of
// eq. SysP times the influence factor of eq. inf_fun; end-point correction of
// the final point for rho(t), Sec. 3.2.1), drops children below theta
// (Sec. 2.1), merges each segment of consecutive parents per pair (sum of the
// surviving weights; representative of largest quantised |w|^2, ties to the
// smaller history read from the oldest point), writes the merged groups to
// their slots, and sets their bits (LDS atomics into the chunk's window of
// output words, then one device atomic OR per word).  Chunks never wait on one
// another.  Each workgroup sums rho(t), the dropped |w| and the survivors over
// its chunks; the next planner adds the workgroups' sums in workgroup order.

#include <hip/hip_runtime.h>

#include "quapi_dense.h"
#include "quapi_device.h"

namespace quapi_dev {

namespace {

constexpr int P4 = 4, BP2 = 2;
constexpr int kWavesD = kDenseThreads / 64;
constexpr int kC = kDenseThreads - (P4 - 1);   // segment heads per chunk
constexpr int kWinD = kDenseThreads + 6;       // nonempty words cached per chunk (>= groups it reads + 1)
constexpr int kTabPtsD = 2;
constexpr int kTabEntriesD = 16;
constexpr int kMaxTabsD = 16;
constexpr int kPlanWavesD = kDensePlanThreads / 64;
constexpr int kOutWin = 8;                     // output bitmap words per pair staged per chunk

// position of the r-th set bit (r < popcount) of v
__device__ inline unsigned int select_bit(unsigned long long v, unsigned int r) {
    unsigned int pos = 0;
    unsigned int c = (unsigned int)__popc((unsigned int)v);
    if (r >= c) { r -= c; pos = 32; v >>= 32; }
    c = (unsigned int)__popc((unsigned int)v & 0xffffu);
    if (r >= c) { r -= c; pos += 16; v >>= 16; }
    c = (unsigned int)__popc((unsigned int)v & 0xffu);
    if (r >= c) { r -= c; pos += 8; v >>= 8; }
    c = (unsigned int)__popc((unsigned int)v & 0xfu);
    if (r >= c) { r -= c; pos += 4; v >>= 4; }
    c = (unsigned int)__popc((unsigned int)v & 0x3u);
    if (r >= c) { r -= c; pos += 2; v >>= 2; }
    c = (unsigned int)(v & 1u);
    if (r >= c) pos += 1;
    return pos;
}

// ------------------------------------------------------------------ planner
// Workgroup w < n_regions plans the words [w * kDenseRegion, (w + 1) * kDenseRegion)
// (thread i owns kDensePlanPer consecutive ones, read as 16-byte pairs), publishes
// its region's totals (groups, nonempty words) tagged with the launch's epoch,
// and adds up the totals of the regions before it in one wave-wide read (every
// region workgroup is resident: there are at most 64); the last workgroup
// reduces the finished step's per-workgroup sums.
constexpr unsigned long long kAggTag = 1ull << 40;   // epoch field of a region total: bits 40..63

__device__ inline unsigned long long pack_sizes_d(unsigned int groups, unsigned int nz) {
    return ((unsigned long long)groups << 32) | nz;       // (groups << 32) | nonempty words
}

__global__ __launch_bounds__(kDensePlanThreads) void dense_plan(const DensePlanArgs a) {
    constexpr int S = partial_stride(P4);
    __shared__ unsigned long long wsum[kPlanWavesD];
    __shared__ unsigned long long before_s;
    __shared__ double wred[kPlanWavesD][S];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const long long NW = a.n_words;
    const int n_regions = (int)((NW + kDenseRegion - 1) / kDenseRegion);
    const int w = (int)blockIdx.x;

    if (w == n_regions) {
        // ---- counters and rho(t) of the step just finished, summed in workgroup order
        if (a.reduce_t <= 0) return;
        const unsigned int nc = (unsigned int)a.n_parts;
        const unsigned int err = error_word(a.error);
        if (err != 0u && (int)(err >> 4) <= a.reduce_t) return;
        double acc[S];
#pragma unroll
        for (int k = 0; k < S; ++k) acc[k] = 0.0;
        for (unsigned int c = i; c < nc; c += kDensePlanThreads)
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] += a.partials[(size_t)k * a.n_parts + c];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) wred[wave][k] = v;
        }
        __syncthreads();
        if (i < S) {
            double v = 0.0;
            for (int q = 0; q < kPlanWavesD; ++q) v += wred[q][i];
            wred[0][i] = v;
        }
        __syncthreads();
        if (i == 0) {
            const unsigned long long ng = a.plan_prev->n_groups;
#pragma unroll
            for (int p = 0; p < P4; ++p)
                a.rho_hist[(size_t)a.reduce_t * P4 + p] = make_double2(wred[0][2 * p], wred[0][2 * p + 1]);
            StepStatsDev* st = a.stats_hist + a.reduce_t;   // n_stored comes from the last region
            st->n_groups = ng;
            st->n_children = ng * (unsigned long long)P4;
            st->n_survivors = (unsigned long long)wred[0][2 * P4 + 1];
            st->dropped_abs = wred[0][2 * P4];
            st->pad = 0.0;
        }
        return;
    }
    if (error_word(a.error) != 0u) return;               // keep the last complete state

    // ---- this thread's words, as 16-byte pairs
    const long long b_lo = (long long)w * kDenseRegion + (long long)i * kDensePlanPer;
    unsigned long long wd[kDensePlanPer];
    if (b_lo + kDensePlanPer <= NW) {
        const ulonglong2* src = reinterpret_cast<const ulonglong2*>(a.bits + b_lo);
#pragma unroll
        for (int k = 0; k < kDensePlanPer / 2; ++k) {
            const ulonglong2 v = src[k];
            wd[2 * k] = v.x;
            wd[2 * k + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kDensePlanPer; ++k) wd[k] = b_lo + k < NW ? a.bits[b_lo + k] : 0ull;
    }
    unsigned int cnt[kDensePlanPer];
    unsigned int g_mine = 0, nz_mine = 0;
#pragma unroll
    for (int k = 0; k < kDensePlanPer; ++k) {
        cnt[k] = (unsigned int)__popcll(wd[k]);
        g_mine += cnt[k];
        nz_mine += wd[k] != 0ull;
    }

    // ---- block scan of this region; publish its totals; the regions before it
    const unsigned long long mine = pack_sizes_d(g_mine, nz_mine);
    unsigned long long incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long v = (unsigned long long)__shfl_up((long long)incl, off, 64);
        if ((int)lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    unsigned long long base = incl - mine, region = 0;
    for (int q = 0; q < kPlanWavesD; ++q) {
        if (q < wave) base += wsum[q];
        region += wsum[q];
    }
    const unsigned long long tag = (unsigned long long)(a.epoch & 0xffffffu) * kAggTag;
    if (i == 0)   // region totals < 2^20 groups and 2^16 words: (groups << 16) | nonempty
        st_relaxed(a.agg + w, tag | ((region >> 32) << 16) | (region & 0xffffull));
    if (wave == 0) {
        unsigned long long g = 0, nz = 0;
        if ((int)lane < w) {
            unsigned long long v;
            unsigned int spins = 0;
            while (((v = ld_relaxed(a.agg + lane)) & ~(kAggTag - 1ull)) != tag) {
                if (++spins == (1u << 24)) {   // a region never published: fail the step, do not hang
                    raise_error(a.error, a.reduce_t + 1, kErrSpin);
                    v = 0ull;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            g = (v >> 16) & 0xffffffull;
            nz = v & 0xffffull;
        }
        unsigned long long b = (g << 32) | nz;
        for (int off = 32; off > 0; off >>= 1) b += (unsigned long long)__shfl_xor((long long)b, off, 64);
        if (lane == 0) before_s = b;
    }
    __syncthreads();
    base += before_s;
    const unsigned long long total = before_s + region;

    // ---- nonempty words; each chunk's first group lies in the one of rank desc[c]
    unsigned int run = (unsigned int)(base >> 32), rank = (unsigned int)base;
#pragma unroll
    for (int k = 0; k < kDensePlanPer; ++k) {
        const unsigned int n = cnt[k];
        if (n == 0u) continue;
        a.nz_word[rank] = (unsigned int)(b_lo + k);
        a.nz_prefix[rank] = run;
        a.nz_bits[rank] = wd[k];
        for (unsigned int c = (run + kC - 1) / kC; c * kC < run + n; ++c)
            if ((int)c < a.max_chunks) a.desc[c] = rank;
        ++rank;
        run += n;
    }

    // ---- clear the next step's output bitmap
    if (b_lo + kDensePlanPer <= NW) {
        ulonglong2* dst = reinterpret_cast<ulonglong2*>(a.bits_next + b_lo);
#pragma unroll
        for (int k = 0; k < kDensePlanPer / 2; ++k) dst[k] = make_ulonglong2(0ull, 0ull);
    } else {
        for (long long b = b_lo; b < NW; ++b) a.bits_next[b] = 0ull;
    }

    // ---- the last region knows the totals
    if (w == n_regions - 1 && i == 0) {
        const unsigned int N = (unsigned int)(total >> 32);
        if (a.reduce_t > 0) a.stats_hist[a.reduce_t].n_stored = N;
        DensePlan pl;
        pl.n_groups = N;
        pl.n_chunks = (N + kC - 1) / kC;
        pl.pad = 0u;
        pl.n_nonempty = (unsigned int)total;
        *a.plan = pl;
    }
}

// ------------------------------------------------------------------ step
struct DLds {
    double k4re[16], k4im[16];
    double ds[4], ss[4];
    double cre[kMaxK + 1], cim[kMaxK + 1], dre[kMaxK + 1], dim[kMaxK + 1];
    double tab[kMaxTabsD][kTabEntriesD][4];     // subset sums of the coefficients (A, B, Ac, Bc)
    double e0, f0;
    double2 cw[P4][kDenseThreads];              // child weights
    unsigned int cq[P4][kDenseThreads];         // their quantised |w|^2, high word (qbits >= 32)
    unsigned long long ctail[kDenseThreads];    // child history tails
    unsigned int surv[kDenseThreads];           // bit p: child p survives
    unsigned long long win_b[kWinD];            // nonempty words around the next chunk ...
    unsigned int win_w[kWinD];                  // ... their index ...
    unsigned int win_p[kWinD];                  // ... and the groups before them
    unsigned long long hmask[kWavesD];          // segment heads, one word per wave
    unsigned long long vmask[kWavesD];          // loaded parents
    unsigned long long obits[P4][kOutWin];      // output bitmap words of the chunk, by pair
    unsigned long long obase;                   // word (within a pair) of obits[.][0]
    double wrho[kWavesD][4][8];                 // rho sums per wave and row of 16 lanes
    double wdrop[kWavesD];
    unsigned int wsurv[kWavesD];
};

// One thread's parent of a chunk.  Lane 0 of each wave also holds the key of
// the group before it.
struct DParent {
    unsigned long long key, tail, pkey;   // key ~0: none
    double2 w;
};

struct DWin {
    unsigned long long b0, b1;
    unsigned int w0, p0, w1, p1;
};

// entries [rb, rb + kWinD) of the nonempty-word list, rb one before the word of
// the chunk's first group; thread i holds entries i and kDenseThreads + i
__device__ inline DWin load_window_d(const DenseArgs& a, unsigned int first_rank, unsigned int n_nz,
                                     unsigned int N, int i) {
    const unsigned int rb = first_rank > 0u ? first_rank - 1u : 0u;
    DWin w;
    const unsigned int k0 = rb + (unsigned int)i, k1 = rb + kDenseThreads + (unsigned int)i;
    const bool h0 = k0 < n_nz, h1 = i < kWinD - kDenseThreads && k1 < n_nz;
    w.w0 = h0 ? a.nz_word[k0] : 0u;
    w.p0 = h0 ? a.nz_prefix[k0] : N;
    w.b0 = h0 ? a.nz_bits[k0] : 0ull;
    w.w1 = h1 ? a.nz_word[k1] : 0u;
    w.p1 = h1 ? a.nz_prefix[k1] : N;
    w.b1 = h1 ? a.nz_bits[k1] : 0ull;
    return w;
}

__device__ inline void store_window_d(DLds& s, const DWin& w, int i) {
    s.win_w[i] = w.w0;
    s.win_p[i] = w.p0;
    s.win_b[i] = w.b0;
    if (i < kWinD - kDenseThreads) {
        s.win_w[kDenseThreads + i] = w.w1;
        s.win_p[kDenseThreads + i] = w.p1;
        s.win_b[kDenseThreads + i] = w.b1;
    }
}

// largest k with win_p[k] <= g
__device__ inline int window_search_d(const DLds& s, unsigned int g) {
    int lo = 0, hi = kWinD - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s.win_p[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ inline unsigned long long slot_of(const DLds& s, int k, unsigned int g) {
    return 64ull * s.win_w[k] + select_bit(s.win_b[k], g - s.win_p[k]);
}

__device__ inline DParent fetch_parent_d(const DenseArgs& a, const DLds& s, unsigned int c, unsigned int N,
                                         int i, unsigned int lane) {
    DParent r;
    r.key = ~0ull;
    r.tail = 0ull;
    r.pkey = ~0ull;
    r.w = make_double2(0.0, 0.0);
    const unsigned int g = c * (unsigned int)kC + (unsigned int)i;
    if (g < N) {
        const int k = window_search_d(s, g);
        const unsigned long long slot = slot_of(s, k, g);
        r.key = slot;
        r.tail = a.tail_in[slot];
        r.w = a.w_in[slot];
        // lane 0: the group before, in the word of g or the nonempty word before it
        if (lane == 0u && g > 0u) {
            const int kn = (g - 1u >= s.win_p[k] || k == 0) ? k : k - 1;
            r.pkey = slot_of(s, kn, g - 1u);
        }
    }
    return r;
}

// thread i < P * kOutWin: word i % kOutWin of pair i / kOutWin of the chunk's
// window, ORed into the bitmap and cleared
__device__ inline void flush_bits(const DenseArgs& a, DLds& s, int i, int pair_words) {
    const int p = i / kOutWin, k = i % kOutWin;
    const unsigned long long v = s.obits[p][k];
    if (v) {
        atomicOr(a.bits_out + (((unsigned long long)p << pair_words) | (s.obase + k)), v);
        s.obits[p][k] = 0ull;
    }
}

__global__ __launch_bounds__(kDenseThreads, 4) void dense_step(const DenseArgs a) {
    constexpr int P = P4, BP = BP2, C = kC;
    constexpr int S = partial_stride(P);
    constexpr unsigned long long DM = (1ull << BP) - 1;
    __shared__ DLds s;
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();

    if (error_word(a.error) != 0u) return;
    const unsigned int N = a.plan->n_groups;
    const unsigned int n_chunks = a.plan->n_chunks;
    const unsigned int n_nz = a.plan->n_nonempty;
    const unsigned int G = gridDim.x;
    unsigned int c = blockIdx.x;
    if (c >= n_chunks) {
        if (i < S) a.partials[(size_t)i * G + blockIdx.x] = 0.0;   // no chunk: zero sums
        return;
    }

    // ---- the first chunk's window and the next one's, in flight during the set-up
    DWin wr = load_window_d(a, a.desc[c], n_nz, N, i);
    DWin wn = {0ull, 0ull, 0u, 0u, 0u, 0u};
    if (c + G < n_chunks) wn = load_window_d(a, a.desc[c + G], n_nz, N, i);
    unsigned int d_after = (c + 2 * G < n_chunks) ? a.desc[c + 2 * G] : 0u;

    // ---- tables and coefficients of this step
    const int K = a.K, L = a.L, t = a.t;
    if (i < P * P) {
        s.k4re[i] = a.tables[2 * i];
        s.k4im[i] = a.tables[2 * i + 1];
    }
    if (i < P) {
        s.ds[i] = a.tables[TableLayout::ds(P) + i];
        s.ss[i] = a.tables[TableLayout::ss(P) + i];
    }
    for (int k = i; k < 4 * (K + 1); k += kDenseThreads) {
        const int r = k / (K + 1), d = k - r * (K + 1);
        double* dst = r == 0 ? s.cre : r == 1 ? s.cim : r == 2 ? s.dre : s.dim;
        dst[d] = a.coef[k];
    }
    store_window_d(s, wr, i);
    if (i < P * kOutWin) s.obits[i / kOutWin][i % kOutWin] = 0ull;
    __syncthreads();
    DParent cur = fetch_parent_d(a, s, c, N, i, lane);
    const int nk = (L + kTabPtsD - 1) / kTabPtsD, nt = (K - L + kTabPtsD - 1) / kTabPtsD;
    const bool use_tabs = nk + nt <= kMaxTabsD;
    if (use_tabs && i < (nk + nt) * kTabEntriesD) {
        const int q = i / kTabEntriesD, v = i - q * kTabEntriesD;
        const bool in_key = q < nk;
        const int st = in_key ? kTabPtsD * q : L + kTabPtsD * (q - nk);
        const int len = in_key ? min(kTabPtsD, L - st) : min(kTabPtsD, K - st);
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
    if (i == 0) {
        const double D = s.ds[1];
        s.e0 = exp(-D * D * s.cre[0]);
        s.f0 = exp(-D * D * s.dre[0]);
    }

    const int dmax = t < K ? t : K;
    const int tail_pts = K - L;
    const unsigned long long tail_mask =
        tail_pts <= 0 ? 0ull : (tail_pts * BP >= 64 ? ~0ull : ((1ull << (tail_pts * BP)) - 1));
    const int top_shift = BP * (L - 1);
    const int pair_words = top_shift - 6;              // log2 of the bitmap words of one pair
    const unsigned long long lane_le = (lane == 63u) ? ~0ull : ((2ull << lane) - 1ull);   // lanes 0..lane
    const bool q32 = (a.qmask & 0xffffffffull) == 0ull;   // the quantised |w|^2 fits its high word

    // the workgroup's sums over its chunks, per wave (row sums of rho by pair,
    // dropped |w|, survivors), added chunk by chunk in chunk order
    if (i < kWavesD * 4 * 8) (&s.wrho[0][0][0])[i] = 0.0;
    if (i < kWavesD) {
        s.wdrop[i] = 0.0;
        s.wsurv[i] = 0u;
    }

    for (;;) {
        // ---- fetch the next chunk's parents now; they arrive while this chunk computes
        const unsigned int c1 = c + G;
        const bool has_next = c1 < n_chunks;
        DParent nxt = cur;
        __syncthreads();                                   // the chunk before is done with the LDS
        if (i < P * kOutWin) flush_bits(a, s, i, pair_words);
        if (has_next) {
            store_window_d(s, wn, i);
            __syncthreads();                               // (also publishes the tables)
            nxt = fetch_parent_d(a, s, c1, N, i, lane);
            if (c1 + G < n_chunks) wn = load_window_d(a, d_after, n_nz, N, i);
            d_after = (c1 + 2 * G < n_chunks) ? a.desc[c1 + 2 * G] : 0u;
        }

        // ---- this chunk: groups [g0, g0 + 256) loaded, segment heads [g0, g0 + H) owned;
        //      for all but the last chunk H = C and positions >= H lie in the last wave
        const unsigned int g0 = c * (unsigned int)C;
        const int H = (int)min((unsigned int)C, N - g0);
        const bool valid = cur.key != ~0ull;
        const unsigned long long key = cur.key, tail = cur.tail;
        const double2 W = cur.w;
        const unsigned long long up_key = (unsigned long long)__shfl_up((long long)key, 1, 64);
        const unsigned long long pk = lane == 0u ? cur.pkey : up_key;
        const bool head = valid && (g0 + i == 0u || (key >> BP) != (pk >> BP));
        const unsigned long long hm = __ballot(head), vm = __ballot(valid);
        if (lane == 0u) {
            s.hmask[wave] = hm;
            s.vmask[wave] = vm;
        }
        if (i == 0) s.obase = valid ? (key >> BP) >> 6 : 0ull;   // the chunk's first output word
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
            const unsigned long long stop_hi = wave + 1 < kWavesD ? (s.hmask[wave + 1] | ~s.vmask[wave + 1]) : ~0ull;
            const unsigned long long after = lane == 63u ? stop_hi : ((stop_lo >> (lane + 1)) | (stop_hi << (63 - lane)));
            len = 1 + (after ? __builtin_ctzll(after) : 64);
            if (len > P) len = P;
        }

        // ---- extend: influence sums of the parent over lags 1..dmax
        double rho_v[2 * P];
#pragma unroll
        for (int k = 0; k < 2 * P; ++k) rho_v[k] = 0.0;
        double dropped = 0.0;
        unsigned int surv_bits = 0;
        unsigned long long ctail = 0;
        if (owned) {
            double A = 0.0, B = 0.0, Ac = 0.0, Bc = 0.0;
            if (use_tabs) {
                for (int q = 0; q < nk; ++q) {
                    const int st = kTabPtsD * q, ln = min(kTabPtsD, L - st);
                    const int v = (int)((key >> (BP * (L - st - ln))) & ((1ull << (BP * ln)) - 1));
                    A += s.tab[q][v][0];
                    B += s.tab[q][v][1];
                    Ac += s.tab[q][v][2];
                    Bc += s.tab[q][v][3];
                }
                for (int q = nk; q < nk + nt; ++q) {
                    const int st = L + kTabPtsD * (q - nk), ln = min(kTabPtsD, K - st);
                    const int v = (int)((tail >> (BP * (st - L))) & ((1ull << (BP * ln)) - 1));
                    A += s.tab[q][v][0];
                    B += s.tab[q][v][1];
                    Ac += s.tab[q][v][2];
                    Bc += s.tab[q][v][3];
                }
            } else {
                for (int d = 1; d <= dmax; ++d) {
                    const int ps = d - 1;
                    const unsigned int x = ps < L ? (unsigned int)((key >> (BP * (L - 1 - ps))) & DM)
                                                  : (unsigned int)((tail >> (BP * (ps - L))) & DM);
                    const double dsx = s.ds[x], ssx = s.ss[x];
                    A = __builtin_fma(s.cre[d], dsx, A);
                    B = __builtin_fma(s.cim[d], ssx, B);
                    Ac = __builtin_fma(s.dre[d], dsx, Ac);
                    Bc = __builtin_fma(s.dim[d], ssx, Bc);
                }
            }
            const int h0 = (int)(key >> top_shift);
            ctail = ((tail << BP) | (key & DM)) & tail_mask;
            // pairs (0,1) and (1,0) have ds = +D, -D and equal ss: their exponents are
            // mirror images and share one exp and one sincos; pairs (0,0), (1,1) have ds = 0
            const double D = s.ds[1], Sg = s.ss[1];
            const double x = D * A, y = D * __builtin_fma(s.cim[0], Sg, B);
            const double xc = D * Ac, yc = D * __builtin_fma(s.dim[0], Sg, Bc);
            const double ex = exp_fast(x), exc = exp_fast(xc);
            const double iex = recip(ex), iexc = recip(exc);
            double sy, cy, syc, cyc;
            sincos_fast(y, &sy, &cy);
            sincos_fast(yc, &syc, &cyc);
            const double e0 = s.e0, f0 = s.f0;    // exp(-D^2 Re c_0), exp(-D^2 Re delta_0)
            double er[P], ei[P], fr[P], fi[P];
            er[0] = 1.0; ei[0] = 0.0; fr[0] = 1.0; fi[0] = 0.0;
            er[3] = 1.0; ei[3] = 0.0; fr[3] = 1.0; fi[3] = 0.0;
            er[1] = e0 * iex * cy;  ei[1] = -(e0 * iex * sy);
            er[2] = e0 * ex * cy;   ei[2] = e0 * ex * sy;
            fr[1] = f0 * iexc * cyc; fi[1] = -(f0 * iexc * syc);
            fr[2] = f0 * exc * cyc;  fi[2] = f0 * exc * syc;
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
                    rho_v[2 * p] = wr2 * fr[p] - wi2 * fi[p];
                    rho_v[2 * p + 1] = wr2 * fi[p] + wi2 * fr[p];
                } else {
                    dropped += sqrt(n2);
                }
                s.cw[p][i] = make_double2(wr2, wi2);
                s.cq[p][i] = (unsigned int)(((unsigned long long)__double_as_longlong(n2) & a.qmask) >> 32);
            }
        }
        s.surv[i] = surv_bits;
        s.ctail[i] = ctail;
        {
            // this chunk's rho, dropped |w| and survivors, added to the wave's sums
            double x0, x1;
            row_sums8(rho_v, lane, x0, x1);
            if ((lane & 15u) >= 12u) {
                const unsigned int r = lane & 3u;
                const int k = 4 * (int)(r & 1u) + 2 * (int)(r >> 1);
                s.wrho[wave][lane >> 4][k] += x0;
                s.wrho[wave][lane >> 4][k + 1] += x1;
            }
            const double dsum = wave_sum(dropped);
            unsigned int ns = 0u;
#pragma unroll
            for (int p = 0; p < P; ++p) ns += (unsigned int)__popcll(__ballot((surv_bits >> p) & 1u));
            if (lane == 0u) {
                s.wdrop[wave] += dsum;
                s.wsurv[wave] += ns;
            }
        }
        __syncthreads();

        // ---- merge each segment per pair (sum of the surviving weights and the
        //      representative), write the merged group to its slot, set its bit
        unsigned int msurv[P];
        unsigned long long mtail[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int j = min(i + m, kDenseThreads - 1);
            msurv[m] = m < len ? s.surv[j] : 0u;
            mtail[m] = s.ctail[j];
        }
#pragma unroll 1
        for (int p = 0; p < P; ++p) {
            bool any = false;
            double sr = 0.0, si = 0.0;
            unsigned long long bq = 0, bt = 0;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                if (!((msurv[m] >> p) & 1u)) continue;
                const int j = min(i + m, kDenseThreads - 1);
                const double2 w = s.cw[p][j];
                sr += w.x;
                si += w.y;
                const unsigned long long q =
                    q32 ? ((unsigned long long)s.cq[p][j] << 32)
                        : ((unsigned long long)__double_as_longlong(norm2_nocontract(w.x, w.y)) & a.qmask);
                if (!any || q > bq || (q == bq && mtail[m] < bt)) { bq = q; bt = mtail[m]; }
                any = true;
            }
            const unsigned long long so = ((unsigned long long)p << top_shift) | (key >> BP);
            if (any) {
                a.tail_out[so] = bt;
                a.w_out[so] = make_double2(sr, si);
            }
            // its bit: into the chunk's window of output words, or straight to the bitmap
            if (any) {
                const unsigned long long wi = (key >> BP) >> 6, idx = wi - s.obase;
                const unsigned long long bit = 1ull << ((key >> BP) & 63ull);
                if (idx < (unsigned long long)kOutWin) atomicOr(&s.obits[p][idx], bit);
                else atomicOr(a.bits_out + (((unsigned long long)p << pair_words) | wi), bit);
            }
        }
        if (!has_next) break;
        cur = nxt;
        c = c1;
    }
    __syncthreads();
    if (i < P * kOutWin) flush_bits(a, s, i, pair_words);

    // ---- the workgroup's sums: rows and waves in order
    if (i < S) {
        double v = 0.0;
        if (i < 2 * P) {
            for (int w = 0; w < kWavesD; ++w)
                for (int r = 0; r < 4; ++r) v += s.wrho[w][r][i];
        } else if (i == 2 * P) {
            for (int w = 0; w < kWavesD; ++w) v += s.wdrop[w];
        } else {
            unsigned int ns = 0u;
            for (int w = 0; w < kWavesD; ++w) ns += s.wsurv[w];
            v = (double)ns;
        }
        a.partials[(size_t)i * G + blockIdx.x] = v;
    }
}

}  // namespace

int dense_chunk_heads() { return kC; }

int dense_step_grid(int n_cu) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dense_step, kDenseThreads, 0) != hipSuccess || nb < 1)
        return 0;
    return nb * n_cu;
}

int launch_dense_step(const DenseArgs& a, int grid, void* stream) {
    hipLaunchKernelGGL(dense_step, dim3(grid), dim3(kDenseThreads), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_dense_plan(const DensePlanArgs& a, void* stream) {
    const int grid = (int)((a.n_words + kDenseRegion - 1) / kDenseRegion) + 1;
    hipLaunchKernelGGL(dense_plan, dim3(grid), dim3(kDensePlanThreads), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

}  // namespace quapi_dev
