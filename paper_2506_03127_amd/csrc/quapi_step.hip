// One time step of the MACGIC-iQUAPI path propagation as a single HIP kernel
// for gfx950 (wave64).
//
// State between steps: the groups the next step extends, kept as P sorted runs
// ("classes", one per value of the newest point).  A group is a merge key
// (points 0..L-1 of its history, point 0 in the top bits), the rest of the
// representative's history (points L..K-1) and the group amplitude.  The
// merge positions are 0..L-1: L = E-1 for pre-merging on the reduced mask
// {mask[i]-1} of a contiguous mask {0..E-1} (Sec. 3.1), L = E for
// post-merging on the mask (Sec. 2.1).
//
// Why one kernel suffices: a child of group g by pair p has key
// (p, points 0..L-2 of g), so the children that merge are the children, by
// the same p, of the groups that agree on points 0..L-2 -- at most P
// consecutive entries of a class run (they differ only in point L-1, the
// lowest digit).  For each p those children land in class p, in the order of
// their parents.  So each step is: read the runs in order, extend each
// parent by every pair (eq. SysP propagator element times the influence factor
// of eq. inf_fun), drop children below theta (Sec. 2.1), merge each segment of
// consecutive parents per p (sum of weights; representative of largest
// quantised |w|^2, ties to the smaller history read from the oldest point;
// Sec. 3.1.2), and append the merged groups to output run p.  rho(t) collects
// the survivors with the end-point correction of the final point
// (Sec. 3.2.1).  Output positions come from a wave-ballot compaction inside
// the tile plus a decoupled look-back over tiles; tiles are taken in order
// from an atomic counter by a persistent grid, so a tile only ever waits on
// tiles already owned by running workgroups.
//
// Determinism: the merge sums in parent order; rho(t) and the counters are
// summed per tile in a fixed order and then over tiles in tile order by the
// last workgroup to finish.

#include <hip/hip_runtime.h>

#include "quapi_host.h"

namespace quapi_dev {

namespace {

constexpr int kWaves = kThreads / 64;
constexpr unsigned long long kStatusAgg = 1ull << 30;
constexpr unsigned long long kStatusIncl = 2ull << 30;
constexpr unsigned long long kValueMask = (1ull << 30) - 1;
constexpr unsigned int kSpinLimit = 1u << 22;

__device__ inline double norm2_nocontract(double re, double im) {
#pragma clang fp contract(off)
    const double a = re * re;
    const double b = im * im;
    return a + b;
}

__device__ inline unsigned int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ inline unsigned int rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned int)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned int)mask, 0u));
}

__device__ inline unsigned long long ld_status(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_status(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

template <int P>
struct Lds {
    double k4re[P * P], k4im[P * P];
    double ds[P], ss[P];
    double cre[kMaxK + 1], cim[kMaxK + 1], dre[kMaxK + 1], dim[kMaxK + 1];
    double2 cw[P][kThreads];               // child weights; reused for the final reduction
    unsigned long long key[kThreads];
    unsigned long long ctail[kThreads];
    unsigned int surv[kThreads];           // bit p: child p survives
    unsigned char flags[kThreads];         // bit 0 valid, bit 1 segment head
    unsigned int wcount[kWaves][P];
    unsigned int excl[P];
    double2 wrho[kWaves][P];
    double wdrop[kWaves];
    unsigned long long wsurv[kWaves];
    double fdrop[kThreads];
    unsigned long long fsurv[kThreads];
    int tile;
    int last;
};

template <int P>
__device__ void finalize(const StepArgs& a, Lds<P>& s, int n_tiles, unsigned long long n_groups) {
    const int i = threadIdx.x;
    // sum the tile partials in tile order: thread i takes tiles i, i+256, ...
    double acc[2 * P];
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) acc[k] = 0.0;
    double drop = 0.0;
    unsigned long long ns = 0;
    for (int tl = i; tl < n_tiles; tl += kThreads) {
        const TilePartial& tp = a.partials[tl];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            acc[2 * k] += tp.rho[k].x;
            acc[2 * k + 1] += tp.rho[k].y;
        }
        drop += tp.dropped;
        ns += tp.n_surv;
    }
    double* buf = reinterpret_cast<double*>(&s.cw[0][0]);   // 2P x kThreads doubles
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) buf[k * kThreads + i] = acc[k];
    s.fdrop[i] = drop;
    s.fsurv[i] = ns;
    __syncthreads();
    for (int half = kThreads / 2; half > 0; half >>= 1) {
        if (i < half) {
#pragma unroll
            for (int k = 0; k < 2 * P; ++k) buf[k * kThreads + i] += buf[k * kThreads + i + half];
            s.fdrop[i] += s.fdrop[i + half];
            s.fsurv[i] += s.fsurv[i + half];
        }
        __syncthreads();
    }
    if (i < P) a.rho_out[i] = make_double2(buf[(2 * i) * kThreads], buf[(2 * i + 1) * kThreads]);
    if (i == 0) {
        unsigned long long stored = 0;
        bool overflow = false;
        for (int c = 0; c < P; ++c) {
            unsigned long long v = 0;
            if (n_tiles > 0) v = ld_status(&a.status[(size_t)c * a.max_tiles + (n_tiles - 1)]) & kValueMask;
            if ((long long)v > a.cap) { overflow = true; v = (unsigned long long)a.cap; }
            a.out_count[c] = (unsigned int)v;
            stored += v;
        }
        StepStatsDev st;
        st.n_groups = n_groups;
        st.n_children = n_groups * (unsigned long long)P;
        st.n_survivors = s.fsurv[0];
        st.n_stored = stored;
        st.dropped_abs = s.fdrop[0];
        st.pad = 0.0;
        *a.stats_out = st;
        if (overflow) {
            atomicCAS(&a.error[0], kErrNone, kErrOverflow);
            a.error[1] = (unsigned int)a.t;
        }
        // counters of the next step start from zero
        const int nxt = (a.epoch + 1) & 1;
        a.counters[nxt] = 0u;
        a.counters[2 + nxt] = 0u;
        __threadfence();
    }
}

template <int P, int BP>
__global__ __launch_bounds__(kThreads) void step_kernel(const StepArgs a) {
    constexpr int C = kThreads - (P - 1);              // segment heads per tile
    constexpr unsigned long long DM = (1ull << BP) - 1;
    __shared__ Lds<P> s;
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();

    if (__hip_atomic_load(&a.error[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone) return;

    // ---- tables and the coefficients of this step
    for (int k = i; k < P * P; k += kThreads) {
        s.k4re[k] = a.tables[2 * k];
        s.k4im[k] = a.tables[2 * k + 1];
    }
    if (i < P) {
        s.ds[i] = a.tables[TableLayout::ds(P) + i];
        s.ss[i] = a.tables[TableLayout::ss(P) + i];
    }
    const int K = a.K, L = a.L, t = a.t;
    if (i <= K) {
        const double* eta = a.tables + TableLayout::eta(P);
        const int n = K + 1;
        const int d = i;
        const double ir = eta[2 * d], ii = eta[2 * d + 1];
        const double hr = eta[2 * (n + d)], hi = eta[2 * (n + d) + 1];
        const double xr = eta[2 * (2 * n + d)], xi = eta[2 * (2 * n + d) + 1];
        double cr = 0, ci = 0, dr = 0, di = 0;
        if (d <= t) {
            if (d == t) { cr = hr; ci = hi; } else { cr = ir; ci = ii; }   // time-0 partner: half window
            if (d == 0) { dr = hr - ir; di = hi - ii; }                     // final point self term
            else if (d == t) { dr = xr - hr; di = xi - hi; }                 // final x initial
            else { dr = hr - ir; di = hi - ii; }                             // final x interior
        }
        s.cre[d] = cr; s.cim[d] = ci; s.dre[d] = dr; s.dim[d] = di;
    }

    // ---- tiling of the input runs
    unsigned int cnt[P];
    int tpre[P + 1];
    tpre[0] = 0;
    unsigned long long n_groups = 0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        cnt[c] = a.in_count[c];
        n_groups += cnt[c];
        tpre[c + 1] = tpre[c] + (int)((cnt[c] + C - 1) / C);
    }
    const int n_tiles = tpre[P];
    __syncthreads();
    if (n_tiles == 0) {
        if (blockIdx.x == 0) finalize<P>(a, s, 0, 0);
        return;
    }

    const int dmax = t < K ? t : K;
    const int tail_pts = K - L;
    const unsigned long long tail_mask =
        tail_pts <= 0 ? 0ull : (tail_pts * BP >= 64 ? ~0ull : ((1ull << (tail_pts * BP)) - 1));
    const int top_shift = BP * (L - 1);
    unsigned int* tile_ctr = &a.counters[a.epoch & 1];
    unsigned int* done_ctr = &a.counters[2 + (a.epoch & 1)];

    for (;;) {
        if (i == 0) s.tile = (int)atomicAdd(tile_ctr, 1u);
        __syncthreads();
        const int tile = s.tile;
        if (tile >= n_tiles) break;
        int c = 0, tbase = 0;
        long long n = 0;
#pragma unroll
        for (int k = 1; k < P; ++k) c += (tile >= tpre[k]) ? 1 : 0;
#pragma unroll
        for (int k = 0; k < P; ++k)
            if (k == c) { tbase = tpre[k]; n = cnt[k]; }
        const long long start = (long long)(tile - tbase) * C;
        const size_t base = (size_t)c * (size_t)a.cap;
        const long long j = start + i;
        const bool valid = j < n;

        // ---- load the parent and find segment heads
        unsigned long long key = ~0ull, tail = 0;
        double2 W = make_double2(0.0, 0.0);
        if (valid) {
            key = a.in.key[base + j];
            tail = a.in.tail[base + j];
            W = a.in.w[base + j];
        }
        s.key[i] = key;
        unsigned long long prev_key = ~0ull;
        if (i == 0 && start > 0) prev_key = a.in.key[base + start - 1];
        __syncthreads();
        if (i > 0) prev_key = s.key[i - 1];
        const bool head = valid && (j == 0 || (key >> BP) != (prev_key >> BP));
        s.flags[i] = (unsigned char)((valid ? 1 : 0) | (head ? 2 : 0));
        __syncthreads();
        // a parent belongs to this tile when its segment head does
        bool owned = false;
        if (valid) {
            if (i < C) {
                for (int k = i; k >= 0 && k > i - P; --k)
                    if (s.flags[k] & 2) { owned = true; break; }
            } else {
                owned = true;
                for (int k = C; k <= i; ++k)
                    if (s.flags[k] & 2) { owned = false; break; }
            }
        }

        // ---- extend: influence sums of the parent over lags 1..dmax
        double rho_re[P], rho_im[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { rho_re[p] = 0.0; rho_im[p] = 0.0; }
        double dropped = 0.0;
        unsigned int n_surv = 0, surv_bits = 0;
        unsigned long long ctail = 0;
        if (owned) {
            double A = 0.0, B = 0.0, Ac = 0.0, Bc = 0.0;
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
            const int h0 = (int)(key >> top_shift);
            ctail = ((tail << BP) | (key & DM)) & tail_mask;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const double k4r = s.k4re[p * P + h0], k4i = s.k4im[p * P + h0];
                const double br = W.x * k4r - W.y * k4i;
                const double bi = W.x * k4i + W.y * k4r;
                const double dsp = s.ds[p], ssp = s.ss[p];
                double wr = br, wi = bi, fr = 1.0, fi = 0.0;
                if (dsp != 0.0) {
                    const double pr = -dsp * (s.cre[0] * dsp + A);
                    const double pi = -dsp * (s.cim[0] * ssp + B);
                    const double e = exp(pr);
                    double sn, cs;
                    sincos(pi, &sn, &cs);
                    const double er = e * cs, ei = e * sn;
                    wr = br * er - bi * ei;
                    wi = br * ei + bi * er;
                    const double qr = -dsp * (s.dre[0] * dsp + Ac);
                    const double qi = -dsp * (s.dim[0] * ssp + Bc);
                    const double f = exp(qr);
                    double fs, fc;
                    sincos(qi, &fs, &fc);
                    fr = f * fc;
                    fi = f * fs;
                }
                const double n2 = norm2_nocontract(wr, wi);
                const bool keep = (a.theta2 == 0.0) || !(n2 < a.theta2);
                if (keep) {
                    surv_bits |= 1u << p;
                    ++n_surv;
                    rho_re[p] = wr * fr - wi * fi;
                    rho_im[p] = wr * fi + wi * fr;
                } else {
                    dropped += sqrt(n2);
                }
                s.cw[p][i] = make_double2(wr, wi);
            }
        }
        s.surv[i] = surv_bits;
        s.ctail[i] = ctail;

        // ---- per-tile partials of rho, dropped weight and survivor count
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double r = rho_re[p], m = rho_im[p];
            for (int off = 32; off > 0; off >>= 1) {
                r += shfl_xor_d(r, off);
                m += shfl_xor_d(m, off);
            }
            if (lane == 0) s.wrho[wave][p] = make_double2(r, m);
        }
        {
            double d = dropped;
            unsigned long long ns = n_surv;
            for (int off = 32; off > 0; off >>= 1) {
                d += shfl_xor_d(d, off);
                ns += __shfl_xor(ns, off, 64);
            }
            if (lane == 0) { s.wdrop[wave] = d; s.wsurv[wave] = ns; }
        }
        __syncthreads();

        // ---- merge each segment per pair
        bool ov[P];
        double2 ow[P];
        unsigned long long otail[P];
        const unsigned char fl = s.flags[i];
        const bool is_head = (i < C) && (fl & 2);
        int len = 0;
        if (is_head) {
            len = 1;
            while (i + len < kThreads && len < P && (s.flags[i + len] & 1) && !(s.flags[i + len] & 2)) ++len;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            bool any = false;
            double sr = 0.0, si = 0.0;
            unsigned long long bq = 0, bt = 0;
            for (int m = 0; m < len; ++m) {
                if (!((s.surv[i + m] >> p) & 1u)) continue;
                const double2 w = s.cw[p][i + m];
                sr += w.x;
                si += w.y;
                const unsigned long long q =
                    (unsigned long long)__double_as_longlong(norm2_nocontract(w.x, w.y)) & a.qmask;
                const unsigned long long ct = s.ctail[i + m];
                if (!any || q > bq || (q == bq && ct < bt)) { bq = q; bt = ct; }
                any = true;
            }
            ov[p] = any;
            ow[p] = make_double2(sr, si);
            otail[p] = bt;
        }

        // ---- compaction: wave ballot per output run, then block prefix
        unsigned int lrank[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const unsigned long long bal = __ballot(ov[p]);
            lrank[p] = rank_below(bal);
            if (lane == 0) s.wcount[wave][p] = (unsigned int)__popcll(bal);
        }
        __syncthreads();
        if (i == 0) {
            TilePartial tp;
            double drop = 0.0;
            unsigned long long ns = 0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                double r = 0.0, m = 0.0;
                for (int w = 0; w < kWaves; ++w) { r += s.wrho[w][p].x; m += s.wrho[w][p].y; }
                tp.rho[p] = make_double2(r, m);
            }
            for (int p = P; p < kMaxP; ++p) tp.rho[p] = make_double2(0.0, 0.0);
            for (int w = 0; w < kWaves; ++w) { drop += s.wdrop[w]; ns += s.wsurv[w]; }
            tp.dropped = drop;
            tp.n_surv = ns;
            a.partials[tile] = tp;
        }
        // ---- decoupled look-back over tiles, one lane per output run
        if (wave == 0 && (int)lane < P) {
            const int p = (int)lane;
            unsigned int agg = 0;
            for (int w = 0; w < kWaves; ++w) agg += s.wcount[w][p];
            unsigned long long* st = a.status + (size_t)p * a.max_tiles;
            const unsigned long long ep = (unsigned long long)a.epoch << 32;
            unsigned long long excl = 0;
            if (tile == 0) {
                st_status(&st[0], ep | kStatusIncl | agg);
            } else {
                st_status(&st[tile], ep | kStatusAgg | agg);
                int k = tile - 1;
                unsigned int spins = 0;
                for (;;) {
                    const unsigned long long v = ld_status(&st[k]);
                    if ((v >> 32) != (unsigned long long)a.epoch || (v & (3ull << 30)) == 0) {
                        if (++spins > kSpinLimit) {
                            atomicCAS(&a.error[0], kErrNone, kErrSpin);
                            a.error[1] = (unsigned int)t;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    excl += v & kValueMask;
                    if (v & kStatusIncl) break;
                    --k;
                }
                st_status(&st[tile], ep | kStatusIncl | ((excl + agg) & kValueMask));
            }
            s.excl[p] = (unsigned int)excl;
        }
        __syncthreads();

        // ---- write merged groups to their runs
#pragma unroll
        for (int p = 0; p < P; ++p) {
            if (!ov[p]) continue;
            unsigned long long idx = s.excl[p] + lrank[p];
            for (int w = 0; w < wave; ++w) idx += s.wcount[w][p];
            if ((long long)idx >= a.cap) {
                atomicCAS(&a.error[0], kErrNone, kErrOverflow);
                a.error[1] = (unsigned int)t;
                continue;
            }
            const size_t o = (size_t)p * (size_t)a.cap + idx;
            a.out.key[o] = ((unsigned long long)p << top_shift) | (key >> BP);
            a.out.tail[o] = otail[p];
            a.out.w[o] = ow[p];
        }

        // ---- tile done; the last one reduces the partials
        __syncthreads();
        if (i == 0) {
            __threadfence();
            const unsigned int prev = atomicAdd(done_ctr, 1u);
            s.last = (prev == (unsigned int)(n_tiles - 1)) ? 1 : 0;
        }
        __syncthreads();
        if (s.last) {
            __threadfence();
            finalize<P>(a, s, n_tiles, n_groups);
            __syncthreads();
        }
    }
}

}  // namespace

int tile_heads(int P) { return kThreads - (P - 1); }

int max_tiles_for(int P, long long cap) {
    const long long C = tile_heads(P);
    return (int)(P * ((cap + C - 1) / C));
}

int launch_step(const StepArgs& a, int grid, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (a.P) {
        case 4: hipLaunchKernelGGL((step_kernel<4, 2>), dim3(grid), dim3(kThreads), 0, st, a); break;
        case 9: hipLaunchKernelGGL((step_kernel<9, 4>), dim3(grid), dim3(kThreads), 0, st, a); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace quapi_dev
