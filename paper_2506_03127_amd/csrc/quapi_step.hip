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
// Planner (between steps): prefix sum of the bucket sizes, so that the next
// step can cut its input into full chunks of consecutive groups regardless
// of bucket boundaries; it also zeroes the next bucket sizes, resets the
// chunk ticket and reduces the finished step's per-chunk sums of rho(t) and
// counters in chunk order (deterministic).
//
// Step: persistent workgroups take chunks in order.  A chunk extends each
// parent by every pair (eq. SysP propagator element times the influence
// factor of eq. inf_fun), drops children below theta (Sec. 2.1), merges each
// segment of consecutive parents per p (sum of weights; representative of
// largest quantised |w|^2, ties to the smaller history read from the oldest
// point; Sec. 3.1.2), ranks the merged groups per output bucket with wave
// ballots and a segmented block scan, and writes them.  rho(t) collects the
// survivors with the end-point correction of the final point (Sec. 3.2.1).
// A super-bucket cut by a chunk boundary continues at the offsets published
// by the chunk before it; only such chunks wait, and only on that one chunk.

#include <hip/hip_runtime.h>

#include "quapi_host.h"

namespace quapi_dev {

namespace {

constexpr int kWaves = kThreads / 64;
constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
constexpr int kWindow = 512;          // prefix entries cached per chunk for the bucket lookup
constexpr int kTabPts = 3;            // points per subset-sum table (two-level systems)
constexpr int kTabEntries = 64;       // 4^3
constexpr int kMaxTabs = 10;
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

// 1/x from the hardware estimate and two Newton steps
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ inline unsigned long long ld_relaxed(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_relaxed(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The error word holds (failing step << 4) | code; the first error wins.
__device__ inline void raise_error(unsigned int* err, int t, unsigned int code) {
    atomicCAS(err, 0u, ((unsigned int)t << 4) | code);
}

__device__ inline unsigned int error_word(const unsigned int* err) {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ planner
template <int P>
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(const PlanArgs a) {
    constexpr int S = partial_stride(P);
    __shared__ unsigned int wsum[kPlanWaves];
    __shared__ double wred[kPlanWaves][S];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const long long NB = a.n_buckets;
    const long long per = (NB + kPlanThreads - 1) / kPlanThreads;
    const long long b_lo = (long long)i * per < NB ? (long long)i * per : NB;
    const long long b_hi = b_lo + per < NB ? b_lo + per : NB;

    // ---- exclusive prefix of the bucket sizes
    unsigned int mine = 0;
    for (long long b = b_lo; b < b_hi; ++b) mine += a.counts[b];
    unsigned int incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned int v = __shfl_up(incl, off, 64);
        if ((int)lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    unsigned int base = incl - mine;
    for (int w = 0; w < wave; ++w) base += wsum[w];
    unsigned int total = 0;
    for (int w = 0; w < kPlanWaves; ++w) total += wsum[w];
    const unsigned int C = (unsigned int)a.chunk_heads;
    unsigned int run = base;
    for (long long b = b_lo; b < b_hi; ++b) {
        const unsigned int n = a.counts[b];
        a.prefix[b] = run;
        if (n) {
            // chunk c starts in bucket b when c*C lies in [run, run+n); the
            // group before it (c*C - 1) lies in b when c*C lies in [run+1, run+n]
            for (unsigned int c = (run + C - 1) / C; c * C < run + n; ++c)
                if ((int)c < a.max_chunks) a.chunk_start[2 * c] = (unsigned int)b;
            for (unsigned int c = run / C + 1; c * C <= run + n; ++c)
                if ((int)c < a.max_chunks) a.chunk_start[2 * c + 1] = (unsigned int)b;
        }
        run += n;
        a.counts_next[b] = 0u;
    }
    if (i == kPlanThreads - 1) a.prefix[NB] = total;

    // ---- counters and rho(t) of the step just finished, summed in chunk order
    const unsigned int err = error_word(a.error);
    const bool reduce = a.reduce_t > 0 && (err == 0u || (int)(err >> 4) > a.reduce_t);
    if (reduce) {
        const unsigned int nc = a.plan_prev->n_chunks;
        double acc[S];
#pragma unroll
        for (int k = 0; k < S; ++k) acc[k] = 0.0;
        for (unsigned int c = i; c < nc; c += kPlanThreads)
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] += a.partials[(size_t)c * S + k];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            double v = acc[k];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) wred[wave][k] = v;
        }
    }
    __syncthreads();
    if (reduce && i == 0) {
        double sum[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            sum[k] = 0.0;
            for (int w = 0; w < kPlanWaves; ++w) sum[k] += wred[w][k];
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
            a.rho_hist[(size_t)a.reduce_t * P + p] = make_double2(sum[2 * p], sum[2 * p + 1]);
        StepStatsDev st;
        st.n_groups = a.plan_prev->n_groups;
        st.n_children = st.n_groups * (unsigned long long)P;
        st.n_survivors = (unsigned long long)sum[2 * P + 1];
        st.n_stored = total;
        st.dropped_abs = sum[2 * P];
        st.pad = 0.0;
        a.stats_hist[a.reduce_t] = st;
    }
    if (i == 0) {
        Plan pl;
        pl.n_groups = total;
        pl.n_chunks = (total + C - 1) / C;
        pl.counter = 0u;
        pl.pad = 0u;
        *a.plan = pl;
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
    unsigned long long key[kThreads];
    unsigned long long ctail[kThreads];
    unsigned int surv[kThreads];           // bit p: child p survives
    unsigned int sig[kThreads];            // super-bucket of each loaded parent
    unsigned int excl[P][kThreads + 1];    // block-exclusive prefix of the output flags
    unsigned int win[kWindow + 1];         // prefix window of the chunk
    unsigned char flags[kThreads];         // bit 0 valid, bit 1 segment head
    unsigned int wcount[kWaves][P];
    int wstart[kWaves];                    // last super-bucket run start in each wave
    unsigned int base[P];                  // offsets of the first run when it continues a chunk
    double2 wrho[kWaves][P];
    double wdrop[kWaves];
    double wsurv[kWaves];
    unsigned long long prev_key;
    double e0, f0;
    int chunk, prev_sig;
};

template <int P, int BP>
__global__ __launch_bounds__(kThreads) void step_kernel(const StepArgs a) {
    constexpr int C = kThreads - (P - 1);              // segment heads per full chunk
    constexpr int S = partial_stride(P);
    constexpr unsigned long long DM = (1ull << BP) - 1;
    __shared__ Lds<P> s;
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();

    if (error_word(a.error) != 0u) return;             // an earlier step failed: leave the state alone

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
    for (int k = i; k < 4 * (K + 1); k += kThreads) {
        const int r = k / (K + 1), d = k - r * (K + 1);
        double* dst = r == 0 ? s.cre : r == 1 ? s.cim : r == 2 ? s.dre : s.dim;
        dst[d] = a.coef[k];
    }
    const int nk = (L + kTabPts - 1) / kTabPts, nt = (K - L + kTabPts - 1) / kTabPts;
    const bool use_tabs = (P == 4) && (nk + nt <= kMaxTabs);
    __syncthreads();
    if constexpr (P == 4) {
        if (use_tabs) {
            // tab[q][v] = sum over the points of table q of coefficient(lag) * (ds, ss)(point)
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

    const unsigned int N = a.plan->n_groups;
    const unsigned int n_chunks = a.plan->n_chunks;
    const int dmax = t < K ? t : K;
    const int tail_pts = K - L;
    const unsigned long long tail_mask =
        tail_pts <= 0 ? 0ull : (tail_pts * BP >= 64 ? ~0ull : ((1ull << (tail_pts * BP)) - 1));
    const int top_shift = BP * (L - 1);
    const unsigned long long ep = (unsigned long long)a.epoch << 32;

    for (;;) {
        __syncthreads();
        if (i == 0) s.chunk = (int)atomicAdd(&a.plan->counter, 1u);
        __syncthreads();
        const int c = s.chunk;
        if (c >= (int)n_chunks) break;
        const unsigned int g0 = (unsigned int)c * C;
        const unsigned int nsz = min((unsigned int)kThreads, N - g0);
        const int H = (c == (int)n_chunks - 1) ? (int)nsz : C;   // heads owned by this chunk: [0, H)

        // ---- bucket lookup: prefix window from the chunk's first bucket
        const unsigned int b0 = a.chunk_start[2 * c];
        const int kw = (int)min((long long)kWindow, a.n_buckets - (long long)b0);
        for (int k = i; k <= kw; k += kThreads) s.win[k] = a.prefix[b0 + k];
        if (i == 0) {
            int psig = -1;
            unsigned long long pk = ~0ull;
            if (g0 > 0) {
                const unsigned int bp = a.chunk_start[2 * c + 1];   // bucket of group g0-1
                const unsigned int off = g0 - 1 - a.prefix[bp];
                pk = a.in.key[(size_t)bp * a.cap + off];
                psig = (int)(bp / P);
            }
            s.prev_key = pk;
            s.prev_sig = psig;
        }
        __syncthreads();
        const unsigned int g = g0 + i;
        const bool valid = i < (int)nsz;
        unsigned long long key = ~0ull, tail = 0;
        double2 W = make_double2(0.0, 0.0);
        unsigned int b = b0;
        if (valid) {
            if (g < s.win[kw]) {                              // largest k with win[k] <= g
                int lo = 0, hi = kw;                           // win[lo] <= g < win[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s.win[mid] <= g) lo = mid; else hi = mid;
                }
                b = b0 + lo;
            } else {                                           // beyond the window: search the prefix
                long long lo = (long long)b0 + kw, hi = a.n_buckets;
                while (hi - lo > 1) {
                    const long long mid = (lo + hi) >> 1;
                    if (a.prefix[mid] <= g) lo = mid; else hi = mid;
                }
                b = (unsigned int)lo;
            }
            const unsigned int pb = ((int)(b - b0) <= kw) ? s.win[b - b0] : a.prefix[b];
            const size_t o = (size_t)b * (size_t)a.cap + (g - pb);
            key = a.in.key[o];
            tail = a.in.tail[o];
            W = a.in.w[o];
        }
        const unsigned int my_sig = valid ? b / P : 0xffffffffu;
        s.key[i] = key;
        s.sig[i] = my_sig;
        __syncthreads();
        const unsigned long long prev_key = i > 0 ? s.key[i - 1] : s.prev_key;
        const bool head = valid && (g == 0 || (key >> BP) != (prev_key >> BP));
        s.flags[i] = (unsigned char)((valid ? 1 : 0) | (head ? 2 : 0));
        __syncthreads();
        // a parent belongs to this chunk when its segment head does
        bool owned = false;
        if (valid) {
            if (i < H) {
                for (int k = i; k >= 0 && k > i - P; --k)
                    if (s.flags[k] & 2) { owned = true; break; }
            } else {
                owned = true;
                for (int k = H; k <= i; ++k)
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
            if (use_tabs) {
                for (int q = 0; q < nk; ++q) {
                    const int st = kTabPts * q, len = min(kTabPts, L - st);
                    const int v = (int)((key >> (BP * (L - st - len))) & ((1ull << (BP * len)) - 1));
                    A += s.tab[q][v][0];
                    B += s.tab[q][v][1];
                    Ac += s.tab[q][v][2];
                    Bc += s.tab[q][v][3];
                }
                for (int q = nk; q < nk + nt; ++q) {
                    const int st = L + kTabPts * (q - nk), len = min(kTabPts, K - st);
                    const int v = (int)((tail >> (BP * (st - L))) & ((1ull << (BP * len)) - 1));
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
                const double ex = exp(x), exc = exp(xc);
                const double iex = recip(ex), iexc = recip(exc);
                double sy, cy, syc, cyc;
                sincos(y, &sy, &cy);
                sincos(yc, &syc, &cyc);
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
                        const double e = exp(-dsp * (s.cre[0] * dsp + A));
                        double sn, cs;
                        sincos(-dsp * (s.cim[0] * ssp + B), &sn, &cs);
                        er[p] = e * cs;
                        ei[p] = e * sn;
                        const double f = exp(-dsp * (s.dre[0] * dsp + Ac));
                        double fs, fc;
                        sincos(-dsp * (s.dim[0] * ssp + Bc), &fs, &fc);
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
                const double wr = br * er[p] - bi * ei[p];
                const double wi = br * ei[p] + bi * er[p];
                const double n2 = norm2_nocontract(wr, wi);
                const bool keep = (a.theta2 == 0.0) || !(n2 < a.theta2);
                if (keep) {
                    surv_bits |= 1u << p;
                    ++n_surv;
                    rho_re[p] = wr * fr[p] - wi * fi[p];
                    rho_im[p] = wr * fi[p] + wi * fr[p];
                } else {
                    dropped += sqrt(n2);
                }
                s.cw[p][i] = make_double2(wr, wi);
            }
        }
        s.surv[i] = surv_bits;
        s.ctail[i] = ctail;

        // ---- partial sums of rho, dropped weight and survivor count
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double r = rho_re[p], m = rho_im[p];
            for (int off = 32; off > 0; off >>= 1) {
                r += __shfl_xor(r, off, 64);
                m += __shfl_xor(m, off, 64);
            }
            if (lane == 0) s.wrho[wave][p] = make_double2(r, m);
        }
        {
            double d = dropped, ns = (double)n_surv;
            for (int off = 32; off > 0; off >>= 1) {
                d += __shfl_xor(d, off, 64);
                ns += __shfl_xor(ns, off, 64);
            }
            if (lane == 0) { s.wdrop[wave] = d; s.wsurv[wave] = ns; }
        }
        __syncthreads();

        // ---- merge each segment per pair
        bool ov[P];
        double2 ow[P];
        unsigned long long otail[P];
        const bool is_head = (i < H) && (s.flags[i] & 2);
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

        // ---- ranks: block prefix of the output flags per pair, segmented by super-bucket
        const bool run_start = valid && (i == 0 || s.sig[i - 1] != my_sig);
        const unsigned long long rs_mask = __ballot(run_start);
        unsigned int lrank[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const unsigned long long bal = __ballot(ov[p]);
            lrank[p] = rank_below(bal);
            if (lane == 0) s.wcount[wave][p] = (unsigned int)__popcll(bal);
        }
        if (lane == 0) s.wstart[wave] = rs_mask ? wave * 64 + 63 - __builtin_clzll(rs_mask) : -1;
        __syncthreads();
#pragma unroll
        for (int p = 0; p < P; ++p) {
            unsigned int e = lrank[p];
            for (int w = 0; w < wave; ++w) e += s.wcount[w][p];
            s.excl[p][i] = e;
            if (i == kThreads - 1) s.excl[p][kThreads] = e + (ov[p] ? 1u : 0u);
        }
        // start of this parent's super-bucket run inside the chunk
        int start;
        {
            const unsigned long long le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
            const unsigned long long m = rs_mask & le;
            if (m) {
                start = wave * 64 + 63 - __builtin_clzll(m);
            } else {
                start = 0;
                for (int w = wave - 1; w >= 0; --w)
                    if (s.wstart[w] >= 0) { start = s.wstart[w]; break; }
            }
        }
        if (i < S) {                                           // this chunk's partial sums
            double v = 0.0;
            if (i < 2 * P) {
                const int p = i >> 1;
                for (int w = 0; w < kWaves; ++w) v += (i & 1) ? s.wrho[w][p].y : s.wrho[w][p].x;
            } else if (i == 2 * P) {
                for (int w = 0; w < kWaves; ++w) v += s.wdrop[w];
            } else {
                for (int w = 0; w < kWaves; ++w) v += s.wsurv[w];
            }
            a.partials[(size_t)c * S + i] = v;
        }
        __syncthreads();

        // ---- chain between chunks: the first run continues a super-bucket cut by the
        //      chunk boundary when the group before the chunk lies in the same one
        const bool first_cont = (g0 > 0) && (s.prev_sig == (int)s.sig[0]);
        const unsigned int last_sig = s.sig[H - 1];
        // publish this chunk's last-run totals; they are final unless that run is the
        // continued first run, which needs the previous chunk's totals first
        const bool last_needs_base = (i == H - 1) && first_cont && (start == 0);
        if (i == H - 1 && !last_needs_base) {
#pragma unroll
            for (int p = 0; p < P; ++p)
                st_relaxed(a.chain + (size_t)(1 + p) * a.max_chunks + c, ep | (s.excl[p][H] - s.excl[p][start]));
            st_relaxed(a.chain + c, ep | last_sig);
        }
        if (wave == 0) {
            unsigned int base_p = 0;
            if (first_cont && (int)lane < P) {
                const unsigned long long* cp = a.chain + (size_t)(1 + lane) * a.max_chunks + (c - 1);
                unsigned int spins = 0;
                for (;;) {
                    const unsigned long long v = ld_relaxed(cp);
                    if ((v >> 32) == (unsigned long long)a.epoch) { base_p = (unsigned int)(v & 0xffffffffu); break; }
                    if (++spins > kSpinLimit) { raise_error(a.error, t, kErrSpin); break; }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if ((int)lane < P) s.base[lane] = first_cont ? base_p : 0u;
        }
        __syncthreads();
        if (last_needs_base) {
#pragma unroll
            for (int p = 0; p < P; ++p)
                st_relaxed(a.chain + (size_t)(1 + p) * a.max_chunks + c,
                           ep | (s.excl[p][H] - s.excl[p][0] + s.base[p]));
            st_relaxed(a.chain + c, ep | last_sig);
        }

        // ---- write merged groups to the output buckets (p, sigma)
        const bool from_prev = (start == 0) && first_cont;
        if (is_head) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (!ov[p]) continue;
                const unsigned long long idx =
                    (unsigned long long)(s.excl[p][i] - s.excl[p][start]) + (from_prev ? s.base[p] : 0u);
                if ((long long)idx >= a.cap) {
                    raise_error(a.error, t, kErrOverflow);
                    continue;
                }
                const size_t o = ((size_t)p * a.n_super + my_sig) * (size_t)a.cap + idx;
                a.out.key[o] = ((unsigned long long)p << top_shift) | (key >> BP);
                a.out.tail[o] = otail[p];
                a.out.w[o] = ow[p];
            }
        }
        // bucket sizes: the last parent of each run records the run totals (a later
        // chunk continuing the run records larger totals; the maximum wins)
        if (i < H && (i == H - 1 || s.sig[i + 1] != my_sig)) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const unsigned int tot = s.excl[p][i] + (ov[p] ? 1u : 0u) - s.excl[p][start] +
                                         (from_prev ? s.base[p] : 0u);
                if (tot) atomicMax(&a.out_count[(size_t)p * a.n_super + my_sig],
                                   tot > (unsigned long long)a.cap ? (unsigned int)a.cap : tot);
            }
        }
    }
}

}  // namespace

int chunk_heads(int P) { return kThreads - (P - 1); }

int launch_step(const StepArgs& a, int grid, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (a.P) {
        case 4: hipLaunchKernelGGL((step_kernel<4, 2>), dim3(grid), dim3(kThreads), 0, st, a); break;
        case 9: hipLaunchKernelGGL((step_kernel<9, 4>), dim3(grid), dim3(kThreads), 0, st, a); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_plan(const PlanArgs& a, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    switch (a.P) {
        case 4: hipLaunchKernelGGL((plan_kernel<4>), dim3(1), dim3(kPlanThreads), 0, st, a); break;
        case 9: hipLaunchKernelGGL((plan_kernel<9>), dim3(1), dim3(kPlanThreads), 0, st, a); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace quapi_dev
