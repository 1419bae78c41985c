// One time step of the MACGIC-iQUAPI path propagation on the direct-mapped
// store (two-level systems, merge positions 0..L-1): a planner and a step
// kernel per step.
//
// The store has a slot for every key of the merge positions (slot = key, point
// 0 most significant): a 32-byte record (amplitude, history tail) and an
// occupancy byte.  The parents whose children merge -- those agreeing on
// points 0..L-2 (Sec. 3.1.2) -- are the occupied slots of one aligned segment
// of four, and the merged child of segment j by pair p has the fixed slot
// (p, points 0..L-2) = p * 4^(L-1) + j: writing it needs no offset from any
// other segment.
//
// Planner (between steps): reads the occupancy of every segment (the bytes
// holding the finished step's tag), lists the nonempty segments by how many
// groups they hold (four lists, each in segment order within a region; a
// decoupled look-back over epoch-tagged region counts places the regions),
// now and then clears the occupancy buffer the planned step writes, and
// reduces the finished step's per-workgroup sums of rho(t) and counters in
// workgroup order (deterministic).
//
// Step: every wave takes chunks of 64 segments of one list (the lists of full
// segments first), one segment per lane, so all lanes extend the same number
// of parents.  A lane sums the lag terms of the points its parents share
// (0..L-2) once, from tables built once per coefficient set, then extends each
// parent by every pair (propagator element of eq. SysP times the influence
// factor of eq. inf_fun; end-point correction of the final point for rho(t),
// Sec. 3.2.1), drops children below theta (Sec. 2.1) and merges the survivors
// of each pair in registers, in slot order (sum of the weights; representative
// of largest quantised |w|^2, ties to the smaller history read from the oldest
// point).  It writes the up to four merged groups to their slots with their
// occupancy bytes.  Each lane adds its segments' rho, and its wave the dropped
// |w| and survivor count; a workgroup's sums are added wave by wave, and the
// next planner adds the workgroups' sums in workgroup order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "quapi_dense.h"
#include "quapi_device.h"

namespace quapi_dev {

namespace {

constexpr int P4 = 4;
constexpr int kWavesD = kDenseThreads / 64;
constexpr int kDies = 8;                                     // XCDs of an MI355X: workgroups go to them in turn
constexpr int kPlanWavesD = kDensePlanThreads / 64;
constexpr int kTabPts = 2;                                   // points per lag-sum table
constexpr int kTabEntries = 1 << (2 * kTabPts);
constexpr int kCountBits = 13;                               // a region's count of one list (<= 4096)
constexpr int kTagShift = 4 * kCountBits;                    // epoch tag: bits 52..63

__device__ inline unsigned int n_shared_tabs(int L) { return (unsigned int)(L - 1 + kTabPts - 1) / kTabPts; }
__device__ inline unsigned int n_tail_tabs(int L, int K) { return (unsigned int)(K - L + kTabPts - 1) / kTabPts; }

__device__ inline unsigned int comp4(const uint4& v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// the four occupancy bits of a segment's word of bytes (slot r: byte r): the
// bytes equal to the tag (x = v ^ tag has a zero byte there; the sum below
// sets bit 7 of every nonzero byte and of no zero one)
__device__ inline unsigned int seg_nibble(unsigned int v, unsigned int tagx4) {
    const unsigned int x = v ^ tagx4;
    const unsigned int z = ~(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x) & 0x80808080u;
    return ((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u);
}

__device__ inline unsigned int wave_sum_u32(unsigned int v) {
    for (int off = 32; off > 0; off >>= 1) v += (unsigned int)__shfl_xor((int)v, off, 64);
    return v;
}

// ------------------------------------------------------------------ planner
// Workgroup w < n_regions plans segments [w * kDenseRegion, (w + 1) * kDenseRegion):
// wave v takes a quarter of them, thread l of the wave the four segments
// base + 256 it + 4 l + (0..3) of iteration it.  Pass 1 counts the segments of
// each list per wave; the region publishes its four counts tagged with the
// epoch and sums those of the regions before it (their workgroups were
// dispatched earlier, so the wait ends); pass 2 writes the entries, list by
// list in (wave, iteration, component, lane) order.  The last workgroup
// reduces the finished step's per-workgroup sums.
__global__ __launch_bounds__(kDensePlanThreads) void dense_plan(const DensePlanArgs a) {
    constexpr int S = partial_stride(P4);
    __shared__ unsigned int wcnt[kPlanWavesD][4];
    __shared__ unsigned int wpre[kPlanWavesD][4];
    __shared__ double wred[kPlanWavesD][S];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const long long NS = a.n_segs;
    const int n_regions = (int)((NS + kDenseRegion - 1) / kDenseRegion);
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

    // ---- pass 1: this wave's segments and their counts per list
    const long long wbase = (long long)w * kDenseRegion + (long long)wave * (kDenseRegion / kPlanWavesD);
    const unsigned int tagx4 = dense_tag(a.reduce_t) * 0x01010101u;   // the finished step's tag in each byte
    uint4 f[kDensePlanIters];
#pragma unroll
    for (int it = 0; it < kDensePlanIters; ++it) {
        const long long s0 = wbase + 256 * it + 4 * (long long)lane;   // NS is a multiple of 4
        f[it] = s0 < NS ? *reinterpret_cast<const uint4*>(a.flags + s0) : make_uint4(0u, 0u, 0u, 0u);
        // the buffer the planned step writes holds the tags of earlier steps, which
        // differ from the tags of the next 508 steps; it is cleared now and then
        if (a.clear_spent && s0 < NS) *reinterpret_cast<uint4*>(a.flags_spent + s0) = make_uint4(0u, 0u, 0u, 0u);
    }
    unsigned int cnt[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int it = 0; it < kDensePlanIters; ++it)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int n = __popc(seg_nibble(comp4(f[it], k), tagx4));
#pragma unroll
            for (int b = 0; b < 4; ++b) cnt[b] += (unsigned int)__popcll(__ballot(n == b + 1));
        }
    if (lane == 0u)
#pragma unroll
        for (int b = 0; b < 4; ++b) wcnt[wave][b] = cnt[b];
    __syncthreads();

    // ---- the region's counts, published; the regions before it, summed
    unsigned long long packed = 0ull;
    unsigned int run[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        unsigned int tot = 0u, before = 0u;
        for (int q = 0; q < kPlanWavesD; ++q) {
            if (q < wave) before += wcnt[q][b];
            tot += wcnt[q][b];
        }
        run[b] = before;
        packed |= (unsigned long long)tot << (kCountBits * b);
    }
    const unsigned long long tag = (unsigned long long)(a.epoch & 0xfffu) << kTagShift;
    if (i == 0) st_relaxed(a.agg + w, tag | packed);
    unsigned int pre[4] = {0u, 0u, 0u, 0u};
    for (int r = i; r < w; r += kDensePlanThreads) {
        unsigned long long v;
        unsigned int spins = 0;
        while (((v = ld_relaxed(a.agg + r)) >> kTagShift) != (tag >> kTagShift)) {
            if (++spins == (1u << 24)) {   // a region never published: fail the step, do not hang
                raise_error(a.error, a.reduce_t + 1, kErrSpin);
                v = 0ull;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) pre[b] += (unsigned int)(v >> (kCountBits * b)) & ((1u << kCountBits) - 1u);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const unsigned int s = wave_sum_u32(pre[b]);
        if (lane == 0u) wpre[wave][b] = s;
    }
    __syncthreads();
    unsigned int before_all[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        before_all[b] = wpre[0][b] + wpre[1][b] + wpre[2][b] + wpre[3][b];
        run[b] += before_all[b];
    }

    // ---- pass 2: the entries
#pragma unroll
    for (int it = 0; it < kDensePlanIters; ++it)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned int nib = seg_nibble(comp4(f[it], k), tagx4);
            const int n = __popc(nib);
            unsigned long long m[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) m[b] = __ballot(n == b + 1);
            if (n > 0) {
                const int b = n - 1;
                const unsigned long long mb = b == 0 ? m[0] : b == 1 ? m[1] : b == 2 ? m[2] : m[3];
                const unsigned int base = b == 0 ? run[0] : b == 1 ? run[1] : b == 2 ? run[2] : run[3];
                const unsigned long long sj = (unsigned long long)(wbase + 256 * it + 4 * (long long)lane + k);
                a.seg[(size_t)b * (size_t)NS + base + rank_below(mb)] = (unsigned int)(sj << 4) | nib;
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) run[b] += (unsigned int)__popcll(m[b]);
        }

    // ---- the last region knows the totals
    if (w == n_regions - 1 && i == 0) {
        DensePlan pl;
        unsigned int ng = 0u, nc = 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            unsigned int tot = before_all[b];
            for (int q = 0; q < kPlanWavesD; ++q) tot += wcnt[q][b];
            pl.n_seg[b] = tot;
            ng += (unsigned int)(b + 1) * tot;
            nc += (tot + kDenseChunk - 1) / kDenseChunk;
        }
        pl.n_groups = ng;
        pl.n_chunks = nc;
        pl.pad[0] = pl.pad[1] = 0u;
        if (a.reduce_t > 0) a.stats_hist[a.reduce_t].n_stored = ng;
        *a.plan = pl;
    }
}

// ------------------------------------------------------------------ step
struct DLds {
    double2 k4[16];                              // K4[p * 4 + h]
    double ds[4], ss[4];
    double e0, f0;                               // exp(-D^2 Re c_0), exp(-D^2 Re delta_0)
    float2 k4f[16];                              // the FP32 form's copies
    float dsf[4], ssf[4];
    double acc[2 * P4][kDenseThreads];           // each lane's rho by pair, re/im, over its segments
    double red[kWavesD][partial_stride(P4)];
};

// ---- lag-sum table sets: workgroup k builds the set of coefficient set k
__global__ __launch_bounds__(256) void dense_tables(const double* __restrict__ coef,
                                                    const double* __restrict__ tables, int L, int K,
                                                    unsigned int set_doubles, double* __restrict__ out) {
    __shared__ double cs[4][kMaxK + 1];
    __shared__ double dsx[4], ssx[4];
    const int i = threadIdx.x;
    const double* cf = coef + (size_t)blockIdx.x * 4 * (K + 1);
    double* o = out + (size_t)blockIdx.x * set_doubles;
    for (int k = i; k < 4 * (K + 1); k += 256) cs[k / (K + 1)][k % (K + 1)] = cf[k];
    if (i < 4) {
        dsx[i] = tables[TableLayout::ds(P4) + i];
        ssx[i] = tables[TableLayout::ss(P4) + i];
    }
    __syncthreads();
    const unsigned int nsh = n_shared_tabs(L), ntl = n_tail_tabs(L, K);
    for (unsigned int k = i; k < (nsh + ntl) * kTabEntries; k += 256) {
        const unsigned int q = k / kTabEntries, v = k % kTabEntries;
        const bool shared = q < nsh;
        const int st = shared ? kTabPts * (int)q : L + kTabPts * (int)(q - nsh);
        const int len = shared ? min(kTabPts, L - 1 - st) : min(kTabPts, K - st);
        double A = 0, B = 0, Ac = 0, Bc = 0;
        if (v < (1u << (2 * len))) {
            for (int m = 0; m < len; ++m) {
                const int x = (int)(v >> (shared ? 2 * (len - 1 - m) : 2 * m)) & 3;
                const int d = st + m + 1;                     // lag of that point
                A += cs[0][d] * dsx[x];
                B += cs[1][d] * ssx[x];
                Ac += cs[2][d] * dsx[x];
                Bc += cs[3][d] * ssx[x];
            }
        }
        o[4 * k] = A;
        o[4 * k + 1] = B;
        o[4 * k + 2] = Ac;
        o[4 * k + 3] = Bc;
    }
    if (i == 0) {
        const double D = dsx[1];
        o[4 * (nsh + ntl) * kTabEntries] = exp(-D * D * cs[0][0]);
        o[4 * (nsh + ntl) * kTabEntries + 1] = exp(-D * D * cs[2][0]);
    }
}

// entry e of table q: (A, B, Ac, Bc) = sums of (cre ds, cim ss, dre ds, dim ss)
// over the table's points at the digits of e
__device__ inline void tab_add(const double* tab, unsigned int q, unsigned int e, double& A, double& B,
                               double& Ac, double& Bc) {
    const double4 v = *reinterpret_cast<const double4*>(tab + 4 * ((size_t)q * kTabEntries + e));
    A += v.x;
    B += v.y;
    Ac += v.z;
    Bc += v.w;
}

__device__ inline void tab_add(const float* tab, unsigned int q, unsigned int e, float& A, float& B, float& Ac,
                               float& Bc) {
    const float4 v = *reinterpret_cast<const float4*>(tab + 4 * ((size_t)q * kTabEntries + e));
    A += v.x;
    B += v.y;
    Ac += v.z;
    Bc += v.w;
}

// fused multiply-add in the precision of its operands
__device__ inline float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ inline double uniform_d(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// chunk c of the plan: list b (segments of b + 1 groups) and its first entry
// Chunks by die.  The lists are in segment order, so slice x of X of every list
// covers about the same range of segments; the workgroups of die x (workgroup
// x mod X: the order in which workgroups are handed to the dies) take slice x of
// lists 3, 2, 1, 0 in turn.  The merged records and occupancy bytes of
// neighbouring segments, which share lines, then meet in one L2.  Chunk v of
// slice x: its list b and first entry, false past the slice's last chunk.
__device__ inline bool slice_chunk(const unsigned int (&n_seg)[4], unsigned int x, unsigned int X, unsigned int v,
                                   int& b, unsigned int& first) {
    unsigned int kk = v;
    bool found = false;
#pragma unroll
    for (int bb = 3; bb >= 0; --bb) {
        const unsigned long long cb = (n_seg[bb] + kDenseChunk - 1) / kDenseChunk;
        const unsigned int lo = (unsigned int)(cb * x / X), hi = (unsigned int)(cb * (x + 1) / X);
        if (!found && kk < hi - lo) {
            b = bb;
            first = (lo + kk) * kDenseChunk;
            found = true;
        }
        if (!found) kk -= hi - lo;
    }
    return found;
}

// Q32: the quantised |w|^2 keeps no bit of the low word (qbits >= 32), so the
// representative's key is the high word alone.
// F32: the precision form.  A parent's amplitude is read as FP32 (ln|w|, arg w)
// and leaves the log domain with FP32 exp and sin/cos; the lag sums, the
// influence exponents and each child's product are FP32; the filter test, the
// merge sums and rho(t) are FP64, and each merged sum returns to the log domain
// through FP32 log and atan2 refined by one FP64 Newton step, rounded once.
template <bool Q32, bool F32>
__global__ __launch_bounds__(kDenseThreads, 4) void dense_step(const DenseArgs a) {
    constexpr int P = P4;
    constexpr int S = partial_stride(P);
    using QT = typename std::conditional<Q32, unsigned int, unsigned long long>::type;
    using Real = typename std::conditional<F32, float, double>::type;
    using Rec = typename std::conditional<F32, DenseRec32, DenseRec>::type;
    extern __shared__ double tab_raw[];
    Real* tab = reinterpret_cast<Real*>(tab_raw);  // [n_tabs][kTabEntries][4]
    __shared__ DLds s;
    const Rec* rec_in;
    Rec* rec_out;
    if constexpr (F32) {
        rec_in = a.rec32_in;
        rec_out = a.rec32_out;
    } else {
        rec_in = a.rec_in;
        rec_out = a.rec_out;
    }
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();

    if (error_word(a.error) != 0u) return;
    const int K = a.K, L = a.L;
    const long long NS = a.n_segs;
    const unsigned int nsh = n_shared_tabs(L), ntl = n_tail_tabs(L, K);

    // ---- this wave's first chunk: its entry in flight during the set-up
    unsigned int n_seg[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) n_seg[b] = a.plan->n_seg[b];
    const unsigned int X = min(gridDim.x, (unsigned int)kDies);
    const unsigned int x = blockIdx.x % X;
    const unsigned int stride = (gridDim.x - x + X - 1) / X * kWavesD;   // waves of slice x
    // the wave's index in slice x (wave-uniform: kept in scalar registers)
    unsigned int v = (unsigned int)__builtin_amdgcn_readfirstlane((int)(blockIdx.x / X * kWavesD + wave));
    int b = 0;
    unsigned int e = 0u, ent = 0u;
    unsigned int first;
    bool have = slice_chunk(n_seg, x, X, v, b, first);
    if (have) {
        e = first + lane;
        if (e < n_seg[b]) ent = a.seg[(size_t)b * (size_t)NS + e];
    }

    // ---- this step's lag-sum tables (built once per coefficient set) and K4
    if (i < P * P) {
        s.k4[i] = make_double2(a.tables[2 * i], a.tables[2 * i + 1]);
        s.k4f[i] = make_float2((float)a.tables[2 * i], (float)a.tables[2 * i + 1]);
    }
    if (i < P) {
        s.ds[i] = a.tables[TableLayout::ds(P) + i];
        s.ss[i] = a.tables[TableLayout::ss(P) + i];
        s.dsf[i] = (float)s.ds[i];
        s.ssf[i] = (float)s.ss[i];
    }
    {
        const unsigned int n4 = (nsh + ntl) * kTabEntries;             // entries of four sums
        const double4* src = reinterpret_cast<const double4*>(a.tabset);
        for (unsigned int k = i; k < n4; k += kDenseThreads) {
            const double4 v = src[k];
            if constexpr (F32)
                reinterpret_cast<float4*>(tab)[k] = make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
            else
                reinterpret_cast<double4*>(tab)[k] = v;
        }
        if (i == 0) {
            s.e0 = a.tabset[4 * n4];
            s.f0 = a.tabset[4 * n4 + 1];
        }
    }
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) s.acc[k][i] = 0.0;
    __syncthreads();

    const int tail_pts = K - L;
    const unsigned long long tail_mask =
        tail_pts <= 0 ? 0ull : (tail_pts * 2 >= 64 ? ~0ull : ((1ull << (tail_pts * 2)) - 1));
    const int q_shift = 2 * (L - 1);                        // output slot = (p << q_shift) | j
    // wave-uniform constants (scalar registers)
    const int n1 = K + 1;
    const Real D = (Real)a.tables[TableLayout::ds(P) + 1], Sg = (Real)a.tables[TableLayout::ss(P) + 1];
    const Real cim0 = (Real)a.coef[n1], dim0 = (Real)a.coef[3 * n1];
    const Real creL = (Real)a.coef[L], cimL = (Real)a.coef[n1 + L], dreL = (Real)a.coef[2 * n1 + L],
               dimL = (Real)a.coef[3 * n1 + L];
    const double e0d = uniform_d(s.e0), f0d = uniform_d(s.f0), theta2 = a.theta2;
    const Real e0 = (Real)e0d, f0 = (Real)f0d;
    const unsigned long long qmask = a.qmask;

    double dropped = 0.0;
    unsigned int n_surv = 0u;                               // this lane's surviving children
    while (have) {
        if (e < n_seg[b]) {
            // ---- segment j of chunk c, its b + 1 parents in slot order
            const unsigned int j = ent >> 4;
            unsigned int nib = ent & 15u;
            int mn = __builtin_ctz(nib);
            nib &= nib - 1u;
            Rec Rn = rec_in[4ull * j + mn];

            // lag sums over the shared points 0..L-2
            Real As = 0, Bs = 0, Acs = 0, Bcs = 0;
            for (unsigned int q = 0; q < nsh; ++q) {
                const int st = kTabPts * (int)q, len = min(kTabPts, L - 1 - st);
                const unsigned int v = (j >> (2 * (L - 1 - st - len))) & ((1u << (2 * len)) - 1u);
                tab_add(tab, q, v, As, Bs, Acs, Bcs);
            }
            const int h0 = (int)(j >> (2 * (L - 2)));      // point 0 of the segment

            bool any[P];
            double sr[P], si[P];
            QT bq[P];
            unsigned long long bt[P];
            double r1r = 0.0, r1i = 0.0, r2r = 0.0, r2i = 0.0;   // rho of pairs 1, 2 (f != 1)
#pragma unroll
            for (int p = 0; p < P; ++p) {
                any[p] = false;
                sr[p] = si[p] = 0.0;
                bq[p] = 0u;
                bt[p] = 0ull;
            }
#pragma unroll 1
            for (int r = 0; r <= b; ++r) {
                // this parent, and the next one's record in flight
                const int mc = mn;
                const unsigned long long Tc = Rn.tail;
                Real Wcx, Wcy;                         // the parent's amplitude (FP32 form: ln|w|, arg w)
                if constexpr (F32) {
                    Wcx = Rn.lw;
                    Wcy = Rn.aw;
                } else {
                    Wcx = Rn.w.x;
                    Wcy = Rn.w.y;
                }
                if (r < b) {
                    mn = __builtin_ctz(nib);
                    nib &= nib - 1u;
                    Rn = rec_in[4ull * j + mn];
                }
                if constexpr (F32) {
                    const float m = expf(Wcx);
                    float sa, ca;
                    sincos_f32(Wcy, sa, ca);
                    Wcx = m * ca;
                    Wcy = m * sa;
                }
                // the propagator row of point 0, read again each parent (held across the
                // loop it would take 16 registers)
                int k4row = h0;
                asm volatile("" : "+v"(k4row));

                // ---- influence sums of the parent over lags 1..K
                Real dsm, ssm;                         // point L-1 of the parent (lag L)
                if constexpr (F32) {
                    dsm = s.dsf[mc];
                    ssm = s.ssf[mc];
                } else {
                    dsm = s.ds[mc];
                    ssm = s.ss[mc];
                }
                Real A = fma_r(creL, dsm, As), B = fma_r(cimL, ssm, Bs);
                Real Ac = fma_r(dreL, dsm, Acs), Bc = fma_r(dimL, ssm, Bcs);
                for (unsigned int q = 0; q < ntl; ++q) {
                    const int len = min(kTabPts, tail_pts - kTabPts * (int)q);
                    const unsigned int v = (unsigned int)(Tc >> (2 * kTabPts * q)) & ((1u << (2 * len)) - 1u);
                    tab_add(tab, nsh + q, v, A, B, Ac, Bc);
                }
                const unsigned long long ctail = ((Tc << 2) | (unsigned long long)mc) & tail_mask;
                // pairs (0,1) and (1,0) have ds = +D, -D and equal ss: their exponents are
                // mirror images and share one exp and one sincos; pairs (0,0), (1,1) have ds = 0
                const Real x = D * A, y = D * fma_r(cim0, Sg, B);
                const Real xc = D * Ac, yc = D * fma_r(dim0, Sg, Bc);
                Real ex, exc, iex, iexc, sy, cy, syc, cyc;
                if constexpr (F32) {
                    ex = expf(x);
                    exc = expf(xc);
                    iex = 1.0f / ex;
                    iexc = 1.0f / exc;
                    sincos_f32(y, sy, cy);
                    sincos_f32(yc, syc, cyc);
                } else {
                    ex = exp_fast(x);
                    exc = exp_fast(xc);
                    iex = recip(ex);
                    iexc = recip(exc);
                    sincos_fast(y, &sy, &cy);
                    sincos_fast(yc, &syc, &cyc);
                }
                Real er[P], ei[P], fr[P], fi[P];
                er[1] = e0 * iex * cy;  ei[1] = -(e0 * iex * sy);
                er[2] = e0 * ex * cy;   ei[2] = e0 * ex * sy;
                fr[1] = f0 * iexc * cyc; fi[1] = -(f0 * iexc * syc);
                fr[2] = f0 * exc * cyc;  fi[2] = f0 * exc * syc;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    Real k4x, k4y;
                    if constexpr (F32) {
                        k4x = s.k4f[p * P + k4row].x;
                        k4y = s.k4f[p * P + k4row].y;
                    } else {
                        k4x = s.k4[p * P + k4row].x;
                        k4y = s.k4[p * P + k4row].y;
                    }
                    const Real br = Wcx * k4x - Wcy * k4y;
                    const Real bi = Wcx * k4y + Wcy * k4x;
                    Real cr = br, ci = bi;                  // pairs 0 and 3: factor 1
                    if (p == 1 || p == 2) {
                        cr = br * er[p] - bi * ei[p];
                        ci = br * ei[p] + bi * er[p];
                    }
                    const double wr2 = (double)cr, wi2 = (double)ci;
                    const double n2 = norm2_nocontract(wr2, wi2);
                    const bool keep = (theta2 == 0.0) || !(n2 < theta2);
                    n_surv += keep ? 1u : 0u;
                    if (keep) {
                        // rho(t) terms: the product in the form's precision, summed in FP64
                        if (p == 1) {
                            r1r += (double)(cr * fr[1] - ci * fi[1]);
                            r1i += (double)(cr * fi[1] + ci * fr[1]);
                        } else if (p == 2) {
                            r2r += (double)(cr * fr[2] - ci * fi[2]);
                            r2i += (double)(cr * fi[2] + ci * fr[2]);
                        }
                        const unsigned long long q64 = (unsigned long long)__double_as_longlong(n2) & qmask;
                        const QT q = Q32 ? (QT)(q64 >> 32) : (QT)q64;
                        if (!any[p] || q > bq[p] || (q == bq[p] && ctail < bt[p])) {
                            bq[p] = q;
                            bt[p] = ctail;
                        }
                        sr[p] += wr2;
                        si[p] += wi2;
                        any[p] = true;
                    } else {
                        dropped += sqrt(n2);
                    }
                }
            }
            // ---- rho of the segment; the merged children at their slots
            s.acc[0][i] += sr[0];          // pairs 0 and 3: the end-point factor is 1
            s.acc[1][i] += si[0];
            s.acc[2][i] += r1r;
            s.acc[3][i] += r1i;
            s.acc[4][i] += r2r;
            s.acc[5][i] += r2i;
            s.acc[6][i] += sr[3];
            s.acc[7][i] += si[3];
            if constexpr (F32) {
                // one pair at a time, its state rotated into index 0 (one set of the
                // conversion's temporaries live at once)
#pragma unroll 1
                for (int p = 0; p < P; ++p) {
                    if (any[0]) {
                        const float2 la = to_log_domain32(sr[0], si[0]);
                        Rec o;
                        o.lw = la.x;
                        o.aw = la.y;
                        o.tail = bt[0];
                        const unsigned long long so = ((unsigned long long)p << q_shift) | j;
                        rec_out[so] = o;
                        a.flag_out[so] = (unsigned char)dense_tag(a.t);
                    }
#pragma unroll
                    for (int k = 0; k + 1 < P; ++k) {
                        any[k] = any[k + 1];
                        sr[k] = sr[k + 1];
                        si[k] = si[k + 1];
                        bt[k] = bt[k + 1];
                    }
                }
            } else {
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    if (!any[p]) continue;
                    const unsigned long long so = ((unsigned long long)p << q_shift) | j;
                    Rec o;
                    o.w = make_double2(sr[p], si[p]);
                    o.tail = bt[p];
                    o.pad = 0ull;
                    rec_out[so] = o;
                    a.flag_out[so] = (unsigned char)dense_tag(a.t);
                }
            }
        }
        // ---- the next chunk of this wave
        v += stride;
        have = slice_chunk(n_seg, x, X, v, b, first);
        if (have) {
            e = first + lane;
            if (e < n_seg[b]) ent = a.seg[(size_t)b * (size_t)NS + e];
        }
    }

    // ---- the workgroup's sums: lanes, then waves, in a fixed order
#pragma unroll
    for (int k = 0; k < 2 * P; ++k) {
        const double t = wave_sum(s.acc[k][i]);
        if (lane == 0u) s.red[wave][k] = t;
    }
    {
        const double t = wave_sum(dropped);
        const unsigned int ns = wave_sum_u32(n_surv);
        if (lane == 0u) {
            s.red[wave][2 * P] = t;
            s.red[wave][2 * P + 1] = (double)ns;
        }
    }
    __syncthreads();
    if (i < S) {
        double t = 0.0;
        for (int q = 0; q < kWavesD; ++q) t += s.red[q][i];
        a.partials[(size_t)i * gridDim.x + blockIdx.x] = t;
    }
}

}  // namespace

int dense_tab_count(int L, int K) {
    return (L - 1 + kTabPts - 1) / kTabPts + (K - L + kTabPts - 1) / kTabPts;
}

size_t dense_tabset_doubles(int L, int K) { return (size_t)dense_tab_count(L, K) * kTabEntries * 4 + 4; }

int dense_lds_bytes(int L, int K, bool f32) {
    return dense_tab_count(L, K) * kTabEntries * 4 * (f32 ? (int)sizeof(float) : (int)sizeof(double));
}

int launch_dense_tables(const double* coef, const double* tables, int L, int K, int n_sets, double* out,
                        void* stream) {
    hipLaunchKernelGGL(dense_tables, dim3(n_sets), dim3(256), 0, (hipStream_t)stream, coef, tables, L, K,
                       (unsigned int)dense_tabset_doubles(L, K), out);
    return (int)hipGetLastError();
}

int dense_max_chunks(long long n_segs) { return (int)((n_segs + kDenseChunk - 1) / kDenseChunk) + 4; }

int dense_step_grid(int n_cu, int lds_bytes, bool f32) {
    int n32 = 0, n64 = 0;
    const hipError_t e1 =
        f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n32, dense_step<true, true>, kDenseThreads, lds_bytes)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n32, dense_step<true, false>, kDenseThreads, lds_bytes);
    const hipError_t e2 =
        f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n64, dense_step<false, true>, kDenseThreads, lds_bytes)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n64, dense_step<false, false>, kDenseThreads, lds_bytes);
    if (e1 != hipSuccess || e2 != hipSuccess) return 0;
    const int nb = std::min(n32, n64);                       // one grid serves either form
    return nb < 1 ? 0 : nb * n_cu;
}

int launch_dense_step(const DenseArgs& a, int grid, int lds_bytes, void* stream) {
    const bool q32 = (a.qmask & 0xffffffffull) == 0ull;
    const hipStream_t st = (hipStream_t)stream;
    if (a.f32 && q32)
        hipLaunchKernelGGL((dense_step<true, true>), dim3(grid), dim3(kDenseThreads), lds_bytes, st, a);
    else if (a.f32)
        hipLaunchKernelGGL((dense_step<false, true>), dim3(grid), dim3(kDenseThreads), lds_bytes, st, a);
    else if (q32)
        hipLaunchKernelGGL((dense_step<true, false>), dim3(grid), dim3(kDenseThreads), lds_bytes, st, a);
    else
        hipLaunchKernelGGL((dense_step<false, false>), dim3(grid), dim3(kDenseThreads), lds_bytes, st, a);
    return (int)hipGetLastError();
}

int launch_dense_plan(const DensePlanArgs& a, void* stream) {
    const int grid = (int)((a.n_segs + kDenseRegion - 1) / kDenseRegion) + 1;
    hipLaunchKernelGGL(dense_plan, dim3(grid), dim3(kDensePlanThreads), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

}  // namespace quapi_dev
