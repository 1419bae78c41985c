// One time step of MACGIC-iQUAPI for masks whose merge positions are not a
// contiguous run 0..L-1 (a MACGIC mask that keeps distant lags, Sec. 2.1).
// The groups a child joins are then not adjacent in key order, so the merge
// goes through an open-addressing hash table in HBM keyed on the child's
// points at the merge positions.
//
// State between steps: groups as full histories (point j = lag j at bits
// [BP*j, BP*j+BP), the newest point lowest) with their amplitudes, in no
// particular order.  One step is three kernels (four in the unpacked form):
//   expand  - extend every group by every pair: weight times the propagator
//             element (eq. SysP) times the influence factor of the new point
//             (eq. inf_fun); drop children below theta (Sec. 2.1); add the
//             survivors to this workgroup's rho(t) sums with the end-point
//             correction of the final point (Sec. 3.2.1); merge the
//             survivors of a pass in an LDS table, then insert each merged
//             key into the table, raise the slot's representative word to
//             the best child's and add the weights to the key's sum (the
//             group amplitude is the sum of all its members, Sec. 3.1.2);
//   resolve - unpacked form only: among the children of a key with its
//             largest quantised |w|^2, keep the smallest history;
//   compact - write one group per used slot, its history rebuilt from the key
//             and the representative word, and clear the slot;
//   reduce  - add up the workgroups' rho(t) and counters in workgroup order.
// The representative is the child with the largest quantised |w|^2 and, among
// those, the history that is smallest read from the oldest point.  Children
// of one key agree at the merge positions, so that order is the order of
// their points at the other positions, packed oldest first; when those fit
// below the quantised |w|^2 in one 64-bit word a single atomic max selects the
// representative (the packed form).
// The table in use has the next power of two above twice the children of the
// step, read from the stored count on the device.  The weight sums of the
// table are atomic and so in no fixed order; rho(t) is summed in a fixed order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "quapi_device.h"
#include "quapi_host.h"
#include "quapi_sparse.h"

namespace quapi_dev {

namespace {

constexpr int kSpWaves = kSparseThreads / 64;
constexpr int kMaxProbe = 1 << 16;
constexpr int kRows = 8;                                  // table rows per compact tile
constexpr unsigned long long kTile = (unsigned long long)kRows * kSparseThreads;

// 64-bit finaliser of the SplitMix64 generator (Steele, Lea, Flood 2014), as
// the hash of a merge key
__device__ inline unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// The table is cut into windows of 2^kWinBits slots.  A key's window is the
// hash of its points at the clustered positions (merge positions q with q+1
// also a merge position), its place inside the window the hash of the whole
// key.  A group's clustered points are the points of its next-step merge
// signature that its key holds, so groups whose children merge at the next
// step share a window, and compact, which scans in slot order, stores them
// side by side: the next expand then meets them in one workgroup pass.
// Smaller windows crowd the keys of a pass into long probe chains, larger ones
// split partners over passes (long memory, K = 40, expand per step: 27.6 ms
// at 128 slots, 5.4 at 512, 3.4 at 1024, 3.5 at 2048, 4.2 at 4096, 4.8 at
// 8192, 5.5 with keys hashed whole).
constexpr int kWinBits = 10;

__device__ inline unsigned long long home_slot(unsigned long long key, unsigned long long cmask,
                                               unsigned long long tm) {
    if (cmask == 0ull) return mix64(key) & tm;
    return ((mix64(key & cmask) << kWinBits) | (mix64(key) & ((1ull << kWinBits) - 1ull))) & tm;
}

// groups a segment holds at parity par, bounded by its size
__device__ inline unsigned long long seg_groups(const SparseArgs& a, int par, int s) {
    const unsigned long long c = a.count[seg_counter(par, s)];
    return c < a.seg_cap ? c : a.seg_cap;
}

// groups stored at t-1 (the step's input), bounded by the capacity
__device__ inline unsigned long long groups_in(const SparseArgs& a) {
    unsigned long long n = 0ull;
    for (int s = 0; s < kSegs; ++s) n += seg_groups(a, (a.t - 1) & 1, s);
    return n < (unsigned long long)a.cap ? n : (unsigned long long)a.cap;
}

// slots in use this step, minus one: the next power of two at or above twice
// the children, at least kMinTable and at most the allocation
__device__ inline unsigned long long table_mask(const SparseArgs& a, unsigned long long n_in) {
    const unsigned long long need = 2ull * (unsigned long long)a.P * n_in;
    unsigned long long ts = kMinTable;
    if (need > ts) ts = 1ull << (64 - __clzll(need - 1ull));
    return (ts < a.tsize ? ts : a.tsize) - 1ull;
}

// partitions in use this step: about one per kPartLoad children of the input,
// a power of two, at most the allocation
__device__ inline unsigned int n_partitions(const SparseArgs& a, unsigned long long n_in) {
    const unsigned long long need = ((unsigned long long)a.P * n_in + kPartLoad - 1) / kPartLoad;
    unsigned long long np = 1;
    while (np < need) np <<= 1;
    return (unsigned int)(np < a.n_part_max ? np : a.n_part_max);
}

// partition of a merge key: high bits of its hash (the LDS table of the
// partition merge takes the low ones)
__device__ inline unsigned int partition_of(unsigned long long key, unsigned int np) {
    return (unsigned int)(mix64(key) >> 32) & (np - 1u);
}

// w bits (at most 64) of the 128-bit number hi:lo from bit s
__device__ inline unsigned long long bits_at(unsigned long long lo, unsigned long long hi, int s, int w) {
    const unsigned long long v = s >= 64 ? hi >> (s - 64) : (s == 0 ? lo : (lo >> s) | (hi << (64 - s)));
    return w >= 64 ? v : v & ((1ull << w) - 1ull);
}

// v (below 2^(128-s)) into the 128-bit number hi:lo at bit s
__device__ inline void put_bits(unsigned long long& lo, unsigned long long& hi, unsigned long long v, int s) {
    if (s >= 64) {
        hi |= v << (s - 64);
    } else {
        lo |= v << s;
        if (s > 0) hi |= v >> (64 - s);
    }
}

// low bits of the packed representative word: the complement of the points
// at the other positions
__device__ inline unsigned long long other_mask(const SparseArgs& a) {
    return (1ull << (a.qbits + 1)) - 1ull;
}

// A history of W 64-bit words: point j at bit BP*j of the W*64-bit number
// (word j*BP/64), the newest point lowest.  BP divides 64, so no point
// straddles two words.
template <int W>
struct Hist {
    unsigned long long w[W];
};

template <int BP, int W>
__device__ inline unsigned long long point_at(const Hist<W>& h, int bit) {
    constexpr unsigned long long DM = (1ull << BP) - 1;
    if (W == 1) return (h.w[0] >> bit) & DM;
    const unsigned long long word = (bit >> 6) == 0 ? h.w[0] : h.w[W - 1];
    return (word >> (bit & 63)) & DM;
}

template <int W>
__device__ inline Hist<W> load_hist(const uint64_t* p, unsigned long long g) {
    Hist<W> h;
#pragma unroll
    for (int k = 0; k < W; ++k) h.w[k] = p[g * W + k];
    return h;
}

// A merged group's history from its key and its representative's other points:
// both are read in 4-bit slices (two points of a two-level system, one of a
// larger one), and a table in the LDS gives each slice value's points at their
// history positions.  Table 0 covers the key (point k of the merge positions
// at key bit BP*(nq-1-k)), table 1 the other word (point k at BP*(nn-1-k)).
constexpr int kSliceBits = 4;
constexpr int kSlices = 64 / kSliceBits;
using HistTab = ulonglong2[2][kSlices][1 << kSliceBits];

template <int BP>
__device__ inline void build_hist_tab(const SparseArgs& a, HistTab& tab) {
    constexpr unsigned int DM = (1u << BP) - 1;
    for (int e = threadIdx.x; e < 2 * kSlices * (1 << kSliceBits); e += blockDim.x) {
        const int side = e / (kSlices << kSliceBits);
        const int sl = (e / (1 << kSliceBits)) % kSlices;
        const unsigned int v = (unsigned int)e & ((1u << kSliceBits) - 1);
        const int n = side ? a.nn : a.nq;
        unsigned long long w0 = 0ull, w1 = 0ull;
        for (int b = 0; b < kSliceBits; b += BP) {
            const int kbit = sl * kSliceBits + b;                 // bit of the key (other word)
            const int k = n - 1 - kbit / BP;                       // its point
            if (k < 0) break;
            const unsigned long long pt = (v >> b) & DM;
            const int bit = BP * (side ? a.npos[k] : a.qpos[k]);   // its history position
            if (bit < 64) w0 |= pt << bit;
            else w1 |= pt << (bit - 64);
        }
        tab[side][sl][v] = make_ulonglong2(w0, w1);
    }
}

// Slices are read four at a time from both tables, up to ns (the larger of the
// two slice counts): the slices above the key's or the other word's points read
// value 0, whose entry is zero.
constexpr int kSliceGroup = 4;

template <int BP, int W>
__device__ inline Hist<W> hist_from(const HistTab& tab, unsigned long long key, unsigned long long nk, int ns) {
    Hist<W> h;
#pragma unroll
    for (int w = 0; w < W; ++w) h.w[w] = 0ull;
    for (int s0 = 0; s0 < ns; s0 += kSliceGroup) {
#pragma unroll
        for (int j = 0; j < kSliceGroup; ++j) {
            const int sl = s0 + j;
            const ulonglong2 t = tab[0][sl][(key >> (kSliceBits * sl)) & ((1u << kSliceBits) - 1)];
            const ulonglong2 u = tab[1][sl][(nk >> (kSliceBits * sl)) & ((1u << kSliceBits) - 1)];
            h.w[0] |= t.x | u.x;
            if (W == 2) h.w[W - 1] |= t.y | u.y;
        }
    }
    return h;
}

// slices a history rebuild reads: the larger of the key's and the other word's
// slice counts, rounded up to whole groups of kSliceGroup (at most kSlices)
template <int BP>
__device__ inline int hist_slices(const SparseArgs& a) {
    const int bits = BP * (a.nq > a.nn ? a.nq : a.nn);
    const int ns = (bits + kSliceBits - 1) / kSliceBits;
    return (ns + kSliceGroup - 1) / kSliceGroup * kSliceGroup;
}

// History chunks of kChunkBits bits (two points of a two-level system, one of
// a three-level one) index two tables built per step and workgroup: the
// chunk's share of the influence sums A, B, Ac, Bc, and its points placed
// where the child holds them (key or other word).  A parent then costs one
// table read per chunk instead of a loop over its points.
constexpr int kChunkBits = 4;
constexpr int kChunkVals = 1 << kChunkBits;
constexpr int kLdsRows = 4;                               // LDS merge slots per thread
constexpr int kLds = kLdsRows * kSparseThreads;           // a pass's children at P = 4 (a share at P = 9)
constexpr int kLdsProbe = 32;
// dynamic LDS of the expand kernel at least this, which with its static LDS
// leaves room for two workgroups per CU: with more in flight the memory-side
// atomics contend (long memory, K = 40, expand per step: 3.5 ms at two per
// CU against 3.8 ms at three with 2048-slot windows; 5.4, 6.1 and 7.1 ms at
// two, three and one with 512-slot windows)
constexpr size_t kExpandLdsFloor = 24 * 1024;

template <int W>
__device__ inline unsigned int chunk_at(const Hist<W>& h, int c) {
    const int bit = kChunkBits * c;
    const unsigned long long word = (W == 1 || bit < 64) ? h.w[0] : h.w[W - 1];
    return (unsigned int)((word >> (bit & 63)) & (unsigned long long)(kChunkVals - 1));
}

// bytes of the influence table of n chunks; the key table follows it
template <bool F32>
__host__ __device__ constexpr size_t sparse_itab_bytes(int n_chunks) {
    return (size_t)n_chunks * kChunkVals * 2 * (F32 ? sizeof(float2) : sizeof(double2));
}
template <bool F32>
__host__ __device__ constexpr size_t sparse_chunk_lds(int n_chunks) {
    return sparse_itab_bytes<F32>(n_chunks) + (size_t)n_chunks * kChunkVals * sizeof(ulonglong2);
}

// F32: the precision form.  A group's amplitude is read as (ln|w|, arg w) in
// FP32; each child adds ln K4 and its influence exponent in FP32, leaves the
// log domain with FP32 exp and sin/cos, and enters the filter, the merge sums
// and rho(t) in FP64.  (Two levels: the parent leaves the log domain once and
// the mirrored pairs share one FP32 exp and sin/cos, as in FP64.)
//
// A workgroup takes kSparseThreads parents per pass.  Their children merge
// first in a table in the LDS (key, best word, weight sums; unpacked form:
// also the smallest other word at the best q); each used LDS slot then makes
// one insertion into the table in HBM, whose atomics are performed at the
// memory side and bound the kernel.  Children that find the LDS table full go
// to the HBM table directly.
template <int P, int BP, int W, bool F32>
__global__ __launch_bounds__(kSparseThreads) void sparse_expand(const SparseArgs a) {
    using Real = typename std::conditional<F32, float, double>::type;
    using Real2 = typename std::conditional<F32, float2, double2>::type;
    constexpr int S = partial_stride(P);
    constexpr int PPC = kChunkBits / BP;                     // points per chunk
    constexpr unsigned long long DM = (1ull << BP) - 1;
    __shared__ double k4re[P * P], k4im[P * P], ds[P], ss[P];
    __shared__ double cre[kMaxK + 1], cim[kMaxK + 1], dre[kMaxK + 1], dim[kMaxK + 1];
    __shared__ double e0f0[2];                               // two levels: exp(-D^2 Re c_0), exp(-D^2 Re delta_0)
    // FP32 precision form: ln|K4|, arg K4 and the exponent tables in FP32
    __shared__ float lk4[F32 ? P * P : 1], ak4[F32 ? P * P : 1], dsf[F32 ? P : 1], ssf[F32 ? P : 1];
    __shared__ float cref[F32 ? kMaxK + 1 : 1], cimf[F32 ? kMaxK + 1 : 1];
    __shared__ float dref[F32 ? kMaxK + 1 : 1], dimf[F32 ? kMaxK + 1 : 1];
    __shared__ double wpart[kSpWaves][S];
    // child position -> its shift in the key, or 256 + its shift in the other word
    __shared__ int pmap[kMaxK];
    // the chunk tables, in dynamic LDS sized for the step's chunks:
    // (A, B), (Ac, Bc) and (key bits, other bits) of each chunk value
    extern __shared__ __align__(16) unsigned char chunk_lds[];
    Real2 (*const itab)[kChunkVals][2] = reinterpret_cast<Real2 (*)[kChunkVals][2]>(chunk_lds);
    // the LDS merge of one pass's children: key + 1 (0: free), best word
    // (unpacked form: then the smallest other word at the best q), weight sums
    __shared__ unsigned long long lkey[kLds], lbest[kLds];
    __shared__ double lwr[kLds], lwi[kLds];
    __shared__ unsigned int loff[kLdsRows][kSpWaves];
    __shared__ unsigned int lovf[2], lused;
    __shared__ unsigned long long seg_pre[kSegs + 1];       // the input's segments: first group of each
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const int K = a.K, t = a.t, nq = a.nq, nn = a.nn;
    const int dmax = t < K ? t : K;
    if (i < nq) pmap[a.qpos[i]] = BP * (nq - 1 - i);
    if (i < nn) pmap[a.npos[i]] = 256 + BP * (nn - 1 - i);
    // where the new point goes: its shift in the key, else in the other word
    int kshift = -1, nshift = -1;
    for (int k = 0; k < nq; ++k)
        if (a.qpos[k] == 0) kshift = BP * (nq - 1 - k);
    for (int k = 0; k < nn; ++k)
        if (a.npos[k] == 0) nshift = BP * (nn - 1 - k);

    for (int k = i; k < kLds; k += kSparseThreads) {
        lkey[k] = 0ull;
        lbest[k] = 0ull;
        lwr[k] = 0.0;
        lwi[k] = 0.0;
    }
    if (i < 2) lovf[i] = 0u;
    for (int k = i; k < P * P; k += kSparseThreads) {
        k4re[k] = a.tables[2 * k];
        k4im[k] = a.tables[2 * k + 1];
    }
    if (i < P) {
        ds[i] = a.tables[TableLayout::ds(P) + i];
        ss[i] = a.tables[TableLayout::ss(P) + i];
    }
    for (int k = i; k < 4 * (K + 1); k += kSparseThreads) {
        const int r = k / (K + 1), d = k - r * (K + 1);
        double* dst = r == 0 ? cre : r == 1 ? cim : r == 2 ? dre : dim;
        dst[d] = a.coef[k];
        if (F32) {
            float* dstf = r == 0 ? cref : r == 1 ? cimf : r == 2 ? dref : dimf;
            dstf[d] = (float)a.coef[k];
        }
    }
    if (F32) {
        for (int k = i; k < P * P; k += kSparseThreads) {
            const double re = a.tables[2 * k], im = a.tables[2 * k + 1];
            lk4[k] = (float)(0.5 * log(re * re + im * im));
            ak4[k] = (float)atan2(im, re);
        }
        if (i < P) {
            dsf[i] = (float)a.tables[TableLayout::ds(P) + i];
            ssf[i] = (float)a.tables[TableLayout::ss(P) + i];
        }
    }
    __syncthreads();
    if (P == 4 && i == 0) {
        const double D = ds[1];
        e0f0[0] = exp(-D * (cre[0] * D));
        e0f0[1] = exp(-D * (dre[0] * D));
    }
    // the chunk tables: parent point j = c*PPC + u lies at lag j+1 and goes to
    // the child's position j+1 (dropped at K)
    const int n_chunks = (K + PPC - 1) / PPC;
    ulonglong2 (*const gtab)[kChunkVals] =
        reinterpret_cast<ulonglong2 (*)[kChunkVals]>(chunk_lds + sparse_itab_bytes<F32>(n_chunks));
    for (int e = i; e < n_chunks * kChunkVals; e += kSparseThreads) {
        const int c = e / kChunkVals, v = e % kChunkVals;
        Real A = 0, B = 0, Ac = 0, Bc = 0;
        unsigned long long kp = 0ull, np = 0ull;
#pragma unroll
        for (int u = 0; u < PPC; ++u) {
            const unsigned int x = (unsigned int)((v >> (BP * u)) & DM);
            const int j = c * PPC + u;
            if ((int)x >= P) continue;                       // not a point (three levels)
            if (j < dmax) {
                if (F32) {
                    A = __builtin_fmaf(cref[j + 1], dsf[x], A);
                    B = __builtin_fmaf(cimf[j + 1], ssf[x], B);
                    Ac = __builtin_fmaf(dref[j + 1], dsf[x], Ac);
                    Bc = __builtin_fmaf(dimf[j + 1], ssf[x], Bc);
                } else {
                    A = __builtin_fma(cre[j + 1], ds[x], A);
                    B = __builtin_fma(cim[j + 1], ss[x], B);
                    Ac = __builtin_fma(dre[j + 1], ds[x], Ac);
                    Bc = __builtin_fma(dim[j + 1], ss[x], Bc);
                }
            }
            if (j + 1 < K) {
                const int m = pmap[j + 1];
                if (m >= 256) np |= (unsigned long long)x << (m - 256);
                else kp |= (unsigned long long)x << m;
            }
        }
        Real2 ab, abc;
        ab.x = A; ab.y = B; abc.x = Ac; abc.y = Bc;
        itab[c][v][0] = ab;
        itab[c][v][1] = abc;
        gtab[c][v] = make_ulonglong2(kp, np);
    }
    if (i == 0) {
        unsigned long long n = 0ull;
        for (int s = 0; s < kSegs; ++s) {
            seg_pre[s] = n;
            n += seg_groups(a, (t - 1) & 1, s);
        }
        seg_pre[kSegs] = n;
    }
    __syncthreads();

    double acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0.0;
    const bool failed = error_word(a.error) != 0u;
    const unsigned long long n_in = groups_in(a);
    // place of input group g: the last segment starting at or before g (empty
    // segments start where the next one does)
    auto at = [&](unsigned long long g) {
        int s = 0;
#pragma unroll
        for (int step = kSegs / 2; step > 0; step >>= 1)
            if (seg_pre[s + step] <= g) s += step;
        return (unsigned long long)s * a.seg_cap + (g - seg_pre[s]);
    };
    const unsigned long long N = failed ? 0ull : n_in;
    const unsigned long long tm = table_mask(a, n_in);
    const bool packed = a.packed != 0;
    const unsigned long long omask = packed ? other_mask(a) : 0ull;
    const unsigned long long qmask = ~((1ull << a.qbits) - 1ull);
    const unsigned long long cmask = a.cmask;
    const unsigned long long stride = (unsigned long long)gridDim.x * kSparseThreads;

    // A slot of the table takes its updates from a child or from a merged LDS
    // slot (all its children's sum and best word).  Unpacked form: the entry
    // (slot, other word, q) that the resolve pass reads.
    auto update = [&](unsigned long long sl, unsigned long long word, unsigned long long nk, double wr, double wi,
                      unsigned long long entry) {
        SpSlot* const e = a.slot + sl;
        atomicMax(&e->best, word);
        if (!packed) {
            a.cslot[entry] = (unsigned int)sl;
            a.cN[entry] = nk;
            a.cq[entry] = word;
        }
        unsafeAtomicAdd(&e->wr, wr);
        unsafeAtomicAdd(&e->wi, wi);
    };
    auto overflow = [&](unsigned long long entry) {
        raise_error(a.error, t, kErrOverflow);
        if (!packed) a.cslot[entry] = ~0u;
    };
    // partition merge: a merged slot (or a child that found the LDS table full)
    // becomes one entry of its key's partition
    const bool parted = a.part != 0;
    const unsigned int n_part = parted ? n_partitions(a, n_in) : 1u;
    auto append = [&](unsigned long long key, unsigned long long best, unsigned long long other, double wr,
                      double wi) {
        const unsigned int pp = partition_of(key, n_part);
        const unsigned int pos = atomicAdd(a.pcount + pp, 1u);
        if (pos < kPartCap) {
            const size_t e = (size_t)pp * kPartCap + pos;
            PartRec r;
            r.x = key;
            r.y = best;
            if (!packed && a.pfit) {
                const int kb = BP * a.nq;
                r.y = 0ull;
                put_bits(r.x, r.y, other, kb);
                put_bits(r.x, r.y, best >> a.qbits, kb + BP * a.nn);
            } else if (!packed) {
                a.pother[e] = other;
            }
            r.wr = wr;
            r.wi = wi;
            a.prec[e] = r;
        } else {
            raise_error(a.error, t, kErrOverflow);
        }
    };

    unsigned int pass = 0u;
    for (unsigned long long base = (unsigned long long)blockIdx.x * kSparseThreads; base < N; base += stride, ++pass) {
        // this pass: parents [base, base + n_par); unpacked-form entries
        // [base*P, base*P + n_ent): merged LDS slots from the bottom, children
        // that found the LDS full from the top, the rest marked unused
        const unsigned int n_par = (unsigned int)((N - base) < kSparseThreads ? (N - base) : kSparseThreads);
        const unsigned int n_ent = n_par * P;
        const unsigned long long ebase = base * P;
        unsigned int* const ovf = &lovf[pass & 1u];
        if (i == 0) lovf[(pass + 1u) & 1u] = 0u;          // the next pass's counter (last read a pass ago)
        unsigned int mls[P];                              // unpacked: LDS slot, q and other word of each child
        unsigned long long mq[P], mnk[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { mls[p] = ~0u; mq[p] = 0ull; mnk[p] = 0ull; }

        const unsigned long long g = base + i;
        if (g < N) {
            const unsigned long long gp = at(g);
            const Hist<W> h = load_hist<W>(a.h_in, gp);
            double2 Wt = make_double2(0.0, 0.0);
            float2 Wl = make_float2(0.0f, 0.0f);
            if (F32) Wl = a.wf_in[gp];
            else Wt = a.w_in[gp];
            // influence sums over lags 1..dmax, and the children's key and other
            // points but for the new point
            Real A = 0, B = 0, Ac = 0, Bc = 0;
            unsigned long long kb = 0ull, nb = 0ull;
            for (int c = 0; c < n_chunks; ++c) {
                const unsigned int v = chunk_at<W>(h, c);
                const Real2 ab = itab[c][v][0], abc = itab[c][v][1];
                const ulonglong2 kn = gtab[c][v];
                A += ab.x;
                B += ab.y;
                Ac += abc.x;
                Bc += abc.y;
                kb |= kn.x;
                nb |= kn.y;
            }
            const int h0 = (int)(h.w[0] & DM);
            // two levels, FP64: pairs (0,1) and (1,0) have ds = +D, -D and equal ss,
            // so their exponents are mirror images and share one exp and one sincos
            double er1 = 1.0, ei1 = 0.0, er2 = 1.0, ei2 = 0.0, fr1 = 1.0, fi1 = 0.0, fr2 = 1.0, fi2 = 0.0;
            if constexpr (P == 4 && !F32) {
                const double D = ds[1], Sg = ss[1];
                const double x = D * A, y = D * __builtin_fma(cim[0], Sg, B);
                const double xc = D * Ac, yc = D * __builtin_fma(dim[0], Sg, Bc);
                const double ex = exp_fast(x), exc = exp_fast(xc);
                const double iex = recip(ex), iexc = recip(exc);
                double sy, cy, syc, cyc;
                sincos_fast(y, &sy, &cy);
                sincos_fast(yc, &syc, &cyc);
                const double e0 = e0f0[0], f0 = e0f0[1];
                er1 = e0 * iex * cy;  ei1 = -(e0 * iex * sy);
                er2 = e0 * ex * cy;   ei2 = e0 * ex * sy;
                fr1 = f0 * iexc * cyc; fi1 = -(f0 * iexc * syc);
                fr2 = f0 * exc * cyc;  fi2 = f0 * exc * syc;
            }
            // two levels, FP32: the same mirror, in FP32; the parent leaves the log
            // domain once and each child is its product with K4 and the factor
            float pwr = 0.f, pwi = 0.f;
            float ger1 = 1.f, gei1 = 0.f, ger2 = 1.f, gei2 = 0.f, gfr1 = 1.f, gfi1 = 0.f, gfr2 = 1.f, gfi2 = 0.f;
            if constexpr (P == 4 && F32) {
                const float m = expf(Wl.x);
                float sa, ca;
                sincos_f32(Wl.y, sa, ca);
                pwr = m * ca;
                pwi = m * sa;
                const float D = dsf[1], Sg = ssf[1];
                const float x = D * (float)A, y = D * __builtin_fmaf(cimf[0], Sg, (float)B);
                const float xc = D * (float)Ac, yc = D * __builtin_fmaf(dimf[0], Sg, (float)Bc);
                const float ex = expf(x), exc = expf(xc);
                const float iex = 1.0f / ex, iexc = 1.0f / exc;
                float sy, cy, syc, cyc;
                sincos_f32(y, sy, cy);
                sincos_f32(yc, syc, cyc);
                const float e0 = (float)e0f0[0], f0 = (float)e0f0[1];
                ger1 = e0 * iex * cy;  gei1 = -(e0 * iex * sy);
                ger2 = e0 * ex * cy;   gei2 = e0 * ex * sy;
                gfr1 = f0 * iexc * cyc; gfi1 = -(f0 * iexc * syc);
                gfr2 = f0 * exc * cyc;  gfi2 = f0 * exc * syc;
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                double wr, wi, rr, ri;   // the child's amplitude; its rho(t) term
                if constexpr (P == 4 && F32) {
                    const float k4r = (float)k4re[p * P + h0], k4i = (float)k4im[p * P + h0];
                    const float br = pwr * k4r - pwi * k4i;
                    const float bi = pwr * k4i + pwi * k4r;
                    float er = 1.f, ei = 0.f, fr = 1.f, fi = 0.f;
                    if (p == 1) { er = ger1; ei = gei1; fr = gfr1; fi = gfi1; }
                    if (p == 2) { er = ger2; ei = gei2; fr = gfr2; fi = gfi2; }
                    const float cr = br * er - bi * ei, ci = br * ei + bi * er;
                    wr = (double)cr;
                    wi = (double)ci;
                    rr = (double)(cr * fr - ci * fi);
                    ri = (double)(cr * fi + ci * fr);
                } else if constexpr (F32) {
                    float lr = Wl.x + lk4[p * P + h0], ph = Wl.y + ak4[p * P + h0];
                    float lc = lr, pc = ph;
                    const float dsp = dsf[p], ssp = ssf[p];
                    if (dsp != 0.0f) {
                        lr += -dsp * (cref[0] * dsp + A);
                        ph += -dsp * (cimf[0] * ssp + B);
                        lc = lr - dsp * (dref[0] * dsp + Ac);
                        pc = ph - dsp * (dimf[0] * ssp + Bc);
                    }
                    const float m = expf(lr), mc = expf(lc);
                    float sn, cs2, snc, csc;
                    sincosf(ph, &sn, &cs2);
                    sincosf(pc, &snc, &csc);
                    wr = (double)(m * cs2);
                    wi = (double)(m * sn);
                    rr = (double)(mc * csc);
                    ri = (double)(mc * snc);
                } else {
                    double er = 1.0, ei = 0.0, fr = 1.0, fi = 0.0;
                    if constexpr (P == 4) {
                        if (p == 1) { er = er1; ei = ei1; fr = fr1; fi = fi1; }
                        if (p == 2) { er = er2; ei = ei2; fr = fr2; fi = fi2; }
                    } else {
                        const double dsp = ds[p], ssp = ss[p];
                        if (dsp != 0.0) {
                            const double e = exp_fast(-dsp * (cre[0] * dsp + A));
                            double sn, cs2;
                            sincos_fast(-dsp * (cim[0] * ssp + B), &sn, &cs2);
                            er = e * cs2;
                            ei = e * sn;
                            const double f = exp_fast(-dsp * (dre[0] * dsp + Ac));
                            double fs, fc;
                            sincos_fast(-dsp * (dim[0] * ssp + Bc), &fs, &fc);
                            fr = f * fc;
                            fi = f * fs;
                        }
                    }
                    const double k4r = k4re[p * P + h0], k4i = k4im[p * P + h0];
                    const double br = Wt.x * k4r - Wt.y * k4i;
                    const double bi = Wt.x * k4i + Wt.y * k4r;
                    wr = br * er - bi * ei;
                    wi = br * ei + bi * er;
                    rr = wr * fr - wi * fi;
                    ri = wr * fi + wi * fr;
                }
                const double n2 = norm2_nocontract(wr, wi);
                if (!((a.theta2 == 0.0) || !(n2 < a.theta2))) {
                    acc[2 * P] += sqrt(n2);
                    continue;
                }
                acc[2 * p] += rr;
                acc[2 * p + 1] += ri;
                acc[2 * P + 1] += 1.0;
                const unsigned long long key = kb | (kshift < 0 ? 0ull : (unsigned long long)p << kshift);
                const unsigned long long kk = key + 1ull;         // stored form: zero is a free slot
                const unsigned long long nk = nb | (nshift < 0 ? 0ull : (unsigned long long)p << nshift);
                const unsigned long long n2b = (unsigned long long)__double_as_longlong(n2);
                const unsigned long long word =
                    packed ? (((n2b >> a.qbits) << (a.qbits + 1)) | (omask ^ nk)) : (n2b & qmask);
                // merge in the LDS first
                unsigned int ls = (unsigned int)(mix64(key) >> 40) & (unsigned int)(kLds - 1);
                bool in_lds = false;
                for (int probe = 0; probe < kLdsProbe; ++probe) {
                    const unsigned long long prev = atomicCAS(&lkey[ls], 0ull, kk);
                    if (prev == 0ull || prev == kk) {
                        in_lds = true;
                        break;
                    }
                    ls = (ls + 1u) & (unsigned int)(kLds - 1);
                }
                if (in_lds) {
                    atomicMax(&lbest[ls], word);
                    unsafeAtomicAdd(&lwr[ls], wr);
                    unsafeAtomicAdd(&lwi[ls], wi);
                    if (!packed) { mls[p] = ls; mq[p] = word; mnk[p] = nk; }
                } else if (parted) {
                    // no room in the LDS: an entry of its own
                    append(key, word, nk, wr, wi);
                } else {
                    // no room in the LDS: straight to the table
                    const unsigned long long entry = packed ? 0ull : ebase + n_ent - 1u - atomicAdd(ovf, 1u);
                    unsigned long long sl = home_slot(key, cmask, tm), prev = 0ull;
                    int probe = 0;
                    for (; probe < kMaxProbe; ++probe) {
                        prev = atomicCAS(&a.slot[sl].key, 0ull, kk);
                        if (prev == 0ull || prev == kk) break;
                        sl = (sl + 1ull) & tm;
                    }
                    if (probe < kMaxProbe) update(sl, word, nk, wr, wi, entry);
                    else overflow(entry);
                }
            }
        }
        __syncthreads();

        // unpacked form: among the LDS children at a slot's largest q, the
        // smallest other word, kept in the best-word array once its q is
        // saved; and the entries of the used LDS slots
        unsigned long long lbal[kLdsRows], savedq[kLdsRows];
        if (!packed) {
            bool win[P];
#pragma unroll
            for (int p = 0; p < P; ++p) win[p] = mls[p] != ~0u && mq[p] == lbest[mls[p]];
#pragma unroll
            for (int r = 0; r < kLdsRows; ++r) {
                const int ls = r * kSparseThreads + i;
                savedq[r] = lbest[ls];
                lbal[r] = __ballot(lkey[ls] != 0ull);
                if (lane == 0u) loff[r][wave] = (unsigned int)__popcll(lbal[r]);
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < kLdsRows; ++r) lbest[r * kSparseThreads + i] = ~0ull;
            if (i == 0) {
                unsigned int tot = 0u;
                for (int r = 0; r < kLdsRows; ++r)
                    for (int w = 0; w < kSpWaves; ++w) {
                        const unsigned int c = loff[r][w];
                        loff[r][w] = tot;
                        tot += c;
                    }
                lused = tot;
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < P; ++p)
                if (win[p]) atomicMin(&lbest[mls[p]], mnk[p]);
            __syncthreads();
        }

        if (parted) {
            // each used LDS slot is one entry of its key's partition
#pragma unroll
            for (int r = 0; r < kLdsRows; ++r) {
                const int ls = r * kSparseThreads + i;
                const unsigned long long kk = lkey[ls];
                if (kk) append(kk - 1ull, packed ? lbest[ls] : savedq[r], packed ? 0ull : lbest[ls], lwr[ls], lwi[ls]);
                lkey[ls] = 0ull;
                lbest[ls] = 0ull;
                lwr[ls] = 0.0;
                lwi[ls] = 0.0;
            }
        } else {
        // each used LDS slot is one insertion into the table; the first probes
        // of a thread's slots are in flight together
            unsigned long long fkk[kLdsRows], fsl[kLdsRows], fprev[kLdsRows];
#pragma unroll
            for (int r = 0; r < kLdsRows; ++r) {
                fkk[r] = lkey[r * kSparseThreads + i];
                fsl[r] = fkk[r] ? home_slot(fkk[r] - 1ull, cmask, tm) : 0ull;
                fprev[r] = 0ull;
            }
#pragma unroll
            for (int r = 0; r < kLdsRows; ++r)
                if (fkk[r]) fprev[r] = atomicCAS(&a.slot[fsl[r]].key, 0ull, fkk[r]);
#pragma unroll
            for (int r = 0; r < kLdsRows; ++r) {
                const int ls = r * kSparseThreads + i;
                if (fkk[r]) {
                    const unsigned long long entry =
                        packed ? 0ull : ebase + loff[r][wave] + rank_below(lbal[r]);
                    for (int probe = 1; fprev[r] != 0ull && fprev[r] != fkk[r] && probe < kMaxProbe; ++probe) {
                        fsl[r] = (fsl[r] + 1ull) & tm;
                        fprev[r] = atomicCAS(&a.slot[fsl[r]].key, 0ull, fkk[r]);
                    }
                    if (fprev[r] == 0ull || fprev[r] == fkk[r]) {
                        if (packed) update(fsl[r], lbest[ls], 0ull, lwr[ls], lwi[ls], entry);
                        else update(fsl[r], savedq[r], lbest[ls], lwr[ls], lwi[ls], entry);
                    } else {
                        overflow(entry);
                    }
                }
                lkey[ls] = 0ull;
                lbest[ls] = 0ull;
                lwr[ls] = 0.0;
                lwi[ls] = 0.0;
            }
        }
        if (!packed && !parted) {
            // entries of this pass that no child took
            const unsigned int lo = lused, hi = n_ent - *ovf;
            for (unsigned int j = lo + (unsigned int)i; j < hi; j += kSparseThreads) a.cslot[ebase + j] = ~0u;
        }
        __syncthreads();   // the LDS table is clear for the next pass
    }

    // this workgroup's sums, in a fixed order
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0u) wpart[wave][k] = v;
    }
    __syncthreads();
    if (i < S) {
        double v = 0.0;
        for (int w = 0; w < kSpWaves; ++w) v += wpart[w][i];
        a.partials[(size_t)i * a.grid + blockIdx.x] = v;
    }
}

// The FP64 sum w of a group back to FP32 (ln|w|, arg w): FP64 log and atan2,
// rounded once.  Not inlined, so that the unrolled rows of the compact loop do
// not each hold the registers of the two functions.

// unpacked form: among the children with the key's largest quantised |w|^2,
// the smallest points at the other positions (oldest first)
template <int P>
__global__ __launch_bounds__(kSparseThreads) void sparse_resolve(const SparseArgs a) {
    if (error_word(a.error) != 0u) return;
    const unsigned long long n = groups_in(a) * P;
    for (unsigned long long ci = (unsigned long long)blockIdx.x * kSparseThreads + threadIdx.x; ci < n;
         ci += (unsigned long long)gridDim.x * kSparseThreads) {
        const unsigned int s = a.cslot[ci];
        if (s == ~0u) continue;
        if (a.cq[ci] == a.slot[s].best) atomicMin(a.tN + s, a.cN[ci]);
    }
}

// Tiles of kRows x kSparseThreads slots: each tile takes its place in the
// output with one counter update and writes its used slots in slot order.
// The used slots of a tile are first listed in the LDS, so that consecutive
// threads rebuild consecutive groups (most slots are free: the table is sized
// for twice the children, and children merge).
template <int BP, int W, bool F32>
__global__ __launch_bounds__(kSparseThreads) void sparse_compact(const SparseArgs a) {
    __shared__ unsigned int wcnt[kRows][kSpWaves];
    __shared__ unsigned int tile_base, tile_used;
    __shared__ unsigned short lpos[kTile];                  // used slots of the tile, in slot order
    __shared__ unsigned long long lkey[kTile];              // and their stored keys
    __shared__ HistTab htab;
    build_hist_tab<BP>(a, htab);
    const int ns = hist_slices<BP>(a);
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const bool failed = error_word(a.error) != 0u;
    // this workgroup's output segment
    const unsigned int seg = blockIdx.x % (unsigned int)kSegs;
    unsigned int* const out_count = a.count + seg_counter(a.t & 1, (int)seg);
    const unsigned long long seg_base = (unsigned long long)seg * a.seg_cap;
    const unsigned long long tm = table_mask(a, groups_in(a));
    const unsigned long long n_tiles = (tm + kTile) / kTile;
    const bool packed = a.packed != 0;
    const unsigned long long omask = packed ? other_mask(a) : 0ull;
    for (unsigned long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const unsigned long long s0 = tile * kTile;
        unsigned long long kk[kRows], bal[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const unsigned long long sl = s0 + (unsigned long long)(r * kSparseThreads + i);
            kk[r] = sl <= tm ? a.slot[sl].key : 0ull;
            bal[r] = __ballot(kk[r] != 0ull);
            if (lane_id() == 0u) wcnt[r][wave] = (unsigned int)__popcll(bal[r]);
        }
        __syncthreads();
        if (i == 0) {
            unsigned int tot = 0u;
            for (int r = 0; r < kRows; ++r)
                for (int w = 0; w < kSpWaves; ++w) {
                    const unsigned int c = wcnt[r][w];
                    wcnt[r][w] = tot;
                    tot += c;
                }
            tile_used = tot;
            tile_base = tot ? atomicAdd(out_count, tot) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            if (kk[r] == 0ull) continue;
            const unsigned int j = wcnt[r][wave] + rank_below(bal[r]);
            lpos[j] = (unsigned short)(r * kSparseThreads + i);
            lkey[j] = kk[r];
        }
        __syncthreads();
        const unsigned int base = tile_base, used = tile_used;
        for (unsigned int j = (unsigned int)i; j < used; j += kSparseThreads) {
            const unsigned long long sl = s0 + lpos[j];
            const unsigned long long idx = (unsigned long long)base + j;
            SpSlot* const e = a.slot + sl;
            unsigned long long nk = 0ull;
            if (packed) {
                nk = (e->best & omask) ^ omask;
            } else {
                nk = a.tN[sl];
                a.tN[sl] = ~0ull;
            }
            if (!failed && idx < a.seg_cap) {
                // the key's points at the merge positions, the representative's elsewhere
                const unsigned long long key = lkey[j] - 1ull;
                const Hist<W> hist = hist_from<BP, W>(htab, key, nk, ns);
                const unsigned long long o = seg_base + idx;
#pragma unroll
                for (int w = 0; w < W; ++w) a.h_out[o * W + w] = hist.w[w];
                if (F32) {
                    a.wf_out[o] = to_log_domain32(e->wr, e->wi);
                } else {
                    a.w_out[o] = make_double2(e->wr, e->wi);
                }
            } else if (!failed) {
                raise_error(a.error, a.t, kErrOverflow);
            }
            e->key = 0ull;
            e->best = 0ull;
            e->wr = 0.0;
            e->wi = 0.0;
        }
        __syncthreads();   // the LDS list and counts are rewritten by the next tile
    }
}

// Partition merge: workgroups take the step's partitions in turn.  A
// partition's entries merge in an LDS table (key, representative word, weight
// sums; unpacked form: then the smallest other points at the largest quantised
// |w|^2), and its groups are written at one counter update, their histories
// rebuilt from the key and the representative's other points.  The partition's
// counter is cleared for the next step.  The rounds are pipelined: a round's
// entries are loaded while the round before takes its place in the output, and
// the count of the round after is loaded with them.
template <int BP, int W, bool F32>
__global__ __launch_bounds__(kSparseThreads) void sparse_pmerge(const SparseArgs a) {
    constexpr int kRowsP = kPartLds / kSparseThreads;
    constexpr int kPer = (kPartCap + kSparseThreads - 1) / kSparseThreads;   // entries per thread
    __shared__ unsigned long long lk[kPartLds], lb[kPartLds], lo[kPartLds];
    __shared__ double lwr[kPartLds], lwi[kPartLds];
    __shared__ unsigned int wcnt[kRowsP][kSpWaves];
    __shared__ unsigned int base_s, used_s;
    __shared__ unsigned short lslot[kPartLds];               // the round's used slots, in slot order
    __shared__ HistTab htab;
    build_hist_tab<BP>(a, htab);
    const int ns = hist_slices<BP>(a);
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const bool failed = error_word(a.error) != 0u;
    // this workgroup's output segment
    const unsigned int seg = blockIdx.x % (unsigned int)kSegs;
    unsigned int* const out_count = a.count + seg_counter(a.t & 1, (int)seg);
    const unsigned long long seg_base = (unsigned long long)seg * a.seg_cap;
    const unsigned int n_part = n_partitions(a, groups_in(a));
    const unsigned int G = gridDim.x;
    const bool packed = a.packed != 0;
    const unsigned long long omask = packed ? other_mask(a) : 0ull;
    for (int k = i; k < kPartLds; k += kSparseThreads) {
        lk[k] = 0ull;
        lb[k] = 0ull;
        lo[k] = ~0ull;
        lwr[k] = 0.0;
        lwi[k] = 0.0;
    }

    const bool fit = !packed && a.pfit != 0;
    const int kb = BP * a.nq, ob = BP * a.nn;
    const unsigned long long kmask = (1ull << kb) - 1ull;
    // the entries of one partition, kPer per thread (beyond kPartCap: reported by
    // expand).  The loads take no branch, so that they are all in flight at once:
    // a thread past the count reads the partition's last entry again (its line is
    // read anyway), a round past the last partition reads partition 0; those
    // values are not used.
    unsigned long long ek[kPer], eb[kPer], eo[kPer];
    double2 ew[kPer];
    auto load = [&](unsigned int pp, unsigned int n) {
        const size_t p0 = (size_t)(pp < n_part ? pp : 0u) * kPartCap;
        const unsigned int last = n ? n - 1u : 0u;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const unsigned int e = (unsigned int)i + (unsigned int)q * kSparseThreads;
            const size_t ge = p0 + (e < last ? e : last);
            const PartRec r = a.prec[ge];
            ek[q] = r.x;
            eb[q] = r.y;
            ew[q] = make_double2(r.wr, r.wi);
            eo[q] = packed || fit ? 0ull : a.pother[ge];
        }
        if (fit) {
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const unsigned long long lo = ek[q], hi = eb[q];
                ek[q] = lo & kmask;
                eo[q] = bits_at(lo, hi, kb, ob);
                eb[q] = bits_at(lo, hi, kb + ob, 63 - a.qbits) << a.qbits;
            }
        }
    };
    // a partition's count as stored (clamped where it is used, so that the
    // load of the next round's count is not waited for at once)
    auto count_of = [&](unsigned int pp) { return pp < n_part ? a.pcount[pp] : 0u; };
    auto clamp = [](unsigned int c) { return c < kPartCap ? c : kPartCap; };
    unsigned int pp = blockIdx.x;
    unsigned int n_cur = clamp(count_of(pp));
    load(pp, n_cur);
    unsigned int n_next = count_of(pp + G);
    __syncthreads();

    for (; pp < n_part; pp += G) {
        // this round's entries into the table: at most kPartCap keys in
        // kPartLds slots, so a free slot is always found
        unsigned int ms[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const unsigned int e = (unsigned int)i + (unsigned int)q * kSparseThreads;
            ms[q] = ~0u;
            if (e < n_cur) {
                const unsigned long long kk = ek[q] + 1ull;
                unsigned int sl = (unsigned int)mix64(ek[q]) & (unsigned int)(kPartLds - 1);
                for (int probe = 0; probe < kPartLds; ++probe) {
                    const unsigned long long prev = atomicCAS(&lk[sl], 0ull, kk);
                    if (prev == 0ull || prev == kk) break;
                    sl = (sl + 1u) & (unsigned int)(kPartLds - 1);
                }
                ms[q] = sl;
                atomicMax(&lb[sl], eb[q]);
                unsafeAtomicAdd(&lwr[sl], ew[q].x);
                unsafeAtomicAdd(&lwi[sl], ew[q].y);
            }
        }
        __syncthreads();
        if (!packed) {
#pragma unroll
            for (int q = 0; q < kPer; ++q)
                if (ms[q] != ~0u && eb[q] == lb[ms[q]]) atomicMin(&lo[ms[q]], eo[q]);
            __syncthreads();
        }
        // the used slots' places: per row and wave, then one counter update
        unsigned long long bal[kRowsP];
#pragma unroll
        for (int r = 0; r < kRowsP; ++r) {
            bal[r] = __ballot(lk[r * kSparseThreads + i] != 0ull);
            if (lane == 0u) wcnt[r][wave] = (unsigned int)__popcll(bal[r]);
        }
        __syncthreads();
        // the next round's entries, and the count of the round after, are in
        // flight while the place is taken
        const unsigned int pn = pp + G;
        n_cur = clamp(n_next);
        load(pn, n_cur);
        n_next = count_of(pn + G);
        if (i == 0) {
            unsigned int tot = 0u;
            for (int r = 0; r < kRowsP; ++r)
                for (int w = 0; w < kSpWaves; ++w) {
                    const unsigned int c = wcnt[r][w];
                    wcnt[r][w] = tot;
                    tot += c;
                }
            base_s = tot ? atomicAdd(out_count, tot) : 0u;
            used_s = tot;
            a.pcount[pp] = 0u;                                // the next step's appends start at zero
        }
        __syncthreads();
        const unsigned int base = base_s, used = used_s;
        // the used slots listed in slot order, so that consecutive threads
        // write consecutive groups
#pragma unroll
        for (int r = 0; r < kRowsP; ++r) {
            const int sl = r * kSparseThreads + i;
            if (lk[sl] != 0ull) lslot[wcnt[r][wave] + rank_below(bal[r])] = (unsigned short)sl;
        }
        __syncthreads();
        // write the groups, and free the slots for the next round
        for (unsigned int j = (unsigned int)i; j < used; j += kSparseThreads) {
            const int sl = lslot[j];
            const unsigned long long kk = lk[sl];
            const unsigned long long idx = (unsigned long long)base + j;
            if (!failed && idx < a.seg_cap) {
                const unsigned long long key = kk - 1ull;
                const unsigned long long nk = packed ? ((lb[sl] & omask) ^ omask) : lo[sl];
                // the key's points at the merge positions, the representative's elsewhere
                const Hist<W> hist = hist_from<BP, W>(htab, key, nk, ns);
                const unsigned long long o = seg_base + idx;
#pragma unroll
                for (int w = 0; w < W; ++w) a.h_out[o * W + w] = hist.w[w];
                if (F32) a.wf_out[o] = to_log_domain32(lwr[sl], lwi[sl]);
                else a.w_out[o] = make_double2(lwr[sl], lwi[sl]);
            } else if (!failed) {
                raise_error(a.error, a.t, kErrOverflow);
            }
            lk[sl] = 0ull;
            lb[sl] = 0ull;
            lo[sl] = ~0ull;
            lwr[sl] = 0.0;
            lwi[sl] = 0.0;
        }
        __syncthreads();   // the table is free for the next round
    }
}

template <int P>
__global__ __launch_bounds__(kSparseThreads) void sparse_reduce(const SparseArgs a) {
    constexpr int S = partial_stride(P);
    __shared__ double wred[kSpWaves][S];
    __shared__ int keep_s;
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const int t = a.t;
    double acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0.0;
    for (int b = i; b < a.grid; b += kSparseThreads)
#pragma unroll
        for (int k = 0; k < S; ++k) acc[k] += a.partials[(size_t)k * a.grid + b];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0u) wred[wave][k] = v;
    }
    __syncthreads();
    if (i == 0) {
        // the groups stored: over the capacity, the step fails
        unsigned long long n_stored = 0ull;
        for (int s = 0; s < kSegs; ++s) n_stored += a.count[seg_counter(t & 1, s)];
        if (n_stored > (unsigned long long)a.cap) raise_error(a.error, t, kErrOverflow);
        const unsigned int err = error_word(a.error);
        const bool keep = err == 0u || (int)(err >> 4) > t;
        keep_s = keep ? 1 : 0;
        const unsigned long long n_in = groups_in(a);
        if (keep) {
            double sum[S];
#pragma unroll
            for (int k = 0; k < S; ++k) {
                sum[k] = 0.0;
                for (int w = 0; w < kSpWaves; ++w) sum[k] += wred[w][k];
            }
#pragma unroll
            for (int p = 0; p < P; ++p) a.rho_hist[(size_t)t * P + p] = make_double2(sum[2 * p], sum[2 * p + 1]);
            StepStatsDev st;
            st.n_groups = n_in;
            st.n_children = n_in * P;
            st.n_survivors = (unsigned long long)sum[2 * P + 1];
            st.n_stored = n_stored;
            st.dropped_abs = sum[2 * P];
            st.pad = 0.0;
            a.stats_hist[t] = st;
        }
    }
    __syncthreads();
    // the counters step t+1 writes: they held this step's input counts
    if (keep_s && i < kSegs) a.count[seg_counter((t + 1) & 1, i)] = 0u;
}

}  // namespace

template <int P, int BP, int W, bool F32>
void launch_sparse(const SparseArgs& a, hipStream_t st, hipEvent_t after_expand) {
    const int g = a.grid;
    constexpr int ppc = kChunkBits / BP;
    const size_t chunk_bytes = std::max(sparse_chunk_lds<F32>((a.K + ppc - 1) / ppc), kExpandLdsFloor);
    hipLaunchKernelGGL((sparse_expand<P, BP, W, F32>), dim3(g), dim3(kSparseThreads), chunk_bytes, st, a);
    if (after_expand) (void)hipEventRecord(after_expand, st);
    if (a.part) {
        hipLaunchKernelGGL((sparse_pmerge<BP, W, F32>), dim3(a.grid_merge), dim3(kSparseThreads), 0, st, a);
    } else {
        if (!a.packed) hipLaunchKernelGGL((sparse_resolve<P>), dim3(g), dim3(kSparseThreads), 0, st, a);
        hipLaunchKernelGGL((sparse_compact<BP, W, F32>), dim3(g), dim3(kSparseThreads), 0, st, a);
    }
    hipLaunchKernelGGL((sparse_reduce<P>), dim3(1), dim3(kSparseThreads), 0, st, a);
}

template <bool F32>
int launch_sparse_form(const SparseArgs& a, hipStream_t st, hipEvent_t ev) {
    if (a.P == 4 && a.hw == 1) launch_sparse<4, 2, 1, F32>(a, st, ev);
    else if (a.P == 4 && a.hw == 2) launch_sparse<4, 2, 2, F32>(a, st, ev);
    else if (a.P == 9 && a.hw == 1) launch_sparse<9, 4, 1, F32>(a, st, ev);
    else if (a.P == 9 && a.hw == 2) launch_sparse<9, 4, 2, F32>(a, st, ev);
    else if (a.P == 16 && a.hw == 1) launch_sparse<16, 4, 1, F32>(a, st, ev);
    else if (a.P == 16 && a.hw == 2) launch_sparse<16, 4, 2, F32>(a, st, ev);
    else return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

template <int BP, int W, bool F32>
int merge_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sparse_pmerge<BP, W, F32>, kSparseThreads, 0) != hipSuccess)
        return 0;
    return n;
}

int sparse_merge_grid(int P, int hw, bool f32, int n_cu) {
    const int bp = P == 4 ? 2 : 4;
    int per_cu = 0;
    if (bp == 2 && hw == 1) per_cu = f32 ? merge_blocks_per_cu<2, 1, true>() : merge_blocks_per_cu<2, 1, false>();
    else if (bp == 2) per_cu = f32 ? merge_blocks_per_cu<2, 2, true>() : merge_blocks_per_cu<2, 2, false>();
    else if (hw == 1) per_cu = f32 ? merge_blocks_per_cu<4, 1, true>() : merge_blocks_per_cu<4, 1, false>();
    else per_cu = f32 ? merge_blocks_per_cu<4, 2, true>() : merge_blocks_per_cu<4, 2, false>();
    const int g = std::max(per_cu, 1) * std::max(n_cu, 1) / kSegs * kSegs;
    return std::max(g, kSegs);
}

int launch_sparse_step(const SparseArgs& a, void* stream, void* after_expand) {
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t ev = (hipEvent_t)after_expand;
    return a.wf_in ? launch_sparse_form<true>(a, st, ev) : launch_sparse_form<false>(a, st, ev);
}

}  // namespace quapi_dev
