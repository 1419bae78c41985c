// One time step of MACGIC-iQUAPI for masks whose merge positions are not a
// contiguous run 0..L-1 (a MACGIC mask that keeps distant lags, Sec. 2.1).
// The groups a child joins are then not adjacent in key order, so the merge
// goes through an open-addressing hash table in HBM keyed on the child's
// points at the merge positions.
//
// State between steps: groups as full histories (point j = lag j at bits
// [BP*j, BP*j+BP), the newest point lowest) with their amplitudes, in no
// particular order.  One step is four kernels:
//   expand  - extend every group by every pair: weight times the propagator
//             element (eq. SysP) times the influence factor of the new point
//             (eq. inf_fun); drop children below theta (Sec. 2.1); add the
//             survivors to this workgroup's rho(t) sums with the end-point
//             correction of the final point (Sec. 3.2.1); insert each
//             survivor's merge key into the table, keep the key's largest
//             quantised |w|^2 and add the weight to the key's sum (the group
//             amplitude is the sum of all its members, Sec. 3.1.2);
//   resolve - among the children of a key with its largest quantised |w|^2,
//             keep the history that is smallest read from the oldest point
//             (the representative; with the newest point in the low bits the
//             packed history is that number);
//   compact - write one group per used slot and clear the slot;
//   reduce  - add up the workgroups' rho(t) and counters in workgroup order.
// The weight sums of the table are atomic and so in no fixed order; rho(t) is
// summed in a fixed order.

#include <hip/hip_runtime.h>

#include "quapi_device.h"
#include "quapi_host.h"

namespace quapi_dev {

namespace {

constexpr int kSpWaves = kSparseThreads / 64;
constexpr int kMaxProbe = 1 << 16;

// 64-bit finaliser of the SplitMix64 generator (Steele, Lea, Flood 2014), as
// the hash of a merge key
__device__ inline unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <int P, int BP>
__global__ __launch_bounds__(kSparseThreads) void sparse_expand(const SparseArgs a) {
    constexpr int S = partial_stride(P);
    constexpr unsigned long long DM = (1ull << BP) - 1;
    __shared__ double k4re[P * P], k4im[P * P], ds[P], ss[P];
    __shared__ double cre[kMaxK + 1], cim[kMaxK + 1], dre[kMaxK + 1], dim[kMaxK + 1];
    __shared__ double wpart[kSpWaves][S];
    __shared__ int qpos[kMaxK];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const int K = a.K, t = a.t, nq = a.nq;
    if (i < nq) qpos[i] = a.qpos[i];

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
    }
    __syncthreads();

    double acc[S];
#pragma unroll
    for (int k = 0; k < S; ++k) acc[k] = 0.0;
    const bool failed = error_word(a.error) != 0u;
    const unsigned int stored = a.count[(t - 1) & 1];
    const unsigned int N = failed ? 0u : (stored < (unsigned long long)a.cap ? stored : (unsigned int)a.cap);
    const int dmax = t < K ? t : K;
    const unsigned long long kmask = K * BP >= 64 ? ~0ull : ((1ull << (K * BP)) - 1ull);
    const unsigned int stride = gridDim.x * kSparseThreads;

    for (unsigned int g = blockIdx.x * kSparseThreads + i; g < N; g += stride) {
        const unsigned long long h = a.h_in[g];
        const double2 W = a.w_in[g];
        double A = 0.0, B = 0.0, Ac = 0.0, Bc = 0.0;
        for (int d = 1; d <= dmax; ++d) {
            const unsigned int x = (unsigned int)((h >> (BP * (d - 1))) & DM);
            A = __builtin_fma(cre[d], ds[x], A);
            B = __builtin_fma(cim[d], ss[x], B);
            Ac = __builtin_fma(dre[d], ds[x], Ac);
            Bc = __builtin_fma(dim[d], ss[x], Bc);
        }
        const int h0 = (int)(h & DM);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double er = 1.0, ei = 0.0, fr = 1.0, fi = 0.0;
            const double dsp = ds[p], ssp = ss[p];
            if (dsp != 0.0) {
                const double e = exp(-dsp * (cre[0] * dsp + A));
                double sn, cs;
                sincos(-dsp * (cim[0] * ssp + B), &sn, &cs);
                er = e * cs;
                ei = e * sn;
                const double f = exp(-dsp * (dre[0] * dsp + Ac));
                double fs, fc;
                sincos(-dsp * (dim[0] * ssp + Bc), &fs, &fc);
                fr = f * fc;
                fi = f * fs;
            }
            const double k4r = k4re[p * P + h0], k4i = k4im[p * P + h0];
            const double br = W.x * k4r - W.y * k4i;
            const double bi = W.x * k4i + W.y * k4r;
            const double wr = br * er - bi * ei;
            const double wi = br * ei + bi * er;
            const double n2 = norm2_nocontract(wr, wi);
            const size_t ci = (size_t)g * P + p;
            if (!((a.theta2 == 0.0) || !(n2 < a.theta2))) {
                acc[2 * P] += sqrt(n2);
                a.cslot[ci] = ~0u;
                continue;
            }
            acc[2 * p] += wr * fr - wi * fi;
            acc[2 * p + 1] += wr * fi + wi * fr;
            acc[2 * P + 1] += 1.0;
            const unsigned long long child = ((h << BP) | (unsigned long long)p) & kmask;
            unsigned long long key = 0;
            for (int k = 0; k < nq; ++k) key = (key << BP) | ((child >> (BP * qpos[k])) & DM);
            unsigned long long slot = mix64(key) & a.tmask;
            bool placed = false;
            for (int probe = 0; probe < kMaxProbe; ++probe) {
                const unsigned long long prev = atomicCAS(a.tkey + slot, kEmptyKey, key);
                if (prev == kEmptyKey || prev == key) {
                    placed = true;
                    break;
                }
                slot = (slot + 1) & a.tmask;
            }
            if (!placed) {
                raise_error(a.error, t, kErrOverflow);
                a.cslot[ci] = ~0u;
                continue;
            }
            const unsigned long long q = (unsigned long long)__double_as_longlong(n2) & a.qmask;
            atomicMax(a.tq + slot, q);
            atomicAdd(&a.tw[slot].x, wr);
            atomicAdd(&a.tw[slot].y, wi);
            a.cslot[ci] = (unsigned int)slot;
            a.cT[ci] = child;   // point j at bits BP*j: as a number it reads from the oldest point
            a.cq[ci] = q;
        }
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

template <int P>
__global__ __launch_bounds__(kSparseThreads) void sparse_resolve(const SparseArgs a) {
    if (error_word(a.error) != 0u) return;
    const unsigned int stored = a.count[(a.t - 1) & 1];
    const unsigned long long n =
        (unsigned long long)(stored < (unsigned long long)a.cap ? stored : (unsigned int)a.cap) * P;
    for (unsigned long long ci = (unsigned long long)blockIdx.x * kSparseThreads + threadIdx.x; ci < n;
         ci += (unsigned long long)gridDim.x * kSparseThreads) {
        const unsigned int slot = a.cslot[ci];
        if (slot == ~0u) continue;
        if (a.cq[ci] == a.tq[slot]) atomicMin(a.tT + slot, a.cT[ci]);
    }
}

__global__ __launch_bounds__(kSparseThreads) void sparse_compact(const SparseArgs a) {
    const bool failed = error_word(a.error) != 0u;
    const unsigned int lane = lane_id();
    unsigned int* const out_count = a.count + (a.t & 1);
    for (unsigned long long s0 = (unsigned long long)blockIdx.x * kSparseThreads;; s0 += (unsigned long long)gridDim.x * kSparseThreads) {
        if (s0 > a.tmask) break;                                   // uniform over the workgroup
        const unsigned long long sl = s0 + threadIdx.x;
        const bool used = sl <= a.tmask && a.tkey[sl] != kEmptyKey;
        // one counter update per wave
        const unsigned long long bal = __ballot(used);
        unsigned int base = 0u;
        if (lane == 0u && bal) base = atomicAdd(out_count, (unsigned int)__popcll(bal));
        base = __shfl(base, 0, 64);
        if (used) {
            const unsigned int idx = base + rank_below(bal);
            if (!failed && (long long)idx < a.cap) {
                a.h_out[idx] = a.tT[sl];                      // the representative's history
                a.w_out[idx] = a.tw[sl];
            } else if (!failed) {
                raise_error(a.error, a.t, kErrOverflow);
            }
            a.tkey[sl] = kEmptyKey;
            a.tq[sl] = 0ull;
            a.tT[sl] = ~0ull;
            a.tw[sl] = make_double2(0.0, 0.0);
        }
    }
}

template <int P>
__global__ __launch_bounds__(kSparseThreads) void sparse_reduce(const SparseArgs a) {
    constexpr int S = partial_stride(P);
    __shared__ double wred[kSpWaves][S];
    const int i = threadIdx.x;
    const int wave = i >> 6;
    const unsigned int lane = lane_id();
    const int t = a.t;
    const unsigned int err = error_word(a.error);
    const bool keep = err == 0u || (int)(err >> 4) > t;
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
        const unsigned int n_in = a.count[(t - 1) & 1];
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
            st.n_children = (unsigned long long)n_in * P;
            st.n_survivors = (unsigned long long)sum[2 * P + 1];
            st.n_stored = a.count[t & 1];
            st.dropped_abs = sum[2 * P];
            st.pad = 0.0;
            a.stats_hist[t] = st;
            // the counter step t+1 writes: it held this step's input count
            a.count[(t + 1) & 1] = 0u;
        }
    }
}

}  // namespace

int launch_sparse_step(const SparseArgs& a, void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int g = a.grid;
    switch (a.P) {
        case 4:
            hipLaunchKernelGGL((sparse_expand<4, 2>), dim3(g), dim3(kSparseThreads), 0, st, a);
            hipLaunchKernelGGL((sparse_resolve<4>), dim3(g), dim3(kSparseThreads), 0, st, a);
            hipLaunchKernelGGL(sparse_compact, dim3(g), dim3(kSparseThreads), 0, st, a);
            hipLaunchKernelGGL((sparse_reduce<4>), dim3(1), dim3(kSparseThreads), 0, st, a);
            break;
        case 9:
            hipLaunchKernelGGL((sparse_expand<9, 4>), dim3(g), dim3(kSparseThreads), 0, st, a);
            hipLaunchKernelGGL((sparse_resolve<9>), dim3(g), dim3(kSparseThreads), 0, st, a);
            hipLaunchKernelGGL(sparse_compact, dim3(g), dim3(kSparseThreads), 0, st, a);
            hipLaunchKernelGGL((sparse_reduce<9>), dim3(1), dim3(kSparseThreads), 0, st, a);
            break;
        default:
            return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace quapi_dev
