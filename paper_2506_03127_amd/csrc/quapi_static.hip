// quapi_run_static: a whole propagation on the direct-mapped store with no
// device allocation, for callers that cannot allocate (code under HIP graph
// capture, serving loops, harnesses that forbid it).
//
// Every buffer of the run -- the two stores, the planner's lists, the
// per-chunk sums, the tables and coefficient sets, the counters -- is carved
// from one file-scope device array, `scratch` (kScratchBytes), whose address
// on each device is taken once with hipGetSymbolAddress.  The caller passes
// the problem and a device buffer for rho(t).  The host tables go to the
// device as kernel arguments (no host buffer outlives the call), and no step
// synchronises.  Calls that overlap on one device share the array and race.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <mutex>

#include "../../include/quapi.h"
#include "quapi_dense.h"
#include "quapi_device.h"
#include "quapi_host.h"

// every buffer of a run; each device holds its own copy until the process ends
static __device__ __align__(256) unsigned char scratch[96ull << 20];

namespace {

using quapi_dev::StepStatsDev;
using quapi_dev::TableLayout;

constexpr size_t kScratchBytes = sizeof(scratch);
constexpr int kStaticMaxK = 40;                 // the coefficient table travels as a kernel argument
constexpr int kStaticMaxL = 10;                 // 4^10 slots: the stores fit the scratch array
constexpr int kMaxDevices = 64;

std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};     // device address of scratch, per device
int g_grid[kMaxDevices] = {};                   // resident step workgroups, per device

// scratch's address and the step grid on the current device (taken once per device)
int device_scratch(unsigned char** ptr, int* grid) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return QUAPI_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return QUAPI_EDEVICE;
        }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return QUAPI_EDEVICE;
        // resident step workgroups with the largest lag-sum tables a run here can need
        const int grid = quapi_dev::dense_step_grid(std::max(ncu, 1), quapi_dev::dense_lds_bytes(kStaticMaxL, kStaticMaxK, false), false);
        if (grid < 1) return QUAPI_EDEVICE;
        g_scratch[dev] = (unsigned char*)p;
        g_grid[dev] = grid;
    }
    *ptr = g_scratch[dev];
    *grid = g_grid[dev];
    return QUAPI_OK;
}

// Host tables of one run, passed by value (under 4 KB).
struct StaticSetup {
    double k4[32];                              // K4[pn][po] re, im
    double ds[4], ss[4];
    double eta[3 * (kStaticMaxK + 1) * 2];      // the three columns, re, im
    double init_w[8];                           // initial groups' amplitudes
    double rho0[8];
    unsigned long long init_slot[4];
    int K, n_init;
    long long n_segs;                           // S/4: occupancy words (four bytes) per buffer
    double* tables;
    double* coef;                               // [(K+1)][4][K+1]
    unsigned int* flag0;                        // occupancy bytes of the two buffers, by segment
    unsigned int* flag1;
    quapi_dev::DenseRec* rec0;
    double2* rho_hist;
    StepStatsDev* stats;
    quapi_dev::DensePlan* plan;                 // [2]
    unsigned long long* agg;                    // [kDenseMaxRegions] planner region counts
    unsigned int* error;
};

// tables, coefficient sets (as quapi_create forms them: interior partners take
// the interior column, the time-0 partner the half-window one; the end-point
// correction swaps the final point's coefficients) and both occupancies cleared
__global__ __launch_bounds__(256) void static_tables(const StaticSetup a) {
    const int K = a.K, n = K + 1;
    const size_t tid = (size_t)blockIdx.x * 256u + threadIdx.x, nth = (size_t)gridDim.x * 256u;
    for (size_t k = tid; k < (size_t)a.n_segs; k += nth) {
        a.flag0[k] = 0u;
        a.flag1[k] = 0u;
    }
    if (blockIdx.x != 0) return;
    const int i = threadIdx.x;
    for (int k = i; k < quapi_dev::kDenseMaxRegions; k += 256) a.agg[k] = 0ull;   // no tag of an earlier call survives
    if (i < 32) a.tables[i] = a.k4[i];
    if (i < 4) {
        a.tables[TableLayout::ds(4) + i] = a.ds[i];
        a.tables[TableLayout::ss(4) + i] = a.ss[i];
    }
    for (int k = i; k < 6 * n; k += 256) a.tables[TableLayout::eta(4) + k] = a.eta[k];
    for (int k = i; k < n * 4 * n; k += 256) {
        const int t = k / (4 * n) + 1, r = (k / n) % 4, d = k % n;
        double v = 0.0;
        if (d <= t) {
            const double in_re = a.eta[2 * d], in_im = a.eta[2 * d + 1];
            const double hf_re = a.eta[2 * (n + d)], hf_im = a.eta[2 * (n + d) + 1];
            const double hh_re = a.eta[2 * (2 * n + d)], hh_im = a.eta[2 * (2 * n + d) + 1];
            if (r == 0) v = d == t ? hf_re : in_re;
            else if (r == 1) v = d == t ? hf_im : in_im;
            else if (d == 0) v = r == 2 ? hf_re - in_re : hf_im - in_im;
            else if (d == t) v = r == 2 ? hh_re - hf_re : hh_im - hf_im;
            else v = r == 2 ? hf_re - in_re : hf_im - in_im;
        }
        a.coef[k] = v;
    }
}

// the initial groups, rho(0), the counters of t = 0, the plans and the error word
__global__ __launch_bounds__(64) void static_initial(const StaticSetup a) {
    const int i = threadIdx.x;
    if (i == 0) {
        for (int k = 0; k < a.n_init; ++k) {
            const unsigned long long s = a.init_slot[k];
            reinterpret_cast<unsigned char*>(a.flag0)[s] = (unsigned char)quapi_dev::dense_tag(0);
            quapi_dev::DenseRec r;
            r.w = make_double2(a.init_w[2 * k], a.init_w[2 * k + 1]);
            r.tail = 0ull;
            r.pad = 0ull;
            a.rec0[s] = r;
        }
        StepStatsDev s0 = {};
        s0.n_stored = (unsigned long long)a.n_init;
        *a.stats = s0;
        quapi_dev::DensePlan z = {};
        a.plan[0] = z;
        a.plan[1] = z;
        *a.error = 0u;
    }
    if (i < 4) a.rho_hist[i] = make_double2(a.rho0[2 * i], a.rho0[2 * i + 1]);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" int quapi_run_static(const quapi_params* p, int n_steps, quapi_c64* rho_out) {
    if (!p || !rho_out || n_steps < 0 || !p->H || !p->q || !p->eta || !p->rho0) return QUAPI_EINVAL;
    const int M = p->M, K = p->dk_max;
    if (M != 2 || p->precision != QUAPI_FP64) return QUAPI_EUNSUPPORTED;
    if (K < 1 || K > kStaticMaxK) return QUAPI_EUNSUPPORTED;
    if (!(p->dt > 0) || !std::isfinite(p->dt) || !(p->theta >= 0) || !std::isfinite(p->theta)) return QUAPI_EINVAL;
    if (p->mode != QUAPI_PRE && p->mode != QUAPI_POST) return QUAPI_EINVAL;
    if (p->merge != QUAPI_MERGE_AUTO && p->merge != QUAPI_MERGE_DIRECT) return QUAPI_EUNSUPPORTED;
    if (!quapi_host::hermitian_ok(M, (const double*)p->H)) return QUAPI_EINVAL;
    for (int k = 0; k < 3 * (K + 1); ++k)
        if (!std::isfinite(p->eta[k].re) || !std::isfinite(p->eta[k].im)) return QUAPI_EINVAL;
    for (int k = 0; k < M * M; ++k)
        if (!std::isfinite(p->rho0[k].re) || !std::isfinite(p->rho0[k].im)) return QUAPI_EINVAL;
    for (int k = 0; k < M; ++k)
        if (!std::isfinite(p->q[k])) return QUAPI_EINVAL;
    // mask: sorted, with 0 and 1, lags < K; merge positions 0..L-1 (the direct-mapped store)
    int mask[kStaticMaxK];
    int nm = 0;
    if (p->mask && p->n_mask > 0) {
        if (p->n_mask > K) return QUAPI_EINVAL;
        for (int k = 0; k < p->n_mask; ++k) mask[nm++] = p->mask[k];
    } else if (p->mask && p->n_mask < 0) {
        return QUAPI_EINVAL;
    } else {
        for (int d = 0; d < K; ++d) mask[nm++] = d;
    }
    if (nm < 2 || mask[0] != 0 || mask[1] != 1) return QUAPI_EINVAL;
    for (int k = 1; k < nm; ++k)
        if (mask[k] <= mask[k - 1] || mask[k] >= K) return QUAPI_EINVAL;
    int L = 0;
    for (int k = (p->mode == QUAPI_PRE ? 1 : 0); k < nm; ++k) {
        const int pos = p->mode == QUAPI_PRE ? mask[k] - 1 : mask[k];
        if (pos != L) return QUAPI_EUNSUPPORTED;          // merge positions not 0..L-1
        ++L;
    }
    if (L < quapi_dev::kDenseMinL || L > kStaticMaxL) return QUAPI_EUNSUPPORTED;

    unsigned char* base = nullptr;
    int grid = 0;
    const int rc = device_scratch(&base, &grid);
    if (rc != QUAPI_OK) return rc;

    // ---- the run's buffers in scratch
    const unsigned long long S = 1ull << (2 * L);
    const size_t ns = (size_t)(S / 4);
    const size_t n_tab = TableLayout::total(4, K), n_coef = (size_t)(K + 1) * 4 * (K + 1);
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_flag0 = take(S), o_flag1 = take(S);
    const size_t o_rec0 = take(S * sizeof(quapi_dev::DenseRec)), o_rec1 = take(S * sizeof(quapi_dev::DenseRec));
    const size_t o_seg = take(S * 4);                    // four lists of S/4 segments
    const size_t o_plan = take(2 * sizeof(quapi_dev::DensePlan));
    const size_t o_agg = take(quapi_dev::kDenseMaxRegions * 8);
    const size_t o_part = take((size_t)grid * quapi_dev::partial_stride(4) * 8);
    const size_t o_tab = take(n_tab * 8), o_coef = take(n_coef * 8);
    const size_t set_d = quapi_dev::dense_tabset_doubles(L, K);
    const size_t o_sets = take((size_t)(K + 1) * set_d * 8);
    const size_t o_stats = take((size_t)(n_steps + 1) * sizeof(StepStatsDev));
    const size_t o_err = take(4);
    if (off > kScratchBytes) return QUAPI_ENOMEM;       // beyond the static scratch array

    // ---- host tables (fixed-size, no heap): K4, ds, ss, eta, initial groups
    StaticSetup su = {};
    double U[8];
    quapi_host::propagator(M, (const double*)p->H, p->dt, U);
    for (int pn = 0; pn < 4; ++pn)
        for (int po = 0; po < 4; ++po) {
            const std::complex<double> u1(U[2 * ((pn / 2) * 2 + po / 2)], U[2 * ((pn / 2) * 2 + po / 2) + 1]);
            const std::complex<double> u2(U[2 * ((pn % 2) * 2 + po % 2)], U[2 * ((pn % 2) * 2 + po % 2) + 1]);
            const std::complex<double> k4 = u1 * std::conj(u2);
            su.k4[2 * (pn * 4 + po)] = k4.real();
            su.k4[2 * (pn * 4 + po) + 1] = k4.imag();
        }
    for (int pp = 0; pp < 4; ++pp) {
        su.ds[pp] = p->q[pp / 2] - p->q[pp % 2];
        su.ss[pp] = p->q[pp / 2] + p->q[pp % 2];
    }
    const int n = K + 1;
    for (int k = 0; k < 3 * n; ++k) {
        su.eta[2 * k] = p->eta[k].re;
        su.eta[2 * k + 1] = p->eta[k].im;
    }
    // phases within the kernels' sine and cosine (as quapi_create checks)
    {
        const double ds_max = std::max(std::fabs(su.ds[1]), std::fabs(su.ds[2]));
        double ss_max = 0.0;
        for (int pp = 0; pp < 4; ++pp) ss_max = std::max(ss_max, std::fabs(su.ss[pp]));
        double worst = 0.0;
        for (int t = 1; t <= n; ++t) {
            double sc = 0.0, sd = 0.0;
            for (int d = 0; d <= K && d <= t; ++d) {
                const double in_im = p->eta[d].im, hf_im = p->eta[n + d].im, hh_im = p->eta[2 * n + d].im;
                sc += std::fabs(d == t ? hf_im : in_im);
                sd += std::fabs(d == 0 ? hf_im - in_im : d == t ? hh_im - hf_im : hf_im - in_im);
            }
            worst = std::max(worst, ds_max * std::max(sc, sd) * ss_max);
        }
        if (!(worst < quapi_dev::kTrigArgMax)) return QUAPI_EUNSUPPORTED;
    }
    const std::complex<double> e0(p->eta[n].re, p->eta[n].im);        // end-point self term
    for (int pp = 0; pp < 4; ++pp) {
        const std::complex<double> r(p->rho0[pp].re, p->rho0[pp].im);
        su.rho0[2 * pp] = r.real();
        su.rho0[2 * pp + 1] = r.imag();
        if (r == std::complex<double>(0, 0)) continue;
        const std::complex<double> w =
            r * std::exp(std::complex<double>(-su.ds[pp] * e0.real() * su.ds[pp], -su.ds[pp] * e0.imag() * su.ss[pp]));
        su.init_slot[su.n_init] = (unsigned long long)pp << (2 * (L - 1));
        su.init_w[2 * su.n_init] = w.real();
        su.init_w[2 * su.n_init + 1] = w.imag();
        ++su.n_init;
    }

    hipStream_t stream = (hipStream_t)p->stream;
    su.K = K;
    su.n_segs = (long long)ns;
    su.tables = (double*)(base + o_tab);
    su.coef = (double*)(base + o_coef);
    su.flag0 = (unsigned int*)(base + o_flag0);
    su.flag1 = (unsigned int*)(base + o_flag1);
    su.rec0 = (quapi_dev::DenseRec*)(base + o_rec0);
    su.rho_hist = (double2*)rho_out;
    su.stats = (StepStatsDev*)(base + o_stats);
    su.plan = (quapi_dev::DensePlan*)(base + o_plan);
    su.agg = (unsigned long long*)(base + o_agg);
    su.error = (unsigned int*)(base + o_err);
    const unsigned int tgrid = (unsigned int)std::min<size_t>(std::max<size_t>((ns + 255) / 256, 1), 1024);
    hipLaunchKernelGGL(static_tables, dim3(tgrid), dim3(256), 0, stream, su);
    double* sets = (double*)(base + o_sets);
    if (quapi_dev::launch_dense_tables(su.coef, su.tables, L, K, K + 1, sets, stream) != (int)hipSuccess)
        return QUAPI_EDEVICE;
    hipLaunchKernelGGL(static_initial, dim3(1), dim3(64), 0, stream, su);
    if (hipGetLastError() != hipSuccess) return QUAPI_EDEVICE;

    // ---- t = 0 planned, then each step: the step kernel and the next planner
    unsigned char* flag[2] = {(unsigned char*)su.flag0, (unsigned char*)su.flag1};
    quapi_dev::DenseRec* rec[2] = {su.rec0, (quapi_dev::DenseRec*)(base + o_rec1)};
    const int lds = quapi_dev::dense_lds_bytes(L, K, false);
    quapi_dev::DensePlanArgs pa;
    pa.seg = (unsigned int*)(base + o_seg);
    pa.n_segs = (long long)ns;
    pa.partials = (double*)(base + o_part);
    pa.n_parts = grid;
    pa.rho_hist = su.rho_hist;
    pa.stats_hist = su.stats;
    pa.error = su.error;
    pa.agg = su.agg;
    quapi_dev::DenseArgs sa;
    sa.seg = pa.seg;
    sa.partials = (double*)(base + o_part);
    sa.n_segs = (long long)ns;
    sa.tables = su.tables;
    sa.L = L;
    sa.K = K;
    sa.theta2 = p->theta * p->theta;
    const int qbits = p->qbits < 0 ? 32 : std::min(p->qbits, 63);
    sa.qmask = qbits >= 64 ? 0ull : ~((1ull << qbits) - 1ull);
    sa.error = su.error;
    sa.f32 = 0;
    sa.rec32_in = nullptr;
    sa.rec32_out = nullptr;
    int cur = 0;
    for (int t = 0; t <= n_steps; ++t) {
        if (t > 0) {
            sa.rec_in = rec[cur];
            sa.rec_out = rec[1 - cur];
            sa.flag_out = flag[1 - cur];
            sa.plan = su.plan + (t & 1);
            sa.t = t;
            sa.coef = su.coef + (size_t)(std::min(t, K + 1) - 1) * 4 * n;
            sa.tabset = sets + (size_t)(std::min(t, K + 1) - 1) * set_d;
            if (quapi_dev::launch_dense_step(sa, grid, lds, stream) != (int)hipSuccess) return QUAPI_EDEVICE;
            cur = 1 - cur;
        }
        // plan step t+1 from the groups after step t (and reduce step t)
        pa.flags = reinterpret_cast<const unsigned int*>(flag[cur]);
        pa.flags_spent = reinterpret_cast<unsigned int*>(flag[1 - cur]);
        pa.plan = su.plan + ((t + 1) & 1);
        pa.plan_prev = su.plan + (t & 1);
        pa.reduce_t = t;
        pa.clear_spent = quapi_dev::dense_clear_due(t);
        pa.epoch = (unsigned int)(t % 4095) + 1u;   // 1..4095: differs from the launch before
        if (quapi_dev::launch_dense_plan(pa, stream) != (int)hipSuccess) return QUAPI_EDEVICE;
    }
    return QUAPI_OK;
}
