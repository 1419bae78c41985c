// C ABI of the path-propagation library: context, host tables, device
// buffers and the step loop.  See include/quapi.h for the contract.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/quapi.h"
#include "quapi_dense.h"
#include "quapi_device.h"
#include "quapi_host.h"
#include "quapi_sparse.h"

using quapi_dev::GroupBuf;
using quapi_dev::StepArgs;
using quapi_dev::StepStatsDev;
using quapi_dev::TableLayout;

struct quapi_ctx {
    int M = 0, P = 0, K = 0, L = 0, bits = 0, mode = 0, qbits = 32;
    int D = 0;                   // bucket key length in points
    int n_super = 0;             // P^(D-1)
    long long n_buckets = 0;     // P^D
    double dt = 0, theta = 0;
    long long cap = 0;           // groups per bucket
    std::vector<double> tables;  // host copy of the device tables
    std::vector<double> coef;    // per-step coefficient sets, t = 1..K+1 (t > K uses set K+1)
    std::vector<double> rho0;    // 2*P
    std::vector<unsigned long long> init_key;
    std::vector<double2> init_w;           // [n_inst][initial groups]
    std::vector<long long> init_bucket;    // bucket inside an instance
    std::vector<int> init_pair;

    // sparse-mask path (merge positions not 0..L-1): hash-table merge
    bool sparse = false;
    std::vector<int> qpos;       // merge positions, most significant first
    std::vector<int> npos;       // the other positions, oldest first
    bool sp_packed = false;      // representative word holds the other positions
    int sp_hw = 1;               // 64-bit words per stored history
    bool f32 = false;            // FP32 precision form: amplitudes as FP32 (ln|w|, arg w)
    float2* sp_wf[2] = {nullptr, nullptr};
    long long sp_cap = 0;        // group capacity
    unsigned long long sp_seg_cap = 0;           // groups per segment (kSegs segments)
    uint64_t* sp_h[2] = {nullptr, nullptr};
    double2* sp_w[2] = {nullptr, nullptr};
    unsigned int* sp_count = nullptr;            // [seg_counter(2, 0)] per segment, by step parity
    quapi_dev::SpSlot* sp_slot = nullptr;        // [sp_tsize] hash table
    unsigned long long sp_tsize = 0;
    bool sp_part = false;                         // partition merge in place of the table
    unsigned int sp_n_part = 0;                   // partitions allocated
    unsigned int* sp_pcount = nullptr;            // [sp_n_part]
    quapi_dev::PartRec* sp_prec = nullptr;        // [sp_n_part * kPartCap] entries
    unsigned long long* sp_pother = nullptr;      // (unpacked form whose entry does not fit 128 bits)
    bool sp_pfit = false;
    unsigned long long* sp_tN = nullptr;         // unpacked form only
    unsigned int* sp_cslot = nullptr;
    unsigned long long* sp_cN = nullptr;
    unsigned long long* sp_cq = nullptr;
    double* sp_partials = nullptr;
    int sp_grid = 0;
    int sp_grid_merge = 0;                       // partition merge

    // direct-mapped store (two-level systems, merge positions 0..L-1, short keys)
    bool dense = false;
    unsigned char* dn_flag[2] = {nullptr, nullptr};        // [S] occupancy bytes by buffer
    quapi_dev::DenseRec* dn_rec[2] = {nullptr, nullptr};   // [S] records by buffer (FP64 form)
    quapi_dev::DenseRec32* dn_rec32[2] = {nullptr, nullptr}; // [S] records by buffer (FP32 form)
    double* dn_tabs = nullptr;                             // [K+1] lag-sum table sets
    unsigned long long dn_slots = 0;                       // S = P^L
    unsigned int* dn_seg = nullptr;                        // [4][S/4] the planner's segment lists
    quapi_dev::DensePlan* dn_plan = nullptr;               // [2] by step parity
    double* dn_partials = nullptr;                         // [partial_stride(4)][dn_grid]
    int dn_grid = 0;
    int dn_lds = 0;                                        // the step kernel's table bytes
    unsigned long long* dn_agg = nullptr;                  // [kDenseMaxRegions] planner region counts
    unsigned int dn_epoch = 0;                             // tag of the last planner launch

    // batched form: n_inst instances (bath parameter points) in one store
    int n_inst = 1;
    bool batch = false;
    long long inst_buckets = 0;              // P^D, buckets of one instance
    unsigned long long* d_totals = nullptr;  // [n_inst]
    unsigned int* d_inst = nullptr;          // [2][n_inst][2] first chunk and groups, by step parity
    int chunk_run = 1;                       // consecutive chunks a step-kernel workgroup takes in turn

    hipStream_t stream = nullptr;
    bool own_stream = false;                 // the device's shared library stream, released at destroy
    int stream_dev = 0;
    int dev = 0;                             // device the context was created on
    GroupBuf buf[2] = {};
    unsigned int* counts[2] = {nullptr, nullptr};
    double* d_tables = nullptr;
    double* d_coef = nullptr;
    std::vector<double> k4_batch;            // batched form with one H_S per instance: [n_inst][P*P] complex
    double* d_k4_batch = nullptr;
    double* d_inst_tabs = nullptr;           // batched form: each instance's subset tables of the current set
    double* d_partials = nullptr;
    unsigned int* d_nz_bucket = nullptr;     // [n_buckets] nonempty buckets of the stored groups
    unsigned int* d_nz_prefix = nullptr;     // [n_buckets] their first global group index
    unsigned int* d_desc = nullptr;          // [max_chunks] bucket rank of each chunk's first group
    quapi_dev::Plan* d_plan = nullptr;       // [2], by step parity
    unsigned long long* d_chain = nullptr;   // [P * max_chunks] look-back words
    int max_chunks = 0;
    int grid = 0;
    double2* d_rho = nullptr;
    StepStatsDev* d_stats = nullptr;
    unsigned int* d_error = nullptr;
    int hist_cap = 0;            // rho/stats history holds steps 0..hist_cap
    int t = 0;                   // steps enqueued
    int cur = 0;                 // buffer holding the state at time t
    unsigned int epoch = 0;
    int err = QUAPI_OK;          // sticky error of a failed step
    size_t device_bytes = 0;
    std::vector<void*> allocations;
    // quapi_step_graph: the last recorded run of steps, replayed while it starts
    // at the context's step and parity with the buffers it recorded
    hipGraphExec_t graph = nullptr;
    int graph_t0 = -1, graph_n = 0, graph_cur0 = 0, graph_run = 0;
    double2* graph_rho = nullptr;
    StepStatsDev* graph_stats = nullptr;
    unsigned int graph_epoch_end = 0;
    bool capturing = false;
    // launch timing: three events per recorded step
    bool prof_on = false;
    int prof_cap = 0, prof_n = 0;
    std::vector<hipEvent_t> prof_ev;
};

namespace {

constexpr int kMaxInstances = 1024;   // instances of one batched context

int hip_to_code(hipError_t e) {
    if (e == hipSuccess) return QUAPI_OK;
    if (e == hipErrorOutOfMemory) return QUAPI_ENOMEM;
    return QUAPI_EDEVICE;
}

template <class T>
int dev_alloc(quapi_ctx* c, T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    void* q = nullptr;
    const hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return hip_to_code(e);
    }
    c->allocations.push_back(q);
    c->device_bytes += bytes;
    *p = (T*)q;
    return QUAPI_OK;
}

void dev_free(quapi_ctx* c, void* p, size_t bytes) {
    if (!p) return;
    auto it = std::find(c->allocations.begin(), c->allocations.end(), p);
    if (it != c->allocations.end()) c->allocations.erase(it);
    c->device_bytes -= bytes;
    (void)hipFree(p);
}

int launch_planner(quapi_ctx* c, int t);

int upload_initial_sparse(quapi_ctx* c) {
    const size_t n0 = c->init_pair.size();
    const size_t hw = (size_t)c->sp_hw;
    std::vector<uint64_t> h(n0 * hw, 0ull);
    for (size_t k = 0; k < n0; ++k) h[k * hw] = (uint64_t)c->init_pair[k];
    // the initial groups fill segments 0, 1, ... in turn
    std::vector<unsigned int> cnt((size_t)quapi_dev::seg_counter(2, 0), 0u);
    for (int s = 0; s < quapi_dev::kSegs; ++s) {
        const unsigned long long lo = (unsigned long long)s * c->sp_seg_cap;
        if (lo < n0) cnt[quapi_dev::seg_counter(0, s)] = (unsigned int)std::min<unsigned long long>(n0 - lo, c->sp_seg_cap);
    }
    const size_t ts = (size_t)c->sp_tsize;
    hipError_t e = hipSuccess;
    // the FP32 precision form stores (ln|w|, arg w)
    std::vector<float2> wl(c->f32 ? n0 : 0);
    for (size_t k = 0; k < wl.size(); ++k) {
        const double re = c->init_w[k].x, im = c->init_w[k].y;
        wl[k] = make_float2((float)(0.5 * std::log(re * re + im * im)), (float)std::atan2(im, re));
    }
    if (n0) {
        e = hipMemcpyAsync(c->sp_h[0], h.data(), h.size() * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && c->f32)
            e = hipMemcpyAsync(c->sp_wf[0], wl.data(), n0 * sizeof(float2), hipMemcpyHostToDevice, c->stream);
        else if (e == hipSuccess)
            e = hipMemcpyAsync(c->sp_w[0], c->init_w.data(), n0 * sizeof(double2), hipMemcpyHostToDevice, c->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->sp_count, cnt.data(), cnt.size() * sizeof(unsigned int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && c->sp_slot) e = hipMemsetAsync(c->sp_slot, 0, ts * sizeof(quapi_dev::SpSlot), c->stream);
    if (e == hipSuccess && c->sp_tN)
        e = hipMemsetAsync(c->sp_tN, 0xff, ts * sizeof(unsigned long long), c->stream);
    if (e == hipSuccess && c->sp_pcount)
        e = hipMemsetAsync(c->sp_pcount, 0, (size_t)c->sp_n_part * sizeof(unsigned int), c->stream);
    // the copies read host vectors of this frame: complete them before returning
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_to_code(e);
}

// Plan step t+1 on the direct-mapped store from the groups stored after step t
// (and reduce step t's sums when t >= 1); clears the bitmap step t+1 writes.
int launch_dense_planner(quapi_ctx* c, int t) {
    quapi_dev::DensePlanArgs pa;
    pa.flags = reinterpret_cast<const unsigned int*>(c->dn_flag[c->cur]);
    pa.flags_spent = reinterpret_cast<unsigned int*>(c->dn_flag[1 - c->cur]);
    pa.seg = c->dn_seg;
    pa.n_segs = (long long)(c->dn_slots / 4);
    pa.plan = c->dn_plan + ((t + 1) & 1);
    pa.plan_prev = c->dn_plan + (t & 1);
    pa.reduce_t = t;
    pa.clear_spent = quapi_dev::dense_clear_due(t);
    pa.partials = c->dn_partials;
    pa.n_parts = c->dn_grid;
    pa.rho_hist = c->d_rho;
    pa.stats_hist = c->d_stats;
    pa.error = c->d_error;
    pa.agg = c->dn_agg;
    c->dn_epoch = c->dn_epoch % 4095u + 1u;               // 1..4095; 0 is the cleared buffer's tag
    pa.epoch = c->dn_epoch;
    return quapi_dev::launch_dense_plan(pa, c->stream) == (int)hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

// t = 0 on the direct-mapped store: the initial groups at their slots, the
// occupancy of the first buffer holding exactly them and that of the second none
int upload_initial_dense(quapi_ctx* c) {
    const size_t S = (size_t)c->dn_slots;
    const size_t n0 = c->init_key.size();
    std::vector<quapi_dev::DenseRec> rec(n0 ? n0 : 1);
    std::vector<quapi_dev::DenseRec32> rec32(n0 ? n0 : 1);
    const unsigned char one = (unsigned char)quapi_dev::dense_tag(0);
    hipError_t e = hipMemsetAsync(c->dn_flag[0], 0, S, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->dn_flag[1], 0, S, c->stream);
    for (size_t k = 0; k < n0 && e == hipSuccess; ++k) {
        const unsigned long long sl = c->init_key[k];
        const double2 w = c->init_w[k];
        if (c->f32) {
            rec32[k].lw = (float)(0.5 * std::log(w.x * w.x + w.y * w.y));
            rec32[k].aw = (float)std::atan2(w.y, w.x);
            rec32[k].tail = 0ull;
            e = hipMemcpyAsync(c->dn_rec32[0] + sl, &rec32[k], sizeof(quapi_dev::DenseRec32), hipMemcpyHostToDevice,
                               c->stream);
        } else {
            rec[k].w = w;
            rec[k].tail = 0ull;
            rec[k].pad = 0ull;
            e = hipMemcpyAsync(c->dn_rec[0] + sl, &rec[k], sizeof(quapi_dev::DenseRec), hipMemcpyHostToDevice,
                               c->stream);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(c->dn_flag[0] + sl, &one, 1, hipMemcpyHostToDevice, c->stream);
    }
    // the copies read host values of this frame: complete them before returning
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_to_code(e);
}

int upload_initial(quapi_ctx* c) {
    hipError_t e = hipSuccess;
    if (c->sparse) {
        if (upload_initial_sparse(c) != QUAPI_OK) e = hipErrorLaunchFailure;
    } else if (c->dense) {
        if (upload_initial_dense(c) != QUAPI_OK) e = hipErrorLaunchFailure;
    } else {
        e = hipMemsetAsync(c->counts[0], 0, (size_t)c->n_buckets * sizeof(unsigned int), c->stream);
    }
    const size_t n0 = c->init_key.size();
    for (size_t j = 0; !c->sparse && !c->dense && j < (size_t)c->n_inst && e == hipSuccess; ++j)
        for (size_t k = 0; k < n0 && e == hipSuccess; ++k) {
            const long long b = (long long)j * c->inst_buckets + c->init_bucket[k];
            const size_t o = (size_t)b * (size_t)c->cap;
            const unsigned long long zero = 0;
            const unsigned int one = 1;
            e = hipMemcpyAsync(c->buf[0].key + o, &c->init_key[k], 8, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(c->buf[0].tail + o, &zero, 8, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(c->buf[0].w + o, &c->init_w[j * n0 + k], 16, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) e = hipMemcpyAsync(c->counts[0] + b, &one, 4, hipMemcpyHostToDevice, c->stream);
            // the copies read host stack values: complete them before the next iteration reuses them
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        }
    if (e == hipSuccess) e = hipMemsetAsync(c->d_error, 0, sizeof(unsigned int), c->stream);
    // t = 0 of every instance
    std::vector<double2> r0((size_t)c->n_inst * c->P);
    for (size_t j = 0; j < (size_t)c->n_inst; ++j)
        for (int p = 0; p < c->P; ++p) r0[j * c->P + p] = make_double2(c->rho0[2 * p], c->rho0[2 * p + 1]);
    std::vector<StepStatsDev> s0((size_t)c->n_inst);
    for (auto& x : s0) {
        x = StepStatsDev{};
        x.n_stored = n0;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_rho, r0.data(), r0.size() * sizeof(double2), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_stats, s0.data(), s0.size() * sizeof(StepStatsDev), hipMemcpyHostToDevice, c->stream);
    c->t = 0;
    c->cur = 0;
    c->err = QUAPI_OK;
    if (e == hipSuccess && !c->sparse && !c->dense && launch_planner(c, 0) != QUAPI_OK) e = hipErrorLaunchFailure;
    if (e == hipSuccess && c->dense && launch_dense_planner(c, 0) != QUAPI_OK) e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_to_code(e);
}

// Plan step t+1 from the groups stored after step t (and reduce step t's sums when t >= 1).
int launch_planner(quapi_ctx* c, int t) {
    quapi_dev::PlanArgs pa;
    pa.counts = c->counts[c->cur];
    pa.counts_next = c->counts[1 - c->cur];
    pa.nz_bucket = c->d_nz_bucket;
    pa.nz_prefix = c->d_nz_prefix;
    pa.desc = c->d_desc;
    pa.plan = c->d_plan + ((t + 1) & 1);
    pa.plan_prev = c->d_plan + (t & 1);
    pa.n_buckets = c->n_buckets;
    pa.max_chunks = c->max_chunks;
    pa.P = c->P;
    pa.reduce_t = t;
    pa.partials = c->d_partials;
    pa.rho_hist = c->d_rho;
    pa.stats_hist = c->d_stats;
    pa.error = c->d_error;
    pa.n_inst = c->n_inst;
    pa.inst_buckets = (int)c->inst_buckets;
    pa.totals = c->d_totals;
    pa.inst_next = c->d_inst ? c->d_inst + (size_t)((t + 1) & 1) * 2 * c->n_inst : nullptr;
    pa.inst_prev = c->d_inst ? c->d_inst + (size_t)(t & 1) * 2 * c->n_inst : nullptr;
    const int e = c->batch ? quapi_dev::launch_plan_batch(pa, c->stream) : quapi_dev::launch_plan(pa, c->stream);
    return e == (int)hipSuccess ? QUAPI_OK : QUAPI_EDEVICE;
}

int grow_history(quapi_ctx* c, int need) {
    if (need <= c->hist_cap) return QUAPI_OK;
    const int ncap = std::max(need, 2 * c->hist_cap);
    const size_t B = (size_t)c->n_inst;             // history rows hold every instance
    double2* nr = nullptr;
    StepStatsDev* ns = nullptr;
    int rc = dev_alloc(c, &nr, (size_t)(ncap + 1) * B * c->P);
    if (rc) return rc;
    rc = dev_alloc(c, &ns, (size_t)(ncap + 1) * B);
    if (rc) { dev_free(c, nr, (size_t)(ncap + 1) * B * c->P * sizeof(double2)); return rc; }
    hipError_t e = hipMemcpyAsync(nr, c->d_rho, (size_t)(c->hist_cap + 1) * B * c->P * sizeof(double2),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ns, c->d_stats, (size_t)(c->hist_cap + 1) * B * sizeof(StepStatsDev),
                           hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        dev_free(c, nr, (size_t)(ncap + 1) * B * c->P * sizeof(double2));
        dev_free(c, ns, (size_t)(ncap + 1) * B * sizeof(StepStatsDev));
        return hip_to_code(e);
    }
    dev_free(c, c->d_rho, (size_t)(c->hist_cap + 1) * B * c->P * sizeof(double2));
    dev_free(c, c->d_stats, (size_t)(c->hist_cap + 1) * B * sizeof(StepStatsDev));
    c->d_rho = nr;
    c->d_stats = ns;
    c->hist_cap = ncap;
    return QUAPI_OK;
}

// Reads the kernel-reported error after a synchronisation and rolls the
// context back to the last complete step.
int check_device_error(quapi_ctx* c) {
    if (c->err) return c->err;
    unsigned int h = 0;
    hipError_t e = hipMemcpy(&h, c->d_error, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) { c->err = hip_to_code(e); return c->err; }
    if (h == 0u) return QUAPI_OK;
    c->err = ((h & 15u) == quapi_dev::kErrOverflow) ? QUAPI_ENOMEM : QUAPI_EDEVICE;
    const int failed = (int)(h >> 4);
    if (failed >= 1 && failed <= c->t) {
        c->t = failed - 1;
        c->cur = c->t & 1;
    }
    return c->err;
}

int sync_ctx(quapi_ctx* c) {
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { c->err = hip_to_code(e); return c->err; }
    return check_device_error(c);
}

bool is_finite_d(double x) { return std::isfinite(x); }

// n time steps on the hash-table path (merge positions other than 0..L-1)
int step_sparse(quapi_ctx* c, int n_steps) {
    quapi_dev::SparseArgs a;
    a.count = c->sp_count;
    a.slot = c->sp_slot;
    a.tsize = c->sp_tsize;
    a.tN = c->sp_tN;
    a.hw = c->sp_hw;
    a.cslot = c->sp_cslot;
    a.cN = c->sp_cN;
    a.cq = c->sp_cq;
    a.part = c->sp_part ? 1 : 0;
    a.grid_merge = c->sp_grid_merge;
    a.n_part_max = c->sp_n_part;
    a.pcount = c->sp_pcount;
    a.prec = c->sp_prec;
    a.pother = c->sp_pother;
    a.pfit = c->sp_pfit ? 1 : 0;
    a.cap = c->sp_cap;
    a.seg_cap = c->sp_seg_cap;
    a.P = c->P;
    a.K = c->K;
    a.theta2 = c->theta * c->theta;
    a.qbits = c->qbits;
    a.packed = c->sp_packed ? 1 : 0;
    a.tables = c->d_tables;
    a.nq = (int)c->qpos.size();
    a.nn = (int)c->npos.size();
    for (int k = 0; k < quapi_dev::kMaxK; ++k) {
        a.qpos[k] = k < a.nq ? c->qpos[k] : 0;
        a.npos[k] = k < a.nn ? c->npos[k] : 0;
    }
    // the clustered positions: merge positions q with q+1 also a merge position
    a.cmask = 0ull;
    for (int k = 0; k < a.nq; ++k)
        if (std::find(c->qpos.begin(), c->qpos.end(), c->qpos[k] + 1) != c->qpos.end())
            a.cmask |= ((1ull << c->bits) - 1ull) << (c->bits * (a.nq - 1 - k));
    a.partials = c->sp_partials;
    a.grid = c->sp_grid;
    a.rho_hist = c->d_rho;
    a.stats_hist = c->d_stats;
    a.error = c->d_error;
    const int n = c->K + 1;
    for (int k = 0; k < n_steps; ++k) {
        const int t = c->t + 1;
        a.h_in = c->sp_h[c->cur];
        a.w_in = c->sp_w[c->cur];
        a.wf_in = c->sp_wf[c->cur];
        a.h_out = c->sp_h[1 - c->cur];
        a.w_out = c->sp_w[1 - c->cur];
        a.wf_out = c->sp_wf[1 - c->cur];
        a.t = t;
        a.coef = c->d_coef + (size_t)(std::min(t, c->K + 1) - 1) * 4 * n;
        hipEvent_t* ev = (c->prof_on && !c->capturing && c->prof_n < c->prof_cap)
                             ? &c->prof_ev[3 * (size_t)c->prof_n++] : nullptr;
        if (ev && hipEventRecord(ev[0], c->stream) != hipSuccess) ev = nullptr;
        // profiled: ev[0]..ev[1] brackets expand, ev[1]..ev[2] the rest of the step
        if (quapi_dev::launch_sparse_step(a, c->stream, ev ? (void*)ev[1] : nullptr) != (int)hipSuccess) {
            c->err = QUAPI_EDEVICE;
            return c->err;
        }
        if (ev) (void)hipEventRecord(ev[2], c->stream);
        c->t = t;
        c->cur = 1 - c->cur;
    }
    return QUAPI_OK;
}

// n time steps on the direct-mapped store: the step kernel, then the planner
// of the next step (which reduces this one's sums)
int step_dense(quapi_ctx* c, int n_steps) {
    quapi_dev::DenseArgs a;
    a.seg = c->dn_seg;
    a.partials = c->dn_partials;
    a.n_segs = (long long)(c->dn_slots / 4);
    a.tables = c->d_tables;
    a.L = c->L;
    a.K = c->K;
    a.theta2 = c->theta * c->theta;
    a.qmask = c->qbits >= 64 ? 0ull : ~((1ull << c->qbits) - 1ull);
    a.error = c->d_error;
    a.f32 = c->f32 ? 1 : 0;
    const int n = c->K + 1;
    for (int k = 0; k < n_steps; ++k) {
        const int t = c->t + 1;
        a.rec_in = c->dn_rec[c->cur];
        a.rec_out = c->dn_rec[1 - c->cur];
        a.rec32_in = c->dn_rec32[c->cur];
        a.rec32_out = c->dn_rec32[1 - c->cur];
        a.flag_out = c->dn_flag[1 - c->cur];
        a.plan = c->dn_plan + (t & 1);
        a.t = t;
        a.coef = c->d_coef + (size_t)(std::min(t, c->K + 1) - 1) * 4 * n;
        a.tabset = c->dn_tabs + (size_t)(std::min(t, c->K + 1) - 1) * quapi_dev::dense_tabset_doubles(c->L, c->K);
        hipEvent_t* ev = (c->prof_on && !c->capturing && c->prof_n < c->prof_cap)
                             ? &c->prof_ev[3 * (size_t)c->prof_n++] : nullptr;
        if (ev && hipEventRecord(ev[0], c->stream) != hipSuccess) ev = nullptr;
        if (quapi_dev::launch_dense_step(a, c->dn_grid, c->dn_lds, c->stream) != (int)hipSuccess) {
            c->err = QUAPI_EDEVICE;
            return c->err;
        }
        if (ev) (void)hipEventRecord(ev[1], c->stream);
        c->t = t;
        c->cur = 1 - c->cur;
        if (launch_dense_planner(c, t) != QUAPI_OK) {
            c->err = QUAPI_EDEVICE;
            return c->err;
        }
        if (ev) (void)hipEventRecord(ev[2], c->stream);
    }
    return QUAPI_OK;
}

long long ipow(long long b, int e) {
    long long r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

}  // namespace

namespace {

// Contexts that pass no stream share one per device.  The step kernel's grid is
// co-resident: its chunks wait on earlier chunks of the same launch, so two step
// kernels side by side, neither with the whole GPU, can wait on each other until
// the look-back's spin limit reports a fault.  One stream orders them.
std::mutex g_stream_mu;
struct SharedStream {
    hipStream_t s = nullptr;
    int refs = 0;
};
std::map<int, SharedStream> g_streams;

hipError_t acquire_shared_stream(int dev, hipStream_t* out) {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    SharedStream& e = g_streams[dev];
    if (!e.s) {
        const hipError_t r = hipStreamCreateWithFlags(&e.s, hipStreamNonBlocking);
        if (r != hipSuccess) {
            e.s = nullptr;
            return r;
        }
    }
    ++e.refs;
    *out = e.s;
    return hipSuccess;
}

void release_shared_stream(int dev) {
    std::lock_guard<std::mutex> lk(g_stream_mu);
    auto it = g_streams.find(dev);
    if (it == g_streams.end()) return;
    if (--it->second.refs == 0) {
        (void)hipStreamDestroy(it->second.s);
        g_streams.erase(it);
    }
}

// Step kernels of one device run one after another, whatever stream they are
// on.  The device remembers the stream of the last step kernel enqueued; a
// launch from another stream first waits for an event recorded on that stream
// (after everything enqueued there so far, the step kernel included).  Launches
// that stay on one stream add nothing to it: stream order already holds.
struct StepOrder {
    std::mutex mu;
    hipEvent_t ev = nullptr;
    hipStream_t last = nullptr;   // stream of the last step kernel enqueued, or none
    bool ev_valid = false;        // ev was recorded on `last` after that kernel
};
std::mutex g_order_mu;
std::map<int, StepOrder*> g_order;   // never freed: lives until the process ends

StepOrder* step_order(int dev) {
    std::lock_guard<std::mutex> lk(g_order_mu);
    StepOrder*& o = g_order[dev];
    if (!o) o = new (std::nothrow) StepOrder();
    return o;
}

// Enqueue `launch` on `stream` after every step kernel enqueued before it on
// the device.
template <class F>
hipError_t ordered_launch(int dev, hipStream_t stream, F&& launch) {
    StepOrder* o = step_order(dev);
    if (!o) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(o->mu);
    if (o->last && o->last != stream) {
        if (!o->ev) {
            const hipError_t e = hipEventCreateWithFlags(&o->ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                o->ev = nullptr;
                return e;
            }
        }
        if (!o->ev_valid) {
            const hipError_t e = hipEventRecord(o->ev, o->last);
            if (e != hipSuccess) return e;
            o->ev_valid = true;
        }
        const hipError_t e = hipStreamWaitEvent(stream, o->ev, 0);
        if (e != hipSuccess) return e;
    }
    const hipError_t e = launch();
    if (e != hipSuccess) return e;
    o->last = stream;
    o->ev_valid = false;
    return hipSuccess;
}

// Record the device's event on `stream` now when the last step kernel is
// there and no event follows it yet, so that later launches from other streams
// wait on that event and never record on `stream` itself: before the stream is
// captured into a graph (nothing may be recorded on it from outside the
// capture) and when a context on it is destroyed (the stream may go away).
hipError_t order_release(int dev, hipStream_t stream) {
    StepOrder* o = step_order(dev);
    if (!o) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(o->mu);
    if (o->last != stream || o->ev_valid) return hipSuccess;
    if (!o->ev) {
        const hipError_t e = hipEventCreateWithFlags(&o->ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            o->ev = nullptr;
            return e;
        }
    }
    const hipError_t e = hipEventRecord(o->ev, stream);
    if (e == hipSuccess) o->ev_valid = true;
    return e;
}

// zero n 64-bit words: a kernel, so that a HIP graph records it as a kernel node
__global__ __launch_bounds__(256) void clear_words(unsigned long long* p, size_t n) {
    for (size_t k = (size_t)blockIdx.x * 256u + threadIdx.x; k < n; k += (size_t)gridDim.x * 256u) p[k] = 0ull;
}

hipError_t launch_clear_words(unsigned long long* p, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const size_t blocks = (n + 255u) / 256u;
    const unsigned int g = (unsigned int)(blocks < 1024u ? blocks : 1024u);
    hipLaunchKernelGGL(clear_words, dim3(g), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace

extern "C" {

const char* quapi_strerror(int code) {
    switch (code) {
        case QUAPI_OK: return "ok";
        case QUAPI_EINVAL: return "invalid argument";
        case QUAPI_ENOMEM: return "out of device memory or group capacity exceeded";
        case QUAPI_EDEVICE: return "HIP runtime error or kernel-reported fault";
        case QUAPI_ESTATE: return "call not valid in the current state";
        case QUAPI_EUNSUPPORTED: return "input not supported by this build";
        default: return "unknown error";
    }
}

int quapi_propagator(int M, const quapi_c64* H, double dt, quapi_c64* U_out) {
    if (M < 1 || M > 8 || !H || !U_out || !is_finite_d(dt)) return QUAPI_EINVAL;
    if (!quapi_host::hermitian_ok(M, (const double*)H)) return QUAPI_EINVAL;
    quapi_host::propagator(M, (const double*)H, dt, (double*)U_out);
    return QUAPI_OK;
}

int quapi_eta(const quapi_bath* bath, double beta, double dt, int dk_max, quapi_c64* eta_out) {
    if (!bath || !eta_out || !(beta > 0) || !(dt > 0) || dk_max < 1 || dk_max > quapi_dev::kMaxK)
        return QUAPI_EINVAL;
    if (bath->ohmic_alpha < 0 || (bath->ohmic_alpha > 0 && !(bath->ohmic_wc > 0))) return QUAPI_EINVAL;
    if (bath->n_peaks < 0 || (bath->n_peaks > 0 && !bath->peaks)) return QUAPI_EINVAL;
    for (int k = 0; k < bath->n_peaks; ++k)
        if (!(bath->peaks[3 * k] > 0) || !(bath->peaks[3 * k + 1] > 0) || bath->peaks[3 * k + 2] < 0)
            return QUAPI_EINVAL;
    return quapi_host::eta_columns(bath->ohmic_alpha, bath->ohmic_wc, bath->n_peaks, bath->peaks, beta,
                                   dt, dk_max, (double*)eta_out) == 0 ? QUAPI_OK : QUAPI_EINVAL;
}

// A context of n_inst instances that share p but for the eta tables (instance
// j's at eta_all + 3*(K+1)*j) and, when H_all is given, the Hamiltonians (j's at
// H_all + M*M*j); batch: the batched form (its planner and layout).
static int create_ctx(const quapi_params* p, int n_inst, const quapi_c64* eta_all, const quapi_c64* H_all,
                      bool batch, quapi_ctx** out) {
    if (!out) return QUAPI_EINVAL;
    *out = nullptr;
    if (!p || !p->H || !p->q || !eta_all || !p->rho0 || n_inst < 1 || n_inst > kMaxInstances) return QUAPI_EINVAL;
    const int M = p->M, K = p->dk_max;
    if (M < 2 || K < 1 || K > quapi_dev::kMaxK || !(p->dt > 0) || !is_finite_d(p->dt)) return QUAPI_EINVAL;
    if (!(p->theta >= 0) || !is_finite_d(p->theta)) return QUAPI_EINVAL;
    if (p->mode != QUAPI_PRE && p->mode != QUAPI_POST) return QUAPI_EINVAL;
    if (p->precision != QUAPI_FP64 && p->precision != QUAPI_FP32_LOG) return QUAPI_EINVAL;
    if (M > 4) return QUAPI_EUNSUPPORTED;
    if (!quapi_host::hermitian_ok(M, (const double*)p->H)) return QUAPI_EINVAL;
    for (int j = 0; H_all && j < n_inst; ++j)
        if (!quapi_host::hermitian_ok(M, (const double*)(H_all + (size_t)M * M * j))) return QUAPI_EINVAL;
    for (int i = 0; i < M; ++i)
        if (!is_finite_d(p->q[i])) return QUAPI_EINVAL;
    for (long long i = 0; i < 3ll * (K + 1) * n_inst; ++i)
        if (!is_finite_d(eta_all[i].re) || !is_finite_d(eta_all[i].im)) return QUAPI_EINVAL;
    for (int i = 0; i < M * M; ++i)
        if (!is_finite_d(p->rho0[i].re) || !is_finite_d(p->rho0[i].im)) return QUAPI_EINVAL;

    // mask: sorted, distinct, contains 0 and 1, lags < K
    std::vector<int> mask;
    if (p->mask && p->n_mask > 0) {
        mask.assign(p->mask, p->mask + p->n_mask);
    } else if (p->mask && p->n_mask < 0) {
        return QUAPI_EINVAL;
    } else {
        for (int d = 0; d < K; ++d) mask.push_back(d);
    }
    if (mask.size() < 2 || mask[0] != 0 || mask[1] != 1) return QUAPI_EINVAL;
    for (size_t i = 1; i < mask.size(); ++i)
        if (mask[i] <= mask[i - 1] || mask[i] >= K) return QUAPI_EINVAL;
    // merge positions: pre-merging {mask[i]-1 : i>=1}, post-merging the mask itself
    std::vector<int> pos;
    if (p->mode == QUAPI_PRE) {
        for (size_t i = 1; i < mask.size(); ++i) pos.push_back(mask[i] - 1);
    } else {
        pos = mask;
    }
    // merge positions 0..L-1 (L >= 2) take the bucketed path; any other set the
    // hash-table path, which keeps each history in one or two 64-bit words, the
    // key in 62 bits and the points at the other positions in one 64-bit word
    // (the FP32 precision form runs on the direct-mapped store and the hash-table merge)
    // (four levels, 16 pairs of 4-bit points, run on the hash-table merge, which takes any P)
    bool contiguous = pos.size() >= 2 && M <= 3;
    for (size_t i = 0; i < pos.size(); ++i)
        if (pos[i] != (int)i) contiguous = false;
    const int L = (int)pos.size();
    const int P = M * M;
    const int bits = P <= 4 ? 2 : 4;
    if (contiguous) {
        if (L * bits > 62 || (K - L) * bits > 64) return QUAPI_EUNSUPPORTED;
    } else {
        if (K * bits > 128 || L * bits > 62 || (K - L) * bits > 64) return QUAPI_EUNSUPPORTED;
    }
    // the batched form is built on the bucketed store (FP64, merge positions 0..L-1)
    if (batch && !contiguous) return QUAPI_EUNSUPPORTED;
    // store: merge positions 0..L-1 of a two-level system with 5 <= L <= 13 (at most
    // 4^13 slots of 24 B) take the direct-mapped store unless the caller asks for
    // another; the bucketed store serves every contiguous mask, the hash table every mask
    const int merge = p->merge;
    if (merge < QUAPI_MERGE_AUTO || merge > QUAPI_MERGE_PARTITION) return QUAPI_EINVAL;
    const bool hash_store = merge == QUAPI_MERGE_HASH || merge == QUAPI_MERGE_PARTITION;
    const bool dense_ok =
        contiguous && !batch && M == 2 && L >= quapi_dev::kDenseMinL && L <= quapi_dev::kDenseMaxL;
    if (merge == QUAPI_MERGE_DIRECT && !dense_ok) return QUAPI_EUNSUPPORTED;
    // the precision form has no bucketed store: its contiguous masks go to the
    // direct-mapped store where that applies, else to the hash table
    const bool f32_form = p->precision == QUAPI_FP32_LOG;
    if (f32_form && batch) return QUAPI_EUNSUPPORTED;      // the batched form is FP64
    if (merge == QUAPI_MERGE_BUCKETED && (!contiguous || f32_form)) return QUAPI_EUNSUPPORTED;
    if (hash_store && batch) return QUAPI_EUNSUPPORTED;
    if (hash_store && contiguous) {
        // the hash table takes any merge positions
        if (K * bits > 128 || L * bits > 62 || (K - L) * bits > 64) return QUAPI_EUNSUPPORTED;
        contiguous = false;
    }
    // AUTO takes the direct-mapped store where it applies (measured the faster of the
    // two on merge positions 0..L-1) and max_groups does not ask for fewer than its 4^L
    // slots, else the bucketed store for 0..L-1, else the table
    const bool auto_dense = merge == QUAPI_MERGE_AUTO && (p->max_groups <= 0 || p->max_groups >= ipow(P, L));
    const bool use_dense = dense_ok && (merge == QUAPI_MERGE_DIRECT || auto_dense);
    if (f32_form && contiguous && !use_dense) {
        if (K * bits > 128 || L * bits > 62 || (K - L) * bits > 64) return QUAPI_EUNSUPPORTED;
        contiguous = false;
    }
    const quapi_c64* const eta0 = eta_all;                // instance 0

    quapi_ctx* c = new (std::nothrow) quapi_ctx();
    if (!c) return QUAPI_ENOMEM;
    c->M = M;
    c->P = P;
    c->K = K;
    c->L = L;
    c->bits = bits;
    c->mode = p->mode;
    // the FP32 form's rounding of |w|^2 (~1e-6 relative) would split values the
    // FP64 form sees as equal across 2^-20 quanta: it compares 12 mantissa bits
    c->qbits = p->qbits < 0 ? (p->precision == QUAPI_FP32_LOG ? 40 : 32) : std::min(p->qbits, 63);
    c->dt = p->dt;
    c->theta = p->theta;
    c->sparse = !contiguous;
    c->dense = use_dense;
    c->f32 = p->precision == QUAPI_FP32_LOG;
    // the hash-table store merges through partitions unless the table is asked for
    c->sp_part = c->sparse && merge != QUAPI_MERGE_HASH;
    c->qpos = pos;
    if (c->sparse) {
        // the other positions, oldest first; the representative word packs
        // them below the quantised |w|^2 when they fit in its qbits+1 low bits
        for (int j = K - 1; j >= 0; --j)
            if (std::find(pos.begin(), pos.end(), j) == pos.end()) c->npos.push_back(j);
        c->sp_packed = c->qbits <= 62 && (int)c->npos.size() * bits <= c->qbits + 1;
        c->sp_hw = K * bits <= 64 ? 1 : 2;
    }

    // buckets: the top D points of the key, D-1 the most points with at most
    // max_super super-buckets (bounded by what the planner is built for); a
    // bucket holds every key of its prefix, or its share of max_groups
    const long long plan_super = quapi_dev::plan_max_buckets() / (M * M);
    long long max_super = 8192;   // tuning knob: upper bound on the number of super-buckets
    if (const char* env = std::getenv("QUAPI_MAX_SUPER")) max_super = std::max(1ll, std::atoll(env));
    max_super = std::min(max_super, plan_super);
    // batched form: one planner workgroup per instance takes all of its buckets
    if (batch) max_super = std::min(max_super, (long long)quapi_dev::plan_batch_max_buckets() / P);
    int dm1 = 0;
    while (!c->sparse && !c->dense && dm1 + 1 <= L - 1 && ipow(P, dm1 + 1) <= max_super) ++dm1;
    c->D = dm1 + 1;
    c->n_super = (int)ipow(P, dm1);
    c->n_inst = n_inst;
    c->batch = batch;
    c->inst_buckets = ipow(P, c->D);
    c->n_buckets = c->inst_buckets * n_inst;
    long long cap = (c->sparse || c->dense) ? 1 : ipow(P, L - c->D);
    // (max_groups counts one instance)
    if (p->max_groups > 0) cap = std::max(1ll, std::min(cap, (p->max_groups + c->inst_buckets - 1) / c->inst_buckets));
    // group indices are 32-bit: keep the whole store below 2^31 groups
    cap = std::min(cap, ((1ll << 31) - 1) / c->n_buckets);
    if (cap < 1) {
        delete c;
        return QUAPI_EUNSUPPORTED;
    }
    c->cap = cap;

    // tables: K4[pn][po] = U[an][ao] conj(U[bn][bo]); ds, ss; eta
    auto k4_of = [&](const quapi_c64* H, double* dst) {
        std::vector<double> U(2 * M * M);
        quapi_host::propagator(M, (const double*)H, p->dt, U.data());
        for (int pn = 0; pn < P; ++pn)
            for (int po = 0; po < P; ++po) {
                const std::complex<double> u1(U[2 * ((pn / M) * M + po / M)], U[2 * ((pn / M) * M + po / M) + 1]);
                const std::complex<double> u2(U[2 * ((pn % M) * M + po % M)], U[2 * ((pn % M) * M + po % M) + 1]);
                const std::complex<double> k4 = u1 * std::conj(u2);
                dst[2 * (pn * P + po)] = k4.real();
                dst[2 * (pn * P + po) + 1] = k4.imag();
            }
    };
    c->tables.assign(TableLayout::total(P, K), 0.0);
    k4_of(H_all ? H_all : p->H, c->tables.data());
    if (H_all) {
        c->k4_batch.assign((size_t)n_inst * 2 * P * P, 0.0);
        for (int j = 0; j < n_inst; ++j) k4_of(H_all + (size_t)M * M * j, c->k4_batch.data() + (size_t)j * 2 * P * P);
    }
    for (int pp = 0; pp < P; ++pp) {
        c->tables[TableLayout::ds(P) + pp] = p->q[pp / M] - p->q[pp % M];
        c->tables[TableLayout::ss(P) + pp] = p->q[pp / M] + p->q[pp % M];
    }
    for (int i = 0; i < 3 * (K + 1); ++i) {
        c->tables[TableLayout::eta(P) + 2 * i] = eta0[i].re;
        c->tables[TableLayout::eta(P) + 2 * i + 1] = eta0[i].im;
    }
    // coefficients of the new point at step t with the point at lag d (eq. inf_fun
    // windows): interior partners use the interior column, the time-0 partner
    // (d == t) the half-window column; the end-point correction of rho(t) swaps
    // the final point's interior coefficients for its half-window ones
    // (one set per instance: [t-1][instance][4][K+1])
    const int n = K + 1;
    c->coef.assign((size_t)(K + 1) * n_inst * 4 * n, 0.0);
    for (int t = 1; t <= K + 1; ++t)
    for (int j = 0; j < n_inst; ++j) {
        const quapi_c64* const eta = eta_all + (size_t)3 * n * j;
        double* cs = c->coef.data() + ((size_t)(t - 1) * n_inst + j) * 4 * n;
        for (int d = 0; d <= K && d <= t; ++d) {
            const quapi_c64 in = eta[d], hf = eta[n + d], hh = eta[2 * n + d];
            const quapi_c64 cc = (d == t) ? hf : in;
            quapi_c64 dd;
            if (d == 0) dd = {hf.re - in.re, hf.im - in.im};
            else if (d == t) dd = {hh.re - hf.re, hh.im - hf.im};
            else dd = {hf.re - in.re, hf.im - in.im};
            cs[d] = cc.re;
            cs[n + d] = cc.im;
            cs[2 * n + d] = dd.re;
            cs[3 * n + d] = dd.im;
        }
    }

    // the kernels' sin/cos take phases below kTrigArgMax: bound every phase a
    // child or an end-point correction can get, |ds_p| sum_d |Im c_d| max|ss|
    {
        double ds_max = 0.0, ss_max = 0.0;
        for (int pp = 0; pp < P; ++pp) {
            ds_max = std::max(ds_max, std::fabs(c->tables[TableLayout::ds(P) + pp]));
            ss_max = std::max(ss_max, std::fabs(c->tables[TableLayout::ss(P) + pp]));
        }
        double worst = 0.0;
        for (size_t set = 0; set < (size_t)(K + 1) * n_inst; ++set)
            for (int col = 1; col <= 3; col += 2) {          // Im of the coefficients and of the corrections
                const double* cs = c->coef.data() + set * 4 * n + (size_t)col * n;
                double sum = 0.0;
                for (int d = 0; d <= K; ++d) sum += std::fabs(cs[d]);
                worst = std::max(worst, ds_max * sum * ss_max);
            }
        if (!(worst < quapi_dev::kTrigArgMax)) {
            delete c;
            return QUAPI_EUNSUPPORTED;
        }
    }

    // t = 0: one group per nonzero element of rho0 with the initial point's self term
    c->rho0.resize(2 * P);
    for (int pp = 0; pp < P; ++pp) {
        const std::complex<double> r(p->rho0[pp].re, p->rho0[pp].im);
        c->rho0[2 * pp] = r.real();
        c->rho0[2 * pp + 1] = r.imag();
        if (r == std::complex<double>(0, 0)) continue;
        c->init_key.push_back(c->sparse ? 0ull : (unsigned long long)pp << (bits * (L - 1)));
        c->init_pair.push_back(pp);
        c->init_bucket.push_back((long long)pp * c->n_super);   // top D points (pp, 0, ..., 0)
    }
    for (int j = 0; j < n_inst; ++j) {
        const quapi_c64 e0c = eta_all[(size_t)3 * n * j + n];     // end-point self term
        const std::complex<double> e0(e0c.re, e0c.im);
        for (int pp : c->init_pair) {
            const std::complex<double> r(p->rho0[pp].re, p->rho0[pp].im);
            const double ds = c->tables[TableLayout::ds(P) + pp], ss = c->tables[TableLayout::ss(P) + pp];
            const std::complex<double> w = r * std::exp(std::complex<double>(-ds * e0.real() * ds, -ds * e0.imag() * ss));
            c->init_w.push_back(make_double2(w.real(), w.imag()));
        }
    }

    int rc = QUAPI_OK;
    if (hipGetDevice(&c->dev) != hipSuccess) {
        delete c;
        return QUAPI_EDEVICE;
    }
    if (p->stream) {
        c->stream = (hipStream_t)p->stream;
    } else {
        if (acquire_shared_stream(c->dev, &c->stream) != hipSuccess) {
            delete c;
            return QUAPI_EDEVICE;
        }
        c->own_stream = true;
        c->stream_dev = c->dev;
    }

    const size_t nrec = (c->sparse || c->dense) ? 1 : (size_t)c->n_buckets * (size_t)cap;
    for (int b = 0; b < 2 && rc == QUAPI_OK; ++b) {
        rc = dev_alloc(c, &c->buf[b].key, nrec);
        if (!rc) rc = dev_alloc(c, &c->buf[b].tail, nrec);
        if (!rc) rc = dev_alloc(c, &c->buf[b].w, nrec);
        if (!rc) rc = dev_alloc(c, &c->counts[b], (size_t)c->n_buckets);
    }
    if (!rc) rc = dev_alloc(c, &c->d_tables, c->tables.size());
    if (!rc) rc = dev_alloc(c, &c->d_coef, c->coef.size());
    if (!rc && !c->k4_batch.empty()) rc = dev_alloc(c, &c->d_k4_batch, c->k4_batch.size());
    if (!rc && batch && P == 4)
        rc = dev_alloc(c, &c->d_inst_tabs, (size_t)n_inst * quapi_dev::instance_table_doubles());
    // (each instance of the batched form starts a chunk: one partial chunk more each)
    c->max_chunks = (int)std::min<long long>((long long)nrec / quapi_dev::chunk_heads(P) + n_inst + 2, 1ll << 30);
    if (!rc) rc = dev_alloc(c, &c->d_partials, (size_t)c->max_chunks * quapi_dev::partial_stride(P));
    if (!rc) rc = dev_alloc(c, &c->d_nz_bucket, (size_t)c->n_buckets + n_inst);
    if (!rc) rc = dev_alloc(c, &c->d_nz_prefix, (size_t)c->n_buckets + n_inst);
    if (!rc && batch) rc = dev_alloc(c, &c->d_totals, (size_t)n_inst);
    if (!rc && batch) rc = dev_alloc(c, &c->d_inst, (size_t)4 * n_inst);
    if (!rc) rc = dev_alloc(c, &c->d_desc, (size_t)c->max_chunks);
    if (!rc) rc = dev_alloc(c, &c->d_plan, 2);
    if (!rc) rc = dev_alloc(c, &c->d_chain, (size_t)P * c->max_chunks);
    if (!rc) rc = dev_alloc(c, &c->d_error, 1);
    if (!rc && c->dense) {
        c->dn_slots = (unsigned long long)ipow(P, L);
        for (int b = 0; b < 2 && !rc; ++b) {
            rc = dev_alloc(c, &c->dn_flag[b], (size_t)c->dn_slots);
            if (!rc && !c->f32) rc = dev_alloc(c, &c->dn_rec[b], (size_t)c->dn_slots);
            if (!rc && c->f32) rc = dev_alloc(c, &c->dn_rec32[b], (size_t)c->dn_slots);
        }
        if (!rc) rc = dev_alloc(c, &c->dn_seg, (size_t)c->dn_slots);   // four lists of S/4
        if (!rc) rc = dev_alloc(c, &c->dn_plan, 2);
        if (!rc) rc = dev_alloc(c, &c->dn_tabs, (size_t)(K + 1) * quapi_dev::dense_tabset_doubles(L, K));
        if (!rc) rc = dev_alloc(c, &c->dn_agg, (size_t)quapi_dev::kDenseMaxRegions);
    }
    if (!rc && c->sparse) {
        // capacity: max_groups, else every key of the merge positions up to 2^21 groups;
        // the table holds twice the children a step can insert
        long long scap = p->max_groups > 0 ? p->max_groups : std::min(ipow(P, std::min(L, 12)), 1ll << 21);
        scap = std::max((long long)c->init_pair.size(), std::min(scap, ((1ll << 31) - 1) / P));
        c->sp_cap = scap;
        // segments: an eighth over an even share, and room for a few merge tiles
        const unsigned long long seg_cap = ((unsigned long long)scap * 9 / 8 + quapi_dev::kSegs - 1) / quapi_dev::kSegs + 4096;
        c->sp_seg_cap = seg_cap;
        const size_t n_slots = (size_t)seg_cap * quapi_dev::kSegs;
        unsigned long long ts = quapi_dev::kMinTable;
        while (ts < 2ull * (unsigned long long)P * (unsigned long long)scap) ts <<= 1;
        c->sp_tsize = ts;
        for (int b = 0; b < 2 && !rc; ++b) {
            rc = dev_alloc(c, &c->sp_h[b], n_slots * c->sp_hw);
            if (!rc && c->f32) rc = dev_alloc(c, &c->sp_wf[b], n_slots);
            if (!rc && !c->f32) rc = dev_alloc(c, &c->sp_w[b], n_slots);
        }
        if (!rc) rc = dev_alloc(c, &c->sp_count, (size_t)quapi_dev::seg_counter(2, 0));
        if (c->sp_part) {
            // partitions for the children of a full store, one per kPartLoad
            unsigned long long np = 1;
            while (np * quapi_dev::kPartLoad < (unsigned long long)P * (unsigned long long)scap) np <<= 1;
            c->sp_n_part = (unsigned int)np;
            const size_t ne = (size_t)np * quapi_dev::kPartCap;
            if (!rc) rc = dev_alloc(c, &c->sp_pcount, (size_t)np);
            // unpacked form: key, other points and quantised |w|^2 in one 128-bit number where they fit
            c->sp_pfit = !c->sp_packed && bits * K + (63 - c->qbits) <= 128;
            if (!rc) rc = dev_alloc(c, &c->sp_prec, ne);
            if (!rc && !c->sp_packed && !c->sp_pfit) rc = dev_alloc(c, &c->sp_pother, ne);
        } else {
        if (!rc) rc = dev_alloc(c, &c->sp_slot, (size_t)ts);
        if (!c->sp_packed) {
            if (!rc) rc = dev_alloc(c, &c->sp_tN, (size_t)ts);
            if (!rc) rc = dev_alloc(c, &c->sp_cslot, (size_t)scap * P);
            if (!rc) rc = dev_alloc(c, &c->sp_cN, (size_t)scap * P);
            if (!rc) rc = dev_alloc(c, &c->sp_cq, (size_t)scap * P);
        }
        }
    }
    c->hist_cap = p->max_steps > 0 ? p->max_steps : 1024;
    if (!rc) rc = dev_alloc(c, &c->d_rho, (size_t)(c->hist_cap + 1) * n_inst * P);
    if (!rc) rc = dev_alloc(c, &c->d_stats, (size_t)(c->hist_cap + 1) * n_inst);
    if (rc) {
        quapi_destroy(c);
        return rc;
    }
    hipError_t e = hipMemcpyAsync(c->d_tables, c->tables.data(), c->tables.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_coef, c->coef.data(), c->coef.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess && c->dense &&
        quapi_dev::launch_dense_tables(c->d_coef, c->d_tables, L, K, K + 1, c->dn_tabs, c->stream) != (int)hipSuccess)
        e = hipErrorLaunchFailure;
    if (e == hipSuccess && c->d_k4_batch)
        e = hipMemcpyAsync(c->d_k4_batch, c->k4_batch.data(), c->k4_batch.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->d_chain, 0, (size_t)P * c->max_chunks * sizeof(unsigned long long), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->d_plan, 0, 2 * sizeof(quapi_dev::Plan), c->stream);
    if (e == hipSuccess && c->d_inst) e = hipMemsetAsync(c->d_inst, 0, (size_t)4 * n_inst * sizeof(unsigned int), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        quapi_destroy(c);
        return hip_to_code(e);
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        quapi_destroy(c);
        return QUAPI_EDEVICE;
    }
    // persistent workgroups: as many as are resident at once (the look-back between
    // chunks needs every workgroup of the grid resident); QUAPI_BLOCKS_PER_CU lowers it
    int per_cu = 0;
    if (const char* env = std::getenv("QUAPI_BLOCKS_PER_CU")) per_cu = std::max(1, std::min(16, std::atoi(env)));
    // (the bucketed step kernel is built for P = 4 and 9; the hash-table merge has grids of its own)
    c->grid = c->sparse ? 1 : quapi_dev::step_grid(P, std::max(ncu, 1), per_cu, n_inst > 1);
    if (c->grid < 1) {
        quapi_destroy(c);
        return QUAPI_EDEVICE;
    }
    if (c->dense) {
        // persistent workgroups, as many as are resident (their chunks never wait on one another)
        c->dn_lds = quapi_dev::dense_lds_bytes(L, K, c->f32);
        c->dn_grid = quapi_dev::dense_step_grid(std::max(ncu, 1), c->dn_lds, c->f32);
        if (per_cu > 0) c->dn_grid = std::min(c->dn_grid, per_cu * std::max(ncu, 1));
        if (c->dn_grid < 1 ||
            dev_alloc(c, &c->dn_partials, (size_t)c->dn_grid * quapi_dev::partial_stride(4)) != QUAPI_OK ||
            hipMemsetAsync(c->dn_plan, 0, 2 * sizeof(quapi_dev::DensePlan), c->stream) != hipSuccess ||
            hipMemsetAsync(c->dn_agg, 0, quapi_dev::kDenseMaxRegions * 8, c->stream) != hipSuccess) {
            quapi_destroy(c);
            return QUAPI_EDEVICE;
        }
    }
    if (c->sparse) {
        // a multiple of kSegs, so that every segment has as many writers
        c->sp_grid = (4 * std::max(ncu, 1) + quapi_dev::kSegs - 1) / quapi_dev::kSegs * quapi_dev::kSegs;
        c->sp_grid_merge = quapi_dev::sparse_merge_grid(P, c->sp_hw, c->f32, ncu);
        if (dev_alloc(c, &c->sp_partials, (size_t)c->sp_grid * quapi_dev::partial_stride(P)) != QUAPI_OK) {
            quapi_destroy(c);
            return QUAPI_ENOMEM;
        }
    }
    rc = upload_initial(c);
    if (rc) {
        quapi_destroy(c);
        return rc;
    }
    *out = c;
    return QUAPI_OK;
}

int quapi_create(const quapi_params* p, quapi_ctx** out) {
    if (!p) {
        if (out) *out = nullptr;
        return QUAPI_EINVAL;
    }
    return create_ctx(p, 1, p->eta, nullptr, false, out);
}

int quapi_create_batch(const quapi_params* p, int n_inst, const quapi_c64* eta_batch, const quapi_c64* H_batch,
                       quapi_ctx** out) {
    return create_ctx(p, n_inst, eta_batch, H_batch, true, out);
}

int quapi_step(quapi_ctx* c, int n_steps) {
    if (!c || n_steps < 0) return QUAPI_EINVAL;
    if (c->err) return QUAPI_ESTATE;
    if (n_steps == 0) return QUAPI_OK;
    int rc = grow_history(c, c->t + n_steps);
    if (rc) return rc;
    if (c->sparse) return step_sparse(c, n_steps);
    if (c->dense) return step_dense(c, n_steps);
    StepArgs a;
    a.cap = c->cap;
    a.P = c->P;
    a.L = c->L;
    a.K = c->K;
    a.n_super = c->n_super;
    a.n_inst = c->n_inst;
    a.chunk_run = c->chunk_run;
    a.k4_batch = c->d_k4_batch;
    a.inst_tabs = c->n_inst > 1 ? c->d_inst_tabs : nullptr;
    a.theta2 = c->theta * c->theta;
    a.qmask = c->qbits >= 64 ? 0ull : ~((1ull << c->qbits) - 1ull);
    a.tables = c->d_tables;
    a.nz_bucket = c->d_nz_bucket;
    a.nz_prefix = c->d_nz_prefix;
    a.desc = c->d_desc;
    a.chain = c->d_chain;
    a.max_chunks = c->max_chunks;
    a.partials = c->d_partials;
    a.error = c->d_error;
    const int n = c->K + 1;
    for (int k = 0; k < n_steps; ++k) {
        const int t = c->t + 1;
        a.in = c->buf[c->cur];
        a.out = c->buf[1 - c->cur];
        a.out_count = c->counts[1 - c->cur];
        a.plan = c->d_plan + (t & 1);
        a.t = t;
        a.epoch = ++c->epoch;
        a.coef = c->d_coef + (size_t)(std::min(t, c->K + 1) - 1) * c->n_inst * 4 * n;
        // the batched form's instance tables follow the coefficient set, which is
        // the same from step K+1 on
        if (a.inst_tabs && t <= c->K + 1 &&
            quapi_dev::launch_instance_tables(a, c->d_inst_tabs, c->stream) != (int)hipSuccess) {
            c->err = QUAPI_EDEVICE;
            return c->err;
        }
        hipEvent_t* ev = (c->prof_on && !c->capturing && c->prof_n < c->prof_cap)
                             ? &c->prof_ev[3 * (size_t)c->prof_n++] : nullptr;
        if (ev && hipEventRecord(ev[0], c->stream) != hipSuccess) ev = nullptr;
        // (inside a graph capture the whole graph is ordered at its launch instead)
        const hipError_t le =
            c->capturing ? (hipError_t)quapi_dev::launch_step(a, c->grid, c->stream)
                         : ordered_launch(c->dev, c->stream, [&] {
                               return (hipError_t)quapi_dev::launch_step(a, c->grid, c->stream);
                           });
        if (le != hipSuccess) {
            c->err = QUAPI_EDEVICE;
            return c->err;
        }
        if (ev) (void)hipEventRecord(ev[1], c->stream);
        c->t = t;
        c->cur = 1 - c->cur;
        // reduce step t and plan step t+1
        if (launch_planner(c, t) != QUAPI_OK) {
            c->err = QUAPI_EDEVICE;
            return c->err;
        }
        if (ev) (void)hipEventRecord(ev[2], c->stream);
    }
    return QUAPI_OK;
}

int quapi_step_graph(quapi_ctx* c, int n_steps) {
    if (!c || n_steps < 1) return QUAPI_EINVAL;
    if (c->err) return QUAPI_ESTATE;
    if (c->sparse) return QUAPI_EUNSUPPORTED;
    int rc = grow_history(c, c->t + n_steps);      // allocations stay outside the capture
    if (rc) return rc;
    const bool hit = c->graph && c->graph_t0 == c->t && c->graph_n == n_steps && c->graph_cur0 == c->cur &&
                     c->graph_run == c->chunk_run && c->graph_rho == c->d_rho && c->graph_stats == c->d_stats;
    if (!hit) {
        if (c->graph) {
            (void)hipGraphExecDestroy(c->graph);
            c->graph = nullptr;
        }
        const int t0 = c->t, cur0 = c->cur;
        hipGraph_t g = nullptr;
        hipError_t e = order_release(c->dev, c->stream);
        if (e != hipSuccess) return hip_to_code(e);
        e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_to_code(e);
        // look-back words of an earlier replay carry the same epochs: clear them first
        hipError_t lr = launch_clear_words(c->d_chain, (size_t)c->P * c->max_chunks, c->stream);
        if (lr == hipSuccess && c->dense)
            lr = launch_clear_words(c->dn_agg, (size_t)quapi_dev::kDenseMaxRegions, c->stream);
        c->capturing = true;
        rc = lr == hipSuccess ? quapi_step(c, n_steps) : QUAPI_EDEVICE;
        c->capturing = false;
        e = hipStreamEndCapture(c->stream, &g);
        // nothing recorded has run: back to the state before the capture
        c->t = t0;
        c->cur = cur0;
        if (rc == QUAPI_EDEVICE) c->err = QUAPI_OK;
        if (rc != QUAPI_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return rc != QUAPI_OK ? rc : hip_to_code(e);
        }
        e = hipGraphInstantiateWithFlags(&c->graph, g, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->graph = nullptr;
            (void)hipGetLastError();
            return hip_to_code(e);
        }
        c->graph_t0 = t0;
        c->graph_n = n_steps;
        c->graph_cur0 = cur0;
        c->graph_run = c->chunk_run;
        c->graph_rho = c->d_rho;
        c->graph_stats = c->d_stats;
        c->graph_epoch_end = c->epoch;
    }
    const hipError_t e = ordered_launch(c->dev, c->stream, [&] { return hipGraphLaunch(c->graph, c->stream); });
    if (e != hipSuccess) {
        c->err = QUAPI_EDEVICE;
        return c->err;
    }
    c->t += n_steps;
    if (n_steps & 1) c->cur = 1 - c->cur;
    // later eager steps take epochs above every recorded one
    if (c->epoch < c->graph_epoch_end) c->epoch = c->graph_epoch_end;
    return QUAPI_OK;
}

int quapi_sync(quapi_ctx* c) {
    if (!c) return QUAPI_EINVAL;
    return sync_ctx(c);
}

int quapi_time(quapi_ctx* c, int* t_out) {
    if (!c || !t_out) return QUAPI_EINVAL;
    const int rc = sync_ctx(c);
    *t_out = c->t;
    return rc == QUAPI_EDEVICE ? rc : QUAPI_OK;
}

int quapi_batch_rho_history(quapi_ctx* c, int inst, int t0, int n, quapi_c64* out) {
    if (!c || !out || t0 < 0 || n < 0 || inst < 0 || inst >= c->n_inst) return QUAPI_EINVAL;
    const int rc = sync_ctx(c);
    if (rc == QUAPI_EDEVICE) return rc;
    if (t0 + n - 1 > c->t) return QUAPI_EINVAL;
    if (n == 0) return QUAPI_OK;
    // history rows hold every instance: [t][instance][P]
    const size_t row = (size_t)c->n_inst * c->P;
    const hipError_t e = hipMemcpy2D(out, (size_t)c->P * sizeof(double2), c->d_rho + (size_t)t0 * row + (size_t)inst * c->P,
                                     row * sizeof(double2), (size_t)c->P * sizeof(double2), (size_t)n,
                                     hipMemcpyDeviceToHost);
    return hip_to_code(e);
}

int quapi_rho_history(quapi_ctx* c, int t0, int n, quapi_c64* out) { return quapi_batch_rho_history(c, 0, t0, n, out); }

int quapi_batch_rho_all(quapi_ctx* c, int t0, int n, quapi_c64* out) {
    if (!c || !out || t0 < 0 || n < 0) return QUAPI_EINVAL;
    const int rc = sync_ctx(c);
    if (rc == QUAPI_EDEVICE) return rc;
    if (t0 + n - 1 > c->t) return QUAPI_EINVAL;
    if (n == 0) return QUAPI_OK;
    const size_t row = (size_t)c->n_inst * c->P;
    return hip_to_code(hipMemcpy(out, c->d_rho + (size_t)t0 * row, (size_t)n * row * sizeof(double2),
                                 hipMemcpyDeviceToHost));
}

int quapi_set_chunk_run(quapi_ctx* c, int run) {
    if (!c || run < 1 || run > 64) return QUAPI_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    c->chunk_run = run;
    return QUAPI_OK;
}

int quapi_autotune(quapi_ctx* c, int n_steps, int* run_out) {
    if (!c || n_steps < 1) return QUAPI_EINVAL;
    if (c->err) return QUAPI_ESTATE;
    // runs matter to the batched form only (they change how often a workgroup
    // switches instance); a lone context keeps round-robin
    static const int kRuns[] = {1, 2, 4, 8, 16};
    int best = 1;
    if (c->n_inst > 1) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            return QUAPI_EDEVICE;
        }
        float best_ms = 0.0f;
        int rc = QUAPI_OK;
        for (int r : kRuns) {
            c->chunk_run = r;
            rc = quapi_reset(c);
            if (rc) break;
            (void)hipEventRecord(e0, c->stream);
            rc = quapi_step(c, n_steps);
            if (rc) break;
            (void)hipEventRecord(e1, c->stream);
            rc = sync_ctx(c);
            if (rc) break;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = QUAPI_EDEVICE; break; }
            if (r == kRuns[0] || ms < best_ms) { best_ms = ms; best = r; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc) return rc;
    }
    c->chunk_run = best;
    if (run_out) *run_out = best;
    return quapi_reset(c);
}

int quapi_rho(quapi_ctx* c, int t, quapi_c64* rho_out) { return quapi_rho_history(c, t, 1, rho_out); }

int quapi_batch_step_stats(quapi_ctx* c, int inst, int t0, int n, quapi_stepstat_t* out) {
    if (!c || !out || t0 < 1 || n < 0 || inst < 0 || inst >= c->n_inst) return QUAPI_EINVAL;
    const int rc = sync_ctx(c);
    if (rc == QUAPI_EDEVICE) return rc;
    if (t0 + n - 1 > c->t) return QUAPI_EINVAL;
    std::vector<StepStatsDev> h(n);
    if (n) {
        const hipError_t e = hipMemcpy2D(h.data(), sizeof(StepStatsDev), c->d_stats + (size_t)t0 * c->n_inst + inst,
                                         (size_t)c->n_inst * sizeof(StepStatsDev), sizeof(StepStatsDev), (size_t)n,
                                         hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_to_code(e);
    }
    for (int k = 0; k < n; ++k) {
        out[k].t = t0 + k;
        out[k].n_groups = (long long)h[k].n_groups;
        out[k].n_children = (long long)h[k].n_children;
        out[k].n_survivors = (long long)h[k].n_survivors;
        out[k].n_stored = (long long)h[k].n_stored;
        out[k].dropped_abs = h[k].dropped_abs;
    }
    return QUAPI_OK;
}

int quapi_step_stats(quapi_ctx* c, int t0, int n, quapi_stepstat_t* out) {
    return quapi_batch_step_stats(c, 0, t0, n, out);
}

int quapi_batch_groups(quapi_ctx* c, int inst, long long cap, unsigned char* hist, quapi_c64* w,
                       long long* n_out) {
    if (!c || !n_out || cap < 0 || (cap > 0 && (!hist || !w)) || inst < 0 || inst >= c->n_inst)
        return QUAPI_EINVAL;
    const int rc = sync_ctx(c);
    if (rc == QUAPI_EDEVICE) return rc;
    if (c->sparse) {
        std::vector<unsigned int> cnt((size_t)quapi_dev::seg_counter(2, 0));
        hipError_t e = hipMemcpy(cnt.data(), c->sp_count, cnt.size() * sizeof(unsigned int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_to_code(e);
        // the segments' groups, one after the other
        unsigned long long seg_n[quapi_dev::kSegs];
        long long n = 0;
        for (int s = 0; s < quapi_dev::kSegs; ++s) {
            seg_n[s] = std::min<unsigned long long>(cnt[quapi_dev::seg_counter(c->t & 1, s)], c->sp_seg_cap);
            n += (long long)seg_n[s];
        }
        *n_out = n;
        if (cap == 0 || n == 0) return QUAPI_OK;
        const int hw = c->sp_hw;
        std::vector<uint64_t> hh((size_t)n * hw);
        std::vector<double2> ww((size_t)n);
        std::vector<float2> wl(c->f32 ? (size_t)n : 0);
        size_t r0 = 0;
        for (int s = 0; s < quapi_dev::kSegs && e == hipSuccess; ++s) {
            if (!seg_n[s]) continue;
            const size_t src = (size_t)s * c->sp_seg_cap;
            e = hipMemcpy(hh.data() + r0 * hw, c->sp_h[c->cur] + src * hw, (size_t)seg_n[s] * hw * 8,
                          hipMemcpyDeviceToHost);
            if (e == hipSuccess && c->f32)
                e = hipMemcpy(wl.data() + r0, c->sp_wf[c->cur] + src, (size_t)seg_n[s] * sizeof(float2),
                              hipMemcpyDeviceToHost);
            else if (e == hipSuccess)
                e = hipMemcpy(ww.data() + r0, c->sp_w[c->cur] + src, (size_t)seg_n[s] * 16, hipMemcpyDeviceToHost);
            r0 += (size_t)seg_n[s];
        }
        if (e != hipSuccess) return hip_to_code(e);
        for (size_t r = 0; r < wl.size(); ++r) {
            const double m = std::exp((double)wl[r].x);
            ww[r] = make_double2(m * std::cos((double)wl[r].y), m * std::sin((double)wl[r].y));
        }
        const unsigned long long dm = (1ull << c->bits) - 1;
        for (long long r = 0; r < n && r < cap; ++r) {
            unsigned char* row = hist + (size_t)r * c->K;
            for (int j = 0; j < c->K; ++j) {
                const int bit = c->bits * j;
                row[j] = (unsigned char)((hh[(size_t)r * hw + bit / 64] >> (bit % 64)) & dm);
            }
            w[r].re = ww[r].x;
            w[r].im = ww[r].y;
        }
        return QUAPI_OK;
    }
    if (c->dense) {
        const size_t S = (size_t)c->dn_slots;
        std::vector<unsigned char> flag(S);
        hipError_t e = hipMemcpy(flag.data(), c->dn_flag[c->cur], S, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_to_code(e);
        long long n = 0;
        const unsigned char tag = (unsigned char)quapi_dev::dense_tag(c->t);
        for (unsigned char f : flag) n += f == tag;
        *n_out = n;
        if (cap == 0 || n == 0) return QUAPI_OK;
        std::vector<quapi_dev::DenseRec> rec(S);
        if (c->f32) {
            std::vector<quapi_dev::DenseRec32> r32(S);
            e = hipMemcpy(r32.data(), c->dn_rec32[c->cur], S * sizeof(quapi_dev::DenseRec32), hipMemcpyDeviceToHost);
            for (size_t o = 0; e == hipSuccess && o < S; ++o) {
                if (flag[o] != tag) continue;
                const double m = std::exp((double)r32[o].lw);
                rec[o].w = make_double2(m * std::cos((double)r32[o].aw), m * std::sin((double)r32[o].aw));
                rec[o].tail = r32[o].tail;
            }
        } else {
            e = hipMemcpy(rec.data(), c->dn_rec[c->cur], S * sizeof(quapi_dev::DenseRec), hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) return hip_to_code(e);
        const unsigned long long dm = (1ull << c->bits) - 1;
        long long written = 0;
        for (size_t o = 0; o < S && written < cap; ++o) {
            if (flag[o] != tag) continue;
            unsigned char* row = hist + (size_t)written * c->K;
            for (int j = 0; j < c->K; ++j) {
                unsigned long long d;
                if (j < c->L) d = ((unsigned long long)o >> (c->bits * (c->L - 1 - j))) & dm;
                else d = (rec[o].tail >> (c->bits * (j - c->L))) & dm;
                row[j] = (unsigned char)d;
            }
            w[written].re = rec[o].w.x;
            w[written].im = rec[o].w.y;
            ++written;
        }
        return QUAPI_OK;
    }
    // the instance's buckets
    const size_t nb = (size_t)c->inst_buckets, b0 = (size_t)inst * nb;
    std::vector<unsigned int> cnt(nb);
    hipError_t e = hipMemcpy(cnt.data(), c->counts[c->cur] + b0, nb * sizeof(unsigned int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_to_code(e);
    long long n = 0;
    for (unsigned int x : cnt) n += x;
    *n_out = n;
    if (cap == 0) return QUAPI_OK;
    const size_t nrec = nb * (size_t)c->cap, r0 = b0 * (size_t)c->cap;
    std::vector<unsigned long long> k(nrec), tl(nrec);
    std::vector<double2> ww(nrec);
    e = hipMemcpy(k.data(), c->buf[c->cur].key + r0, nrec * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(tl.data(), c->buf[c->cur].tail + r0, nrec * 8, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ww.data(), c->buf[c->cur].w + r0, nrec * 16, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_to_code(e);
    const unsigned long long dm = (1ull << c->bits) - 1;
    long long written = 0;
    for (long long b = 0; b < (long long)nb && written < cap; ++b) {
        for (unsigned int r = 0; r < cnt[b] && written < cap; ++r) {
            const size_t o = (size_t)b * (size_t)c->cap + r;
            unsigned char* row = hist + (size_t)written * c->K;
            for (int j = 0; j < c->K; ++j) {
                unsigned long long d;
                if (j < c->L) d = (k[o] >> (c->bits * (c->L - 1 - j))) & dm;
                else d = (tl[o] >> (c->bits * (j - c->L))) & dm;
                row[j] = (unsigned char)d;
            }
            w[written].re = ww[o].x;
            w[written].im = ww[o].y;
            ++written;
        }
    }
    return QUAPI_OK;
}

int quapi_groups(quapi_ctx* c, long long cap, unsigned char* hist, quapi_c64* w, long long* n_out) {
    return quapi_batch_groups(c, 0, cap, hist, w, n_out);
}

int quapi_reset(quapi_ctx* c) {
    if (!c) return QUAPI_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    return upload_initial(c);
}

int quapi_info(quapi_ctx* c, quapi_info_t* out) {
    if (!c || !out) return QUAPI_EINVAL;
    out->M = c->M;
    out->P = c->P;
    out->K = c->K;
    out->L = c->L;
    out->bits_per_point = c->bits;
    out->record_bytes = c->sparse ? (c->f32 ? 8 : 16) + 8 * c->sp_hw : c->dense ? (c->f32 ? 16 : 24) : 32;
    out->capacity = c->sparse ? c->sp_cap : c->dense ? (long long)c->dn_slots : c->inst_buckets * c->cap;
    out->device_bytes = c->device_bytes;
    out->precision = c->f32 ? QUAPI_FP32_LOG : QUAPI_FP64;
    out->hash_merge = c->sparse ? 1 : 0;
    out->store = c->sparse ? (c->sp_part ? QUAPI_MERGE_PARTITION : QUAPI_MERGE_HASH)
                           : c->dense ? QUAPI_MERGE_DIRECT : QUAPI_MERGE_BUCKETED;
    out->n_instances = c->n_inst;
    return QUAPI_OK;
}

void* quapi_stream(quapi_ctx* c) { return c ? (void*)c->stream : nullptr; }

int quapi_profile_begin(quapi_ctx* c, int max_launches) {
    if (!c || max_launches < 1) return QUAPI_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    const size_t need = 3 * (size_t)max_launches;
    while (c->prof_ev.size() < need) {
        hipEvent_t e = nullptr;
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            (void)hipGetLastError();
            return hip_to_code(r);
        }
        c->prof_ev.push_back(e);
    }
    c->prof_cap = max_launches;
    c->prof_n = 0;
    c->prof_on = true;
    return QUAPI_OK;
}

int quapi_profile_end(quapi_ctx* c, int cap, double* step_ms, double* plan_ms, int* n_out) {
    if (!c || !n_out || cap < 0) return QUAPI_EINVAL;
    if (!c->prof_on) return QUAPI_ESTATE;
    c->prof_on = false;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return QUAPI_EDEVICE;
    *n_out = c->prof_n;
    for (int k = 0; k < c->prof_n && k < cap; ++k) {
        float a = 0.f, b = 0.f;
        if (hipEventElapsedTime(&a, c->prof_ev[3 * k], c->prof_ev[3 * k + 1]) != hipSuccess ||
            hipEventElapsedTime(&b, c->prof_ev[3 * k + 1], c->prof_ev[3 * k + 2]) != hipSuccess)
            return QUAPI_EDEVICE;
        if (step_ms) step_ms[k] = a;
        if (plan_ms) plan_ms[k] = b;
    }
    return QUAPI_OK;
}

void quapi_destroy(quapi_ctx* c) {
    if (!c) return;
    if (c->stream) {
        (void)order_release(c->dev, c->stream);
        (void)hipStreamSynchronize(c->stream);
    }
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    c->prof_ev.clear();
    for (void* p : c->allocations) (void)hipFree(p);
    c->allocations.clear();
    if (c->own_stream && c->stream) release_shared_stream(c->stream_dev);
    delete c;
}

}  // extern "C"
