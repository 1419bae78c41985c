// Plain FP64 reference of the MACGIC-iQUAPI path propagation.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
// this file; only tests/, __graft_entry__.smoke() and the cpu_baseline leg of
// bench.py may.  It shares no code with the HIP library.
//
// What it computes, in the paper's order (Sec. 2, 2.1, 3.1, 3.2.1):
//   * the short-time propagator S of eq. SysP from U = exp(-i H dt), with U
//     taken from its power series (scaling and squaring);
//   * the influence factor of eq. inf_fun, truncated to the finite memory of
//     Sec. 2 (lags 0..dk_max), with window-typed eta coefficients supplied by
//     the caller (interior / half-window end point / initial x final point);
//   * per time step, for the pre-merging variant (Sec. 3.1, Scheme premerging):
//       premerging()  - group the stored paths on the reduced mask
//                       {mask[i]-1 : i>=1}; a group keeps the member of largest
//                       |w| as its representative and the sum of all member
//                       weights (Sec. 3.1.2; the sum always includes every
//                       member, which is what preserves the trace, Sec. 2.1);
//       propagation() - extend each group by every forward/backward pair,
//                       multiply S and the influence factor, drop weights
//                       below theta (Sec. 2.1, path filtering), add the
//                       survivors to rho(t) (Sec. 3.2.1);
//     and for the original post-merging variant (Sec. 2.1, Scheme MACGIC):
//       propagation(), filtering, rho(t), then merging of the children that
//       agree on the mask.
//
// Readings of points the paper leaves open (each is listed with its reason
// in the design notes of the repository):
//   * a stored path holds dk_max points (lags 0..dk_max-1 of its newest
//     point); the new point couples to lags 0..dk_max;
//   * stored weights treat the newest point as interior; rho(t) multiplies
//     each survivor by the end-point correction exp(Phi_corr) that replaces
//     the interior coefficients of the final point by the half-window ones;
//   * the representative is the member with the largest quantised |w|^2
//     (low qbits mantissa bits cleared, |w|^2 = re*re + im*im without fused
//     multiply-add); ties go to the history that is smallest when read as a
//     number whose most significant digit is the oldest point;
//   * the filter drops a child when |w|^2 < theta^2 (theta = 0: no filter).
//
// Data layout: a path is a std::string of pair indices, h[j] = a*M+b at lag j
// (j = 0 is the newest point), plus a std::complex<double> weight.  Paths of
// one step all hold the same number of points, min(t+1, dk_max).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

typedef std::complex<double> cplx;

extern "C" {

typedef struct {
    int M;                 // number of system states
    const double* H;       // M*M complex, row-major, (re, im) interleaved
    const double* q;       // M coupling eigenvalues
    double dt;
    int K;                 // dk_max
    const double* eta;     // 3*(K+1) complex: eta_int, eta_half, eta_hh
    const int* mask;       // sorted lags, mask[0]=0, mask[1]=1; NULL -> all K lags
    int n_mask;
    double theta;
    const double* rho0;    // M*M complex
    int mode;              // 0: pre-merging, 1: post-merging
    int qbits;             // mantissa bits cleared in the quantised |w|^2
    double amb_eps;        // relative perturbation used to flag ambiguous decisions
} oracle_params;

typedef struct {
    long long n_groups;       // groups expanded at this step
    long long n_children;     // n_groups * M^2
    long long n_survivors;    // children that passed the filter
    long long n_stored;       // size of the stored set after the step
    long long n_amb_rep;      // representative choices that a perturbation of amb_eps could flip
    long long n_amb_theta;    // filter decisions within amb_eps of theta^2
    double dropped_abs;       // sum of |w| of the filtered children
    double theta_margin;      // min | |w|^2/theta^2 - 1 | over children (inf if theta = 0)
} oracle_stats;

}  // extern "C"

namespace {

struct Path {
    std::string h;   // pair index per lag, h[0] newest
    cplx w;
};

struct Group {
    Path rep;        // member of largest |w|
    cplx sum;        // sum of all member weights
    int n_members;
    bool amb;        // some member could have been chosen under a perturbation
};

struct Ctx {
    int M, P, K, mode, qbits;
    double dt, theta, theta2, amb_eps;
    std::vector<cplx> K4;        // K4[pn*P + po] = U[an][ao] * conj(U[bn][bo])
    std::vector<double> ds, ss;  // per pair: q_a - q_b, q_a + q_b
    std::vector<cplx> eta_int, eta_half, eta_hh;
    std::vector<int> mask;       // lags of the mask (POST key positions)
    std::vector<int> rmask;      // reduced mask {mask[i]-1 : i>=1} (PRE key positions)
    std::vector<cplx> rho0;
    int t;
    std::vector<Path> omega;     // PRE: survivors of the last step; POST: merged groups (w = sum)
    std::vector<std::vector<cplx>> rho_hist;
    std::vector<oracle_stats> stats_hist;
};

// ---------------------------------------------------------------- U = exp(-i H dt)
typedef std::vector<cplx> Mat;   // row-major n x n

Mat matmul(const Mat& A, const Mat& B, int n) {
    Mat C(n * n, cplx(0, 0));
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) C[i * n + j] += A[i * n + k] * B[k * n + j];
    return C;
}

// exp(A) = (sum_k (A/2^s)^k / k!)^(2^s), with 2^s >= ||A||_1 so the series converges fast.
Mat expm_series(const Mat& A, int n) {
    double norm = 0.0;
    for (int j = 0; j < n; ++j) {
        double col = 0.0;
        for (int i = 0; i < n; ++i) col += std::abs(A[i * n + j]);
        norm = std::max(norm, col);
    }
    int s = 0;
    while (norm > 0.5) { norm *= 0.5; ++s; }
    const double scale = std::ldexp(1.0, -s);
    Mat B(A);
    for (auto& x : B) x *= scale;
    Mat E(n * n, cplx(0, 0)), term(n * n, cplx(0, 0));
    for (int i = 0; i < n; ++i) { E[i * n + i] = 1.0; term[i * n + i] = 1.0; }
    for (int k = 1; k <= 40; ++k) {
        term = matmul(term, B, n);
        for (auto& x : term) x /= double(k);
        for (int i = 0; i < n * n; ++i) E[i] += term[i];
    }
    for (int i = 0; i < s; ++i) E = matmul(E, E, n);
    return E;
}

// ---------------------------------------------------------------- decisions
uint64_t quantised_norm2(cplx w, int qbits) {
    const double re = w.real(), im = w.imag();
    const double n2 = re * re + im * im;            // built with -ffp-contract=off
    uint64_t b;
    std::memcpy(&b, &n2, sizeof b);
    const uint64_t keep = qbits >= 64 ? 0 : ~((uint64_t(1) << qbits) - 1);
    return b & keep;
}

double norm2(cplx w) {
    const double re = w.real(), im = w.imag();
    return re * re + im * im;
}

uint64_t quantise_value(double n2, int qbits) {
    uint64_t b;
    std::memcpy(&b, &n2, sizeof b);
    const uint64_t keep = qbits >= 64 ? 0 : ~((uint64_t(1) << qbits) - 1);
    return b & keep;
}

// History order used for ties: compare from the oldest point to the newest.
bool history_less(const std::string& a, const std::string& b) {
    for (size_t j = a.size(); j-- > 0;) {
        const unsigned char x = (unsigned char)a[j], y = (unsigned char)b[j];
        if (x != y) return x < y;
    }
    return false;
}

// true when path c should replace the current representative r
bool better(const Path& c, const Path& r, int qbits) {
    const uint64_t qc = quantised_norm2(c.w, qbits), qr = quantised_norm2(r.w, qbits);
    if (qc != qr) return qc > qr;
    return history_less(c.h, r.h);
}

// Could a relative perturbation eps of the two |w|^2 values change which of
// them wins?  (The exact-tie case that stays a tie under the perturbation is
// decided by the history and is not ambiguous.)
bool could_flip(const cplx& winner, const cplx& other, int qbits, double eps) {
    const double vw = norm2(winner), vo = norm2(other);
    const uint64_t lw = quantise_value(vw * (1.0 - eps), qbits);
    const uint64_t hw = quantise_value(vw * (1.0 + eps), qbits);
    const uint64_t lo = quantise_value(vo * (1.0 - eps), qbits);
    const uint64_t ho = quantise_value(vo * (1.0 + eps), qbits);
    if (ho < lw) return false;                       // other stays strictly below
    if (lw == hw && lo == ho && lw == lo) return false;   // certain tie, broken by history
    return true;
}

std::string key_of(const std::string& h, const std::vector<int>& positions) {
    std::string k;
    for (int pos : positions)
        if (pos < (int)h.size()) k.push_back(h[pos]);
    return k;
}

// Group a set of paths on the given history positions (Sec. 3.1.2 for the
// reduced mask, Sec. 2.1 for the mask of the post-merging variant).
std::vector<Group> merge_on(const std::vector<Path>& paths, const std::vector<int>& positions,
                            int qbits) {
    std::unordered_map<std::string, size_t> index;
    std::vector<Group> groups;
    for (const Path& x : paths) {
        const std::string key = key_of(x.h, positions);
        auto it = index.find(key);
        if (it == index.end()) {
            index.emplace(key, groups.size());
            groups.push_back(Group{x, x.w, 1, false});
        } else {
            Group& g = groups[it->second];
            g.sum += x.w;
            g.n_members += 1;
            if (better(x, g.rep, qbits)) g.rep = x;
        }
    }
    return groups;
}

void flag_ambiguous(std::vector<Group>& groups, const std::vector<Path>& paths,
                    const std::vector<int>& positions, int qbits, double eps) {
    std::unordered_map<std::string, size_t> index;
    for (size_t i = 0; i < groups.size(); ++i) index.emplace(key_of(groups[i].rep.h, positions), i);
    for (const Path& x : paths) {
        Group& g = groups[index[key_of(x.h, positions)]];
        if (x.h == g.rep.h) continue;
        if (could_flip(g.rep.w, x.w, qbits, eps)) g.amb = true;
    }
}

// ---------------------------------------------------------------- one step
// Coefficient of the new point at time t paired with the point at lag d.
cplx coef(const Ctx& c, int d, int t) {
    if (d == t) return c.eta_half[d];        // partner is the time-0 point
    return c.eta_int[d];
}

// Difference between the final-point coefficient and the stored one.
cplx corr(const Ctx& c, int d, int t) {
    if (d == 0) return c.eta_half[0] - c.eta_int[0];
    if (d == t) return c.eta_hh[d] - c.eta_half[d];
    return c.eta_half[d] - c.eta_int[d];
}

// Extend one group (history h, amplitude W) at time t by every pair; filter;
// accumulate rho(t).  Children are appended to `out`.
void expand(Ctx& c, const std::string& h, cplx W, int t, std::vector<Path>& out,
            std::vector<cplx>& rho, oracle_stats& st) {
    const int dmax = std::min(t, c.K);
    for (int p = 0; p < c.P; ++p) {
        cplx phi(0, 0), phic(0, 0);
        for (int d = 0; d <= dmax; ++d) {
            const int x = (d == 0) ? p : (unsigned char)h[d - 1];
            const cplx cd = coef(c, d, t), dd = corr(c, d, t);
            phi += cplx(cd.real() * c.ds[x], cd.imag() * c.ss[x]);
            phic += cplx(dd.real() * c.ds[x], dd.imag() * c.ss[x]);
        }
        phi *= -c.ds[p];
        phic *= -c.ds[p];
        const cplx w = W * c.K4[p * c.P + (unsigned char)h[0]] * std::exp(phi);
        st.n_children += 1;
        if (c.theta > 0.0) {
            const double n2 = norm2(w);
            const double margin = std::fabs(n2 / c.theta2 - 1.0);
            st.theta_margin = std::min(st.theta_margin, margin);
            if (margin < c.amb_eps) st.n_amb_theta += 1;
            if (n2 < c.theta2) {
                st.dropped_abs += std::abs(w);
                continue;
            }
        }
        st.n_survivors += 1;
        rho[p] += w * std::exp(phic);
        Path child;
        child.h.push_back((char)p);
        const size_t keep = std::min(h.size(), (size_t)(c.K - 1));
        child.h.append(h, 0, keep);
        child.w = w;
        out.push_back(std::move(child));
    }
}

void do_step(Ctx& c) {
    const int t = c.t + 1;
    oracle_stats st;
    std::memset(&st, 0, sizeof st);
    st.theta_margin = INFINITY;
    std::vector<cplx> rho(c.P, cplx(0, 0));
    std::vector<Path> children;

    if (c.mode == 0) {
        // premerging() on the reduced mask, then propagation()
        std::vector<Group> groups = merge_on(c.omega, c.rmask, c.qbits);
        flag_ambiguous(groups, c.omega, c.rmask, c.qbits, c.amb_eps);
        for (const Group& g : groups) st.n_amb_rep += g.amb ? 1 : 0;
        st.n_groups = (long long)groups.size();
        for (const Group& g : groups) expand(c, g.rep.h, g.sum, t, children, rho, st);
        c.omega.swap(children);
    } else {
        // propagation() of the merged set, filtering, then merging on the mask
        st.n_groups = (long long)c.omega.size();
        for (const Path& g : c.omega) expand(c, g.h, g.w, t, children, rho, st);
        std::vector<Group> groups = merge_on(children, c.mask, c.qbits);
        flag_ambiguous(groups, children, c.mask, c.qbits, c.amb_eps);
        for (const Group& g : groups) st.n_amb_rep += g.amb ? 1 : 0;
        c.omega.clear();
        for (const Group& g : groups) c.omega.push_back(Path{g.rep.h, g.sum});
    }
    st.n_stored = (long long)c.omega.size();
    c.t = t;
    c.rho_hist.push_back(rho);
    c.stats_hist.push_back(st);
}

}  // namespace

extern "C" {

void* oracle_create(const oracle_params* p) {
    if (!p || p->M < 1 || p->K < 1 || p->dt <= 0.0 || p->theta < 0.0) return nullptr;
    Ctx* c = new Ctx();
    c->M = p->M;
    c->P = p->M * p->M;
    c->K = p->K;
    c->mode = p->mode;
    c->qbits = p->qbits;
    c->dt = p->dt;
    c->theta = p->theta;
    c->theta2 = p->theta * p->theta;
    c->amb_eps = p->amb_eps;
    const int M = c->M, P = c->P;

    // U = exp(-i H dt)  and  K4 of eq. SysP
    Mat A(M * M);
    for (int i = 0; i < M * M; ++i) A[i] = cplx(0, -p->dt) * cplx(p->H[2 * i], p->H[2 * i + 1]);
    const Mat U = expm_series(A, M);
    c->K4.assign(P * P, cplx(0, 0));
    for (int pn = 0; pn < P; ++pn)
        for (int po = 0; po < P; ++po) {
            const int an = pn / M, bn = pn % M, ao = po / M, bo = po % M;
            c->K4[pn * P + po] = U[an * M + ao] * std::conj(U[bn * M + bo]);
        }
    c->ds.resize(P);
    c->ss.resize(P);
    for (int pp = 0; pp < P; ++pp) {
        c->ds[pp] = p->q[pp / M] - p->q[pp % M];
        c->ss[pp] = p->q[pp / M] + p->q[pp % M];
    }
    const int n = p->K + 1;
    for (int d = 0; d < n; ++d) {
        c->eta_int.push_back(cplx(p->eta[2 * d], p->eta[2 * d + 1]));
        c->eta_half.push_back(cplx(p->eta[2 * (n + d)], p->eta[2 * (n + d) + 1]));
        c->eta_hh.push_back(cplx(p->eta[2 * (2 * n + d)], p->eta[2 * (2 * n + d) + 1]));
    }
    if (p->mask && p->n_mask > 0) c->mask.assign(p->mask, p->mask + p->n_mask);
    else for (int d = 0; d < p->K; ++d) c->mask.push_back(d);
    for (size_t i = 1; i < c->mask.size(); ++i) c->rmask.push_back(c->mask[i] - 1);
    for (int i = 0; i < M * M; ++i) c->rho0.push_back(cplx(p->rho0[2 * i], p->rho0[2 * i + 1]));

    // t = 0: one path per nonzero element of rho(0), carrying the self-term of
    // the initial point (half window)
    c->t = 0;
    const cplx e0 = c->eta_half[0];
    for (int pp = 0; pp < P; ++pp) {
        if (c->rho0[pp] == cplx(0, 0)) continue;
        const cplx phi = -c->ds[pp] * cplx(e0.real() * c->ds[pp], e0.imag() * c->ss[pp]);
        Path x;
        x.h.push_back((char)pp);
        x.w = c->rho0[pp] * std::exp(phi);
        c->omega.push_back(x);
    }
    c->rho_hist.push_back(c->rho0);
    oracle_stats st0;
    std::memset(&st0, 0, sizeof st0);
    st0.n_stored = (long long)c->omega.size();
    st0.theta_margin = INFINITY;
    c->stats_hist.push_back(st0);
    return c;
}

int oracle_step(void* h, int n) {
    Ctx* c = (Ctx*)h;
    if (!c || n < 0) return -1;
    for (int i = 0; i < n; ++i) do_step(*c);
    return 0;
}

int oracle_time(void* h) { return h ? ((Ctx*)h)->t : -1; }

int oracle_rho(void* h, int t, double* out) {
    Ctx* c = (Ctx*)h;
    if (!c || t < 0 || t > c->t) return -1;
    for (int i = 0; i < c->P; ++i) {
        out[2 * i] = c->rho_hist[t][i].real();
        out[2 * i + 1] = c->rho_hist[t][i].imag();
    }
    return 0;
}

int oracle_stats_at(void* h, int t, oracle_stats* out) {
    Ctx* c = (Ctx*)h;
    if (!c || t < 0 || t > c->t) return -1;
    *out = c->stats_hist[t];
    return 0;
}

// The groups that the next step expands (PRE: the pre-merge of the stored
// survivors; POST: the stored merged set), as histories (n x K bytes, lags
// beyond the held points set to 0) and amplitudes (n complex).  Returns the
// number of groups; writes at most `cap`.
long long oracle_groups(void* h, unsigned char* hist, double* w, long long cap) {
    Ctx* c = (Ctx*)h;
    if (!c) return -1;
    std::vector<Path> g;
    if (c->mode == 0) {
        for (const Group& x : merge_on(c->omega, c->rmask, c->qbits)) g.push_back(Path{x.rep.h, x.sum});
    } else {
        g = c->omega;
    }
    const long long n = (long long)g.size();
    for (long long i = 0; i < std::min(n, cap); ++i) {
        for (int j = 0; j < c->K; ++j)
            hist[i * c->K + j] = j < (int)g[i].h.size() ? (unsigned char)g[i].h[j] : 0;
        w[2 * i] = g[i].w.real();
        w[2 * i + 1] = g[i].w.imag();
    }
    return n;
}

// Stored set itself (PRE: survivors; POST: merged groups).
long long oracle_stored(void* h, unsigned char* hist, double* w, long long cap) {
    Ctx* c = (Ctx*)h;
    if (!c) return -1;
    const long long n = (long long)c->omega.size();
    for (long long i = 0; i < std::min(n, cap); ++i) {
        for (int j = 0; j < c->K; ++j)
            hist[i * c->K + j] = j < (int)c->omega[i].h.size() ? (unsigned char)c->omega[i].h[j] : 0;
        w[2 * i] = c->omega[i].w.real();
        w[2 * i + 1] = c->omega[i].w.imag();
    }
    return n;
}

void oracle_destroy(void* h) { delete (Ctx*)h; }

// U = exp(-i H dt) as the oracle computes it (M*M complex, row-major).
int oracle_propagator(int M, const double* H, double dt, double* U_out) {
    if (M < 1) return -1;
    Mat A(M * M);
    for (int i = 0; i < M * M; ++i) A[i] = cplx(0, -dt) * cplx(H[2 * i], H[2 * i + 1]);
    const Mat U = expm_series(A, M);
    for (int i = 0; i < M * M; ++i) { U_out[2 * i] = U[i].real(); U_out[2 * i + 1] = U[i].imag(); }
    return 0;
}

// Merge an explicit set of paths on the given positions (for unit tests of
// the merge rule).  hist: n x L bytes; w: n complex.  Writes, per group in
// order of first appearance, the representative's index and the sum.
int oracle_merge_demo(const unsigned char* hist, const double* w, int n, int L,
                      const int* positions, int n_pos, int qbits,
                      int* rep_index, double* sums) {
    std::vector<Path> paths(n);
    for (int i = 0; i < n; ++i) {
        paths[i].h.assign((const char*)hist + (size_t)i * L, L);
        paths[i].w = cplx(w[2 * i], w[2 * i + 1]);
    }
    std::vector<int> pos(positions, positions + n_pos);
    std::vector<Group> groups = merge_on(paths, pos, qbits);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        int idx = -1;
        for (int i = 0; i < n; ++i)
            if (paths[i].h == groups[gi].rep.h) { idx = i; break; }
        rep_index[gi] = idx;
        sums[2 * gi] = groups[gi].sum.real();
        sums[2 * gi + 1] = groups[gi].sum.imag();
    }
    return (int)groups.size();
}

}  // extern "C"

extern "C" {

// Test hooks of the decision log (Sec. 3.1.2 representative choice, with the
// quantised comparison and tie rule of the header).  could_flip for two
// amplitudes given as (re, im) pairs; returns 1 when a relative perturbation
// eps of the two |w|^2 could change which one wins.
int oracle_could_flip(const double* winner, const double* other, int qbits, double eps) {
    return could_flip(cplx(winner[0], winner[1]), cplx(other[0], other[1]), qbits, eps) ? 1 : 0;
}

// Merge explicit paths on the given positions and flag the groups whose
// representative choice a perturbation eps could flip.  Writes, per group in
// order of first appearance, the representative's index and the flag (0/1);
// returns the number of groups.
int oracle_flag_demo(const unsigned char* hist, const double* w, int n, int L, const int* positions,
                     int n_pos, int qbits, double eps, int* rep_index, int* amb) {
    std::vector<Path> paths(n);
    for (int i = 0; i < n; ++i) {
        paths[i].h.assign((const char*)hist + (size_t)i * L, L);
        paths[i].w = cplx(w[2 * i], w[2 * i + 1]);
    }
    std::vector<int> pos(positions, positions + n_pos);
    std::vector<Group> groups = merge_on(paths, pos, qbits);
    flag_ambiguous(groups, paths, pos, qbits, eps);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        int idx = -1;
        for (int i = 0; i < n; ++i)
            if (paths[i].h == groups[gi].rep.h) { idx = i; break; }
        rep_index[gi] = idx;
        amb[gi] = groups[gi].amb ? 1 : 0;
    }
    return (int)groups.size();
}

}  // extern "C"
