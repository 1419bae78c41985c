// Sanitizer run of the library's host paths (AddressSanitizer +
// UndefinedBehaviorSanitizer on the host code only; device code is built as
// usual and never launched here): the host tables (propagator, eta quadrature),
// the argument validation of every create call, the error strings, and the
// null-context guards of the stepping, reading and network calls.  On a host
// without a GPU a valid create returns an error code; on a GPU host it makes a
// context, which is destroyed at once.  Exits 0 when every call returns as
// documented; any sanitizer report aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "quapi.h"
#include "quapi_mlp.h"

namespace {

int n_fail = 0;

void expect(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "library_host_driver: %s\n", what);
        ++n_fail;
    }
}

struct Case {
    std::vector<quapi_c64> H, eta, rho0;
    std::vector<double> q;
    std::vector<int> mask;
    quapi_params p{};

    Case(int M, int K) : H((size_t)M * M), eta(3 * (size_t)(K + 1)), rho0((size_t)M * M), q(M) {
        for (int i = 0; i < M; ++i) {
            q[i] = 1.0 - 2.0 * i / (M > 1 ? M - 1 : 1);
            H[(size_t)i * M + i] = {0.25 * (i ? -1 : 1), 0.0};
            if (i + 1 < M) {
                H[(size_t)i * M + i + 1] = {0.5, 0.0};
                H[(size_t)(i + 1) * M + i] = {0.5, 0.0};
            }
        }
        rho0[0] = {1.0, 0.0};
        for (size_t k = 0; k < eta.size(); ++k) eta[k] = {0.01 / (1.0 + (double)k), -0.002};
        for (int d = 0; d < K / 2; ++d) mask.push_back(d);
        p.M = M;
        p.H = H.data();
        p.q = q.data();
        p.dt = 0.2;
        p.dk_max = K;
        p.eta = eta.data();
        p.mask = mask.data();
        p.n_mask = (int)mask.size();
        p.theta = 1e-8;
        p.rho0 = rho0.data();
        p.mode = QUAPI_PRE;
        p.qbits = -1;
        p.max_groups = 0;
        p.max_steps = 16;
        p.stream = nullptr;
        p.precision = QUAPI_FP64;
    }
};

int create(const quapi_params& p) {
    quapi_ctx* c = reinterpret_cast<quapi_ctx*>(&n_fail);   // must be overwritten
    const int rc = quapi_create(&p, &c);
    if (rc != QUAPI_OK) expect(c == nullptr, "failed create leaves *out set");
    else quapi_destroy(c);
    return rc;
}

}  // namespace

int main() {
    // error strings
    for (int code = 1; code >= -6; --code) expect(quapi_strerror(code) != nullptr, "strerror");

    // host tables
    {
        Case c(2, 24);
        quapi_c64 U[4];
        expect(quapi_propagator(2, c.H.data(), 0.2, U) == QUAPI_OK, "propagator");
        const double n0 = U[0].re * U[0].re + U[0].im * U[0].im + U[2].re * U[2].re + U[2].im * U[2].im;
        expect(std::fabs(n0 - 1.0) < 1e-13, "propagator column norm");
        quapi_c64 bad[4] = {{0, 0}, {1, 0}, {0.5, 0}, {0, 0}};
        expect(quapi_propagator(2, bad, 0.2, U) == QUAPI_EINVAL, "non-Hermitian propagator");
        expect(quapi_propagator(9, c.H.data(), 0.2, U) == QUAPI_EINVAL, "propagator M range");
        const double peaks[3] = {1.0, 0.05, 0.1};
        quapi_bath b{0.05, 5.0, 1, peaks};
        std::vector<quapi_c64> eta(3 * 25);
        expect(quapi_eta(&b, 5.0, 0.2, 24, eta.data()) == QUAPI_OK, "eta");
        for (const auto& z : eta) expect(std::isfinite(z.re) && std::isfinite(z.im), "eta finite");
        quapi_bath nb{-1.0, 5.0, 0, nullptr};
        expect(quapi_eta(&nb, 5.0, 0.2, 24, eta.data()) == QUAPI_EINVAL, "eta negative alpha");
        expect(quapi_eta(&b, 0.0, 0.2, 24, eta.data()) == QUAPI_EINVAL, "eta beta");
        expect(quapi_eta(&b, 5.0, 0.2, 65, eta.data()) == QUAPI_EINVAL, "eta dk_max");
        expect(quapi_eta(nullptr, 5.0, 0.2, 24, eta.data()) == QUAPI_EINVAL, "eta null bath");
    }

    // argument validation of create
    {
        expect(quapi_create(nullptr, nullptr) == QUAPI_EINVAL, "null create");
        quapi_ctx* out = nullptr;
        expect(quapi_create(nullptr, &out) == QUAPI_EINVAL && out == nullptr, "null params");
        Case c(2, 12);
        quapi_params p = c.p;
        p.M = 1;
        expect(create(p) == QUAPI_EINVAL, "M = 1");
        p = c.p;
        p.dk_max = 0;
        expect(create(p) == QUAPI_EINVAL, "dk_max = 0");
        p = c.p;
        p.dt = -0.1;
        expect(create(p) == QUAPI_EINVAL, "dt < 0");
        p = c.p;
        p.theta = -1.0;
        expect(create(p) == QUAPI_EINVAL, "theta < 0");
        p = c.p;
        p.mode = 7;
        expect(create(p) == QUAPI_EINVAL, "mode");
        p = c.p;
        p.precision = 3;
        expect(create(p) == QUAPI_EINVAL, "precision");
        std::vector<int> bad_mask = {0, 2, 3};
        p = c.p;
        p.mask = bad_mask.data();
        p.n_mask = 3;
        expect(create(p) == QUAPI_EINVAL, "mask without lag 1");
        std::vector<int> long_mask = {0, 1, 12};
        p.mask = long_mask.data();
        expect(create(p) == QUAPI_EINVAL, "mask lag >= K");
        p = c.p;
        std::vector<quapi_c64> Hn = c.H;
        Hn[1] = {0.7, 0.0};
        p.H = Hn.data();
        expect(create(p) == QUAPI_EINVAL, "non-Hermitian H");
        p = c.p;
        std::vector<quapi_c64> en = c.eta;
        en[3].re = NAN;
        p.eta = en.data();
        expect(create(p) == QUAPI_EINVAL, "NaN eta");
        Case c5(5, 6);
        expect(create(c5.p) == QUAPI_EUNSUPPORTED, "M = 5");
        Case c4(4, 6);
        c4.p.merge = QUAPI_MERGE_BUCKETED;
        expect(create(c4.p) == QUAPI_EUNSUPPORTED, "M = 4 on the bucketed store");
        Case c3(3, 40);
        c3.mask.assign({0, 1, 20});
        c3.p.mask = c3.mask.data();
        c3.p.n_mask = 3;
        expect(create(c3.p) == QUAPI_EUNSUPPORTED, "three levels, history over 128 bits");
        // phases beyond the range of the kernels' sine and cosine
        Case cp(2, 8);
        for (auto& z : cp.eta) z.im = 1e4;
        expect(create(cp.p) == QUAPI_EUNSUPPORTED, "phase bound");
        // batched create
        quapi_ctx* bo = nullptr;
        expect(quapi_create_batch(&c.p, 0, c.eta.data(), nullptr, &bo) == QUAPI_EINVAL && !bo, "batch n = 0");
        expect(quapi_create_batch(&c.p, 1025, c.eta.data(), nullptr, &bo) == QUAPI_EINVAL, "batch n > 1024");
        expect(quapi_create_batch(&c.p, 2, nullptr, nullptr, &bo) == QUAPI_EINVAL, "batch null eta");
        // a valid create: an error code without a GPU, a context with one
        const int rc = create(c.p);
        expect(rc == QUAPI_OK || rc == QUAPI_EDEVICE || rc == QUAPI_ENOMEM, "valid create");
    }

    // null-context guards
    {
        quapi_c64 r[4];
        quapi_stepstat_t st;
        quapi_info_t info;
        long long n = 0;
        int t = 0, run = 0;
        double ms[2];
        expect(quapi_step(nullptr, 1) == QUAPI_EINVAL, "step null");
        expect(quapi_step_graph(nullptr, 1) == QUAPI_EINVAL, "step_graph null");
        expect(quapi_sync(nullptr) == QUAPI_EINVAL, "sync null");
        expect(quapi_time(nullptr, &t) == QUAPI_EINVAL, "time null");
        expect(quapi_rho(nullptr, 0, r) == QUAPI_EINVAL, "rho null");
        expect(quapi_rho_history(nullptr, 0, 1, r) == QUAPI_EINVAL, "rho_history null");
        expect(quapi_step_stats(nullptr, 1, 1, &st) == QUAPI_EINVAL, "step_stats null");
        expect(quapi_groups(nullptr, 0, nullptr, nullptr, &n) == QUAPI_EINVAL, "groups null");
        expect(quapi_batch_rho_all(nullptr, 0, 1, r) == QUAPI_EINVAL, "rho_all null");
        expect(quapi_set_chunk_run(nullptr, 1) == QUAPI_EINVAL, "chunk_run null");
        expect(quapi_autotune(nullptr, 1, &run) == QUAPI_EINVAL, "autotune null");
        expect(quapi_reset(nullptr) == QUAPI_EINVAL, "reset null");
        expect(quapi_info(nullptr, &info) == QUAPI_EINVAL, "info null");
        expect(quapi_stream(nullptr) == nullptr, "stream null");
        expect(quapi_profile_begin(nullptr, 1) == QUAPI_EINVAL, "profile_begin null");
        expect(quapi_profile_end(nullptr, 2, ms, ms, &t) == QUAPI_EINVAL, "profile_end null");
        quapi_destroy(nullptr);
    }

    // network calls
    {
        quapi_mlp* m = nullptr;
        expect(quapi_mlp_create(0, 256, 4, 4, 64, 1ull, nullptr, &m) != 0 && m == nullptr, "mlp bad shape");
        long long np = 0;
        expect(quapi_mlp_n_params(nullptr, &np) != 0, "mlp null");
        expect(quapi_mlp_forward(nullptr, nullptr, 1, nullptr) != 0, "mlp forward null");
        quapi_mlp_destroy(nullptr);
    }

    std::printf("library_host_driver: %s\n", n_fail ? "FAILED" : "ok");
    return n_fail ? 1 : 0;
}
