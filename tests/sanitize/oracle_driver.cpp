// Sanitizer run of the oracle (AddressSanitizer + UndefinedBehaviorSanitizer,
// host only): builds the oracle source into this program and drives every
// exported entry point on small cases -- both merging orders, a mask, a
// filter, three levels, the dumps and the decision-log hooks.  Exits 0 when
// every call returns as documented; any sanitizer report aborts the run.
#include "../../oracle/quapi_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

int fail(const char* what) {
    std::fprintf(stderr, "oracle_driver: %s\n", what);
    return 1;
}

int run(int M, int K, int mode, const std::vector<int>& mask, double theta, int steps) {
    const int P = M * M;
    std::vector<double> H(2 * M * M, 0.0), q(M), rho0(2 * P, 0.0), eta(2 * 3 * (K + 1));
    for (int i = 0; i < M; ++i) {
        q[i] = 1.0 - 2.0 * i / (M - 1);
        H[2 * (i * M + i)] = 0.3 * i;
        if (i + 1 < M) {
            H[2 * (i * M + i + 1)] = 0.5;
            H[2 * ((i + 1) * M + i)] = 0.5;
        }
    }
    rho0[0] = 1.0;
    for (int k = 0; k < 3 * (K + 1); ++k) {
        eta[2 * k] = 0.02 / (1 + k % (K + 1));
        eta[2 * k + 1] = -0.01 / (1 + k % (K + 1));
    }
    oracle_params p{};
    p.M = M;
    p.H = H.data();
    p.q = q.data();
    p.dt = 0.2;
    p.K = K;
    p.eta = eta.data();
    p.mask = mask.empty() ? nullptr : mask.data();
    p.n_mask = (int)mask.size();
    p.theta = theta;
    p.rho0 = rho0.data();
    p.mode = mode;
    p.qbits = 32;
    p.amb_eps = 1e-12;
    void* o = oracle_create(&p);
    if (!o) return fail("oracle_create");
    if (oracle_step(o, steps) != 0) return fail("oracle_step");
    if (oracle_time(o) != steps) return fail("oracle_time");
    std::vector<double> r(2 * P);
    oracle_stats st;
    for (int t = 0; t <= steps; ++t) {
        if (oracle_rho(o, t, r.data()) != 0) return fail("oracle_rho");
        if (oracle_stats_at(o, t, &st) != 0) return fail("oracle_stats_at");
    }
    if (oracle_rho(o, steps + 1, r.data()) == 0) return fail("rho past the end accepted");
    const long long n = oracle_groups(o, nullptr, nullptr, 0);
    std::vector<unsigned char> hist((size_t)(n > 0 ? n : 1) * K);
    std::vector<double> w(2 * (size_t)(n > 0 ? n : 1));
    if (oracle_groups(o, hist.data(), w.data(), n) != n) return fail("oracle_groups");
    const long long ns = oracle_stored(o, nullptr, nullptr, 0);
    hist.resize((size_t)(ns > 0 ? ns : 1) * K);
    w.resize(2 * (size_t)(ns > 0 ? ns : 1));
    if (oracle_stored(o, hist.data(), w.data(), ns) != ns) return fail("oracle_stored");
    oracle_destroy(o);
    return 0;
}

}  // namespace

int main() {
    int rc = 0;
    rc |= run(2, 6, 0, {0, 1, 2, 3}, 1e-6, 20);
    rc |= run(2, 6, 1, {0, 1, 2, 3}, 0.0, 12);
    rc |= run(2, 5, 1, {}, 0.0, 8);
    rc |= run(3, 4, 0, {0, 1, 2}, 1e-7, 10);
    rc |= run(2, 8, 0, {0, 1, 2, 5}, 1e-6, 16);
    // decision-log hooks and the merge demo
    const unsigned char hist[6 * 2] = {0, 1, 0, 2, 0, 3, 1, 1, 1, 0, 2, 0};
    const double w[12] = {1.0, 0.0, 0.999, 0.0, 0.5, 0.0, 0.7, 0.1, 0.7, 0.1, 0.3, 0.0};
    const int pos[1] = {0};
    int rep[6], amb[6];
    double sums[12];
    if (oracle_flag_demo(hist, w, 6, 2, pos, 1, 32, 1e-12, rep, amb) != 3) rc |= fail("flag_demo");
    if (oracle_merge_demo(hist, w, 6, 2, pos, 1, 32, rep, sums) != 3) rc |= fail("merge_demo");
    const double a[2] = {1.0, 0.5}, b[2] = {0.5, 1.0};
    (void)oracle_could_flip(a, b, 32, 1e-12);
    double U[8];
    const double H2[8] = {0.25, 0, 0.5, 0, 0.5, 0, -0.25, 0};
    if (oracle_propagator(2, H2, 0.2, U) != 0) rc |= fail("propagator");
    if (oracle_create(nullptr) != nullptr) rc |= fail("null params accepted");
    std::printf("oracle_driver: %s\n", rc ? "FAILED" : "ok");
    return rc;
}
