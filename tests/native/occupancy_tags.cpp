// The direct-mapped store's occupancy protocol, run on the host with the
// library's own tag and clear schedule (dense_tag, dense_clear_due): two byte
// buffers; step t writes the tag of t at its occupied slots of buffer t & 1 and
// leaves every other byte as it was; the planner after step t counts the bytes
// of buffer t & 1 equal to the tag of t and, when the schedule says so, zeroes
// buffer (t + 1) & 1 before step t + 1 writes it.  Over seeded random
// occupancies (per-slot rates from 1/1000 to 1/2, so that some slots stay empty
// for hundreds of steps) the counted slots must be exactly the occupied ones at
// every step.  A schedule that never clears must fail the same check (a stale
// tag 510 steps old is counted), which shows the check can fail.
#include <cstdint>
#include <cstdio>
#include <functional>
#include <vector>

#include "quapi_dense.h"

namespace {

uint64_t state = 0x2545F4914F6CDD1Dull;
double uniform01() {    // SplitMix64 draws
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

// number of steps at which the counted set differed from the occupied set
long long run(const std::function<int(int)>& clear_due, int n_slots, int n_steps) {
    state = 0x2545F4914F6CDD1Dull;
    std::vector<double> rate(n_slots);
    for (int s = 0; s < n_slots; ++s) rate[s] = 0.001 + (0.5 - 0.001) * (double)s / (n_slots - 1);
    std::vector<unsigned char> buf[2] = {std::vector<unsigned char>(n_slots, 0u),
                                         std::vector<unsigned char>(n_slots, 0u)};
    std::vector<char> occ(n_slots);
    for (int s = 0; s < n_slots; ++s) {
        occ[s] = uniform01() < 0.5;
        if (occ[s]) buf[0][s] = (unsigned char)quapi_dev::dense_tag(0);
    }
    long long bad = 0;
    for (int t = 0;; ++t) {
        // planner after step t
        const unsigned char tag = (unsigned char)quapi_dev::dense_tag(t);
        bool ok = true;
        for (int s = 0; s < n_slots; ++s) ok &= (buf[t & 1][s] == tag) == (bool)occ[s];
        bad += !ok;
        if (t == n_steps) break;
        if (clear_due(t)) std::fill(buf[(t + 1) & 1].begin(), buf[(t + 1) & 1].end(), 0u);
        // step t + 1
        const unsigned char next = (unsigned char)quapi_dev::dense_tag(t + 1);
        for (int s = 0; s < n_slots; ++s) {
            occ[s] = uniform01() < rate[s];
            if (occ[s]) buf[(t + 1) & 1][s] = next;
        }
    }
    return bad;
}

}  // namespace

int main() {
    const int n_slots = 512, n_steps = 5000;
    const long long lib = run([](int t) { return quapi_dev::dense_clear_due(t); }, n_slots, n_steps);
    const long long never = run([](int) { return 0; }, n_slots, n_steps);
    int cleared_even = 0, cleared_odd = 0, max_gap[2] = {0, 0}, last[2] = {0, 0};
    for (int t = 0; t < n_steps; ++t)
        if (quapi_dev::dense_clear_due(t)) {
            const int b = (t + 1) & 1;
            (b ? cleared_odd : cleared_even)++;
            if (t + 1 - last[b] > max_gap[b]) max_gap[b] = t + 1 - last[b];
            last[b] = t + 1;
        }
    std::printf("steps with a wrong count: library schedule %lld, never clearing %lld\n", lib, never);
    std::printf("clears: buffer 0 %d, buffer 1 %d; longest gap %d and %d steps\n", cleared_even, cleared_odd,
                max_gap[0], max_gap[1]);
    const bool ok = lib == 0 && never > 0 && cleared_even > 0 && cleared_odd > 0 && max_gap[0] < 510 &&
                    max_gap[1] < 510;
    return ok ? 0 : 1;
}
