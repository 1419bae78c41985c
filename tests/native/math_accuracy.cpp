// Accuracy of the library's reduced-argument FP64 exp and sincos, and of the
// FP32 sincos of the precision form (the host build of the same inline
// functions the kernels use) against the C library,
// which is within one ulp of the correctly rounded value: the largest error in
// ulps over seeded random arguments spanning the reduced range, and the
// quadrant signs.  Prints the maxima; exits non-zero above the bound.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "quapi_device.h"

namespace {

double ulp_diff(double a, double b) {
    if (a == b) return 0.0;
    const double u = std::nextafter(std::fabs(b), INFINITY) - std::fabs(b);
    return std::fabs(a - b) / u;
}

uint64_t state = 0x1234567ull;
double uniform(double lo, double hi) {    // SplitMix64 draws
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return lo + (hi - lo) * (double)(z >> 11) * 0x1.0p-53;
}

}  // namespace

int main() {
    double e_exp = 0, e_sin = 0, e_cos = 0;
    for (int i = 0; i < 2000000; ++i) {
        const double span = (i % 4 == 0) ? 1.0 : (i % 4 == 1) ? 20.0 : (i % 4 == 2) ? 690.0 : 1e5;
        const double x = uniform(-span, span);
        if (std::fabs(x) < 700.0) e_exp = std::fmax(e_exp, ulp_diff(quapi_dev::exp_fast(x), std::exp(x)));
        double s, c;
        if (std::fabs(x) < quapi_dev::kTrigArgMax) {
            quapi_dev::sincos_reduced(x, s, c);
            // the sin/cos error is measured against the larger of |value| and 1e-3
            // (absolute near the zeros, where any reduced form loses relative accuracy)
            const double rs = std::sin(x), rc = std::cos(x);
            e_sin = std::fmax(e_sin, ulp_diff(s, rs) * std::fmin(1.0, std::fabs(rs) / 1e-3 + 1e-300));
            e_cos = std::fmax(e_cos, ulp_diff(c, rc) * std::fmin(1.0, std::fabs(rc) / 1e-3 + 1e-300));
        }
    }
    int bad = 0;
    // exact points and quadrant signs
    const double pts[] = {0.0, 1e-300, -1e-300, 0.5, -0.5, 1.5707963267948966, 3.141592653589793,
                          -3.141592653589793, 4.71238898038469, 100.0, -100.0};
    for (double x : pts) {
        double s, c;
        quapi_dev::sincos_reduced(x, s, c);
        if (std::fabs(s - std::sin(x)) > 4e-16 * (1 + std::fabs(x)) || std::fabs(c - std::cos(x)) > 4e-16 * (1 + std::fabs(x))) {
            std::printf("sincos(%g) = (%.17g, %.17g) vs (%.17g, %.17g)\n", x, s, c, std::sin(x), std::cos(x));
            ++bad;
        }
    }
    if (quapi_dev::exp_fast(0.0) != 1.0) ++bad;
    // the clamped tails: zero below the subnormal range, infinity above the largest finite value
    if (quapi_dev::exp_fast(-800.0) != 0.0 || quapi_dev::exp_fast(-1e30) != 0.0) ++bad;
    if (!std::isinf(quapi_dev::exp_fast(720.0)) || !std::isinf(quapi_dev::exp_fast(1e30))) ++bad;
    if (std::fabs(quapi_dev::exp_fast(709.0) / std::exp(709.0) - 1.0) > 1e-15) ++bad;
    if (std::fabs(quapi_dev::exp_fast(-707.0) / std::exp(-707.0) - 1.0) > 1e-15) ++bad;
    std::printf("max ulp: exp %.2f  sin %.2f  cos %.2f\n", e_exp, e_sin, e_cos);
    if (e_exp > 4.0 || e_sin > 4.0 || e_cos > 4.0) ++bad;
    // the precision form's FP32 sincos: error in units of 2^-24 times the larger of
    // |value| and 1e-3, against the FP64 value of the same FP32 argument
    double f_sin = 0, f_cos = 0;
    for (int i = 0; i < 2000000; ++i) {
        const double span = (i % 3 == 0) ? 3.2 : (i % 3 == 1) ? 100.0 : 0.99e5;
        const float x = (float)uniform(-span, span);
        float s, c;
        quapi_dev::sincos_f32(x, s, c);
        const double rs = std::sin((double)x), rc = std::cos((double)x);
        f_sin = std::fmax(f_sin, std::fabs((double)s - rs) / std::fmax(std::fabs(rs), 1e-3) * 0x1.0p24);
        f_cos = std::fmax(f_cos, std::fabs((double)c - rc) / std::fmax(std::fabs(rc), 1e-3) * 0x1.0p24);
    }
    std::printf("FP32 sincos, max error in 2^-24 relative units: sin %.2f  cos %.2f\n", f_sin, f_cos);
    if (f_sin > 8.0 || f_cos > 8.0) ++bad;
    return bad ? 1 : 0;
}
