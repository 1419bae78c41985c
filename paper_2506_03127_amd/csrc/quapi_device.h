// Device helpers shared by the HIP kernels of the library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace quapi_dev {

__device__ inline double norm2_nocontract(double re, double im) {
#pragma clang fp contract(off)
    const double a = re * re;
    const double b = im * im;
    return a + b;
}

__device__ inline unsigned int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ inline unsigned int rank_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned int)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned int)mask, 0u));
}

// 1/x from the hardware estimate and two Newton steps
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Sum over the 64 lanes of a wave, in a fixed order, returned to every lane:
// butterflies inside each row of 16 lanes by DPP (quad_perm xor 1, xor 2,
// half-row mirror, row mirror), then the four row sums read from lanes 0, 16,
// 32, 48.
template <int CTRL>
__device__ inline double dpp_pair(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane_d(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

__device__ inline double wave_sum(double v) {
    v += dpp_pair<0xB1>(v);      // quad_perm [1,0,3,2]
    v += dpp_pair<0x4E>(v);      // quad_perm [2,3,0,1]
    v += dpp_pair<0x141>(v);     // row_half_mirror
    v += dpp_pair<0x140>(v);     // row_mirror
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Eight per-lane values reduced over the lanes of each row of 16, four rows
// per wave, in a fixed order: two butterfly levels (partners lane^1, lane^2)
// that each keep half of the values, then a shift-add scan by 4 and 8 lanes
// inside the row.  Afterwards lane 12 + r of a row holds the row sums of
// values 4*(r&1) + 2*(r>>1) + {0, 1}.
__device__ inline double dpp_sel_xor(double keep, double send, int level) {
    return keep + (level == 1 ? dpp_pair<0xB1>(send) : dpp_pair<0x4E>(send));
}

__device__ inline void row_sums8(const double (&v)[8], unsigned int lane, double& x0, double& x1) {
    const bool h1 = lane & 1u, h2 = (lane >> 1) & 1u;
    double u[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = dpp_sel_xor(h1 ? v[4 + j] : v[j], h1 ? v[j] : v[4 + j], 1);
    double x[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) x[j] = dpp_sel_xor(h2 ? u[2 + j] : u[j], h2 ? u[j] : u[2 + j], 2);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        x[j] += dpp_pair<0x114>(x[j]);   // row_shr:4 (lanes 0..3 of a row add 0)
        x[j] += dpp_pair<0x118>(x[j]);   // row_shr:8
    }
    x0 = x[0];
    x1 = x[1];
}

__device__ inline unsigned long long ld_relaxed(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void st_relaxed(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- FP64 exp and sincos
// The influence factors need exp and sin/cos of one FP64 argument per child
// pair.  The general library sin/cos also carries the reduction for huge
// arguments (Payne-Hanek), which the compiler evaluates beside the common path
// when it turns their branch into selects.  These use Cody-Waite reduction and
// truncated Taylor series instead, each within a few ulp of the correctly
// rounded value: exp for every argument (clamped where the result under- or
// overflows anyway), sin/cos for |y| < kTrigArgMax.  The host checks before a
// run that no phase the coefficient table can produce reaches that bound.
//
// Split constants: ln 2 = kLn2Hi + kLn2Lo and pi/2 = kPio2A + kPio2B + kPio2C,
// each leading part holding at most 33 significant bits, so that k times it is
// exact for the k these arguments take.
constexpr double kLog2e = 1.4426950408889634;           // 1 / ln 2
constexpr double kLn2Hi = 0.69314718060195446;          // 0x3fe62e42ff000000
constexpr double kLn2Lo = -4.2009150726810846e-11;      // ln 2 - kLn2Hi
constexpr double kTwoOverPi = 0.63661977236758138;
constexpr double kPio2A = 1.5707963267341256;           // 0x3ff921fb54400000
constexpr double kPio2B = 6.077100506303966e-11;        // 0x3dd0b4611a600000
constexpr double kPio2C = 2.0222662487959506e-21;       // pi/2 - kPio2A - kPio2B
constexpr double kTrigArgMax = 1.0e5;                   // sincos_fast: |y| below this

// exp(r) for |r| <= ln2/2 by its Taylor series through r^13 (the next term is
// below 1e-17 relative there), coefficients 1/n!.
__host__ __device__ inline double exp_poly(double r) {
    double p = 1.0 / 6227020800.0;                       // 1/13!
    p = __builtin_fma(p, r, 1.0 / 479001600.0);
    p = __builtin_fma(p, r, 1.0 / 39916800.0);
    p = __builtin_fma(p, r, 1.0 / 3628800.0);
    p = __builtin_fma(p, r, 1.0 / 362880.0);
    p = __builtin_fma(p, r, 1.0 / 40320.0);
    p = __builtin_fma(p, r, 1.0 / 5040.0);
    p = __builtin_fma(p, r, 1.0 / 720.0);
    p = __builtin_fma(p, r, 1.0 / 120.0);
    p = __builtin_fma(p, r, 1.0 / 24.0);
    p = __builtin_fma(p, r, 1.0 / 6.0);
    p = __builtin_fma(p, r, 0.5);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_fma(p, r, 1.0);
}

// exp(x) = 2^k exp(r), k = rint(x / ln 2), r = x - k ln 2 (Cody-Waite).
__host__ __device__ inline double exp_reduced(double x) {
    const double k = __builtin_rint(x * kLog2e);
    double r = __builtin_fma(-k, kLn2Hi, x);
    r = __builtin_fma(-k, kLn2Lo, r);
    return __builtin_ldexp(exp_poly(r), (int)k);
}

// exp for any argument: below -746 the result is zero and above 710 infinite,
// which the clamped arguments still give
__host__ __device__ inline double exp_fast(double x) {
    return exp_reduced(__builtin_fmin(__builtin_fmax(x, -746.0), 710.0));
}

// sin and cos of r, |r| <= pi/4: Taylor series through r^17 and r^16 (the next
// terms are below 1e-17 relative), Horner in z = r^2, coefficients 1/n!.
__host__ __device__ inline void sincos_poly(double r, double& sn, double& cs) {
    const double z = r * r;
    double ps = -1.0 / 355687428096000.0;                // -1/17!  (times r^17)
    ps = __builtin_fma(ps, z, 1.0 / 1307674368000.0);    //  1/15!
    ps = __builtin_fma(ps, z, -1.0 / 6227020800.0);      // -1/13!
    ps = __builtin_fma(ps, z, 1.0 / 39916800.0);         //  1/11!
    ps = __builtin_fma(ps, z, -1.0 / 362880.0);          // -1/9!
    ps = __builtin_fma(ps, z, 1.0 / 5040.0);             //  1/7!
    ps = __builtin_fma(ps, z, -1.0 / 120.0);             // -1/5!
    ps = __builtin_fma(ps, z, 1.0 / 6.0);                //  1/3!
    sn = __builtin_fma(-(r * z), ps, r);                 // r - r^3 (1/3! - z/5! + ...)
    double pc = 1.0 / 20922789888000.0;                  //  1/16!
    pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);     // -1/14!
    pc = __builtin_fma(pc, z, 1.0 / 479001600.0);        //  1/12!
    pc = __builtin_fma(pc, z, -1.0 / 3628800.0);         // -1/10!
    pc = __builtin_fma(pc, z, 1.0 / 40320.0);            //  1/8!
    pc = __builtin_fma(pc, z, -1.0 / 720.0);             // -1/6!
    pc = __builtin_fma(pc, z, 1.0 / 24.0);               //  1/4!
    pc = __builtin_fma(pc, z, -0.5);                     // -1/2!
    cs = __builtin_fma(pc, z, 1.0);
}

__host__ __device__ inline void sincos_reduced(double y, double& sn, double& cs) {
    const double k = __builtin_rint(y * kTwoOverPi);
    double r = __builtin_fma(-k, kPio2A, y);
    r = __builtin_fma(-k, kPio2B, r);
    r = __builtin_fma(-k, kPio2C, r);
    double s0, c0;
    sincos_poly(r, s0, c0);
    // quadrant q of y = q pi/2 + r: (sin, cos) = (s, c), (c, -s), (-s, -c), (-c, s)
    const int q = (int)k & 3;
    const double a = (q & 1) ? c0 : s0;
    const double b = (q & 1) ? s0 : c0;
    sn = (q & 2) ? -a : a;
    cs = ((q + 1) & 2) ? -b : b;
}

// |y| < kTrigArgMax (checked on the host for every phase of a run)
__device__ inline void sincos_fast(double y, double* sn, double* cs) { sincos_reduced(y, *sn, *cs); }

// FP32 sin and cos for the precision form, |y| < kTrigArgMax: the quadrant and
// the reduced argument r = y - k pi/2 in FP64 (as above; exact to FP32
// rounding), then Taylor series in FP32 through r^9 and r^10 on |r| <= pi/4
// (the next terms are below 3e-9 there), coefficients 1/n!.
__host__ __device__ inline void sincos_f32(float y, float& sn, float& cs) {
    const double yd = (double)y;
    const double k = __builtin_rint(yd * kTwoOverPi);
    double rd = __builtin_fma(-k, kPio2A, yd);
    rd = __builtin_fma(-k, kPio2B, rd);
    const float r = (float)rd, z = r * r;
    float ps = 1.0f / 362880.0f;                          //  1/9!
    ps = __builtin_fmaf(ps, z, -1.0f / 5040.0f);         // -1/7!
    ps = __builtin_fmaf(ps, z, 1.0f / 120.0f);           //  1/5!
    ps = __builtin_fmaf(ps, z, -1.0f / 6.0f);            // -1/3!
    const float s0 = __builtin_fmaf(ps * z, r, r);
    float pc = -1.0f / 3628800.0f;                        // -1/10!
    pc = __builtin_fmaf(pc, z, 1.0f / 40320.0f);         //  1/8!
    pc = __builtin_fmaf(pc, z, -1.0f / 720.0f);          // -1/6!
    pc = __builtin_fmaf(pc, z, 1.0f / 24.0f);            //  1/4!
    pc = __builtin_fmaf(pc, z, -0.5f);                   // -1/2!
    const float c0 = __builtin_fmaf(pc, z, 1.0f);
    const int q = (int)k & 3;
    const float a = (q & 1) ? c0 : s0;
    const float b = (q & 1) ? s0 : c0;
    sn = (q & 2) ? -a : a;
    cs = ((q + 1) & 2) ? -b : b;
}

// (ln|w|, arg w) of w = (re, im) in FP32 for the precision form's stores: FP32
// log and atan2, then one Newton step each in FP64 (ln|w| = l0 + ln(1 + u) / 2
// with u = |w|^2 e^(-2 l0) - 1; arg w = a0 + atan of w turned by -a0), rounded
// once.  Out of line: its temporaries do not add to the calling kernel's registers.
__device__ __noinline__ float2 to_log_domain32(double re, double im) {
    const double n2 = norm2_nocontract(re, im);
    const float l0 = 0.5f * logf((float)n2);
    const double u = __builtin_fma(n2, exp_fast(-2.0 * (double)l0), -1.0);
    const float a0 = atan2f((float)im, (float)re);
    double sa, ca;
    sincos_fast((double)a0, &sa, &ca);
    const double num = im * ca - re * sa, den = re * ca + im * sa;
    return make_float2((float)((double)l0 + __builtin_fma(-0.25 * u, u, 0.5 * u)),
                       (float)((double)a0 + num * recip(den)));
}

// The error word holds (failing step << 4) | code; the first error wins.
__device__ inline void raise_error(unsigned int* err, int t, unsigned int code) {
    atomicCAS(err, 0u, ((unsigned int)t << 4) | code);
}

__device__ inline unsigned int error_word(const unsigned int* err) {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace quapi_dev
