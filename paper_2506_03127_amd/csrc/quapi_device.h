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

// The error word holds (failing step << 4) | code; the first error wins.
__device__ inline void raise_error(unsigned int* err, int t, unsigned int code) {
    atomicCAS(err, 0u, ((unsigned int)t << 4) | code);
}

__device__ inline unsigned int error_word(const unsigned int* err) {
    return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace quapi_dev
