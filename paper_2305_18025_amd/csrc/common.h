// Device helpers shared by the exchange kernels (exchange.h, compiled once
// per launch variant from exchange_inst.hip) and the other kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include "internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace pimdb {

constexpr double LN2 = 0.6931471805599453;
constexpr double LOG2E = 1.4426950408889634;
constexpr double XLO = -536870912.0;     // -2^29: lower clamp of an exported term exponent
constexpr double XHI = 268435456.0;      //  2^28: bound on h = -kappa |d_ref|^2
constexpr int EMIN = -(1 << 30);         // exponent of an empty accumulator
constexpr int EZ_LIM = 1 << 29;          // bound on the exponent of a published Z value
constexpr int EMASK = -(3 << 29);        // term exponent that adds nothing (below EMIN)

enum StatusBits { ST_NONFINITE_IN = 1, ST_NONFINITE_OUT = 2, ST_RANGE = 4, ST_PRECISION = 8, ST_TIMEOUT = 16 };
// |kappa| max |p - o|^2 up to which the open FP64 dot form keeps the 1e-10
// accuracy with margin (measured 4e-12 in the forces at 2.5e6)
constexpr double DOT_LIM = 8388608.0; // 2^23

// 2^f for |f| <= 1/2: degree-10 minimax polynomial (relative approximation
// error 2.1e-16, about one rounding; coefficients from gen_exp2_coeffs.py),
// highest degree first.  Kept in constant memory so the wave-uniform
// coefficients live in scalar registers and every Horner step is one
// v_fma_f64.  The array has external linkage, so the compiler cannot fold
// the values into 64-bit literals (each would take two VGPRs); every
// translation unit names its own copy (PIMDB_EXP2_SYM) so the host-side
// shadows of the copies do not collide at link time.
#ifndef PIMDB_EXP2_SYM
#define PIMDB_EXP2_SYM exp2_c_misc
#endif
#define EXP2_C PIMDB_EXP2_SYM
constexpr int EXP2_N = 11;
__constant__ double EXP2_C[EXP2_N] = {
    7.037278846726901e-09,  1.0208537929657404e-07, 1.3215662835959238e-06, 1.5252658116409854e-05,
    0.00015403529961127076, 0.0013333558228561767,  0.009618129108034596,   0.05550410866445883,
    0.24022650695908768,    0.6931471805599497,     1.0};

__device__ __forceinline__ double exp2_frac(double f) {
    double p = EXP2_C[0];
#pragma unroll
    for (int i = 1; i < EXP2_N; ++i) p = fma(p, f, EXP2_C[i]);
    return p;
}

template <bool BOX>
__device__ __forceinline__ double mimg(double d, double box, double inv_box) {
    if (BOX) return fma(-box, rint(d * inv_box), d);
    return d;
}

// |d|^2 in FP32 with exact products (FMA) and compensated summation; the
// displacement itself is formed in FP64 and rounded to FP32 once.
__device__ __forceinline__ double sqlen_f32c(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    const float x = (float)dx, y = (float)dy, z = (float)dz;
    const float px = x * x, ex = fmaf(x, x, -px);
    const float py = y * y, ey = fmaf(y, y, -py);
    const float pz = z * z, ez = fmaf(z, z, -pz);
    float s1 = px + py;
    float bb = s1 - px;
    const float e1 = (px - (s1 - bb)) + (py - bb);
    const float s2 = s1 + pz;
    bb = s2 - s1;
    const float e2 = (s1 - (s2 - bb)) + (pz - bb);
    const float lo = ((ex + ey) + ez) + (e1 + e2);
    return (double)s2 + (double)lo;
}

template <bool MIXED>
__device__ __forceinline__ double sqlen(double dx, double dy, double dz) {
    if (MIXED) return sqlen_f32c(dx, dy, dz);
    return fma(dx, dx, fma(dy, dy, dz * dz));
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int t = threadIdx.x, T = blockDim.x; // T is a power of two
    red[t] = v;
    __syncthreads();
    for (int s = T >> 1; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Workgroup barrier ordering LDS alone: a wave's global stores still in
// flight need not complete first (the recursion workgroups never read back
// another wave's global stores within a launch: results go to the next
// launch, exchange-area payloads to other workgroups behind their own
// flags), so the stores of one phase overlap the next.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ void set_flag(int32_t *flags, int bits) {
    __hip_atomic_fetch_or(flags, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 2^x as mantissa p in [0.7, 1.42] and integer exponent n; n saturates for
// |x| >= 2^31 (such terms then add nothing).
__device__ __forceinline__ void exp2x(double x, double &p, int &n) {
    const double r = rint(x);
    p = exp2_frac(x - r);
    n = (int)r;
}

} // namespace pimdb
