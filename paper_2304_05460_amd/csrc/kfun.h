// Kernel functions of the device code (Eq. (1.2) and the Matern-3/2 kernel of
// Section 5), r = ||x - y||:
//   AFN_KERNEL_GAUSSIAN   K = exp(-r^2 / l^2)
//   AFN_KERNEL_MATERN32   K = (1 + sqrt(3) r / l) exp(-sqrt(3) r / l)
//
// The tile kernels of the matvec read coordinates pre-scaled by
// kernel_scale(kind, l), so that the squared distance t of two scaled points
// gives the kernel value without a division:
//   Gaussian   scale sqrt(log2 e) / l           K = 2^(-t)
//   Matern     scale sqrt(3) log2(e) / l        s = sqrt(t), K = (1 + s ln 2) 2^(-s)
// Both are decreasing in t, so a lower bound on t over a pair of tiles bounds
// every kernel value in it; kernel_cut_t(kind, cut) is the t at which the
// kernel value is 2^-cut.
//
// 2^(-t) in FP64 (t >= 0): t clamped to 2000 (the result underflows long
// before; the bounded form leaves that to its caller), k = rint(t) from
// c - t with c = 1.5 * 2^52 (ulp 1 there, so the subtraction rounds t to
// the nearest integer, ties to even, and the low word of c - t is -k as a
// 32-bit integer), f = k - t in [-1/2, 1/2] exactly, and
// 2^(-t) = p(f) 2^(-k) with p the degree-11 polynomial interpolating 2^f at
// the Chebyshev nodes of [-1/2, 1/2] (interpolation error 4.4e-18 relative;
// Horner in FP64 <= 1.7 ulp).  No FP64 round or convert instruction (both
// slower than an FMA on this hardware).  FP32: the hardware base-2
// exponential.
#pragma once

#include <hip/hip_runtime.h>

#include "afn.h"

namespace afn {

constexpr double kLn2 = 0.6931471805599453;

// 2^(-t) for t < 2^31 (also slightly below 0, from rounding): the caller
// bounds t, so no clamp (whose minimum on an MFMA result also costs a NaN
// canonicalization) is needed.
__device__ __forceinline__ double exp2_neg_bounded(double t)
{
    const double kb = 6755399441055744.0 - t;
    const double kd = 6755399441055744.0 - kb;
    const double f = kd - t;
    double p = 4.45594401136235e-10;
    p = __builtin_fma(p, f, 7.074200215313511e-09);
    p = __builtin_fma(p, f, 1.0178056459844976e-07);
    p = __builtin_fma(p, f, 1.3215432494521488e-06);
    p = __builtin_fma(p, f, 1.5252733842373628e-05);
    p = __builtin_fma(p, f, 0.00015403530463828206);
    p = __builtin_fma(p, f, 0.0013333558146406623);
    p = __builtin_fma(p, f, 0.009618129107587145);
    p = __builtin_fma(p, f, 0.05550410866482162);
    p = __builtin_fma(p, f, 0.2402265069591016);
    p = __builtin_fma(p, f, 0.6931471805599453);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_ldexp(p, __double2loint(kb));
}

__device__ __forceinline__ double exp2_neg(double t) { return exp2_neg_bounded(t < 2000.0 ? t : 2000.0); }

__device__ __forceinline__ float exp2_neg(float t) { return __builtin_amdgcn_exp2f(-t); }
__device__ __forceinline__ float exp2_neg_bounded(float t) { return exp2_neg(t); }

__device__ __forceinline__ double sqrtT(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float sqrtT(float x) { return __builtin_sqrtf(x); }

// Kernel value from the squared distance t of pre-scaled points.
template <int KIND, typename T>
__device__ __forceinline__ T kernel_scaled(T t)
{
    if constexpr (KIND == AFN_KERNEL_MATERN32) {
        const T s = sqrtT(t);
        return (T(1) + s * T(kLn2)) * exp2_neg(s);
    } else {
        return exp2_neg(t);
    }
}

// kernel_scaled without the clamp, for t below 2^31 (Gaussian) or 2^62
// (Matern, whose exponent is sqrt(t)).
template <int KIND, typename T>
__device__ __forceinline__ T kernel_scaled_bounded(T t)
{
    if constexpr (KIND == AFN_KERNEL_MATERN32) {
        const T s = sqrtT(t);
        return (T(1) + s * T(kLn2)) * exp2_neg_bounded(s);
    } else {
        return exp2_neg_bounded(t);
    }
}

// Kernel value from the plain squared distance d2 (l2 = l^2); for the setup
// kernels, which take the kind at run time.
__device__ __forceinline__ double kernel_d2(double d2, double l2, int kind)
{
    if (kind == AFN_KERNEL_MATERN32) {
        const double s = __builtin_sqrt(3.0 * d2 / l2);
        return (1.0 + s) * exp(-s);
    }
    return exp(-(d2 / l2));
}

// Host side (kmv.hip): scale of the packed coordinates, and the scaled
// squared distance beyond which every kernel value is below 2^-cut.
double kernel_scale(int kind, double l);
double kernel_cut_t(int kind, double cut);

}  // namespace afn
