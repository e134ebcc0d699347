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
// the Chebyshev nodes of [-1/2, 1/2] (with the coefficients rounded to FP64
// as stored, 2.8e-17 relative, about 0.25 ulp; Horner in FP64 <= 1.7 ulp).  No FP64 round or convert instruction (both
// slower than an FMA on this hardware).  Where the tile boxes bound t, the
// tile kernel takes the table-driven form below instead, without the clamp
// (whose minimum on an MFMA result also costs a NaN canonicalization).
// FP32: the hardware base-2 exponential.
#pragma once

#include <hip/hip_runtime.h>

#include "afn.h"

namespace afn {

constexpr double kLn2 = 0.6931471805599453;

// 2^(-t) for t < 2^31 (also slightly below 0, from rounding), no clamp.
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

// 2^(j/64), j = 0 .. 63, correctly rounded.
constexpr double kExp2Tab64[64] = {
    1.0, 1.0108892860517005, 1.0218971486541166, 1.0330248790212284,
    1.0442737824274138, 1.0556451783605572, 1.0671404006768237, 1.0787607977571199,
    1.0905077326652577, 1.102382583307841, 1.1143867425958924, 1.1265216186082418,
    1.1387886347566916, 1.1511892299529827, 1.1637248587775775, 1.1763969916502812,
    1.189207115002721, 1.202156731452703, 1.215247359980469, 1.22848053610687,
    1.241857812073484, 1.255380757024691, 1.2690509571917332, 1.2828700160787783,
    1.2968395546510096, 1.3109612115247644, 1.3252366431597413, 1.339667524053303,
    1.3542555469368927, 1.3690024229745905, 1.383909881963832, 1.3989796725383112,
    1.4142135623730951, 1.42961333839197, 1.4451808069770467, 1.460917794180647,
    1.4768261459394993, 1.4929077282912648, 1.5091644275934228, 1.5255981507445384,
    1.5422108254079407, 1.559004400237837, 1.5759808451078865, 1.593142151342267,
    1.6104903319492543, 1.6280274218573478, 1.645755478153965, 1.6636765803267364,
    1.681792830507429, 1.7001063537185235, 1.718619298122478, 1.7373338352737062,
    1.7562521603732995, 1.7753764925265212, 1.7947090750031072, 1.8142521755003989,
    1.8340080864093424, 1.8539791250833855, 1.8741676341103, 1.8945759815869656,
    1.9152065613971474, 1.9360617934922943, 1.9571441241754002, 1.978456026387951,
};

// 2^(-t) for t < 2^25 (also slightly below 0) by Tang's table-driven method:
// N = rint(64 t) from c - t with c = 1.5 * 2^46 (ulp 1/64 there; the low word
// of c - t is -N as a 32-bit integer), f = N/64 - t in [-1/128, 1/128]
// exactly, and with -N = 64 e + j (0 <= j < 64)
//   2^(-t) = 2^e * tab[j] * 2^f,   tab[j] = 2^(j/64) (kExp2Tab64, staged in
// LDS by the caller), 2^f by the degree-5 polynomial interpolating it at the
// Chebyshev nodes of [-1/128, 1/128] (2.4e-18 relative).  Two FP64
// instructions fewer than the degree-11 form, for one LDS read.
__device__ __forceinline__ double exp2_neg_tab(double t, const double *tab)
{
    const double kb = 105553116266496.0 - t;
    const double kd = 105553116266496.0 - kb;
    const double f = kd - t;
    const int lo = __double2loint(kb);
    const double tj = tab[lo & 63];
    double p = 0.0013333572110729706;
    p = __builtin_fma(p, f, 0.00961814320999005);
    p = __builtin_fma(p, f, 0.055504108664789616);
    p = __builtin_fma(p, f, 0.24022650695877792);
    p = __builtin_fma(p, f, 0.6931471805599453);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_ldexp(p * tj, lo >> 6);
}

__device__ __forceinline__ float exp2_neg(float t) { return __builtin_amdgcn_exp2f(-t); }

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

// kernel_scaled by the table-driven exponential (FP64), for t below 2^25
// (Gaussian) or 2^50 (Matern); FP32: the hardware exponential.
template <int KIND, typename T>
__device__ __forceinline__ T kernel_scaled_tab(T t, const T *tab)
{
    if constexpr (sizeof(T) == 4) {
        return kernel_scaled<KIND, T>(t);
    } else if constexpr (KIND == AFN_KERNEL_MATERN32) {
        const T s = sqrtT(t);
        return (T(1) + s * T(kLn2)) * exp2_neg_tab(s, tab);
    } else {
        return exp2_neg_tab(t, tab);
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
