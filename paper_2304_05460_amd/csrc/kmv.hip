// Kernel matvec y = (K + mu I) v with the Gaussian kernel evaluated on the fly
// (Eq. (1.1), Eq. (1.2)).  FP64 path.
//
// Layout: X row-major n x d FP64.  A workgroup owns 256 consecutive rows (one
// per thread, point coordinates in registers) and one of S contiguous column
// ranges; the column range is streamed through LDS in tiles of BN points
// (coordinates stored coordinate-major so that every lane reads the same
// address: LDS broadcast).  Each (row, split) partial sum goes to a workspace;
// a second pass adds the S partials in ascending split order, so the result
// is deterministic and independent of scheduling.
#include "afn_internal.h"

namespace afn {
namespace {

constexpr int kRows = 256;

template <int D, int BN>
__global__ __launch_bounds__(256) void kmv_f64_partial(const double *__restrict__ X, int64_t n,
                                                       int d_rt, double neg_inv_l2,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ part,
                                                       int64_t split_len)
{
    constexpr int DC = D > 0 ? D : 1;
    __shared__ double sx[(D > 0 ? D : kMaxD) * BN];
    __shared__ double sv[BN];
    const int d = D > 0 ? D : d_rt;
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kRows + tid;
    const int64_t c0 = (int64_t)blockIdx.y * split_len;
    const int64_t c1 = c0 + split_len < n ? c0 + split_len : n;
    const bool row_ok = i < n;

    double xi[DC];
    if (D > 0) {
#pragma unroll
        for (int t = 0; t < DC; ++t) xi[t] = row_ok ? X[i * D + t] : 0.0;
    }
    double acc = 0.0;
    for (int64_t j0 = c0; j0 < c1; j0 += BN) {
        const int jn = (int)(c1 - j0 < BN ? c1 - j0 : BN);
        for (int e = tid; e < BN * d; e += blockDim.x) {
            int j = e / d, t = e - j * d;
            sx[t * BN + j] = j < jn ? X[(j0 + j) * d + t] : 0.0;
        }
        for (int j = tid; j < BN; j += blockDim.x) sv[j] = j < jn ? v[j0 + j] : 0.0;
        __syncthreads();
        if (D > 0) {
#pragma unroll 4
            for (int j = 0; j < jn; ++j) {
                double d2 = 0.0;
#pragma unroll
                for (int t = 0; t < DC; ++t) {
                    double del = xi[t] - sx[t * BN + j];
                    d2 = __builtin_fma(del, del, d2);
                }
                acc = __builtin_fma(exp(d2 * neg_inv_l2), sv[j], acc);
            }
        } else {
            for (int j = 0; j < jn; ++j) {
                double d2 = 0.0;
                for (int t = 0; t < d; ++t) {
                    double xit = row_ok ? X[i * d + t] : 0.0;
                    double del = xit - sx[t * BN + j];
                    d2 = __builtin_fma(del, del, d2);
                }
                acc = __builtin_fma(exp(d2 * neg_inv_l2), sv[j], acc);
            }
        }
        __syncthreads();
    }
    if (row_ok) part[(int64_t)blockIdx.y * n + i] = acc;
}

// FP32 tiles: coordinates rounded to FP32 on load, squared distance and the
// kernel value in FP32 (exp via the hardware base-2 exponential with log2(e)
// folded into the scale), FP32 accumulation within a split; the S split
// partials are added in FP64 by kmv_reduce.
template <int D, int BN>
__global__ __launch_bounds__(256) void kmv_f32_partial(const double *__restrict__ X, int64_t n,
                                                       int d_rt, float neg_log2e_inv_l2,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ part,
                                                       int64_t split_len)
{
    constexpr int DC = D > 0 ? D : 1;
    __shared__ float sx[(D > 0 ? D : kMaxD) * BN];
    __shared__ float sv[BN];
    const int d = D > 0 ? D : d_rt;
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kRows + tid;
    const int64_t c0 = (int64_t)blockIdx.y * split_len;
    const int64_t c1 = c0 + split_len < n ? c0 + split_len : n;
    const bool row_ok = i < n;
    float xi[DC];
    if (D > 0) {
#pragma unroll
        for (int t = 0; t < DC; ++t) xi[t] = row_ok ? (float)X[i * D + t] : 0.0f;
    }
    float acc = 0.0f;
    for (int64_t j0 = c0; j0 < c1; j0 += BN) {
        const int jn = (int)(c1 - j0 < BN ? c1 - j0 : BN);
        for (int e = tid; e < BN * d; e += blockDim.x) {
            int j = e / d, t = e - j * d;
            sx[t * BN + j] = j < jn ? (float)X[(j0 + j) * d + t] : 0.0f;
        }
        for (int j = tid; j < BN; j += blockDim.x) sv[j] = j < jn ? (float)v[j0 + j] : 0.0f;
        __syncthreads();
        if (D > 0) {
#pragma unroll 8
            for (int j = 0; j < jn; ++j) {
                float d2 = 0.0f;
#pragma unroll
                for (int t = 0; t < DC; ++t) {
                    float del = xi[t] - sx[t * BN + j];
                    d2 = __builtin_fmaf(del, del, d2);
                }
                acc = __builtin_fmaf(__builtin_amdgcn_exp2f(d2 * neg_log2e_inv_l2), sv[j], acc);
            }
        } else {
            for (int j = 0; j < jn; ++j) {
                float d2 = 0.0f;
                for (int t = 0; t < d; ++t) {
                    float xit = row_ok ? (float)X[i * d + t] : 0.0f;
                    float del = xit - sx[t * BN + j];
                    d2 = __builtin_fmaf(del, del, d2);
                }
                acc = __builtin_fmaf(__builtin_amdgcn_exp2f(d2 * neg_log2e_inv_l2), sv[j], acc);
            }
        }
        __syncthreads();
    }
    if (row_ok) part[(int64_t)blockIdx.y * n + i] = (double)acc;
}

__global__ __launch_bounds__(256) void kmv_reduce(const double *__restrict__ part, int64_t n,
                                                  int splits, double mu,
                                                  const double *__restrict__ v,
                                                  double *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += part[(int64_t)k * n + i];
    y[i] = s + mu * v[i];
}

template <int D, int BN>
void launch_partial(dim3 grid, const double *X, int64_t n, int d, double nil2, const double *v,
                    double *part, int64_t split_len, hipStream_t s)
{
    hipLaunchKernelGGL((kmv_f64_partial<D, BN>), grid, dim3(256), 0, s, X, n, d, nil2, v, part,
                       split_len);
}

template <int D, int BN>
void launch_partial32(dim3 grid, const double *X, int64_t n, int d, float sc, const double *v,
                      double *part, int64_t split_len, hipStream_t s)
{
    hipLaunchKernelGGL((kmv_f32_partial<D, BN>), grid, dim3(256), 0, s, X, n, d, sc, v, part,
                       split_len);
}

}  // namespace

int64_t kmv_splits(int64_t n)
{
    int64_t rb = ceil_div(n, kRows);
    int64_t s = ceil_div(2048, rb);
    int64_t smax = n / 256 > 1 ? n / 256 : 1;
    if (s > smax) s = smax;
    if (s > 64) s = 64;
    return s < 1 ? 1 : s;
}

int64_t kmv_workspace_doubles(int64_t n) { return kmv_splits(n) * n; }

afn_status kmv_f64(const double *X, int64_t n, int d, double l, double mu, const double *v,
                   int64_t ldv, double *y, int64_t ldy, int nrhs, double *work, hipStream_t s,
                   hipEvent_t ev0, hipEvent_t ev1)
{
    const int64_t S = kmv_splits(n);
    const int64_t split_len = ceil_div(n, S);
    const double nil2 = -1.0 / (l * l);
    dim3 grid((unsigned)ceil_div(n, kRows), (unsigned)S);
    for (int c = 0; c < nrhs; ++c) {
        const double *vc = v + c * ldv;
        if (ev0) AFN_HIP(hipEventRecord(ev0, s));
        switch (d) {
            case 1: launch_partial<1, 512>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 2: launch_partial<2, 512>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 3: launch_partial<3, 512>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 4: launch_partial<4, 512>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 5: launch_partial<5, 256>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 6: launch_partial<6, 256>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 7: launch_partial<7, 256>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            case 8: launch_partial<8, 256>(grid, X, n, d, nil2, vc, work, split_len, s); break;
            default: launch_partial<0, 32>(grid, X, n, d, nil2, vc, work, split_len, s); break;
        }
        AFN_HIP(hipGetLastError());
        if (ev1) AFN_HIP(hipEventRecord(ev1, s));
        hipLaunchKernelGGL(kmv_reduce, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, work, n,
                           (int)S, mu, vc, y + c * ldy);
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

}  // namespace afn

namespace afn {

afn_status kmv_f32(const double *X, int64_t n, int d, double l, double mu, const double *v,
                   int64_t ldv, double *y, int64_t ldy, int nrhs, void *work, hipStream_t s)
{
    const int64_t S = kmv_splits(n);
    const int64_t split_len = ceil_div(n, S);
    const float sc = (float)(-1.4426950408889634 / (l * l));
    double *part = (double *)work;
    dim3 grid((unsigned)ceil_div(n, kRows), (unsigned)S);
    for (int c = 0; c < nrhs; ++c) {
        const double *vc = v + c * ldv;
        switch (d) {
            case 1: launch_partial32<1, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 2: launch_partial32<2, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 3: launch_partial32<3, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 4: launch_partial32<4, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 5: launch_partial32<5, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 6: launch_partial32<6, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 7: launch_partial32<7, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            case 8: launch_partial32<8, 512>(grid, X, n, d, sc, vc, part, split_len, s); break;
            default: launch_partial32<0, 32>(grid, X, n, d, sc, vc, part, split_len, s); break;
        }
        AFN_HIP(hipGetLastError());
        hipLaunchKernelGGL(kmv_reduce, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, n,
                           (int)S, mu, vc, y + c * ldy);
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

}  // namespace afn
