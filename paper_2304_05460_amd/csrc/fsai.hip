// FSAI of the Schur complement (Algorithm 1 applied as in Algorithm 2).
//
// Row p of G (pattern s, m = |s| <= 64 entries, p last):
//   S_ss = K22[s,s] + mu I - V_s^T V_s          (V = L^{-1} K12, k x nr)
//   S_ss = R R^T (Cholesky),   g = R^{-T} e_m
// which equals Algorithm 1's  e_m^T S_ss^{-1} / sqrt(e_m^T S_ss^{-1} e_m):
// with y = S_ss^{-1} e_m = R^{-T} R^{-1} e_m and R^{-1} e_m = e_m / R_mm,
// y_m = 1 / R_mm^2, so y / sqrt(y_m) = R^{-T} e_m.
//
// One workgroup per row: the k x m gathered columns of V stream through LDS
// in chunks of 32 rows; each thread accumulates a 4 x 4 block of the Gram
// matrix; the m x m Schur block is factored in LDS.
#include "afn_internal.h"

namespace afn {
namespace {

constexpr int W = 64;
constexpr int TK = 32;

__global__ __launch_bounds__(256) void fsai_row_kernel(const double *__restrict__ Xp, int k, int d,
                                                       double l2, double mu,
                                                       const double *__restrict__ V,
                                                       const int32_t *__restrict__ cols, int w,
                                                       double *__restrict__ gval, int *info,
                                                       int64_t row0)
{
    __shared__ int s[W];
    __shared__ double Vt[TK][W + 1];
    __shared__ double S[W][W + 1];    // S[col][row]
    __shared__ double g[W];
    const int tid = threadIdx.x;
    const int64_t p = row0 + blockIdx.x;
    const int m = (int)(p + 1 < w ? p + 1 : w);
    if (tid < W) s[tid] = tid < m ? cols[p * w + tid] : 0;
    __syncthreads();
    const int ty = tid / 16, tx = tid % 16;
    double acc[4][4] = {};
    for (int t0 = 0; t0 < k; t0 += TK) {
        for (int e = tid; e < TK * W; e += 256) {
            int a = e / TK, tt = e - a * TK;
            Vt[tt][a] = (a < m && t0 + tt < k) ? V[(int64_t)(t0 + tt) + (int64_t)s[a] * k] : 0.0;
        }
        __syncthreads();
        for (int tt = 0; tt < TK; ++tt) {
            double x[4], y[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) { x[q] = Vt[tt][ty * 4 + q]; y[q] = Vt[tt][tx * 4 + q]; }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[q][u] = __builtin_fma(x[q], y[u], acc[q][u]);
        }
        __syncthreads();
    }
    const double *Xr = Xp + (int64_t)k * d;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int a = ty * 4 + q, b = tx * 4 + u;
            double v = 0.0;
            if (a < m && b < m) {
                const double *xa = Xr + (int64_t)s[a] * d, *xb = Xr + (int64_t)s[b] * d;
                double dd = 0.0;
                for (int t = 0; t < d; ++t) {
                    double del = xa[t] - xb[t];
                    dd = __builtin_fma(del, del, dd);
                }
                v = exp(-(dd / l2)) + (a == b ? mu : 0.0) - acc[q][u];
            }
            S[b][a] = v;
        }
    __syncthreads();
    // Cholesky S = R R^T (lower R stored in S[col][row], row >= col)
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            double pv = S[j][j];
            if (!(pv > 0.0)) {
                atomicCAS(info, 0, 1);
                pv = 1.0;
            }
            S[j][j] = sqrt(pv);
        }
        __syncthreads();
        const double piv = S[j][j];
        for (int r = j + 1 + tid; r < m; r += 256) S[j][r] /= piv;
        __syncthreads();
        const int mm = m - j - 1;
        for (int e = tid; e < mm * mm; e += 256) {
            int c = j + 1 + e / mm, r = j + 1 + e % mm;
            if (r >= c) S[c][r] -= S[j][r] * S[j][c];
        }
        __syncthreads();
    }
    // g = R^{-T} e_m by back substitution, one wavefront
    if (tid < 64) {
        const int lane = tid;
        double gl = 0.0;   // g[lane] once known
        if (lane == m - 1) gl = 1.0 / S[m - 1][m - 1];
        for (int i = m - 2; i >= 0; --i) {
            // sum_{t > i} R[t][i] g[t],  R[t][i] = S[i][t]
            double term = (lane > i && lane < m) ? S[i][lane] * gl : 0.0;
            for (int off = 32; off > 0; off >>= 1) term += __shfl_xor(term, off, 64);
            if (lane == i) gl = -term / S[i][i];
        }
        if (lane < w) gval[p * w + lane] = lane < m ? gl : 0.0;
        (void)g;
    }
}

__global__ __launch_bounds__(256) void count_cols(const int32_t *cols, int64_t nr, int w,
                                                  unsigned long long *cnt)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nr * w) return;
    int64_t p = e / w;
    int a = (int)(e - p * w);
    int m = (int)(p + 1 < w ? p + 1 : w);
    if (a < m) atomicAdd(&cnt[cols[e]], 1ULL);
}

// Exclusive scan of nr counts into ptr[0..nr] by one workgroup.
__global__ __launch_bounds__(1024) void scan_counts(const unsigned long long *cnt, int64_t nr,
                                                    int64_t *ptr)
{
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nr; base += 1024) {
        int64_t i = base + threadIdx.x;
        int64_t v = i < nr ? (int64_t)cnt[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int64_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nr) ptr[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) ptr[nr] = carry;
}

__global__ __launch_bounds__(256) void fill_transpose(const int32_t *cols, const double *gval,
                                                      int64_t nr, int w, const int64_t *ptr,
                                                      unsigned long long *cursor, int32_t *trow,
                                                      double *tval)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nr * w) return;
    int64_t p = e / w;
    int a = (int)(e - p * w);
    int m = (int)(p + 1 < w ? p + 1 : w);
    if (a >= m) return;
    int c = cols[e];
    unsigned long long pos = atomicAdd(&cursor[c], 1ULL);
    int64_t at = ptr[c] + (int64_t)pos;
    trow[at] = (int32_t)p;
    tval[at] = gval[e];
}

// Order every column of G^T's CSR by row index (deterministic layout).
__global__ __launch_bounds__(256) void sort_segments(const int64_t *ptr, int64_t nr, int32_t *trow,
                                                     double *tval)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nr) return;
    int64_t b = ptr[c], e = ptr[c + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        int32_t r = trow[i];
        double v = tval[i];
        int64_t j = i;
        while (j > b && trow[j - 1] > r) {
            trow[j] = trow[j - 1];
            tval[j] = tval[j - 1];
            --j;
        }
        trow[j] = r;
        tval[j] = v;
    }
}

}  // namespace

afn_status fsai_rows(const double *Xp, int64_t n, int k, int d, double l, double mu,
                     const double *V, const int32_t *cols, int w, double *gval, int *info,
                     hipStream_t s)
{
    const int64_t nr = n - k;
    if (nr <= 0) return AFN_OK;
    const int64_t chunk = 1 << 20;
    for (int64_t r0 = 0; r0 < nr; r0 += chunk) {
        int64_t cnt = nr - r0 < chunk ? nr - r0 : chunk;
        hipLaunchKernelGGL(fsai_row_kernel, dim3((unsigned)cnt), dim3(256), 0, s, Xp, k, d, l * l, mu,
                           V, cols, w, gval, info, r0);
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

afn_status fsai_transpose(const int32_t *cols, const double *gval, int64_t nr, int w,
                          int64_t *tptr, int32_t *trow, double *tval, int64_t *work,
                          hipStream_t s)
{
    if (nr <= 0) {
        AFN_HIP(hipMemsetAsync(tptr, 0, sizeof(int64_t), s));
        return AFN_OK;
    }
    unsigned long long *cnt = (unsigned long long *)work;
    AFN_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)nr, s));
    const unsigned blocks = (unsigned)ceil_div(nr * w, 256);
    hipLaunchKernelGGL(count_cols, dim3(blocks), dim3(256), 0, s, cols, nr, w, cnt);
    hipLaunchKernelGGL(scan_counts, dim3(1), dim3(1024), 0, s, cnt, nr, tptr);
    AFN_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)nr, s));
    hipLaunchKernelGGL(fill_transpose, dim3(blocks), dim3(256), 0, s, cols, gval, nr, w, tptr, cnt,
                       trow, tval);
    hipLaunchKernelGGL(sort_segments, dim3((unsigned)ceil_div(nr, 256)), dim3(256), 0, s, tptr, nr,
                       trow, tval);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
