// Vector kernels of the AFN apply (Algorithm 3) and of PCG.  Every reduction
// has a fixed order (per-workgroup partials, then one ordered pass), so results
// are bitwise reproducible run to run.
#include <cstdio>

#include "afn_internal.h"
#include "group.h"

namespace afn {
namespace {

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_sumT(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_sumT(double v) { return wave_sum(v); }

__device__ double block_sum(double v)
{
    __shared__ double ws[16];
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (int)(blockDim.x >> 6);
    for (int i = 0; i < nw; ++i) s += ws[i];
    __syncthreads();
    return s;
}

constexpr int kDotBlocks = 512;

// Each kernel below that a PCG iteration launches has its body in a device
// function taking the block coordinates, an argument struct, the kernel of
// one launch (its usual name) and a grouped kernel (suffix _g, see group.h)
// that runs the same body for several solves in one launch.
#define AFN_GROUPED_ARGS(Args)                                                                  \
    static void launch1(const Args &p, dim3 grid, size_t lds, hipStream_t s);                  \
    static void launchG(const GroupTable<Args> &t, unsigned blocks, size_t lds, hipStream_t s);

template <typename T>
struct DotArgs {
    const T *a, *b;
    int64_t n, chunk;
    double *part;
    AFN_GROUPED_ARGS(DotArgs)
};

template <typename T>
__device__ __forceinline__ void dot_stage1_body(const DotArgs<T> &p, int64_t bx)
{
    const int64_t i0 = bx * p.chunk;
    const int64_t i1 = i0 + p.chunk < p.n ? i0 + p.chunk : p.n;
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
        s = __builtin_fma((double)p.a[i], (double)p.b[i], s);
    s = block_sum(s);
    if (threadIdx.x == 0) p.part[bx] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void dot_stage1(DotArgs<T> p) { dot_stage1_body(p, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void dot_stage1_g(GroupTable<DotArgs<T>> t)
{
    const GroupPos q = group_pos(t);
    dot_stage1_body(t.a[q.g], q.bx);
}

struct SumArgs {
    const double *part;
    int np;
    int step;          // -1: plain sum into *out; else the PCG scalar step
    double *out;       // the sum (step -1) or the PCG scalars
    AFN_GROUPED_ARGS(SumArgs)
};

// The ordered sum of the partials; for the PCG dot products followed by the
// scalar step (alpha = rho / p'q, or beta = rho_new / rho and rho = rho_new).
__device__ __forceinline__ void sum_stage2_body(const SumArgs &p)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < p.np; i += blockDim.x) s += p.part[i];
    s = block_sum(s);
    if (threadIdx.x == 0) {
        double *sc = p.out;
        if (p.step < 0) {
            *sc = s;
        } else if (p.step == kPcgAlpha) {
            sc[1] = s;
            sc[4] = sc[0] / s;
        } else {
            sc[3] = s;
            sc[5] = s / sc[0];
            sc[0] = s;
        }
    }
}

__global__ __launch_bounds__(256) void sum_stage2(SumArgs p) { sum_stage2_body(p); }

__global__ __launch_bounds__(256) void sum_stage2_g(GroupTable<SumArgs> t)
{
    const GroupPos q = group_pos(t);
    sum_stage2_body(t.a[q.g]);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Loads in flight per thread in the GEMV loops (the sums stay in index order).
constexpr int kGemvUnroll = 8;

// y[i] (+)= sum over column chunk of A[i + j*lda] x[j]; partial per split.
template <typename T, typename M>
struct GemvNArgs {
    const M *A;
    int64_t lda, m, ncols;
    const T *x;
    int64_t chunk;
    T *part;
    AFN_GROUPED_ARGS(GemvNArgs)
};

template <typename T, typename M>
__device__ __forceinline__ void gemv_n_partial_body(const GemvNArgs<T, M> &p, int64_t bx, int64_t by)
{
    const M *__restrict__ A = p.A;
    const T *__restrict__ x = p.x;
    const int64_t lda = p.lda, m = p.m, ncols = p.ncols, chunk = p.chunk;
    T *__restrict__ part = p.part;
    const int64_t i = bx * blockDim.x + threadIdx.x;
    const int64_t j0 = by * chunk;
    const int64_t j1 = j0 + chunk < ncols ? j0 + chunk : ncols;
    if (i >= m) return;
    T s = T(0);
    int64_t j = j0;
    for (; j + kGemvUnroll <= j1; j += kGemvUnroll) {
        T a[kGemvUnroll];
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) a[u] = widen<T>(A[i + (j + u) * lda]);
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) s = fmaT(a[u], x[j + u], s);
    }
    for (; j < j1; ++j) s = fmaT(widen<T>(A[i + j * lda]), x[j], s);
    part[by * m + i] = s;
}

template <typename T, typename M>
__global__ __launch_bounds__(256) void gemv_n_partial(GemvNArgs<T, M> p) { gemv_n_partial_body(p, blockIdx.x, blockIdx.y); }

template <typename T, typename M>
__global__ __launch_bounds__(256) void gemv_n_partial_g(GroupTable<GemvNArgs<T, M>> t)
{
    const GroupPos q = group_pos(t);
    gemv_n_partial_body(t.a[q.g], q.bx, q.by);
}

// y[i] = base[i] + sign * sum_s part[s][i]   (base may be null -> 0);
// WAVE: one wavefront per row, for many splits: lane q adds splits q, q + 64,
// ... in order, then the 64 lane sums are added by a fixed butterfly
// (deterministic).
template <typename T, bool WAVE>
struct GemvRedArgs {
    const T *part;
    int64_t m;
    int splits;
    T sign;
    const T *base;
    T *y;
    AFN_GROUPED_ARGS(GemvRedArgs)
};

template <typename T, bool WAVE>
__device__ __forceinline__ void gemv_n_reduce_body(const GemvRedArgs<T, WAVE> &p, int64_t bx)
{
    if constexpr (WAVE) {
        const int lane = threadIdx.x & 63;
        const int64_t i = bx * 4 + (threadIdx.x >> 6);
        if (i >= p.m) return;
        T s = T(0);
        for (int k = lane; k < p.splits; k += 64) s += p.part[(int64_t)k * p.m + i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) p.y[i] = (p.base ? p.base[i] : T(0)) + p.sign * s;
    } else {
        const int64_t i = bx * blockDim.x + threadIdx.x;
        if (i >= p.m) return;
        T s = T(0);
        for (int k = 0; k < p.splits; ++k) s += p.part[(int64_t)k * p.m + i];
        p.y[i] = (p.base ? p.base[i] : T(0)) + p.sign * s;
    }
}

template <typename T, bool WAVE>
__global__ __launch_bounds__(256) void gemv_n_reduce(GemvRedArgs<T, WAVE> p) { gemv_n_reduce_body(p, blockIdx.x); }

template <typename T, bool WAVE>
__global__ __launch_bounds__(256) void gemv_n_reduce_g(GroupTable<GemvRedArgs<T, WAVE>> t)
{
    const GroupPos q = group_pos(t);
    gemv_n_reduce_body(t.a[q.g], q.bx);
}

template <typename T, typename M, bool FOUR>
struct GemvTArgs {
    const M *A;
    int64_t lda, m, ncols;
    const T *x, *base;
    T sign;
    T *y;
    AFN_GROUPED_ARGS(GemvTArgs)
};

// y[j] = base[j] + sign * sum_i A[i + j*lda] x[i], one wavefront per column.
template <typename T, typename M>
__device__ __forceinline__ void gemv_t_body(const GemvTArgs<T, M, false> &p, int64_t bx)
{
    const M *__restrict__ A = p.A;
    const T *__restrict__ x = p.x;
    const T *__restrict__ base = p.base;
    T *__restrict__ y = p.y;
    const int64_t lda = p.lda, m = p.m, ncols = p.ncols;
    const T sign = p.sign;
    const int lane = threadIdx.x & 63;
    const int64_t j = (bx * blockDim.x + threadIdx.x) >> 6;
    if (j >= ncols) return;
    const M *col = A + j * lda;
    T s = T(0);
    int64_t i = lane;
    for (; i + 64 * (kGemvUnroll - 1) < m; i += 64 * kGemvUnroll) {
        T a[kGemvUnroll], b[kGemvUnroll];
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) {
            a[u] = widen<T>(col[i + 64 * u]);
            b[u] = x[i + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < kGemvUnroll; ++u) s = fmaT(a[u], b[u], s);
    }
    for (; i < m; i += 64) s = fmaT(widen<T>(col[i]), x[i], s);
    s = wave_sumT(s);
    if (lane == 0) y[j] = (base ? base[j] : T(0)) + sign * s;
}

template <typename T, typename M>
__global__ __launch_bounds__(256) void gemv_t_kernel(GemvTArgs<T, M, false> p) { gemv_t_body(p, blockIdx.x); }

// The same sums with four columns per wavefront and x staged in LDS (m T
// values of dynamic LDS): per lane the rows lane, lane + 64, ... of each
// column in order, then the butterfly, as in gemv_t_kernel; x is read from
// HBM once per workgroup instead of once per column.
template <typename T, typename M>
__device__ __forceinline__ void gemv_t4_body(const GemvTArgs<T, M, true> &p, int64_t bx)
{
    const M *__restrict__ A = p.A;
    const T *__restrict__ x = p.x;
    const T *__restrict__ base = p.base;
    T *__restrict__ y = p.y;
    const int64_t lda = p.lda, m = p.m, ncols = p.ncols;
    const T sign = p.sign;
    extern __shared__ char gemv_smem[];
    T *xs = reinterpret_cast<T *>(gemv_smem);
    for (int64_t i = threadIdx.x; i < m; i += 256) xs[i] = x[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t j0 = (bx * 4 + (threadIdx.x >> 6)) * 4;
    if (j0 >= ncols) return;
    const int nc = ncols - j0 < 4 ? (int)(ncols - j0) : 4;
    const M *col[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) col[c] = A + (j0 + (c < nc ? c : nc - 1)) * lda;
    constexpr int U = 4;
    T s[4] = {T(0), T(0), T(0), T(0)};
    int64_t i = lane;
    for (; i + 64 * (U - 1) < m; i += 64 * U) {
        T a[4][U];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int u = 0; u < U; ++u) a[c][u] = widen<T>(col[c][i + 64 * u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T xv = xs[i + 64 * u];
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] = fmaT(a[c][u], xv, s[c]);
        }
    }
    for (; i < m; i += 64) {
        const T xv = xs[i];
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] = fmaT(widen<T>(col[c][i]), xv, s[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const T t = wave_sumT(s[c]);
        if (c < nc && lane == 0) y[j0 + c] = (base ? base[j0 + c] : T(0)) + sign * t;
    }
}

template <typename T, typename M>
__global__ __launch_bounds__(256) void gemv_t4_kernel(GemvTArgs<T, M, true> p) { gemv_t4_body(p, blockIdx.x); }

template <typename T, typename M, bool FOUR>
__global__ __launch_bounds__(256) void gemv_t_g(GroupTable<GemvTArgs<T, M, FOUR>> t)
{
    const GroupPos q = group_pos(t);
    if constexpr (FOUR) gemv_t4_body(t.a[q.g], q.bx);
    else gemv_t_body(t.a[q.g], q.bx);
}

// Sum over the 16 lanes of each lane group (lanes 16 g .. 16 g + 15), a
// fixed butterfly: every lane of the group ends with the total.
template <typename T>
__device__ __forceinline__ T group16_sum(T s)
{
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off);
    return s;
}

// u[p] = sum_a gval[p*w + a] t[cols[p*w + a]], a < min(p+1, w) (w <= 16 RP):
// 16 lanes per row, lane q taking a = q, q + 16, ..., q + 16 (RP - 1) (each
// load instruction reads 16 consecutive entries of a row; 4 rows per wave);
// RP = 4 up to w = 64, 8 up to w = 128.
template <typename T, typename M, int RP>
struct SpmvGArgs {
    const int32_t *cols;
    const M *gval;
    int64_t nr;
    int w;
    const T *t;
    T *u;
    const int32_t *order;
    AFN_GROUPED_ARGS(SpmvGArgs)
};

template <typename T, typename M, int RP>
__device__ __forceinline__ void spmv_padded_body(const SpmvGArgs<T, M, RP> &pa, int64_t bx, int64_t gx)
{
    const int32_t *__restrict__ cols = pa.cols;
    const M *__restrict__ gval = pa.gval;
    const T *__restrict__ t = pa.t;
    T *__restrict__ u = pa.u;
    const int32_t *__restrict__ order = pa.order;
    const int64_t nr = pa.nr;
    const int w = pa.w;
    const int q = threadIdx.x & 15;
    const int64_t blk = order ? xcd_contiguous(bx, gx) : bx;
    const int64_t slot = blk * 16 + (threadIdx.x >> 4);
    if (slot >= nr) return;
    const int64_t p = order ? (int64_t)order[slot] : slot;
    const int m = (int)(p + 1 < w ? p + 1 : w);
    const int64_t base = p * w;
    // entries past the row's end load entry m - 1 (in bounds) and count zero,
    // so that every load is issued before the first wait
    T g[RP], tv[RP];
    int32_t cj[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
        const int a = q + 16 * r < m ? q + 16 * r : m - 1;
        g[r] = widen<T>(gval[base + a]);
        cj[r] = cols[base + a];
    }
#pragma unroll
    for (int r = 0; r < RP; ++r) tv[r] = t[cj[r]];
    T s = T(0);
#pragma unroll
    for (int r = 0; r < RP; ++r) s = fmaT(q + 16 * r < m ? g[r] : T(0), tv[r], s);
    s = group16_sum(s);
    if (q == 0) u[p] = s;
}

template <typename T, typename M, int RP>
__global__ __launch_bounds__(256) void spmv_padded(SpmvGArgs<T, M, RP> p) { spmv_padded_body(p, blockIdx.x, gridDim.x); }

template <typename T, typename M, int RP>
__global__ __launch_bounds__(256) void spmv_padded_g(GroupTable<SpmvGArgs<T, M, RP>> t)
{
    const GroupPos q = group_pos(t);
    spmv_padded_body(t.a[q.g], q.bx, q.gx);
}

// s[c] = sum_e tval[e] u[trow[e]] over e in [ptr[c], ptr[c+1]): 16 lanes per
// row, up to 4 entries per lane in flight per pass (4 rows per wave).
template <typename T, typename M>
struct SpmvCsrArgs {
    const int64_t *ptr;
    const int32_t *idx;
    const M *val;
    int64_t nrows;
    const T *u;
    T *out;
    const int32_t *order;
    AFN_GROUPED_ARGS(SpmvCsrArgs)
};

template <typename T, typename M>
__device__ __forceinline__ void spmv_csr_body(const SpmvCsrArgs<T, M> &pa, int64_t bx, int64_t gx)
{
    const int64_t *__restrict__ ptr = pa.ptr;
    const int32_t *__restrict__ idx = pa.idx;
    const M *__restrict__ val = pa.val;
    const T *__restrict__ u = pa.u;
    T *__restrict__ out = pa.out;
    const int32_t *__restrict__ order = pa.order;
    const int64_t nrows = pa.nrows;
    const int q = threadIdx.x & 15;
    const int64_t blk = order ? xcd_contiguous(bx, gx) : bx;
    const int64_t slot = blk * 16 + (threadIdx.x >> 4);
    if (slot >= nrows) return;
    const int64_t c = order ? (int64_t)order[slot] : slot;
    const int64_t e1 = ptr[c + 1];
    T s = T(0);
    for (int64_t e = ptr[c] + q; e < e1; e += 64) {
        // entries past the row's end load entry e1 - 1 and count zero
        T a[4], b[4];
        int32_t ri[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t f = e + 16 * r < e1 ? e + 16 * r : e1 - 1;
            a[r] = widen<T>(val[f]);
            ri[r] = idx[f];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = u[ri[r]];
#pragma unroll
        for (int r = 0; r < 4; ++r) s = fmaT(e + 16 * r < e1 ? a[r] : T(0), b[r], s);
    }
    s = group16_sum(s);
    if (q == 0) out[c] = s;
}

template <typename T, typename M>
__global__ __launch_bounds__(256) void spmv_csr(SpmvCsrArgs<T, M> p) { spmv_csr_body(p, blockIdx.x, gridDim.x); }

template <typename T, typename M>
__global__ __launch_bounds__(256) void spmv_csr_g(GroupTable<SpmvCsrArgs<T, M>> t)
{
    const GroupPos q = group_pos(t);
    spmv_csr_body(t.a[q.g], q.bx, q.gx);
}

__global__ __launch_bounds__(256) void gather_kernel(const double *__restrict__ src, int64_t lds,
                                                     double *__restrict__ dst, int64_t ldd,
                                                     const int32_t *__restrict__ perm, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = blockIdx.y;
    dst[i + c * ldd] = src[perm[i] + c * lds];
}

__global__ __launch_bounds__(256) void scatter_kernel(const double *__restrict__ src, int64_t lds,
                                                      double *__restrict__ dst, int64_t ldd,
                                                      const int32_t *__restrict__ perm, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = blockIdx.y;
    dst[perm[i] + c * ldd] = src[i + c * lds];
}

__global__ __launch_bounds__(256) void gather_points_kernel(const double *__restrict__ X,
                                                            const int32_t *__restrict__ perm,
                                                            int64_t n, int d,
                                                            double *__restrict__ Xp)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t i = e / d;
    const int t = (int)(e - i * d);
    Xp[e] = X[(int64_t)perm[i] * d + t];
}

// x += alpha p; r -= alpha q; partial sums of r.r (FP64 scalars, vectors in T)
template <typename T>
struct PcgXrArgs {
    T *x, *r;
    const T *p, *q;
    const double *sc;
    int64_t n, chunk;
    double *part;
    AFN_GROUPED_ARGS(PcgXrArgs)
};

template <typename T>
__device__ __forceinline__ void pcg_xr_body(const PcgXrArgs<T> &a, int64_t bx)
{
    T *__restrict__ x = a.x;
    T *__restrict__ r = a.r;
    const T *__restrict__ p = a.p;
    const T *__restrict__ q = a.q;
    const T alpha = (T)a.sc[4];
    const int64_t i0 = bx * a.chunk;
    const int64_t i1 = i0 + a.chunk < a.n ? i0 + a.chunk : a.n;
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        x[i] = fmaT(alpha, p[i], x[i]);
        const T ri = fmaT(-alpha, q[i], r[i]);
        r[i] = ri;
        s = __builtin_fma((double)ri, (double)ri, s);
    }
    s = block_sum(s);
    if (threadIdx.x == 0) a.part[bx] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void pcg_xr(PcgXrArgs<T> a) { pcg_xr_body(a, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void pcg_xr_g(GroupTable<PcgXrArgs<T>> t)
{
    const GroupPos q = group_pos(t);
    pcg_xr_body(t.a[q.g], q.bx);
}

// p = z + beta p
template <typename T>
struct PcgPArgs {
    T *p;
    const T *z;
    const double *sc;
    int64_t n;
    AFN_GROUPED_ARGS(PcgPArgs)
};

template <typename T>
__device__ __forceinline__ void pcg_p_body(const PcgPArgs<T> &a, int64_t bx)
{
    const int64_t i = bx * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    a.p[i] = fmaT((T)a.sc[5], a.p[i], a.z[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void pcg_p(PcgPArgs<T> a) { pcg_p_body(a, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void pcg_p_g(GroupTable<PcgPArgs<T>> t)
{
    const GroupPos q = group_pos(t);
    pcg_p_body(t.a[q.g], q.bx);
}

// r32 = r * scale (rounded to FP32)
__global__ __launch_bounds__(256) void to_f32_scaled(const double *__restrict__ r, double scale,
                                                     float *__restrict__ r32, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    r32[i] = (float)(r[i] * scale);
}

// x += a * e (e in FP32)
__global__ __launch_bounds__(256) void axpy_f32_into_f64(double a, const float *__restrict__ e,
                                                         double *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] = __builtin_fma(a, (double)e[i], x[i]);
}

// FP32 copy of an FP64 array
__global__ __launch_bounds__(256) void to_f32(const double *__restrict__ a, float *__restrict__ b,
                                              int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    b[i] = (float)a[i];
}

// x *= a
template <typename T>
struct ScaleArgs {
    T *x;
    T a;
    int64_t n;
    AFN_GROUPED_ARGS(ScaleArgs)
};

template <typename T>
__device__ __forceinline__ void scale_body(const ScaleArgs<T> &p, int64_t bx)
{
    const int64_t i = bx * blockDim.x + threadIdx.x;
    if (i < p.n) p.x[i] *= p.a;
}

template <typename T>
__global__ __launch_bounds__(256) void scale_kernel(ScaleArgs<T> p) { scale_body(p, blockIdx.x); }

template <typename T>
__global__ __launch_bounds__(256) void scale_g(GroupTable<ScaleArgs<T>> t)
{
    const GroupPos q = group_pos(t);
    scale_body(t.a[q.g], q.bx);
}

// The launchers of the argument structs.
#define AFN_DEFINE_LAUNCH(TPL, Args, k1, kg)                                                          \
    TPL void Args::launch1(const Args &p, dim3 grid, size_t lds, hipStream_t s)                     \
    {                                                                                                \
        hipLaunchKernelGGL(k1, grid, dim3(256), lds, s, p);                                          \
    }                                                                                                \
    TPL void Args::launchG(const GroupTable<Args> &t, unsigned blocks, size_t lds, hipStream_t s)   \
    {                                                                                                \
        hipLaunchKernelGGL(kg, dim3(blocks), dim3(256), lds, s, t);                                  \
    }

AFN_DEFINE_LAUNCH(template <typename T>, DotArgs<T>, dot_stage1<T>, dot_stage1_g<T>)
AFN_DEFINE_LAUNCH(, SumArgs, sum_stage2, sum_stage2_g)
#define AFN_COMMA ,
AFN_DEFINE_LAUNCH(template <typename T AFN_COMMA typename M>, GemvNArgs<T AFN_COMMA M>, (gemv_n_partial<T, M>),
                  (gemv_n_partial_g<T, M>))
AFN_DEFINE_LAUNCH(template <typename T AFN_COMMA bool WAVE>, GemvRedArgs<T AFN_COMMA WAVE>, (gemv_n_reduce<T, WAVE>),
                  (gemv_n_reduce_g<T, WAVE>))
template <typename T, typename M, bool FOUR>
void GemvTArgs<T, M, FOUR>::launch1(const GemvTArgs &p, dim3 grid, size_t lds, hipStream_t s)
{
    if constexpr (FOUR) hipLaunchKernelGGL((gemv_t4_kernel<T, M>), grid, dim3(256), lds, s, p);
    else hipLaunchKernelGGL((gemv_t_kernel<T, M>), grid, dim3(256), lds, s, p);
}
template <typename T, typename M, bool FOUR>
void GemvTArgs<T, M, FOUR>::launchG(const GroupTable<GemvTArgs> &t, unsigned blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((gemv_t_g<T, M, FOUR>), dim3(blocks), dim3(256), lds, s, t);
}
AFN_DEFINE_LAUNCH(template <typename T AFN_COMMA typename M AFN_COMMA int RP>, SpmvGArgs<T AFN_COMMA M AFN_COMMA RP>,
                  (spmv_padded<T, M, RP>), (spmv_padded_g<T, M, RP>))
AFN_DEFINE_LAUNCH(template <typename T AFN_COMMA typename M>, SpmvCsrArgs<T AFN_COMMA M>, (spmv_csr<T, M>),
                  (spmv_csr_g<T, M>))
AFN_DEFINE_LAUNCH(template <typename T>, PcgXrArgs<T>, pcg_xr<T>, pcg_xr_g<T>)
AFN_DEFINE_LAUNCH(template <typename T>, PcgPArgs<T>, pcg_p<T>, pcg_p_g<T>)
AFN_DEFINE_LAUNCH(template <typename T>, ScaleArgs<T>, scale_kernel<T>, scale_g<T>)

__global__ __launch_bounds__(256) void sub_kernel(const double *__restrict__ b,
                                                  const double *__restrict__ y,
                                                  double *__restrict__ r, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    r[i] = b[i] - y[i];
}

__global__ __launch_bounds__(256) void finite_check(const double *__restrict__ a, int64_t n,
                                                    int *flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = a[i];
    if (!(v - v == 0.0)) atomicOr(flag, 1);
}

}  // namespace

int64_t dot_partials(int64_t n)
{
    int64_t b = ceil_div(n, 2048);
    return b < 1 ? 1 : (b > kDotBlocks ? kDotBlocks : b);
}

int64_t gemv_splits(int64_t m, int64_t ncols)
{
    if (m <= 0 || ncols <= 0) return 1;
    int64_t rb = ceil_div(m, 256);
    int64_t s = ceil_div(1024, rb);
    int64_t smax = ceil_div(ncols, 32);
    if (s > smax) s = smax;
    if (s > 512) s = 512;
    return s < 1 ? 1 : s;
}

int64_t gemv_partials(int64_t m, int64_t ncols) { return gemv_splits(m, ncols) * m; }

namespace {

template <typename T>
afn_status dotT(const T *a, int64_t lda, const T *b, int64_t ldb, int64_t n, int nrhs, double *out,
                double *part, hipStream_t s)
{
    const int64_t nb = dot_partials(n);
    const int64_t chunk = ceil_div(n, nb);
    for (int c = 0; c < nrhs; ++c) {
        AFN_TRY(dlaunch(dim3((unsigned)nb), 0, s, DotArgs<T>{a + c * lda, b + c * ldb, n, chunk, part}));
        AFN_TRY(dlaunch(dim3(1), 0, s, SumArgs{part, (int)nb, -1, out + c}));
    }
    return AFN_OK;
}

template <typename T>
afn_status dot_pcgT(const T *a, const T *b, int64_t n, double *sc, PcgDotStep step, double *part,
                    hipStream_t s)
{
    const int64_t nb = dot_partials(n);
    const int64_t chunk = ceil_div(n, nb);
    AFN_TRY(dlaunch(dim3((unsigned)nb), 0, s, DotArgs<T>{a, b, n, chunk, part}));
    return dlaunch(dim3(1), 0, s, SumArgs{part, (int)nb, (int)step, sc});
}

template <typename T, typename M = T>
afn_status gemv_nT(const M *A, int64_t lda, int64_t m, int64_t ncols, const T *x, const T *base,
                   T sign, T *y, T *part, hipStream_t s)
{
    if (m <= 0) return AFN_OK;
    // split counts: the heuristic's, and a half and a quarter of it (the
    // partial buffer holds the heuristic's)
    const int64_t S0 = gemv_splits(m, ncols);
    int64_t cand[3];
    int nc = 0;
    for (int64_t q : {S0, S0 / 2, S0 / 4}) {
        q = q < 1 ? 1 : q;
        bool dup = false;
        for (int c = 0; c < nc; ++c) dup = dup || cand[c] == q;
        if (!dup) cand[nc++] = q;
    }
    auto launch = [&](int c) -> afn_status {
        const int64_t S = cand[c];
        const int64_t chunk = ceil_div(ncols, S);
        AFN_TRY(dlaunch(dim3((unsigned)ceil_div(m, 256), (unsigned)S), 0, s,
                        GemvNArgs<T, M>{A, lda, m, ncols, x, chunk, part}));
        if (S > 32)
            return dlaunch(dim3((unsigned)ceil_div(m, 4)), 0, s, GemvRedArgs<T, true>{part, m, (int)S, sign, base, y});
        return dlaunch(dim3((unsigned)ceil_div(m, 256)), 0, s, GemvRedArgs<T, false>{part, m, (int)S, sign, base, y});
    };
    int pick = 0;
    if ((const void *)base != (const void *)y && (const void *)x != (const void *)y) {
        char shape[96];
        snprintf(shape, sizeof shape, "m%lld_n%lld_%s", (long long)m, (long long)ncols,
                 sizeof(M) == 2 ? "bf16" : (sizeof(T) == 8 ? "f64" : "f32"));
        pick = tune_pick("gemv_n_splits", shape, nc, 0, launch, s);
    }
    return launch(pick);
}

template <typename T, typename M = T>
afn_status gemv_tT(const M *A, int64_t lda, int64_t m, int64_t ncols, const T *x, const T *base,
                   T sign, T *y, hipStream_t s)
{
    if (ncols <= 0) return AFN_OK;
    const size_t lds = sizeof(T) * (size_t)(m > 0 ? m : 1);
    if (ncols >= 4096 && lds <= 32768)
        return dlaunch(dim3((unsigned)ceil_div(ncols, 16)), lds, s, GemvTArgs<T, M, true>{A, lda, m, ncols, x, base, sign, y});
    return dlaunch(dim3((unsigned)ceil_div(ncols, 4)), 0, s, GemvTArgs<T, M, false>{A, lda, m, ncols, x, base, sign, y});
}

template <typename T, typename M = T>
afn_status spmv_gT(const int32_t *cols, const M *gval, int64_t nr, int w, const T *t, T *u,
                   const int32_t *order, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    const dim3 grid((unsigned)ceil_div(nr, 16));
    if (w > 64) return dlaunch(grid, 0, s, SpmvGArgs<T, M, 8>{cols, gval, nr, w, t, u, order});
    return dlaunch(grid, 0, s, SpmvGArgs<T, M, 4>{cols, gval, nr, w, t, u, order});
}

template <typename T, typename M = T>
afn_status spmv_gtT(const int64_t *ptr, const int32_t *idx, const M *val, int64_t nr, const T *u,
                    T *out, const int32_t *order, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    return dlaunch(dim3((unsigned)ceil_div(nr, 16)), 0, s, SpmvCsrArgs<T, M>{ptr, idx, val, nr, u, out, order});
}

template <typename T>
afn_status pcg_xrT(T *x, T *r, const T *p, const T *q, const double *sc, int64_t n, double *part,
                   double *rr_out, hipStream_t s)
{
    const int64_t nb = dot_partials(n);
    const int64_t chunk = ceil_div(n, nb);
    AFN_TRY(dlaunch(dim3((unsigned)nb), 0, s, PcgXrArgs<T>{x, r, p, q, sc, n, chunk, part}));
    return dlaunch(dim3(1), 0, s, SumArgs{part, (int)nb, -1, rr_out});
}

template <typename T>
afn_status pcg_pT(T *p, const T *z, const double *sc, int64_t n, hipStream_t s)
{
    return dlaunch(dim3((unsigned)ceil_div(n, 256)), 0, s, PcgPArgs<T>{p, z, sc, n});
}

}  // namespace

afn_status dot(const double *a, int64_t lda, const double *b, int64_t ldb, int64_t n, int nrhs,
               double *out, double *part, hipStream_t s)
{
    return dotT(a, lda, b, ldb, n, nrhs, out, part, s);
}
afn_status dot(const float *a, int64_t lda, const float *b, int64_t ldb, int64_t n, int nrhs,
               double *out, double *part, hipStream_t s)
{
    return dotT(a, lda, b, ldb, n, nrhs, out, part, s);
}
afn_status gemv_n(const double *A, int64_t lda, int64_t m, int64_t ncols, const double *x,
                  const double *base, double sign, double *y, double *part, hipStream_t s)
{
    return gemv_nT(A, lda, m, ncols, x, base, sign, y, part, s);
}
afn_status gemv_n(const float *A, int64_t lda, int64_t m, int64_t ncols, const float *x,
                  const float *base, float sign, float *y, float *part, hipStream_t s)
{
    return gemv_nT(A, lda, m, ncols, x, base, sign, y, part, s);
}
afn_status gemv_t(const double *A, int64_t lda, int64_t m, int64_t ncols, const double *x,
                  const double *base, double sign, double *y, hipStream_t s)
{
    return gemv_tT(A, lda, m, ncols, x, base, sign, y, s);
}
afn_status gemv_t(const float *A, int64_t lda, int64_t m, int64_t ncols, const float *x,
                  const float *base, float sign, float *y, hipStream_t s)
{
    return gemv_tT(A, lda, m, ncols, x, base, sign, y, s);
}
afn_status spmv_g(const int32_t *cols, const double *gval, int64_t nr, int w, const double *t,
                  double *u, const int32_t *order, hipStream_t s)
{
    return spmv_gT(cols, gval, nr, w, t, u, order, s);
}
afn_status spmv_g(const int32_t *cols, const float *gval, int64_t nr, int w, const float *t, float *u,
                  const int32_t *order, hipStream_t s)
{
    return spmv_gT(cols, gval, nr, w, t, u, order, s);
}
afn_status spmv_gt(const int64_t *ptr, const int32_t *idx, const double *val, int64_t nr,
                   const double *u, double *out, const int32_t *order, hipStream_t s)
{
    return spmv_gtT(ptr, idx, val, nr, u, out, order, s);
}
afn_status spmv_gt(const int64_t *ptr, const int32_t *idx, const float *val, int64_t nr,
                   const float *u, float *out, const int32_t *order, hipStream_t s)
{
    return spmv_gtT(ptr, idx, val, nr, u, out, order, s);
}
afn_status gemv_n(const bf16_t *A, int64_t lda, int64_t m, int64_t ncols, const float *x, const float *base,
                  float sign, float *y, float *part, hipStream_t s)
{
    return gemv_nT<float, bf16_t>(A, lda, m, ncols, x, base, sign, y, part, s);
}
afn_status gemv_t(const bf16_t *A, int64_t lda, int64_t m, int64_t ncols, const float *x, const float *base,
                  float sign, float *y, hipStream_t s)
{
    return gemv_tT<float, bf16_t>(A, lda, m, ncols, x, base, sign, y, s);
}
afn_status spmv_g(const int32_t *cols, const bf16_t *gval, int64_t nr, int w, const float *t, float *u,
                  const int32_t *order, hipStream_t s)
{
    return spmv_gT<float, bf16_t>(cols, gval, nr, w, t, u, order, s);
}
afn_status spmv_gt(const int64_t *ptr, const int32_t *idx, const bf16_t *val, int64_t nr, const float *u,
                   float *out, const int32_t *order, hipStream_t s)
{
    return spmv_gtT<float, bf16_t>(ptr, idx, val, nr, u, out, order, s);
}

namespace {

// FP32 bits to BF16 bits, nearest with ties to even (a NaN stays a NaN).
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const double *__restrict__ a, bf16_t *__restrict__ b,
                                                      int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i].bits = f32_to_bf16_bits((float)a[i]);
}

__global__ __launch_bounds__(256) void round_bf16_kernel(double *__restrict__ a, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = (double)bf16_to_f32(bf16_t{f32_to_bf16_bits((float)a[i])});
}

}  // namespace

afn_status to_bf16_launch(const double *a, bf16_t *b, int64_t n, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, a, b, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status round_bf16_inplace_launch(double *a, int64_t n, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    hipLaunchKernelGGL(round_bf16_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, a, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status pcg_xr_launch(double *x, double *r, const double *p, const double *q, const double *sc,
                         int64_t n, double *part, double *rr_out, hipStream_t s)
{
    return pcg_xrT(x, r, p, q, sc, n, part, rr_out, s);
}
afn_status pcg_xr_launch(float *x, float *r, const float *p, const float *q, const double *sc,
                         int64_t n, double *part, double *rr_out, hipStream_t s)
{
    return pcg_xrT(x, r, p, q, sc, n, part, rr_out, s);
}
afn_status pcg_p_launch(double *p, const double *z, const double *sc, int64_t n, hipStream_t s)
{
    return pcg_pT(p, z, sc, n, s);
}
afn_status pcg_p_launch(float *p, const float *z, const double *sc, int64_t n, hipStream_t s)
{
    return pcg_pT(p, z, sc, n, s);
}

afn_status to_f32_scaled_launch(const double *r, double scale, float *r32, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(to_f32_scaled, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, r, scale, r32, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status axpy_f32_into_f64_launch(double a, const float *e, double *x, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(axpy_f32_into_f64, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, a, e, x, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status to_f32_launch(const double *a, float *b, int64_t n, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    hipLaunchKernelGGL(to_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, a, b, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status permute_gather(const double *src, int64_t lds, double *dst, int64_t ldd,
                          const int32_t *perm, int64_t n, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)ceil_div(n, 256), (unsigned)nrhs), dim3(256), 0, s,
                       src, lds, dst, ldd, perm, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status permute_scatter(const double *src, int64_t lds, double *dst, int64_t ldd,
                           const int32_t *perm, int64_t n, int nrhs, hipStream_t s)
{
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)ceil_div(n, 256), (unsigned)nrhs), dim3(256), 0, s,
                       src, lds, dst, ldd, perm, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status gather_points(const double *X, const int32_t *perm, int64_t n, int d, double *Xp,
                         hipStream_t s)
{
    hipLaunchKernelGGL(gather_points_kernel, dim3((unsigned)ceil_div(n * d, 256)), dim3(256), 0, s, X,
                       perm, n, d, Xp);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status dot_pcg(const double *a, const double *b, int64_t n, double *sc, PcgDotStep step,
                   double *partials, hipStream_t s)
{
    return dot_pcgT(a, b, n, sc, step, partials, s);
}
afn_status dot_pcg(const float *a, const float *b, int64_t n, double *sc, PcgDotStep step,
                   double *partials, hipStream_t s)
{
    return dot_pcgT(a, b, n, sc, step, partials, s);
}

afn_status sub_launch(const double *b, const double *y, double *r, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(sub_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, b, y, r, n);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status scale_launch(double *x, double a, int64_t n, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    return dlaunch(dim3((unsigned)ceil_div(n, 256)), 0, s, ScaleArgs<double>{x, a, n});
}

afn_status scale_launch(float *x, float a, int64_t n, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    return dlaunch(dim3((unsigned)ceil_div(n, 256)), 0, s, ScaleArgs<float>{x, a, n});
}

afn_status finite_launch(const double *a, int64_t n, int *flag, hipStream_t s)
{
    if (n <= 0) return AFN_OK;
    hipLaunchKernelGGL(finite_check, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, a, n, flag);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
