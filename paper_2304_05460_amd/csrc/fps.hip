// Farthest point sampling (Algorithm 6, Section 4.5) on the GPU.
//
// Bit-exact contract with a sequential reading of the algorithm:
//  - squared distances by the fixed chain acc = fma(x_t - y_t, x_t - y_t, acc)
//    over t = 0..d-1 (this file is compiled with -ffp-contract=off);
//  - centroid summed per coordinate over blocks of 256 ascending indices, then
//    over the block sums in ascending order, then divided by n;
//  - arg-min / arg-max ties go to the smallest index; selected points are
//    masked (running distance -1) so they are never chosen again.
// Max/min reductions are order-independent, so the result does not depend on
// how points are spread over workgroups.
//
// Schedule: one launch per selection step.  Every workgroup owns a contiguous
// range of points; step s first reduces the per-workgroup winners of step s-1
// (each workgroup redundantly, same order), updates the running distances of
// its points with the new landmark, and publishes its local winner.
#include <cfloat>
#include <climits>

#include "afn_internal.h"

namespace afn {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxWG = 256;

struct Ws {
    double *dist;      // n running squared distances (-1 = selected)
    double *bsum;      // d * nb block sums
    double *cen;       // d
    double *slot_d;    // 2 * kMaxWG
    int *slot_i;       // 2 * kMaxWG
    double *min_d;     // kMaxWG
    int *min_i;        // kMaxWG
};

__device__ __forceinline__ double sqdist_chain(const double *a, const double *b, int d)
{
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double del = a[t] - b[t];
        acc = __builtin_fma(del, del, acc);
    }
    return acc;
}

// (d1, i1) better than (d2, i2) for an arg-max with ties to the smaller index
__device__ __forceinline__ bool amax_better(double d1, int i1, double d2, int i2)
{
    return d1 > d2 || (d1 == d2 && i1 < i2);
}
__device__ __forceinline__ bool amin_better(double d1, int i1, double d2, int i2)
{
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

template <bool MAX>
__device__ void block_reduce(double &bd, int &bi)
{
    __shared__ double sd[kThreads / 64];
    __shared__ int si[kThreads / 64];
    for (int off = 32; off > 0; off >>= 1) {
        double od = __shfl_xor(bd, off, 64);
        int oi = __shfl_xor(bi, off, 64);
        bool take = MAX ? amax_better(od, oi, bd, bi) : amin_better(od, oi, bd, bi);
        if (take) { bd = od; bi = oi; }
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) { sd[wid] = bd; si[wid] = bi; }
    __syncthreads();
    bd = sd[0];
    bi = si[0];
    for (int w = 1; w < kThreads / 64; ++w) {
        bool take = MAX ? amax_better(sd[w], si[w], bd, bi) : amin_better(sd[w], si[w], bd, bi);
        if (take) { bd = sd[w]; bi = si[w]; }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void centroid_blocks(const double *__restrict__ X, int64_t n,
                                                            int d, double *__restrict__ bsum,
                                                            int64_t nb)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nb * d) return;
    int t = (int)(e / nb);
    int64_t b = e - (int64_t)t * nb;
    int64_t j0 = b * 256, j1 = j0 + 256 < n ? j0 + 256 : n;
    double s = 0.0;
    for (int64_t j = j0; j < j1; ++j) s += X[j * d + t];
    bsum[(int64_t)t * nb + b] = s;
}

__global__ void centroid_final(const double *__restrict__ bsum, int64_t nb, int64_t n, int d,
                               double *__restrict__ cen)
{
    int t = threadIdx.x;
    if (t >= d) return;
    double total = 0.0;
    for (int64_t b = 0; b < nb; ++b) total += bsum[(int64_t)t * nb + b];
    cen[t] = total / (double)n;
}

// Per-workgroup arg-min of the squared distance to the centroid; also sets the
// running distances to +inf.
__global__ __launch_bounds__(kThreads) void nearest_centroid(const double *__restrict__ X, int64_t n,
                                                             int d, const double *__restrict__ cen,
                                                             double *__restrict__ dist,
                                                             int64_t chunk, double *min_d, int *min_i)
{
    __shared__ double sc[kMaxD];
    if (threadIdx.x < d) sc[threadIdx.x] = cen[threadIdx.x];
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    double bd = DBL_MAX;
    int bi = INT_MAX;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
        dist[j] = __builtin_inf();
        double dj = sqdist_chain(X + j * d, sc, d);
        if (amin_better(dj, (int)j, bd, bi)) { bd = dj; bi = (int)j; }
    }
    block_reduce<false>(bd, bi);
    if (threadIdx.x == 0) { min_d[blockIdx.x] = bd; min_i[blockIdx.x] = bi; }
}

// First landmark = overall arg-min; seeds the step-0 winner slots.
__global__ __launch_bounds__(kThreads) void fps_first(const double *min_d, const int *min_i, int nwg,
                                                      int64_t n, double *slot_d, int *slot_i,
                                                      int *err)
{
    double bd = DBL_MAX;
    int bi = INT_MAX;
    for (int g = threadIdx.x; g < nwg; g += kThreads)
        if (amin_better(min_d[g], min_i[g], bd, bi)) { bd = min_d[g]; bi = min_i[g]; }
    block_reduce<false>(bd, bi);
    if (bi < 0 || bi >= n) { if (threadIdx.x == 0) *err = 1; bi = 0; }
    for (int g = threadIdx.x; g < kMaxWG; g += kThreads) {
        slot_d[g] = g == 0 ? __builtin_inf() : -__builtin_inf();
        slot_i[g] = g == 0 ? bi : INT_MAX;
    }
}

// Step s: winner of step s-1 -> idx[s-1]; if !final, update distances with it
// and publish this workgroup's arg-max for step s.
__global__ __launch_bounds__(kThreads) void fps_step(const double *__restrict__ X, int64_t n, int d,
                                                     double *__restrict__ dist, int64_t chunk,
                                                     int nwg, const double *prev_d,
                                                     const int *prev_i, double *next_d,
                                                     int *next_i, int32_t *idx, double *seld,
                                                     int s, int final_step, int *err)
{
    __shared__ double sw[kMaxD];
    double wd = -__builtin_inf();
    int wi = INT_MAX;
    for (int g = threadIdx.x; g < nwg; g += kThreads)
        if (amax_better(prev_d[g], prev_i[g], wd, wi)) { wd = prev_d[g]; wi = prev_i[g]; }
    block_reduce<true>(wd, wi);
    if (wi < 0 || wi >= n) {      // cannot happen for finite inputs; keep accesses in bounds
        if (threadIdx.x == 0) *err = 1;
        wi = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        idx[s - 1] = wi;
        if (seld) seld[s - 1] = wd;
    }
    if (final_step) return;
    if (threadIdx.x < d) sw[threadIdx.x] = X[(int64_t)wi * d + threadIdx.x];
    __syncthreads();
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    double bd = -__builtin_inf();
    int bi = INT_MAX;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
        double cur = dist[j];
        if (j == wi) {
            cur = -1.0;
            dist[j] = cur;
        } else if (cur >= 0.0) {
            double dj = sqdist_chain(X + j * d, sw, d);
            if (dj < cur) {
                cur = dj;
                dist[j] = cur;
            }
        }
        if (amax_better(cur, (int)j, bd, bi)) { bd = cur; bi = (int)j; }
    }
    block_reduce<true>(bd, bi);
    if (threadIdx.x == 0) { next_d[blockIdx.x] = bd; next_i[blockIdx.x] = bi; }
}

Ws carve(void *work, int64_t n, int d)
{
    Ws w;
    char *p = (char *)work;
    auto take = [&](size_t bytes) {
        char *q = p;
        p += round_up((int64_t)bytes, 256);
        return q;
    };
    int64_t nb = ceil_div(n, 256);
    w.dist = (double *)take(sizeof(double) * n);
    w.bsum = (double *)take(sizeof(double) * nb * kMaxD);
    w.cen = (double *)take(sizeof(double) * kMaxD);
    w.slot_d = (double *)take(sizeof(double) * 2 * kMaxWG);
    w.slot_i = (int *)take(sizeof(int) * 2 * kMaxWG);
    w.min_d = (double *)take(sizeof(double) * kMaxWG);
    w.min_i = (int *)take(sizeof(int) * kMaxWG);
    (void)d;
    return w;
}

}  // namespace

size_t fps_workspace_bytes(int64_t n)
{
    int64_t nb = ceil_div(n, 256);
    return (size_t)(round_up(8 * n, 256) + round_up(8 * nb * kMaxD, 256) + round_up(8 * kMaxD, 256) +
                    round_up(16 * kMaxWG, 256) + round_up(8 * kMaxWG, 256) +
                    round_up(8 * kMaxWG, 256) + round_up(4 * kMaxWG, 256) + 256);
}

// First landmark (nearest to the centroid) into the step-0 slots.
afn_status fps_start(const double *X, int64_t n, int d, void *work, hipStream_t s, int *err)
{
    Ws w = carve(work, n, d);
    const int64_t nb = ceil_div(n, 256);
    const int nwg = (int)(ceil_div(n, kThreads) < kMaxWG ? ceil_div(n, kThreads) : kMaxWG);
    const int64_t chunk = ceil_div(n, nwg);
    hipLaunchKernelGGL(centroid_blocks, dim3((unsigned)ceil_div(nb * d, kThreads)), dim3(kThreads), 0,
                       s, X, n, d, w.bsum, nb);
    hipLaunchKernelGGL(centroid_final, dim3(1), dim3(64), 0, s, w.bsum, nb, n, d, w.cen);
    hipLaunchKernelGGL(nearest_centroid, dim3(nwg), dim3(kThreads), 0, s, X, n, d, w.cen, w.dist,
                       chunk, w.min_d, w.min_i);
    hipLaunchKernelGGL(fps_first, dim3(1), dim3(kThreads), 0, s, w.min_d, w.min_i, nwg, n, w.slot_d,
                       w.slot_i, err);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

// Selection steps st0+1 .. st1 (step st writes idx[st-1]); the step k_total
// only reports its winner.  A later call resumes from st1.
afn_status fps_advance(const double *X, int64_t n, int d, int st0, int st1, int k_total, int32_t *idx,
                       double *seld, void *work, hipStream_t s, int *err)
{
    Ws w = carve(work, n, d);
    const int nwg = (int)(ceil_div(n, kThreads) < kMaxWG ? ceil_div(n, kThreads) : kMaxWG);
    const int64_t chunk = ceil_div(n, nwg);
    for (int st = st0 + 1; st <= st1; ++st) {
        const int pb = (st - 1) & 1, nbuf = st & 1;
        const int fin = st == k_total ? 1 : 0;
        hipLaunchKernelGGL(fps_step, dim3(fin ? 1 : nwg), dim3(kThreads), 0, s, X, n, d, w.dist, chunk,
                           nwg, w.slot_d + pb * kMaxWG, w.slot_i + pb * kMaxWG,
                           w.slot_d + nbuf * kMaxWG, w.slot_i + nbuf * kMaxWG, idx, seld, st, fin, err);
    }
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status fps(const double *X, int64_t n, int d, int k, int32_t *idx, double *seld, void *work,
               hipStream_t s, int *err)
{
    if (k <= 0) return AFN_OK;
    AFN_TRY(fps_start(X, n, d, work, s, err));
    return fps_advance(X, n, d, 0, k, k, idx, seld, work, s, err);
}

namespace {

__global__ __launch_bounds__(256) void mark_selected(const int32_t *idx, int k, int64_t n, int *sel,
                                                     int32_t *perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k) return;
    int j = idx[i];
    if (j >= 0 && j < n) sel[j] = 1;
    perm[i] = j;
}

// Unselected indices in ascending order after the k landmarks (one workgroup).
__global__ __launch_bounds__(1024) void compact_rest(const int *sel, int64_t n, int k, int32_t *perm)
{
    __shared__ int part[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t j = base + threadIdx.x;
        const int f = (j < n && !sel[j]) ? 1 : 0;
        part[threadIdx.x] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        if (f) {
            int64_t pos = (int64_t)k + carry + part[threadIdx.x] - 1;
            if (pos < n) perm[pos] = (int32_t)j;
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
}

}  // namespace

afn_status landmark_permutation(const int32_t *idx, int k, int64_t n, int32_t *perm, int *sel,
                                hipStream_t s)
{
    AFN_HIP(hipMemsetAsync(sel, 0, sizeof(int) * (size_t)n, s));
    if (k > 0)
        hipLaunchKernelGGL(mark_selected, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, idx, k, n,
                           sel, perm);
    hipLaunchKernelGGL(compact_rest, dim3(1), dim3(1024), 0, s, sel, n, k, perm);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
