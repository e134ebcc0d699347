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
// its points with the new landmark, and publishes its local winner.  Point
// sets whose coordinates fit in LDS run a range of steps in one workgroup
// instead (fps_lds).
#include <cfloat>
#include <climits>
#include <type_traits>

#include "afn_internal.h"

namespace afn {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxWG = 256;
constexpr int kPubD = 8;       // d up to which slots also carry their point's coordinates

struct Ws {
    double *dist;      // n running squared distances (-1 = selected)
    double *bsum;      // d * nb block sums
    double *cen;       // d
    double *slot_d;    // 2 * kMaxWG
    int *slot_i;       // 2 * kMaxWG
    double *min_d;     // kMaxWG
    int *min_i;        // kMaxWG
    double *slot_x;    // 2 * kMaxWG * kPubD: coordinates of each slot's point (d <= kPubD)
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
                                                      const double *X, int d, double *slot_x, int *err)
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
    if (d <= kPubD && (int)threadIdx.x < d) slot_x[threadIdx.x] = X[(int64_t)bi * d + threadIdx.x];
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

// Step s as fps_step, for d = D <= kPubD and at most PT points per thread:
// the thread's points (running distances and coordinates) and the previous
// slots with their points' coordinates are loaded first, none of them
// waiting for the previous winner; the thread holding the winning slot
// passes its coordinates on through LDS, and the thread holding this
// workgroup's winner publishes the winner's coordinates with its slot.
template <int D, int PT>
__global__ __launch_bounds__(kThreads) void fps_step_pf(const double *__restrict__ X, int64_t n,
                                                        double *__restrict__ dist, int64_t chunk, int nwg,
                                                        const double *prev_d, const int *prev_i,
                                                        const double *prev_x, double *next_d, int *next_i,
                                                        double *next_x, int32_t *idx, double *seld, int s,
                                                        int final_step, int *err)
{
    __shared__ double sw[D];
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    double cur[PT], xj[PT][D];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int64_t j = j0 + tid + (int64_t)kThreads * u;
        const bool in = !final_step && j < j1;
        cur[u] = in ? dist[j] : -1.0;
#pragma unroll
        for (int t = 0; t < D; ++t) xj[u][t] = in ? X[j * D + t] : 0.0;
    }
    double wd = -__builtin_inf(), px[D];
    int wi = INT_MAX;
    if (tid < nwg) {
        wd = prev_d[tid];
        wi = prev_i[tid];
#pragma unroll
        for (int t = 0; t < D; ++t) px[t] = prev_x[tid * D + t];
    }
    const int pi = wi;
    block_reduce<true>(wd, wi);
    const bool bad = wi < 0 || wi >= n;
    if (bad) {                    // cannot happen for finite inputs; keep accesses in bounds
        if (tid == 0) *err = 1;
        wi = 0;
    }
    if (blockIdx.x == 0 && tid == 0) {
        idx[s - 1] = wi;
        if (seld) seld[s - 1] = wd;
    }
    if (final_step) return;
    if (!bad) {
        if (tid < nwg && pi == wi) {
#pragma unroll
            for (int t = 0; t < D; ++t) sw[t] = px[t];
        }
    } else if (tid < D) {
        sw[tid] = X[tid];
    }
    __syncthreads();
    double sx[D];
#pragma unroll
    for (int t = 0; t < D; ++t) sx[t] = sw[t];
    double bd = -__builtin_inf();
    int bi = INT_MAX;
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int64_t j = j0 + tid + (int64_t)kThreads * u;
        if (j >= j1) continue;
        double c = cur[u];
        if (j == wi) {
            c = -1.0;
            dist[j] = c;
        } else if (c >= 0.0) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const double del = xj[u][t] - sx[t];
                acc = __builtin_fma(del, del, acc);
            }
            if (acc < c) {
                c = acc;
                dist[j] = c;
            }
        }
        cur[u] = c;
        if (amax_better(c, (int)j, bd, bi)) { bd = c; bi = (int)j; }
    }
    block_reduce<true>(bd, bi);
    if (tid == 0) { next_d[blockIdx.x] = bd; next_i[blockIdx.x] = bi; }
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int64_t j = j0 + tid + (int64_t)kThreads * u;
        if (j < j1 && j == bi) {
#pragma unroll
            for (int t = 0; t < D; ++t) next_x[blockIdx.x * D + t] = xj[u][t];
        }
    }
}

// Steps st0+1 .. st1 in one workgroup, for point sets whose coordinates fit
// in LDS (n d <= kLdsFpsMax, n <= 16 kLdsThreads): the coordinates copied
// into LDS (read back for the selected point only), each thread's points
// (j = tid + kLdsThreads u) with their coordinates (D > 0, d = D) and running
// distances in registers, one block arg-max per step (wave shuffles, then the
// eight wave winners in a slot pair chosen by step parity, so one barrier per
// step).  Same distances, masking and tie rule as fps_step; it starts from
// the slots the previous step published (nwg of them) and, unless its last
// step is the final one, publishes its winner as slot 0 of the next buffer
// (the others empty), so launches of either kind can follow each other.
// D = 0: any d, each point's coordinates read from LDS.
constexpr int kLdsThreads = 512;
constexpr int kLdsFpsMax = 20224;   // doubles of coordinates in LDS (158 KiB)

template <int PT, int D>
__global__ __launch_bounds__(kLdsThreads) void fps_lds(const double *__restrict__ X, int n, int d,
                                                       double *__restrict__ dist, int nwg,
                                                       const double *prev_d, const int *prev_i,
                                                       double *next_d, int *next_i, double *next_x,
                                                       int32_t *idx, double *seld, int st0, int st1,
                                                       int k_total, int *err)
{
    extern __shared__ double xs[];          // xs[j * d + t], as X
    __shared__ double wdd[2][kLdsThreads / 64];
    __shared__ int wii[2][kLdsThreads / 64];
    constexpr int DR = D > 0 ? D : 1;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // eight loads in flight per thread (clamped in-range addresses, the stores
    // masked): one load per iteration would wait out the latency each time,
    // and every launch of a chunked run fills LDS again
    const int nd = n * d;
    for (int e0 = 0; e0 < nd; e0 += 8 * kLdsThreads) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + tid + kLdsThreads * u;
            v[u] = X[e < nd ? e : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + tid + kLdsThreads * u;
            if (e < nd) xs[e] = v[u];
        }
    }
    double cur[PT], own[PT][DR];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int j = tid + kLdsThreads * u;
        cur[u] = j < n ? dist[j] : -__builtin_inf();
        if constexpr (D > 0) {
#pragma unroll
            for (int t = 0; t < D; ++t) own[u][t] = j < n ? X[(int64_t)j * D + t] : 0.0;
        }
    }
    // the winner published by step st0
    double wd = -__builtin_inf();
    int wi = INT_MAX;
    for (int g = tid; g < nwg; g += kLdsThreads)
        if (amax_better(prev_d[g], prev_i[g], wd, wi)) { wd = prev_d[g]; wi = prev_i[g]; }
    auto reduce = [&](int par) {
        for (int off = 32; off > 0; off >>= 1) {
            const double od = __shfl_xor(wd, off, 64);
            const int oi = __shfl_xor(wi, off, 64);
            if (amax_better(od, oi, wd, wi)) { wd = od; wi = oi; }
        }
        if (lane == 0) { wdd[par][wv] = wd; wii[par][wv] = wi; }
        __syncthreads();
        wd = wdd[par][0];
        wi = wii[par][0];
        for (int w = 1; w < kLdsThreads / 64; ++w)
            if (amax_better(wdd[par][w], wii[par][w], wd, wi)) { wd = wdd[par][w]; wi = wii[par][w]; }
    };
    reduce(0);     // also orders the coordinate stores before the first reads
    int par = 1;
    for (int st = st0 + 1; st <= st1; ++st) {
        if (wi < 0 || wi >= n) {      // cannot happen for finite inputs; keep accesses in bounds
            if (tid == 0) *err = 1;
            wi = 0;
        }
        if (tid == 0) {
            idx[st - 1] = wi;
            if (seld) seld[st - 1] = wd;
        }
        if (st == k_total) break;
        const int sel = wi;
        double sx[DR];
        if constexpr (D > 0) {
#pragma unroll
            for (int t = 0; t < D; ++t) sx[t] = xs[sel * D + t];
        }
        wd = -__builtin_inf();
        wi = INT_MAX;
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int j = tid + kLdsThreads * u;
            if (j >= n) continue;
            double c = cur[u];
            if (j == sel) {
                c = -1.0;
            } else if (c >= 0.0) {
                double acc = 0.0;
                if constexpr (D > 0) {
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        const double del = own[u][t] - sx[t];
                        acc = __builtin_fma(del, del, acc);
                    }
                } else {
                    for (int t = 0; t < d; ++t) {
                        const double del = xs[j * d + t] - xs[sel * d + t];
                        acc = __builtin_fma(del, del, acc);
                    }
                }
                if (acc < c) c = acc;
            }
            cur[u] = c;
            if (amax_better(c, j, wd, wi)) { wd = c; wi = j; }
        }
        reduce(par);
        par ^= 1;
        if (st == st1) {
            // published for the next call, which starts at step st1 + 1
            for (int g = tid; g < nwg; g += kLdsThreads) {
                next_d[g] = g == 0 ? wd : -__builtin_inf();
                next_i[g] = g == 0 ? wi : INT_MAX;
            }
            if (d <= kPubD && tid < d) next_x[tid] = wi >= 0 && wi < n ? xs[wi * d + tid] : 0.0;
        }
    }
#pragma unroll
    for (int u = 0; u < PT; ++u) {
        const int j = tid + kLdsThreads * u;
        if (j < n) dist[j] = cur[u];
    }
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
    w.slot_x = (double *)take(sizeof(double) * 2 * kMaxWG * kPubD);
    (void)d;
    return w;
}

}  // namespace

size_t fps_workspace_bytes(int64_t n)
{
    int64_t nb = ceil_div(n, 256);
    return (size_t)(round_up(8 * n, 256) + round_up(8 * nb * kMaxD, 256) + round_up(8 * kMaxD, 256) +
                    round_up(16 * kMaxWG, 256) + round_up(8 * kMaxWG, 256) +
                    round_up(8 * kMaxWG, 256) + round_up(4 * kMaxWG, 256) +
                    round_up(8 * 2 * kMaxWG * kPubD, 256) + 256);
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
                       w.slot_i, X, d, w.slot_x, err);
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
    if (st1 <= st0) return AFN_OK;
    if (n * d <= kLdsFpsMax && n <= 16 * kLdsThreads && st1 - st0 > 1) {
        // one workgroup for the whole range; the slots of step st0 are in
        // buffer st0 & 1 and the winner of step st1 goes to buffer st1 & 1
        const size_t lds = sizeof(double) * (size_t)(n * d);
        const int pb = st0 & 1, nbuf = st1 & 1;
        auto go = [&](auto kern) -> afn_status {
            // one value for every launch: setups on other threads launch the
            // same function with other sizes at the same time
            AFN_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)(sizeof(double) * kLdsFpsMax)));
            hipLaunchKernelGGL(kern, dim3(1), dim3(kLdsThreads), lds, s, X, (int)n, d, w.dist, nwg,
                               w.slot_d + pb * kMaxWG, w.slot_i + pb * kMaxWG, w.slot_d + nbuf * kMaxWG,
                               w.slot_i + nbuf * kMaxWG, w.slot_x + nbuf * kMaxWG * kPubD, idx, seld,
                               st0, st1, k_total, err);
            return AFN_OK;
        };
        // points per thread: 4, 8 or 16; registers for 64 coordinates at most
        auto by_n = [&](auto dtag) -> afn_status {
            constexpr int D = decltype(dtag)::value;
            if (n <= 4 * kLdsThreads) return go(fps_lds<4, D>);
            if constexpr (8 * D <= 64) {
                if (n <= 8 * kLdsThreads) return go(fps_lds<8, D>);
            }
            if constexpr (16 * D <= 64) return go(fps_lds<16, D>);
            return go(fps_lds<16, 0>);
        };
        switch (d) {
        case 1: AFN_TRY(by_n(std::integral_constant<int, 1>{})); break;
        case 2: AFN_TRY(by_n(std::integral_constant<int, 2>{})); break;
        case 3: AFN_TRY(by_n(std::integral_constant<int, 3>{})); break;
        case 4: AFN_TRY(by_n(std::integral_constant<int, 4>{})); break;
        case 5: AFN_TRY(by_n(std::integral_constant<int, 5>{})); break;
        case 6: AFN_TRY(by_n(std::integral_constant<int, 6>{})); break;
        case 7: AFN_TRY(by_n(std::integral_constant<int, 7>{})); break;
        case 8: AFN_TRY(by_n(std::integral_constant<int, 8>{})); break;
        default:
            if (n <= 4 * kLdsThreads) AFN_TRY(go(fps_lds<4, 0>));
            else AFN_TRY(go(fps_lds<16, 0>));
        }
        AFN_HIP(hipGetLastError());
        return AFN_OK;
    }
    // d <= kPubD and at most 4 points per thread: the prefetching step
    auto pf = [&](auto dtag) -> bool {
        constexpr int D = decltype(dtag)::value;
        auto run = [&](auto kern) {
            for (int st = st0 + 1; st <= st1; ++st) {
                const int pb = (st - 1) & 1, nbuf = st & 1;
                const int fin = st == k_total ? 1 : 0;
                hipLaunchKernelGGL(kern, dim3(fin ? 1 : nwg), dim3(kThreads), 0, s, X, n, w.dist, chunk,
                                   nwg, w.slot_d + pb * kMaxWG, w.slot_i + pb * kMaxWG,
                                   w.slot_x + pb * kMaxWG * kPubD, w.slot_d + nbuf * kMaxWG,
                                   w.slot_i + nbuf * kMaxWG, w.slot_x + nbuf * kMaxWG * kPubD, idx, seld,
                                   st, fin, err);
            }
        };
        if (chunk <= kThreads) run(fps_step_pf<D, 1>);
        else if (chunk <= 4 * kThreads) run(fps_step_pf<D, 4>);
        else return false;
        return true;
    };
    bool done = false;
    switch (d) {
    case 1: done = pf(std::integral_constant<int, 1>{}); break;
    case 2: done = pf(std::integral_constant<int, 2>{}); break;
    case 3: done = pf(std::integral_constant<int, 3>{}); break;
    case 4: done = pf(std::integral_constant<int, 4>{}); break;
    case 5: done = pf(std::integral_constant<int, 5>{}); break;
    case 6: done = pf(std::integral_constant<int, 6>{}); break;
    case 7: done = pf(std::integral_constant<int, 7>{}); break;
    case 8: done = pf(std::integral_constant<int, 8>{}); break;
    default: break;
    }
    for (int st = st0 + 1; !done && st <= st1; ++st) {
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
