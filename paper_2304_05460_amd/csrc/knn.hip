// FSAI sparsity pattern (Section 3.1): row p of the non-landmark points X_r
// holds the w-1 nearest earlier-numbered points q < p -- keys (squared
// distance, q) compared lexicographically -- plus p itself, columns ascending
// (p last).  Rows p < w-1 hold all p predecessors.
//
// One wavefront per query p.  The 64 lanes evaluate 64 candidates at a time
// (squared distance by the fixed fma chain, -ffp-contract=off, so keys are
// bit-identical to a sequential evaluation); candidates whose key beats the
// current (w-1)-th best enter a sorted list held NE entries per lane (entry
// 64 e + l in lane l; NE = 1 for w <= 64, 2 for w <= 128), by a wave-wide
// rank-and-shift.  The final set is unique, so the pattern does not
// depend on the candidate order.  Queries are dealt round-robin to waves,
// which balances the O(p) cost per query.
//
// With a spatial (Hilbert) order of Xr, d <= 8: queries are taken in that
// order, the order is cut into 64-point tiles with their bounding boxes and
// smallest index, and a query with p >= nr/4 first takes the candidates of
// its own tile and the two on either side, then every other tile whose
// smallest index is below p and whose box is not farther than the current
// (w-1)-th key (the box distance, by the same fma chain over per-coordinate
// gaps, is a lower bound of every candidate's key: rounding is monotone).
// A query whose list is not full after those five tiles, and every query
// with p < nr/4, scans all its predecessors as above.  Both give the same
// unique set.
#include <climits>

#include "afn_internal.h"

namespace afn {
namespace {

__device__ __forceinline__ bool key_less(double d1, int q1, double d2, int q2)
{
    return d1 < d2 || (d1 == d2 && q1 < q2);
}

// The sorted list of a query: NE entries per lane (ld, lq), cnt entries, and
// the key of the (w-1)-th entry once the list is full.
template <int NE>
struct KnnList {
    double ld[NE];
    int lq[NE];
    int cnt = 0;
    double thr_d = __builtin_inf();
    int thr_q = INT_MAX;
    __device__ KnnList()
    {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            ld[e] = __builtin_inf();
            lq[e] = INT_MAX;
        }
    }
};

// Offer this lane's candidate (dq, qi) if pass; the wave's passing candidates
// enter one at a time, lowest lane first.  want <= 64 NE.
template <int NE>
__device__ __forceinline__ void knn_offer(KnnList<NE> &L, int want, bool pass, double dq, int qi)
{
    const int lane = threadIdx.x & 63;
    pass = pass && (L.cnt < want || key_less(dq, qi, L.thr_d, L.thr_q));
    uint64_t mask = __ballot(pass);
    while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        const double nd = __shfl(dq, src, 64);
        const int nq = __shfl(qi, src, 64);
        int pos = 0;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const bool lt = 64 * e + lane < L.cnt && key_less(L.ld[e], L.lq[e], nd, nq);
            pos += __popcll(__ballot(lt));
        }
        // entries at positions >= pos move up by one; position 64 e takes the
        // old entry 64 e - 1 (lane 63 of the entry below, read before it moves)
#pragma unroll
        for (int e = NE - 1; e >= 0; --e) {
            double upd = __shfl_up(L.ld[e], 1, 64);
            int upq = __shfl_up(L.lq[e], 1, 64);
            if (e > 0) {
                const double bd = __shfl(L.ld[e > 0 ? e - 1 : 0], 63, 64);
                const int bq = __shfl(L.lq[e > 0 ? e - 1 : 0], 63, 64);
                if (lane == 0) { upd = bd; upq = bq; }
            }
            const int idx = 64 * e + lane;
            if (idx > pos) { L.ld[e] = upd; L.lq[e] = upq; }
            if (idx == pos) { L.ld[e] = nd; L.lq[e] = nq; }
            if (idx >= want) { L.ld[e] = __builtin_inf(); L.lq[e] = INT_MAX; }
        }
        L.cnt = L.cnt + 1 < want ? L.cnt + 1 : want;
        mask &= mask - 1;
        if (L.cnt == want) {
            const int te = (want - 1) >> 6, tl = (want - 1) & 63;
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                const double td = __shfl(L.ld[e], tl, 64);
                const int tq = __shfl(L.lq[e], tl, 64);
                if (e == te) { L.thr_d = td; L.thr_q = tq; }
            }
            mask &= __ballot(pass && key_less(dq, qi, L.thr_d, L.thr_q));
        }
    }
}

// Row p of the pattern from the final list: the cnt neighbours in ascending
// index (each entry's rank among them), then p, then -1 up to w.
template <int NE>
__device__ __forceinline__ void knn_write_row(const KnnList<NE> &L, int64_t p, int w, int32_t *__restrict__ cols)
{
    const int lane = threadIdx.x & 63;
    int rank[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) rank[e] = 0;
#pragma unroll
    for (int e2 = 0; e2 < NE; ++e2) {
        const int lim = L.cnt - 64 * e2;
        for (int j = 0; j < lim && j < 64; ++j) {
            const int oq = __shfl(L.lq[e2], j, 64);
#pragma unroll
            for (int e = 0; e < NE; ++e) rank[e] += (oq < L.lq[e]) ? 1 : 0;
        }
    }
    int32_t *row = cols + p * w;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const int idx = 64 * e + lane;
        if (idx < L.cnt) row[rank[e]] = L.lq[e];
        if (idx > L.cnt && idx < w) row[idx] = -1;
    }
    if (lane == 0) row[L.cnt] = (int32_t)p;
}

// D >= d: the query's coordinates sit in registers, zero-padded to D; the
// candidate's coordinates beyond d are taken as zero too, so the squared
// distance is the fma chain over t = 0..d-1 followed by additions of +0.
template <int D, int NE>
__global__ __launch_bounds__(256) void knn_pred(const double *__restrict__ Xr, int64_t nr, int d,
                                                int w, int32_t *__restrict__ cols)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int want = w - 1;
    for (int64_t p = wave; p < nr; p += nwaves) {
        double xp[D];
#pragma unroll
        for (int t = 0; t < D; ++t) xp[t] = t < d ? Xr[p * d + t] : 0.0;
        KnnList<NE> L;
        if (want > 0) {
            for (int64_t q0 = 0; q0 < p; q0 += 64) {
                const int64_t q = q0 + lane;
                const bool valid = q < p;
                double dq = __builtin_inf();
                if (valid) {
                    double acc = 0.0;
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        if (t < d) {
                            const double del = xp[t] - Xr[q * d + t];
                            acc = __builtin_fma(del, del, acc);
                        }
                    }
                    dq = acc;
                }
                knn_offer(L, want, valid, dq, (int)q);
            }
        }
        knn_write_row(L, p, w, cols);
    }
}

// Tile t of the ordered points: box[(t*d + c)*2 + {0,1}] = min / max of
// coordinate c, tmin[t] = smallest index.
__global__ __launch_bounds__(256) void knn_tile_boxes(const double *__restrict__ Xr, int64_t nr, int d,
                                                      const int32_t *__restrict__ order, int64_t ntiles,
                                                      double *__restrict__ box, int32_t *__restrict__ tmin)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntiles * (d + 1)) return;
    const int64_t t = e / (d + 1);
    const int c = (int)(e - t * (d + 1));
    const int64_t j0 = t * 64, j1 = j0 + 64 < nr ? j0 + 64 : nr;
    if (c == d) {
        int32_t m = INT_MAX;
        for (int64_t j = j0; j < j1; ++j) m = order[j] < m ? order[j] : m;
        tmin[t] = m;
        return;
    }
    double lo = __builtin_inf(), hi = -__builtin_inf();
    for (int64_t j = j0; j < j1; ++j) {
        const double x = Xr[(int64_t)order[j] * d + c];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
    box[(t * d + c) * 2] = lo;
    box[(t * d + c) * 2 + 1] = hi;
}

template <int D, int NE>
__global__ __launch_bounds__(256) void knn_pred_tiles(const double *__restrict__ Xr, int64_t nr, int d, int w,
                                                      const int32_t *__restrict__ order,
                                                      const double *__restrict__ box,
                                                      const int32_t *__restrict__ tmin, int64_t ntiles,
                                                      int32_t *__restrict__ cols)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int want = w - 1;
    for (int64_t j = wave; j < nr; j += nwaves) {
        const int64_t p = order[j];
        double xp[D];
#pragma unroll
        for (int t = 0; t < D; ++t) xp[t] = t < d ? Xr[p * d + t] : 0.0;
        auto key = [&](int64_t q) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                if (t < d) {
                    const double del = xp[t] - Xr[q * d + t];
                    acc = __builtin_fma(del, del, acc);
                }
            }
            return acc;
        };
        KnnList<NE> L;
        auto scan_tile = [&](int64_t tt) {
            const int64_t jj = tt * 64 + lane;
            const int64_t q = jj < nr ? (int64_t)order[jj] : nr;
            const bool valid = q < p;
            knn_offer(L, want, valid, valid ? key(q) : __builtin_inf(), (int)q);
        };
        bool brute = want == 0 || 4 * p < nr;
        const int64_t T = j / 64;
        if (!brute) {
            for (int64_t tt = T - 2; tt <= T + 2; ++tt)
                if (tt >= 0 && tt < ntiles) scan_tile(tt);
            brute = L.cnt < want;
        }
        if (!brute) {
            for (int64_t t0 = 0; t0 < ntiles; t0 += 64) {
                const int64_t t = t0 + lane;
                double g2 = __builtin_inf();
                if (t < ntiles && (t < T - 2 || t > T + 2) && tmin[t] < p) {
                    double acc = 0.0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        if (c < d) {
                            const double lo = box[(t * d + c) * 2], hi = box[(t * d + c) * 2 + 1];
                            const double gap = xp[c] < lo ? lo - xp[c] : (xp[c] > hi ? xp[c] - hi : 0.0);
                            acc = __builtin_fma(gap, gap, acc);
                        }
                    }
                    g2 = acc;
                }
                uint64_t mask = __ballot(g2 <= L.thr_d);
                while (mask) {
                    const int src = __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1;
                    // the threshold may have dropped since the ballot
                    if (__shfl(g2, src, 64) <= L.thr_d) scan_tile(t0 + src);
                }
            }
        } else if (want > 0) {
            L = KnnList<NE>();
            for (int64_t q0 = 0; q0 < p; q0 += 64) {
                const int64_t q = q0 + lane;
                const bool valid = q < p;
                knn_offer(L, want, valid, valid ? key(q) : __builtin_inf(), (int)q);
            }
        }
        knn_write_row(L, p, w, cols);
    }
}

template <int NE>
void launch_tiles(dim3 grid, dim3 block, hipStream_t s, const double *Xr, int64_t nr, int d, int w,
                  const int32_t *order, const double *box, const int32_t *tmin, int64_t nt, int32_t *cols)
{
    switch (d) {
        case 1: hipLaunchKernelGGL((knn_pred_tiles<1, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        case 2: hipLaunchKernelGGL((knn_pred_tiles<2, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        case 3: hipLaunchKernelGGL((knn_pred_tiles<3, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        case 4: hipLaunchKernelGGL((knn_pred_tiles<4, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        case 5: hipLaunchKernelGGL((knn_pred_tiles<5, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        case 6: hipLaunchKernelGGL((knn_pred_tiles<6, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        case 7: hipLaunchKernelGGL((knn_pred_tiles<7, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
        default: hipLaunchKernelGGL((knn_pred_tiles<8, NE>), grid, block, 0, s, Xr, nr, d, w, order, box, tmin, nt, cols); break;
    }
}

template <int NE>
void launch_brute(dim3 grid, dim3 block, hipStream_t s, const double *Xr, int64_t nr, int d, int w, int32_t *cols)
{
    switch (d) {
        case 1: hipLaunchKernelGGL((knn_pred<1, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 2: hipLaunchKernelGGL((knn_pred<2, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 3: hipLaunchKernelGGL((knn_pred<3, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 4: hipLaunchKernelGGL((knn_pred<4, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 5: hipLaunchKernelGGL((knn_pred<5, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 6: hipLaunchKernelGGL((knn_pred<6, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 7: hipLaunchKernelGGL((knn_pred<7, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 8: hipLaunchKernelGGL((knn_pred<8, NE>), grid, block, 0, s, Xr, nr, d, w, cols); break;
        default:
            if (d <= 12) hipLaunchKernelGGL((knn_pred<12, NE>), grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 16) hipLaunchKernelGGL((knn_pred<16, NE>), grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 24) hipLaunchKernelGGL((knn_pred<24, NE>), grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 32) hipLaunchKernelGGL((knn_pred<32, NE>), grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 48) hipLaunchKernelGGL((knn_pred<48, NE>), grid, block, 0, s, Xr, nr, d, w, cols);
            else hipLaunchKernelGGL((knn_pred<64, NE>), grid, block, 0, s, Xr, nr, d, w, cols);
            break;
    }
}

}  // namespace

size_t knn_work_bytes(int64_t nr, int d)
{
    const int64_t nt = (nr + 63) / 64;
    return (size_t)(nt * d * 2 * 8 + 256 + nt * 4 + 256);
}

afn_status knn_pattern_ordered(const double *Xr, int64_t nr, int d, int w, const int32_t *order, void *work,
                               int32_t *cols, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    if (w < 1 || w > kMaxW) {
        set_error("knn_pattern: w=%d outside [1, %d]", w, kMaxW);
        return AFN_EINVAL;
    }
    if (d > 8 || !order || !work) return knn_pattern(Xr, nr, d, w, cols, s);
    const int64_t nt = (nr + 63) / 64;
    double *box = (double *)work;
    int32_t *tmin = (int32_t *)((char *)work + ((nt * d * 2 * 8 + 255) / 256) * 256);
    hipLaunchKernelGGL(knn_tile_boxes, dim3((unsigned)ceil_div(nt * (d + 1), 256)), dim3(256), 0, s, Xr, nr, d,
                       order, nt, box, tmin);
    int64_t waves = nr < 16384 ? nr : 16384;
    dim3 grid((unsigned)ceil_div(waves, 4)), block(256);
    if (w > 64) launch_tiles<2>(grid, block, s, Xr, nr, d, w, order, box, tmin, nt, cols);
    else launch_tiles<1>(grid, block, s, Xr, nr, d, w, order, box, tmin, nt, cols);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status knn_pattern(const double *Xr, int64_t nr, int d, int w, int32_t *cols, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    if (w < 1 || w > kMaxW) {
        set_error("knn_pattern: w=%d outside [1, %d]", w, kMaxW);
        return AFN_EINVAL;
    }
    int64_t waves = nr < 16384 ? nr : 16384;
    dim3 grid((unsigned)ceil_div(waves, 4)), block(256);
    if (w > 64) launch_brute<2>(grid, block, s, Xr, nr, d, w, cols);
    else launch_brute<1>(grid, block, s, Xr, nr, d, w, cols);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
