// FSAI sparsity pattern (Section 3.1): row p of the non-landmark points X_r
// holds the w-1 nearest earlier-numbered points q < p -- keys (squared
// distance, q) compared lexicographically -- plus p itself, columns ascending
// (p last).  Rows p < w-1 hold all p predecessors.
//
// One wavefront per query p.  The 64 lanes evaluate 64 candidates at a time
// (squared distance by the fixed fma chain, -ffp-contract=off, so keys are
// bit-identical to a sequential evaluation); candidates whose key beats the
// current (w-1)-th best enter a sorted list held one entry per lane, by a
// wave-wide rank-and-shift.  The final set is unique, so the pattern does not
// depend on the candidate order.  Queries are dealt round-robin to waves,
// which balances the O(p) cost per query.
#include <climits>

#include "afn_internal.h"

namespace afn {
namespace {

__device__ __forceinline__ bool key_less(double d1, int q1, double d2, int q2)
{
    return d1 < d2 || (d1 == d2 && q1 < q2);
}

// D >= d: the query's coordinates sit in registers, zero-padded to D; the
// candidate's coordinates beyond d are taken as zero too, so the squared
// distance is the fma chain over t = 0..d-1 followed by additions of +0.
template <int D>
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
        double ld = __builtin_inf();   // this lane's list entry
        int lq = INT_MAX;
        int cnt = 0;
        double thr_d = __builtin_inf();
        int thr_q = INT_MAX;
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
                const int qi = (int)q;
                bool pass = valid && (cnt < want || key_less(dq, qi, thr_d, thr_q));
                uint64_t mask = __ballot(pass);
                while (mask) {
                    const int src = __ffsll((unsigned long long)mask) - 1;
                    const double nd = __shfl(dq, src, 64);
                    const int nq = __shfl(qi, src, 64);
                    const bool lt = lane < cnt && key_less(ld, lq, nd, nq);
                    const int pos = __popcll(__ballot(lt));
                    const double upd = __shfl_up(ld, 1, 64);
                    const int upq = __shfl_up(lq, 1, 64);
                    if (lane > pos) { ld = upd; lq = upq; }
                    if (lane == pos) { ld = nd; lq = nq; }
                    if (lane >= want) { ld = __builtin_inf(); lq = INT_MAX; }
                    cnt = cnt + 1 < want ? cnt + 1 : want;
                    mask &= mask - 1;
                    if (cnt == want) {
                        thr_d = __shfl(ld, want - 1, 64);
                        thr_q = __shfl(lq, want - 1, 64);
                        mask &= __ballot(pass && key_less(dq, qi, thr_d, thr_q));
                    }
                }
            }
        }
        // rank of this lane's neighbour among the cnt selected, by index
        int rank = 0;
        for (int j = 0; j < cnt; ++j) {
            int oq = __shfl(lq, j, 64);
            rank += (oq < lq) ? 1 : 0;
        }
        int32_t *row = cols + p * w;
        if (lane < cnt) row[rank] = lq;
        if (lane == 0) row[cnt] = (int32_t)p;
        if (lane > cnt && lane < w) row[lane] = -1;
    }
}

}  // namespace

afn_status knn_pattern(const double *Xr, int64_t nr, int d, int w, int32_t *cols, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    if (w < 1 || w > 64) {
        set_error("knn_pattern: w=%d outside [1, 64]", w);
        return AFN_EINVAL;
    }
    int64_t waves = nr < 16384 ? nr : 16384;
    dim3 grid((unsigned)ceil_div(waves, 4)), block(256);
    switch (d) {
        case 1: hipLaunchKernelGGL(knn_pred<1>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 2: hipLaunchKernelGGL(knn_pred<2>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 3: hipLaunchKernelGGL(knn_pred<3>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 4: hipLaunchKernelGGL(knn_pred<4>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 5: hipLaunchKernelGGL(knn_pred<5>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 6: hipLaunchKernelGGL(knn_pred<6>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 7: hipLaunchKernelGGL(knn_pred<7>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        case 8: hipLaunchKernelGGL(knn_pred<8>, grid, block, 0, s, Xr, nr, d, w, cols); break;
        default:
            if (d <= 12) hipLaunchKernelGGL(knn_pred<12>, grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 16) hipLaunchKernelGGL(knn_pred<16>, grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 24) hipLaunchKernelGGL(knn_pred<24>, grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 32) hipLaunchKernelGGL(knn_pred<32>, grid, block, 0, s, Xr, nr, d, w, cols);
            else if (d <= 48) hipLaunchKernelGGL(knn_pred<48>, grid, block, 0, s, Xr, nr, d, w, cols);
            else hipLaunchKernelGGL(knn_pred<64>, grid, block, 0, s, Xr, nr, d, w, cols);
            break;
    }
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
