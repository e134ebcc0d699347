// Many right-hand sides at once.
//
// Kernel matvec Y = (K + mu I) P for R <= 64 columns: per 64 x 64 tile the
// kernel values E are formed on the VALU (from the same pre-scaled
// coordinates as the single-vector kernels, kfun.h) and stored transposed in LDS; the product E P_J is
// a GEMM with K = 64 and runs on the matrix cores (MFMA 16x16x4, FP32 or
// FP64).  A workgroup owns 64 rows and a range of column tiles; split
// partials are added in order by a second pass (deterministic).
//
// The batched apply (Algorithm 3 for R columns) uses an MFMA GEMM with split
// K for the L^{-1} and V products and SpMMs for G and G^T.  Vectors of R
// columns are point-major (row-major n x R, columns contiguous) inside the
// solver so that the SpMM gathers and the kernel tile loads are coalesced.
//
// MFMA operand layouts: mfma.h.
#include <cmath>

#include <cstdio>

#include "afn_internal.h"
#include "kfun.h"
#include "mfma.h"

namespace afn {
namespace {

constexpr int TL = 64;      // tile edge (points / rows / k-chunk)
constexpr int LS = 80;      // LDS row stride: (lane/16) * LS = 16 (mod 64) -> conflict-free MFMA reads

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// part[s][i * RP + c] = sum over the column tiles of split s of K_ij P_jc.
// Xs: packed scaled coordinates (npad a multiple of 128, zero padded).
// P: row-major n x R (leading dimension ldp).  RP = 16 * NB >= R.
// 128 rows per workgroup (8 waves).  Kernel values: lane = row within a
// 64-row half, wave pair = 16-column group, so the transposed stores into
// LDS are consecutive and the column coordinates are broadcast reads.
constexpr int BM = 128;
constexpr int LSE = 144;    // (lane/16) * 144 = 16 (mod 64): conflict-free MFMA A reads

// perm (may be null): row q of P is row perm[q] of the caller's array.  box
// (may be null): per 64-point tile, [min, max] of each packed coordinate; a
// column tile whose box gap^2 to this block's rows is >= tcut is skipped.
template <int KIND, int D, typename T, int NB>
__global__ __launch_bounds__(512) void kmv_mrhs(const T *__restrict__ Xs, int64_t npad, int64_t n,
                                                const T *__restrict__ P, int64_t ldp, int R,
                                                int tiles_per_split, T *__restrict__ part,
                                                const int32_t *__restrict__ perm, const T *__restrict__ box,
                                                T tcut)
{
    using M = Mfma<T>;
    constexpr int RP = 16 * NB;
    __shared__ T cx[D][TL];
    __shared__ T EsT[TL][LSE];      // EsT[j][i] = K(row i, column j)
    __shared__ T PJ[TL][LS];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int half = wave & 1, cgrp = wave >> 1;     // rows half*64 + lane, columns cgrp*16 ..
    const int64_t i0 = (int64_t)blockIdx.x * BM;
    const int64_t ntiles = npad / TL;
    const int64_t J0 = (int64_t)blockIdx.y * tiles_per_split;
    const int64_t J1 = J0 + tiles_per_split < ntiles ? J0 + tiles_per_split : ntiles;
    T xi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = Xs[(int64_t)t * npad + i0 + half * 64 + lane];
    typename M::acc_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = typename M::acc_t{};
    // box of this block's 128 rows (tiles 2 blockIdx.x and 2 blockIdx.x + 1)
    T rlo[D], rhi[D];
    if (box) {
        const int64_t ta = 2 * (int64_t)blockIdx.x, tb = ta + 1;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            const T alo = box[(ta * D + t) * 2], ahi = box[(ta * D + t) * 2 + 1];
            const T blo = box[(tb * D + t) * 2], bhi = box[(tb * D + t) * 2 + 1];
            rlo[t] = alo < blo ? alo : blo;
            rhi[t] = ahi > bhi ? ahi : bhi;
        }
    }
    // candidate column tiles in chunks of 512: every thread tests one, the
    // survivors are listed in ascending order (the summation order over tiles
    // is the same as without pruning)
    __shared__ int jlist[512];
    __shared__ int wcnt[8];
    for (int64_t Jc = J0; Jc < J1; Jc += 512) {
        const int64_t Jt = Jc + tid;
        bool keep = Jt < J1;
        if (keep && box) {
            T g2 = T(0);
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const T blo = box[(Jt * D + t) * 2], bhi = box[(Jt * D + t) * 2 + 1];
                T gap = blo - rhi[t] > rlo[t] - bhi ? blo - rhi[t] : rlo[t] - bhi;
                gap = gap > T(0) ? gap : T(0);
                g2 = fmaT(gap, gap, g2);
            }
            keep = g2 < tcut;
        }
        const unsigned long long mask = __ballot(keep);
        __syncthreads();
        if (lane == 0) wcnt[wave] = (int)__popcll(mask);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w2 = 0; w2 < 8; ++w2) {
            before += w2 < wave ? wcnt[w2] : 0;
            total += wcnt[w2];
        }
        if (keep) jlist[before + (int)__popcll(mask & ((1ull << lane) - 1ull))] = tid;
        __syncthreads();
        for (int qj = 0; qj < total; ++qj) {
            const int64_t j0 = (Jc + jlist[qj]) * TL;
            __syncthreads();
            for (int e = tid; e < D * TL; e += 512) {
                const int t = e / TL, j = e % TL;
                cx[t][j] = Xs[(int64_t)t * npad + j0 + j];
            }
            for (int e = tid; e < TL * RP; e += 512) {
                const int k = e / RP, c = e % RP;
                const int64_t q = j0 + k;
                PJ[k][c] = (q < n && c < R) ? P[(perm ? (int64_t)perm[q] : q) * ldp + c] : T(0);
            }
            __syncthreads();
#pragma unroll 4
            for (int c = 0; c < 16; ++c) {
                const int j = cgrp * 16 + c;
                T d2 = T(0);
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const T del = xi[t] - cx[t][j];
                    d2 = fmaT(del, del, d2);
                }
                EsT[j][half * 64 + lane] = kernel_scaled<KIND, T>(d2);
            }
            __syncthreads();
#pragma unroll 4
            for (int kk = 0; kk < TL / 4; ++kk) {
                const int k = 4 * kk + (lane >> 4);
                const T a = EsT[k][16 * wave + (lane & 15)];
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[b] = M::op(a, PJ[k][16 * b + (lane & 15)], acc[b]);
            }
        }
    }
    T *out = part + (int64_t)blockIdx.y * npad * RP;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = i0 + 16 * wave + M::row(lane, q);
            out[row * RP + 16 * b + (lane & 15)] = acc[b][q];
        }
}

// FP32 variant, software-pipelined.  64 rows per workgroup (4 waves); for
// each kept column tile the MFMAs consume the kernel-value tile E and the
// vector block P_J staged in LDS by the previous step, while the same waves
// compute E and load P_J for the next kept tile into the other buffer (the
// two parts sit in one basic block, so the scheduler can interleave the
// VALU work with the matrix-core work).  One barrier per tile.  LDS tiles
// are XOR-swizzled instead of padded (two workgroups fit per CU):
//   E:   element (k, r) at k * 64 + (r ^ 16 (k & 3))
//   P_J: element (k, c) at k * LD + (c ^ 16 (k & 3)) for R = 64; rows of
//        16 or 48 values (LD = 16, 48) need no swizzle
// so the MFMA operand reads of the four lane groups (rows 4 kk + g) fall in
// four different 16-bank groups.
template <int NB>
struct PjLayout {
    static constexpr int RP = 16 * NB;
    static constexpr int LD = NB == 2 ? 48 : RP;
    static __device__ __forceinline__ int at(int k, int c)
    {
        return k * LD + (NB == 4 ? (c ^ (16 * (k & 3))) : c);
    }
};

template <int KIND, int D, int NB>
__global__ __launch_bounds__(256) void kmv_mrhs_pipe(const float *__restrict__ Xs, int64_t npad, int64_t n,
                                                     const float *__restrict__ P, int64_t ldp, int R,
                                                     int tiles_per_split, float *__restrict__ part,
                                                     const int32_t *__restrict__ perm, const float *__restrict__ box,
                                                     float tcut)
{
    using M = Mfma<float>;
    using L = PjLayout<NB>;
    constexpr int RP = L::RP;
    constexpr int PV4 = NB;             // groups of 4 P values per thread and tile (64 RP / 1024)
    constexpr int CHUNK = 2048;         // column tiles listed at a time
    __shared__ float Es[2][TL * TL];
    __shared__ float Pj[2][TL * L::LD];
    __shared__ int jlist[CHUNK];
    __shared__ int wcnt[4];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, lc = lane & 15, g = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * TL;
    const int64_t ntiles = npad / TL;
    const int64_t J0 = (int64_t)blockIdx.y * tiles_per_split;
    const int64_t J1 = J0 + tiles_per_split < ntiles ? J0 + tiles_per_split : ntiles;
    float xi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = Xs[(int64_t)t * npad + r0 + lane];
    float rlo[D], rhi[D];
    if (box) {
#pragma unroll
        for (int t = 0; t < D; ++t) {
            rlo[t] = box[((int64_t)blockIdx.x * D + t) * 2];
            rhi[t] = box[((int64_t)blockIdx.x * D + t) * 2 + 1];
        }
    }
    typename M::acc_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = typename M::acc_t{};
    // staging of the next tile: values 4 e .. 4 e + 3 of P_J for
    // e = tid + 256 i (row 4 e / RP), so that 16 / NB consecutive lanes read
    // a row and write it to LDS as whole 16-byte words; coordinates of this
    // wave's 16 columns
    float pv[PV4][4], xc[16][D];
    auto load_next = [&](int64_t j0) {
#pragma unroll
        for (int i = 0; i < PV4; ++i) {
            const int e = 4 * (tid + 256 * i), k = e / RP, c = e % RP;
            const int64_t q = j0 + k;
            const float *src = P + (q < n ? (perm ? (int64_t)perm[q] : q) * ldp : 0);
#pragma unroll
            for (int u = 0; u < 4; ++u) pv[i][u] = (q < n && c + u < R) ? src[c + u] : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < 16; ++c)
#pragma unroll
            for (int t = 0; t < D; ++t) xc[c][t] = Xs[(int64_t)t * npad + j0 + 16 * wave + c];
    };
    auto stage_next = [&](int b) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int col = 16 * wave + c;
            float d2 = 0.0f;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const float del = xi[t] - xc[c][t];
                d2 = __builtin_fmaf(del, del, d2);
            }
            Es[b][col * TL + (lane ^ (16 * (col & 3)))] = kernel_scaled<KIND, float>(d2);
        }
#pragma unroll
        for (int i = 0; i < PV4; ++i) {
            const int e = 4 * (tid + 256 * i);
            float *dst = &Pj[b][L::at(e / RP, e % RP)];
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = pv[i][u];
        }
    };
    for (int64_t Jc = J0; Jc < J1; Jc += CHUNK) {
        const int64_t Je = Jc + CHUNK < J1 ? Jc + CHUNK : J1;
        // kept column tiles of this chunk in ascending order (the summation
        // order over tiles is the same as without pruning)
        int total = 0;
        for (int64_t Jr = Jc; Jr < Je; Jr += 256) {
            const int64_t Jt = Jr + tid;
            bool keep = Jt < Je;
            if (keep && box) {
                float g2 = 0.0f;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const float blo = box[(Jt * D + t) * 2], bhi = box[(Jt * D + t) * 2 + 1];
                    float gap = blo - rhi[t] > rlo[t] - bhi ? blo - rhi[t] : rlo[t] - bhi;
                    gap = gap > 0.0f ? gap : 0.0f;
                    g2 = __builtin_fmaf(gap, gap, g2);
                }
                keep = g2 < tcut;
            }
            const unsigned long long mask = __ballot(keep);
            __syncthreads();
            if (lane == 0) wcnt[wave] = (int)__popcll(mask);
            __syncthreads();
            int before = 0, cnt = 0;
#pragma unroll
            for (int w2 = 0; w2 < 4; ++w2) {
                before += w2 < wave ? wcnt[w2] : 0;
                cnt += wcnt[w2];
            }
            if (keep) jlist[total + before + (int)__popcll(mask & ((1ull << lane) - 1ull))] = (int)(Jt - Jc);
            total += cnt;
        }
        __syncthreads();
        if (total == 0) continue;
        load_next((Jc + jlist[0]) * TL);
        stage_next(0);
        __syncthreads();
        for (int qj = 0; qj < total; ++qj) {
            const int b = qj & 1;
            // the next kept tile (past the end: the first one again; staged
            // into the unused buffer and never read)
            const int64_t jn = (Jc + jlist[qj + 1 < total ? qj + 1 : 0]) * TL;
            load_next(jn);
#pragma unroll
            for (int kk = 0; kk < TL / 4; ++kk) {
                const int k = 4 * kk + g;
                const float a = Es[b][k * TL + ((16 * wave + lc) ^ (16 * (k & 3)))];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb] = M::op(a, Pj[b][L::at(k, 16 * nb + lc)], acc[nb]);
            }
            stage_next(b ^ 1);
            __syncthreads();
        }
    }
    float *out = part + (int64_t)blockIdx.y * npad * RP;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = r0 + 16 * wave + M::row(lane, q);
            out[row * RP + 16 * nb + lc] = acc[nb][q];
        }
}

// Y[i * ldy + c] = sum_s part[s][i * RP + c] + mu P[i * ldp + c]
template <typename T>
__global__ __launch_bounds__(256) void mrhs_reduce(const T *__restrict__ part, int64_t npad, int RP,
                                                   int splits, int64_t n, int R, double mu,
                                                   const T *__restrict__ P, int64_t ldp,
                                                   T *__restrict__ Y, int64_t ldy,
                                                   const int32_t *__restrict__ perm)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int64_t i = e / R;
    const int c = (int)(e - i * R);
    const int64_t o = perm ? (int64_t)perm[i] : i;
    double s = 0.0;
    for (int q = 0; q < splits; ++q) s += (double)part[(int64_t)q * npad * RP + i * RP + c];
    Y[o * ldy + c] = (T)(s + mu * (double)P[o * ldp + c]);
}

// part[s][i * RP + c] = sum_{t in split s} A(i, t) B(t, c), A(i,t) = A[i*ars + t*acs],
// B row-major (ldb).  64 rows per workgroup, K in chunks of 64, each chunk
// read with 16-byte loads along the contiguous dimension of A (t when
// KF, i otherwise) and of B while the MFMAs run on the previous chunk
// (double-buffered in LDS, one barrier per chunk).  LDS layouts (conflict-
// free MFMA operand reads by the four lane groups): KF: A as [i][k] with
// row stride 68; otherwise A as [k][i] and B as [k][c], row stride 80.
// VEC: every 4-element group is 16-byte aligned (strides and bases checked
// on the host); groups at the edges are read element by element.
template <typename T, bool VEC>
__device__ __forceinline__ void load4(const T *p, bool whole, int nvalid, int64_t step, T (&o)[4])
{
    if (VEC && whole) {
        if constexpr (sizeof(T) == 4) {
            const float4 x = *reinterpret_cast<const float4 *>(p);
            o[0] = x.x; o[1] = x.y; o[2] = x.z; o[3] = x.w;
        } else {
            const double2 x = *reinterpret_cast<const double2 *>(p);
            const double2 y = *reinterpret_cast<const double2 *>(p + 2);
            o[0] = x.x; o[1] = x.y; o[2] = y.x; o[3] = y.y;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) o[u] = u < nvalid ? p[u * step] : T(0);
    }
}

// LDS row strides of gemm_splitk's tiles (A along k, A along i, B).
constexpr int kGemmLAk = 68, kGemmLAi = 80, kGemmLB = 80;

template <typename T, int NB, bool KF, bool VEC>
__global__ __launch_bounds__(256) void gemm_splitk(const T *__restrict__ A, int64_t ars, int64_t acs,
                                                   int64_t m, int64_t K, const T *__restrict__ B,
                                                   int64_t ldb, int R, int64_t k_per_split,
                                                   T *__restrict__ part, int64_t mpad)
{
    using M = Mfma<T>;
    constexpr int RP = 16 * NB;
    constexpr int LA = KF ? kGemmLAk : kGemmLAi;
    constexpr int LB = kGemmLB;
    // FP64: one LDS buffer (two workgroups per CU), FP32: two
    constexpr int NBUF = sizeof(T) == 8 ? 1 : 2;
    __shared__ T As[NBUF][TL * LA];
    __shared__ T Bs[NBUF][TL * LB];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, lc = lane & 15, g = lane >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * TL;
    const int64_t t0 = (int64_t)blockIdx.y * k_per_split;
    const int64_t t1 = t0 + k_per_split < K ? t0 + k_per_split : K;
    typename M::acc_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = typename M::acc_t{};
    T pa[4][4], pb[NB][4];
    auto load = [&](int64_t tc) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            if constexpr (KF) {
                const int i = e / 16, k = 4 * (e % 16);
                const int64_t gi = i0 + i, gt = tc + k;
                const int nv = gi < m ? (int)(t1 - gt < 4 ? (t1 - gt > 0 ? t1 - gt : 0) : 4) : 0;
                load4<T, VEC>(A + (gi < m ? gi : 0) * ars + (gt < t1 ? gt : t0) * acs, nv == 4, nv, acs, pa[q]);
            } else {
                const int k = e / 16, i = 4 * (e % 16);
                const int64_t gi = i0 + i, gt = tc + k;
                const int nv = gt < t1 ? (int)(m - gi < 4 ? (m - gi > 0 ? m - gi : 0) : 4) : 0;
                load4<T, VEC>(A + (gi < m ? gi : 0) * ars + (gt < t1 ? gt : t0) * acs, nv == 4, nv, ars, pa[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q;
            const int k = e / (RP / 4), c = 4 * (e % (RP / 4));
            const int64_t gt = tc + k;
            const int nv = gt < t1 ? (R - c < 4 ? (R - c > 0 ? R - c : 0) : 4) : 0;
            load4<T, VEC>(B + (gt < t1 ? gt : t0) * ldb + (c < R ? c : 0), nv == 4, nv, 1, pb[q]);
        }
    };
    auto store = [&](int b) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            T *dst;
            if constexpr (KF) dst = &As[b][(e / 16) * LA + 4 * (e % 16)];
            else dst = &As[b][(e / 16) * LA + 4 * (e % 16)];
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = pa[q][u];
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int e = tid + 256 * q;
            T *dst = &Bs[b][(e / (RP / 4)) * LB + 4 * (e % (RP / 4))];
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = pb[q][u];
        }
    };
    const int64_t nchunk = t1 > t0 ? ceil_div(t1 - t0, TL) : 0;
    if (nchunk > 0) {
        load(t0);
        store(0);
        __syncthreads();
        for (int64_t ch = 0; ch < nchunk; ++ch) {
            const int b = NBUF == 1 ? 0 : (int)(ch & 1);
            // the next chunk (past the end: the last one again, staged and
            // never read)
            load(t0 + (ch + 1 < nchunk ? ch + 1 : ch) * TL);
#pragma unroll
            for (int kk = 0; kk < TL / 4; ++kk) {
                const int k = 4 * kk + g, i = 16 * wave + lc;
                const T a = KF ? As[b][i * LA + k] : As[b][k * LA + i];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb] = M::op(a, Bs[b][k * LB + 16 * nb + lc], acc[nb]);
            }
            if constexpr (NBUF == 1) {
                __syncthreads();      // every wave is done with the buffer
                store(0);
            } else {
                store(b ^ 1);
            }
            __syncthreads();
        }
    }
    T *out = part + (int64_t)blockIdx.y * mpad * RP;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = i0 + 16 * wave + M::row(lane, q);
            out[row * RP + 16 * b + lc] = acc[b][q];
        }
}

// C[i * ldc + c] = base[i * ldc + c] + sign * sum_s part[s][i * RP + c]
template <typename T>
__global__ __launch_bounds__(256) void gemm_reduce(const T *__restrict__ part, int64_t mpad, int RP,
                                                   int splits, int64_t m, int R,
                                                   const T *__restrict__ base, T sign,
                                                   T *__restrict__ C, int64_t ldc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * R) return;
    const int64_t i = e / R;
    const int c = (int)(e - i * R);
    T s = T(0);
    for (int q = 0; q < splits; ++q) s += part[(int64_t)q * mpad * RP + i * RP + c];
    C[i * ldc + c] = (base ? base[i * ldc + c] : T(0)) + sign * s;
}

// U[p*ld + c] = sum_a g[p*w + a] T[cols[p*w + a]*ld + c]  (wave per row, lane = column)
template <typename T>
__global__ __launch_bounds__(256) void spmm_padded(const int32_t *__restrict__ cols,
                                                   const T *__restrict__ g, int64_t nr, int w,
                                                   const T *__restrict__ X, int64_t ld, int R,
                                                   T *__restrict__ U, const int32_t *__restrict__ order)
{
    const int lane = threadIdx.x & 63;
    const int64_t blk = order ? xcd_contiguous(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t slot = blk * 4 + (threadIdx.x >> 6);
    if (slot >= nr || lane >= R) return;
    const int64_t p = order ? (int64_t)order[slot] : slot;
    const int m = (int)(p + 1 < w ? p + 1 : w);
    T s = T(0);
    // 8 gathers in flight; entries past the row's end repeat entry m - 1
    // with weight zero (the sum stays in entry order)
    for (int a0 = 0; a0 < m; a0 += 8) {
        T gv[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int a = a0 + u < m ? a0 + u : m - 1;
            gv[u] = a0 + u < m ? g[p * w + a] : T(0);
            xv[u] = X[(int64_t)cols[p * w + a] * ld + lane];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fmaT(gv[u], xv[u], s);
    }
    U[p * ld + lane] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void spmm_csr(const int64_t *__restrict__ ptr,
                                                const int32_t *__restrict__ idx,
                                                const T *__restrict__ val, int64_t nrows,
                                                const T *__restrict__ X, int64_t ld, int R,
                                                T *__restrict__ U, const int32_t *__restrict__ order)
{
    const int lane = threadIdx.x & 63;
    const int64_t blk = order ? xcd_contiguous(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t slot = blk * 4 + (threadIdx.x >> 6);
    if (slot >= nrows || lane >= R) return;
    const int64_t q = order ? (int64_t)order[slot] : slot;
    T s = T(0);
    const int64_t e1 = ptr[q + 1];
    for (int64_t e0 = ptr[q]; e0 < e1; e0 += 8) {
        T vv[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t e = e0 + u < e1 ? e0 + u : e1 - 1;
            vv[u] = e0 + u < e1 ? val[e] : T(0);
            xv[u] = X[(int64_t)idx[e] * ld + lane];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fmaT(vv[u], xv[u], s);
    }
    U[q * ld + lane] = s;
}

// Per-column dot products of row-major n x R blocks: stage 1 (4 row groups x
// 64 columns per workgroup), stage 2 sums the block partials in order.
template <typename T>
__global__ __launch_bounds__(256) void coldot_stage1(const T *__restrict__ A, const T *__restrict__ B,
                                                     int64_t n, int R, int64_t chunk,
                                                     double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
    double s = 0.0;
    if (c < R)
        for (int64_t i = i0 + g; i < i1; i += 16) {
            // four rows' loads in flight; the products are added in row order
            T a[4], b[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t r = i + 4 * u < i1 ? i + 4 * u : i;
                a[u] = i + 4 * u < i1 ? A[r * R + c] : T(0);
                b[u] = B[r * R + c];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) s = __builtin_fma((double)a[u], (double)b[u], s);
        }
    red[g][c] = s;
    __syncthreads();
    if (g == 0 && c < R) part[(int64_t)blockIdx.x * R + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

__global__ __launch_bounds__(64) void coldot_stage2(const double *__restrict__ part, int nb, int R,
                                                    double *__restrict__ out)
{
    const int c = threadIdx.x;
    if (c >= R) return;
    double s = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 8) {
        double q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = b0 + u < nb ? part[(int64_t)(b0 + u) * R + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) s += q[u];
    }
    out[c] = s;
}

// Per-column scalars (arrays of R): alpha = rho / pq for active columns.
__global__ __launch_bounds__(64) void col_alpha(const double *rho, const double *pq, int *active,
                                                double *alpha, int R, int *bad)
{
    const int c = threadIdx.x;
    if (c >= R) return;
    double a = 0.0;
    if (active[c]) {
        if (pq[c] > 0.0) {
            a = rho[c] / pq[c];
        } else {
            atomicOr(bad, 2);     // p'Ap <= 0 or NaN: breakdown of this column
            active[c] = 0;
        }
    }
    alpha[c] = a;
}

__global__ __launch_bounds__(64) void col_beta(double *rho, const double *rho_new, const int *active,
                                               double *beta, int R)
{
    const int c = threadIdx.x;
    if (c >= R) return;
    beta[c] = active[c] ? rho_new[c] / rho[c] : 0.0;
    rho[c] = rho_new[c];
}

// x += alpha_c p; r -= alpha_c q; partial r.r per column
template <typename T>
__global__ __launch_bounds__(256) void col_xr(T *__restrict__ X, T *__restrict__ Rv,
                                              const T *__restrict__ Pv, const T *__restrict__ Q,
                                              const double *__restrict__ alpha, int64_t n, int R,
                                              int64_t chunk, double *__restrict__ part)
{
    __shared__ double red[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * chunk;
    const int64_t i1 = i0 + chunk < n ? i0 + chunk : n;
    double s = 0.0;
    if (c < R) {
        const T a = (T)alpha[c];
        for (int64_t i = i0 + g; i < i1; i += 16) {
            // four rows' loads in flight, updated and summed in row order
            T xv[4], pv[4], qv[4], rv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = (i + 4 * u < i1 ? i + 4 * u : i) * R + c;
                xv[u] = X[e];
                pv[u] = Pv[e];
                qv[u] = Q[e];
                rv[u] = Rv[e];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i + 4 * u < i1) {
                    const int64_t e = (i + 4 * u) * R + c;
                    X[e] = fmaT(a, pv[u], xv[u]);
                    const T r = fmaT(-a, qv[u], rv[u]);
                    Rv[e] = r;
                    s = __builtin_fma((double)r, (double)r, s);
                }
            }
        }
    }
    red[g][c] = s;
    __syncthreads();
    if (g == 0 && c < R) part[(int64_t)blockIdx.x * R + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}

template <typename T>
__global__ __launch_bounds__(256) void col_p(T *__restrict__ Pv, const T *__restrict__ Z,
                                             const double *__restrict__ beta, int64_t n, int R)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int c = (int)(e % R);
    Pv[e] = fmaT((T)beta[c], Pv[e], Z[e]);
}

// active_c &= (sqrt(rr_c / bnorm2_c) > tol_c); count of active columns.
__global__ __launch_bounds__(64) void col_converged(const double *rr, const double *bnorm2,
                                                    const double *tol, int *active, int *count, int R,
                                                    int *bad)
{
    const int c = threadIdx.x;
    int a = 0;
    if (c < R && active[c]) {
        const double rel = sqrt(rr[c] / bnorm2[c]);
        if (!(rel == rel)) atomicOr(bad, 1);
        a = rel > tol[c] && rel == rel;
        active[c] = a;
    }
    const uint64_t m = __ballot(a);
    if (c == 0) *count = __popcll(m);
}

// Gather columns from a column-major block into a row-major one, with the
// point permutation: Y[i * R + c] = (T) (X[perm[i] + c * ld] * scale_c).
template <typename T>
__global__ __launch_bounds__(256) void gather_rowmajor(const double *__restrict__ X, int64_t ld,
                                                       const int32_t *__restrict__ perm, int64_t n,
                                                       int R, const double *__restrict__ scale,
                                                       T *__restrict__ Y)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int64_t i = e / R;
    const int c = (int)(e - i * R);
    const double v = X[(perm ? perm[i] : i) + c * ld];
    Y[e] = (T)(scale ? v * scale[c] : v);
}

__global__ __launch_bounds__(256) void scatter_rowmajor(const double *__restrict__ Y,
                                                        const int32_t *__restrict__ perm, int64_t n,
                                                        int R, double *__restrict__ X, int64_t ld)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int64_t i = e / R;
    const int c = (int)(e - i * R);
    X[(perm ? perm[i] : i) + c * ld] = Y[e];
}

// X[i + c * ld] = Y[i * R + c] for FP32 Y (identity order)
__global__ __launch_bounds__(256) void scatter_rowmajor_f32(const float *__restrict__ Y, int64_t n, int R,
                                                            double *__restrict__ X, int64_t ld)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int64_t i = e / R;
    const int c = (int)(e - i * R);
    X[i + c * ld] = (double)Y[e];
}

// R64 = B64 - A64 (row-major n x R)
__global__ __launch_bounds__(256) void sub_rows(const double *__restrict__ B, const double *__restrict__ Y,
                                                double *__restrict__ Rr, int64_t total)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    Rr[e] = B[e] - Y[e];
}

// r32[i*R + c] = r64[i*R + c] * inv_c ; x64 += norm_c * e32
__global__ __launch_bounds__(256) void scale_to_f32(const double *__restrict__ r, const double *__restrict__ inv,
                                                    float *__restrict__ r32, int64_t n, int R)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    r32[e] = (float)(r[e] * inv[e % R]);
}

__global__ __launch_bounds__(256) void axpy_cols_f32(const double *__restrict__ a, const float *__restrict__ e32,
                                                     double *__restrict__ x, int64_t n, int R)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    x[e] = __builtin_fma(a[e % R], (double)e32[e], x[e]);
}

template <int KIND, int D, typename T, int NB>
void launch_mrhs(dim3 g, const T *Xs, int64_t npad, int64_t n, const T *P, int64_t ldp, int R, int tps,
                 T *part, const int32_t *perm, const T *box, T tcut, hipStream_t s)
{
    if constexpr (sizeof(T) == 4) {
        // 64-row workgroups: twice the row blocks of the 128-row grid
        hipLaunchKernelGGL((kmv_mrhs_pipe<KIND, D, NB>), dim3(2 * g.x, g.y), dim3(256), 0, s, Xs, npad, n, P, ldp,
                           R, tps, part, perm, box, tcut);
    } else {
        hipLaunchKernelGGL((kmv_mrhs<KIND, D, T, NB>), g, dim3(512), 0, s, Xs, npad, n, P, ldp, R, tps, part,
                           perm, box, tcut);
    }
}

template <int KIND, typename T, int NB>
void launch_mrhs_d(int d, dim3 g, const T *Xs, int64_t npad, int64_t n, const T *P, int64_t ldp, int R,
                   int tps, T *part, const int32_t *perm, const T *box, T tcut, hipStream_t s)
{
    switch (d) {
        case 1: launch_mrhs<KIND, 1, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 2: launch_mrhs<KIND, 2, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 3: launch_mrhs<KIND, 3, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 4: launch_mrhs<KIND, 4, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 5: launch_mrhs<KIND, 5, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 6: launch_mrhs<KIND, 6, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 7: launch_mrhs<KIND, 7, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        default: launch_mrhs<KIND, 8, T, NB>(g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
    }
}

template <int KIND, typename T>
void launch_mrhs_nb(int NBk, int d, dim3 g, const T *Xs, int64_t npad, int64_t n, const T *P, int64_t ldp,
                    int R, int tps, T *part, const int32_t *perm, const T *box, T tcut, hipStream_t s)
{
    switch (NBk) {
        case 1: launch_mrhs_d<KIND, T, 1>(d, g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 2: launch_mrhs_d<KIND, T, 2>(d, g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        case 3: launch_mrhs_d<KIND, T, 3>(d, g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
        default: launch_mrhs_d<KIND, T, 4>(d, g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s); break;
    }
}

}  // namespace

// ------------------------------------------------------------------ host side

int mrhs_splits(int64_t npad)
{
    // enough (row block, split) workgroups that the last wave of them is a
    // small part of the launch: pruning makes their work uneven
    const int64_t rt = npad / BM;
    int64_t s = ceil_div(4096, rt);
    if (s > rt) s = rt;
    if (s > 64) s = 64;
    return (int)(s < 1 ? 1 : s);
}

int64_t mrhs_part_elems(int64_t npad) { return (int64_t)mrhs_splits(npad) * npad * 64; }

template <typename T>
afn_status kmv_mrhs_run(const T *Xs, int64_t npad, int64_t n, int d, double mu, int kind, const T *P,
                        int64_t ldp, T *Y, int64_t ldy, int R, T *part, hipStream_t s,
                        hipEvent_t e0, hipEvent_t e1, const int32_t *perm, const T *box)
{
    if (R < 1 || R > 64 || d < 1 || d > 8) {
        set_error("kmv_mrhs: R=%d d=%d outside [1, 64] x [1, 8]", R, d);
        return AFN_EINVAL;
    }
    if (npad % BM != 0) {
        set_error("kmv_mrhs: padded size %lld is not a multiple of %d", (long long)npad, BM);
        return AFN_EINVAL;
    }
    const int NBk = (R + 15) / 16;
    const int S = mrhs_splits(npad);
    const int64_t ntiles = npad / TL;
    const int tps = (int)ceil_div(ntiles, S);
    dim3 g((unsigned)(npad / BM), (unsigned)S);
    const T tcut = (T)kernel_cut_t(kind, sizeof(T) == 8 ? kCullF64 : kCullF32);
    if (e0) AFN_HIP(hipEventRecord(e0, s));
    if (kind == AFN_KERNEL_MATERN32)
        launch_mrhs_nb<AFN_KERNEL_MATERN32, T>(NBk, d, g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s);
    else
        launch_mrhs_nb<AFN_KERNEL_GAUSSIAN, T>(NBk, d, g, Xs, npad, n, P, ldp, R, tps, part, perm, box, tcut, s);
    AFN_HIP(hipGetLastError());
    if (e1) AFN_HIP(hipEventRecord(e1, s));
    hipLaunchKernelGGL((mrhs_reduce<T>), dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, part, npad,
                       16 * NBk, S, n, R, mu, P, ldp, Y, ldy, perm);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

template afn_status kmv_mrhs_run<float>(const float *, int64_t, int64_t, int, double, int, const float *,
                                        int64_t, float *, int64_t, int, float *, hipStream_t,
                                        hipEvent_t, hipEvent_t, const int32_t *, const float *);
template afn_status kmv_mrhs_run<double>(const double *, int64_t, int64_t, int, double, int, const double *,
                                         int64_t, double *, int64_t, int, double *, hipStream_t,
                                         hipEvent_t, hipEvent_t, const int32_t *, const double *);

int gemm_splits(int64_t m, int64_t K)
{
    const int64_t rt = ceil_div(m, TL);
    int64_t s = ceil_div(1024, rt);
    const int64_t smax = ceil_div(K, TL);
    if (s > smax) s = smax;
    if (s > 256) s = 256;
    return (int)(s < 1 ? 1 : s);
}

namespace {

// Workgroups of gemm_splitk that fit on one CU by LDS (double-buffered tiles).
template <typename T>
int gemm_wgs_per_cu(bool kf)
{
    const size_t nbuf = sizeof(T) == 8 ? 1 : 2;
    const size_t lds = nbuf * (size_t)TL * (kf ? kGemmLAk : kGemmLAi) * sizeof(T) + nbuf * (size_t)TL * kGemmLB * sizeof(T);
    const int per = (int)((160 * 1024) / lds);
    return per < 1 ? 1 : per;
}

int device_cus()
{
    static const int cus = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            v = 0;
        return v > 0 ? v : 256;
    }();
    return cus;
}

// Splits of one launch: at most gemm_splits(m, K) (the partial buffers are
// sized for that), chosen so that the workgroups fill whole rounds of the
// chip.  The time per row block goes as rounds / splits; take the fewest
// splits within 2% of the least.
int gemm_splits_launch(int64_t m, int64_t K, int per_cu)
{
    const int smax = gemm_splits(m, K);
    const int64_t rt = ceil_div(m, TL), cap = (int64_t)device_cus() * per_cu;
    double best = 1e300;
    for (int sp = 1; sp <= smax; ++sp) {
        const double c = (double)ceil_div(rt * sp, cap) / sp;
        best = c < best ? c : best;
    }
    for (int sp = 1; sp <= smax; ++sp)
        if ((double)ceil_div(rt * sp, cap) / sp <= best * 1.02) return sp;
    return smax;
}

}  // namespace

int64_t gemm_part_elems(int64_t m, int64_t K)
{
    return (int64_t)gemm_splits(m, K) * round_up(m, TL) * 64;
}

// gemm_part_elems(m, K) is not monotone in m (fewer row blocks get more
// splits): for every m <= mmax and any K, splits x row blocks <= row blocks
// of mmax + 1023, since ceil(1024 / rt) rt < 1024 + rt.
int64_t gemm_part_bound(int64_t mmax)
{
    return (ceil_div(mmax, TL) + 1023) * TL * 64;
}

namespace {

template <typename T, bool KF, bool VEC>
void launch_gemm(int NBk, dim3 g, const T *A, int64_t ars, int64_t acs, int64_t m, int64_t K, const T *B,
                 int64_t ldb, int R, int64_t kps, T *part, int64_t mpad, hipStream_t s)
{
    switch (NBk) {
        case 1: hipLaunchKernelGGL((gemm_splitk<T, 1, KF, VEC>), g, dim3(256), 0, s, A, ars, acs, m, K, B, ldb, R, kps, part, mpad); break;
        case 2: hipLaunchKernelGGL((gemm_splitk<T, 2, KF, VEC>), g, dim3(256), 0, s, A, ars, acs, m, K, B, ldb, R, kps, part, mpad); break;
        case 3: hipLaunchKernelGGL((gemm_splitk<T, 3, KF, VEC>), g, dim3(256), 0, s, A, ars, acs, m, K, B, ldb, R, kps, part, mpad); break;
        default: hipLaunchKernelGGL((gemm_splitk<T, 4, KF, VEC>), g, dim3(256), 0, s, A, ars, acs, m, K, B, ldb, R, kps, part, mpad); break;
    }
}

}  // namespace

// C = base + sign * A B  (A(i,t) = A[i*ars + t*acs], m x K; B row-major K x R)
template <typename T>
afn_status gemm_rows(const T *A, int64_t ars, int64_t acs, int64_t m, int64_t K, const T *B,
                     int64_t ldb, int R, const T *base, T sign, T *C, int64_t ldc, T *part,
                     hipStream_t s)
{
    if (m <= 0 || R <= 0) return AFN_OK;
    const int NBk = (R + 15) / 16;
    // A is read along t when its t stride is 1 (KF), along i otherwise
    const bool kf = acs == 1;
    const int smax = gemm_splits(m, K);      // the partial buffer holds this many
    const int S0 = gemm_splits_launch(m, K, gemm_wgs_per_cu<T>(kf));
    // split counts: the heuristic's (whole rounds of the chip), half of it and
    // twice it, within what the partial buffer holds
    int cand[3];
    int nc = 0;
    for (int q : {S0, S0 / 2, 2 * S0}) {
        q = q < 1 ? 1 : (q > smax ? smax : q);
        bool dup = false;
        for (int c = 0; c < nc; ++c) dup = dup || cand[c] == q;
        if (!dup) cand[nc++] = q;
    }
    const int64_t mpad = round_up(m, TL);
    const auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
    const bool vec = al16(A) && al16(B) && ldb % 4 == 0 && (kf ? ars % 4 == 0 : (ars == 1 && acs % 4 == 0));
    auto launch = [&](int c) -> afn_status {
        const int S = cand[c];
        const int64_t kps = round_up(ceil_div(K, S), TL);
        dim3 g((unsigned)ceil_div(m, TL), (unsigned)S);
        if (kf && vec) launch_gemm<T, true, true>(NBk, g, A, ars, acs, m, K, B, ldb, R, kps, part, mpad, s);
        else if (kf) launch_gemm<T, true, false>(NBk, g, A, ars, acs, m, K, B, ldb, R, kps, part, mpad, s);
        else if (vec) launch_gemm<T, false, true>(NBk, g, A, ars, acs, m, K, B, ldb, R, kps, part, mpad, s);
        else launch_gemm<T, false, false>(NBk, g, A, ars, acs, m, K, B, ldb, R, kps, part, mpad, s);
        AFN_HIP(hipGetLastError());
        hipLaunchKernelGGL((gemm_reduce<T>), dim3((unsigned)ceil_div(m * R, 256)), dim3(256), 0, s, part, mpad,
                           16 * NBk, S, m, R, base, sign, C, ldc);
        AFN_HIP(hipGetLastError());
        return AFN_OK;
    };
    int pick = 0;
    if ((const void *)base != (const void *)C && (const void *)A != (const void *)C &&
        (const void *)B != (const void *)C) {
        char shape[112];
        snprintf(shape, sizeof shape, "m%lld_K%lld_R%d_%s%s", (long long)m, (long long)K, R,
                 sizeof(T) == 8 ? "f64" : "f32", kf ? "_kf" : "");
        pick = tune_pick("gemm_splits", shape, nc, 0, launch, s);
    }
    return launch(pick);
}

template afn_status gemm_rows<float>(const float *, int64_t, int64_t, int64_t, int64_t, const float *,
                                     int64_t, int, const float *, float, float *, int64_t, float *,
                                     hipStream_t);
template afn_status gemm_rows<double>(const double *, int64_t, int64_t, int64_t, int64_t,
                                      const double *, int64_t, int, const double *, double, double *,
                                      int64_t, double *, hipStream_t);

template <typename T>
afn_status spmm_g(const int32_t *cols, const T *g, int64_t nr, int w, const T *X, int R, T *U,
                  const int32_t *order, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    hipLaunchKernelGGL((spmm_padded<T>), dim3((unsigned)ceil_div(nr, 4)), dim3(256), 0, s, cols, g, nr, w, X,
                       (int64_t)R, R, U, order);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

template <typename T>
afn_status spmm_gt(const int64_t *ptr, const int32_t *idx, const T *val, int64_t nr, const T *X, int R,
                   T *U, const int32_t *order, hipStream_t s)
{
    if (nr <= 0) return AFN_OK;
    hipLaunchKernelGGL((spmm_csr<T>), dim3((unsigned)ceil_div(nr, 4)), dim3(256), 0, s, ptr, idx, val, nr, X,
                       (int64_t)R, R, U, order);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

template afn_status spmm_g<float>(const int32_t *, const float *, int64_t, int, const float *, int,
                                  float *, const int32_t *, hipStream_t);
template afn_status spmm_g<double>(const int32_t *, const double *, int64_t, int, const double *, int,
                                  double *, const int32_t *, hipStream_t);
template afn_status spmm_gt<float>(const int64_t *, const int32_t *, const float *, int64_t,
                                   const float *, int, float *, const int32_t *, hipStream_t);
template afn_status spmm_gt<double>(const int64_t *, const int32_t *, const double *, int64_t,
                                    const double *, int, double *, const int32_t *, hipStream_t);

int64_t coldot_blocks(int64_t n)
{
    int64_t b = ceil_div(n, 256);
    return b < 1 ? 1 : (b > 2048 ? 2048 : b);
}

template <typename T>
afn_status coldot(const T *A, const T *B, int64_t n, int R, double *out, double *part, hipStream_t s)
{
    const int64_t nb = coldot_blocks(n);
    hipLaunchKernelGGL((coldot_stage1<T>), dim3((unsigned)nb), dim3(256), 0, s, A, B, n, R, ceil_div(n, nb),
                       part);
    hipLaunchKernelGGL(coldot_stage2, dim3(1), dim3(64), 0, s, part, (int)nb, R, out);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}
template afn_status coldot<float>(const float *, const float *, int64_t, int, double *, double *,
                                  hipStream_t);
template afn_status coldot<double>(const double *, const double *, int64_t, int, double *, double *,
                                   hipStream_t);

template <typename T>
afn_status col_xr_launch(T *X, T *Rv, const T *Pv, const T *Q, const double *alpha, int64_t n, int R,
                         double *rr, double *part, hipStream_t s)
{
    const int64_t nb = coldot_blocks(n);
    hipLaunchKernelGGL((col_xr<T>), dim3((unsigned)nb), dim3(256), 0, s, X, Rv, Pv, Q, alpha, n, R,
                       ceil_div(n, nb), part);
    hipLaunchKernelGGL(coldot_stage2, dim3(1), dim3(64), 0, s, part, (int)nb, R, rr);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}
template afn_status col_xr_launch<float>(float *, float *, const float *, const float *, const double *,
                                         int64_t, int, double *, double *, hipStream_t);
template afn_status col_xr_launch<double>(double *, double *, const double *, const double *,
                                          const double *, int64_t, int, double *, double *, hipStream_t);

template <typename T>
afn_status col_p_launch(T *Pv, const T *Z, const double *beta, int64_t n, int R, hipStream_t s)
{
    hipLaunchKernelGGL((col_p<T>), dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, Pv, Z, beta, n, R);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}
template afn_status col_p_launch<float>(float *, const float *, const double *, int64_t, int, hipStream_t);
template afn_status col_p_launch<double>(double *, const double *, const double *, int64_t, int,
                                         hipStream_t);

afn_status col_alpha_launch(const double *rho, const double *pq, const int *active, double *alpha, int R,
                            int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(col_alpha, dim3(1), dim3(64), 0, s, rho, pq, (int *)active, alpha, R, bad);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status col_beta_launch(double *rho, const double *rho_new, const int *active, double *beta, int R,
                           hipStream_t s)
{
    hipLaunchKernelGGL(col_beta, dim3(1), dim3(64), 0, s, rho, rho_new, active, beta, R);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status col_converged_launch(const double *rr, const double *bnorm2, const double *tol, int *active,
                                int *count, int R, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(col_converged, dim3(1), dim3(64), 0, s, rr, bnorm2, tol, active, count, R, bad);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

template <typename T>
afn_status gather_rows(const double *X, int64_t ld, const int32_t *perm, int64_t n, int R,
                       const double *scale, T *Y, hipStream_t s)
{
    hipLaunchKernelGGL((gather_rowmajor<T>), dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, X, ld,
                       perm, n, R, scale, Y);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}
template afn_status gather_rows<float>(const double *, int64_t, const int32_t *, int64_t, int,
                                       const double *, float *, hipStream_t);
template afn_status gather_rows<double>(const double *, int64_t, const int32_t *, int64_t, int,
                                        const double *, double *, hipStream_t);

afn_status scatter_rows(const double *Y, const int32_t *perm, int64_t n, int R, double *X, int64_t ld,
                        hipStream_t s)
{
    hipLaunchKernelGGL(scatter_rowmajor, dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, Y, perm, n,
                       R, X, ld);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status scatter_rows_f32(const float *Y, int64_t n, int R, double *X, int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(scatter_rowmajor_f32, dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, Y, n, R,
                       X, ld);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status sub_rows_launch(const double *B, const double *Y, double *Rr, int64_t total, hipStream_t s)
{
    hipLaunchKernelGGL(sub_rows, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, B, Y, Rr, total);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status scale_to_f32_launch(const double *r, const double *inv, float *r32, int64_t n, int R,
                               hipStream_t s)
{
    hipLaunchKernelGGL(scale_to_f32, dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, r, inv, r32, n, R);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status axpy_cols_f32_launch(const double *a, const float *e32, double *x, int64_t n, int R,
                                hipStream_t s)
{
    hipLaunchKernelGGL(axpy_cols_f32, dim3((unsigned)ceil_div(n * R, 256)), dim3(256), 0, s, a, e32, x, n, R);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
