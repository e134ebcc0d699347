// FSAI of the Schur complement (Algorithm 1 applied as in Algorithm 2).
//
// Row p of G (pattern s, m = |s| <= w <= 128 entries, p last):
//   S_ss = K22[s,s] + mu I - V_s^T V_s          (V = L^{-1} K12, k x nr)
//   S_ss = R R^T (Cholesky),   g = R^{-T} e_m
// which equals Algorithm 1's  e_m^T S_ss^{-1} / sqrt(e_m^T S_ss^{-1} e_m):
// with y = S_ss^{-1} e_m = R^{-T} R^{-1} e_m and R^{-1} e_m = e_m / R_mm,
// y_m = 1 / R_mm^2, so y / sqrt(y_m) = R^{-T} e_m.
//
// One wavefront (workgroup of 64) per row, pattern padded to N = 16 NT:
//  1. Gram V_s^T V_s on MFMA (v_mfma_f64_16x16x4f64): the k x N gathered
//     columns of V stream through LDS in chunks of 16 (coalesced along k);
//     the same 16 x 4 fragment of a tile row serves as A and B operand, and
//     only the NT (NT + 1) / 2 tiles on and below the diagonal are formed.
//  2. S_ss = K22[s,s] + mu I - Gram in the accumulator layout; padding
//     rows/columns (a >= m) become the identity.  The lower triangle goes to
//     LDS (packed) and comes back one row per lane.
//  3. Cholesky S_ss = R R^T in registers: lane r holds row r; the column of
//     step j is broadcast lane by lane (v_readlane).
//  4. g = R^{-T} e_m by back substitution (a wavefront sum per entry).
//
// Patterns wider than 64 (w <= 128) take one workgroup of four waves per row
// with the pattern padded to 128: the Gram tiles are shared among the waves,
// S_ss sits in LDS, and the Cholesky factor and the substitution go by
// 64 x 64 blocks, each diagonal block by the register Cholesky above.
//
// The transpose G^T (CSR over columns) is filled with atomic cursors and
// then put in ascending row order per column: one wavefront per column ranks
// each entry among its column's entries (rows in a column are distinct), so
// the layout, and every sum over it, does not depend on scheduling.
#include "afn_internal.h"
#include "kfun.h"

namespace afn {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

constexpr int tile_index(int I, int J) { return I * (I + 1) / 2 + J; }

// Two waves per SIMD: without the bound the compiler keeps the Gram tiles
// in accumulation registers on top of 221 others (one wave per SIMD, a
// third slower on the gathers); with it they share the 256 registers, no
// spill.
template <int NT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void fsai_row_mfma(const double *__restrict__ Xp, int k, int d, double l2,
                                                    int kind, double mu, const double *__restrict__ V,
                                                    const int32_t *__restrict__ cols, int w,
                                                    double *__restrict__ gval, int *info,
                                                    const int32_t *__restrict__ order, int64_t row0,
                                                    int64_t G, int64_t vbase)
{
    constexpr int N = 16 * NT;
    constexpr int TK = 16;
    constexpr int QN = N * TK / 64;          // staged values per lane and chunk
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int PACK = N * (N + 1) / 2;
    constexpr int STAGE = TK * (N + 1);
    __shared__ double lds[PACK > STAGE ? PACK : STAGE];
    __shared__ int sidx[N];
    const int lane = threadIdx.x;
    const int64_t slot = row0 + xcd_contiguous(blockIdx.x, G);
    const int64_t p = order ? (int64_t)order[slot] : slot;
    const int m = (int)(p + 1 < w ? p + 1 : w);
    if (lane < N) sidx[lane] = lane < m ? cols[p * w + lane] : -1;
    __syncthreads();

    // chunk t0 of the gathered columns: lane takes entries e = lane + 64 q,
    // column a = e / TK, row t0 + e % TK (16 consecutive lanes read 128
    // contiguous bytes of one column); out-of-range entries load a valid
    // address and are zeroed, so all loads issue back to back.  The column of
    // pattern entry a is V[:, s_a], or column (p - vbase) w + a of a batch of
    // recomputed pattern columns (vbase >= 0).
    auto load_chunk = [&](int t0, double (&dst)[QN]) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int e = lane + 64 * q;
            const int a = e / TK, tt = e - a * TK;
            const int c = sidx[a];
            const bool ok = c >= 0 && t0 + tt < k;
            const int64_t vc = vbase >= 0 ? (p - vbase) * w + a : (int64_t)c;
            dst[q] = V[ok ? (int64_t)(t0 + tt) + vc * k : 0];
            if (!ok) dst[q] = 0.0;
        }
    };
    doublex4 acc[NTILE];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    double nxt[QN];
    if (k > 0) load_chunk(0, nxt);
    for (int t0 = 0; t0 < k; t0 += TK) {
        double cur[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) cur[q] = nxt[q];
        if (t0 + TK < k) load_chunk(t0 + TK, nxt);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int e = lane + 64 * q;
            const int a = e / TK, tt = e - a * TK;
            lds[tt * (N + 1) + a] = cur[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TK / 4; ++q) {
            double f[NT];
#pragma unroll
            for (int I = 0; I < NT; ++I) f[I] = lds[(4 * q + (lane >> 4)) * (N + 1) + 16 * I + (lane & 15)];
#pragma unroll
            for (int I = 0; I < NT; ++I)
#pragma unroll
                for (int J = 0; J <= I; ++J)
                    acc[tile_index(I, J)] =
                        __builtin_amdgcn_mfma_f64_16x16x4f64(f[I], f[J], acc[tile_index(I, J)], 0, 0, 0);
        }
        __syncthreads();
    }

    // S_ss entries of the lower tiles: lane l, element i -> (16I + l/16 + 4i, 16J + l%16)
    const double *Xr = Xp + (int64_t)k * d;
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * I + (lane >> 4) + 4 * i, c = 16 * J + (lane & 15);
                if (r < c) continue;
                double v;
                if (r < m && c < m) {
                    const double *xa = Xr + (int64_t)sidx[r] * d, *xb = Xr + (int64_t)sidx[c] * d;
                    double dd = 0.0;
                    for (int t = 0; t < d; ++t) {
                        const double del = xa[t] - xb[t];
                        dd = __builtin_fma(del, del, dd);
                    }
                    v = kernel_d2(dd, l2, kind) + (r == c ? mu : 0.0) - acc[tile_index(I, J)][i];
                } else {
                    v = r == c ? 1.0 : 0.0;
                }
                lds[r * (r + 1) / 2 + c] = v;
            }
    __syncthreads();
    double a[N];
#pragma unroll
    for (int c = 0; c < N; ++c) a[c] = (lane < N && c <= lane) ? lds[lane * (lane + 1) / 2 + c] : 0.0;

    // Cholesky: after step j, lane r holds R[r][j] in a[j] (r >= j)
    bool bad = false;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double djj = readlane_f64(a[j], j);
        bad = bad || !(djj > 0.0);
        const double rjj = sqrt(djj > 0.0 ? djj : 1.0);
        const double lr = lane == j ? rjj : a[j] / rjj;
        a[j] = lr;
#pragma unroll
        for (int c = j + 1; c < N; ++c) a[c] = __builtin_fma(-lr, readlane_f64(lr, c), a[c]);
    }
    if (bad && lane == 0) atomicAdd(info, 1);     // rows whose block is not positive definite

    // R^T g = e_{m-1} column by column: R goes back through LDS so that lane t
    // holds column t (a[i] = R[i][t], i >= t); b is the running right-hand side.
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N; ++c)
        if (lane < N && c <= lane) lds[lane * (lane + 1) / 2 + c] = a[c];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = (lane < N && i >= lane) ? lds[i * (i + 1) / 2 + lane] : 0.0;
    double b = lane == m - 1 ? 1.0 : 0.0, g = 0.0;
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        const double gi = readlane_f64(b, i) / readlane_f64(a[i], i);
        if (lane == i) g = gi;
        b = __builtin_fma(-a[i], gi, b);
    }
    if (lane < w) gval[p * w + lane] = lane < m ? g : 0.0;
}

__device__ __forceinline__ int packed(int r, int c) { return r * (r + 1) / 2 + c; }

// Cholesky of a 64 x 64 block in registers: lane r holds row r (a[c], c <=
// r, zero above); on return a[c] = R[r][c].  False if a pivot is not positive.
__device__ __forceinline__ bool chol64_regs(double (&a)[64], int lane)
{
    bool bad = false;
#pragma unroll
    for (int j = 0; j < 64; ++j) {
        const double djj = readlane_f64(a[j], j);
        bad = bad || !(djj > 0.0);
        const double rjj = sqrt(djj > 0.0 ? djj : 1.0);
        const double lr = lane == j ? rjj : a[j] / rjj;
        a[j] = lr;
#pragma unroll
        for (int c = j + 1; c < 64; ++c) a[c] = __builtin_fma(-lr, readlane_f64(lr, c), a[c]);
    }
    return !bad;
}

// R^T g = b for a 64 x 64 lower R: lane t holds column t (a[i] = R[i][t],
// i >= t) and b[t]; returns g[t].
__device__ __forceinline__ double backsub64(const double (&a)[64], double b, int lane)
{
    double g = 0.0;
#pragma unroll
    for (int i = 63; i >= 0; --i) {
        const double gi = readlane_f64(b, i) / readlane_f64(a[i], i);
        if (lane == i) g = gi;
        b = __builtin_fma(-a[i], gi, b);
    }
    return g;
}

// FSAI row for 64 < w <= 128: one workgroup of 256 per row, N = 128.
//  1. Gram on MFMA: the 36 lower 16 x 16 tiles go to the waves round-robin
//     (tile t to wave t mod 4), the gathered 16-deep chunks of the pattern
//     columns are staged once in LDS for all four.
//  2. S_ss (lower, packed) in LDS; padding rows/columns are the identity.
//  3. With S = [S11 .; S21 S22] in 64-blocks: R11 = chol(S11) (wave 0);
//     R21 = S21 R11^{-T} (wave 1, row 64 + l in lane l, forward substitution
//     against R11 read from LDS); S22 -= R21 R21^T on MFMA (the ten lower
//     tiles over the four waves); R22 = chol(S22) (wave 0).
//  4. g = R^{-T} e_m (wave 0): R22^T g2 = e2, then R11^T g1 = e1 - R21^T g2.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void fsai_row_wide(
    const double *__restrict__ Xp, int k, int d, double l2, int kind, double mu, const double *__restrict__ V,
    const int32_t *__restrict__ cols, int w, double *__restrict__ gval, int *info, const int32_t *__restrict__ order,
    int64_t row0, int64_t G, int64_t vbase)
{
    constexpr int N = 128;
    constexpr int TK = 16;
    constexpr int LD = N + 1;                  // staging row stride (doubles)
    constexpr int QN = N * TK / 256;           // staged values per thread and chunk
    constexpr int PACK = N * (N + 1) / 2;
    static_assert(TK * LD <= PACK, "staging area inside the packed triangle");
    __shared__ double lds[PACK];
    __shared__ int sidx[N];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t slot = row0 + xcd_contiguous(blockIdx.x, G);
    const int64_t p = order ? (int64_t)order[slot] : slot;
    const int m = (int)(p + 1 < w ? p + 1 : w);
    if (tid < N) sidx[tid] = tid < m ? cols[p * w + tid] : -1;
    __syncthreads();

    // this wave's Gram tiles t = wave + 4 u = I (I + 1) / 2 + J, J <= I < 8
    int TI[9], TJ[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) {
        const int t = wave + 4 * u;
        const int I = (int)((__builtin_sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        TI[u] = I;
        TJ[u] = t - I * (I + 1) / 2;
    }
    auto load_chunk = [&](int t0, double (&dst)[QN]) {
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int e = tid + 256 * q;
            const int a = e / TK, tt = e - a * TK;
            const int c = sidx[a];
            const bool ok = c >= 0 && t0 + tt < k;
            const int64_t vc = vbase >= 0 ? (p - vbase) * w + a : (int64_t)c;
            dst[q] = V[ok ? (int64_t)(t0 + tt) + vc * k : 0];
            if (!ok) dst[q] = 0.0;
        }
    };
    doublex4 acc[9];
#pragma unroll
    for (int u = 0; u < 9; ++u) acc[u] = doublex4{0.0, 0.0, 0.0, 0.0};
    double nxt[QN];
    if (k > 0) load_chunk(0, nxt);
    for (int t0 = 0; t0 < k; t0 += TK) {
        double cur[QN];
#pragma unroll
        for (int q = 0; q < QN; ++q) cur[q] = nxt[q];
        if (t0 + TK < k) load_chunk(t0 + TK, nxt);
#pragma unroll
        for (int q = 0; q < QN; ++q) {
            const int e = tid + 256 * q;
            const int a = e / TK, tt = e - a * TK;
            lds[tt * LD + a] = cur[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TK / 4; ++q) {
            const double *row = lds + (4 * q + lk) * LD + lr;
#pragma unroll
            for (int u = 0; u < 9; ++u)
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[16 * TI[u]], row[16 * TJ[u]], acc[u], 0, 0, 0);
        }
        __syncthreads();
    }

    // S_ss: lane l, element i of tile (I, J) -> (16I + l/16 + 4i, 16J + l%16)
    const double *Xr = Xp + (int64_t)k * d;
#pragma unroll
    for (int u = 0; u < 9; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * TI[u] + lk + 4 * i, c = 16 * TJ[u] + lr;
            if (r < c) continue;
            double v;
            if (r < m && c < m) {
                const double *xa = Xr + (int64_t)sidx[r] * d, *xb = Xr + (int64_t)sidx[c] * d;
                double dd = 0.0;
                for (int t = 0; t < d; ++t) {
                    const double del = xa[t] - xb[t];
                    dd = __builtin_fma(del, del, dd);
                }
                v = kernel_d2(dd, l2, kind) + (r == c ? mu : 0.0) - acc[u][i];
            } else {
                v = r == c ? 1.0 : 0.0;
            }
            lds[packed(r, c)] = v;
        }
    __syncthreads();

    bool ok = true;
    double a[64];
#pragma nounroll
    for (int blk = 0; blk < 2; ++blk) {
        const int o = 64 * blk;
        if (wave == 0) {
#pragma unroll
            for (int c = 0; c < 64; ++c) a[c] = c <= lane ? lds[packed(o + lane, o + c)] : 0.0;
            ok = chol64_regs(a, lane) && ok;
#pragma unroll
            for (int c = 0; c < 64; ++c)
                if (c <= lane) lds[packed(o + lane, o + c)] = a[c];
        }
        __syncthreads();
        if (blk == 1) break;
        if (wave == 1) {
            // row 64 + lane of R21: R11 x = S21[row, :]^T by forward substitution
#pragma unroll
            for (int c = 0; c < 64; ++c) a[c] = lds[packed(64 + lane, c)];
#pragma unroll
            for (int c = 0; c < 64; ++c) {
                double sc = a[c];
#pragma unroll
                for (int t = 0; t < c; ++t) sc = __builtin_fma(-lds[packed(c, t)], a[t], sc);
                a[c] = sc / lds[packed(c, c)];
            }
#pragma unroll
            for (int c = 0; c < 64; ++c) lds[packed(64 + lane, c)] = a[c];
        }
        __syncthreads();
        // S22 -= R21 R21^T: lower tile t = I (I + 1) / 2 + J of the 4 x 4 tiles
        for (int t = wave; t < 10; t += 4) {
            const int I = t < 1 ? 0 : (t < 3 ? 1 : (t < 6 ? 2 : 3));
            const int J = t - I * (I + 1) / 2;
            doublex4 s4 = doublex4{0.0, 0.0, 0.0, 0.0};
            const double *ra = lds + packed(64 + 16 * I + lr, 0) + lk;
            const double *rb = lds + packed(64 + 16 * J + lr, 0) + lk;
#pragma unroll
            for (int q = 0; q < 16; ++q) s4 = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[4 * q], rb[4 * q], s4, 0, 0, 0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * I + lk + 4 * i, c = 16 * J + lr;
                if (r >= c) lds[packed(64 + r, 64 + c)] -= s4[i];
            }
        }
        __syncthreads();
    }
    if (wave != 0) return;
    if (!ok && lane == 0) atomicAdd(info, 1);

    // R22^T g2 = e2, then R11^T g1 = e1 - R21^T g2 (lane t holds column t)
    double rhs = lane == m - 1 - 64 ? 1.0 : 0.0;
    double g1 = 0.0, g2 = 0.0;
#pragma nounroll
    for (int blk = 1; blk >= 0; --blk) {
        const int o = 64 * blk;
#pragma unroll
        for (int i = 0; i < 64; ++i) a[i] = i >= lane ? lds[packed(o + i, o + lane)] : 0.0;
        const double g = backsub64(a, rhs, lane);
        if (blk == 1) {
            g2 = g;
            rhs = lane == m - 1 ? 1.0 : 0.0;
#pragma unroll
            for (int i = 0; i < 64; ++i) rhs = __builtin_fma(-lds[packed(64 + i, lane)], readlane_f64(g, i), rhs);
        } else {
            g1 = g;
        }
    }
    if (lane < w) gval[p * w + lane] = lane < m ? g1 : 0.0;
    if (64 + lane < w) gval[p * w + 64 + lane] = 64 + lane < m ? g2 : 0.0;
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

// Entry i of column c goes to position ptr[c] + #{entries of c with a smaller
// row} (ties by fill position, so the placement is a permutation even for
// malformed input); one wavefront per column.
__global__ __launch_bounds__(256) void place_sorted(const int64_t *__restrict__ ptr, int64_t nr,
                                                    const int32_t *__restrict__ urow,
                                                    const double *__restrict__ uval,
                                                    int32_t *__restrict__ trow, double *__restrict__ tval)
{
    const int lane = threadIdx.x & 63;
    const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nr) return;
    const int64_t b = ptr[c], len = ptr[c + 1] - b;
    for (int64_t i = lane; i < len; i += 64) {
        const int32_t r = urow[b + i];
        int64_t rank = 0;
        for (int64_t j = 0; j < len; ++j) {
            const int32_t q = urow[b + j];
            rank += (q < r || (q == r && j < i)) ? 1 : 0;
        }
        trow[b + rank] = r;
        tval[b + rank] = uval[b + i];
    }
}

}  // namespace

afn_status fsai_rows(const double *Xp, int64_t n, int k, int d, double l, int kind, double mu,
                     const double *V, const int32_t *cols, int w, double *gval, int *info,
                     const int32_t *order, hipStream_t s)
{
    const int64_t nr = n - k;
    if (nr <= 0) return AFN_OK;
    const int64_t chunk = 1 << 20;
    for (int64_t r0 = 0; r0 < nr; r0 += chunk) {
        const int64_t cnt = nr - r0 < chunk ? nr - r0 : chunk;
        const dim3 grid((unsigned)cnt), block(64);
        if (w > 64) {
            hipLaunchKernelGGL(fsai_row_wide, grid, dim3(256), 0, s, Xp, k, d, l * l, kind, mu, V, cols, w, gval, info, order, r0, cnt, (int64_t)-1);
            AFN_HIP(hipGetLastError());
            continue;
        }
        switch ((w + 15) / 16) {
            case 1: hipLaunchKernelGGL(fsai_row_mfma<1>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, V, cols, w, gval, info, order, r0, cnt, (int64_t)-1); break;
            case 2: hipLaunchKernelGGL(fsai_row_mfma<2>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, V, cols, w, gval, info, order, r0, cnt, (int64_t)-1); break;
            case 3: hipLaunchKernelGGL(fsai_row_mfma<3>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, V, cols, w, gval, info, order, r0, cnt, (int64_t)-1); break;
            default: hipLaunchKernelGGL(fsai_row_mfma<4>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, V, cols, w, gval, info, order, r0, cnt, (int64_t)-1); break;
        }
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

int64_t fsai_batch_rows(int k, int w)
{
    // about 256 MB of recomputed columns per batch, between 16 and 4096 rows
    const int64_t per_row = (int64_t)(k > 0 ? k : 1) * w * 8;
    int64_t b = ((int64_t)256 << 20) / per_row;
    b = b < 16 ? 16 : (b > 4096 ? 4096 : b);
    return b;
}

int64_t fsai_batch_doubles(int k, int w)
{
    const int64_t cols = fsai_batch_rows(k, w) * w;
    // the last batch is shorter: its GEMMs may use more splits than a full one
    return 2 * (int64_t)(k > 0 ? k : 1) * cols + gemm_part_bound(cols);
}

afn_status fsai_rows_batched(const double *Xp, int64_t n, int k, int d, double l, int kind, double mu,
                             const double *Linv, const int32_t *cols, int w, double *gval, int *info,
                             double *work, hipStream_t s)
{
    const int64_t nr = n - k;
    if (nr <= 0) return AFN_OK;
    const int64_t B = fsai_batch_rows(k, w);
    const int64_t kk = k > 0 ? k : 1;
    double *kb = work;                       // K12 columns of the batch's patterns (k x B w)
    double *vb = kb + kk * B * w;            // L^{-1} times them
    double *gp = vb + kk * B * w;            // GEMM partial sums
    for (int64_t r0 = 0; r0 < nr; r0 += B) {
        const int64_t cnt = nr - r0 < B ? nr - r0 : B;
        if (k > 0) {
            AFN_TRY(fill_k12_patterns(Xp, n, k, d, l, kind, cols, w, r0, cnt, kb, s));
            // vb = L^{-1} kb, as vb^T = kb^T L^{-T} in 64-column blocks of L^{-T}
            // (row-major with leading dimension k: L^{-T}(t, c) = Linv[c + t k])
            for (int c0 = 0; c0 < k; c0 += 64) {
                const int rc = k - c0 < 64 ? k - c0 : 64;
                AFN_TRY(gemm_rows<double>(kb, k, 1, cnt * w, k, Linv + c0, k, rc, nullptr, 1.0, vb + c0, k, gp, s));
            }
        }
        const dim3 grid((unsigned)cnt), block(64);
        if (w > 64) {
            hipLaunchKernelGGL(fsai_row_wide, grid, dim3(256), 0, s, Xp, k, d, l * l, kind, mu, vb, cols, w, gval, info, nullptr, r0, cnt, r0);
            AFN_HIP(hipGetLastError());
            continue;
        }
        switch ((w + 15) / 16) {
            case 1: hipLaunchKernelGGL(fsai_row_mfma<1>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, vb, cols, w, gval, info, nullptr, r0, cnt, r0); break;
            case 2: hipLaunchKernelGGL(fsai_row_mfma<2>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, vb, cols, w, gval, info, nullptr, r0, cnt, r0); break;
            case 3: hipLaunchKernelGGL(fsai_row_mfma<3>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, vb, cols, w, gval, info, nullptr, r0, cnt, r0); break;
            default: hipLaunchKernelGGL(fsai_row_mfma<4>, grid, block, 0, s, Xp, k, d, l * l, kind, mu, vb, cols, w, gval, info, nullptr, r0, cnt, r0); break;
        }
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

size_t fsai_transpose_work_bytes(int64_t nr, int w)
{
    const int64_t nnz = nr * w;
    return (size_t)(round_up(8 * (nr > 0 ? nr : 1), 256) + round_up(4 * (nnz > 0 ? nnz : 1), 256) +
                    round_up(8 * (nnz > 0 ? nnz : 1), 256));
}

afn_status fsai_transpose(const int32_t *cols, const double *gval, int64_t nr, int w,
                          int64_t *tptr, int32_t *trow, double *tval, void *work, hipStream_t s)
{
    if (nr <= 0) {
        AFN_HIP(hipMemsetAsync(tptr, 0, sizeof(int64_t), s));
        return AFN_OK;
    }
    char *base = (char *)work;
    unsigned long long *cnt = (unsigned long long *)base;
    int32_t *urow = (int32_t *)(base + round_up(8 * nr, 256));
    double *uval = (double *)(base + round_up(8 * nr, 256) + round_up(4 * nr * w, 256));
    AFN_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)nr, s));
    const unsigned blocks = (unsigned)ceil_div(nr * w, 256);
    hipLaunchKernelGGL(count_cols, dim3(blocks), dim3(256), 0, s, cols, nr, w, cnt);
    hipLaunchKernelGGL(scan_counts, dim3(1), dim3(1024), 0, s, cnt, nr, tptr);
    AFN_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)nr, s));
    hipLaunchKernelGGL(fill_transpose, dim3(blocks), dim3(256), 0, s, cols, gval, nr, w, tptr, cnt,
                       urow, uval);
    hipLaunchKernelGGL(place_sorted, dim3((unsigned)ceil_div(nr, 4)), dim3(256), 0, s, tptr, nr, urow,
                       uval, trow, tval);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
