// Kernel matvec y = (K + mu I) v with the kernel evaluated on the fly
// (Eq. (1.1); Gaussian Eq. (1.2) or Matern-3/2, Section 5).
//
// FP64 path (d <= 8): symmetric tiles.  Coordinates are pre-scaled by
// kernel_scale(kind, l) (SoA, zero-padded), so K_ij is a function of the
// squared distance t of the scaled points alone (kfun.h).  The 64-point tile partition is grouped into
// super-blocks of ST tiles; one workgroup owns a super-block pair (BI <= BJ)
// and evaluates every unique pair once, adding K_ij v_j to row i and K_ij v_i
// to row j.  Row partials stay in registers across the column tiles; column
// partials are reduced over the 16 thread-rows through LDS in a fixed order.
// Each workgroup writes one row-partial and one column-partial vector; a final
// pass adds them in ascending super-block order (deterministic result).
// Diagonal 64 x 64 tiles are evaluated in full and feed rows only.
//
// Generic d (> 8) and the FP32 variant use row-block x column-split tiles:
// 256 rows per workgroup, columns streamed through LDS, S split partials
// added in order by kmv_reduce.
#include <cmath>
#include <type_traits>

#include <cstdio>

#include "afn_internal.h"
#include "group.h"
#include "kfun.h"
#include "mfma.h"

namespace afn {
namespace {

constexpr int kRows = 256;

constexpr int kTile = 64;
constexpr int kMaxST = 16;      // super-block edge (tiles), plain kernel
constexpr int kMaxSTmf = 8;     // MFMA variant (per-wave column accumulators in LDS)
// Largest squared half-diagonal (scaled units) of a row tile whose distances
// the MFMA variant forms from norms and dot products.
constexpr double kCentredR2Max = 16.0;
// Tile pairs whose largest squared distance (scaled units) is below this take
// the table-driven FP64 exponential (valid for t < 2^25) without a clamp.
constexpr double kBoundedT = 16777216.0;

constexpr int kOriginSample = 255;

// Xs[t * npad + q] = (X[perm[q]*d + t] - o_t) * scale for q < n (perm may be
// null: identity), 0 beyond (rounded to T); grid (ceil(npad / 256), d).  o_t
// is the median of coordinate t over kOriginSample points at a fixed stride
// of the packed order (all points if fewer), found by each workgroup for
// itself.  The kernel depends on differences only; with the origin inside
// the bulk of the points, FP32 copies keep their precision for data far from
// the origin, and outliers do not move it.
template <typename T>
__global__ __launch_bounds__(256) void pack_scaled(const double *__restrict__ X,
                                                   const int32_t *__restrict__ perm, int64_t n, int d,
                                                   int64_t npad, double scale, T *__restrict__ Xs)
{
    __shared__ double smp[kOriginSample];
    __shared__ double org;
    const int t = (int)blockIdx.y, tid = (int)threadIdx.x;
    const int ns = n < kOriginSample ? (int)n : kOriginSample;
    if (tid == 0) org = 0.0;
    if (tid < ns) {
        const int64_t q = (int64_t)tid * n / ns;
        smp[tid] = X[(perm ? (int64_t)perm[q] : q) * d + t];
    }
    __syncthreads();
    if (tid < ns) {
        // rank in the order (value, sample index): the middle one is the median
        const double x = smp[tid];
        int rank = 0;
        for (int k = 0; k < ns; ++k) {
            const double y = smp[k];
            rank += y < x || (y == x && k < tid) ? 1 : 0;
        }
        if (rank == ns / 2) org = x;
    }
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * 256 + tid;
    if (q >= npad) return;
    const int64_t i = q < n ? (perm ? (int64_t)perm[q] : q) : 0;
    Xs[(int64_t)t * npad + q] = (T)(q < n ? (X[i * d + t] - org) * scale : 0.0);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// box[(tile * d + t) * 2 + {0, 1}] = min / max of the packed coordinate t over
// the valid points of the 64-point tile; an empty tile gets [+inf, -inf].
template <typename T>
__global__ __launch_bounds__(256) void tile_boxes(const T *__restrict__ Xs, int64_t npad, int64_t n, int d,
                                                  T *__restrict__ box)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = npad / kTile;
    if (e >= ntiles * d) return;
    const int64_t tile = e / d;
    const int t = (int)(e - tile * d);
    T lo = (T)__builtin_inf(), hi = -(T)__builtin_inf();
    for (int j = 0; j < kTile; ++j) {
        const int64_t q = tile * kTile + j;
        if (q >= n) break;
        const T x = Xs[(int64_t)t * npad + q];
        lo = x < lo ? x : lo;
        hi = x > hi ? x : hi;
    }
    box[e * 2] = lo;
    box[e * 2 + 1] = hi;
}

// Squared gap between the boxes of tiles a and b (0 where they overlap).
template <int D, typename T>
__device__ __forceinline__ T box_gap2(const T *__restrict__ box, int64_t a, int64_t b)
{
    T g2 = T(0);
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const T alo = box[(a * D + t) * 2], ahi = box[(a * D + t) * 2 + 1];
        const T blo = box[(b * D + t) * 2], bhi = box[(b * D + t) * 2 + 1];
        T gap = blo - ahi > alo - bhi ? blo - ahi : alo - bhi;
        gap = gap > T(0) ? gap : T(0);
        g2 = fmaT(gap, gap, g2);
    }
    return g2;
}

// Largest squared distance between a point of box a and one of box b.
template <int D, typename T>
__device__ __forceinline__ T box_span2(const T *__restrict__ box, int64_t a, int64_t b)
{
    T s2 = T(0);
#pragma unroll
    for (int t = 0; t < D; ++t) {
        const T alo = box[(a * D + t) * 2], ahi = box[(a * D + t) * 2 + 1];
        const T blo = box[(b * D + t) * 2], bhi = box[(b * D + t) * 2 + 1];
        const T span = (ahi > bhi ? ahi : bhi) - (alo < blo ? alo : blo);
        s2 = fmaT(span, span, s2);
    }
    return s2;
}

__device__ __forceinline__ void decode_pair(int q, int S, int &BI, int &BJ)
{
    int bi = 0, rem = q;
    while (rem >= S - bi) {
        rem -= S - bi;
        ++bi;
    }
    BI = bi;
    BJ = bi + rem;
}

// perm (may be null): v is indexed through it (v[perm[q]] for packed point
// q).  box (may be null): a tile pair whose box gap^2 is >= tcut is skipped:
// every kernel value in it is below the cut tcut was derived from.
template <int KIND, int D, typename T, typename VT>
__global__ __launch_bounds__(256) void kmv_sym(const T *__restrict__ Xs, int64_t npad, int64_t n,
                                               const VT *__restrict__ v, const int32_t *__restrict__ perm,
                                               const T *__restrict__ box, T tcut, int S, int ST,
                                               T *__restrict__ part)
{
    __shared__ T cx[D][kTile];
    __shared__ T cv[kTile];
    __shared__ T red[16][kTile + 1];
    __shared__ T colacc[kMaxST][kTile];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    int BI, BJ;
    decode_pair(blockIdx.x, S, BI, BJ);
    const int64_t SB = (int64_t)ST * kTile;
    const bool diag_super = BI == BJ;
    for (int e = tid; e < kMaxST * kTile; e += 256) (&colacc[0][0])[e] = T(0);
    // pruning decisions for all ST x ST tile pairs, one per thread
    __shared__ unsigned char keep[kMaxST * kMaxST];
    if (tid < ST * ST)
        keep[tid] = !box || box_gap2<D, T>(box, (int64_t)BI * ST + tid / ST, (int64_t)BJ * ST + tid % ST) < tcut;
    __syncthreads();
    T *rowout = part + (int64_t)blockIdx.x * 2 * SB;
    T *colout = rowout + SB;
    for (int ti = 0; ti < ST; ++ti) {
        const int64_t i0 = BI * SB + (int64_t)ti * kTile + ty * 4;
        T xi[4][D], vi[4], racc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int t = 0; t < D; ++t) xi[r][t] = Xs[(int64_t)t * npad + i0 + r];
            const int64_t q = i0 + r;
            vi[r] = q < n ? (T)v[perm ? (int64_t)perm[q] : q] : T(0);
            racc[r] = T(0);
        }
        for (int tj = diag_super ? ti : 0; tj < ST; ++tj) {
            const int64_t j0 = BJ * SB + (int64_t)tj * kTile;
            if (!keep[ti * ST + tj]) continue;
            __syncthreads();
            for (int e = tid; e < kTile * (D + 1); e += 256) {
                const int t = e / kTile, j = e % kTile;
                const int64_t q = j0 + j;
                if (t < D) cx[t][j] = Xs[(int64_t)t * npad + q];
                else cv[j] = q < n ? (T)v[perm ? (int64_t)perm[q] : q] : T(0);
            }
            __syncthreads();
            const bool diag_tile = diag_super && tj == ti;
            T cacc[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                T xj[D];
#pragma unroll
                for (int t = 0; t < D; ++t) xj[t] = cx[t][tx * 4 + c];
                const T vj = cv[tx * 4 + c];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    T d2 = T(0);
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        const T del = xi[r][t] - xj[t];
                        d2 = fmaT(del, del, d2);
                    }
                    const T kij = kernel_scaled<KIND, T>(d2);
                    racc[r] = fmaT(kij, vj, racc[r]);
                    cacc[c] = fmaT(kij, vi[r], cacc[c]);
                }
            }
            if (!diag_tile) {
#pragma unroll
                for (int c = 0; c < 4; ++c) red[ty][tx * 4 + c] = cacc[c];
                __syncthreads();
                if (tid < kTile) {
                    T s = T(0);
#pragma unroll
                    for (int y = 0; y < 16; ++y) s += red[y][tid];
                    colacc[tj][tid] += s;
                }
            }
        }
        // rows of tile ti: add the 16 thread-columns in order
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) red[tx][ty * 4 + r] = racc[r];
        __syncthreads();
        if (tid < kTile) {
            T s = T(0);
#pragma unroll
            for (int x = 0; x < 16; ++x) s += red[x][tid];
            rowout[(int64_t)ti * kTile + tid] = s;
        }
    }
    __syncthreads();
    for (int e = tid; e < ST * kTile; e += 256) colout[e] = (&colacc[0][0])[e];
}

// Cross-lane sums in a fixed order.  Each step keeps half of a lane's values
// and trades the other half with its partner (the empty asm keeps the
// selects on values; otherwise they are folded into a runtime index into the
// array, which becomes a compare-and-select chain).
template <typename T>
__device__ __forceinline__ void keep_or_send(bool hi, T &a, T &b, T &keep, T &send)
{
    asm volatile("" : "+v"(a), "+v"(b));
    keep = hi ? b : a;
    send = hi ? a : b;
}

// Lanes 32..63 of x trade places with lanes 0..31 of y (v_permlane32_swap),
// and, within each half, lanes 16..31 of x with lanes 0..15 of y
// (v_permlane16_swap): a transposition across lane groups with no LDS
// traffic and no lane-index arithmetic.
__device__ __forceinline__ void swap_lanes32(float &x, float &y)
{
    auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                              false, false);
    x = __builtin_bit_cast(float, (unsigned)r[0]);
    y = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void swap_lanes16(float &x, float &y)
{
    auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y),
                                              false, false);
    x = __builtin_bit_cast(float, (unsigned)r[0]);
    y = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void swap_lanes32(double &x, double &y)
{
    const unsigned long long a = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long b = __builtin_bit_cast(unsigned long long, y);
    auto lo = __builtin_amdgcn_permlane32_swap((unsigned)a, (unsigned)b, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
    x = __builtin_bit_cast(double, (unsigned long long)(unsigned)lo[0] | ((unsigned long long)(unsigned)hi[0] << 32));
    y = __builtin_bit_cast(double, (unsigned long long)(unsigned)lo[1] | ((unsigned long long)(unsigned)hi[1] << 32));
}
__device__ __forceinline__ void swap_lanes16(double &x, double &y)
{
    const unsigned long long a = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long b = __builtin_bit_cast(unsigned long long, y);
    auto lo = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
    x = __builtin_bit_cast(double, (unsigned long long)(unsigned)lo[0] | ((unsigned long long)(unsigned)hi[0] << 32));
    y = __builtin_bit_cast(double, (unsigned long long)(unsigned)lo[1] | ((unsigned long long)(unsigned)hi[1] << 32));
}

// Four values over the four lane groups (lanes l, l + 16, l + 32, l + 48):
// on return lane l holds the total of value l >> 4.  After swap_lanes32 of
// (v[j], v[2 + j]) a lane of the lower half holds its own v[j] and its
// partner's, a lane of the upper half both v[2 + j]; swap_lanes16 does the
// same between the two groups of each half.
template <typename T>
__device__ __forceinline__ T groups4_sum(T (&v)[4], int)
{
    T h[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        T x = v[j], y = v[2 + j];
        swap_lanes32(x, y);
        h[j] = x + y;
    }
    T x = h[0], y = h[1];
    swap_lanes16(x, y);
    return x + y;
}

// Four values over the 16 lanes of a lane group: on return lane l holds the
// total of value (l & 15) >> 2.
template <typename T>
__device__ __forceinline__ T lanes16_sum4(T (&v)[4], int lane)
{
    T h[2], keep, send;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        keep_or_send((lane & 8) != 0, v[j], v[2 + j], keep, send);
        h[j] = keep + __shfl_xor(send, 8);
    }
    keep_or_send((lane & 4) != 0, h[0], h[1], keep, send);
    T q = keep + __shfl_xor(send, 4);
    q += __shfl_xor(q, 2);
    q += __shfl_xor(q, 1);
    return q;
}

// The symmetric tile kernel with the distance contraction on the matrix
// cores (Hilbert-ordered points with tile boxes).
//
// In a 64 x 64 tile pair, wave w owns rows 16 w .. 16 w + 15 and all 64
// columns.  Coordinates are centred on the middle of the row tile's box; for
// each 16-column block one MFMA 16x16x4 per 4 coordinates forms
// |x_i|^2 + |x_j|^2 - 2 x_i . x_j: for d < 4 the unused coordinate slot d
// holds 1 for the rows and |x_j|^2 for the columns, and the row norms are
// the accumulator input, so no addition per pair is left (d = 4: the
// accumulator starts at the two norms).  Centring bounds the cancellation:
// with h2 the squared
// half-diagonal of the row tile's box, the distance carries an absolute
// error of about 2 (h2 + (sqrt(t) + sqrt(h2))^2) (d + 2) u, and a row tile
// with h2 > r2max uses the plain differences instead.
//
// A lane holds 4 rows x 4 columns of each tile pair.  Its column sums are
// transposed over the four lane groups so that lane l ends with column l,
// which it adds to its wave's own LDS accumulator (no barrier); the four
// waves' accumulators are added in order at the end.  Row sums are added
// over the lane group once per row tile.  Column tiles are centred and
// staged in LDS.  FP32: all kept column tiles of a row tile at once (loads
// from every thread in flight together), so the tile loop has no barrier.
// FP64 (whose registers allow 4 waves per SIMD only with a small LDS
// footprint): two buffers, the next kept tile read into registers while the
// current one is evaluated, one barrier per tile pair.  Each 16-column
// block's distances become kernel values before the next block's MFMA, and
// the box centre that column staging needs sits in LDS: that keeps the FP64
// kernel within 128 registers without spills in its loops.
template <int KIND, int D, typename T, typename VT>
struct KmvMfArgs {
    const T *Xs;
    int64_t npad, n;
    const VT *v;
    const int32_t *perm;
    const T *box;
    T tcut, tfar, r2max;
    int S, ST;
    T *part;
    static void launch1(const KmvMfArgs &p, dim3 grid, size_t lds, hipStream_t s);
    static void launchG(const GroupTable<KmvMfArgs> &t, unsigned blocks, size_t lds, hipStream_t s);
};

template <int KIND, int D, typename T, typename VT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : (D <= 4 ? 4 : 2)))) void kmv_sym_mf(
    const T *__restrict__ Xs, int64_t npad, int64_t n, const VT *__restrict__ v, const int32_t *__restrict__ perm,
    const T *__restrict__ box, T tcut, T tfar, T r2max, int S, int ST, T *__restrict__ part)
{
#define KMV_SYM_MF_BID blockIdx.x
#include "kmv_sym_mf_body.inc"
#undef KMV_SYM_MF_BID
}

// The same for several solves in one launch (group.h).
template <int KIND, int D, typename T, typename VT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 5 : (D <= 4 ? 4 : 2)))) void kmv_sym_mf_g(
    GroupTable<KmvMfArgs<KIND, D, T, VT>> t)
{
    const GroupPos q = group_pos(t);
    const KmvMfArgs<KIND, D, T, VT> &a = t.a[q.g];
    const T *__restrict__ Xs = a.Xs;
    const int64_t npad = a.npad, n = a.n;
    const VT *__restrict__ v = a.v;
    const int32_t *__restrict__ perm = a.perm;
    const T *__restrict__ box = a.box;
    const T tcut = a.tcut, tfar = a.tfar, r2max = a.r2max;
    const int S = a.S, ST = a.ST;
    T *__restrict__ part = a.part;
    const unsigned bid = (unsigned)q.bx;
#define KMV_SYM_MF_BID bid
#include "kmv_sym_mf_body.inc"
#undef KMV_SYM_MF_BID
}

template <int KIND, int D, typename T, typename VT>
void KmvMfArgs<KIND, D, T, VT>::launch1(const KmvMfArgs &p, dim3 grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((kmv_sym_mf<KIND, D, T, VT>), grid, dim3(256), lds, s, p.Xs, p.npad, p.n, p.v, p.perm, p.box,
                       p.tcut, p.tfar, p.r2max, p.S, p.ST, p.part);
}

template <int KIND, int D, typename T, typename VT>
void KmvMfArgs<KIND, D, T, VT>::launchG(const GroupTable<KmvMfArgs> &t, unsigned blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((kmv_sym_mf_g<KIND, D, T, VT>), dim3(blocks), dim3(256), lds, s, t);
}

// y_i = sum over BJ >= s of row partials + sum over BI <= s of column
// partials (ascending) + mu v_i, s = super-block of i.
template <typename T, typename VT>
struct KmvRedArgs {
    const T *part;
    int64_t n;
    int S, ST;
    double mu;
    const VT *v;
    const int32_t *perm;
    VT *y;
    static void launch1(const KmvRedArgs &p, dim3 grid, size_t lds, hipStream_t s);
    static void launchG(const GroupTable<KmvRedArgs> &t, unsigned blocks, size_t lds, hipStream_t s);
};

template <typename T, typename VT>
__device__ __forceinline__ void kmv_sym_reduce_body(const KmvRedArgs<T, VT> &args, int64_t bx)
{
    const T *__restrict__ part = args.part;
    const int64_t n = args.n;
    const int S = args.S, ST = args.ST;
    const double mu = args.mu;
    const VT *__restrict__ v = args.v;
    const int32_t *__restrict__ perm = args.perm;
    VT *__restrict__ y = args.y;
    const int64_t i = bx * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = perm ? (int64_t)perm[i] : i;
    const int64_t SB = (int64_t)ST * kTile;
    const int s = (int)(i / SB);
    const int64_t ii = i - (int64_t)s * SB;
    double acc = 0.0;
    const int64_t qs = (int64_t)s * S - (int64_t)s * (s - 1) / 2;   // q(s, s)
    // 8 loads in flight per thread; the additions stay in index order
    constexpr int U = 8;
    int bj = s;
    for (; bj + U <= S; bj += U) {
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = part[(qs + bj + u - s) * 2 * SB + ii];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)a[u];
    }
    for (; bj < S; ++bj) acc += (double)part[(qs + bj - s) * 2 * SB + ii];
    auto colq = [&](int bi) { return (int64_t)bi * S - (int64_t)bi * (bi - 1) / 2 + (s - bi); };
    int bi = 0;
    for (; bi + U <= s + 1; bi += U) {
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) a[u] = part[colq(bi + u) * 2 * SB + SB + ii];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)a[u];
    }
    for (; bi <= s; ++bi) acc += (double)part[colq(bi) * 2 * SB + SB + ii];
    y[o] = (VT)(acc + mu * (double)v[o]);
}

template <typename T, typename VT>
__global__ __launch_bounds__(256) void kmv_sym_reduce(KmvRedArgs<T, VT> args) { kmv_sym_reduce_body(args, blockIdx.x); }

template <typename T, typename VT>
__global__ __launch_bounds__(256) void kmv_sym_reduce_g(GroupTable<KmvRedArgs<T, VT>> t)
{
    const GroupPos q = group_pos(t);
    kmv_sym_reduce_body(t.a[q.g], q.bx);
}

template <typename T, typename VT>
void KmvRedArgs<T, VT>::launch1(const KmvRedArgs &p, dim3 grid, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((kmv_sym_reduce<T, VT>), grid, dim3(256), lds, s, p);
}

template <typename T, typename VT>
void KmvRedArgs<T, VT>::launchG(const GroupTable<KmvRedArgs> &t, unsigned blocks, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((kmv_sym_reduce_g<T, VT>), dim3(blocks), dim3(256), lds, s, t);
}

// Generic tiles (any d <= D): one thread per row, the row's coordinates in
// registers zero-padded to D, column coordinates staged through LDS (also
// zero-padded, so the padding adds nothing to the distance).  Unscaled
// coordinates; c2 = kernel_scale(kind, l)^2 turns the squared distance into
// the scaled one.
template <int KIND, int D, int BN>
__global__ __launch_bounds__(256) void kmv_f64_partial(const double *__restrict__ X, int64_t n,
                                                       int d, double c2,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ part,
                                                       int64_t split_len)
{
    __shared__ double sx[D * BN];
    __shared__ double sv[BN];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kRows + tid;
    const int64_t c0 = (int64_t)blockIdx.y * split_len;
    const int64_t c1 = c0 + split_len < n ? c0 + split_len : n;
    const bool row_ok = i < n;
    double xi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = (row_ok && t < d) ? X[i * d + t] : 0.0;
    double acc = 0.0;
    for (int64_t j0 = c0; j0 < c1; j0 += BN) {
        const int jn = (int)(c1 - j0 < BN ? c1 - j0 : BN);
        for (int e = tid; e < BN * D; e += blockDim.x) {
            const int j = e / D, t = e - j * D;
            sx[t * BN + j] = (j < jn && t < d) ? X[(j0 + j) * d + t] : 0.0;
        }
        for (int j = tid; j < BN; j += blockDim.x) sv[j] = j < jn ? v[j0 + j] : 0.0;
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < jn; ++j) {
            double d2 = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const double del = xi[t] - sx[t * BN + j];
                d2 = __builtin_fma(del, del, d2);
            }
            acc = __builtin_fma(kernel_scaled<KIND, double>(d2 * c2), sv[j], acc);
        }
        __syncthreads();
    }
    if (row_ok) part[(int64_t)blockIdx.y * n + i] = acc;
}

// FP32 tiles: coordinates rounded to FP32 on load, squared distance and the
// kernel value in FP32 (the hardware base-2 exponential), FP32 accumulation
// within a split; the S split partials are added in FP64 by kmv_reduce.  Same
// layout as above.
template <int KIND, int D, int BN>
__global__ __launch_bounds__(256) void kmv_f32_partial(const double *__restrict__ X, int64_t n,
                                                       int d, float c2,
                                                       const double *__restrict__ v,
                                                       double *__restrict__ part,
                                                       int64_t split_len)
{
    __shared__ float sx[D * BN];
    __shared__ float sv[BN];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * kRows + tid;
    const int64_t c0 = (int64_t)blockIdx.y * split_len;
    const int64_t c1 = c0 + split_len < n ? c0 + split_len : n;
    const bool row_ok = i < n;
    float xi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = (row_ok && t < d) ? (float)X[i * d + t] : 0.0f;
    float acc = 0.0f;
    for (int64_t j0 = c0; j0 < c1; j0 += BN) {
        const int jn = (int)(c1 - j0 < BN ? c1 - j0 : BN);
        for (int e = tid; e < BN * D; e += blockDim.x) {
            const int j = e / D, t = e - j * D;
            sx[t * BN + j] = (j < jn && t < d) ? (float)X[(j0 + j) * d + t] : 0.0f;
        }
        for (int j = tid; j < BN; j += blockDim.x) sv[j] = j < jn ? (float)v[j0 + j] : 0.0f;
        __syncthreads();
#pragma unroll 8
        for (int j = 0; j < jn; ++j) {
            float d2 = 0.0f;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                const float del = xi[t] - sx[t * BN + j];
                d2 = __builtin_fmaf(del, del, d2);
            }
            acc = __builtin_fmaf(kernel_scaled<KIND, float>(d2 * c2), sv[j], acc);
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
void launch_partial(int kind, dim3 grid, const double *X, int64_t n, int d, double c2, const double *v,
                    double *part, int64_t split_len, hipStream_t s)
{
    if (kind == AFN_KERNEL_MATERN32)
        hipLaunchKernelGGL((kmv_f64_partial<AFN_KERNEL_MATERN32, D, BN>), grid, dim3(256), 0, s, X, n, d, c2,
                           v, part, split_len);
    else
        hipLaunchKernelGGL((kmv_f64_partial<AFN_KERNEL_GAUSSIAN, D, BN>), grid, dim3(256), 0, s, X, n, d, c2,
                           v, part, split_len);
}

template <int D, int BN>
void launch_partial32(int kind, dim3 grid, const double *X, int64_t n, int d, float c2, const double *v,
                      double *part, int64_t split_len, hipStream_t s)
{
    if (kind == AFN_KERNEL_MATERN32)
        hipLaunchKernelGGL((kmv_f32_partial<AFN_KERNEL_MATERN32, D, BN>), grid, dim3(256), 0, s, X, n, d, c2,
                           v, part, split_len);
    else
        hipLaunchKernelGGL((kmv_f32_partial<AFN_KERNEL_GAUSSIAN, D, BN>), grid, dim3(256), 0, s, X, n, d, c2,
                           v, part, split_len);
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

namespace {

// Super-block size: enough workgroups to fill the chip, at most kMaxSTmf
// tiles where the MFMA variant runs (d <= 4), kMaxST otherwise.
struct SymShape {
    int ST, S;
    int64_t npad, nwg;
};

SymShape sym_shape(int64_t n, int d)
{
    SymShape sh;
    int64_t tiles = ceil_div(n, kTile);
    int64_t st = tiles / 45;
    const int cap = d <= 8 ? kMaxSTmf : kMaxST;
    sh.ST = (int)(st < 1 ? 1 : (st > cap ? cap : st));
    sh.ST = sh.ST > 1 ? sh.ST & ~1 : 1;       // even: packed length a multiple of 128
    sh.S = (int)ceil_div(tiles, sh.ST);
    if (sh.ST == 1 && (sh.S & 1)) ++sh.S;
    sh.npad = (int64_t)sh.S * sh.ST * kTile;
    sh.nwg = (int64_t)sh.S * (sh.S + 1) / 2;
    return sh;
}

}  // namespace

int64_t kmv_workspace_doubles(int64_t n, int d)
{
    const int64_t split = kmv_splits(n) * n;     // generic-d and FP32 paths
    if (d >= 1 && d <= 8) {
        SymShape sh = sym_shape(n, d);
        const int64_t sym = sh.npad * d + sh.nwg * 2 * sh.npad / sh.S;
        return sym > split ? sym : split;
    }
    return split;
}

namespace {

template <int KIND, int D, typename T, typename VT>
void launch_mf(dim3 grid, const T *Xs, int64_t npad, int64_t n, const VT *v, const int32_t *perm, const T *box,
               T tcut, T tfar, T r2, int S, int ST, T *part, hipStream_t s)
{
    (void)dlaunch(grid, 0, s, KmvMfArgs<KIND, D, T, VT>{Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part});
}

template <int KIND, typename T, typename VT>
void launch_sym(int d, dim3 grid, const T *Xs, int64_t npad, int64_t n, const VT *v, const int32_t *perm,
                const T *box, T tcut, T tfar, int S, int ST, T *part, hipStream_t s, bool mf)
{
    const dim3 block(256);
    // the MFMA variant needs tile boxes (d <= 8: one MFMA per 4 coordinates
    // and 16 x 16 block); mf = false takes the plain differences
    if (box && d <= 8 && mf) {
        const T r2 = T(kCentredR2Max);
        switch (d) {
            case 1: launch_mf<KIND, 1, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            case 2: launch_mf<KIND, 2, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            case 3: launch_mf<KIND, 3, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            case 4: launch_mf<KIND, 4, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            case 5: launch_mf<KIND, 5, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            case 6: launch_mf<KIND, 6, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            case 7: launch_mf<KIND, 7, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
            default: launch_mf<KIND, 8, T, VT>(grid, Xs, npad, n, v, perm, box, tcut, tfar, r2, S, ST, part, s); break;
        }
        return;
    }
    // plain differences: deferred like the rest, no grouped form
    (void)defer(s, [=](hipStream_t st) {
        switch (d) {
            case 1: hipLaunchKernelGGL((kmv_sym<KIND, 1, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            case 2: hipLaunchKernelGGL((kmv_sym<KIND, 2, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            case 3: hipLaunchKernelGGL((kmv_sym<KIND, 3, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            case 4: hipLaunchKernelGGL((kmv_sym<KIND, 4, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            case 5: hipLaunchKernelGGL((kmv_sym<KIND, 5, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            case 6: hipLaunchKernelGGL((kmv_sym<KIND, 6, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            case 7: hipLaunchKernelGGL((kmv_sym<KIND, 7, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
            default: hipLaunchKernelGGL((kmv_sym<KIND, 8, T, VT>), grid, block, 0, st, Xs, npad, n, v, perm, box, tcut, S, ST, part); break;
        }
        return hipGetLastError();
    });
}

template <typename T, typename VT>
afn_status kmv_sym_run(const T *Xs, const SymShape &sh, int64_t n, int d, double mu, int kind, const VT *v,
                       int64_t ldv, VT *y, int64_t ldy, int nrhs, T *part, hipStream_t s,
                       hipEvent_t ev0, hipEvent_t ev1, const int32_t *perm, const T *box)
{
    const T tcut = (T)kernel_cut_t(kind, sizeof(T) == 8 ? kCullF64 : kCullF32);
    const T tfar = sizeof(T) == 8 ? (T)kernel_cut_t(kind, kFarF64) : (T)__builtin_inf();
    const dim3 grid((unsigned)sh.nwg);
    auto tile = [&](const VT *vc, bool mf) {
        if (kind == AFN_KERNEL_MATERN32)
            launch_sym<AFN_KERNEL_MATERN32, T, VT>(d, grid, Xs, sh.npad, n, vc, perm, box, tcut, tfar, sh.S, sh.ST,
                                                   part, s, mf);
        else
            launch_sym<AFN_KERNEL_GAUSSIAN, T, VT>(d, grid, Xs, sh.npad, n, vc, perm, box, tcut, tfar, sh.S, sh.ST,
                                                   part, s, mf);
    };
    // d = 5..8 with tile boxes: MFMA distance contraction (candidate 0) or
    // plain differences (1), by the autotuner; one column and its reduction
    // per timed run (y is written again below)
    bool mf = true;
    if (box && d >= 5 && d <= 8 && (const void *)y != (const void *)v) {
        char shape[96];
        snprintf(shape, sizeof shape, "d%d_n%lld_%s_k%d", d, (long long)n, sizeof(T) == 8 ? "f64" : "f32", kind);
        const int pick = tune_pick("kmv_tile", shape, 2, 0, [&](int c) -> afn_status {
            tile(v, c == 0);
            AFN_HIP(hipGetLastError());
            return dlaunch(dim3((unsigned)ceil_div(n, 256)), 0, s,
                           KmvRedArgs<T, VT>{part, n, sh.S, sh.ST, mu, v, perm, y});
        }, s);
        mf = pick == 0;
    }
    for (int c = 0; c < nrhs; ++c) {
        const VT *vc = v + c * ldv;
        if (ev0) AFN_TRY(defer(s, [=](hipStream_t st) { return hipEventRecord(ev0, st); }));
        tile(vc, mf);
        AFN_HIP(hipGetLastError());
        if (ev1) AFN_TRY(defer(s, [=](hipStream_t st) { return hipEventRecord(ev1, st); }));
        AFN_TRY(dlaunch(dim3((unsigned)ceil_div(n, 256)), 0, s,
                        KmvRedArgs<T, VT>{part, n, sh.S, sh.ST, mu, vc, perm, y + c * ldy}));
    }
    return AFN_OK;
}

}  // namespace

double kernel_scale(int kind, double l)
{
    if (kind == AFN_KERNEL_MATERN32) return std::sqrt(3.0) * 1.4426950408889634 / l;
    return std::sqrt(1.4426950408889634) / l;
}

// Gaussian: 2^-t = 2^-cut at t = cut.  Matern: (1 + s ln 2) 2^-s = 2^-cut at
// the root of g(s) = s - log2(1 + s ln 2) - cut, convex and increasing for
// s > 0, so Newton's method from a point right of the root decreases
// monotonically onto it; t = s^2.
double kernel_cut_t(int kind, double cut)
{
    if (kind != AFN_KERNEL_MATERN32) return cut;
    const double ln2 = 0.6931471805599453;
    double s = 2.0 * cut + 16.0;
    for (int it = 0; it < 60; ++it) {
        const double g = s - std::log2(1.0 + s * ln2) - cut;
        const double dg = s * ln2 / (1.0 + s * ln2);
        const double step = g / dg;
        s -= step;
        if (step < 1e-13 * s) break;
    }
    return s * s;
}

int64_t kmv_packed_doubles(int64_t n, int d)
{
    const SymShape sh = sym_shape(n, d);
    return sh.npad * d;
}

afn_status kmv_pack(const double *X, int64_t n, int d, double l, int kind, void *Xs, bool f32, hipStream_t s,
                    const int32_t *perm)
{
    const SymShape sh = sym_shape(n, d);
    const double scale = kernel_scale(kind, l);
    if (f32)
        hipLaunchKernelGGL(pack_scaled<float>, dim3((unsigned)ceil_div(sh.npad, 256), (unsigned)d), dim3(256), 0, s,
                           X, perm, n, d, sh.npad, scale, (float *)Xs);
    else
        hipLaunchKernelGGL(pack_scaled<double>, dim3((unsigned)ceil_div(sh.npad, 256), (unsigned)d), dim3(256), 0, s,
                           X, perm, n, d, sh.npad, scale, (double *)Xs);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

int64_t kmv_box_count(int64_t n, int d) { return sym_shape(n, d).npad / kTile * d * 2; }

namespace {

// Unordered pairs (a <= b) of non-empty tiles that the pruned kernels evaluate
// at cut^2 = tcut, and all such pairs (counts[0], counts[1]).
template <int D>
__global__ __launch_bounds__(256) void count_kept_pairs(const double *__restrict__ box, int64_t ntiles,
                                                        int64_t a0, double tcut, unsigned long long *counts)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t a = a0 + blockIdx.y;
    if (b >= ntiles || b < a) return;
    if (!(box[a * D * 2] <= box[a * D * 2 + 1]) || !(box[b * D * 2] <= box[b * D * 2 + 1])) return;
    atomicAdd(&counts[1], 1ULL);
    if (box_gap2<D, double>(box, a, b) < tcut) atomicAdd(&counts[0], 1ULL);
}

}  // namespace

afn_status kmv_kept_fraction(const double *box, int64_t n, int d, double tcut, unsigned long long *counts,
                             hipStream_t s)
{
    const int64_t ntiles = sym_shape(n, d).npad / kTile;
    AFN_HIP(hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s));
    for (int64_t a0 = 0; a0 < ntiles; a0 += 32768) {
        const int64_t rows = ntiles - a0 < 32768 ? ntiles - a0 : 32768;
        const dim3 g((unsigned)ceil_div(ntiles, 256), (unsigned)rows);
        switch (d) {
            case 1: hipLaunchKernelGGL(count_kept_pairs<1>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            case 2: hipLaunchKernelGGL(count_kept_pairs<2>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            case 3: hipLaunchKernelGGL(count_kept_pairs<3>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            case 4: hipLaunchKernelGGL(count_kept_pairs<4>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            case 5: hipLaunchKernelGGL(count_kept_pairs<5>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            case 6: hipLaunchKernelGGL(count_kept_pairs<6>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            case 7: hipLaunchKernelGGL(count_kept_pairs<7>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
            default: hipLaunchKernelGGL(count_kept_pairs<8>, g, dim3(256), 0, s, box, ntiles, a0, tcut, counts); break;
        }
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

afn_status kmv_boxes(const void *Xs, int64_t n, int d, bool f32, void *box, hipStream_t s)
{
    const SymShape sh = sym_shape(n, d);
    const unsigned g = (unsigned)ceil_div(sh.npad / kTile * d, 256);
    if (f32)
        hipLaunchKernelGGL(tile_boxes<float>, dim3(g), dim3(256), 0, s, (const float *)Xs, sh.npad, n, d,
                           (float *)box);
    else
        hipLaunchKernelGGL(tile_boxes<double>, dim3(g), dim3(256), 0, s, (const double *)Xs, sh.npad, n, d,
                           (double *)box);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status kmv_packed_f64(const double *Xs, int64_t n, int d, double mu, int kind, const double *v, int64_t ldv,
                          double *y, int64_t ldy, int nrhs, double *part, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1, const int32_t *perm, const double *box)
{
    return kmv_sym_run<double, double>(Xs, sym_shape(n, d), n, d, mu, kind, v, ldv, y, ldy, nrhs, part, s, ev0,
                                       ev1, perm, box);
}

afn_status kmv_packed_f32(const float *Xs, int64_t n, int d, double mu, int kind, const float *v, int64_t ldv,
                          float *y, int64_t ldy, int nrhs, float *part, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1, const int32_t *perm, const float *box)
{
    return kmv_sym_run<float, float>(Xs, sym_shape(n, d), n, d, mu, kind, v, ldv, y, ldy, nrhs, part, s, ev0,
                                     ev1, perm, box);
}

afn_status kmv_packed_f32_dvec(const float *Xs, int64_t n, int d, double mu, int kind, const double *v,
                               int64_t ldv, double *y, int64_t ldy, int nrhs, float *part, hipStream_t s,
                               const int32_t *perm, const float *box)
{
    return kmv_sym_run<float, double>(Xs, sym_shape(n, d), n, d, mu, kind, v, ldv, y, ldy, nrhs, part, s, nullptr,
                                      nullptr, perm, box);
}

afn_status kmv_f64(const double *X, int64_t n, int d, double l, double mu, int kind, const double *v,
                   int64_t ldv, double *y, int64_t ldy, int nrhs, double *work, hipStream_t s,
                   hipEvent_t ev0, hipEvent_t ev1)
{
    if (d >= 1 && d <= 8) {
        const SymShape sh = sym_shape(n, d);
        double *Xs = work;
        double *part = work + sh.npad * d;
        AFN_TRY(kmv_pack(X, n, d, l, kind, Xs, false, s));
        return kmv_sym_run<double, double>(Xs, sh, n, d, mu, kind, v, ldv, y, ldy, nrhs, part, s, ev0, ev1,
                                           nullptr, nullptr);
    }
    const int64_t S = kmv_splits(n);
    const int64_t split_len = ceil_div(n, S);
    const double c2 = kernel_scale(kind, l) * kernel_scale(kind, l);
    dim3 grid((unsigned)ceil_div(n, kRows), (unsigned)S);
    for (int c = 0; c < nrhs; ++c) {
        const double *vc = v + c * ldv;
        if (ev0) AFN_HIP(hipEventRecord(ev0, s));
        if (d <= 12) launch_partial<12, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
        else if (d <= 16) launch_partial<16, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
        else if (d <= 20) launch_partial<20, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
        else if (d <= 24) launch_partial<24, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
        else if (d <= 32) launch_partial<32, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
        else if (d <= 48) launch_partial<48, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
        else launch_partial<64, 32>(kind, grid, X, n, d, c2, vc, work, split_len, s);
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

afn_status kmv_f32(const double *X, int64_t n, int d, double l, double mu, int kind, const double *v,
                   int64_t ldv, double *y, int64_t ldy, int nrhs, void *work, hipStream_t s)
{
    if (d >= 1 && d <= 8) {
        const SymShape sh = sym_shape(n, d);
        float *Xs = (float *)work;
        float *part = Xs + round_up(sh.npad * d, 64);
        AFN_TRY(kmv_pack(X, n, d, l, kind, Xs, true, s));
        return kmv_sym_run<float, double>(Xs, sh, n, d, mu, kind, v, ldv, y, ldy, nrhs, part, s, nullptr,
                                          nullptr, nullptr, nullptr);
    }
    const int64_t S = kmv_splits(n);
    const int64_t split_len = ceil_div(n, S);
    const float c2 = (float)(kernel_scale(kind, l) * kernel_scale(kind, l));
    double *part = (double *)work;
    dim3 grid((unsigned)ceil_div(n, kRows), (unsigned)S);
    for (int c = 0; c < nrhs; ++c) {
        const double *vc = v + c * ldv;
        if (d <= 12) launch_partial32<12, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        else if (d <= 16) launch_partial32<16, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        else if (d <= 20) launch_partial32<20, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        else if (d <= 24) launch_partial32<24, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        else if (d <= 32) launch_partial32<32, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        else if (d <= 48) launch_partial32<48, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        else launch_partial32<64, 32>(kind, grid, X, n, d, c2, vc, part, split_len, s);
        AFN_HIP(hipGetLastError());
        hipLaunchKernelGGL(kmv_reduce, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, n,
                           (int)S, mu, vc, y + c * ldy);
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

}  // namespace afn
