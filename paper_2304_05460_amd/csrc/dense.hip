// Dense factors of the landmark block (Algorithm 2):
//   L = chol(K11 + mu I)           blocked right-looking Cholesky, 64-wide panels
//   Linv = L^{-1}, V = L^{-1} K12   left-looking blocked triangular solve
// All matrices column-major FP64.  Kernel values kernel_d2 (kfun.h) of the
// squared distance by the fixed fma chain.
#include "afn_internal.h"
#include "kfun.h"
#include "mfma.h"

namespace afn {
namespace {

constexpr int NB = 64;

__device__ __forceinline__ double kval(const double *a, const double *b, int d, double l2, int kind)
{
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double del = a[t] - b[t];
        acc = __builtin_fma(del, del, acc);
    }
    return kernel_d2(acc, l2, kind);
}

__global__ __launch_bounds__(256) void k11_fill(const double *__restrict__ Xp, int k, int d,
                                                double l2, int kind, double mu, double *__restrict__ A,
                                                int64_t lda)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    int j = (int)(e / k), i = (int)(e - (int64_t)j * k);
    if (i < j) {     // only the lower triangle is factored; keep the upper zero
        A[i + (int64_t)j * lda] = 0.0;
        return;
    }
    double v = kval(Xp + (int64_t)i * d, Xp + (int64_t)j * d, d, l2, kind);
    A[i + (int64_t)j * lda] = v + (i == j ? mu : 0.0);
}

__global__ __launch_bounds__(256) void k12_fill(const double *__restrict__ Xp, int64_t n, int k,
                                                int d, double l2, int kind, double *__restrict__ K12)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nr = n - k;
    if (e >= (int64_t)k * nr) return;
    int64_t p = e / k;
    int t = (int)(e - p * k);
    K12[e] = kval(Xp + (int64_t)t * d, Xp + (k + p) * d, d, l2, kind);
}

// Columns of K12 for the FSAI patterns of rows r0 .. r0+B-1: column
// c = (q - r0) w + a holds K(x_t, x_{k + cols[q w + a]}) for t < k (the same
// values k12_fill computes), zero for padding entries (a >= min(q + 1, w)).
// Tiled: a workgroup takes 256 landmarks and 16 pattern columns, stages the
// 16 points in LDS and keeps each thread's landmark in registers (d <= D),
// so a landmark's coordinates are read once per 16 entries and the writes of
// a column are contiguous.  Same arithmetic as kval, entry for entry.
template <int D>
__global__ __launch_bounds__(256) void k12_pattern_fill_tiled(const double *__restrict__ Xp, int64_t nr, int k,
                                                              int d, double l2, int kind,
                                                              const int32_t *__restrict__ cols, int w, int64_t r0,
                                                              int64_t B, double *__restrict__ Kb)
{
    constexpr int CB = 16;
    __shared__ double pts[CB][D];
    __shared__ int ok[CB];
    const int64_t ncol = B * w;
    const int64_t c0 = (int64_t)blockIdx.y * CB;
    for (int e = threadIdx.x; e < CB * d; e += 256) {
        const int cc = e / d, t = e - cc * d;
        const int64_t c = c0 + cc;
        const int64_t q = r0 + c / w;
        const int a = (int)(c - (c / w) * w);
        const int64_t m = q + 1 < w ? q + 1 : w;
        const bool valid = c < ncol && q < nr && a < m;
        pts[cc][t] = valid ? Xp[(k + (int64_t)cols[q * w + a]) * d + t] : 0.0;
        if (t == 0) ok[cc] = valid;
    }
    __syncthreads();
    const int64_t lt = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (lt >= k) return;
    double xl[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xl[t] = t < d ? Xp[lt * d + t] : 0.0;
    for (int cc = 0; cc < CB; ++cc) {
        const int64_t c = c0 + cc;
        if (c >= ncol) break;
        double v = 0.0;
        if (ok[cc]) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < D; ++t) {
                if (t < d) {
                    const double del = xl[t] - pts[cc][t];
                    acc = __builtin_fma(del, del, acc);
                }
            }
            v = kernel_d2(acc, l2, kind);
        }
        Kb[c * k + lt] = v;
    }
}

__device__ __forceinline__ double readlane_f64(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Step j0 of the blocked Cholesky, diagonal block: one wavefront factors the
// jb x jb block (lane r holds row r, the identity past jb) left-looking in
// chunks of eight columns.  A chunk takes the contributions of the columns
// already in LDS (the lane's own entry and the chunk rows' entries, read as
// broadcasts), then factors its eight columns in registers with the pivots
// and the entries L[c][j] taken from their lanes.  Every entry receives the
// same fused multiply-adds in the same ascending column order as a
// right-looking register sweep, while the loops stay rolled: code that runs
// once per launch and is unrolled over the whole block spends its time on
// instruction fetch.  Writes L11 (zero above the diagonal).  A pivot that is
// not positive is recorded in *info (first failing column, 1-based) and
// replaced by 1.  A separate kernel (potrf_rows) then solves the rows below
// against the finished L11: a workgroup of one launch that read the diagonal
// block while another wrote it back would see a partly factored block.
constexpr int kChol = 8;   // columns per chunk

__global__ __launch_bounds__(64) void potrf_diag(double *A, int64_t lda, int j0, int jb, int *info)
{
    __shared__ double Lc[NB][NB];   // Lc[c][r]: A[r][c], then L[r][c] (zero above the diagonal)
    const int lane = threadIdx.x;
    // the whole block first, sixteen loads in flight at a time (a load per
    // chunk or per column would wait out the memory latency each time), from
    // clamped in-range addresses and masked afterwards, so that no branch
    // separates the loads
    const int lr = lane < jb ? lane : 0;
    for (int c0 = 0; c0 < NB; c0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = A[(j0 + lr) + (int64_t)(j0 + (c0 + u < jb ? c0 + u : 0)) * lda];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = c0 + u;
            Lc[c][lane] = lane < jb && c < jb ? (c <= lane ? v[u] : 0.0) : (lane == c ? 1.0 : 0.0);
        }
    }
    int badj = -1;
    for (int q = 0; q < NB; q += kChol) {
        double a[kChol];
#pragma unroll
        for (int t = 0; t < kChol; ++t) a[t] = Lc[q + t][lane];
        for (int c = 0; c < q; ++c) {
            const double lr = Lc[c][lane];
#pragma unroll
            for (int t = 0; t < kChol; ++t) a[t] = __builtin_fma(-lr, Lc[c][q + t], a[t]);
        }
#pragma unroll
        for (int t = 0; t < kChol; ++t) {
            const int j = q + t;
            const double djj = readlane_f64(a[t], j);
            const bool bad = !(djj > 0.0);
            if (bad && badj < 0) badj = j;
            const double rjj = sqrt(bad ? 1.0 : djj);
            const double lr = lane == j ? rjj : (lane > j ? a[t] / rjj : 0.0);
            a[t] = lr;
#pragma unroll
            for (int u = t + 1; u < kChol; ++u) a[u] = __builtin_fma(-lr, readlane_f64(lr, q + u), a[u]);
        }
#pragma unroll
        for (int t = 0; t < kChol; ++t) {
            Lc[q + t][lane] = a[t];
            if (lane < jb && q + t < jb) A[(j0 + lane) + (int64_t)(j0 + q + t) * lda] = a[t];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0 && badj >= 0) atomicCAS(info, 0, j0 + badj + 1);
}

// Step j0, the rows below: workgroup b solves rows j0 + jb + 64 b + lane of
// L21 = A21 L11^{-T} by forward substitution, after potrf_diag has written
// L11: left-looking in chunks of eight columns against the solved entries of
// the lane's row kept in LDS, the same operations in the same order as a
// right-looking sweep (and rolled for the reason given above).
__global__ __launch_bounds__(64) void potrf_rows(double *A, int64_t lda, int j0, int jb, int k)
{
    __shared__ double Ls[NB][NB];   // Ls[c][r] = L11[r][c]
    __shared__ double Xs[NB][NB];   // Xs[c][lane]: entry c of the lane's row, then its solution
    const int lane = threadIdx.x;
    const int64_t row = (int64_t)j0 + jb + (int64_t)blockIdx.x * 64 + lane;
    // L11 and the lane's row first, sixteen loads in flight at a time
    // (clamped in-range addresses, masked afterwards: no branch between loads)
    const int lr = lane < jb ? lane : 0;
    const int64_t rr = row < k ? row : (int64_t)j0;
    for (int c0 = 0; c0 < NB; c0 += 16) {
        double lv[16], xv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int64_t col = (int64_t)(j0 + (c0 + u < jb ? c0 + u : 0)) * lda;
            lv[u] = A[(j0 + lr) + col];
            xv[u] = A[rr + col];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = c0 + u;
            Ls[c][lane] = lane < jb && c < jb && c <= lane ? lv[u] : 0.0;
            Xs[c][lane] = row < k && c < jb ? xv[u] : 0.0;
        }
    }
    __syncthreads();
    if (row >= k) return;
    for (int q = 0; q < jb; q += kChol) {
        double x[kChol];
#pragma unroll
        for (int t = 0; t < kChol; ++t) x[t] = Xs[q + t][lane];
        for (int c = 0; c < q; ++c) {
            const double xc = Xs[c][lane];
#pragma unroll
            for (int t = 0; t < kChol; ++t) x[t] = __builtin_fma(-Ls[c][q + t], xc, x[t]);
        }
#pragma unroll
        for (int t = 0; t < kChol; ++t) {
            if (q + t < jb) {
                const double xt = x[t] / Ls[q + t][q + t];
                x[t] = xt;
#pragma unroll
                for (int u = t + 1; u < kChol; ++u) x[u] = __builtin_fma(-Ls[q + t][q + u], xt, x[u]);
            }
        }
#pragma unroll
        for (int t = 0; t < kChol; ++t) {
            Xs[q + t][lane] = x[t];
            if (q + t < jb) A[row + (int64_t)(j0 + q + t) * lda] = x[t];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Inverse of each 64 x 64 lower diagonal block of L; identity-padded past k.
// Dinv[b] column-major 64 x 64.  Thread c forms column c by forward
// substitution on e_c.
__global__ __launch_bounds__(64) void diag_inverse(const double *L, int k, double *Dinv)
{
    __shared__ double Ls[NB][NB + 1];  // Ls[col][row]
    __shared__ double Ys[NB][NB + 1];  // Ys[c][row]: column c of the inverse
    const int b = blockIdx.x, c = threadIdx.x;
    const int j0 = b * NB;
    const int jb = k - j0 < NB ? k - j0 : NB;
    for (int col = 0; col < NB; ++col)
        Ls[col][c] = (c < jb && col < jb) ? L[(j0 + c) + (int64_t)(j0 + col) * k]
                                          : (c == col ? 1.0 : 0.0);
    __syncthreads();
    for (int i = 0; i < NB; ++i) {
        double s = (i == c) ? 1.0 : 0.0;
        if (i > c)
            for (int t = c; t < i; ++t) s -= Ls[t][i] * Ys[c][t];
        Ys[c][i] = i < c ? 0.0 : s / Ls[i][i];
    }
    double *out = Dinv + (int64_t)b * NB * NB + (int64_t)c * NB;
    for (int i = 0; i < NB; ++i) out[i] = Ys[c][i];
}

// The same solve with the 64 x 64 x 64 products on FP64 MFMA 16x16x4: wave
// w of the workgroup owns rows 16 w .. 16 w + 15 of the row block and all 64
// columns of the strip (four 16 x 16 accumulators), for the updates
// B_I -= L_IT X_T (T < I) and for X_I = Dinv_I B_I alike.  Tiles are staged
// k-index major in LDS with a row stride of TSM doubles, so each 16-lane
// group of an operand read touches consecutive doubles.
constexpr int TSM = NB + 4;

__device__ __forceinline__ void mfma_tile64(const double *__restrict__ As, const double *__restrict__ Bs, int wave,
                                            int lr, int lk, double sign, doublex4 (&acc)[4])
{
#pragma unroll 2
    for (int kk = 0; kk < NB / 4; ++kk) {
        const double a = sign * As[(4 * kk + lk) * TSM + 16 * wave + lr];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const double b = Bs[(4 * kk + lk) * TSM + 16 * cb + lr];
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
        }
    }
}

// Trailing update A22 -= L21 L21^T of the blocked Cholesky on lower 64 x 64
// tiles with FP64 MFMA: tile (I, C) takes the jb-column panel rows of both
// row blocks as k-index-major operands (zero past k and past jb) and one
// 64 x 64 x 64 product, as the triangular solve does.
__global__ __launch_bounds__(256) void syrk_update_mf(double *A, int64_t lda, int j0, int jb, int k)
{
    const int I = blockIdx.y, C = blockIdx.x;
    if (C > I) return;
    __shared__ double As[NB * TSM];    // As[t * TSM + r] = L21[r0 + r, t]
    __shared__ double Bs[NB * TSM];    // Bs[t * TSM + c] = L21[c0 + c, t]
    const int base = j0 + jb;
    const int r0 = base + I * NB, c0 = base + C * NB;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    for (int e = tid; e < NB * NB; e += 256) {
        const int t = e >> 6, r = e & 63;
        As[t * TSM + r] = (t < jb && r0 + r < k) ? A[(r0 + r) + (int64_t)(j0 + t) * lda] : 0.0;
        Bs[t * TSM + r] = (t < jb && c0 + r < k) ? A[(c0 + r) + (int64_t)(j0 + t) * lda] : 0.0;
    }
    __syncthreads();
    doublex4 acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = doublex4{0.0, 0.0, 0.0, 0.0};
    mfma_tile64(As, Bs, wave, lr, lk, 1.0, acc);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + 16 * wave + lk + 4 * i, c = c0 + 16 * cb + lr;
            if (r < k && c < k && r >= c) A[r + (int64_t)c * lda] -= acc[cb][i];
        }
}

// 64 x NC product on FP64 MFMA: wave w takes rows 16 w .. 16 w + 15, both
// operands k-index major in LDS (A with row stride TSM, B with NC + 4).
template <int NC>
__device__ __forceinline__ void mfma_tile_nc(const double *__restrict__ As, const double *__restrict__ Bs, int wave,
                                             int lr, int lk, double sign, doublex4 (&acc)[NC / 16])
{
    constexpr int TSB = NC + 4;
#pragma unroll 2
    for (int kk = 0; kk < NB / 4; ++kk) {
        const double a = sign * As[(4 * kk + lk) * TSM + 16 * wave + lr];
#pragma unroll
        for (int cb = 0; cb < NC / 16; ++cb) {
            const double b = Bs[(4 * kk + lk) * TSB + 16 * cb + lr];
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[cb], 0, 0, 0);
        }
    }
}

// B (k x ncols, ld k) := L^{-1} B, left-looking by 64-row blocks; one
// workgroup per NC-column strip (so every strip is solved by one workgroup in
// order and no cross-workgroup synchronization is needed): B_I -= L_IT X_T
// for T < I, then X_I = Dinv_I B_I, as 64 x 64 x NC products on FP64 MFMA.
// unit: B is the identity, so the strip's rows above its first column are
// zero in X and stay as they are (the solve starts at that row block).
template <int NC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void trsm_left_lower_mf(
    const double *__restrict__ L, const double *__restrict__ Dinv, int k, double *B, int64_t ncols, int unit)
{
    constexpr int CB = NC / 16, TSB = NC + 4, XQ = NC / 4;
    __shared__ double As[NB * TSM];    // As[t * TSM + r]: A[r][t]
    __shared__ double Bs[NB * TSB];    // Bs[t * TSB + c]: B[t][c]
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lk = lane >> 4;
    const int64_t c0 = (int64_t)blockIdx.x * NC;
    const int nblk = (int)ceil_div(k, NB);
    const int first = unit ? (int)(c0 / NB) : 0;
    for (int I = first; I < nblk; ++I) {
        const int r0 = I * NB;
        doublex4 acc[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 16 * wave + lk + 4 * i;
                const int64_t c = c0 + 16 * cb + lr;
                acc[cb][i] = (r < k && c < ncols) ? B[r + c * k] : 0.0;
            }
        // the tiles of step T + 1 are read into registers while the MFMAs
        // of step T run (16 doubles of L and NC / 4 of X per thread)
        double la[16], xa[XQ];
        // thread (r, t0) = (tid & 63, tid >> 6) takes L[r0 + r, T NB + t0 + 4 q] (q < 16)
        // and B[T NB + r, c0 + t0 + 4 q] (q < NC / 4): one base address, stride 4 k
        const int rr = tid & 63, t0 = tid >> 6;
        const bool rok = r0 + rr < k;
        const int64_t st4 = 4 * (int64_t)k;
        auto fetch = [&](int T) {
            const double *lp = L + (r0 + rr) + (int64_t)(T * NB + t0) * k;
            const double *xp = B + (T * NB + rr) + (c0 + t0) * k;
#pragma unroll
            for (int q = 0; q < 16; ++q) la[q] = rok ? lp[q * st4] : 0.0;
#pragma unroll
            for (int q = 0; q < XQ; ++q) xa[q] = c0 + t0 + 4 * q < ncols ? xp[q * st4] : 0.0;
        };
        if (I > first) fetch(first);
        for (int T = first; T < I; ++T) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 16; ++q) As[(t0 + 4 * q) * TSM + rr] = la[q];
#pragma unroll
            for (int q = 0; q < XQ; ++q) Bs[rr * TSB + t0 + 4 * q] = xa[q];
            __syncthreads();
            if (T + 1 < I) fetch(T + 1);
            mfma_tile_nc<NC>(As, Bs, wave, lr, lk, -1.0, acc);
        }
        // X_I = Dinv_I acc
        __syncthreads();
        for (int e = tid; e < NB * NB; e += 256) {
            const int t = e >> 6, r = e & 63;
            As[t * TSM + r] = Dinv[(int64_t)I * NB * NB + r + (int64_t)t * NB];
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) Bs[(16 * wave + lk + 4 * i) * TSB + 16 * cb + lr] = acc[cb][i];
        __syncthreads();
        doublex4 out[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) out[cb] = doublex4{0.0, 0.0, 0.0, 0.0};
        mfma_tile_nc<NC>(As, Bs, wave, lr, lk, 1.0, out);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = r0 + 16 * wave + lk + 4 * i;
                const int64_t c = c0 + 16 * cb + lr;
                if (r < k && c < ncols) B[r + c * k] = out[cb][i];
            }
        // each wave stored 16 rows of X_I, and the next row block's first
        // fetch reads X tiles back across waves (X_I itself when I is the
        // strip's first block): every store lands before any wave goes on
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void set_identity(double *A, int k)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    int j = (int)(e / k), i = (int)(e - (int64_t)j * k);
    A[e] = i == j ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void add_diag_kernel(double *A, int k, int64_t lda, double shift)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) A[i + (int64_t)i * lda] += shift;
}

__global__ __launch_bounds__(256) void transpose_kernel(const double *A, int k, int64_t lda, double *B,
                                                        int64_t ldb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    const int i = (int)(e / k), t = (int)(e - (int64_t)i * k);
    B[t + (int64_t)i * ldb] = A[i + (int64_t)t * lda];
}

__global__ __launch_bounds__(256) void zero_upper_kernel(double *A, int k, int64_t lda)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)k * k) return;
    const int j = (int)(e / k), i = (int)(e - (int64_t)j * k);
    if (i < j) A[i + (int64_t)j * lda] = 0.0;
}

}  // namespace

afn_status zero_upper(double *A, int k, int64_t lda, hipStream_t s)
{
    if (k <= 0) return AFN_OK;
    hipLaunchKernelGGL(zero_upper_kernel, dim3((unsigned)ceil_div((int64_t)k * k, 256)), dim3(256), 0, s, A, k,
                       lda);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status add_diagonal(double *A, int k, int64_t lda, double shift, hipStream_t s)
{
    if (k <= 0) return AFN_OK;
    hipLaunchKernelGGL(add_diag_kernel, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, s, A, k, lda, shift);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status transpose_square(const double *A, int k, int64_t lda, double *B, int64_t ldb, hipStream_t s)
{
    if (k <= 0) return AFN_OK;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)ceil_div((int64_t)k * k, 256)), dim3(256), 0, s, A, k,
                       lda, B, ldb);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status fill_k11(const double *Xp, int k, int d, double l, int kind, double mu, double *A, int64_t lda,
                    hipStream_t s)
{
    if (k <= 0) return AFN_OK;
    hipLaunchKernelGGL(k11_fill, dim3((unsigned)ceil_div((int64_t)k * k, 256)), dim3(256), 0, s, Xp,
                       k, d, l * l, kind, mu, A, lda);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status fill_k12(const double *Xp, int64_t n, int k, int d, double l, int kind, double *K12,
                    hipStream_t s)
{
    int64_t total = (int64_t)k * (n - k);
    if (total <= 0) return AFN_OK;
    hipLaunchKernelGGL(k12_fill, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, Xp, n, k, d,
                       l * l, kind, K12);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status fill_k12_patterns(const double *Xp, int64_t n, int k, int d, double l, int kind, const int32_t *cols,
                             int w, int64_t r0, int64_t B, double *Kb, hipStream_t s)
{
    const int64_t total = (int64_t)k * B * w;
    if (total <= 0) return AFN_OK;
    const dim3 g((unsigned)ceil_div(k, 256), (unsigned)ceil_div(B * w, 16));
    const double l2 = l * l;
    const int64_t nr = n - k;
    if (d <= 8) hipLaunchKernelGGL(k12_pattern_fill_tiled<8>, g, dim3(256), 0, s, Xp, nr, k, d, l2, kind, cols, w, r0, B, Kb);
    else if (d <= 16) hipLaunchKernelGGL(k12_pattern_fill_tiled<16>, g, dim3(256), 0, s, Xp, nr, k, d, l2, kind, cols, w, r0, B, Kb);
    else if (d <= 24) hipLaunchKernelGGL(k12_pattern_fill_tiled<24>, g, dim3(256), 0, s, Xp, nr, k, d, l2, kind, cols, w, r0, B, Kb);
    else if (d <= 32) hipLaunchKernelGGL(k12_pattern_fill_tiled<32>, g, dim3(256), 0, s, Xp, nr, k, d, l2, kind, cols, w, r0, B, Kb);
    else if (d <= 48) hipLaunchKernelGGL(k12_pattern_fill_tiled<48>, g, dim3(256), 0, s, Xp, nr, k, d, l2, kind, cols, w, r0, B, Kb);
    else hipLaunchKernelGGL(k12_pattern_fill_tiled<64>, g, dim3(256), 0, s, Xp, nr, k, d, l2, kind, cols, w, r0, B, Kb);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status cholesky(double *A, int k, int64_t lda, int *info, hipStream_t s)
{
    for (int j0 = 0; j0 < k; j0 += NB) {
        const int jb = k - j0 < NB ? k - j0 : NB;
        const int rest = k - j0 - jb;
        hipLaunchKernelGGL(potrf_diag, dim3(1), dim3(64), 0, s, A, lda, j0, jb, info);
        if (rest > 0) {
            hipLaunchKernelGGL(potrf_rows, dim3((unsigned)ceil_div(rest, 64)), dim3(64), 0, s, A, lda, j0, jb, k);
            const unsigned T = (unsigned)ceil_div(rest, NB);
            hipLaunchKernelGGL(syrk_update_mf, dim3(T, T), dim3(256), 0, s, A, lda, j0, jb, k);
        }
        AFN_HIP(hipGetLastError());
    }
    return AFN_OK;
}

int64_t dinv_doubles(int k) { return ceil_div(k, NB) * NB * NB; }

afn_status diag_inverses(const double *L, int k, double *Dinv, hipStream_t s)
{
    if (k <= 0) return AFN_OK;
    hipLaunchKernelGGL(diag_inverse, dim3((unsigned)ceil_div(k, NB)), dim3(64), 0, s, L, k, Dinv);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status trsm_lower(const double *L, const double *Dinv, int k, double *B, int64_t ncols,
                      hipStream_t s, bool unit)
{
    if (k <= 0 || ncols <= 0) return AFN_OK;
    // strips of 16 columns while 64-column strips would not fill the CUs
    // (128-column strips, half the passes over L for very wide B, measured
    // slower: one workgroup per CU)
    if (ncols < 64 * 256)
        hipLaunchKernelGGL(trsm_left_lower_mf<16>, dim3((unsigned)ceil_div(ncols, 16)), dim3(256), 0, s, L,
                           Dinv, k, B, ncols, unit ? 1 : 0);
    else
        hipLaunchKernelGGL(trsm_left_lower_mf<64>, dim3((unsigned)ceil_div(ncols, 64)), dim3(256), 0, s, L,
                           Dinv, k, B, ncols, unit ? 1 : 0);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

afn_status identity(double *A, int k, hipStream_t s)
{
    if (k <= 0) return AFN_OK;
    hipLaunchKernelGGL(set_identity, dim3((unsigned)ceil_div((int64_t)k * k, 256)), dim3(256), 0, s,
                       A, k);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

}  // namespace afn
