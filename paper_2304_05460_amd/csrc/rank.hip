// Nystrom rank estimation (Algorithm 4, Section 3.3) on the GPU.
//
// 1. Subsample m of the n points: the first m entries of a Fisher-Yates
//    shuffle of 0..n-1 driven by splitmix64(seed) (Steele, Lea & Flood 2014),
//    position i swapping with i + (draw mod (n - i)).  One thread keeps the
//    touched positions in an LDS hash table.
// 2. Scale the subsample by (m/n)^{1/d}; form K_m; order it by FPS.
// 3. Nested Nystrom errors ||K_m - K_m[:,I] K_m[I,I]^+ K_m[I,:]||_F / ||K_m||_F
//    for I = the first r FPS points: successive rank-one eliminations of K_m
//    in FPS order (the residual is the Schur complement); a pivot <= 1e-14 m
//    adds nothing (pseudoinverse) and its row and column are set to zero.
//    The smallest r in {8, 16, ...} (or m) with error < 0.1 is the rank r.
// 4. k_est = floor(r n / m); below the switch (2000) the count of eigenvalues
//    of K_m on the unscaled subsample above 0.1 mu replaces it (Householder
//    tridiagonalization, then the Sturm / LDL^T inertia count).
#include <cmath>
#include <vector>

#include "afn_internal.h"
#include "kfun.h"

namespace afn {

namespace {

constexpr int kMaxM = 4096;

__device__ __forceinline__ uint64_t splitmix64_next(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Partial Fisher-Yates over the virtual array a[j] = j: step i swaps
// positions i and p_i = i + draw_i mod (n - i) and takes sub[i] = the value
// found at p_i.  Draw i is the (i+1)-th splitmix64 output, a function of
// seed + (i+1) gamma alone, so every draw is formed in parallel, and so are
// the swaps: the only writes read later are those of a step's own value a_t
// (the value at position t just before step t) into position p_t.  Hence
// sub[i] = a_s for the last step s < i with p_s = p_i (else p_i itself), and
// a_t = a_w for the last step w < t with p_w = t (else t), a chain that
// pointer jumping resolves.  The previous step with the same partner, and the
// last writer of each position, come from the steps sorted by (p_t, t).  The
// result is the serial sequence of swaps, element for element.
constexpr int kSubThreads = 1024;

__global__ __launch_bounds__(kSubThreads) void subsample_kernel(int64_t n, int m, uint64_t seed, int32_t *sub)
{
    __shared__ unsigned long long srt[kMaxM];   // p_t << 32 | t, sorted; then jump buffer
    __shared__ int prv[kMaxM];                  // previous step with the same partner, or -1
    __shared__ int aux[kMaxM];                  // last sorted position of partner t; then chains
    constexpr int PER = kMaxM / kSubThreads;
    const int tid = threadIdx.x;
    int N = 1;
    while (N < m) N <<= 1;
    auto partner_of = [&](int i) -> int64_t {
        uint64_t st = seed + (uint64_t)i * 0x9E3779B97F4A7C15ULL;
        const uint64_t draw = splitmix64_next(st);
        return i + (int64_t)(draw % (uint64_t)(n - i));
    };
    for (int i = tid; i < N; i += kSubThreads) {
        srt[i] = i < m ? ((unsigned long long)partner_of(i) << 32) | (unsigned)i : ~0ull;
        if (i < m) {
            prv[i] = -1;
            aux[i] = -1;
        }
    }
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < N; i += kSubThreads) {
                const int ij = i ^ j;
                if (ij > i) {
                    const unsigned long long x = srt[i], y = srt[ij];
                    if ((x > y) == ((i & k) == 0)) {
                        srt[i] = y;
                        srt[ij] = x;
                    }
                }
            }
            __syncthreads();
        }
    auto key = [&](int q) { return (int)(srt[q] >> 32); };
    auto step = [&](int q) { return (int)(srt[q] & 0xffffffffu); };
    for (int q = tid; q < m; q += kSubThreads) {
        const int kq = key(q);
        if (q > 0 && key(q - 1) == kq) prv[step(q)] = step(q - 1);
        if ((q + 1 == m || key(q + 1) != kq) && kq < m) aux[kq] = q;
    }
    __syncthreads();
    // w_t: the last step before t whose partner is t (those steps are <= t)
    int w[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = tid + kSubThreads * u;
        w[u] = t;
        if (t < m) {
            int q = aux[t];
            if (q >= 0 && step(q) == t) q = q > 0 && key(q - 1) == t ? q - 1 : -1;
            if (q >= 0) w[u] = step(q);
        }
    }
    __syncthreads();    // aux read everywhere before it holds the chains
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int t = tid + kSubThreads * u;
        if (t < m) aux[t] = w[u];
    }
    __syncthreads();
    // after r rounds each entry points 2^r links down its chain (or to its
    // end, a step nothing wrote before, whose value is its own index)
    int *cur = aux, *nxt = (int *)srt;
    for (int r = 0; (1 << r) < m; ++r) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int t = tid + kSubThreads * u;
            if (t < m) nxt[t] = cur[cur[t]];
        }
        __syncthreads();
        int *tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = tid + kSubThreads * u;
        if (i < m) sub[i] = prv[i] >= 0 ? cur[prv[i]] : (int32_t)partner_of(i);
    }
}

__global__ __launch_bounds__(256) void gather_scaled(const double *X, const int32_t *sub, int m, int d,
                                                     double scale, double *Xm)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * d) return;
    int i = e / d, t = e - i * d;
    Xm[e] = X[(int64_t)sub[i] * d + t] * scale;
}

__global__ __launch_bounds__(256) void kmat_fill(const double *Xm, int m, int d, double l2, int kind, double *K)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double del = Xm[i * d + t] - Xm[j * d + t];
        acc = __builtin_fma(del, del, acc);
    }
    K[e] = kernel_d2(acc, l2, kind);
}

// Block partial of sum of squares of K (m x m).
__global__ __launch_bounds__(256) void sumsq_partial(const double *K, int64_t total, double *part)
{
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        s += K[e] * K[e];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ws[0] + ws[1] + ws[2] + ws[3];
}

__global__ __launch_bounds__(256) void sum_parts(const double *part, int np, double *out)
{
    __shared__ double ws[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    ws[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) ws[threadIdx.x] += ws[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = ws[0];
}

// Blocked form of the elimination scan.  A step r with pivot point pj takes
// the column c = S[:, pj] of the current residual S and its pivot p = S[pj, pj];
// it either updates S[x, y] = S[x, y] - c[x] (c[y] / p) everywhere, or, with
// p <= pivtol, sets row and column pj of S to zero.  32 successive steps are
// applied by one pass over S (two passes per FPS chunk of 64): scan_panel
// forms, row by row, the columns c_i and the scaled columns q_i = c_i / p_i
// of the steps from their pivot columns of S (the same arithmetic, in the
// same order, as the steps one at a time), and scan_update applies the terms
// to every entry in step order, so S after the pass is bitwise S after the
// single steps.  A skipped step's zero row and column are applied lazily: a
// zeroed row contributes c = 0 to every later step (as the zero row would), a
// zeroed column (a repeated pivot) gives c = 0 at the step that takes it.
// The update also sums the squares of S after every eighth step (and after
// the last), the Nystrom errors, in per-workgroup partials.  This file is
// compiled without contraction: each term is a product, then a difference.
constexpr int kScanB = 32;     // steps per pass
constexpr int kScanE = 4;      // errors per pass, one every 8 steps

// Out: C[i m + x] = c_i(x), Q[i m + x] = c_i(x) / p_i, skip[i] (workgroup 0).
// Every workgroup first runs the nb x nb block of the pivot rows (wave 0, one
// lane per row) to obtain the pivots, the skip flags and q_i(piv_j), then its
// 256 rows.  A row goes left-looking in chunks of eight columns: a chunk's
// entries (registers) first take the terms c_i q_i(piv_j) of the earlier
// chunks' steps (c_i from the thread's history in LDS, q_i and the skip
// flags as broadcasts), then its eight steps run as before, each updating
// the chunk's later entries.  Every entry thus receives the same products
// and differences in the same step order as in a right-looking sweep over
// all 32 columns, while the code stays rolled (unrolled over all 32 steps it
// waited on instruction fetch: it runs once per launch).  The next chunk's
// entries are loaded while a chunk is processed.
constexpr int kScanC = 8;      // columns per chunk

__global__ __launch_bounds__(256) void scan_panel(const double *__restrict__ K, int m,
                                                  const int32_t *__restrict__ ord, int r0, int nb,
                                                  double pivtol, double *__restrict__ C,
                                                  double *__restrict__ Q, int *__restrict__ skip)
{
    __shared__ int piv[kScanB];
    __shared__ double qb[kScanB][kScanB];     // qb[i][j] = q_i(piv_j)
    __shared__ double pvt[kScanB];
    __shared__ int skp[kScanB], zc[kScanB];   // zc[j]: column piv_j zeroed before step j
    __shared__ double hist[kScanB - kScanC][256];   // hist[i][tid]: the thread's c_i
    const int tid = threadIdx.x;
    if (tid < kScanB) {
        piv[tid] = tid < nb ? ord[r0 + tid] : -1;
        zc[tid] = 0;
    }
    __syncthreads();
    // row x (the rowzero test; -1 for none) with its entries read from row xl
    // (in range) when real; at_step(i, c_i(x)) returns whether step i is skipped
    auto run_row = [&](int x, int xl, bool real, auto at_step) {
        auto load = [&](int q, double (&R)[kScanC]) {
#pragma unroll
            for (int t = 0; t < kScanC; ++t) {
                const int col = q + t < nb ? piv[q + t] : piv[0];
                R[t] = K[xl + (int64_t)col * m];
            }
        };
        double Pn[kScanC];
        load(0, Pn);
        bool rowzero = false;
        for (int q = 0; q < nb; q += kScanC) {
            double P[kScanC];
#pragma unroll
            for (int t = 0; t < kScanC; ++t) P[t] = real && q + t < nb ? Pn[t] : 0.0;
            if (q + kScanC < nb) load(q + kScanC, Pn);
            for (int i = 0; i < q; ++i) {
                if (skp[i]) continue;
                const double ci = hist[i][tid];
#pragma unroll
                for (int t = 0; t < kScanC; ++t) P[t] = P[t] - ci * qb[i][q + t];
            }
#pragma unroll
            for (int t = 0; t < kScanC; ++t) {
                const int i = q + t;
                if (i < nb) {
                    const double ci = rowzero || zc[i] ? 0.0 : P[t];
                    if (at_step(i, ci)) {
                        if (x == piv[i]) rowzero = true;
                    } else {
#pragma unroll
                        for (int u = t + 1; u < kScanC; ++u) P[u] = P[u] - ci * qb[i][q + u];
                    }
                    if (i < kScanB - kScanC) hist[i][tid] = ci;
                }
            }
        }
    };
    if (tid < 64) {
        // the pivot rows: lane a holds row piv_a; step i takes its pivot from
        // lane i, and q_i(piv_j) from lane j through qb (one wave: its LDS
        // accesses complete in program order)
        const int a = tid;
        auto at_step = [&](int i, double cai) {
            const double p = __shfl(cai, i, 64);
            const bool sk = !(p > pivtol);
            if (a == 0) {
                pvt[i] = p;
                skp[i] = sk ? 1 : 0;
            }
            if (a < nb) qb[i][a] = cai / p;
            if (sk && a > i && a < nb && piv[a] == piv[i]) zc[a] = 1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            return sk;
        };
        run_row(a < nb ? piv[a] : -1, a < nb ? piv[a] : piv[0], a < nb, at_step);
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < nb) skip[tid] = skp[tid];
    const int x = blockIdx.x * 256 + tid;
    if (x >= m) return;
    auto at_step = [&](int i, double ci) {
        C[(int64_t)i * m + x] = ci;
        Q[(int64_t)i * m + x] = ci / pvt[i];
        return skp[i] != 0;
    };
    run_row(x, x, true, at_step);
}

// S[x, y] after the nb steps on a 64 x 64 tile (each thread: rows
// x0 + lr + 16 a, columns y0 + 4 lc + b, a, b < 4); part[e * nblk + block] =
// the sum of the squares of the tile after step min(8 e + 7, nb - 1).
constexpr int kUT = 64;

__global__ __launch_bounds__(256) void scan_update(double *__restrict__ K, int m,
                                                   const int32_t *__restrict__ ord, int r0, int nb,
                                                   const double *__restrict__ C,
                                                   const double *__restrict__ Q,
                                                   const int *__restrict__ skip, double *__restrict__ part)
{
    __shared__ double cs[kScanB][kUT], qs[kScanB][kUT];
    __shared__ int piv[kScanB];
    __shared__ unsigned long long skm_s;
    __shared__ double ws[4];
    const int tid = threadIdx.x, lr = tid & 15, lc = tid >> 4;
    const int x0 = blockIdx.x * kUT, y0 = blockIdx.y * kUT;
    double v[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int x = x0 + lr + 16 * a, y = y0 + 4 * lc + b;
            v[a][b] = x < m && y < m ? K[x + (int64_t)y * m] : 0.0;
        }
    for (int e = tid; e < kScanB * kUT; e += 256) {
        const int i = e / kUT, r = e % kUT;
        cs[i][r] = i < nb && x0 + r < m ? C[(int64_t)i * m + x0 + r] : 0.0;
        qs[i][r] = i < nb && y0 + r < m ? Q[(int64_t)i * m + y0 + r] : 0.0;
    }
    if (tid < 64) {
        if (tid < kScanB) piv[tid] = tid < nb ? ord[r0 + tid] : -1;
        const unsigned long long bm = __ballot(tid < nb && skip[tid] != 0);
        if (tid == 0) skm_s = bm;
    }
    __syncthreads();
    const unsigned long long skm = skm_s;
    const int nblk = (int)(gridDim.x * gridDim.y), blk = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    for (int e = 0; 8 * e < nb; ++e) {
        const int iend = 8 * e + 8 < nb ? 8 * e + 8 : nb;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int i = 8 * e + k;
            if (i >= iend) break;
            double c[4], q[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) c[a] = cs[i][lr + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) q[b] = qs[i][4 * lc + b];
            if (!((skm >> i) & 1ull)) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) v[a][b] = v[a][b] - c[a] * q[b];
            } else {
                const int p = piv[i];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (x0 + lr + 16 * a == p || y0 + 4 * lc + b == p) v[a][b] = 0.0;
            }
        }
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) t = __builtin_fma(v[a][b], v[a][b], t);
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
        if ((tid & 63) == 0) ws[tid >> 6] = t;
        __syncthreads();
        if (tid == 0) part[(int64_t)e * nblk + blk] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
        __syncthreads();      // ws read before the next group writes it
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int x = x0 + lr + 16 * a, y = y0 + 4 * lc + b;
            if (x < m && y < m) K[x + (int64_t)y * m] = v[a][b];
        }
}

// errs[r0 + min(8 e + 7, nb - 1)] = sum of part[e * np ...] (one workgroup per e)
__global__ __launch_bounds__(256) void scan_errors(const double *__restrict__ part, int np, int r0, int nb,
                                                   double *__restrict__ errs)
{
    __shared__ double ws[256];
    const int e = blockIdx.x;
    if (8 * e >= nb) return;
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[(int64_t)e * np + i];
    ws[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) ws[threadIdx.x] += ws[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) errs[r0 + (8 * e + 7 < nb - 1 ? 8 * e + 7 : nb - 1)] = ws[0];
}

// ---------------------------------------------------------------- eigen count
// Householder tridiagonalization of the symmetric A (m x m, column-major),
// one launch per step j = 0 .. m-3 after the first product.  The reflector of step j is
// H = I - beta v v^T with v supported on rows j+1 .. m-1, kept in one of two
// buffers (step parity) with beta in sc[0]; the step replaces the trailing
// block B = A[j+1:, j+1:] by H B H = B - v w^T - w v^T with p = beta B v,
// K = beta/2 v^T p and w = p - K v.  Each column of B is handled by two
// wavefronts (alternate blocks of 64 rows): reads along the column are
// coalesced, and every sum runs in a fixed order (lane partials in row order,
// then a butterfly, then the two halves), so the result does not depend on
// scheduling.  The steps are short and dependent, so a launch issues all its
// loads that do not wait for the step's reductions at once.  Rows and columns <= j+1 are never read
// after step j, so the update writes only A[j+2:, j+2:].  The launch of
// step j also does the product of step j+1: every workgroup forms the
// updated column j+1 and from it the reflector of step j+1 (the same
// arithmetic in each), then updates its columns and takes their products
// with the new reflector while the values are in registers.
// diag[c] / off[c] collect the tridiagonal T (the sub-diagonal up to sign).

__device__ __forceinline__ double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

constexpr int kUnroll = 8;     // rows per lane with loads in flight together

// Reflector of the column whose entries at rows r0 .. m-1 are colval(i):
// v[r0] = x0 - snew, v[i] = colval(i) beyond, snew = -sign(x0) alpha with
// alpha = ||col||, and v^T v = 2 alpha (alpha + |x0|) (both terms >= 0).
template <class F>
__device__ void house_wave(F colval, int r0, int m, double *v, double *sc, double *offp)
{
    const int lane = threadIdx.x & 63;
    double a2 = 0.0, x0 = 0.0;
    for (int base = r0 + lane; base < m; base += 64 * kUnroll) {
        double a[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int i = base + 64 * u;
            a[u] = i < m ? colval(i) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int i = base + 64 * u;
            if (i < m) v[i] = a[u];
            a2 = __builtin_fma(a[u], a[u], a2);
        }
        if (base == r0) x0 = a[0];
    }
    a2 = wave_sum(a2);
    x0 = __shfl(x0, 0, 64);
    const double alpha = sqrt(a2);
    const double snew = x0 >= 0.0 ? -alpha : alpha;
    if (lane == 0) {
        const double vn2 = 2.0 * alpha * (alpha + fabs(x0));
        v[r0] = x0 - snew;
        sc[0] = alpha == 0.0 || !(vn2 > 0.0) ? 0.0 : 2.0 / vn2;
        *offp = snew;
    }
}

// One wavefront: diag[0], and the reflector of step 0 (m >= 3) or T (m <= 2).
__global__ __launch_bounds__(64) void hh_init(const double *A, int m, double *v, double *sc, double *diag,
                                              double *off)
{
    const int lane = threadIdx.x;
    if (lane == 0) diag[0] = A[0];
    if (m == 2 && lane == 0) {
        diag[1] = A[1 + m];
        off[0] = A[1];
    }
    if (m < 3) return;
    house_wave([&](int i) { return A[i]; }, 1, m, v, sc, off);
}

// p[c] = beta * sum_{i > j} A[i,c] v[i] for c > j; part[b] = sum over the
// block's (<= 4) columns of v[c] p[c].
__global__ __launch_bounds__(256) void hh_mv(const double *__restrict__ A, int m, int j,
                                             const double *__restrict__ v, const double *__restrict__ sc,
                                             double *__restrict__ p, double *__restrict__ part)
{
    __shared__ double ws[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = j + 1 + (int)blockIdx.x * 4 + wv;
    double dotc = 0.0;
    if (c < m) {
        const double *col = A + (int64_t)c * m;
        double s = 0.0;
        for (int base = j + 1 + lane; base < m; base += 64 * kUnroll) {
            double a[kUnroll], b[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = base + 64 * u;
                a[u] = i < m ? col[i] : 0.0;
                b[u] = i < m ? v[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) s = __builtin_fma(a[u], b[u], s);
        }
        s = wave_sum(s);
        const double pc = sc[0] * s;
        if (lane == 0) p[c] = pc;
        dotc = v[c] * pc;
    }
    if (lane == 0) ws[wv] = dotc;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

// Step j's rank-two update fused with step j+1's product.  In: v, sc (beta),
// p and the nb partials of v^T p of step j.  Out: the reflector of step j+1
// (vn, scn, off[j+1]; written by workgroup 0), diag[j+1], the updated
// A[j+2:, j+2:], pn[c] = beta' sum_{i >= j+2} A'[i,c] v'[i] for c >= j+2 and
// per-workgroup partials partn of v'^T pn (four columns per workgroup, two
// wavefronts each).  Dynamic LDS: 3 (m - j - 2) doubles.
constexpr int kHhPart = 8;     // partials of v^T p per lane loaded up front (nb <= 512)
constexpr int kHhPre = 4;      // rows of v, p and column j+1 per thread up front (s <= 2048)
constexpr int kHhCol = 16;     // rows of the wavefront's column per lane up front (s <= 2048)

__global__ __launch_bounds__(512) void hh_step(double *__restrict__ A, int m, int j,
                                               const double *__restrict__ v, const double *__restrict__ sc,
                                               const double *__restrict__ p, const double *__restrict__ part,
                                               int nb, double *__restrict__ vn, double *__restrict__ scn,
                                               double *__restrict__ pn, double *__restrict__ partn,
                                               double *__restrict__ diag, double *__restrict__ off)
{
    // rows r0 .. m-1 (index i - r0): the new reflector, v, and w = p - K v of step j
    extern __shared__ double hh_lds[];
    __shared__ double red[8];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c1 = j + 1, r0 = j + 2, s = m - r0;
    double *vl = hh_lds, *vs = hh_lds + s, *ws = hh_lds + 2 * s;
    const double *col1 = A + (int64_t)c1 * m;
    // the workgroup's four columns, two wavefronts each (rows r0 + 64 h + 128 u + lane)
    const int c = r0 + (int)blockIdx.x * 4 + (wv & 3), h = wv >> 2;
    double *col = c < m ? A + (int64_t)c * m : A;
    // every load that does not wait for this step's reductions, issued together
    double q[kHhPart], pv[kHhPre], pp[kHhPre], pc[kHhPre], a[kHhCol];
#pragma unroll
    for (int u = 0; u < kHhPart; ++u) q[u] = lane + 64 * u < nb ? part[lane + 64 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < kHhPre; ++u) {
        const int i = r0 + tid + 512 * u;
        pv[u] = i < m ? v[i] : 0.0;
        pp[u] = i < m ? p[i] : 0.0;
        pc[u] = i < m ? col1[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kHhCol; ++u) {
        const int i = r0 + 64 * h + lane + 128 * u;
        a[u] = c < m && i < m ? col[i] : 0.0;
    }
    const double v1 = v[c1], p1 = p[c1], d1 = col1[c1];
    // K = beta/2 v^T p, every wavefront in the same order
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < kHhPart; ++u) sum += q[u];
    for (int b0 = lane + 64 * kHhPart; b0 < nb; b0 += 64) sum += part[b0];
    const double K = 0.5 * sc[0] * wave_sum(sum);
    // the updated column j+1 below the diagonal, and its squared norm
    const double w1 = p1 - K * v1;
    double a2 = 0.0;
    auto prefix_row = [&](int i, double vi, double pi, double ci) {
        const double wi = pi - K * vi;
        const double x = ci - (vi * w1 + wi * v1);
        vl[i - r0] = x;
        vs[i - r0] = vi;
        ws[i - r0] = wi;
        a2 = __builtin_fma(x, x, a2);
    };
#pragma unroll
    for (int u = 0; u < kHhPre; ++u) {
        const int i = r0 + tid + 512 * u;
        if (i < m) prefix_row(i, pv[u], pp[u], pc[u]);
    }
    for (int i = r0 + tid + 512 * kHhPre; i < m; i += 512) prefix_row(i, v[i], p[i], col1[i]);
    a2 = wave_sum(a2);
    if (lane == 0) red[wv] = a2;
    __syncthreads();
    const double x0 = vl[0];
    const double alpha = sqrt(((((((red[0] + red[1]) + red[2]) + red[3]) + red[4]) + red[5]) + red[6]) + red[7]);
    const double snew = x0 >= 0.0 ? -alpha : alpha;
    const double vn2 = 2.0 * alpha * (alpha + fabs(x0));
    const double beta1 = alpha == 0.0 || !(vn2 > 0.0) ? 0.0 : 2.0 / vn2;
    __syncthreads();    // x0 and red[] read everywhere before they are replaced
    if (tid == 0) vl[0] = x0 - snew;
    __syncthreads();
    if (blockIdx.x == 0) {
        for (int i = tid; i < s; i += 512) vn[r0 + i] = vl[i];
        if (tid == 0) {
            scn[0] = beta1;
            off[c1] = snew;
            diag[c1] = d1 - (v1 * w1 + w1 * v1);
        }
    }
    // the columns: update, then the product with the new reflector
    double acc = 0.0;
    if (c < m) {
        const double vc = vs[c - r0], wc = ws[c - r0];
        auto col_row = [&](int i, double ai) {
            const double x = ai - (vs[i - r0] * wc + ws[i - r0] * vc);
            col[i] = x;
            if (i == c) diag[c] = x;
            acc = __builtin_fma(x, vl[i - r0], acc);
        };
#pragma unroll
        for (int u = 0; u < kHhCol; ++u) {
            const int i = r0 + 64 * h + lane + 128 * u;
            if (i < m) col_row(i, a[u]);
        }
        for (int base = r0 + 64 * h + lane + 128 * kHhCol; base < m; base += 128 * kUnroll) {
            double b[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = base + 128 * u;
                b[u] = i < m ? col[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int i = base + 128 * u;
                if (i < m) col_row(i, b[u]);
            }
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    double dotc = 0.0;
    if (h == 0 && c < m) {
        const double pcn = beta1 * (red[wv] + red[wv + 4]);
        if (lane == 0) pn[c] = pcn;
        dotc = vl[c - r0] * pcn;
    }
    __syncthreads();    // red[] reused
    if (lane == 0 && h == 0) red[wv] = dotc;
    __syncthreads();
    if (tid == 0) partn[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Number of eigenvalues of T above tau: positive pivots of the LDL^T of
// T - tau I (Sylvester's law of inertia / Sturm sequence).
__global__ void sturm_count(const double *diag, const double *off, int m, double tau, int *count)
{
    int cnt = 0;
    double q = 0.0;
    for (int i = 0; i < m; ++i) {
        double qi = diag[i] - tau;
        if (i > 0) qi -= off[i - 1] * off[i - 1] / q;
        if (qi == 0.0) qi = -1e-300;
        if (qi > 0.0) ++cnt;
        q = qi;
    }
    *count = cnt;
}

}  // namespace

afn_status uniform_landmarks(int64_t n, int k, uint64_t seed, int32_t *idx, hipStream_t s)
{
    if (k < 0 || k > n || k > kMaxM) {
        set_error("uniform landmarks: k=%d outside [0, min(n, %d)]", k, kMaxM);
        return AFN_EINVAL;
    }
    if (k == 0) return AFN_OK;
    hipLaunchKernelGGL(subsample_kernel, dim3(1), dim3(kSubThreads), 0, s, n, k, seed, idx);
    AFN_HIP(hipGetLastError());
    return AFN_OK;
}

namespace {

int64_t scan_parts(int m)
{
    const int64_t p = kScanE * ceil_div(m, kUT) * ceil_div(m, kUT);
    return p > 256 ? p : 256;
}

}  // namespace

size_t rank_workspace_bytes(int m, int d)
{
    // every buffer rank_estimate carves, in its order, each from a 256-byte boundary
    const int64_t sizes[] = {4 * (int64_t)m, 4 * (int64_t)m, 8 * (int64_t)m * d, 8 * (int64_t)m * m,
                             8 * (int64_t)kScanB * m, 8 * (int64_t)kScanB * m, 8 * scan_parts(m),
                             8 * ((int64_t)m + 1), 4, 4 * kScanB, (int64_t)fps_workspace_bytes(m),
                             16 * (int64_t)m, 16 * (int64_t)m, 64, 4, 16 * (ceil_div(m, 4) + 1),
                             8 * (int64_t)m, 8 * (int64_t)m};
    int64_t total = 0;
    for (int64_t b : sizes) total += round_up(b, 256);
    return (size_t)total;
}

afn_status rank_estimate(const double *X, int64_t n, int d, double l, int kind, double mu, int m, int kmax,
                         uint64_t seed, DevArena &tmp, hipStream_t s, afn_setup_info *info, int *k_out)
{
    if (m < 1 || m > n || m > kMaxM) {
        set_error("rank estimation: subsample size m=%d outside [1, min(n, %d)]", m, kMaxM);
        return AFN_EINVAL;
    }
    int32_t *sub = nullptr, *ord = nullptr;
    double *Xm = nullptr, *K = nullptr, *C = nullptr, *Q = nullptr, *part = nullptr, *errs = nullptr;
    double *v = nullptr, *pw = nullptr, *gp = nullptr, *sc = nullptr, *tdiag = nullptr, *toff = nullptr;
    int *cnt = nullptr, *err = nullptr, *skip = nullptr;
    void *fws = nullptr;
    const int nparts = 256;
    AFN_TRY(tmp.alloc_n(&sub, m));
    AFN_TRY(tmp.alloc_n(&ord, m));
    AFN_TRY(tmp.alloc_n(&Xm, (int64_t)m * d));
    AFN_TRY(tmp.alloc_n(&K, (int64_t)m * m));
    AFN_TRY(tmp.alloc_n(&C, (int64_t)kScanB * m));
    AFN_TRY(tmp.alloc_n(&Q, (int64_t)kScanB * m));
    AFN_TRY(tmp.alloc_n(&part, scan_parts(m)));
    AFN_TRY(tmp.alloc_n(&errs, m + 1));
    AFN_TRY(tmp.alloc_n(&err, 1));
    AFN_TRY(tmp.alloc_n(&skip, kScanB));
    AFN_TRY(tmp.alloc(&fws, fps_workspace_bytes(m)));
    AFN_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
    const double l2 = l * l;
    const int64_t mm = (int64_t)m * m;
    const unsigned gmm = (unsigned)ceil_div(mm, 256);
    hipLaunchKernelGGL(subsample_kernel, dim3(1), dim3(kSubThreads), 0, s, n, m, seed, sub);
    const double scale = std::pow((double)m / (double)n, 1.0 / (double)d);
    hipLaunchKernelGGL(gather_scaled, dim3((unsigned)ceil_div((int64_t)m * d, 256)), dim3(256), 0, s, X,
                       sub, m, d, scale, Xm);
    hipLaunchKernelGGL(kmat_fill, dim3(gmm), dim3(256), 0, s, Xm, m, d, l2, kind, K);
    // FPS order of the subsample, produced 64 positions at a time as the scan
    // needs them, on a second stream one chunk ahead of the scan: chunk c + 1
    // runs while the passes of chunk c do (the scan reads only ord, at
    // positions an earlier chunk wrote; events ev0 / ev1 mark even / odd chunks)
    AFN_TRY(fps_start(Xm, m, d, fws, s, err));
    SideStream side;
    AFN_TRY(side.open());
    AFN_HIP(hipEventRecord(side.ev0, s));
    AFN_HIP(hipStreamWaitEvent(side.st, side.ev0, 0));
    AFN_TRY(fps_advance(Xm, m, d, 0, m < 64 ? m : 64, m, ord, nullptr, fws, side.st, err));
    AFN_HIP(hipEventRecord(side.ev0, side.st));
    hipLaunchKernelGGL(sumsq_partial, dim3(nparts), dim3(256), 0, s, K, mm, part);
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(256), 0, s, part, nparts, errs + m);
    AFN_HIP(hipGetLastError());
    // nested Nystrom scan, one pass over the residual per 32 eliminations (two
    // per FPS chunk of 64), the errors read back after each chunk
    std::vector<double> herr((size_t)m + 1, -1.0);
    AFN_HIP(hipMemcpyAsync(&herr[m], errs + m, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    const double f0 = std::sqrt(herr[m]);
    const double pivtol = 1e-14 * (double)m;
    const dim3 gpanel((unsigned)ceil_div(m, 256));
    const dim3 gupd((unsigned)ceil_div(m, kUT), (unsigned)ceil_div(m, kUT));
    const int nupd = (int)(gupd.x * gupd.y);
    int r_found = m;
    for (int r0 = 0; r0 < m && r_found == m; r0 += 64) {
        const int r1 = r0 + 64 < m ? r0 + 64 : m;
        const bool odd = (r0 / 64) & 1;
        if (r1 < m) {
            AFN_TRY(fps_advance(Xm, m, d, r1, r1 + 64 < m ? r1 + 64 : m, m, ord, nullptr, fws, side.st, err));
            AFN_HIP(hipEventRecord(odd ? side.ev0 : side.ev1, side.st));
        }
        AFN_HIP(hipStreamWaitEvent(s, odd ? side.ev1 : side.ev0, 0));
        for (int b0 = r0; b0 < r1; b0 += kScanB) {
            const int nb = b0 + kScanB < r1 ? kScanB : r1 - b0;
            hipLaunchKernelGGL(scan_panel, gpanel, dim3(256), 0, s, K, m, ord, b0, nb, pivtol, C, Q, skip);
            hipLaunchKernelGGL(scan_update, gupd, dim3(256), 0, s, K, m, ord, b0, nb, C, Q, skip, part);
            hipLaunchKernelGGL(scan_errors, dim3(kScanE), dim3(256), 0, s, part, nupd, b0, nb, errs);
        }
        AFN_HIP(hipGetLastError());
        AFN_HIP(hipMemcpyAsync(&herr[r0], errs + r0, sizeof(double) * (r1 - r0),
                               hipMemcpyDeviceToHost, s));
        AFN_HIP(hipStreamSynchronize(s));
        for (int r = r0; r < r1; ++r) {
            const int rr = r + 1;
            if (rr % 8 == 0 || rr == m) {
                const double e = f0 > 0.0 ? std::sqrt(herr[r]) / f0 : 0.0;
                if (e < 0.1) {
                    r_found = rr;
                    break;
                }
            }
        }
    }
    // the chunk ahead may still run, and the eigenvalue branch rewrites Xm
    AFN_HIP(hipStreamSynchronize(side.st));
    const int64_t kest = (int64_t)std::floor((double)r_found * (double)n / (double)m);
    int64_t k = kest;
    info->rank_r = r_found;
    info->rank_k_est = kest;
    info->rank_eig_branch = 0;
    info->rank_eig_count = -1;
    if (kest < 2000) {
        // eigenvalues of K(X_m, X_m) on the unscaled subsample above 0.1 mu
        AFN_TRY(tmp.alloc_n(&v, 2 * (int64_t)m));
        AFN_TRY(tmp.alloc_n(&pw, 2 * (int64_t)m));
        AFN_TRY(tmp.alloc_n(&sc, 8));
        AFN_TRY(tmp.alloc_n(&cnt, 1));
        const int64_t gps = ceil_div(m, 4) + 1;
        AFN_TRY(tmp.alloc_n(&gp, 2 * gps));
        AFN_TRY(tmp.alloc_n(&tdiag, m));
        AFN_TRY(tmp.alloc_n(&toff, m));
        hipLaunchKernelGGL(gather_scaled, dim3((unsigned)ceil_div((int64_t)m * d, 256)), dim3(256), 0, s,
                           X, sub, m, d, 1.0, Xm);
        hipLaunchKernelGGL(kmat_fill, dim3(gmm), dim3(256), 0, s, Xm, m, d, l2, kind, K);
        hipLaunchKernelGGL(hh_init, dim3(1), dim3(64), 0, s, K, m, v, sc, tdiag, toff);
        if (m >= 3)
            hipLaunchKernelGGL(hh_mv, dim3((unsigned)ceil_div(m - 1, 4)), dim3(256), 0, s, K, m, 0, v, sc, pw,
                               gp);
        // one limit for every launch (the largest subsample's): setups on
        // other threads launch hh_step with other sizes at the same time
        if (3 * sizeof(double) * (size_t)(m - 2) > 64 * 1024)
            AFN_HIP(hipFuncSetAttribute((const void *)hh_step, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)(3 * sizeof(double) * (size_t)(kMaxM - 2))));
        // step j reads buffer set j & 1 (v, beta, p, partials) and writes the other
        for (int j = 0; j + 2 < m; ++j) {
            const int nb = (int)ceil_div(m - j - 1, 4);         // workgroups of the previous launch
            const int nbn = (int)ceil_div(m - j - 2, 4);        // of this one (>= 1: j + 2 < m)
            const int cur = j & 1, nxt = cur ^ 1;
            const size_t lds = 3 * sizeof(double) * (size_t)(m - j - 2);
            hipLaunchKernelGGL(hh_step, dim3((unsigned)nbn), dim3(512), lds, s, K, m, j, v + (int64_t)cur * m,
                               sc + 4 * cur, pw + (int64_t)cur * m, gp + cur * gps, nb, v + (int64_t)nxt * m,
                               sc + 4 * nxt, pw + (int64_t)nxt * m, gp + nxt * gps, tdiag, toff);
        }
        hipLaunchKernelGGL(sturm_count, dim3(1), dim3(1), 0, s, tdiag, toff, m, 0.1 * mu, cnt);
        AFN_HIP(hipGetLastError());
        int hc = 0;
        AFN_HIP(hipMemcpyAsync(&hc, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        AFN_HIP(hipStreamSynchronize(s));
        k = hc;
        info->rank_eig_branch = 1;
        info->rank_eig_count = hc;
    }
    int herr_flag = 0;
    AFN_HIP(hipMemcpy(&herr_flag, err, sizeof(int), hipMemcpyDeviceToHost));
    if (herr_flag) {
        set_error("rank estimation: landmark ordering produced an invalid index");
        return AFN_EDEVICE;
    }
    const int64_t cap = kmax < n ? kmax : n;
    if (k > cap) k = cap;
    if (k < 1) k = 1;
    *k_out = (int)k;
    return AFN_OK;
}

}  // namespace afn
