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

namespace afn {

afn_status fps(const double *X, int64_t n, int d, int k, int32_t *idx, double *seld, void *work,
               hipStream_t s, int *err);
namespace {

constexpr int kMaxM = 4096;
constexpr int kHash = 4 * kMaxM;

__device__ __forceinline__ uint64_t splitmix64_next(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Partial Fisher-Yates over the virtual array a[j] = j, storing only the
// positions that were written (open addressing in LDS).
__global__ __launch_bounds__(64) void subsample_kernel(int64_t n, int m, uint64_t seed, int32_t *sub)
{
    __shared__ int keys[kHash];
    __shared__ int vals[kHash];
    for (int i = threadIdx.x; i < kHash; i += 64) keys[i] = -1;
    __syncthreads();
    if (threadIdx.x != 0) return;
    auto slot = [&](int pos) {
        unsigned h = ((unsigned)pos * 2654435761u) & (kHash - 1);
        while (keys[h] != -1 && keys[h] != pos) h = (h + 1) & (kHash - 1);
        return h;
    };
    auto get = [&](int pos) {
        unsigned h = slot(pos);
        return keys[h] == pos ? vals[h] : pos;
    };
    auto put = [&](int pos, int v) {
        unsigned h = slot(pos);
        keys[h] = pos;
        vals[h] = v;
    };
    uint64_t st = seed;
    for (int i = 0; i < m; ++i) {
        uint64_t draw = splitmix64_next(st);
        int j = (int)(i + (int64_t)(draw % (uint64_t)(n - i)));
        int ai = get(i), aj = get(j);
        put(i, aj);
        put(j, ai);
        sub[i] = aj;
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

__global__ __launch_bounds__(256) void kmat_fill(const double *Xm, int m, int d, double l2, double *K)
{
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double del = Xm[i * d + t] - Xm[j * d + t];
        acc = __builtin_fma(del, del, acc);
    }
    K[e] = exp(-(acc / l2));
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

// c = K[:, pj], piv = K[pj, pj]; skip flag if piv <= pivtol.
__global__ __launch_bounds__(256) void scan_column(const double *K, int m, const int32_t *ord, int r,
                                                   double pivtol, double *c, double *pv)
{
    const int pj = ord[r];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        c[i] = K[i + (int64_t)pj * m];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double p = K[pj + (int64_t)pj * m];
        pv[0] = p;
        pv[1] = p > pivtol ? 0.0 : 1.0;
    }
}

// K -= c c^T / piv  (entry-wise: K[i,j] -= c[i] * (c[j] / piv)), or zero the
// row and column of a skipped pivot.
__global__ __launch_bounds__(256) void scan_update(double *K, int m, const int32_t *ord, int r,
                                                   const double *c, const double *pv)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)m * m) return;
    const int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    if (pv[1] != 0.0) {
        const int pj = ord[r];
        if (i == pj || j == pj) K[e] = 0.0;
        return;
    }
    const double cj = c[j] / pv[0];
    K[e] -= c[i] * cj;
}

// ---------------------------------------------------------------- eigen count
// Householder step j on A (m x m, column-major): scalars sc[0] = beta,
// sc[1] = s (new sub-diagonal), sc[2] = skip flag; v (m, zero outside j+1..).
__global__ __launch_bounds__(256) void hh_vector(double *A, int m, int j, double *v, double *sc)
{
    __shared__ double ws[4];
    const int tid = threadIdx.x;
    double a2 = 0.0;
    for (int i = j + 1 + tid; i < m; i += 256) a2 += A[i + (int64_t)j * m] * A[i + (int64_t)j * m];
    for (int off = 32; off > 0; off >>= 1) a2 += __shfl_xor(a2, off, 64);
    if ((tid & 63) == 0) ws[tid >> 6] = a2;
    __syncthreads();
    const double alpha2 = ws[0] + ws[1] + ws[2] + ws[3];
    __syncthreads();
    const double alpha = sqrt(alpha2);
    const double x0 = A[j + 1 + (int64_t)j * m];
    const double snew = x0 >= 0.0 ? -alpha : alpha;
    for (int i = tid; i < m; i += 256) {
        double vi = 0.0;
        if (i == j + 1) vi = x0 - snew;
        else if (i > j + 1) vi = A[i + (int64_t)j * m];
        v[i] = vi;
    }
    double vn = 0.0;
    for (int i = j + 1 + tid; i < m; i += 256) {
        double vi = (i == j + 1) ? x0 - snew : A[i + (int64_t)j * m];
        vn += vi * vi;
    }
    for (int off = 32; off > 0; off >>= 1) vn += __shfl_xor(vn, off, 64);
    if ((tid & 63) == 0) ws[tid >> 6] = vn;
    __syncthreads();
    if (tid == 0) {
        const double vnorm2 = ws[0] + ws[1] + ws[2] + ws[3];
        const bool skip = alpha == 0.0 || vnorm2 == 0.0;
        sc[0] = skip ? 0.0 : 2.0 / vnorm2;
        sc[1] = snew;
        sc[2] = skip ? 1.0 : 0.0;
    }
}

// pw[i] = beta * sum_t A[i,t] v[t] for i > j, partial over column chunks
__global__ __launch_bounds__(256) void hh_matvec(const double *A, int m, int j, const double *v,
                                                 int chunk, double *part)
{
    const int i = j + 1 + blockIdx.x * blockDim.x + threadIdx.x;
    const int t0 = j + 1 + blockIdx.y * chunk;
    const int t1 = t0 + chunk < m ? t0 + chunk : m;
    if (i >= m) return;
    double s = 0.0;
    for (int t = t0; t < t1; ++t) s = __builtin_fma(A[i + (int64_t)t * m], v[t], s);
    part[(int64_t)blockIdx.y * m + i] = s;
}

__global__ __launch_bounds__(256) void hh_pw(const double *part, int splits, int m, int j,
                                             const double *v, const double *sc, double *pw)
{
    __shared__ double ws[4];
    const int tid = threadIdx.x;
    const double beta = sc[0];
    double vtp = 0.0;
    for (int i = j + 1 + tid; i < m; i += 256) {
        double s = 0.0;
        for (int q = 0; q < splits; ++q) s += part[(int64_t)q * m + i];
        double p = beta * s;
        pw[i] = p;
        vtp += v[i] * p;
    }
    for (int off = 32; off > 0; off >>= 1) vtp += __shfl_xor(vtp, off, 64);
    if ((tid & 63) == 0) ws[tid >> 6] = vtp;
    __syncthreads();
    const double kk = 0.5 * beta * (ws[0] + ws[1] + ws[2] + ws[3]);
    for (int i = j + 1 + tid; i < m; i += 256) pw[i] -= kk * v[i];
}

__global__ __launch_bounds__(256) void hh_update(double *A, int m, int j, const double *v,
                                                 const double *pw, const double *sc)
{
    const int64_t mm = m - j - 1;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool skip = sc[2] != 0.0;
    if (e < mm * mm && !skip) {
        const int c = j + 1 + (int)(e / mm), i = j + 1 + (int)(e % mm);
        A[i + (int64_t)c * m] -= v[i] * pw[c] + pw[i] * v[c];
    }
    // column / row j: new sub-diagonal, zeros below
    if (!skip && e < m) {
        const int i = (int)e;
        if (i == j + 1) {
            A[i + (int64_t)j * m] = sc[1];
            A[j + (int64_t)i * m] = sc[1];
        } else if (i > j + 1) {
            A[i + (int64_t)j * m] = 0.0;
            A[j + (int64_t)i * m] = 0.0;
        }
    }
}

__global__ void sturm_count(const double *A, int m, double tau, int *count)
{
    int cnt = 0;
    double q = 0.0;
    for (int i = 0; i < m; ++i) {
        double qi = A[i + (int64_t)i * m] - tau;
        if (i > 0) {
            double b = A[i + (int64_t)(i - 1) * m];
            qi -= b * b / q;
        }
        if (qi == 0.0) qi = -1e-300;
        if (qi > 0.0) ++cnt;
        q = qi;
    }
    *count = cnt;
}

}  // namespace

afn_status rank_estimate(const double *X, int64_t n, int d, double l, double mu, int m, int kmax,
                         uint64_t seed, hipStream_t s, afn_setup_info *info, int *k_out)
{
    if (m < 1 || m > n || m > kMaxM) {
        set_error("rank estimation: subsample size m=%d outside [1, min(n, %d)]", m, kMaxM);
        return AFN_EINVAL;
    }
    DevArena tmp;
    struct G {
        DevArena &a;
        ~G() { a.release(); }
    } guard{tmp};
    int32_t *sub = nullptr, *ord = nullptr;
    double *Xm = nullptr, *K = nullptr, *c = nullptr, *pv = nullptr, *part = nullptr, *errs = nullptr;
    double *v = nullptr, *pw = nullptr, *gp = nullptr, *sc = nullptr;
    int *cnt = nullptr, *err = nullptr;
    void *fws = nullptr;
    const int nparts = 256;
    AFN_TRY(tmp.alloc_n(&sub, m));
    AFN_TRY(tmp.alloc_n(&ord, m));
    AFN_TRY(tmp.alloc_n(&Xm, (int64_t)m * d));
    AFN_TRY(tmp.alloc_n(&K, (int64_t)m * m));
    AFN_TRY(tmp.alloc_n(&c, m));
    AFN_TRY(tmp.alloc_n(&pv, 4));
    AFN_TRY(tmp.alloc_n(&part, nparts));
    AFN_TRY(tmp.alloc_n(&errs, m + 1));
    AFN_TRY(tmp.alloc_n(&err, 1));
    AFN_TRY(tmp.alloc(&fws, fps_workspace_bytes(m)));
    AFN_HIP(hipMemsetAsync(err, 0, sizeof(int), s));
    const double l2 = l * l;
    const int64_t mm = (int64_t)m * m;
    const unsigned gmm = (unsigned)ceil_div(mm, 256);
    hipLaunchKernelGGL(subsample_kernel, dim3(1), dim3(64), 0, s, n, m, seed, sub);
    const double scale = std::pow((double)m / (double)n, 1.0 / (double)d);
    hipLaunchKernelGGL(gather_scaled, dim3((unsigned)ceil_div((int64_t)m * d, 256)), dim3(256), 0, s, X,
                       sub, m, d, scale, Xm);
    hipLaunchKernelGGL(kmat_fill, dim3(gmm), dim3(256), 0, s, Xm, m, d, l2, K);
    AFN_TRY(fps(Xm, m, d, m, ord, nullptr, fws, s, err));
    hipLaunchKernelGGL(sumsq_partial, dim3(nparts), dim3(256), 0, s, K, mm, part);
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(256), 0, s, part, nparts, errs + m);
    AFN_HIP(hipGetLastError());
    // nested Nystrom scan in batches of 64 eliminations
    std::vector<double> herr((size_t)m + 1, -1.0);
    AFN_HIP(hipMemcpyAsync(&herr[m], errs + m, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    const double f0 = std::sqrt(herr[m]);
    const double pivtol = 1e-14 * (double)m;
    int r_found = m;
    for (int r0 = 0; r0 < m && r_found == m; r0 += 64) {
        const int r1 = r0 + 64 < m ? r0 + 64 : m;
        for (int r = r0; r < r1; ++r) {
            hipLaunchKernelGGL(scan_column, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, s, K, m, ord,
                               r, pivtol, c, pv);
            hipLaunchKernelGGL(scan_update, dim3(gmm), dim3(256), 0, s, K, m, ord, r, c, pv);
            const int rr = r + 1;
            if (rr % 8 == 0 || rr == m) {
                hipLaunchKernelGGL(sumsq_partial, dim3(nparts), dim3(256), 0, s, K, mm, part);
                hipLaunchKernelGGL(sum_parts, dim3(1), dim3(256), 0, s, part, nparts, errs + rr - 1);
            }
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
    const int64_t kest = (int64_t)std::floor((double)r_found * (double)n / (double)m);
    int64_t k = kest;
    info->rank_r = r_found;
    info->rank_k_est = kest;
    info->rank_eig_branch = 0;
    info->rank_eig_count = -1;
    if (kest < 2000) {
        // eigenvalues of K(X_m, X_m) on the unscaled subsample above 0.1 mu
        AFN_TRY(tmp.alloc_n(&v, m));
        AFN_TRY(tmp.alloc_n(&pw, m));
        AFN_TRY(tmp.alloc_n(&sc, 4));
        AFN_TRY(tmp.alloc_n(&cnt, 1));
        hipLaunchKernelGGL(gather_scaled, dim3((unsigned)ceil_div((int64_t)m * d, 256)), dim3(256), 0, s,
                           X, sub, m, d, 1.0, Xm);
        hipLaunchKernelGGL(kmat_fill, dim3(gmm), dim3(256), 0, s, Xm, m, d, l2, K);
        const int splits = 8;
        AFN_TRY(tmp.alloc_n(&gp, (int64_t)splits * m));
        for (int j = 0; j + 2 < m; ++j) {
            const int rows = m - j - 1;
            const int chunk = (int)ceil_div(rows, splits);
            hipLaunchKernelGGL(hh_vector, dim3(1), dim3(256), 0, s, K, m, j, v, sc);
            hipLaunchKernelGGL(hh_matvec, dim3((unsigned)ceil_div(rows, 256), (unsigned)splits),
                               dim3(256), 0, s, K, m, j, v, chunk, gp);
            hipLaunchKernelGGL(hh_pw, dim3(1), dim3(256), 0, s, gp, splits, m, j, v, sc, pw);
            const int64_t upd = (int64_t)rows * rows > m ? (int64_t)rows * rows : m;
            hipLaunchKernelGGL(hh_update, dim3((unsigned)ceil_div(upd, 256)), dim3(256), 0, s, K, m, j, v,
                               pw, sc);
        }
        hipLaunchKernelGGL(sturm_count, dim3(1), dim3(1), 0, s, K, m, 0.1 * mu, cnt);
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
