/*
 * afn_oracle.c -- plain, slow, FP64 CPU oracle for AFN-preconditioned CG.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * shares no code, header, table or helper with it.
 *
 * Source: "An Adaptive Factorized Nystrom Preconditioner for Regularized
 * Kernel Matrices" (Zhao, Xu, Huang, Chow, Xi; arXiv 2304.05460).
 * Every function names the passage it follows.  Where the paper is silent or
 * ambiguous the reading taken is stated in the comment (and listed in the
 * design notes of the repository).
 *
 * Arithmetic: IEEE FP64, compiled with -ffp-contract=off so that every fused
 * multiply-add is an explicit fma() call and every other operation rounds on
 * its own.  OpenMP is used only as "parallel for" over independent outputs,
 * each computed in a fixed order, so results do not depend on thread count.
 *
 * Status codes: 0 ok, 1 invalid argument, 2 out of memory, 3 matrix not SPD,
 * 4 no convergence within maxit, 5 CG breakdown (p'Ap <= 0 or NaN).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_EINVAL 1
#define ORA_ENOMEM 2
#define ORA_ENOTSPD 3
#define ORA_ENOCONV 4
#define ORA_EBREAKDOWN 5

/* ------------------------------------------------------------------------ */
/* Kernel function (Eq. (1.2), the Gaussian kernel; no factor 1/2).         */
/* ------------------------------------------------------------------------ */

/* Squared Euclidean distance as the fixed chain
 *   acc = 0; for t: delta = a[t]-b[t]; acc = fma(delta, delta, acc).
 * Symmetric bit-for-bit because round(a-b) = -round(b-a). */
double ora_sqdist(const double *a, const double *b, int d)
{
    double acc = 0.0;
    for (int t = 0; t < d; ++t) {
        double del = a[t] - b[t];
        acc = fma(del, del, acc);
    }
    return acc;
}

/* The kernel function (Section 5): kind 0 = Gaussian
 *   K(x,y) = exp(-||x-y||^2 / l^2)                     (Eq. (1.2)),
 * kind 1 = Matern-3/2
 *   K(x,y) = (1 + sqrt(3) ||x-y|| / l) exp(-sqrt(3) ||x-y|| / l).
 * The kind is process-wide state of this test library (ora_set_kernel). */
static int g_kernel_kind = 0;

int ora_set_kernel(int kind)
{
    if (kind != 0 && kind != 1) return ORA_EINVAL;
    g_kernel_kind = kind;
    return ORA_OK;
}

double ora_kernel(const double *a, const double *b, int d, double l)
{
    if (g_kernel_kind == 1) {
        const double s = sqrt(3.0) * sqrt(ora_sqdist(a, b, d)) / l;
        return (1.0 + s) * exp(-s);
    }
    return exp(-(ora_sqdist(a, b, d) / (l * l)));
}

/* ------------------------------------------------------------------------ */
/* Regularized kernel matvec  y = (K + mu I) v   (Eq. (1.1)).               */
/* v, y: column-major n x nrhs, leading dimension n.                        */
/* ------------------------------------------------------------------------ */
int ora_kernel_matvec(const double *X, int64_t n, int d, double l, double mu,
                      const double *v, int64_t nrhs, double *y)
{
    if (n < 0 || d < 1 || !(l > 0) || nrhs < 1) return ORA_EINVAL;
    int bad = 0;
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * (size_t)nrhs);
        if (!acc) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; ++i) {
            if (!acc) continue;
            for (int64_t r = 0; r < nrhs; ++r) acc[r] = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                double kij = ora_kernel(X + i * d, X + j * d, d, l);
                for (int64_t r = 0; r < nrhs; ++r) acc[r] += kij * v[j + r * n];
            }
            for (int64_t r = 0; r < nrhs; ++r) y[i + r * n] = acc[r] + mu * v[i + r * n];
        }
        free(acc);
    }
    return bad ? ORA_ENOMEM : ORA_OK;
}

/* Selected rows of (K + mu I) v for one right-hand side, plus the absolute
 * sums  sum_j |K_ij v_j| + mu |v_i|  that bound the rounding error of any
 * summation order (used for tolerances at sizes the full product is too slow). */
int ora_kernel_matvec_rows(const double *X, int64_t n, int d, double l, double mu,
                           const double *v, const int64_t *rows, int64_t nrows,
                           double *y_rows, double *abs_rows)
{
    if (n < 0 || d < 1 || !(l > 0)) return ORA_EINVAL;
    for (int64_t s = 0; s < nrows; ++s)
        if (rows[s] < 0 || rows[s] >= n) return ORA_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nrows; ++s) {
        int64_t i = rows[s];
        double acc = 0.0, aabs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            double t = ora_kernel(X + i * d, X + j * d, d, l) * v[j];
            acc += t;
            aabs += fabs(t);
        }
        y_rows[s] = acc + mu * v[i];
        abs_rows[s] = aabs + fabs(mu * v[i]);
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Farthest point sampling (Algorithm 6, Section 4.5).                      */
/* ------------------------------------------------------------------------ */

/* Centroid (Algorithm 6, the mean of the data points).  The paper does not
 * fix a summation order; a near tie in the first landmark would flip every
 * later one, so the order is fixed: per coordinate, sequential sums over
 * consecutive blocks of 256 ascending indices, then a sequential sum of the
 * block sums in ascending block order, then one division by n. */
int ora_centroid(const double *X, int64_t n, int d, double *c)
{
    if (n < 1 || d < 1) return ORA_EINVAL;
    for (int t = 0; t < d; ++t) {
        double total = 0.0;
        for (int64_t b0 = 0; b0 < n; b0 += 256) {
            int64_t b1 = b0 + 256 < n ? b0 + 256 : n;
            double s = 0.0;
            for (int64_t j = b0; j < b1; ++j) s += X[j * d + t];
            total += s;
        }
        c[t] = total / (double)n;
    }
    return ORA_OK;
}

/* FPS, Algorithm 6.  First landmark: the point nearest the centroid (ties:
 * smallest index).  Then k-1 steps: update the running distance with the last
 * landmark, take the arg-max.  Readings:
 *  - squared distances replace distances (same arg-max/arg-min, no sqrt);
 *  - the arg-max runs over unselected points only and ties go to the smallest
 *    index, so duplicates (all remaining distances 0) never re-select a
 *    landmark.
 * idx[i] = i-th landmark (selection order).  seld[i] = running squared
 * distance of landmark i when it was chosen (seld[0] = +inf), i.e. the squared
 * fill distance of the first i landmarks over the data set. */
int ora_fps(const double *X, int64_t n, int d, int64_t k, int32_t *idx, double *seld)
{
    if (n < 1 || d < 1 || k < 0 || k > n) return ORA_EINVAL;
    if (k == 0) return ORA_OK;
    double c[64];
    if (d > 64) return ORA_EINVAL;
    ora_centroid(X, n, d, c);
    int64_t l0 = 0;
    double best = ora_sqdist(X, c, d);
    for (int64_t j = 1; j < n; ++j) {
        double dj = ora_sqdist(X + j * d, c, d);
        if (dj < best) { best = dj; l0 = j; }
    }
    double *dist = (double *)malloc(sizeof(double) * (size_t)n);
    unsigned char *sel = (unsigned char *)calloc((size_t)n, 1);
    if (!dist || !sel) { free(dist); free(sel); return ORA_ENOMEM; }
    for (int64_t j = 0; j < n; ++j) dist[j] = INFINITY;
    idx[0] = (int32_t)l0;
    sel[l0] = 1;
    if (seld) seld[0] = INFINITY;
    for (int64_t i = 1; i < k; ++i) {
        const double *xl = X + (int64_t)idx[i - 1] * d;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            if (sel[j]) continue;
            double dj = ora_sqdist(X + j * d, xl, d);
            if (dj < dist[j]) dist[j] = dj;
        }
        int64_t arg = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (sel[j]) continue;
            if (arg < 0 || dist[j] > dist[arg]) arg = j;
        }
        idx[i] = (int32_t)arg;
        sel[arg] = 1;
        if (seld) seld[i] = dist[arg];
    }
    free(dist);
    free(sel);
    return ORA_OK;
}

/* Point order of the 2x2 block partition (Section 2: landmarks indexed first).
 * perm = [landmarks in FPS order ; the remaining points by ascending original
 * index] (reading: the paper does not number X \ X_k; ascending order is
 * taken). */
int ora_permutation(int64_t n, int64_t k, const int32_t *idx, int32_t *perm)
{
    if (k < 0 || k > n) return ORA_EINVAL;
    unsigned char *sel = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!sel) return ORA_ENOMEM;
    for (int64_t i = 0; i < k; ++i) {
        if (idx[i] < 0 || idx[i] >= n || sel[idx[i]]) { free(sel); return ORA_EINVAL; }
        sel[idx[i]] = 1;
        perm[i] = idx[i];
    }
    int64_t p = k;
    for (int64_t j = 0; j < n; ++j)
        if (!sel[j]) perm[p++] = (int32_t)j;
    free(sel);
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense Cholesky and triangular solves (Algorithm 2, L = chol(K11 + mu I)).*/
/* ------------------------------------------------------------------------ */

/* Textbook right-looking Cholesky without pivoting, in place on the lower
 * triangle of a column-major k x k matrix (leading dimension lda).  A pivot
 * that is not > 0 gives ORA_ENOTSPD.  The strict upper triangle is zeroed. */
int ora_cholesky(double *A, int64_t k, int64_t lda)
{
    for (int64_t j = 0; j < k; ++j) {
        double djj = A[j + j * lda];
        if (!(djj > 0.0)) return ORA_ENOTSPD;
        double ljj = sqrt(djj);
        A[j + j * lda] = ljj;
        for (int64_t i = j + 1; i < k; ++i) A[i + j * lda] /= ljj;
#pragma omp parallel for schedule(dynamic, 16) if (k - j > 256)
        for (int64_t c = j + 1; c < k; ++c) {
            double lcj = A[c + j * lda];
            for (int64_t i = c; i < k; ++i) A[i + c * lda] -= A[i + j * lda] * lcj;
        }
    }
    for (int64_t j = 0; j < k; ++j)
        for (int64_t i = 0; i < j; ++i) A[i + j * lda] = 0.0;
    return ORA_OK;
}

/* Solve L y = b (forward substitution), L lower, column-major. */
static void fwd_subst(const double *L, int64_t k, int64_t lda, const double *b, double *y)
{
    for (int64_t i = 0; i < k; ++i) {
        double s = b[i];
        for (int64_t t = 0; t < i; ++t) s -= L[i + t * lda] * y[t];
        y[i] = s / L[i + i * lda];
    }
}

/* Solve L^T x = y (backward substitution), L lower, column-major. */
static void bwd_subst(const double *L, int64_t k, int64_t lda, const double *y, double *x)
{
    for (int64_t i = k - 1; i >= 0; --i) {
        double s = y[i];
        for (int64_t t = i + 1; t < k; ++t) s -= L[t + i * lda] * x[t];
        x[i] = s / L[i + i * lda];
    }
}

int ora_fwd_subst(const double *L, int64_t k, const double *b, double *y)
{
    fwd_subst(L, k, k, b, y);
    return ORA_OK;
}

int ora_bwd_subst(const double *L, int64_t k, const double *y, double *x)
{
    bwd_subst(L, k, k, y, x);
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* FSAI sparsity pattern (Section 3.1).                                     */
/* ------------------------------------------------------------------------ */

/* Row p of the lower-triangular pattern over the non-landmark points X_r
 * (positions 0..nr-1 in the order of ora_permutation): the w-1 nearest
 * earlier-numbered points q < p, with keys (squared distance, q) compared
 * lexicographically, plus p itself; columns sorted ascending, so p is last.
 * Rows with p < w-1 hold all p predecessors (shorter rows).  Xr is row-major
 * nr x d in X_r order.  cols receives the row (length returned). */
static int64_t knn_row(const double *Xr, int d, int64_t w, int64_t p,
                       double *kd, int64_t *kq, int32_t *cols)
{
    int64_t want = w - 1;
    int64_t cnt = 0;
    const double *xp = Xr + p * d;
    for (int64_t q = 0; q < p; ++q) {
        double dq = ora_sqdist(xp, Xr + q * d, d);
        /* keep the 'want' smallest keys in kd/kq sorted ascending */
        if (cnt < want) {
            int64_t pos = cnt++;
            while (pos > 0 && (kd[pos - 1] > dq || (kd[pos - 1] == dq && kq[pos - 1] > q))) {
                kd[pos] = kd[pos - 1];
                kq[pos] = kq[pos - 1];
                --pos;
            }
            kd[pos] = dq;
            kq[pos] = q;
        } else if (want > 0 && (dq < kd[want - 1] || (dq == kd[want - 1] && q < kq[want - 1]))) {
            int64_t pos = want - 1;
            while (pos > 0 && (kd[pos - 1] > dq || (kd[pos - 1] == dq && kq[pos - 1] > q))) {
                kd[pos] = kd[pos - 1];
                kq[pos] = kq[pos - 1];
                --pos;
            }
            kd[pos] = dq;
            kq[pos] = q;
        }
    }
    /* sort the selected neighbour positions ascending (simple insertion sort) */
    for (int64_t a = 0; a < cnt; ++a) cols[a] = (int32_t)kq[a];
    for (int64_t a = 1; a < cnt; ++a) {
        int32_t v = cols[a];
        int64_t b = a;
        while (b > 0 && cols[b - 1] > v) { cols[b] = cols[b - 1]; --b; }
        cols[b] = v;
    }
    cols[cnt] = (int32_t)p;
    return cnt + 1;
}

/* Full pattern in CSR: rowptr (nr+1, int64), cols (capacity nr*w). */
int ora_knn_pattern(const double *Xr, int64_t nr, int d, int64_t w,
                    int64_t *rowptr, int32_t *cols)
{
    if (nr < 0 || d < 1 || w < 1) return ORA_EINVAL;
    rowptr[0] = 0;
    for (int64_t p = 0; p < nr; ++p) rowptr[p + 1] = rowptr[p] + (p + 1 < w ? p + 1 : w);
    int bad = 0;
#pragma omp parallel
    {
        double *kd = (double *)malloc(sizeof(double) * (size_t)w);
        int64_t *kq = (int64_t *)malloc(sizeof(int64_t) * (size_t)w);
        if (!kd || !kq) {
#pragma omp atomic write
            bad = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < nr; ++p) {
            if (!kd || !kq) continue;
            knn_row(Xr, d, w, p, kd, kq, cols + rowptr[p]);
        }
        free(kd);
        free(kq);
    }
    return bad ? ORA_ENOMEM : ORA_OK;
}

/* Selected rows of the pattern: out (nrows x w, padded with -1), len (nrows). */
int ora_knn_rows(const double *Xr, int64_t nr, int d, int64_t w,
                 const int64_t *rows, int64_t nrows, int32_t *out, int32_t *len)
{
    if (nr < 0 || d < 1 || w < 1) return ORA_EINVAL;
    for (int64_t s = 0; s < nrows; ++s)
        if (rows[s] < 0 || rows[s] >= nr) return ORA_EINVAL;
#pragma omp parallel
    {
        double *kd = (double *)malloc(sizeof(double) * (size_t)w);
        int64_t *kq = (int64_t *)malloc(sizeof(int64_t) * (size_t)w);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < nrows; ++s) {
            for (int64_t a = 0; a < w; ++a) out[s * w + a] = -1;
            len[s] = (int32_t)knn_row(Xr, d, w, rows[s], kd, kq, out + s * w);
        }
        free(kd);
        free(kq);
    }
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* AFN construction (Algorithm 2) on an explicit landmark set.              */
/* ------------------------------------------------------------------------ */

/* Gathers the points in block order: Xp = X[perm] (row-major n x d). */
static void gather_points(const double *X, int64_t n, int d, const int32_t *perm, double *Xp)
{
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < d; ++t) Xp[i * d + t] = X[(int64_t)perm[i] * d + t];
}

/* L = chol(K11 + mu I) over the first k points of Xp (Algorithm 2). */
int ora_landmark_cholesky(const double *Xp, int64_t k, int d, double l, double mu, double *L)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < k; ++j)
        for (int64_t i = 0; i < k; ++i)
            L[i + j * k] = ora_kernel(Xp + i * d, Xp + j * d, d, l) + (i == j ? mu : 0.0);
    return ora_cholesky(L, k, k);
}

/* Column p of V = L^{-1} K12 (K12 over landmarks x non-landmarks). */
static void v_column(const double *Xp, int64_t k, int d, double l, const double *L,
                     int64_t p, double *kcol, double *vcol)
{
    const double *xr = Xp + (k + p) * d;
    for (int64_t t = 0; t < k; ++t) kcol[t] = ora_kernel(Xp + t * d, xr, d, l);
    fwd_subst(L, k, k, kcol, vcol);
}

/* One FSAI row (Algorithm 1 applied to the Schur complement
 *   S = K22 + mu I - K12^T (K11 + mu I)^{-1} K12,  Algorithm 2):
 *   S_ss[a][b] = K(s_a, s_b) + mu delta_ab - sum_t V[t][s_a] V[t][s_b]
 *   solve S_ss y = e_last (dense Cholesky + two substitutions)
 *   g = y / sqrt(y_last).
 * V columns of the pattern are passed in (vcols: k x m, column-major). */
static int fsai_row(const double *Xp, int64_t k, int d, double l, double mu,
                    const int32_t *s, int64_t m, const double *vcols,
                    double *S, double *e, double *y, double *g)
{
    for (int64_t b = 0; b < m; ++b)
        for (int64_t a = 0; a < m; ++a) {
            double kab = ora_kernel(Xp + (k + s[a]) * d, Xp + (k + s[b]) * d, d, l);
            double acc = 0.0;
            for (int64_t t = 0; t < k; ++t) acc += vcols[t + a * k] * vcols[t + b * k];
            S[a + b * m] = kab + (a == b ? mu : 0.0) - acc;
        }
    int st = ora_cholesky(S, m, m);
    if (st) return st;
    for (int64_t a = 0; a < m; ++a) e[a] = (a == m - 1) ? 1.0 : 0.0;
    double *tmp = g; /* reuse as scratch */
    fwd_subst(S, m, m, e, tmp);
    bwd_subst(S, m, m, tmp, y);
    double scale = sqrt(y[m - 1]);
    for (int64_t a = 0; a < m; ++a) g[a] = y[a] / scale;
    return ORA_OK;
}

/* Complete AFN construction on given landmarks (Algorithm 2 after the
 * landmark choice).  Outputs, all in block order:
 *   perm  (n)           block order -> original index
 *   L     (k x k)       chol(K11 + mu I), column-major
 *   rowptr(nr+1), cols (nr*w), gval (nr*w): FSAI factor G in CSR.
 * k = 0 gives plain FSAI of K + mu I; k = n gives no FSAI rows. */
int ora_afn_build(const double *X, int64_t n, int d, double l, double mu,
                  int64_t k, const int32_t *idx, int64_t w,
                  int32_t *perm, double *L, int64_t *rowptr, int32_t *cols, double *gval)
{
    if (n < 1 || d < 1 || !(l > 0) || !(mu >= 0) || k < 0 || k > n || w < 1) return ORA_EINVAL;
    int st = ora_permutation(n, k, idx, perm);
    if (st) return st;
    int64_t nr = n - k;
    double *Xp = (double *)malloc(sizeof(double) * (size_t)(n * d));
    double *V = (double *)malloc(sizeof(double) * (size_t)(k * nr > 0 ? k * nr : 1));
    if (!Xp || !V) { free(Xp); free(V); return ORA_ENOMEM; }
    gather_points(X, n, d, perm, Xp);
    if (k > 0) {
        st = ora_landmark_cholesky(Xp, k, d, l, mu, L);
        if (st) { free(Xp); free(V); return st; }
    }
    /* V = L^{-1} K12, column by column */
#pragma omp parallel
    {
        double *kcol = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < nr; ++p)
            if (k > 0) v_column(Xp, k, d, l, L, p, kcol, V + p * k);
        free(kcol);
    }
    st = ora_knn_pattern(Xp + k * d, nr, d, w, rowptr, cols);
    if (st) { free(Xp); free(V); return st; }
    int bad = 0;
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)(w * w));
        double *e = (double *)malloc(sizeof(double) * (size_t)w);
        double *y = (double *)malloc(sizeof(double) * (size_t)w);
        double *vc = (double *)malloc(sizeof(double) * (size_t)(w * (k > 0 ? k : 1)));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < nr; ++p) {
            int64_t m = rowptr[p + 1] - rowptr[p];
            const int32_t *s = cols + rowptr[p];
            for (int64_t a = 0; a < m; ++a)
                for (int64_t t = 0; t < k; ++t) vc[t + a * k] = V[t + (int64_t)s[a] * k];
            int rs = fsai_row(Xp, k, d, l, mu, s, m, vc, S, e, y, gval + rowptr[p]);
            if (rs) {
#pragma omp atomic write
                bad = rs;
            }
        }
        free(S); free(e); free(y); free(vc);
    }
    free(Xp);
    free(V);
    return bad;
}

/* Selected FSAI rows at sizes where the full build is too slow.  Needs the
 * landmark factor L (from ora_landmark_cholesky) and perm.  Row patterns are
 * recomputed here (ora_knn_rows); V columns are formed one by one.
 * out_cols/out_g: nrows x w (padded with -1 / 0), out_len: nrows. */
int ora_fsai_rows(const double *X, int64_t n, int d, double l, double mu,
                  int64_t k, const int32_t *perm, const double *L, int64_t w,
                  const int64_t *rows, int64_t nrows,
                  int32_t *out_cols, int32_t *out_len, double *out_g)
{
    if (n < 1 || d < 1 || k < 0 || k > n || w < 1) return ORA_EINVAL;
    int64_t nr = n - k;
    double *Xp = (double *)malloc(sizeof(double) * (size_t)(n * d));
    if (!Xp) return ORA_ENOMEM;
    gather_points(X, n, d, perm, Xp);
    int st = ora_knn_rows(Xp + k * d, nr, d, w, rows, nrows, out_cols, out_len);
    if (st) { free(Xp); return st; }
    int bad = 0;
#pragma omp parallel
    {
        double *S = (double *)malloc(sizeof(double) * (size_t)(w * w));
        double *e = (double *)malloc(sizeof(double) * (size_t)w);
        double *y = (double *)malloc(sizeof(double) * (size_t)w);
        double *vc = (double *)malloc(sizeof(double) * (size_t)(w * (k > 0 ? k : 1)));
        double *kc = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t m = out_len[r];
            const int32_t *s = out_cols + r * w;
            for (int64_t a = 0; a < m; ++a)
                if (k > 0) v_column(Xp, k, d, l, L, s[a], kc, vc + a * k);
            for (int64_t a = 0; a < w; ++a) out_g[r * w + a] = 0.0;
            int rs = fsai_row(Xp, k, d, l, mu, s, m, vc, S, e, y, out_g + r * w);
            if (rs) {
#pragma omp atomic write
                bad = rs;
            }
        }
        free(S); free(e); free(y); free(vc); free(kc);
    }
    free(Xp);
    return bad;
}

/* ------------------------------------------------------------------------ */
/* AFN application (Algorithm 3), literally, with K12 recomputed.           */
/* ------------------------------------------------------------------------ */

/* s = M^{-1} r for one vector, r and s in ORIGINAL point order:
 *   z  = L^{-T} L^{-1} r1
 *   s2 = G^T G (r2 - K12^T z)
 *   s1 = L^{-T} L^{-1} (r1 - K12 s2)                                       */
int ora_afn_apply(const double *X, int64_t n, int d, double l,
                  int64_t k, const int32_t *perm, const double *L,
                  const int64_t *rowptr, const int32_t *cols, const double *gval,
                  const double *r, double *s)
{
    int64_t nr = n - k;
    double *Xp = (double *)malloc(sizeof(double) * (size_t)(n * d));
    double *rp = (double *)malloc(sizeof(double) * (size_t)n);
    double *sp = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    double *tk = (double *)malloc(sizeof(double) * (size_t)(k + 1));
    double *t2 = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
    double *u = (double *)malloc(sizeof(double) * (size_t)(nr + 1));
    if (!Xp || !rp || !sp || !z || !tk || !t2 || !u) {
        free(Xp); free(rp); free(sp); free(z); free(tk); free(t2); free(u);
        return ORA_ENOMEM;
    }
    gather_points(X, n, d, perm, Xp);
    for (int64_t i = 0; i < n; ++i) rp[i] = r[perm[i]];
    const double *r1 = rp, *r2 = rp + k;
    double *s1 = sp, *s2 = sp + k;
    /* z = L^{-T} L^{-1} r1 */
    if (k > 0) {
        fwd_subst(L, k, k, r1, tk);
        bwd_subst(L, k, k, tk, z);
    }
    /* t2 = r2 - K12^T z */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nr; ++p) {
        double acc = 0.0;
        for (int64_t t = 0; t < k; ++t) acc += ora_kernel(Xp + t * d, Xp + (k + p) * d, d, l) * z[t];
        t2[p] = r2[p] - acc;
    }
    /* u = G t2 */
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nr; ++p) {
        double acc = 0.0;
        for (int64_t a = rowptr[p]; a < rowptr[p + 1]; ++a) acc += gval[a] * t2[cols[a]];
        u[p] = acc;
    }
    /* s2 = G^T u (sequential scatter in ascending row order) */
    for (int64_t p = 0; p < nr; ++p) s2[p] = 0.0;
    for (int64_t p = 0; p < nr; ++p)
        for (int64_t a = rowptr[p]; a < rowptr[p + 1]; ++a) s2[cols[a]] += gval[a] * u[p];
    /* s1 = L^{-T} L^{-1} (r1 - K12 s2) */
    if (k > 0) {
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < k; ++t) {
            double acc = 0.0;
            for (int64_t p = 0; p < nr; ++p) acc += ora_kernel(Xp + t * d, Xp + (k + p) * d, d, l) * s2[p];
            z[t] = r1[t] - acc;
        }
        fwd_subst(L, k, k, z, tk);
        bwd_subst(L, k, k, tk, s1);
    }
    for (int64_t i = 0; i < n; ++i) s[perm[i]] = sp[i];
    free(Xp); free(rp); free(sp); free(z); free(tk); free(t2); free(u);
    return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Preconditioned conjugate gradient (Algorithm 5; stopping rule of         */
/* Section 5: relative residual norm; 500 iterations as the cap).           */
/* ------------------------------------------------------------------------ */

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Textbook PCG from x0 = 0 (the paper prints no PCG listing):
 *   r = b; z = M^{-1} r; p = z; rho = r'z
 *   repeat: q = A p; alpha = rho / p'q  (p'q <= 0 or NaN: breakdown)
 *           x += alpha p; r -= alpha q; stop if ||r|| / ||b|| <= tol
 *           z = M^{-1} r; rho' = r'z; p = z + (rho'/rho) p
 * A = K + mu I.  iters = number of products with A.  relres = recurrence
 * residual; true_relres = ||b - A x|| / ||b|| recomputed at exit.
 * If k == n, G is empty and M = K + mu I.  b == 0 returns x = 0, 0 iters. */
int ora_pcg(const double *X, int64_t n, int d, double l, double mu,
            int64_t k, const int32_t *perm, const double *L,
            const int64_t *rowptr, const int32_t *cols, const double *gval,
            const double *b, double tol, int64_t maxit,
            double *x, int64_t *iters, double *relres, double *true_relres)
{
    if (!(tol > 0) || maxit < 1) return ORA_EINVAL;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *q = (double *)malloc(sizeof(double) * (size_t)n);
    if (!r || !z || !p || !q) { free(r); free(z); free(p); free(q); return ORA_ENOMEM; }
    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; r[i] = b[i]; }
    double bnorm = sqrt(dot(b, b, n));
    *iters = 0;
    *relres = 0.0;
    *true_relres = 0.0;
    int status = ORA_OK;
    if (bnorm == 0.0) goto done;
    ora_afn_apply(X, n, d, l, k, perm, L, rowptr, cols, gval, r, z);
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(r, z, n);
    *relres = 1.0;
    status = ORA_ENOCONV;
    for (int64_t it = 0; it < maxit; ++it) {
        ora_kernel_matvec(X, n, d, l, mu, p, 1, q);
        double pq = dot(p, q, n);
        *iters = it + 1;
        if (!(pq > 0.0)) { status = ORA_EBREAKDOWN; break; }
        double alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        double rel = sqrt(dot(r, r, n)) / bnorm;
        *relres = rel;
        if (!(rel == rel)) { status = ORA_EBREAKDOWN; break; }
        if (rel <= tol) { status = ORA_OK; break; }
        ora_afn_apply(X, n, d, l, k, perm, L, rowptr, cols, gval, r, z);
        double rho_new = dot(r, z, n);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    ora_kernel_matvec(X, n, d, l, mu, x, 1, q);
    for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
    *true_relres = sqrt(dot(q, q, n)) / bnorm;
done:
    free(r); free(z); free(p); free(q);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Nystrom rank estimation (Algorithm 4, Section 3.3).                      */
/* ------------------------------------------------------------------------ */

/* splitmix64 (Steele, Lea & Flood, OOPSLA 2014): counter-based generator;
 * the state advances by the golden-ratio increment and is then mixed. */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Raw splitmix64 outputs for a seed (exposed so tests can pin the generator
 * to its published reference outputs). */
int ora_splitmix64_stream(uint64_t seed, int64_t count, uint64_t *out)
{
    uint64_t st = seed;
    for (int64_t i = 0; i < count; ++i) out[i] = splitmix64_next(&st);
    return ORA_OK;
}

/* Random subsample of Algorithm 4 (reading: the first m entries of a
 * Fisher-Yates shuffle of 0..n-1 driven by splitmix64(seed); position i
 * swaps with i + (draw mod (n - i))).  Integer arithmetic only. */
int ora_subsample(int64_t n, int64_t m, uint64_t seed, int32_t *sub)
{
    if (m < 0 || m > n) return ORA_EINVAL;
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!a) return ORA_ENOMEM;
    for (int64_t i = 0; i < n; ++i) a[i] = (int32_t)i;
    uint64_t st = seed;
    for (int64_t i = 0; i < m; ++i) {
        uint64_t draw = splitmix64_next(&st);
        int64_t j = i + (int64_t)(draw % (uint64_t)(n - i));
        int32_t tmp = a[i]; a[i] = a[j]; a[j] = tmp;
        sub[i] = a[i];
    }
    free(a);
    return ORA_OK;
}

/* Relative Frobenius Nystrom error of the FPS-ordered landmark prefixes of
 * a dense SPSD matrix Km (m x m, column-major, overwritten):
 *   err(r) = ||Km - Km[:,I] Km[I,I]^+ Km[I,:]||_F / ||Km||_F,  I = ord[0..r)
 * (Eq. (2.1)/(2.2)).  The residual Km - Nystrom(I) is the Schur complement
 * after r steps of Cholesky elimination with pivots ord[0..r), so nested
 * prefixes follow from successive rank-one eliminations.  A pivot <= pivtol
 * is a landmark that is numerically dependent on the earlier ones; with the
 * pseudoinverse of Eq. (2.1) it adds nothing, and its (numerically zero)
 * residual row and column are set to zero.  errs[r-1] is written at every
 * checked r (r = step, 2*step, ... and r = m); returns the first checked r
 * with err(r) < tol, or m. */
int64_t ora_nystrom_scan(double *Km, int64_t m, const int32_t *ord, int64_t step,
                         double tol, double pivtol, double *errs)
{
    double f0 = 0.0;
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i) f0 += Km[i + j * m] * Km[i + j * m];
    f0 = sqrt(f0);
    double *c = (double *)malloc(sizeof(double) * (size_t)m);
    for (int64_t r = 1; r <= m; ++r) {
        int64_t pj = ord[r - 1];
        double piv = Km[pj + pj * m];
        if (piv > pivtol) {
            /* rank-one elimination: Km -= c c^T / piv with c = Km[:, pj] */
            for (int64_t i = 0; i < m; ++i) c[i] = Km[i + pj * m];
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < m; ++j) {
                double cj = c[j] / piv;
                for (int64_t i = 0; i < m; ++i) Km[i + j * m] -= c[i] * cj;
            }
        } else {
            for (int64_t i = 0; i < m; ++i) { Km[i + pj * m] = 0.0; Km[pj + i * m] = 0.0; }
        }
        if (r % step == 0 || r == m) {
            double f = 0.0;
            for (int64_t j = 0; j < m; ++j)
                for (int64_t i = 0; i < m; ++i) f += Km[i + j * m] * Km[i + j * m];
            double e = (f0 > 0.0) ? sqrt(f) / f0 : 0.0;
            if (errs) errs[r - 1] = e;
            if (e < tol) { free(c); return r; }
        }
    }
    free(c);
    return m;
}

/* Number of eigenvalues of a dense symmetric matrix A (m x m, column-major,
 * overwritten) that are > tau: Householder reduction to tridiagonal form
 * T = Q^T A Q (textbook, Golub & Van Loan Alg. 8.3.1), then Sylvester's law of
 * inertia on T - tau I through the Sturm/LDL^T recurrence
 *   q_1 = a_1 - tau,  q_i = (a_i - tau) - b_{i-1}^2 / q_{i-1},
 * counting the q_i > 0 (a zero q is replaced by a tiny negative value). */
int64_t ora_count_eigs_above(double *A, int64_t m, double tau)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)m);
    double *pw = (double *)malloc(sizeof(double) * (size_t)m);
    double *diag = (double *)malloc(sizeof(double) * (size_t)m);
    double *off = (double *)malloc(sizeof(double) * (size_t)(m > 1 ? m : 1));
    for (int64_t j = 0; j + 2 < m; ++j) {
        /* Householder vector annihilating A[j+2:, j] */
        double alpha2 = 0.0;
        for (int64_t i = j + 1; i < m; ++i) alpha2 += A[i + j * m] * A[i + j * m];
        double alpha = sqrt(alpha2);
        if (alpha == 0.0) continue;
        double x0 = A[j + 1 + j * m];
        double s = (x0 >= 0.0) ? -alpha : alpha; /* new sub-diagonal value */
        for (int64_t i = 0; i < m; ++i) v[i] = 0.0;
        v[j + 1] = x0 - s;
        for (int64_t i = j + 2; i < m; ++i) v[i] = A[i + j * m];
        double vnorm2 = 0.0;
        for (int64_t i = j + 1; i < m; ++i) vnorm2 += v[i] * v[i];
        if (vnorm2 == 0.0) continue;
        double beta = 2.0 / vnorm2;
        /* A <- H A H with H = I - beta v v^T on the trailing block j+1.. */
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < m; ++i) {
            double acc = 0.0;
            for (int64_t t = j + 1; t < m; ++t) acc += A[i + t * m] * v[t];
            pw[i] = beta * acc;
        }
        double vtp = 0.0;
        for (int64_t i = j + 1; i < m; ++i) vtp += v[i] * pw[i];
        double kk = 0.5 * beta * vtp;
        for (int64_t i = j + 1; i < m; ++i) pw[i] -= kk * v[i];
#pragma omp parallel for schedule(static)
        for (int64_t c = j + 1; c < m; ++c)
            for (int64_t i = j + 1; i < m; ++i)
                A[i + c * m] -= v[i] * pw[c] + pw[i] * v[c];
        A[j + 1 + j * m] = s;
        A[j + (j + 1) * m] = s;
        for (int64_t i = j + 2; i < m; ++i) { A[i + j * m] = 0.0; A[j + i * m] = 0.0; }
    }
    for (int64_t i = 0; i < m; ++i) diag[i] = A[i + i * m];
    for (int64_t i = 0; i + 1 < m; ++i) off[i] = A[i + 1 + i * m];
    int64_t count = 0;
    double q = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double qi = diag[i] - tau;
        if (i > 0) qi -= off[i - 1] * off[i - 1] / q;
        if (qi == 0.0) qi = -1e-300;
        if (qi > 0.0) ++count;
        q = qi;
    }
    free(v); free(pw); free(diag); free(off);
    return count;
}

/* Algorithm 4 with the readings: m = given subsample size; scaled copy
 * X_m * (m/n)^{1/d}; error = relative Frobenius norm; ranks scanned in steps
 * of 8 until the error is < 0.1 (giving r); k_est = floor(r n / m); when
 * k_est < kswitch the count of eigenvalues > 0.1 mu of K(X_m, X_m) built on
 * the UNSCALED subsample replaces it; the result is clamped to [1, min(kmax,n)].
 * info[0] = r, info[1] = k_est before the eigenvalue branch, info[2] = 1 if
 * the eigenvalue branch was taken, info[3] = the eigenvalue count. */
int ora_rank_estimate(const double *X, int64_t n, int d, double l, double mu,
                      int64_t m, int64_t kmax, int64_t kswitch, uint64_t seed,
                      int64_t *k_out, int64_t *info)
{
    if (n < 1 || d < 1 || m < 1 || m > n || kmax < 1) return ORA_EINVAL;
    int32_t *sub = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    double *Xm = (double *)malloc(sizeof(double) * (size_t)(m * d));
    double *Km = (double *)malloc(sizeof(double) * (size_t)(m * m));
    int32_t *ord = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    if (!sub || !Xm || !Km || !ord) { free(sub); free(Xm); free(Km); free(ord); return ORA_ENOMEM; }
    ora_subsample(n, m, seed, sub);
    double scale = pow((double)m / (double)n, 1.0 / (double)d);
    for (int64_t i = 0; i < m; ++i)
        for (int t = 0; t < d; ++t) Xm[i * d + t] = X[(int64_t)sub[i] * d + t] * scale;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        for (int64_t i = 0; i < m; ++i) Km[i + j * m] = ora_kernel(Xm + i * d, Xm + j * d, d, l);
    ora_fps(Xm, m, d, m, ord, NULL);
    int64_t r = ora_nystrom_scan(Km, m, ord, 8, 0.1, 1e-14 * (double)m, NULL);
    int64_t kest = (int64_t)floor((double)r * (double)n / (double)m);
    int64_t k = kest;
    int64_t eigbranch = 0, cnt = -1;
    if (kest < kswitch) {
        for (int64_t i = 0; i < m; ++i)
            for (int t = 0; t < d; ++t) Xm[i * d + t] = X[(int64_t)sub[i] * d + t];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < m; ++j)
            for (int64_t i = 0; i < m; ++i) Km[i + j * m] = ora_kernel(Xm + i * d, Xm + j * d, d, l);
        cnt = ora_count_eigs_above(Km, m, 0.1 * mu);
        k = cnt;
        eigbranch = 1;
    }
    int64_t cap = kmax < n ? kmax : n;
    if (k > cap) k = cap;
    if (k < 1) k = 1;
    *k_out = k;
    if (info) { info[0] = r; info[1] = kest; info[2] = eigbranch; info[3] = cnt; }
    free(sub); free(Xm); free(Km); free(ord);
    return ORA_OK;
}
