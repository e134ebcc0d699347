// C-ABI of libafn: preconditioner construction (Algorithm 2), application
// (Algorithm 3) and preconditioned CG (Algorithm 5, AFN branch).
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "afn_internal.h"
#include "kfun.h"

namespace afn {

// Rank estimation (Algorithm 4); defined in rank.hip.
afn_status uniform_landmarks(int64_t n, int k, uint64_t seed, int32_t *idx, hipStream_t s);
afn_status rank_estimate(const double *X, int64_t n, int d, double l, int kind, double mu, int m,
                         int kmax, uint64_t seed, hipStream_t s, afn_setup_info *info, int *k_out);

namespace {

struct Timer {
    hipEvent_t ev[8] = {};
    int used = 0;
    bool ok = true;
    Timer()
    {
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) ok = false;
    }
    ~Timer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void mark(int i, hipStream_t s)
    {
        if (ok) (void)hipEventRecord(ev[i], s);
    }
    double ms(int a, int b)
    {
        float t = 0.f;
        if (!ok || hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return -1.0;
        return t;
    }
};

// Workspace layout inside afn_handle::work (doubles).
struct WorkLayout {
    double *kmv, *dotp, *gemvp, *y1, *t, *u, *y1b, *y2, *x, *r, *z, *p, *q, *bp, *tmp, *rp, *sp, *sc;
};

int64_t work_doubles(int64_t n, int d, int k, int64_t nr, WorkLayout *L, double *base)
{
    int64_t off = 0;
    auto take = [&](int64_t cnt) {
        double *ptr = base ? base + off : nullptr;
        off += round_up(cnt > 0 ? cnt : 1, 32);
        return ptr;
    };
    WorkLayout w;
    int64_t gp = gemv_partials(k, n > k ? n : k);
    int64_t gp2 = gemv_partials(k, k);
    w.kmv = take(kmv_workspace_doubles(n, d));
    w.dotp = take(dot_partials(n));
    w.gemvp = take(gp > gp2 ? gp : gp2);
    w.y1 = take(k);
    w.t = take(nr);
    w.u = take(nr);
    w.y1b = take(k);
    w.y2 = take(k);
    w.x = take(n);
    w.r = take(n);
    w.z = take(n);
    w.p = take(n);
    w.q = take(n);
    w.bp = take(n);
    w.tmp = take(n);
    w.rp = take(n);
    w.sp = take(n);
    w.sc = take(16);
    if (L) *L = w;
    return off;
}

// Workspace of the FP32 inner solves (floats).
struct WorkLayout32 {
    float *kmv, *gemvp, *y1, *t, *u, *y1b, *y2, *r, *z, *p, *q, *e;
};

int64_t work32_floats(int64_t n, int d, int k, int64_t nr, WorkLayout32 *L, float *base)
{
    int64_t off = 0;
    auto take = [&](int64_t cnt) {
        float *ptr = base ? base + off : nullptr;
        off += round_up(cnt > 0 ? cnt : 1, 64);
        return ptr;
    };
    WorkLayout32 w;
    int64_t gp = gemv_partials(k, n > k ? n : k);
    int64_t gp2 = gemv_partials(k, k);
    w.kmv = take(2 * kmv_workspace_doubles(n, d));
    w.gemvp = take(gp > gp2 ? gp : gp2);
    w.y1 = take(k);
    w.t = take(nr);
    w.u = take(nr);
    w.y1b = take(k);
    w.y2 = take(k);
    w.r = take(n);
    w.z = take(n);
    w.p = take(n);
    w.q = take(n);
    w.e = take(n);
    if (L) *L = w;
    return off;
}

// The factors Algorithm 3 needs, in one precision.
template <typename T>
struct Factors {
    const T *Linv, *V, *gval, *tval;
};

// s = M^{-1} r in block order (landmarks first): Algorithm 3 with
// V = L^{-1} K12 and Linv = L^{-1}:
//   y1 = Linv r1 ; t = r2 - V^T y1 ; s2 = G^T (G t) ; s1 = Linv^T (y1 - V s2)
template <typename T>
afn_status apply_blockT(const afn_handle *h, const Factors<T> &f, const T *rp, T *sp, T *y1, T *tt,
                        T *u, T *y1b, T *gemvp, hipStream_t s)
{
    const int k = h->k;
    const int64_t nr = h->nr;
    if (k > 0) AFN_TRY(gemv_n(f.Linv, k, k, k, rp, (const T *)nullptr, T(1), y1, gemvp, s));
    if (nr > 0) {
        const T *t = rp + k;
        if (k > 0) {
            AFN_TRY(gemv_t(f.V, k, k, nr, y1, rp + k, T(-1), tt, s));
            t = tt;
        }
        // G in spatial row order (its gathers of t stay close); G^T in its
        // own order, where the contiguous value stream matters more
        AFN_TRY(spmv_g(h->cols, f.gval, nr, h->w, t, u, h->rorder, s));
        AFN_TRY(spmv_gt(h->tptr, h->trow, f.tval, nr, u, sp + k, nullptr, s));
    }
    if (k > 0) {
        const T *y = y1;
        if (nr > 0) {
            AFN_TRY(gemv_n(f.V, k, k, nr, sp + k, (const T *)y1, T(-1), y1b, gemvp, s));
            y = y1b;
        }
        AFN_TRY(gemv_t(f.Linv, k, k, k, y, (const T *)nullptr, T(1), sp, s));
    }
    return AFN_OK;
}

// s = M^{-1} r for the Nystrom preconditioner M = B B^T + mu I, B = W^T
// (block order): Sherman-Morrison-Woodbury with B^T B + mu I = Rg Rg^T,
//   y1 = W r ; y2 = Rg^{-T} Rg^{-1} y1 ; s = (r - W^T y2) / mu.
template <typename T>
afn_status apply_nysT(const afn_handle *h, const T *W, const T *Rginv, const T *rp, T *sp, T *y1, T *y1b,
                      T *y2, T *gemvp, hipStream_t s)
{
    const int k = h->k;
    const int64_t n = h->n;
    if (k > 0) {
        AFN_TRY(gemv_n(W, k, k, n, rp, (const T *)nullptr, T(1), y1, gemvp, s));
        AFN_TRY(gemv_n(Rginv, k, k, k, y1, (const T *)nullptr, T(1), y1b, gemvp, s));
        AFN_TRY(gemv_t(Rginv, k, k, k, y1b, (const T *)nullptr, T(1), y2, s));
        AFN_TRY(gemv_t(W, k, k, n, y2, rp, T(-1), sp, s));
    } else {
        AFN_HIP(hipMemcpyAsync(sp, rp, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
    }
    return scale_launch(sp, T(1.0 / h->mu), n, s);
}

afn_status apply_block(afn_handle *h, const double *rp, double *sp, const WorkLayout &w,
                       hipStream_t s)
{
    if (h->method == AFN_METHOD_NYSTROM)
        return apply_nysT<double>(h, h->W, h->Rginv, rp, sp, w.y1, w.y1b, w.y2, w.gemvp, s);
    Factors<double> f{h->Linv, h->V, h->gval, h->tval};
    return apply_blockT<double>(h, f, rp, sp, w.y1, w.t, w.u, w.y1b, w.gemvp, s);
}

afn_status apply_block32(afn_handle *h, const float *rp, float *sp, const WorkLayout32 &w,
                         hipStream_t s)
{
    if (h->method == AFN_METHOD_NYSTROM)
        return apply_nysT<float>(h, h->W32, h->Rginv32, rp, sp, w.y1, w.y1b, w.y2, w.gemvp, s);
    Factors<float> f{h->Linv32, h->V32, h->gval32, h->tval32};
    return apply_blockT<float>(h, f, rp, sp, w.y1, w.t, w.u, w.y1b, w.gemvp, s);
}

// (K + mu I) v on the handle's points, FP64
afn_status op_f64(afn_handle *h, const double *v, double *y, const WorkLayout &w, hipStream_t s,
                  hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr)
{
    if (h->Xs64)
        return kmv_packed_f64(h->Xs64, h->n, h->d, h->mu, h->kind, v, h->n, y, h->n, 1, w.kmv, s, e0, e1, h->kperm,
                              h->box64);
    return kmv_f64(h->Xp, h->n, h->d, h->l, h->mu, h->kind, v, h->n, y, h->n, 1, w.kmv, s, e0, e1);
}

afn_status check_flags(afn_handle *h, hipStream_t s)
{
    int f[6] = {0, 0, 0, 0, 0, 0};
    AFN_HIP(hipMemcpyAsync(f, h->flags, sizeof f, hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    if (f[0]) {
        set_error("afn_setup: X holds a non-finite coordinate");
        return AFN_EINVAL;
    }
    if (f[1]) {
        set_error("afn_setup: the landmark block K11 + shift I is not positive definite (pivot %d)",
                  f[1] - 1);
        return AFN_ENOTSPD;
    }
    if (f[2]) {
        set_error("afn_setup: an FSAI block of the Schur complement is not positive definite");
        return AFN_ENOTSPD;
    }
    if (f[3]) {
        set_error("afn_setup: landmark selection produced an invalid index");
        return AFN_EDEVICE;
    }
    if (f[5]) {
        set_error("afn_setup: B^T B + mu I of the Nystrom preconditioner is not positive definite");
        return AFN_ENOTSPD;
    }
    return AFN_OK;
}

// Nystrom factors (see afn_method): L = chol(K11 + nu I) with
// nu = eps ||K[:, S]||_F, W = [L^T | L^{-1} K12], Rginv = inverse of the lower
// Cholesky factor of W W^T + mu I.  Marks timer slots 3 .. 6.
afn_status nystrom_factors(afn_handle *h, DevArena &tmp, Timer &tm, hipStream_t s)
{
    const int64_t n = h->n, nr = h->nr;
    const int k = h->k, d = h->d;
    h->info.nu = 0.0;
    if (k == 0) {
        for (int m = 3; m <= 6; ++m) tm.mark(m, s);
        return AFN_OK;
    }
    const int64_t kk = (int64_t)k * k, knr = (int64_t)k * nr;
    AFN_TRY(h->arena.alloc_n(&h->L, kk));
    AFN_TRY(h->arena.alloc_n(&h->Dinv, dinv_doubles(k)));
    AFN_TRY(h->arena.alloc_n(&h->W, (int64_t)k * n));
    h->V = h->W + kk;
    AFN_TRY(fill_k11(h->Xp, k, d, h->l, h->kind, 0.0, h->L, k, s));    // lower triangle, unit diagonal
    if (nr > 0) AFN_TRY(fill_k12(h->Xp, n, k, d, h->l, h->kind, h->V, s));
    // ||K[:, S]||_F^2 = ||K12||_F^2 + 2 (lower triangle of K11)^2 - k
    double *dp = nullptr, *sc = nullptr;
    AFN_TRY(tmp.alloc_n(&dp, dot_partials(kk > knr ? kk : knr)));
    AFN_TRY(tmp.alloc_n(&sc, 2));
    AFN_HIP(hipMemsetAsync(sc, 0, 2 * sizeof(double), s));
    AFN_TRY(dot(h->L, kk, h->L, kk, kk, 1, sc, dp, s));
    if (nr > 0) AFN_TRY(dot(h->V, knr, h->V, knr, knr, 1, sc + 1, dp, s));
    double hs[2] = {0.0, 0.0};
    AFN_HIP(hipMemcpyAsync(hs, sc, sizeof hs, hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    const double f2 = 2.0 * hs[0] - (double)k + hs[1];
    const double nu = DBL_EPSILON * std::sqrt(f2 > 0.0 ? f2 : 0.0);
    h->info.nu = nu;
    AFN_TRY(add_diagonal(h->L, k, k, nu, s));
    AFN_TRY(cholesky(h->L, k, k, h->flags + 1, s));
    AFN_TRY(diag_inverses(h->L, k, h->Dinv, s));
    tm.mark(3, s);
    tm.mark(4, s);
    if (nr > 0) AFN_TRY(trsm_lower(h->L, h->Dinv, k, h->V, nr, s));
    AFN_TRY(transpose_square(h->L, k, k, h->W, k, s));
    tm.mark(5, s);
    // W W^T + mu I by 64-column blocks on FP64 MFMA, its factor and inverse
    double *G = nullptr, *Dg = nullptr, *part = nullptr;
    AFN_TRY(tmp.alloc_n(&G, kk));
    AFN_TRY(tmp.alloc_n(&Dg, dinv_doubles(k)));
    AFN_TRY(tmp.alloc_n(&part, gemm_part_elems(k, n)));
    for (int c0 = 0; c0 < k; c0 += 64) {
        const int R = k - c0 < 64 ? k - c0 : 64;
        AFN_TRY(gemm_rows<double>(h->W, 1, k, k, n, h->W + c0, k, R, nullptr, 1.0, G + c0, k, part, s));
    }
    AFN_TRY(zero_upper(G, k, k, s));
    AFN_TRY(add_diagonal(G, k, k, h->mu, s));
    AFN_TRY(cholesky(G, k, k, h->flags + 5, s));
    AFN_TRY(diag_inverses(G, k, Dg, s));
    AFN_TRY(h->arena.alloc_n(&h->Rginv, kk));
    AFN_TRY(identity(h->Rginv, k, s));
    AFN_TRY(trsm_lower(G, Dg, k, h->Rginv, k, s));
    tm.mark(6, s);
    return AFN_OK;
}

afn_status setup_impl(const double *X, int64_t n, int d, double l, double mu, const afn_params *prm,
                      hipStream_t s, afn_handle *h)
{
    Timer tm;
    tm.mark(0, s);
    AFN_HIP(hipGetDevice(&h->device));
    h->n = n;
    h->d = d;
    h->l = l;
    h->mu = mu;
    h->kind = prm->kernel;
    h->w = prm->w;
    AFN_TRY(h->arena.alloc_n(&h->flags, 16));
    AFN_HIP(hipMemsetAsync(h->flags, 0, sizeof(int) * 16, s));
    AFN_TRY(finite_launch(X, n * d, h->flags + 0, s));
    // landmark count
    h->info.rank_r = -1;
    h->info.rank_k_est = -1;
    h->info.rank_eig_branch = 0;
    h->info.rank_eig_count = -1;
    int k = prm->k;
    if (k < 0) {
        const int m = prm->m > 0 ? (int)(prm->m < n ? prm->m : n) : (int)(n < 2000 ? n : 2000);
        const int kmax = prm->k_max > 0 ? prm->k_max : 2000;
        AFN_TRY(rank_estimate(X, n, d, l, h->kind, mu, m, kmax, prm->seed, s, &h->info, &k));
    }
    tm.mark(1, s);
    // Algorithm 5: the rank decides between AFN and Nystrom
    h->method = prm->method;
    if (h->method == AFN_METHOD_AUTO) {
        const int64_t rank = prm->k >= 0 ? (int64_t)prm->k
                                         : (h->info.rank_eig_branch ? (int64_t)h->info.rank_eig_count
                                                                    : h->info.rank_k_est);
        h->method = rank < 2000 ? AFN_METHOD_NYSTROM : AFN_METHOD_AFN;
    }
    if (h->method == AFN_METHOD_NYSTROM && !(mu > 0.0)) {
        set_error("afn_setup: the Nystrom preconditioner needs mu > 0");
        return AFN_EINVAL;
    }
    h->k = k;
    h->nr = n - k;
    const int64_t nr = h->nr;
    // FPS and the block order
    DevArena tmp;
    struct TmpGuard {
        DevArena &a;
        ~TmpGuard() { a.release(); }
    } guard{tmp};
    AFN_TRY(h->arena.alloc_n(&h->perm, n));
    int32_t *idx = nullptr;
    void *fws = nullptr;
    int *sel = nullptr;
    AFN_TRY(tmp.alloc_n(&idx, k));
    AFN_TRY(tmp.alloc(&fws, fps_workspace_bytes(n)));
    AFN_TRY(tmp.alloc_n(&sel, n));
    // landmarks (Algorithm 2): FPS in low dimension, uniform sampling above d = 10
    const int lm = prm->landmarks == AFN_LANDMARKS_AUTO ? (d <= 10 ? AFN_LANDMARKS_FPS : AFN_LANDMARKS_UNIFORM)
                                                        : prm->landmarks;
    h->info.landmarks = lm;
    if (lm == AFN_LANDMARKS_UNIFORM)
        AFN_TRY(uniform_landmarks(n, k, prm->seed + 1, idx, s));
    else
        AFN_TRY(fps(X, n, d, k, idx, nullptr, fws, s, h->flags + 3));
    AFN_TRY(landmark_permutation(idx, k, n, h->perm, sel, s));
    AFN_TRY(h->arena.alloc_n(&h->Xp, n * d));
    AFN_TRY(gather_points(X, h->perm, n, d, h->Xp, s));
    tm.mark(2, s);
    if (h->method == AFN_METHOD_NYSTROM) {
        AFN_TRY(nystrom_factors(h, tmp, tm, s));
    } else {
    // L = chol(K11 + mu I), Linv, V = L^{-1} K12
    if (k > 0) {
        AFN_TRY(h->arena.alloc_n(&h->L, (int64_t)k * k));
        AFN_TRY(h->arena.alloc_n(&h->Linv, (int64_t)k * k));
        AFN_TRY(h->arena.alloc_n(&h->Dinv, dinv_doubles(k)));
        AFN_TRY(fill_k11(h->Xp, k, d, l, h->kind, mu, h->L, k, s));
        AFN_TRY(cholesky(h->L, k, k, h->flags + 1, s));
        AFN_TRY(diag_inverses(h->L, k, h->Dinv, s));
        AFN_TRY(identity(h->Linv, k, s));
        AFN_TRY(trsm_lower(h->L, h->Dinv, k, h->Linv, k, s));
    }
    tm.mark(3, s);
    // spatial order of the non-landmark points: tiles for the pattern search,
    // the row order of the FSAI gathers and of the G / G^T products (d <= 10)
    int32_t *rorder = nullptr;
    if (nr > 0 && d <= 10) {
        void *ows = nullptr;
        AFN_TRY(h->arena.alloc_n(&h->rorder, nr));
        rorder = h->rorder;
        AFN_TRY(tmp.alloc(&ows, spatial_order_work_bytes(nr, d)));
        AFN_TRY(spatial_order(h->Xp + (int64_t)k * d, nr, d, rorder, ows, s));
    }
    if (nr > 0) {
        void *kws = nullptr;
        AFN_TRY(h->arena.alloc_n(&h->cols, nr * h->w));
        AFN_TRY(tmp.alloc(&kws, knn_work_bytes(nr, d)));
        AFN_TRY(knn_pattern_ordered(h->Xp + (int64_t)k * d, nr, d, h->w, rorder, kws, h->cols, s));
    }
    tm.mark(4, s);
    if (k > 0 && nr > 0) {
        AFN_TRY(h->arena.alloc_n(&h->V, (int64_t)k * nr));
        AFN_TRY(fill_k12(h->Xp, n, k, d, l, h->kind, h->V, s));
        AFN_TRY(trsm_lower(h->L, h->Dinv, k, h->V, nr, s));
    }
    tm.mark(5, s);
    if (nr > 0) {
        AFN_TRY(h->arena.alloc_n(&h->gval, nr * h->w));
        // above d = 10 the pattern neighbourhoods share few columns, so each
        // row's columns of V are recomputed in batches rather than gathered
        // (AFN_FSAI_RECOMPUTE=0/1 overrides the choice)
        const char *fr = std::getenv("AFN_FSAI_RECOMPUTE");
        const bool recompute = fr && (fr[0] == '0' || fr[0] == '1') ? fr[0] == '1' : d > 10;
        if (recompute) {
            double *fb = nullptr;
            AFN_TRY(tmp.alloc_n(&fb, fsai_batch_doubles(k, h->w)));
            AFN_TRY(fsai_rows_batched(h->Xp, n, k, d, l, h->kind, mu, h->Linv, h->cols, h->w, h->gval,
                                      h->flags + 2, fb, s));
        } else {
            if (!rorder) {
                void *ows = nullptr;
                AFN_TRY(tmp.alloc_n(&rorder, nr));
                AFN_TRY(tmp.alloc(&ows, spatial_order_work_bytes(nr, d)));
                AFN_TRY(spatial_order(h->Xp + (int64_t)k * d, nr, d, rorder, ows, s));
            }
            AFN_TRY(fsai_rows(h->Xp, n, k, d, l, h->kind, mu, h->V, h->cols, h->w, h->gval, h->flags + 2, rorder, s));
        }
        AFN_TRY(h->arena.alloc_n(&h->tptr, nr + 1));
        AFN_TRY(h->arena.alloc_n(&h->trow, nr * h->w));
        AFN_TRY(h->arena.alloc_n(&h->tval, nr * h->w));
        void *tws = nullptr;
        AFN_TRY(tmp.alloc(&tws, fsai_transpose_work_bytes(nr, h->w)));
        AFN_TRY(fsai_transpose(h->cols, h->gval, nr, h->w, h->tptr, h->trow, h->tval, tws, s));
    }
    tm.mark(6, s);
    }
    // points packed for the symmetric tile kernel; FP32 copies for mixed solves
    h->precision = prm->precision;
    if (d <= 8) {
        // spatial order of all points for the tile kernels: far-apart tile
        // pairs (kernel values below 2^-cut) are skipped
        void *kws = nullptr;
        AFN_TRY(h->arena.alloc_n(&h->kperm, n));
        AFN_TRY(tmp.alloc(&kws, spatial_order_work_bytes(n, d)));
        AFN_TRY(spatial_order(h->Xp, n, d, h->kperm, kws, s));
        AFN_TRY(h->arena.alloc_n(&h->Xs64, kmv_packed_doubles(n, d)));
        AFN_TRY(kmv_pack(h->Xp, n, d, l, h->kind, h->Xs64, false, s, h->kperm));
        AFN_TRY(h->arena.alloc_n(&h->box64, kmv_box_count(n, d)));
        AFN_TRY(kmv_boxes(h->Xs64, n, d, false, h->box64, s));
        unsigned long long *cnt = nullptr, hc[6] = {0, 0, 0, 0, 0, 0};
        AFN_TRY(tmp.alloc_n(&cnt, 6));
        AFN_TRY(kmv_kept_fraction(h->box64, n, d, kernel_cut_t(h->kind, kCullF64), cnt, s));
        AFN_TRY(kmv_kept_fraction(h->box64, n, d, kernel_cut_t(h->kind, kCullF32), cnt + 2, s));
        AFN_TRY(kmv_kept_fraction(h->box64, n, d, kernel_cut_t(h->kind, kFarF64), cnt + 4, s));
        AFN_HIP(hipMemcpyAsync(hc, cnt, sizeof hc, hipMemcpyDeviceToHost, s));
        AFN_HIP(hipStreamSynchronize(s));
        h->info.kmv_kept_f64 = hc[1] ? (double)hc[0] / (double)hc[1] : 1.0;
        h->info.kmv_kept_f32 = hc[3] ? (double)hc[2] / (double)hc[3] : 1.0;
        h->info.kmv_far_f64 = (d <= 4 && hc[1]) ? (double)(hc[0] - hc[4]) / (double)hc[1] : 0.0;
    } else {
        h->info.kmv_kept_f64 = h->info.kmv_kept_f32 = 1.0;
        h->info.kmv_far_f64 = 0.0;
    }
    if (h->precision == AFN_FP32) {
        AFN_TRY(h->arena.alloc_n(&h->Xs32, kmv_packed_doubles(n, d)));
        AFN_TRY(kmv_pack(h->Xp, n, d, l, h->kind, h->Xs32, true, s, h->kperm));
        AFN_TRY(h->arena.alloc_n(&h->box32, kmv_box_count(n, d)));
        AFN_TRY(kmv_boxes(h->Xs32, n, d, true, h->box32, s));
        if (h->method == AFN_METHOD_NYSTROM) {
            if (k > 0) {
                AFN_TRY(h->arena.alloc_n(&h->W32, (int64_t)k * n));
                AFN_TRY(to_f32_launch(h->W, h->W32, (int64_t)k * n, s));
                AFN_TRY(h->arena.alloc_n(&h->Rginv32, (int64_t)k * k));
                AFN_TRY(to_f32_launch(h->Rginv, h->Rginv32, (int64_t)k * k, s));
            }
        }
        if (h->method != AFN_METHOD_NYSTROM && k > 0) {
            AFN_TRY(h->arena.alloc_n(&h->Linv32, (int64_t)k * k));
            AFN_TRY(to_f32_launch(h->Linv, h->Linv32, (int64_t)k * k, s));
        }
        if (h->method != AFN_METHOD_NYSTROM && k > 0 && nr > 0) {
            AFN_TRY(h->arena.alloc_n(&h->V32, (int64_t)k * nr));
            AFN_TRY(to_f32_launch(h->V, h->V32, (int64_t)k * nr, s));
        }
        if (h->method != AFN_METHOD_NYSTROM && nr > 0) {
            AFN_TRY(h->arena.alloc_n(&h->gval32, nr * h->w));
            AFN_TRY(h->arena.alloc_n(&h->tval32, nr * h->w));
            AFN_TRY(to_f32_launch(h->gval, h->gval32, nr * h->w, s));
            AFN_TRY(to_f32_launch(h->tval, h->tval32, nr * h->w, s));
        }
        AFN_TRY(h->arena.alloc_n(&h->work32, work32_floats(n, d, k, nr, nullptr, nullptr)));
    }
    // workspace for apply / PCG
    h->work_doubles = work_doubles(n, d, k, nr, nullptr, nullptr);
    AFN_TRY(h->arena.alloc_n(&h->work, h->work_doubles));
    AFN_HIP(hipHostMalloc((void **)&h->host_sc, 16 * sizeof(double), hipHostMallocDefault));
    AFN_HIP(hipEventCreate(&h->kmv_ev[0]));
    AFN_HIP(hipEventCreate(&h->kmv_ev[1]));
    AFN_HIP(hipEventCreateWithFlags(&h->chk_ev, hipEventDisableTiming));
    AFN_TRY(check_flags(h, s));
    h->nnz = 0;
    if (nr > 0 && h->tptr) AFN_HIP(hipMemcpy(&h->nnz, h->tptr + nr, sizeof(int64_t), hipMemcpyDeviceToHost));
    tm.mark(7, s);
    AFN_HIP(hipStreamSynchronize(s));
    afn_setup_info &inf = h->info;
    inf.n = n;
    inf.d = d;
    inf.k = k;
    inf.w = h->w;
    inf.nnz_g = h->nnz;
    inf.ms_rank = tm.ms(0, 1);
    inf.ms_fps = tm.ms(1, 2);
    inf.ms_chol = tm.ms(2, 3);
    inf.ms_knn = tm.ms(3, 4);
    inf.ms_v = tm.ms(4, 5);
    inf.ms_fsai = tm.ms(5, 6);
    inf.ms_total = tm.ms(0, 7);
    inf.method = h->method;
    return AFN_OK;
}

// FP64 PCG iterations from the state x = w.x, r = w.r = b - (K + mu I) x (block
// order): stops when ||r|| <= tol * bnorm (recurrence residual), on a
// breakdown, or after maxit products.
afn_status pcg64_iterate(afn_handle *h, double bnorm, double tol, int maxit, const WorkLayout &w,
                         hipStream_t s, int *iters, double *relres, double *ms_kmv, int *n_kmv)
{
    const int64_t n = h->n;
    double *sc = w.sc;
    double *hs = h->host_sc;
    AFN_TRY(apply_block(h, w.r, w.z, w, s));
    AFN_HIP(hipMemcpyAsync(w.p, w.z, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AFN_TRY(dot(w.r, n, w.z, n, n, 1, sc + 0, w.dotp, s));
    *iters = 0;
    for (int it = 0; it < maxit; ++it) {
        AFN_TRY(op_f64(h, w.p, w.q, w, s, h->kmv_ev[0], h->kmv_ev[1]));
        AFN_TRY(dot_pcg(w.p, w.q, n, sc, kPcgAlpha, w.dotp, s));
        AFN_TRY(pcg_xr_launch(w.x, w.r, w.p, w.q, sc, n, w.dotp, sc + 2, s));
        AFN_HIP(hipMemcpyAsync(hs + 1, sc + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        AFN_HIP(hipEventRecord(h->chk_ev, s));
        // z = M^{-1} r and r'z go on the stream before the host reads the
        // residual (x, r and p stay as they are, so a check that ends the
        // loop discards only z): the device never waits for the host
        if (it + 1 < maxit) {
            AFN_TRY(apply_block(h, w.r, w.z, w, s));
            AFN_TRY(dot_pcg(w.r, w.z, n, sc, kPcgBeta, w.dotp, s));
        }
        AFN_HIP(hipEventSynchronize(h->chk_ev));
        {
            float t = 0.f;
            if (hipEventElapsedTime(&t, h->kmv_ev[0], h->kmv_ev[1]) == hipSuccess) {
                *ms_kmv += t;
                *n_kmv += 1;
            }
        }
        *iters = it + 1;
        const double pq = hs[1];
        const double rel = std::sqrt(hs[2]) / bnorm;
        *relres = rel;
        if (!(pq > 0.0) || !(rel == rel)) {
            set_error("afn_pcg_solve: breakdown at iteration %d (p'Ap = %g)", it + 1, pq);
            return AFN_EBREAKDOWN;
        }
        if (rel <= tol) return AFN_OK;
        AFN_TRY(pcg_p_launch(w.p, w.z, sc, n, s));
    }
    return AFN_ENOCONV;
}

// ||b - (K + mu I) x|| / bnorm in FP64 (block order; w.tmp clobbered).
afn_status true_relres(afn_handle *h, double bnorm, const WorkLayout &w, hipStream_t s, double *out)
{
    const int64_t n = h->n;
    AFN_TRY(op_f64(h, w.x, w.q, w, s));
    AFN_TRY(sub_launch(w.bp, w.q, w.tmp, n, s));
    AFN_TRY(dot(w.tmp, n, w.tmp, n, n, 1, w.sc + 7, w.dotp, s));
    AFN_HIP(hipMemcpyAsync(h->host_sc + 7, w.sc + 7, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    *out = std::sqrt(h->host_sc[7]) / bnorm;
    return AFN_OK;
}

afn_status pcg_one(afn_handle *h, const double *b, double *xout, double tol, int maxit,
                   const WorkLayout &w, hipStream_t s, int *iters, double *relres,
                   double *relres_true, int *converged, double *ms_kmv, int *n_kmv)
{
    const int64_t n = h->n;
    double *sc = w.sc;
    double *hs = h->host_sc;
    AFN_TRY(permute_gather(b, n, w.bp, n, h->perm, n, 1, s));
    AFN_TRY(dot(w.bp, n, w.bp, n, n, 1, sc + 6, w.dotp, s));
    AFN_HIP(hipMemsetAsync(w.x, 0, sizeof(double) * n, s));
    AFN_HIP(hipMemcpyAsync(w.r, w.bp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AFN_HIP(hipMemcpyAsync(hs + 6, sc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(hs[6]);
    *iters = 0;
    *relres = 0.0;
    *relres_true = 0.0;
    *converged = 1;
    if (!(bnorm > 0.0)) {
        if (!(bnorm == 0.0)) {
            set_error("afn_pcg_solve: right-hand side holds a non-finite value");
            *converged = 0;
            *relres = NAN;
            AFN_TRY(permute_scatter(w.x, n, xout, n, h->perm, n, 1, s));
            return AFN_EBREAKDOWN;
        }
        AFN_TRY(permute_scatter(w.x, n, xout, n, h->perm, n, 1, s));
        return AFN_OK;
    }
    *converged = 0;
    *relres = 1.0;
    const afn_status status = pcg64_iterate(h, bnorm, tol, maxit, w, s, iters, relres, ms_kmv, n_kmv);
    *converged = status == AFN_OK ? 1 : 0;
    AFN_TRY(true_relres(h, bnorm, w, s, relres_true));
    AFN_TRY(permute_scatter(w.x, n, xout, n, h->perm, n, 1, s));
    AFN_HIP(hipStreamSynchronize(s));
    if (status == AFN_ENOCONV)
        set_error("afn_pcg_solve: no convergence in %d iterations (relres %g)", maxit, *relres);
    return status;
}

// Inner PCG in FP32 (operator, preconditioner and vectors), FP64 scalars:
// solve (K + mu I) e = r0 to relative recurrence residual tol_in.  r0 in w32.r
// on entry (overwritten), e in w32.e on exit.  sc: 8 device scalar slots.
afn_status pcg_inner32(afn_handle *h, double r0norm, double tol_in, int maxit, const WorkLayout32 &w,
                       double *dotp, double *sc, hipStream_t s, int *iters, double *rel_out,
                       double *ms_kmv, int *n_kmv)
{
    const int64_t n = h->n;
    double *hs = h->host_sc;
    AFN_HIP(hipMemsetAsync(w.e, 0, sizeof(float) * n, s));
    AFN_TRY(apply_block32(h, w.r, w.z, w, s));
    AFN_HIP(hipMemcpyAsync(w.p, w.z, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    AFN_TRY(dot(w.r, n, w.z, n, n, 1, sc + 0, dotp, s));
    *iters = 0;
    *rel_out = 1.0;
    for (int it = 0; it < maxit; ++it) {
        AFN_TRY(kmv_packed_f32(h->Xs32, n, h->d, h->mu, h->kind, w.p, n, w.q, n, 1, w.kmv, s, h->kmv_ev[0],
                               h->kmv_ev[1], h->kperm, h->box32));
        AFN_TRY(dot_pcg(w.p, w.q, n, sc, kPcgAlpha, dotp, s));
        AFN_TRY(pcg_xr_launch(w.e, w.r, w.p, w.q, sc, n, dotp, sc + 2, s));
        AFN_HIP(hipMemcpyAsync(hs + 9, sc + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        AFN_HIP(hipEventRecord(h->chk_ev, s));
        // the next z = M^{-1} r and r'z are queued before the check (as in
        // the FP64 loop)
        if (it + 1 < maxit) {
            AFN_TRY(apply_block32(h, w.r, w.z, w, s));
            AFN_TRY(dot_pcg(w.r, w.z, n, sc, kPcgBeta, dotp, s));
        }
        AFN_HIP(hipEventSynchronize(h->chk_ev));
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->kmv_ev[0], h->kmv_ev[1]) == hipSuccess) {
            *ms_kmv += t;
            *n_kmv += 1;
        }
        *iters = it + 1;
        const double pq = hs[9];
        const double rel = std::sqrt(hs[10]) / r0norm;
        *rel_out = rel;
        if (!(pq > 0.0) || !(rel == rel)) {
            set_error("afn_pcg_solve: inner FP32 breakdown at iteration %d (p'Ap = %g)", it + 1, pq);
            return AFN_EBREAKDOWN;
        }
        if (rel <= tol_in) break;
        AFN_TRY(pcg_p_launch(w.p, w.z, sc, n, s));
    }
    return AFN_OK;
}

// Iterative refinement: x_0 = 0; r = b - (K + mu I) x in FP64; correction
// from the FP32 inner PCG on r / ||r||; stop when ||r|| / ||b|| <= tol.
afn_status pcg_refine(afn_handle *h, const double *b, double *xout, double tol, int maxit,
                      const WorkLayout &w, const WorkLayout32 &w32, hipStream_t s, int *iters,
                      int *outer, int *iters64, double *relres, double *relres_true, int *converged,
                      double *ms_kmv, int *n_kmv)
{
    *iters64 = 0;
    const int64_t n = h->n;
    double *sc = w.sc;
    double *hs = h->host_sc;
    AFN_TRY(permute_gather(b, n, w.bp, n, h->perm, n, 1, s));
    AFN_HIP(hipMemsetAsync(w.x, 0, sizeof(double) * n, s));
    AFN_HIP(hipMemcpyAsync(w.r, w.bp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AFN_TRY(dot(w.bp, n, w.bp, n, n, 1, sc + 6, w.dotp, s));
    AFN_HIP(hipMemcpyAsync(hs + 6, sc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(hs[6]);
    *iters = 0;
    *outer = 0;
    *relres = 0.0;
    *relres_true = 0.0;
    *converged = 1;
    if (!(bnorm > 0.0)) {
        AFN_TRY(permute_scatter(w.x, n, xout, n, h->perm, n, 1, s));
        if (!(bnorm == 0.0)) {
            set_error("afn_pcg_solve: right-hand side holds a non-finite value");
            *converged = 0;
            *relres = NAN;
            return AFN_EBREAKDOWN;
        }
        return AFN_OK;
    }
    *converged = 0;
    afn_status status = AFN_ENOCONV;
    double prev = INFINITY;
    const int max_outer = 40;
    bool fallback = false;     // the FP32 corrections stopped helping: finish in FP64
    for (int o = 0;; ++o) {
        AFN_TRY(dot(w.r, n, w.r, n, n, 1, sc + 7, w.dotp, s));
        AFN_HIP(hipMemcpyAsync(hs + 7, sc + 7, sizeof(double), hipMemcpyDeviceToHost, s));
        AFN_HIP(hipStreamSynchronize(s));
        double rnorm = std::sqrt(hs[7]);
        double rel = rnorm / bnorm;
        if (o > 0 && !(rel <= prev)) {
            // the last FP32 correction made things worse: take it back (x and
            // its residual were kept in rp / sp) and finish in FP64
            AFN_HIP(hipMemcpyAsync(w.x, w.rp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            AFN_HIP(hipMemcpyAsync(w.r, w.sp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            rel = prev;
            rnorm = prev * bnorm;
            fallback = true;
        }
        *relres = rel;
        *relres_true = rel;
        if (!(rel == rel)) {
            set_error("afn_pcg_solve: refinement produced a non-finite residual");
            status = AFN_EBREAKDOWN;
            break;
        }
        if (rel <= tol) {
            status = AFN_OK;
            *converged = 1;
            break;
        }
        if (o >= max_outer || (o >= 3 && rel > 0.5 * prev) || *iters >= maxit * 4) fallback = true;
        if (fallback) {
            // textbook FP64 PCG from the current x and its FP64 residual
            int it64 = 0;
            double rel64 = rel;
            const afn_status st64 =
                pcg64_iterate(h, bnorm, tol, maxit, w, s, &it64, &rel64, ms_kmv, n_kmv);
            *iters64 = it64;
            *outer = o + 1;
            double rt = 0.0;
            AFN_TRY(true_relres(h, bnorm, w, s, &rt));
            *relres = rel64;
            *relres_true = rt;
            if (st64 == AFN_OK) {
                status = AFN_OK;
                *converged = 1;
            } else {
                status = st64;
                if (st64 == AFN_ENOCONV)
                    set_error("afn_pcg_solve: no convergence (FP64 after refinement, relres %g)", rel64);
            }
            break;
        }
        prev = rel;
        AFN_HIP(hipMemcpyAsync(w.rp, w.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        AFN_HIP(hipMemcpyAsync(w.sp, w.r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        // inner tolerance: what this step needs, but at least 3e-2 of its
        // start: the FP32 operator and apply bound what one step gains in
        // FP64, and a tighter inner solve spends iterations that the next
        // refinement step does more cheaply
        double tol_in = 0.5 * tol / rel;
        tol_in = tol_in > 3e-2 ? tol_in : 3e-2;
        tol_in = tol_in < 0.5 ? tol_in : 0.5;
        AFN_TRY(to_f32_scaled_launch(w.r, 1.0 / rnorm, w32.r, n, s));
        int it = 0;
        double rel_in = 0;
        afn_status st = pcg_inner32(h, 1.0, tol_in, maxit, w32, w.dotp, sc + 8, s, &it, &rel_in,
                                    ms_kmv, n_kmv);
        *iters += it;
        *outer = o + 1;
        if (st == AFN_EBREAKDOWN) {
            // the FP32 operator or apply lost definiteness: redo this step in FP64
            fallback = true;
            --o;
            continue;
        }
        if (st != AFN_OK) {
            status = st;
            break;
        }
        AFN_TRY(axpy_f32_into_f64_launch(rnorm, w32.e, w.x, n, s));
        AFN_TRY(op_f64(h, w.x, w.q, w, s));
        AFN_TRY(sub_launch(w.bp, w.q, w.r, n, s));
    }
    AFN_TRY(permute_scatter(w.x, n, xout, n, h->perm, n, 1, s));
    AFN_HIP(hipStreamSynchronize(s));
    return status;
}

}  // namespace
}  // namespace afn

using namespace afn;

extern "C" {

afn_status afn_setup(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                     const afn_params *prm, void *stream, afn_handle **out)
{
    clear_error();
    if (!out) {
        set_error("afn_setup: out is NULL");
        return AFN_EINVAL;
    }
    *out = nullptr;
    if (!X_dev || !prm || n < 1 || n > INT32_MAX - 1 || d < 1 || d > kMaxD || !(l > 0) ||
        !std::isfinite(l) || !(mu >= 0) || !std::isfinite(mu) || prm->k < -1 || prm->k > n ||
        prm->w < 1 || prm->w > kMaxW || prm->method < AFN_METHOD_AFN || prm->method > AFN_METHOD_AUTO ||
        prm->landmarks < AFN_LANDMARKS_AUTO || prm->landmarks > AFN_LANDMARKS_UNIFORM ||
        (prm->kernel != AFN_KERNEL_GAUSSIAN && prm->kernel != AFN_KERNEL_MATERN32) ||
        (prm->precision != AFN_FP64 && prm->precision != AFN_FP32) ||
        (prm->precision == AFN_FP32 && d > 8)) {
        set_error("afn_setup: invalid argument (n=%lld d=%d l=%g mu=%g k=%d w=%d)", (long long)n, d,
                  l, mu, prm ? prm->k : 0, prm ? prm->w : 0);
        return AFN_EINVAL;
    }
    std::unique_ptr<afn_handle> h(new afn_handle());
    afn_status st = setup_impl(X_dev, n, d, l, mu, prm, (hipStream_t)stream, h.get());
    if (st != AFN_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        if (h->host_sc) (void)hipHostFree(h->host_sc);
        for (auto &e : h->kmv_ev)
            if (e) (void)hipEventDestroy(e);
        if (h->chk_ev) (void)hipEventDestroy(h->chk_ev);
        h->arena.release();
        return st;
    }
    *out = h.release();
    return AFN_OK;
}

afn_status afn_apply(afn_handle *h, const double *r_dev, double *z_dev, int32_t nrhs, int64_t ld,
                     void *stream)
{
    clear_error();
    if (!h || !r_dev || !z_dev || nrhs < 1 || ld < h->n) {
        set_error("afn_apply: invalid argument");
        return AFN_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    WorkLayout w;
    work_doubles(h->n, h->d, h->k, h->nr, &w, h->work);
    for (int c = 0; c < nrhs; ++c) {
        AFN_TRY(permute_gather(r_dev + c * ld, h->n, w.rp, h->n, h->perm, h->n, 1, s));
        AFN_TRY(apply_block(h, w.rp, w.sp, w, s));
        AFN_TRY(permute_scatter(w.sp, h->n, z_dev + c * ld, h->n, h->perm, h->n, 1, s));
    }
    return AFN_OK;
}

afn_status afn_pcg_solve(afn_handle *h, const double *b_dev, double *x_dev, int32_t nrhs,
                         int64_t ld, double tol, int32_t maxit, afn_solve_info *info,
                         void *stream)
{
    clear_error();
    if (!h || !b_dev || !x_dev || nrhs < 1 || ld < h->n || !(tol > 0) || maxit < 1) {
        set_error("afn_pcg_solve: invalid argument");
        return AFN_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    WorkLayout w;
    work_doubles(h->n, h->d, h->k, h->nr, &w, h->work);
    WorkLayout32 w32{};
    if (h->precision == AFN_FP32) work32_floats(h->n, h->d, h->k, h->nr, &w32, h->work32);
    Timer tm;
    tm.mark(0, s);
    int outer_max = 0, it64_max = 0;
    afn_status worst = AFN_OK;
    int it_max = 0, conv_all = 1, n_kmv = 0;
    double ms_kmv = 0.0;
    double rel_max = 0.0, true_max = 0.0;
    // columns still to solve one at a time (all of them outside the block path)
    std::vector<int> single;
    if (nrhs >= 2 && h->precision == AFN_FP32 && h->d <= 8) {
        std::vector<int> col_ok(64);
        for (int c0 = 0; c0 < nrhs; c0 += 64) {
            const int Rc = nrhs - c0 < 64 ? nrhs - c0 : 64;
            int it = 0, outer = 0, conv = 0;
            double rel = 0.0;
            afn_status st = block_refine_solve(h, b_dev + c0 * ld, ld, x_dev + c0 * ld, Rc, tol, maxit,
                                               s, &it, &outer, &rel, &conv, col_ok.data());
            if (st != AFN_OK && st != AFN_ENOCONV && st != AFN_EBREAKDOWN && st != AFN_ESTAGNATION)
                return st;
            it_max = it > it_max ? it : it_max;
            outer_max = outer > outer_max ? outer : outer_max;
            for (int c = 0; c < Rc; ++c) {
                if (col_ok[c]) continue;
                if (st == AFN_OK) continue;
                single.push_back(c0 + c);   // re-solved below (refinement with FP64 fallback)
            }
            if (st == AFN_OK) rel_max = rel > rel_max || rel != rel ? rel : rel_max;
            else
                for (int c = 0; c < Rc; ++c)
                    if (col_ok[c]) rel_max = rel_max > tol ? rel_max : tol;
        }
        true_max = rel_max;
    } else {
        for (int c = 0; c < nrhs; ++c) single.push_back(c);
    }
    for (const int c : single) {
        int it = 0, conv = 0, outer = 0, it64 = 0;
        double rel = 0, rt = 0;
        afn_status st =
            h->precision == AFN_FP32
                ? pcg_refine(h, b_dev + c * ld, x_dev + c * ld, tol, maxit, w, w32, s, &it, &outer,
                             &it64, &rel, &rt, &conv, &ms_kmv, &n_kmv)
                : pcg_one(h, b_dev + c * ld, x_dev + c * ld, tol, maxit, w, s, &it, &rel, &rt, &conv,
                          &ms_kmv, &n_kmv);
        outer_max = outer > outer_max ? outer : outer_max;
        it64_max = it64 > it64_max ? it64 : it64_max;
        if (st != AFN_OK && st != AFN_ENOCONV && st != AFN_EBREAKDOWN && st != AFN_ESTAGNATION)
            return st;
        if (st != AFN_OK && worst == AFN_OK) worst = st;
        if (st == AFN_EBREAKDOWN) worst = st;
        it_max = it > it_max ? it : it_max;
        conv_all &= conv;
        rel_max = rel > rel_max || rel != rel ? rel : rel_max;
        true_max = rt > true_max || rt != rt ? rt : true_max;
    }
    tm.mark(1, s);
    AFN_HIP(hipStreamSynchronize(s));
    if (info) {
        info->iterations = it_max;
        info->converged = conv_all;
        info->relres = rel_max;
        info->relres_true = true_max;
        info->ms_solve = tm.ms(0, 1);
        info->ms_matvec = ms_kmv;
        info->matvec_launches = n_kmv;
        info->outer_iterations = outer_max;
        info->fp64_iterations = it64_max;
        info->reserved = 0;
    }
    return worst;
}

afn_status afn_get_info(const afn_handle *h, afn_setup_info *info)
{
    clear_error();
    if (!h || !info) {
        set_error("afn_get_info: invalid argument");
        return AFN_EINVAL;
    }
    *info = h->info;
    return AFN_OK;
}

afn_status afn_get_landmarks(const afn_handle *h, int32_t *idx_host, int64_t cap, int64_t *k_out)
{
    clear_error();
    if (!h || !k_out || (h->k > 0 && (!idx_host || cap < h->k))) {
        set_error("afn_get_landmarks: invalid argument");
        return AFN_EINVAL;
    }
    *k_out = h->k;
    if (h->k > 0)
        AFN_HIP(hipMemcpy(idx_host, h->perm, sizeof(int32_t) * h->k, hipMemcpyDeviceToHost));
    return AFN_OK;
}

afn_status afn_get_fsai(const afn_handle *h, int64_t *rowptr, int32_t *cols_host, double *vals_host,
                        int64_t cap, int64_t *nnz_out)
{
    clear_error();
    if (!h || !rowptr || !nnz_out || (h->nnz > 0 && (!cols_host || cap < h->nnz))) {
        set_error("afn_get_fsai: invalid argument");
        return AFN_EINVAL;
    }
    const int64_t nr = h->nr, w = h->w;
    *nnz_out = h->nnz;
    rowptr[0] = 0;
    if (nr <= 0) return AFN_OK;
    if (!h->cols) {     // Nystrom preconditioner: no FSAI factor
        for (int64_t p = 0; p < nr; ++p) rowptr[p + 1] = 0;
        return AFN_OK;
    }
    std::vector<int32_t> c((size_t)(nr * w));
    std::vector<double> g(vals_host ? (size_t)(nr * w) : 0);
    AFN_HIP(hipMemcpy(c.data(), h->cols, sizeof(int32_t) * nr * w, hipMemcpyDeviceToHost));
    if (vals_host)
        AFN_HIP(hipMemcpy(g.data(), h->gval, sizeof(double) * nr * w, hipMemcpyDeviceToHost));
    int64_t e = 0;
    for (int64_t p = 0; p < nr; ++p) {
        const int64_t m = p + 1 < w ? p + 1 : w;
        for (int64_t a = 0; a < m; ++a, ++e) {
            cols_host[e] = c[(size_t)(p * w + a)];
            if (vals_host) vals_host[e] = g[(size_t)(p * w + a)];
        }
        rowptr[p + 1] = e;
    }
    return AFN_OK;
}

afn_status afn_get_cholesky(const afn_handle *h, double *L_host, int64_t ld)
{
    clear_error();
    if (!h || (h->k > 0 && (!L_host || ld < h->k))) {
        set_error("afn_get_cholesky: invalid argument");
        return AFN_EINVAL;
    }
    const int k = h->k;
    if (k == 0) return AFN_OK;
    AFN_HIP(hipMemcpy2D(L_host, sizeof(double) * ld, h->L, sizeof(double) * k, sizeof(double) * k, k,
                        hipMemcpyDeviceToHost));
    return AFN_OK;
}

afn_status afn_footprint_bytes(int64_t n, int32_t d, const afn_params *prm, size_t *bytes)
{
    clear_error();
    if (!prm || !bytes || n < 1 || d < 1 || d > kMaxD || prm->w < 1 || prm->w > kMaxW ||
        prm->k < -1 || prm->k > n || prm->method < AFN_METHOD_AFN || prm->method > AFN_METHOD_AUTO) {
        set_error("afn_footprint_bytes: invalid argument");
        return AFN_EINVAL;
    }
    const int64_t kmax = prm->k_max > 0 ? prm->k_max : 2000;
    const int64_t k = prm->k >= 0 ? prm->k : (kmax < n ? kmax : n);
    const int64_t nr = n - k, w = prm->w;
    const bool f32 = prm->precision == AFN_FP32;
    auto r = [](int64_t b) { return (size_t)round_up(b > 0 ? b : 1, 256); };
    // shared by both preconditioners: flags, perm, Xp, packed points, workspaces
    size_t base = r(64) + r(4 * n) + r(8 * n * d);
    if (d <= 8) base += r(8 * kmv_packed_doubles(n, d)) + r(4 * n) + r(8 * kmv_box_count(n, d));
    if (f32) base += r(4 * kmv_packed_doubles(n, d)) + r(4 * kmv_box_count(n, d)) +
                     r(4 * work32_floats(n, d, (int)k, nr, nullptr, nullptr));
    base += r(8 * work_doubles(n, d, (int)k, nr, nullptr, nullptr));
    size_t tmp_base = r(4 * k) + (size_t)fps_workspace_bytes(n) + r(4 * n) +
                      r((int64_t)spatial_order_work_bytes(n, d));
    if (prm->k < 0) {
        const int64_t m = prm->m > 0 ? (prm->m < n ? prm->m : n) : (n < 2000 ? n : 2000);
        tmp_base += r(8 * m * m) + r(8 * m * (d + 16)) + (size_t)fps_workspace_bytes(m) + r(8 * 8 * m);
    }
    // AFN: L, Linv, Dinv, pattern, G, G^T, V (+ FP32 copies); transpose and row-order temporaries
    size_t afn = 0;
    if (k > 0) afn += 2 * r(8 * k * k) + r(8 * dinv_doubles((int)k));
    if (nr > 0) afn += r(4 * nr * w) + r(8 * nr * w) + r(8 * (nr + 1)) + r(4 * nr * w) + r(8 * nr * w);
    if (k > 0 && nr > 0) afn += r(8 * k * nr);
    if (f32) afn += r(4 * k * k) + r(4 * k * nr) + 2 * r(4 * nr * w);
    afn += r((int64_t)fsai_transpose_work_bytes(nr, prm->w)) + r(4 * nr) + r((int64_t)knn_work_bytes(nr, d));
    if (d <= 10) afn += r((int64_t)spatial_order_work_bytes(nr, d));
    if (d > 10) afn += r(8 * fsai_batch_doubles((int)k, (int)w));
    // Nystrom: L, Dinv, W, Rginv (+ FP32 W, Rginv); G, its block inverses and GEMM partials
    size_t nys = 0;
    if (k > 0) {
        nys += 2 * r(8 * k * k) + r(8 * dinv_doubles((int)k)) + r(8 * k * n);
        if (f32) nys += r(4 * k * n) + r(4 * k * k);
        nys += r(8 * k * k) + r(8 * dinv_doubles((int)k)) + r(8 * gemm_part_elems(k, n)) +
               r(8 * dot_partials(k * (nr > k ? nr : k))) + r(16);
    }
    size_t extra = prm->method == AFN_METHOD_AFN ? afn
                   : prm->method == AFN_METHOD_NYSTROM ? nys
                                                       : (afn > nys ? afn : nys);
    *bytes = base + tmp_base + extra;
    return AFN_OK;
}

void afn_destroy(afn_handle *h)
{
    if (!h) return;
    if (h->host_sc) (void)hipHostFree(h->host_sc);
    for (auto &e : h->kmv_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->chk_ev) (void)hipEventDestroy(h->chk_ev);
    if (h->mrhs_ws) (void)hipFree(h->mrhs_ws);
    h->arena.release();
    delete h;
}

}  // extern "C"
