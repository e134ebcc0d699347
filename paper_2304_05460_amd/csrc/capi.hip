// C-ABI of libafn: preconditioner construction (Algorithm 2), application
// (Algorithm 3) and preconditioned CG (Algorithm 5, AFN branch).
#include <cfloat>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "afn_internal.h"
#include "group.h"
#include "kfun.h"

namespace afn {

// Rank estimation (Algorithm 4); defined in rank.hip.
afn_status uniform_landmarks(int64_t n, int k, uint64_t seed, int32_t *idx, hipStream_t s);
afn_status rank_estimate(const double *X, int64_t n, int d, double l, int kind, double mu, int m,
                         int kmax, uint64_t seed, DevArena &tmp, hipStream_t s, afn_setup_info *info,
                         int *k_out);
// Bytes rank_estimate carves for a subsample of m points in d dimensions (its
// eigenvalue branch included), as whole 256-byte blocks.
size_t rank_workspace_bytes(int m, int d);

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
template <typename T, typename M>
afn_status apply_blockT(const afn_handle *h, const Factors<M> &f, const T *rp, T *sp, T *y1, T *tt,
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
template <typename T, typename M>
afn_status apply_nysT(const afn_handle *h, const M *W, const T *Rginv, const T *rp, T *sp, T *y1, T *y1b,
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
        AFN_TRY(defer(s, [=](hipStream_t q) { return hipMemcpyAsync(sp, rp, sizeof(T) * n, hipMemcpyDeviceToDevice, q); }));
    }
    return scale_launch(sp, T(1.0 / h->mu), n, s);
}

afn_status apply_block(afn_handle *h, const double *rp, double *sp, const WorkLayout &w,
                       hipStream_t s)
{
    if (h->method == AFN_METHOD_NYSTROM)
        return apply_nysT<double, double>(h, h->W, h->Rginv, rp, sp, w.y1, w.y1b, w.y2, w.gemvp, s);
    Factors<double> f{h->Linv, h->V, h->gval, h->tval};
    return apply_blockT<double, double>(h, f, rp, sp, w.y1, w.t, w.u, w.y1b, w.gemvp, s);
}

afn_status apply_block32(afn_handle *h, const float *rp, float *sp, const WorkLayout32 &w,
                         hipStream_t s)
{
    if (h->precision == AFN_BF16) {
        if (h->method == AFN_METHOD_NYSTROM)
            return apply_nysT<float, bf16_t>(h, h->W16, h->Rginv32, rp, sp, w.y1, w.y1b, w.y2, w.gemvp, s);
        Factors<bf16_t> f{h->Linv16, h->V16, h->gval16, h->tval16};
        return apply_blockT<float, bf16_t>(h, f, rp, sp, w.y1, w.t, w.u, w.y1b, w.gemvp, s);
    }
    if (h->method == AFN_METHOD_NYSTROM)
        return apply_nysT<float, float>(h, h->W32, h->Rginv32, rp, sp, w.y1, w.y1b, w.y2, w.gemvp, s);
    Factors<float> f{h->Linv32, h->V32, h->gval32, h->tval32};
    return apply_blockT<float, float>(h, f, rp, sp, w.y1, w.t, w.u, w.y1b, w.gemvp, s);
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
        set_error("afn_setup: the FSAI blocks of the Schur complement of %d rows are not positive definite",
                  f[2]);
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
    // AFN_BF16: the inner apply uses W rounded to BF16, so W W^T + mu I is
    // formed from the rounded W (kept in FP64): the Woodbury identity then
    // holds for the operator applied, which stays symmetric positive definite
    if (h->precision == AFN_BF16) AFN_TRY(round_bf16_inplace_launch(h->W, (int64_t)k * n, s));
    tm.mark(5, s);
    // W W^T + mu I by 64-column blocks on FP64 MFMA (block c0 needs the rows
    // up to c0 + 63 only: the upper triangle is not used), its factor and
    // inverse
    double *G = nullptr, *Dg = nullptr, *part = nullptr;
    AFN_TRY(tmp.alloc_n(&G, kk));
    AFN_TRY(tmp.alloc_n(&Dg, dinv_doubles(k)));
    AFN_TRY(tmp.alloc_n(&part, gemm_part_bound(k)));      // any m <= k
    for (int c0 = 0; c0 < k; c0 += 64) {
        const int R = k - c0 < 64 ? k - c0 : 64;
        AFN_TRY(gemm_rows<double>(h->W, 1, k, c0 + R, n, h->W + c0, k, R, nullptr, 1.0, G + c0, k, part, s));
    }
    AFN_TRY(zero_upper(G, k, k, s));
    AFN_TRY(add_diagonal(G, k, k, h->mu, s));
    AFN_TRY(cholesky(G, k, k, h->flags + 5, s));
    AFN_TRY(diag_inverses(G, k, Dg, s));
    AFN_TRY(h->arena.alloc_n(&h->Rginv, kk));
    AFN_TRY(identity(h->Rginv, k, s));
    AFN_TRY(trsm_lower(G, Dg, k, h->Rginv, k, s, true));
    tm.mark(6, s);
    return AFN_OK;
}

// Columns of the block-solve workspace a setup provisions (0: none).
int block_columns(const afn_params *prm, int d)
{
    if (prm->precision != AFN_FP32 || d > 8 || prm->nrhs_max < 2) return 0;
    return prm->nrhs_max < 64 ? prm->nrhs_max : 64;
}

// Landmark index slots setup_impl carves: k when it is given, else the
// largest k the rank estimate can return (min(k_max, n)), since the FPS
// order then runs beside the estimate up to that count.
int64_t landmark_slots(int64_t n, const afn_params *prm)
{
    if (prm->k >= 0) return prm->k;
    const int64_t kmax = prm->k_max > 0 ? prm->k_max : 2000;
    return kmax < n ? kmax : n;
}

// A second host thread that enqueues a chain of launches (on a SideStream)
// while this thread enqueues and waits on its own: a chain of a few thousand
// short launches costs the host about as long as the GPU takes to run it, so
// enqueued from the thread that runs the rest it would hold that work back.
// Joined by the destructor (also on error paths, before the side stream is
// released); join() hands on the worker's status and message.
struct HostWorker {
    std::thread th;
    afn_status st = AFN_OK;
    std::string msg;
    template <class F>
    void start(int device, F f)
    {
        try {
            th = std::thread([this, device, f]() {
                hipError_t e = hipSetDevice(device);
                st = e == hipSuccess ? f() : AFN_EDEVICE;
                if (e != hipSuccess) msg = std::string("hipSetDevice: ") + hipGetErrorString(e);
                else if (st != AFN_OK) msg = afn_last_error();
            });
        } catch (...) {
            // no thread to be had: the same launches from this thread
            st = f();
            if (st != AFN_OK) msg = afn_last_error();
        }
    }
    afn_status join()
    {
        if (th.joinable()) th.join();
        if (st != AFN_OK) set_error("%s", msg.c_str());
        return st;
    }
    ~HostWorker()
    {
        if (th.joinable()) th.join();
    }
};

// Bytes setup_impl carves from the workspace when it ends with k landmarks
// and the given method: the same allocations in the same order (each starts
// on a 256-byte boundary), the temporaries included.  rank_m > 0: the rank
// estimation ran on a subsample of rank_m points (its eigenvalue branch
// included).
size_t setup_carve_bytes(int64_t n, int d, int64_t k, int rank_m, int w, const afn_params *prm, int method)
{
    size_t off = 0;
    auto take = [&](size_t bytes) { off = (size_t)round_up((int64_t)off, 256) + bytes; };
    auto n8 = [](int64_t c) { return (size_t)8 * (size_t)(c > 0 ? c : 1); };
    auto n4 = [](int64_t c) { return (size_t)4 * (size_t)(c > 0 ? c : 1); };
    const int64_t nr = n - k, kk = k * k;
    const bool f32 = prm->precision == AFN_FP32, b16 = prm->precision == AFN_BF16;
    take(n4(16));                                            // flags
    take(n4(landmark_slots(n, prm))); take(fps_workspace_bytes(n));   // landmark indices, FPS
    if (rank_m > 0) {
        take(rank_workspace_bytes(rank_m, d));
    }
    take(n4(n)); take(n4(n)); take(n8(n * d));               // perm, selection marks, Xp
    if (method == AFN_METHOD_NYSTROM) {
        if (k > 0) {
            take(n8(kk)); take(n8(dinv_doubles((int)k))); take(n8(k * n));
            take(n8(dot_partials(kk > k * nr ? kk : k * nr))); take(n8(2));
            take(n8(kk)); take(n8(dinv_doubles((int)k))); take(n8(gemm_part_bound(k))); take(n8(kk));
        }
    } else {
        if (k > 0) { take(n8(kk)); take(n8(kk)); take(n8(dinv_doubles((int)k))); }
        if (nr > 0 && d <= 10) { take(n4(nr)); take(spatial_order_work_bytes(nr, d)); }
        if (nr > 0) { take(n4(nr * w)); take(knn_work_bytes(nr, d)); }
        if (k > 0 && nr > 0) take(n8(k * nr));
        if (nr > 0) {
            take(n8(nr * w));
            if (d > 10) take(n8(fsai_batch_doubles((int)k, w)));
            take(n8(nr + 1)); take(n4(nr * w)); take(n8(nr * w)); take(fsai_transpose_work_bytes(nr, w));
        }
    }
    if (d <= 8) {
        take(n4(n)); take(spatial_order_work_bytes(n, d)); take(n8(kmv_packed_doubles(n, d)));
        take(n8(kmv_box_count(n, d))); take(n8(6));
    }
    if (f32 || b16) {
        auto nf = [&](int64_t c) { return b16 ? (size_t)2 * (size_t)(c > 0 ? c : 1) : n4(c); };
        take(n4(kmv_packed_doubles(n, d))); take(n4(kmv_box_count(n, d)));
        if (method == AFN_METHOD_NYSTROM && k > 0) { take(nf(k * n)); take(n4(kk)); }
        if (method != AFN_METHOD_NYSTROM && k > 0) take(nf(kk));
        if (method != AFN_METHOD_NYSTROM && k > 0 && nr > 0) take(nf(k * nr));
        if (method != AFN_METHOD_NYSTROM && nr > 0) { take(nf(nr * w)); take(nf(nr * w)); }
        take(n4(work32_floats(n, d, (int)k, nr, nullptr, nullptr)));
    }
    take(n8(work_doubles(n, d, (int)k, nr, nullptr, nullptr)));
    const int rb = block_columns(prm, d);
    if (rb >= 2) take(block_workspace_bytes(n, d, k, rb));
    return (size_t)round_up((int64_t)off, 256);
}

// afn_workspace_size: the largest carve over every landmark count and method
// the setup can end with.
size_t workspace_bytes(int64_t n, int d, const afn_params *prm)
{
    const int64_t kmax = prm->k_max > 0 ? prm->k_max : 2000;
    const int m = prm->k >= 0 ? 0 : (int)(prm->m > 0 ? (prm->m < n ? prm->m : n) : (n < 2000 ? n : 2000));
    const int64_t klo = prm->k >= 0 ? prm->k : 1;
    const int64_t khi = prm->k >= 0 ? prm->k : (kmax < n ? kmax : n);
    size_t best = 0;
    for (int meth = AFN_METHOD_AFN; meth <= AFN_METHOD_NYSTROM; ++meth) {
        if (prm->method != AFN_METHOD_AUTO && prm->method != meth) continue;
        for (int64_t k = klo; k <= khi; ++k) {
            const size_t b = setup_carve_bytes(n, d, k, m, prm->w, prm, meth);
            best = b > best ? b : best;
        }
    }
    return best;
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
    h->precision = prm->precision;
    AFN_TRY(h->arena.alloc_n(&h->flags, 16));
    AFN_HIP(hipMemsetAsync(h->flags, 0, sizeof(int) * 16, s));
    AFN_TRY(finite_launch(X, n * d, h->flags + 0, s));
    // landmark count
    h->info.rank_r = -1;
    h->info.rank_k_est = -1;
    h->info.rank_eig_branch = 0;
    h->info.rank_eig_count = -1;
    // landmarks (Algorithm 2): FPS in low dimension, uniform sampling above d = 10
    const int lm = prm->landmarks == AFN_LANDMARKS_AUTO ? (d <= 10 ? AFN_LANDMARKS_FPS : AFN_LANDMARKS_UNIFORM)
                                                        : prm->landmarks;
    h->info.landmarks = lm;
    DevArena &tmp = h->arena;
    const int64_t kslots = landmark_slots(n, prm);
    int32_t *idx = nullptr;
    void *fws = nullptr;
    AFN_TRY(tmp.alloc_n(&idx, kslots));
    AFN_TRY(tmp.alloc(&fws, fps_workspace_bytes(n)));
    // the FPS order does not depend on k (a run of k steps gives the first k
    // positions of any longer run), so with k still to be estimated the
    // min(k_max, n) steps run on a second stream beside the rank estimate:
    // two chains of short dependent launches that overlap
    SideStream side;
    HostWorker fps_host;   // declared after side: joined before the stream goes
    const bool overlap = prm->k < 0 && lm == AFN_LANDMARKS_FPS && kslots > 0;
    if (overlap) {
        AFN_TRY(side.open());
        AFN_HIP(hipEventRecord(side.ev0, s));
        AFN_HIP(hipStreamWaitEvent(side.st, side.ev0, 0));
        int *fflag = h->flags + 3;
        const hipStream_t fst = side.st;
        const hipEvent_t fev = side.ev1;
        fps_host.start(h->device, [=]() -> afn_status {
            AFN_TRY(fps(X, n, d, (int)kslots, idx, nullptr, fws, fst, fflag));
            AFN_HIP(hipEventRecord(fev, fst));
            return AFN_OK;
        });
    }
    int k = prm->k;
    if (k < 0) {
        const int m = prm->m > 0 ? (int)(prm->m < n ? prm->m : n) : (int)(n < 2000 ? n : 2000);
        const int kmax = prm->k_max > 0 ? prm->k_max : 2000;
        AFN_TRY(rank_estimate(X, n, d, l, h->kind, mu, m, kmax, prm->seed, h->arena, s, &h->info, &k));
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
    // the landmarks and the block order (temporaries are carved from the same workspace)
    AFN_TRY(h->arena.alloc_n(&h->perm, n));
    int *sel = nullptr;
    AFN_TRY(tmp.alloc_n(&sel, n));
    if (overlap) {
        AFN_TRY(fps_host.join());
        AFN_HIP(hipStreamWaitEvent(s, side.ev1, 0));
    } else if (lm == AFN_LANDMARKS_UNIFORM)
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
    // the kNN pattern of the non-landmark points (and their spatial order)
    // needs none of the factors: it runs on a second stream beside the
    // Cholesky, L^{-1} and V, and the FSAI rows wait for it
    SideStream kside;
    if (nr > 0) {
        AFN_TRY(kside.open());
        AFN_HIP(hipEventRecord(kside.ev0, s));
        AFN_HIP(hipStreamWaitEvent(kside.st, kside.ev0, 0));
    }
    const hipStream_t ks = nr > 0 ? kside.st : s;
    // L = chol(K11 + mu I), Linv, V = L^{-1} K12
    if (k > 0) {
        AFN_TRY(h->arena.alloc_n(&h->L, (int64_t)k * k));
        AFN_TRY(h->arena.alloc_n(&h->Linv, (int64_t)k * k));
        AFN_TRY(h->arena.alloc_n(&h->Dinv, dinv_doubles(k)));
        AFN_TRY(fill_k11(h->Xp, k, d, l, h->kind, mu, h->L, k, s));
        AFN_TRY(cholesky(h->L, k, k, h->flags + 1, s));
        AFN_TRY(diag_inverses(h->L, k, h->Dinv, s));
        AFN_TRY(identity(h->Linv, k, s));
        AFN_TRY(trsm_lower(h->L, h->Dinv, k, h->Linv, k, s, true));
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
        AFN_TRY(spatial_order(h->Xp + (int64_t)k * d, nr, d, rorder, ows, ks));
    }
    if (nr > 0) {
        void *kws = nullptr;
        AFN_TRY(h->arena.alloc_n(&h->cols, nr * h->w));
        AFN_TRY(tmp.alloc(&kws, knn_work_bytes(nr, d)));
        AFN_TRY(knn_pattern_ordered(h->Xp + (int64_t)k * d, nr, d, h->w, rorder, kws, h->cols, ks));
        AFN_HIP(hipEventRecord(kside.ev1, ks));
    }
    tm.mark(4, s);
    if (k > 0 && nr > 0) {
        AFN_TRY(h->arena.alloc_n(&h->V, (int64_t)k * nr));
        AFN_TRY(fill_k12(h->Xp, n, k, d, l, h->kind, h->V, s));
        AFN_TRY(trsm_lower(h->L, h->Dinv, k, h->V, nr, s));
    }
    tm.mark(5, s);
    if (nr > 0) {
        AFN_HIP(hipStreamWaitEvent(s, kside.ev1, 0));
        AFN_TRY(h->arena.alloc_n(&h->gval, nr * h->w));
        // above d = 10 the pattern neighbourhoods share few columns, so each
        // row's columns of V are recomputed in batches rather than gathered
        const bool recompute = d > 10;
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
    if (h->precision == AFN_FP32 || h->precision == AFN_BF16) {
        // the FP32 operator of the inner solves; the factors of the inner
        // apply in FP32, or in BF16 (AFN_BF16: V, L^{-1}, G, G^T and the
        // Nystrom W, whose W W^T + mu I was formed from the rounded W; the
        // k x k inverse factor of that stays FP32)
        const bool b16 = h->precision == AFN_BF16;
        AFN_TRY(h->arena.alloc_n(&h->Xs32, kmv_packed_doubles(n, d)));
        AFN_TRY(kmv_pack(h->Xp, n, d, l, h->kind, h->Xs32, true, s, h->kperm));
        AFN_TRY(h->arena.alloc_n(&h->box32, kmv_box_count(n, d)));
        AFN_TRY(kmv_boxes(h->Xs32, n, d, true, h->box32, s));
        auto copy = [&](const double *src, int64_t cnt, float **f32, bf16_t **f16) -> afn_status {
            if (b16) {
                AFN_TRY(h->arena.alloc_n(f16, cnt));
                return to_bf16_launch(src, *f16, cnt, s);
            }
            AFN_TRY(h->arena.alloc_n(f32, cnt));
            return to_f32_launch(src, *f32, cnt, s);
        };
        if (h->method == AFN_METHOD_NYSTROM) {
            if (k > 0) {
                AFN_TRY(copy(h->W, (int64_t)k * n, &h->W32, &h->W16));
                AFN_TRY(h->arena.alloc_n(&h->Rginv32, (int64_t)k * k));
                AFN_TRY(to_f32_launch(h->Rginv, h->Rginv32, (int64_t)k * k, s));
            }
        }
        if (h->method != AFN_METHOD_NYSTROM && k > 0) AFN_TRY(copy(h->Linv, (int64_t)k * k, &h->Linv32, &h->Linv16));
        if (h->method != AFN_METHOD_NYSTROM && k > 0 && nr > 0)
            AFN_TRY(copy(h->V, (int64_t)k * nr, &h->V32, &h->V16));
        if (h->method != AFN_METHOD_NYSTROM && nr > 0) {
            AFN_TRY(copy(h->gval, nr * h->w, &h->gval32, &h->gval16));
            AFN_TRY(copy(h->tval, nr * h->w, &h->tval32, &h->tval16));
        }
        AFN_TRY(h->arena.alloc_n(&h->work32, work32_floats(n, d, k, nr, nullptr, nullptr)));
    }
    // workspace for apply / PCG
    h->work_doubles = work_doubles(n, d, k, nr, nullptr, nullptr);
    AFN_TRY(h->arena.alloc_n(&h->work, h->work_doubles));
    // block solves of several right-hand sides (FP32 copies, d <= 8)
    h->nrhs_block = 0;
    const int rb = block_columns(prm, d);
    if (rb >= 2) {
        AFN_TRY(h->arena.alloc(&h->mrhs_ws, block_workspace_bytes(n, d, k, rb)));
        AFN_HIP(hipStreamCreateWithFlags(&h->block_stream, hipStreamNonBlocking));
        AFN_HIP(hipEventCreateWithFlags(&h->block_ev, hipEventDisableTiming));
        h->nrhs_block = rb;
    }
    AFN_HIP(hipHostMalloc((void **)&h->host_sc, 16 * sizeof(double), hipHostMallocDefault));
    AFN_HIP(hipEventCreate(&h->kmv_ev[0]));
    AFN_HIP(hipEventCreate(&h->kmv_ev[1]));
    AFN_HIP(hipEventCreateWithFlags(&h->chk_ev, hipEventDisableTiming));
    AFN_HIP(hipEventCreateWithFlags(&h->end_ev, hipEventDisableTiming));
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
    inf.ws_bytes = (int64_t)h->arena.cap;
    inf.ws_bytes_used = (int64_t)h->arena.high;
    return AFN_OK;
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

}  // namespace
}  // namespace afn

// One single-right-hand-side solve, advanced a product at a time.  Every
// solve path goes through it: afn_pcg_solve column by column and the
// step-wise API, so both take the same launches in the same order.
//
// FP64 handle: textbook PCG from x0 = 0 (Algorithm 5's solve), stopping at
// ||r|| / ||b|| <= tol (recurrence), a breakdown, or maxit products.
// AFN_FP32 handle: iterative refinement -- x0 = 0; r = b - (K + mu I) x in
// FP64; a correction e from an inner FP32 PCG on r / ||r|| (FP32 operator,
// apply and vectors, FP64 scalars) stopped at what the step needs but no
// lower than 3e-2 of its start; x += ||r|| e; stop when the FP64 ||r|| / ||b||
// <= tol.  A correction that raised the FP64 residual is taken back, and
// textbook FP64 PCG finishes from the best iterate when the corrections stop
// halving the residual, an inner solve breaks down, 40 steps are used, or
// the inner products pass 4 maxit.
//
// Each round queues the next unit of work (begin: the norm of b; an FP64 or
// FP32 PCG iteration, with the next preconditioner apply queued behind the
// residual copy; a refinement step's residual norm) ending in an event; the
// host then waits on the event and takes the stopping decision, queueing
// what the decision implies.
struct afn_pcg_state {
    enum Phase { kStart, kFp64, kOuter, kInner, kDone };
    afn_handle *h = nullptr;
    const double *b = nullptr;
    double *xout = nullptr;
    double tol = 0.0;
    int maxit = 0;
    Phase phase = kStart;
    bool mixed = false;
    afn::WorkLayout w{};
    afn::WorkLayout32 w32{};
    double bnorm = 0.0;
    // FP64 PCG (also the fallback of a mixed solve)
    int it64 = 0;
    bool p_pending = false;   // p = z + beta p is due before the next product
    bool fp64_started = false;
    // refinement
    int outer = 0;            // refinement steps begun
    int inner_total = 0;
    int inner_it = 0;
    double tol_in = 0.0, rnorm = 0.0, prev = INFINITY;
    bool fallback = false, fallback_redo = false;
    // result
    afn_status status = AFN_OK;
    double relres = 0.0, relres_true = 0.0;
    int converged = 0;
    double ms_kmv = 0.0;
    int n_kmv = 0;
    double t_begin = 0.0, t_end = 0.0;
    hipStream_t stream = nullptr;   // the stream given to afn_pcg_begin
    hipStream_t last = nullptr;     // the stream of the last work queued for it
    int grouped = 0;                // units advanced inside grouped launches
    bool queued = false;            // a unit of work is in flight (afn_pcg_step_many)
};

namespace afn {
namespace {

// Grouped launches in afn_pcg_step_many (afn_group_config; the environment
// variable AFN_NO_GROUP=1 sets the initial value to off).
std::atomic<int> &grouping_flag()
{
    static std::atomic<int> on{[] {
        const char *e = std::getenv("AFN_NO_GROUP");
        return (e && e[0] == '1') ? 0 : 1;
    }()};
    return on;
}

bool grouping_enabled() { return grouping_flag().load(std::memory_order_relaxed) != 0; }

double host_ms()
{
    return 1e3 * (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
                     std::chrono::steady_clock::now().time_since_epoch()).count() * 1e-9;
}

void take_kmv_time(afn_pcg_state *st)
{
    float t = 0.f;
    if (hipEventElapsedTime(&t, st->h->kmv_ev[0], st->h->kmv_ev[1]) == hipSuccess) {
        st->ms_kmv += t;
        st->n_kmv += 1;
    }
}

// x back to the original order, the true FP64 residual, the end of the solve.
afn_status finish(afn_pcg_state *st, afn_status status, bool true_res, hipStream_t s)
{
    afn_handle *h = st->h;
    if (true_res) AFN_TRY(true_relres(h, st->bnorm, st->w, s, &st->relres_true));
    AFN_TRY(permute_scatter(st->w.x, h->n, st->xout, h->n, h->perm, h->n, 1, s));
    AFN_HIP(hipStreamSynchronize(s));
    st->status = status;
    st->converged = status == AFN_OK ? 1 : 0;
    st->phase = afn_pcg_state::kDone;
    st->t_end = host_ms();
    return AFN_OK;
}

// FP64 PCG: its start (z = M^{-1} r, p = z, r'z) from the current x and r.
afn_status fp64_start(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    const WorkLayout &w = st->w;
    AFN_TRY(apply_block(h, w.r, w.z, w, s));
    AFN_HIP(hipMemcpyAsync(w.p, w.z, sizeof(double) * h->n, hipMemcpyDeviceToDevice, s));
    AFN_TRY(dot(w.r, h->n, w.z, h->n, h->n, 1, w.sc + 0, w.dotp, s));
    st->fp64_started = true;
    st->p_pending = false;
    st->it64 = 0;
    return AFN_OK;
}

// One FP64 PCG iteration up to the residual copy, then the next apply.
afn_status fp64_queue(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    const WorkLayout &w = st->w;
    const int64_t n = h->n;
    if (!st->fp64_started) AFN_TRY(fp64_start(st, s));
    if (st->p_pending) AFN_TRY(pcg_p_launch(w.p, w.z, w.sc, n, s));
    st->p_pending = false;
    AFN_TRY(op_f64(h, w.p, w.q, w, s, h->kmv_ev[0], h->kmv_ev[1]));
    AFN_TRY(dot_pcg(w.p, w.q, n, w.sc, kPcgAlpha, w.dotp, s));
    AFN_TRY(pcg_xr_launch(w.x, w.r, w.p, w.q, w.sc, n, w.dotp, w.sc + 2, s));
    AFN_HIP(hipMemcpyAsync(h->host_sc + 1, w.sc + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipEventRecord(h->chk_ev, s));
    // z = M^{-1} r and r'z go on the stream before the host reads the
    // residual (x, r and p stay as they are, so a check that ends the solve
    // discards only z): the device never waits for the host
    if (st->it64 + 1 < st->maxit) {
        AFN_TRY(apply_block(h, w.r, w.z, w, s));
        AFN_TRY(dot_pcg(w.r, w.z, n, w.sc, kPcgBeta, w.dotp, s));
    }
    return AFN_OK;
}

afn_status fp64_decide(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    take_kmv_time(st);
    st->it64 += 1;
    const double pq = h->host_sc[1];
    const double rel = std::sqrt(h->host_sc[2]) / st->bnorm;
    st->relres = rel;
    if (!(pq > 0.0) || !(rel == rel)) {
        set_error("afn_pcg_solve: breakdown at iteration %d (p'Ap = %g)", st->it64, pq);
        return finish(st, AFN_EBREAKDOWN, true, s);
    }
    if (rel <= st->tol) return finish(st, AFN_OK, true, s);
    if (st->it64 >= st->maxit) {
        set_error("afn_pcg_solve: no convergence in %d iterations (relres %g)", st->maxit, rel);
        return finish(st, AFN_ENOCONV, true, s);
    }
    st->p_pending = true;
    return AFN_OK;
}

// Refinement: ||r||^2 of the FP64 residual to the host.
afn_status outer_queue(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    const WorkLayout &w = st->w;
    AFN_TRY(dot(w.r, h->n, w.r, h->n, h->n, 1, w.sc + 7, w.dotp, s));
    AFN_HIP(hipMemcpyAsync(h->host_sc + 7, w.sc + 7, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipEventRecord(h->chk_ev, s));
    return AFN_OK;
}

afn_status outer_decide(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    const WorkLayout &w = st->w;
    const int64_t n = h->n;
    double rnorm = std::sqrt(h->host_sc[7]);
    double rel = rnorm / st->bnorm;
    const int o = st->outer;
    if (o > 0 && !st->fallback_redo && !(rel <= st->prev)) {
        // the last FP32 correction made things worse: take it back (x and
        // its residual were kept in rp / sp) and finish in FP64
        AFN_HIP(hipMemcpyAsync(w.x, w.rp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        AFN_HIP(hipMemcpyAsync(w.r, w.sp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        rel = st->prev;
        rnorm = st->prev * st->bnorm;
        st->fallback = true;
    }
    st->fallback_redo = false;
    st->relres = rel;
    st->relres_true = rel;
    if (!(rel == rel)) {
        set_error("afn_pcg_solve: refinement produced a non-finite residual");
        return finish(st, AFN_EBREAKDOWN, false, s);
    }
    if (rel <= st->tol) return finish(st, AFN_OK, false, s);
    if (o >= 40 || (o >= 3 && rel > 0.5 * st->prev) || st->inner_total >= st->maxit * 4) st->fallback = true;
    if (st->fallback) {
        // textbook FP64 PCG from the current x and its FP64 residual
        st->outer = o + 1;
        st->phase = afn_pcg_state::kFp64;
        st->fp64_started = false;
        return AFN_OK;
    }
    st->prev = rel;
    st->rnorm = rnorm;
    AFN_HIP(hipMemcpyAsync(w.rp, w.x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AFN_HIP(hipMemcpyAsync(w.sp, w.r, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    // inner tolerance: what this step needs, but at least 3e-2 of its
    // start: the FP32 operator and apply bound what one step gains in FP64,
    // and a tighter inner solve spends iterations that the next refinement
    // step does more cheaply
    double tol_in = 0.5 * st->tol / rel;
    tol_in = tol_in > 3e-2 ? tol_in : 3e-2;
    st->tol_in = tol_in < 0.5 ? tol_in : 0.5;
    const WorkLayout32 &v = st->w32;
    AFN_TRY(to_f32_scaled_launch(w.r, 1.0 / rnorm, v.r, n, s));
    // inner FP32 PCG start on r / ||r||: e = 0, z = M^{-1} r, p = z, r'z
    AFN_HIP(hipMemsetAsync(v.e, 0, sizeof(float) * n, s));
    AFN_TRY(apply_block32(h, v.r, v.z, v, s));
    AFN_HIP(hipMemcpyAsync(v.p, v.z, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    AFN_TRY(dot(v.r, n, v.z, n, n, 1, w.sc + 8, w.dotp, s));
    st->inner_it = 0;
    st->p_pending = false;
    st->outer = o + 1;
    st->phase = afn_pcg_state::kInner;
    return AFN_OK;
}

afn_status inner_queue(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    const WorkLayout32 &v = st->w32;
    double *sc = st->w.sc + 8;
    const int64_t n = h->n;
    if (st->p_pending) AFN_TRY(pcg_p_launch(v.p, v.z, sc, n, s));
    st->p_pending = false;
    AFN_TRY(kmv_packed_f32(h->Xs32, n, h->d, h->mu, h->kind, v.p, n, v.q, n, 1, v.kmv, s, h->kmv_ev[0],
                           h->kmv_ev[1], h->kperm, h->box32));
    AFN_TRY(dot_pcg(v.p, v.q, n, sc, kPcgAlpha, st->w.dotp, s));
    AFN_TRY(pcg_xr_launch(v.e, v.r, v.p, v.q, sc, n, st->w.dotp, sc + 2, s));
    double *hs = h->host_sc + 9;
    hipEvent_t chk = h->chk_ev;
    AFN_TRY(defer(s, [=](hipStream_t q) { return hipMemcpyAsync(hs, sc + 1, 2 * sizeof(double), hipMemcpyDeviceToHost, q); }));
    AFN_TRY(defer(s, [=](hipStream_t q) { return hipEventRecord(chk, q); }));
    // the next z = M^{-1} r and r'z are queued before the check (as in the
    // FP64 iteration)
    if (st->inner_it + 1 < st->maxit) {
        AFN_TRY(apply_block32(h, v.r, v.z, v, s));
        AFN_TRY(dot_pcg(v.r, v.z, n, sc, kPcgBeta, st->w.dotp, s));
    }
    return AFN_OK;
}

afn_status inner_decide(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    take_kmv_time(st);
    st->inner_it += 1;
    st->inner_total += 1;
    const double pq = h->host_sc[9];
    const double rel = std::sqrt(h->host_sc[10]);     // relative to ||r / ||r|| || = 1
    if (!(pq > 0.0) || !(rel == rel)) {
        // the FP32 operator or apply lost definiteness: redo this step in FP64
        st->fallback = true;
        st->fallback_redo = true;
        st->outer -= 1;
        st->phase = afn_pcg_state::kOuter;
        return AFN_OK;
    }
    if (rel <= st->tol_in || st->inner_it >= st->maxit) {
        const WorkLayout &w = st->w;
        const int64_t n = h->n;
        AFN_TRY(axpy_f32_into_f64_launch(st->rnorm, st->w32.e, w.x, n, s));
        AFN_TRY(op_f64(h, w.x, w.q, w, s));
        AFN_TRY(sub_launch(w.bp, w.q, w.r, n, s));
        st->phase = afn_pcg_state::kOuter;
        return AFN_OK;
    }
    st->p_pending = true;
    return AFN_OK;
}

// begin: b into block order, ||b||^2 to the host, x = 0, r = b.
afn_status state_begin(afn_pcg_state *st, hipStream_t s)
{
    afn_handle *h = st->h;
    const WorkLayout &w = st->w;
    const int64_t n = h->n;
    st->t_begin = host_ms();
    AFN_TRY(permute_gather(st->b, n, w.bp, n, h->perm, n, 1, s));
    AFN_TRY(dot(w.bp, n, w.bp, n, n, 1, w.sc + 6, w.dotp, s));
    AFN_HIP(hipMemsetAsync(w.x, 0, sizeof(double) * n, s));
    AFN_HIP(hipMemcpyAsync(w.r, w.bp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    AFN_HIP(hipMemcpyAsync(h->host_sc + 6, w.sc + 6, sizeof(double), hipMemcpyDeviceToHost, s));
    AFN_HIP(hipEventRecord(h->chk_ev, s));
    return AFN_OK;
}

afn_status start_decide(afn_pcg_state *st, hipStream_t s)
{
    st->bnorm = std::sqrt(st->h->host_sc[6]);
    if (!(st->bnorm > 0.0)) {
        if (!(st->bnorm == 0.0)) {
            set_error("afn_pcg_solve: right-hand side holds a non-finite value");
            st->relres = NAN;
            return finish(st, AFN_EBREAKDOWN, false, s);
        }
        return finish(st, AFN_OK, false, s);
    }
    st->relres = 1.0;
    st->phase = st->mixed ? afn_pcg_state::kOuter : afn_pcg_state::kFp64;
    return AFN_OK;
}

// Queue the next unit of work of an unfinished solve (ends with chk_ev).
afn_status state_queue(afn_pcg_state *st, hipStream_t s)
{
    switch (st->phase) {
        case afn_pcg_state::kStart: return AFN_OK;    // begin queued the norm of b
        case afn_pcg_state::kFp64: return fp64_queue(st, s);
        case afn_pcg_state::kOuter: return outer_queue(st, s);
        case afn_pcg_state::kInner: return inner_queue(st, s);
        default: return AFN_OK;
    }
}

afn_status state_decide(afn_pcg_state *st, hipStream_t s)
{
    AFN_HIP(hipEventSynchronize(st->h->chk_ev));
    switch (st->phase) {
        case afn_pcg_state::kStart: return start_decide(st, s);
        case afn_pcg_state::kFp64: return fp64_decide(st, s);
        case afn_pcg_state::kOuter: return outer_decide(st, s);
        case afn_pcg_state::kInner: return inner_decide(st, s);
        default: return AFN_OK;
    }
}

// A unit of work counts as a product with K + mu I except the start and
// the refinement's residual norm (whose FP64 product was queued with the
// previous inner step).
bool counts_as_product(const afn_pcg_state *st)
{
    return st->phase == afn_pcg_state::kFp64 || st->phase == afn_pcg_state::kInner;
}

afn_status state_init(afn_handle *h, const double *b, double *x, double tol, int maxit, afn_pcg_state *st)
{
    st->h = h;
    st->b = b;
    st->xout = x;
    st->tol = tol;
    st->maxit = maxit;
    st->mixed = h->precision == AFN_FP32 || h->precision == AFN_BF16;
    work_doubles(h->n, h->d, h->k, h->nr, &st->w, h->work);
    if (st->mixed) work32_floats(h->n, h->d, h->k, h->nr, &st->w32, h->work32);
    return AFN_OK;
}

void state_info(const afn_pcg_state *st, afn_solve_info *info)
{
    info->iterations = st->mixed ? st->inner_total : st->it64;
    info->converged = st->converged;
    info->relres = st->relres;
    info->relres_true = st->relres_true;
    info->ms_solve = (st->phase == afn_pcg_state::kDone ? st->t_end : host_ms()) - st->t_begin;
    info->ms_matvec = st->ms_kmv;
    info->matvec_launches = st->n_kmv;
    info->outer_iterations = st->mixed ? st->outer : 0;
    info->fp64_iterations = st->mixed ? (st->fallback ? st->it64 : 0) : 0;
    info->grouped_units = st->grouped;
}

// Run one solve to its end on stream s (afn_pcg_solve's column loop).
afn_status solve_one(afn_handle *h, const double *b, double *x, double tol, int maxit, hipStream_t s,
                     afn_pcg_state *st)
{
    AFN_TRY(state_init(h, b, x, tol, maxit, st));
    AFN_TRY(state_begin(st, s));
    while (st->phase != afn_pcg_state::kDone) {
        AFN_TRY(state_queue(st, s));
        AFN_TRY(state_decide(st, s));
    }
    return AFN_OK;
}

}  // namespace
}  // namespace afn

using namespace afn;

namespace afn {
namespace {

bool params_valid(int64_t n, int32_t d, const afn_params *prm)
{
    return prm && n >= 1 && n <= INT32_MAX - 1 && d >= 1 && d <= kMaxD && prm->k >= -1 && prm->k <= n &&
           prm->w >= 1 && prm->w <= kMaxW && prm->method >= AFN_METHOD_AFN && prm->method <= AFN_METHOD_AUTO &&
           prm->landmarks >= AFN_LANDMARKS_AUTO && prm->landmarks <= AFN_LANDMARKS_UNIFORM &&
           (prm->kernel == AFN_KERNEL_GAUSSIAN || prm->kernel == AFN_KERNEL_MATERN32) &&
           (prm->precision == AFN_FP64 || prm->precision == AFN_FP32 || prm->precision == AFN_BF16) &&
           !(prm->precision != AFN_FP64 && d > 8) &&
           prm->nrhs_max >= 0 && prm->m >= 0;
}

void release_handle(afn_handle *h)
{
    if (h->host_sc) (void)hipHostFree(h->host_sc);
    for (auto &e : h->kmv_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->chk_ev) (void)hipEventDestroy(h->chk_ev);
    if (h->end_ev) (void)hipEventDestroy(h->end_ev);
    if (h->block_ev) (void)hipEventDestroy(h->block_ev);
    if (h->block_stream) (void)hipStreamDestroy(h->block_stream);
    if (h->ws_owned) (void)hipFree(h->ws_owned);
    delete h;
}

}  // namespace
}  // namespace afn

extern "C" {

afn_status afn_workspace_size(int64_t n, int32_t d, const afn_params *prm, size_t *bytes)
{
    clear_error();
    if (!bytes || !params_valid(n, d, prm)) {
        set_error("afn_workspace_size: invalid argument");
        return AFN_EINVAL;
    }
    *bytes = workspace_bytes(n, d, prm);
    return AFN_OK;
}

afn_status afn_footprint_bytes(int64_t n, int32_t d, const afn_params *prm, size_t *bytes)
{
    return afn_workspace_size(n, d, prm, bytes);
}

afn_status afn_setup(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                     const afn_params *prm, void *ws_dev, size_t ws_bytes, void *stream, afn_handle **out)
{
    clear_error();
    if (!out) {
        set_error("afn_setup: out is NULL");
        return AFN_EINVAL;
    }
    *out = nullptr;
    if (!X_dev || !params_valid(n, d, prm) || !(l > 0) || !std::isfinite(l) || !(mu >= 0) ||
        !std::isfinite(mu) || ((uintptr_t)ws_dev & 255) != 0) {
        set_error("afn_setup: invalid argument (n=%lld d=%d l=%g mu=%g k=%d w=%d ws=%p)", (long long)n, d, l,
                  mu, prm ? prm->k : 0, prm ? prm->w : 0, ws_dev);
        return AFN_EINVAL;
    }
    const size_t need = workspace_bytes(n, d, prm);
    std::unique_ptr<afn_handle, void (*)(afn_handle *)> h(new afn_handle(), release_handle);
    if (ws_dev) {
        if (ws_bytes < need) {
            set_error("afn_setup: workspace of %zu bytes, afn_workspace_size gives %zu", ws_bytes, need);
            return AFN_ENOMEM;
        }
    } else {
        const hipError_t e = hipMalloc(&h->ws_owned, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->ws_owned = nullptr;
            set_error("afn_setup: allocating the %zu-byte workspace failed: %s", need, hipGetErrorString(e));
            return AFN_ENOMEM;
        }
        ws_dev = h->ws_owned;
        ws_bytes = need;
    }
    h->arena.base = (char *)ws_dev;
    h->arena.cap = ws_bytes;
    afn_status st = setup_impl(X_dev, n, d, l, mu, prm, (hipStream_t)stream, h.get());
    if (st != AFN_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
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
    if (h->active) {
        set_error("afn_apply: a step-wise solve is started on this handle");
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
    if (h->active) {
        set_error("afn_pcg_solve: a step-wise solve is started on this handle");
        return AFN_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    WorkLayout w;
    work_doubles(h->n, h->d, h->k, h->nr, &w, h->work);
    WorkLayout32 w32{};
    if (h->work32) work32_floats(h->n, h->d, h->k, h->nr, &w32, h->work32);
    Timer tm;
    tm.mark(0, s);
    int outer_max = 0, it64_max = 0;
    afn_status worst = AFN_OK;
    int it_max = 0, conv_all = 1, n_kmv = 0;
    double ms_kmv = 0.0;
    double rel_max = 0.0, true_max = 0.0;
    // columns still to solve one at a time (all of them outside the block path)
    std::vector<int> single;
    if (nrhs >= 2 && h->nrhs_block >= 2) {
        const int RB = h->nrhs_block;
        std::vector<int> col_ok(RB);
        for (int c0 = 0; c0 < nrhs; c0 += RB) {
            const int Rc = nrhs - c0 < RB ? nrhs - c0 : RB;
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
        afn_pcg_state st;
        AFN_TRY(solve_one(h, b_dev + c * ld, x_dev + c * ld, tol, maxit, s, &st));
        afn_solve_info ci{};
        state_info(&st, &ci);
        ms_kmv += ci.ms_matvec;
        n_kmv += ci.matvec_launches;
        outer_max = ci.outer_iterations > outer_max ? ci.outer_iterations : outer_max;
        it64_max = ci.fp64_iterations > it64_max ? ci.fp64_iterations : it64_max;
        if (st.status != AFN_OK && worst == AFN_OK) worst = st.status;
        if (st.status == AFN_EBREAKDOWN) worst = st.status;
        it_max = ci.iterations > it_max ? ci.iterations : it_max;
        conv_all &= ci.converged;
        rel_max = ci.relres > rel_max || ci.relres != ci.relres ? ci.relres : rel_max;
        true_max = ci.relres_true > true_max || ci.relres_true != ci.relres_true ? ci.relres_true : true_max;
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
        info->grouped_units = 0;
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

afn_status afn_pcg_begin(afn_handle *h, const double *b_dev, double *x_dev, double tol, int32_t maxit,
                         void *stream, afn_pcg_state **out)
{
    clear_error();
    if (!out) {
        set_error("afn_pcg_begin: out is NULL");
        return AFN_EINVAL;
    }
    *out = nullptr;
    if (!h || !b_dev || !x_dev || !(tol > 0) || maxit < 1) {
        set_error("afn_pcg_begin: invalid argument");
        return AFN_EINVAL;
    }
    if (h->active) {
        set_error("afn_pcg_begin: a solve is already started on this handle");
        return AFN_EINVAL;
    }
    std::unique_ptr<afn_pcg_state> st(new afn_pcg_state());
    AFN_TRY(state_init(h, b_dev, x_dev, tol, maxit, st.get()));
    st->stream = (hipStream_t)stream;
    st->last = st->stream;
    AFN_TRY(state_begin(st.get(), st->stream));
    h->active = true;
    *out = st.release();
    return AFN_OK;
}

afn_status afn_pcg_step_many(afn_pcg_state *const *states, int32_t count, int32_t iters, void *stream)
{
    clear_error();
    if (!states || count < 1 || iters < 1) {
        set_error("afn_pcg_step_many: invalid argument");
        return AFN_EINVAL;
    }
    for (int32_t i = 0; i < count; ++i) {
        if (!states[i]) {
            set_error("afn_pcg_step_many: state %d is NULL", i);
            return AFN_EINVAL;
        }
        for (int32_t j = 0; j < i; ++j)
            if (states[j]->h == states[i]->h) {
                set_error("afn_pcg_step_many: states %d and %d share a handle", j, i);
                return AFN_EINVAL;
            }
    }
    // stream NULL: each solve on the stream it was begun on (solves overlap
    // on the device); otherwise every solve on 'stream'
    auto sof = [&](const afn_pcg_state *st) { return stream ? (hipStream_t)stream : st->stream; };
    // Every solve keeps one unit of work in flight; the host polls their
    // events and takes each decision as soon as its unit is done, so a small
    // solve is not held to the pace of a large one.  A solve stops at its
    // budget of products; the call returns when every solve has finished or
    // spent its budget, or at the end of the first polling pass in which a
    // solve finished (its caller can then release it and start another).
    // Units in flight at the return stay queued for the next call.
    //
    // The units due in one polling pass are queued together at its end:
    // inner iterations of like mixed-precision solves (same d, kernel,
    // precision, method, pattern width, n within a factor of 2) are recorded
    // and replayed as grouped launches on the first one's stream (group.h);
    // the rest are queued one by one.  An inner iteration that is due while a
    // like solve's inner iteration is still in flight waits for it (one unit
    // of a solve at most 4 times as costly), so that the two are queued
    // together from then on; nothing waits past the end of the call.  A solve whose next unit goes to
    // another stream than its last one's first waits there for all its work
    // so far (end_ev), and its decisions are taken on the stream of its last
    // unit, so each solve's work stays in order.
    std::vector<int> products(count, 0);
    bool finished_one = false;
    std::vector<afn_pcg_state *> pend;
    pend.reserve(count);
    auto move_to = [](afn_pcg_state *st, hipStream_t q) -> afn_status {
        if (st->last != q) {
            AFN_HIP(hipEventRecord(st->h->end_ev, st->last));
            AFN_HIP(hipStreamWaitEvent(q, st->h->end_ev, 0));
            st->last = q;
        }
        return AFN_OK;
    };
    auto like = [](const afn_pcg_state *a, const afn_pcg_state *b) {
        const afn_handle *x = a->h, *y = b->h;
        auto cls = [](int64_t n) { return 63 - __builtin_clzll((unsigned long long)(n > 0 ? n : 1)); };
        return x->d == y->d && x->kind == y->kind && x->precision == y->precision && x->method == y->method &&
               (x->w > 64) == (y->w > 64) && cls(x->n) == cls(y->n);
    };
    auto inflight_like = [&](const afn_pcg_state *x) {
        for (int32_t i = 0; i < count; ++i) {
            const afn_pcg_state *y = states[i];
            if (y != x && y->queued && y->phase == afn_pcg_state::kInner && like(x, y)) return true;
        }
        return false;
    };
    std::vector<afn_pcg_state *> held;
    auto flush = [&](bool final) -> afn_status {
        held.clear();
        if (!final && grouping_enabled()) {
            size_t m = 0;
            for (afn_pcg_state *st : pend) {
                if (st->phase == afn_pcg_state::kInner && inflight_like(st)) held.push_back(st);
                else pend[m++] = st;
            }
            pend.resize(m);
        }
        std::vector<char> taken(pend.size(), 0);
        if (grouping_enabled()) {
            std::vector<afn_pcg_state *> grp;
            for (size_t i = 0; i < pend.size(); ++i) {
                if (taken[i] || pend[i]->phase != afn_pcg_state::kInner) continue;
                grp.assign(1, pend[i]);
                for (size_t j = i + 1; j < pend.size(); ++j)
                    if (!taken[j] && pend[j]->phase == afn_pcg_state::kInner && like(pend[i], pend[j])) {
                        grp.push_back(pend[j]);
                        taken[j] = 1;
                    }
                if (grp.size() < 2) continue;
                taken[i] = 1;
                const hipStream_t q = sof(grp[0]);
                std::vector<Recorder> recs(grp.size());
                std::vector<Recorder *> rp(grp.size());
                for (size_t g = 0; g < grp.size(); ++g) {
                    AFN_TRY(move_to(grp[g], q));
                    recorder() = &recs[g];
                    const afn_status stq = state_queue(grp[g], q);
                    recorder() = nullptr;
                    AFN_TRY(stq);
                    rp[g] = &recs[g];
                }
                std::vector<char> merged(grp.size(), 0);
                AFN_TRY(replay_grouped(rp.data(), (int)rp.size(), q, merged.data()));
                for (size_t g = 0; g < grp.size(); ++g) {
                    grp[g]->queued = true;
                    grp[g]->grouped += merged[g] ? 1 : 0;
                }
            }
        }
        for (size_t i = 0; i < pend.size(); ++i) {
            if (taken[i]) continue;
            afn_pcg_state *st = pend[i];
            AFN_TRY(move_to(st, sof(st)));
            AFN_TRY(state_queue(st, sof(st)));
            st->queued = true;
        }
        pend.swap(held);
        return AFN_OK;
    };
    for (int32_t i = 0; i < count; ++i) {
        afn_pcg_state *st = states[i];
        if (st->phase == afn_pcg_state::kDone || st->queued) continue;
        pend.push_back(st);
    }
    AFN_TRY(flush(false));
    for (;;) {
        bool waiting = false, progressed = false;
        for (int32_t i = 0; i < count; ++i) {
            afn_pcg_state *st = states[i];
            if (!st->queued) continue;
            const hipError_t q = hipEventQuery(st->h->chk_ev);
            if (q == hipErrorNotReady) {
                waiting = true;
                continue;
            }
            if (q != hipSuccess) {
                set_error("afn_pcg_step_many: hipEventQuery: %s", hipGetErrorString(q));
                return AFN_EDEVICE;
            }
            st->queued = false;
            progressed = true;
            if (counts_as_product(st)) products[i] += 1;
            AFN_TRY(state_decide(st, st->last));
            if (st->phase == afn_pcg_state::kDone) {
                finished_one = true;
            } else if (products[i] < iters) {
                pend.push_back(st);
                waiting = true;
            }
        }
        const bool last = !(waiting || !pend.empty()) || finished_one;
        AFN_TRY(flush(last));
        if (last) break;
        if (!progressed) std::this_thread::yield();
    }
    return AFN_OK;
}

void afn_group_config(int32_t on) { grouping_flag().store(on ? 1 : 0, std::memory_order_relaxed); }

afn_status afn_pcg_query(const afn_pcg_state *st, int32_t *done, afn_solve_info *info)
{
    clear_error();
    if (!st || !done) {
        set_error("afn_pcg_query: invalid argument");
        return AFN_EINVAL;
    }
    *done = st->phase == afn_pcg_state::kDone ? 1 : 0;
    if (info) state_info(st, info);
    return *done ? st->status : AFN_OK;
}

void afn_pcg_end(afn_pcg_state *st)
{
    if (!st) return;
    // the unit in flight and the work queued behind its check
    if (st->queued && st->h) (void)hipEventSynchronize(st->h->chk_ev);
    if (st->h) (void)hipStreamSynchronize(st->last);
    if (st->h) st->h->active = false;
    delete st;
}

void afn_destroy(afn_handle *h)
{
    if (!h) return;
    release_handle(h);
}

}  // extern "C"
