// Block solve of R <= 64 right-hand sides with one AFN preconditioner.
//
// Per-column iterative refinement in FP64 (residual B - (K + mu I) X by the
// FP64 MFMA tile kernel) with corrections from one block PCG in FP32 that
// advances all columns together: per-column FP64 scalars, converged columns
// masked (their step length is zero).  One block-PCG iteration (operator,
// per-column dots and updates, batched Algorithm 3) is captured once as a
// HIP graph and replayed; the host reads back only the count of active
// columns after each replay.  Setting AFN_NO_GRAPH=1 runs the same launches
// eagerly (used to check replays against eager execution).
#include <cmath>
#include <cstdlib>
#include <vector>

#include "afn_internal.h"

namespace afn {

namespace {

struct BlockWs {
    // FP64, row-major n x R unless noted
    double *Bp, *X64, *R64, *Y64, *part64;
    double *bn2, *rr64, *inv, *amul, *tolc;       // R each
    // FP32
    float *Rr, *Rw, *Z, *P, *Q, *E, *Y1, *Y1b, *Y2, *T, *U, *gpart, *kpart;
    // FP64 scalars of the inner solve (R each) and dot partials
    double *rho, *pq, *rr, *rho_new, *alpha, *beta, *bn2_in, *dotp;
    int *active, *count, *bad;
};

size_t block_ws_layout(int64_t n, int d, int64_t k, int R, BlockWs *w, char *base)
{
    const int64_t nr = n - k;
    const int64_t npad = kmv_packed_doubles(n, d) / d;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    BlockWs t{};
    const int64_t nR = n * R;
    t.Bp = (double *)take(8 * nR);
    t.X64 = (double *)take(8 * nR);
    t.R64 = (double *)take(8 * nR);
    t.Y64 = (double *)take(8 * nR);
    t.part64 = (double *)take(8 * (size_t)mrhs_part_elems(npad));
    t.bn2 = (double *)take(8 * 64);
    t.rr64 = (double *)take(8 * 64);
    t.inv = (double *)take(8 * 64);
    t.amul = (double *)take(8 * 64);
    t.tolc = (double *)take(8 * 64);
    t.Rr = (float *)take(4 * nR);
    t.Rw = (float *)take(4 * nR);
    t.Z = (float *)take(4 * nR);
    t.P = (float *)take(4 * nR);
    t.Q = (float *)take(4 * nR);
    t.E = (float *)take(4 * nR);
    t.Y1 = (float *)take(4 * (size_t)(k * R + 1));
    t.Y1b = (float *)take(4 * (size_t)(k * R + 1));
    t.Y2 = (float *)take(4 * (size_t)(k * R + 1));
    t.T = (float *)take(4 * (size_t)(nr * R + 1));
    t.U = (float *)take(4 * (size_t)(nr * R + 1));
    int64_t gp = gemm_part_elems(k, k);
    const int64_t g2 = gemm_part_elems(nr, k), g3 = gemm_part_elems(k, nr);
    const int64_t g4 = gemm_part_elems(n, k), g5 = gemm_part_elems(k, n);    // Nystrom
    gp = gp > g2 ? gp : g2;
    gp = gp > g3 ? gp : g3;
    gp = gp > g4 ? gp : g4;
    gp = gp > g5 ? gp : g5;
    t.gpart = (float *)take(4 * (size_t)(gp + 1));
    t.kpart = (float *)take(4 * (size_t)mrhs_part_elems(npad));
    t.rho = (double *)take(8 * 64);
    t.pq = (double *)take(8 * 64);
    t.rr = (double *)take(8 * 64);
    t.rho_new = (double *)take(8 * 64);
    t.alpha = (double *)take(8 * 64);
    t.beta = (double *)take(8 * 64);
    t.bn2_in = (double *)take(8 * 64);
    t.dotp = (double *)take(8 * (size_t)coldot_blocks(n) * 64);
    t.active = (int *)take(4 * 64);
    t.count = (int *)take(4 * 4);
    t.bad = (int *)take(4 * 4);
    if (w) *w = t;
    return off;
}

size_t block_ws(const afn_handle *h, int R, BlockWs *w, char *base)
{
    return block_ws_layout(h->n, h->d, h->k, R, w, base);
}

__global__ void init_active(const double *bn2, int *active, int R)
{
    const int c = threadIdx.x;
    if (c < R) active[c] = bn2[c] > 0.0 ? 1 : 0;
}

// Z = M^{-1} Rin for the Nystrom preconditioner (see apply_nysT), R columns.
afn_status apply32_block_nys(afn_handle *h, const float *Rin, float *Zout, int R, const BlockWs &w,
                             hipStream_t s)
{
    const int k = h->k;
    const int64_t n = h->n;
    if (k > 0) {
        AFN_TRY(gemm_rows<float>(h->W32, 1, k, k, n, Rin, R, R, nullptr, 1.0f, w.Y1, R, w.gpart, s));
        AFN_TRY(gemm_rows<float>(h->Rginv32, 1, k, k, k, w.Y1, R, R, nullptr, 1.0f, w.Y1b, R, w.gpart, s));
        AFN_TRY(gemm_rows<float>(h->Rginv32, k, 1, k, k, w.Y1b, R, R, nullptr, 1.0f, w.Y2, R, w.gpart, s));
        AFN_TRY(gemm_rows<float>(h->W32, k, 1, n, k, w.Y2, R, R, Rin, -1.0f, Zout, R, w.gpart, s));
    } else {
        AFN_HIP(hipMemcpyAsync(Zout, Rin, sizeof(float) * n * R, hipMemcpyDeviceToDevice, s));
    }
    return scale_launch(Zout, (float)(1.0 / h->mu), n * R, s);
}

// Z = M^{-1} Rin for R columns (row-major blocks, block order).
afn_status apply32_block(afn_handle *h, const float *Rin, float *Zout, int R, const BlockWs &w,
                         hipStream_t s)
{
    if (h->method == AFN_METHOD_NYSTROM) return apply32_block_nys(h, Rin, Zout, R, w, s);
    const int k = h->k;
    const int64_t nr = h->nr;
    if (k > 0)
        AFN_TRY(gemm_rows<float>(h->Linv32, 1, k, k, k, Rin, R, R, nullptr, 1.0f, w.Y1, R, w.gpart, s));
    if (nr > 0) {
        const float *t = Rin + (int64_t)k * R;
        if (k > 0) {
            AFN_TRY(gemm_rows<float>(h->V32, k, 1, nr, k, w.Y1, R, R, Rin + (int64_t)k * R, -1.0f, w.T, R,
                                     w.gpart, s));
            t = w.T;
        }
        AFN_TRY(spmm_g<float>(h->cols, h->gval32, nr, h->w, t, R, w.U, h->rorder, s));
        AFN_TRY(spmm_gt<float>(h->tptr, h->trow, h->tval32, nr, w.U, R, Zout + (int64_t)k * R, nullptr, s));
    }
    if (k > 0) {
        const float *y = w.Y1;
        if (nr > 0) {
            AFN_TRY(gemm_rows<float>(h->V32, 1, k, k, nr, Zout + (int64_t)k * R, R, R, w.Y1, -1.0f, w.Y1b, R,
                                     w.gpart, s));
            y = w.Y1b;
        }
        AFN_TRY(gemm_rows<float>(h->Linv32, k, 1, k, k, y, R, R, nullptr, 1.0f, Zout, R, w.gpart, s));
    }
    return AFN_OK;
}

afn_status inner_body(afn_handle *h, int R, const BlockWs &w, hipStream_t s)
{
    const int64_t n = h->n;
    const int64_t npad = kmv_packed_doubles(n, h->d) / h->d;
    AFN_TRY(kmv_mrhs_run<float>(h->Xs32, npad, n, h->d, h->mu, h->kind, w.P, R, w.Q, R, R, w.kpart, s, nullptr, nullptr,
                                h->kperm, h->box32));
    AFN_TRY(coldot<float>(w.P, w.Q, n, R, w.pq, w.dotp, s));
    AFN_TRY(col_alpha_launch(w.rho, w.pq, w.active, w.alpha, R, w.bad, s));
    AFN_TRY(col_xr_launch<float>(w.E, w.Rw, w.P, w.Q, w.alpha, n, R, w.rr, w.dotp, s));
    AFN_TRY(col_converged_launch(w.rr, w.bn2_in, w.tolc, w.active, w.count, R, w.bad, s));
    AFN_TRY(apply32_block(h, w.Rw, w.Z, R, w, s));
    AFN_TRY(coldot<float>(w.Rw, w.Z, n, R, w.rho_new, w.dotp, s));
    AFN_TRY(col_beta_launch(w.rho, w.rho_new, w.active, w.beta, R, s));
    AFN_TRY(col_p_launch<float>(w.P, w.Z, w.beta, n, R, s));
    return AFN_OK;
}

struct GraphHolder {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    ~GraphHolder()
    {
        if (e) (void)hipGraphExecDestroy(e);
        if (g) (void)hipGraphDestroy(g);
    }
};

// Block PCG on the normalized residual columns in w.Rr (tolerances w.tolc):
// correction in w.E.  Returns the iteration count.
afn_status inner_block(afn_handle *h, int R, int maxit, const BlockWs &w, hipStream_t s,
                       GraphHolder &gh, bool use_graph, int *iters, int *bad_out)
{
    const int64_t n = h->n;
    int *hi = reinterpret_cast<int *>(h->host_sc + 12);
    AFN_HIP(hipMemsetAsync(w.E, 0, sizeof(float) * n * R, s));
    AFN_HIP(hipMemsetAsync(w.bad, 0, sizeof(int), s));
    AFN_HIP(hipMemcpyAsync(w.Rw, w.Rr, sizeof(float) * n * R, hipMemcpyDeviceToDevice, s));
    AFN_TRY(coldot<float>(w.Rr, w.Rr, n, R, w.bn2_in, w.dotp, s));
    hipLaunchKernelGGL(init_active, dim3(1), dim3(64), 0, s, w.bn2_in, w.active, R);
    AFN_HIP(hipGetLastError());
    AFN_TRY(apply32_block(h, w.Rw, w.Z, R, w, s));
    AFN_HIP(hipMemcpyAsync(w.P, w.Z, sizeof(float) * n * R, hipMemcpyDeviceToDevice, s));
    AFN_TRY(coldot<float>(w.Rw, w.Z, n, R, w.rho, w.dotp, s));
    if (use_graph && !gh.e) {
        AFN_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        afn_status st = inner_body(h, R, w, s);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(s, &g);
        if (st != AFN_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        AFN_HIP(ce);
        gh.g = g;
        AFN_HIP(hipGraphInstantiate(&gh.e, gh.g, nullptr, nullptr, 0));
    }
    *iters = 0;
    *bad_out = 0;
    for (int it = 0; it < maxit; ++it) {
        if (use_graph) AFN_HIP(hipGraphLaunch(gh.e, s));
        else AFN_TRY(inner_body(h, R, w, s));
        AFN_HIP(hipMemcpyAsync(hi, w.count, sizeof(int), hipMemcpyDeviceToHost, s));
        AFN_HIP(hipMemcpyAsync(hi + 1, w.bad, sizeof(int), hipMemcpyDeviceToHost, s));
        AFN_HIP(hipStreamSynchronize(s));
        *iters = it + 1;
        if (hi[1]) {
            *bad_out = hi[1];
            break;
        }
        if (hi[0] == 0) break;
    }
    return AFN_OK;
}

}  // namespace

size_t block_workspace_bytes(int64_t n, int d, int64_t k, int R)
{
    return block_ws_layout(n, d, k, R, nullptr, nullptr);
}

afn_status block_refine_solve(afn_handle *h, const double *B, int64_t ld, double *Xout, int R,
                              double tol, int maxit, hipStream_t user_s, int *iters, int *outer,
                              double *relres_max, int *conv_all, int *col_ok)
{
    const int64_t n = h->n;
    const int64_t npad = kmv_packed_doubles(n, h->d) / h->d;
    // every early return leaves the columns marked unsolved, so the caller
    // re-solves them one at a time
    for (int c = 0; c < R; ++c) col_ok[c] = 0;
    if (R > h->nrhs_block || !h->mrhs_ws || !h->block_stream) {
        set_error("block solve: %d columns, but the handle's block workspace holds %d", R, h->nrhs_block);
        return AFN_EINVAL;
    }
    BlockWs w;
    block_ws(h, R, &w, (char *)h->mrhs_ws);
    // the handle's own stream (default priority; created at setup), ordered
    // after the caller's and the caller's after it
    hipStream_t s = h->block_stream;
    hipEvent_t ev = h->block_ev;
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamSynchronize(s); }
    } sg{s};
    AFN_HIP(hipEventRecord(ev, user_s));
    AFN_HIP(hipStreamWaitEvent(s, ev, 0));

    const char *ng = std::getenv("AFN_NO_GRAPH");
    const bool use_graph = !(ng && ng[0] == '1');
    GraphHolder gh;
    double *hd = h->host_sc;   // host scratch (pinned, 16 doubles): not enough for R values
    std::vector<double> bn2(R), rr(R), inv(R), amul(R), tolc(R);
    (void)hd;

    AFN_TRY(gather_rows<double>(B, ld, h->perm, n, R, nullptr, w.Bp, s));
    AFN_HIP(hipMemsetAsync(w.X64, 0, sizeof(double) * n * R, s));
    AFN_HIP(hipMemcpyAsync(w.R64, w.Bp, sizeof(double) * n * R, hipMemcpyDeviceToDevice, s));
    AFN_TRY(coldot<double>(w.Bp, w.Bp, n, R, w.bn2, w.dotp, s));
    AFN_HIP(hipMemcpyAsync(bn2.data(), w.bn2, sizeof(double) * R, hipMemcpyDeviceToHost, s));
    AFN_HIP(hipStreamSynchronize(s));
    for (int c = 0; c < R; ++c)
        if (!(bn2[c] == bn2[c]) || std::isinf(bn2[c])) {
            set_error("afn_pcg_solve: right-hand side %d holds a non-finite value", c);
            return AFN_EBREAKDOWN;
        }
    *iters = 0;
    *outer = 0;
    *conv_all = 0;
    afn_status status = AFN_ENOCONV;
    double prev = INFINITY;
    for (int o = 0;; ++o) {
        AFN_TRY(coldot<double>(w.R64, w.R64, n, R, w.rr64, w.dotp, s));
        AFN_HIP(hipMemcpyAsync(rr.data(), w.rr64, sizeof(double) * R, hipMemcpyDeviceToHost, s));
        AFN_HIP(hipStreamSynchronize(s));
        double worst = 0.0;
        int nactive = 0;
        for (int c = 0; c < R; ++c) {
            const double rel = bn2[c] > 0.0 ? std::sqrt(rr[c] / bn2[c]) : 0.0;
            if (!(rel == rel)) worst = NAN;
            else if (rel > worst) worst = rel;
            const bool act = rel > tol;
            col_ok[c] = act ? 0 : 1;
            nactive += act;
            inv[c] = act ? 1.0 / std::sqrt(rr[c]) : 0.0;
            amul[c] = act ? std::sqrt(rr[c]) : 0.0;
            double ti = act ? 0.5 * tol / rel : 0.5;
            ti = ti > 3e-2 ? ti : 3e-2;      // as for single solves: FP32 bounds a step's gain
            tolc[c] = ti < 0.5 ? ti : 0.5;
        }
        *relres_max = worst;
        if (!(worst == worst)) {
            set_error("afn_pcg_solve: block refinement produced a non-finite residual");
            status = AFN_EBREAKDOWN;
            break;
        }
        if (nactive == 0) {
            status = AFN_OK;
            *conv_all = 1;
            break;
        }
        if (o >= 40 || (o >= 3 && worst > 0.5 * prev)) {
            set_error("afn_pcg_solve: block refinement stagnated at relative residual %g", worst);
            status = AFN_ESTAGNATION;
            break;
        }
        if (*iters >= 4 * maxit) {
            set_error("afn_pcg_solve: block solve did not converge (relres %g)", worst);
            status = AFN_ENOCONV;
            break;
        }
        prev = worst;
        AFN_HIP(hipMemcpyAsync(w.inv, inv.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
        AFN_HIP(hipMemcpyAsync(w.amul, amul.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
        AFN_HIP(hipMemcpyAsync(w.tolc, tolc.data(), sizeof(double) * R, hipMemcpyHostToDevice, s));
        AFN_TRY(scale_to_f32_launch(w.R64, w.inv, w.Rr, n, R, s));
        int it = 0, bad = 0;
        AFN_TRY(inner_block(h, R, maxit, w, s, gh, use_graph, &it, &bad));
        *iters += it;
        *outer = o + 1;
        if (bad) {
            set_error("afn_pcg_solve: block inner PCG breakdown (flag %d)", bad);
            status = AFN_EBREAKDOWN;
            break;
        }
        AFN_TRY(axpy_cols_f32_launch(w.amul, w.E, w.X64, n, R, s));
        AFN_TRY(kmv_mrhs_run<double>(h->Xs64, npad, n, h->d, h->mu, h->kind, w.X64, R, w.Y64, R, R, w.part64, s,
                                     nullptr, nullptr, h->kperm, h->box64));
        AFN_TRY(sub_rows_launch(w.Bp, w.Y64, w.R64, n * R, s));
    }
    AFN_TRY(scatter_rows(w.X64, h->perm, n, R, Xout, ld, s));
    AFN_HIP(hipStreamSynchronize(s));
    AFN_HIP(hipEventRecord(ev, s));
    AFN_HIP(hipStreamWaitEvent(user_s, ev, 0));
    return status;
}

}  // namespace afn
