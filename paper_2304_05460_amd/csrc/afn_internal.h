// Internal declarations of libafn (gfx950).  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "afn.h"

namespace afn {

// Thread-local error message (afn_last_error()).
void set_error(const char *fmt, ...);
void clear_error();

#define AFN_HIP(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::afn::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                \
            return AFN_EDEVICE;                                                        \
        }                                                                              \
    } while (0)

#define AFN_TRY(expr)                      \
    do {                                   \
        afn_status s_ = (expr);            \
        if (s_ != AFN_OK) return s_;       \
    } while (0)

constexpr int kMaxD = 64;
constexpr int kMaxW = 128;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Block b of a launch of G blocks, in XCD-aware order: blocks are dealt to
// the 8 XCDs round-robin, so XCD x gets b = x, x+8, ...; giving it a
// contiguous range of spatially ordered rows keeps each XCD's gathers within
// its own L2.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t G)
{
    const int64_t x = b & 7, j = b >> 3;
    int64_t start = 0;
    for (int64_t y = 0; y < x; ++y) start += (G - y + 7) >> 3;
    return start + j;
}

// BF16 storage of preconditioner factors (AFN_BF16): the upper 16 bits of an
// FP32 value.  Loads widen to FP32 exactly; sums stay in FP32.
struct bf16_t {
    uint16_t bits;
};
__host__ __device__ inline float bf16_to_f32(bf16_t b) { return __builtin_bit_cast(float, (uint32_t)b.bits << 16); }
// Value of type M in the arithmetic type T.
template <typename T, typename M>
__host__ __device__ inline T widen(M v) { return (T)v; }
template <>
__host__ __device__ inline float widen<float, bf16_t>(bf16_t v) { return bf16_to_f32(v); }

// Autotuner (tune.hip): the candidate to run for shape class 'shape' of
// tunable 'kernel' (see afn_tune_config); run(i) queues candidate i on s.
int tune_pick(const char *kernel, const std::string &shape, int ncand, int heuristic,
              const std::function<afn_status(int)> &run, hipStream_t s);

// Device memory of a handle: a bump allocator over one region (the caller's
// workspace, or one block the library allocated for the handle).  Buffers
// start on 256-byte boundaries; temporaries of the setup are carved like
// everything else and never reclaimed, so the region's size bounds the sum
// of every allocation (afn_workspace_size).
struct DevArena {
    char *base = nullptr;
    size_t cap = 0, off = 0, high = 0;
    afn_status alloc(void **p, size_t bytes);
    template <class T>
    afn_status alloc_n(T **p, int64_t count) {
        return alloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)(count > 0 ? count : 1));
    }
};

// Per-device scratch for entry points that do not own a handle.  Grows on
// demand; calls that share it must be stream-ordered by the caller.
afn_status library_scratch(size_t bytes, void **ptr);

// ---------------------------------------------------------------- kernel matvec
// kind: afn_kernel (kfun.h defines the kernel functions and the coordinate
// scaling of the packed layout).
// Partial-sum workspace for kmv_f64 (doubles).
int64_t kmv_splits(int64_t n);
int64_t kmv_workspace_doubles(int64_t n, int d);
// y[:, c] = (K + mu I) v[:, c] for c < nrhs; X row-major n x d FP64.
// ev0/ev1 (optional, single right-hand side): recorded around the tile kernel.
afn_status kmv_f64(const double *X, int64_t n, int d, double l, double mu, int kind, const double *v,
                   int64_t ldv, double *y, int64_t ldy, int nrhs, double *work,
                   hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Pre-scaled SoA copy of the points for the symmetric tile kernels
// (kmv_packed_doubles(n, d) doubles, or as many floats when f32).
// perm (optional): packed position q holds point perm[q] (vectors stay in
// the caller's order and are indexed through perm).
int64_t kmv_packed_doubles(int64_t n, int d);
afn_status kmv_pack(const double *X, int64_t n, int d, double l, int kind, void *Xs, bool f32, hipStream_t s,
                    const int32_t *perm = nullptr);
// Tile pruning.  Per 64-point tile of the packed layout, the box of its
// scaled coordinates (kmv_box_count(n, d) values of the packed type).  A pair
// of tiles whose boxes are at least sqrt(kernel_cut_t(kind, cut)) apart in
// scaled units holds only kernel values below 2^-cut and is skipped: cut =
// kCullF64 for FP64 tiles, kCullF32 for FP32 tiles.  The dropped part of row
// i is below 2^-cut sum_j |v_j|.
constexpr double kCullF64 = 64.0;
constexpr double kCullF32 = 44.0;
// FP64 tile pairs whose kernel values are all below 2^-kFarF64 evaluate the
// exponential in FP32 (the MFMA tile kernel, d <= 4): for t >= 46 the relative
// error ln 2 * 2^-24 t (t rounded to FP32) + 2^-23 (the hardware exponential)
// times 2^-t stays below 2^-64, the bound of the skipped pairs (the Matern
// value likewise).
constexpr double kFarF64 = 46.0;
int64_t kmv_box_count(int64_t n, int d);
// counts[0] = unordered pairs of non-empty tiles kept at cut tcut, counts[1] =
// all such pairs (FP64 boxes, d <= 8).
afn_status kmv_kept_fraction(const double *box, int64_t n, int d, double tcut, unsigned long long *counts,
                             hipStream_t s);
afn_status kmv_boxes(const void *Xs, int64_t n, int d, bool f32, void *box, hipStream_t s);
// y = (K + mu I) v on packed points (d <= 8); part: kmv_workspace_doubles(n, d)
// doubles (or floats for the FP32 variant).  box (optional) enables pruning.
afn_status kmv_packed_f64(const double *Xs, int64_t n, int d, double mu, int kind, const double *v, int64_t ldv,
                          double *y, int64_t ldy, int nrhs, double *part, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                          const int32_t *perm = nullptr, const double *box = nullptr);
afn_status kmv_packed_f32(const float *Xs, int64_t n, int d, double mu, int kind, const float *v, int64_t ldv,
                          float *y, int64_t ldy, int nrhs, float *part, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                          const int32_t *perm = nullptr, const float *box = nullptr);
// FP32 tiles on packed points with FP64 vectors (part: floats).
afn_status kmv_packed_f32_dvec(const float *Xs, int64_t n, int d, double mu, int kind, const double *v,
                               int64_t ldv, double *y, int64_t ldy, int nrhs, float *part, hipStream_t s,
                               const int32_t *perm, const float *box);
// FP32 tiles and accumulation; FP64 vectors at the interface.
afn_status kmv_f32(const double *X, int64_t n, int d, double l, double mu, int kind, const double *v,
                   int64_t ldv, double *y, int64_t ldy, int nrhs, void *work, hipStream_t s);

// ---------------------------------------------------------------- FPS
// Landmarks in selection order (Algorithm 6); idx_dev gets k entries, seld_dev
// (optional) the squared selection distances.  work: fps_workspace_bytes(n).
// err_dev is set to 1 if an invalid winner index ever appears.
size_t fps_workspace_bytes(int64_t n);
afn_status fps(const double *X, int64_t n, int d, int k, int32_t *idx_dev, double *seld_dev,
               void *work, hipStream_t s, int *err_dev);
// A second stream with two events for work that runs beside the setup
// stream.  Streams and events come from a pool of the calling host thread
// (per device; created on first use and kept for the thread's lifetime, as
// creating them cost about as much as the work they overlap); the destructor
// waits for the stream's work (also on error paths, so nothing outlives the
// caller's workspace) and returns it to the pool.
struct SideStream {
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int slot = -1;
    SideStream() = default;
    SideStream(const SideStream &) = delete;
    SideStream &operator=(const SideStream &) = delete;
    afn_status open();
    ~SideStream();
};

// The same selection in pieces: fps_start picks the first point, fps_advance
// runs steps st0+1 .. st1 of a k_total-step selection and can be resumed.
afn_status fps_start(const double *X, int64_t n, int d, void *work, hipStream_t s, int *err);
afn_status fps_advance(const double *X, int64_t n, int d, int st0, int st1, int k_total, int32_t *idx,
                       double *seld, void *work, hipStream_t s, int *err);
// perm = [idx (k entries) ; the other indices ascending]; sel: n ints scratch.
afn_status landmark_permutation(const int32_t *idx, int k, int64_t n, int32_t *perm, int *sel,
                                hipStream_t s);

// ---------------------------------------------------------------- kNN pattern
// Row p (0 <= p < nr) of the predecessor pattern over Xr (row-major nr x d):
// cols[p*w .. p*w+len) (ascending, p last), len = min(p+1, w), the rest -1.
afn_status knn_pattern(const double *Xr, int64_t nr, int d, int w, int32_t *cols,
                       hipStream_t s);
// The same pattern with the help of a spatial order of Xr (order[q] = index
// at position q, d <= 8; otherwise as knn_pattern): 64-point tiles of the
// order with boxes prune candidate tiles.  work: knn_work_bytes(nr, d).
size_t knn_work_bytes(int64_t nr, int d);
afn_status knn_pattern_ordered(const double *Xr, int64_t nr, int d, int w, const int32_t *order, void *work,
                               int32_t *cols, hipStream_t s);

// ---------------------------------------------------------------- dense factors
// A = K11 + mu I for the first k points of Xp, column-major lda.
afn_status fill_k11(const double *Xp, int k, int d, double l, int kind, double mu, double *A, int64_t lda,
                    hipStream_t s);
// K12[t + p*k] = K(x_t, x_{k+p}) for t < k, p < n - k.
afn_status fill_k12(const double *Xp, int64_t n, int k, int d, double l, int kind, double *K12,
                    hipStream_t s);
// K12 columns of the FSAI patterns of rows r0 .. r0+B-1 (k x B w, see
// fsai_rows_batched).
afn_status fill_k12_patterns(const double *Xp, int64_t n, int k, int d, double l, int kind, const int32_t *cols,
                             int w, int64_t r0, int64_t B, double *Kb, hipStream_t s);
// In-place lower Cholesky; *info_dev = 1 + index of the first non-positive pivot.
afn_status cholesky(double *A, int k, int64_t lda, int *info_dev, hipStream_t s);
// Inverses of the 64 x 64 diagonal blocks of L (dinv_doubles(k) doubles).
int64_t dinv_doubles(int k);
afn_status diag_inverses(const double *L, int k, double *Dinv, hipStream_t s);
// B (k x ncols, ld k) := L^{-1} B.  unit: B is the identity (k = ncols), so
// the rows above each column's diagonal are not touched.
afn_status trsm_lower(const double *L, const double *Dinv, int k, double *B, int64_t ncols,
                      hipStream_t s, bool unit = false);
afn_status identity(double *A, int k, hipStream_t s);
// A[i + j lda] = 0 for i < j < k.
afn_status zero_upper(double *A, int k, int64_t lda, hipStream_t s);
// A[i + i lda] += shift for i < k.
afn_status add_diagonal(double *A, int k, int64_t lda, double shift, hipStream_t s);
// B[t + i ldb] = A[i + t lda] for i, t < k (B = A^T of a k x k block).
afn_status transpose_square(const double *A, int k, int64_t lda, double *B, int64_t ldb, hipStream_t s);

// ---------------------------------------------------------------- FSAI
// Padded rows of G (nr x w; row p has min(p+1, w) entries) for the Schur
// complement, from V = L^{-1} K12 (k x nr) and the points.  *info_dev = 1 on
// a non-positive pivot of a Schur block.
// order (optional, nr entries): the sequence in which rows are processed.
afn_status fsai_rows(const double *Xp, int64_t n, int k, int d, double l, int kind, double mu,
                     const double *V, const int32_t *cols, int w, double *gval, int *info_dev,
                     const int32_t *order, hipStream_t s);
// The same rows with the V columns of each row's pattern recomputed instead of
// gathered from V: batches of rows whose pattern columns of K12 are filled
// and multiplied by L^{-1} (an MFMA GEMM), then read contiguously.  For point
// sets whose neighbourhoods share few columns (high dimension), where
// gathers from V would come from HBM.  The columns equal V's to within the
// rounding of the two products (V comes from a triangular solve).
// work: fsai_batch_doubles(k, w) doubles.
int64_t fsai_batch_rows(int k, int w);
int64_t fsai_batch_doubles(int k, int w);
afn_status fsai_rows_batched(const double *Xp, int64_t n, int k, int d, double l, int kind, double mu,
                             const double *Linv, const int32_t *cols, int w, double *gval, int *info,
                             double *work, hipStream_t s);

// ---------------------------------------------------------------- spatial order
// order[q] = index of the point at position q: Hilbert order of grid cells over
// the points X (n x d row-major), ascending index inside a cell.
// Deterministic.  work: spatial_order_work_bytes(n, d).
size_t spatial_order_work_bytes(int64_t n, int d);
afn_status spatial_order(const double *X, int64_t n, int d, int32_t *order, void *work, hipStream_t s);
// CSR of G^T: tptr (nr+1), trow/tval (nnz), rows of each column ascending.
// work: fsai_transpose_work_bytes(nr, w) bytes.
size_t fsai_transpose_work_bytes(int64_t nr, int w);
afn_status fsai_transpose(const int32_t *cols, const double *gval, int64_t nr, int w,
                          int64_t *tptr, int32_t *trow, double *tval, void *work, hipStream_t s);

// ---------------------------------------------------------------- vectors
int64_t dot_partials(int64_t n);
// out[c] = sum_i a[i + c*lda] b[i + c*ldb] (fixed reduction order).
afn_status dot(const double *a, int64_t lda, const double *b, int64_t ldb, int64_t n, int nrhs,
               double *out_dev, double *partials, hipStream_t s);
afn_status dot(const float *a, int64_t lda, const float *b, int64_t ldb, int64_t n, int nrhs,
               double *out_dev, double *partials, hipStream_t s);
int64_t gemv_partials(int64_t m, int64_t ncols);
// y = base + sign * A x  (A m x ncols, column-major lda; base may be null)
afn_status gemv_n(const double *A, int64_t lda, int64_t m, int64_t ncols, const double *x,
                  const double *base, double sign, double *y, double *part, hipStream_t s);
afn_status gemv_n(const float *A, int64_t lda, int64_t m, int64_t ncols, const float *x,
                  const float *base, float sign, float *y, float *part, hipStream_t s);
// y = base + sign * A^T x
afn_status gemv_t(const double *A, int64_t lda, int64_t m, int64_t ncols, const double *x,
                  const double *base, double sign, double *y, hipStream_t s);
afn_status gemv_t(const float *A, int64_t lda, int64_t m, int64_t ncols, const float *x,
                  const float *base, float sign, float *y, hipStream_t s);
// u = G t (padded rows) ;  out = G^T u (CSR of G^T).  order (optional): the
// rows are visited in this order, each XCD taking a contiguous range of it
// (a spatial order keeps the gathers of concurrent rows in one L2); results
// do not depend on it.
afn_status spmv_g(const int32_t *cols, const double *gval, int64_t nr, int w, const double *t,
                  double *u, const int32_t *order, hipStream_t s);
afn_status spmv_g(const int32_t *cols, const float *gval, int64_t nr, int w, const float *t, float *u,
                  const int32_t *order, hipStream_t s);
afn_status spmv_gt(const int64_t *ptr, const int32_t *idx, const double *val, int64_t nr,
                   const double *u, double *out, const int32_t *order, hipStream_t s);
afn_status spmv_gt(const int64_t *ptr, const int32_t *idx, const float *val, int64_t nr,
                   const float *u, float *out, const int32_t *order, hipStream_t s);
// The FP32 products with BF16 factors (AFN_BF16).
afn_status gemv_n(const bf16_t *A, int64_t lda, int64_t m, int64_t ncols, const float *x, const float *base,
                  float sign, float *y, float *part, hipStream_t s);
afn_status gemv_t(const bf16_t *A, int64_t lda, int64_t m, int64_t ncols, const float *x, const float *base,
                  float sign, float *y, hipStream_t s);
afn_status spmv_g(const int32_t *cols, const bf16_t *gval, int64_t nr, int w, const float *t, float *u,
                  const int32_t *order, hipStream_t s);
afn_status spmv_gt(const int64_t *ptr, const int32_t *idx, const bf16_t *val, int64_t nr, const float *u,
                   float *out, const int32_t *order, hipStream_t s);
// b[i] = a[i] rounded to BF16 (nearest, ties to even, through FP32); n values.
afn_status to_bf16_launch(const double *a, bf16_t *b, int64_t n, hipStream_t s);
// a[i] = a[i] rounded to BF16 precision (kept in FP64; exact in BF16 after).
afn_status round_bf16_inplace_launch(double *a, int64_t n, hipStream_t s);
afn_status permute_gather(const double *src, int64_t lds, double *dst, int64_t ldd,
                          const int32_t *perm, int64_t n, int nrhs, hipStream_t s);
afn_status permute_scatter(const double *src, int64_t lds, double *dst, int64_t ldd,
                           const int32_t *perm, int64_t n, int nrhs, hipStream_t s);
afn_status gather_points(const double *X, const int32_t *perm, int64_t n, int d, double *Xp,
                         hipStream_t s);
// PCG scalar slots: sc[0] rho, sc[1] p'q, sc[2] r'r, sc[3] rho_new, sc[4] alpha,
// sc[5] beta, sc[6] b'b, sc[7] true residual squared.
// The same dot product as dot(), fused with the PCG scalar step that follows
// it: kPcgAlpha puts a.b in sc[1] and alpha = sc[0] / sc[1] in sc[4];
// kPcgBeta puts a.b in sc[3], then beta = sc[3] / sc[0] in sc[5] and sc[3]
// in sc[0].
enum PcgDotStep { kPcgAlpha = 1, kPcgBeta = 2 };
afn_status dot_pcg(const double *a, const double *b, int64_t n, double *sc, PcgDotStep step,
                   double *partials, hipStream_t s);
afn_status dot_pcg(const float *a, const float *b, int64_t n, double *sc, PcgDotStep step,
                   double *partials, hipStream_t s);
afn_status pcg_xr_launch(double *x, double *r, const double *p, const double *q, const double *sc,
                         int64_t n, double *part, double *rr_out, hipStream_t s);
afn_status pcg_xr_launch(float *x, float *r, const float *p, const float *q, const double *sc,
                         int64_t n, double *part, double *rr_out, hipStream_t s);
afn_status pcg_p_launch(double *p, const double *z, const double *sc, int64_t n, hipStream_t s);
afn_status pcg_p_launch(float *p, const float *z, const double *sc, int64_t n, hipStream_t s);
// r32 = r * scale; x += a * e; b = (float) a
afn_status to_f32_scaled_launch(const double *r, double scale, float *r32, int64_t n, hipStream_t s);
afn_status axpy_f32_into_f64_launch(double a, const float *e, double *x, int64_t n, hipStream_t s);
afn_status to_f32_launch(const double *a, float *b, int64_t n, hipStream_t s);
afn_status sub_launch(const double *b, const double *y, double *r, int64_t n, hipStream_t s);
afn_status scale_launch(double *x, double a, int64_t n, hipStream_t s);
afn_status scale_launch(float *x, float a, int64_t n, hipStream_t s);
// *flag |= 1 if a value is not finite
afn_status finite_launch(const double *a, int64_t n, int *flag, hipStream_t s);

// ---------------------------------------------------------------- many right-hand sides
// Row-major (point-major) n x R blocks, R <= 64.
int mrhs_splits(int64_t npad);
int64_t mrhs_part_elems(int64_t npad);
template <typename T>
afn_status kmv_mrhs_run(const T *Xs, int64_t npad, int64_t n, int d, double mu, int kind, const T *P,
                        int64_t ldp, T *Y, int64_t ldy, int R, T *part, hipStream_t s,
                        hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                        const int32_t *perm = nullptr, const T *box = nullptr);
int gemm_splits(int64_t m, int64_t K);
int64_t gemm_part_elems(int64_t m, int64_t K);
// Partial-sum elements enough for gemm_rows with any m <= mmax.
int64_t gemm_part_bound(int64_t mmax);
template <typename T>
afn_status gemm_rows(const T *A, int64_t ars, int64_t acs, int64_t m, int64_t K, const T *B,
                     int64_t ldb, int R, const T *base, T sign, T *C, int64_t ldc, T *part,
                     hipStream_t s);
// G and G^T on R columns (row-major blocks); order as for spmv_g.
template <typename T>
afn_status spmm_g(const int32_t *cols, const T *g, int64_t nr, int w, const T *X, int R, T *U,
                  const int32_t *order, hipStream_t s);
template <typename T>
afn_status spmm_gt(const int64_t *ptr, const int32_t *idx, const T *val, int64_t nr, const T *X,
                   int R, T *U, const int32_t *order, hipStream_t s);
int64_t coldot_blocks(int64_t n);
template <typename T>
afn_status coldot(const T *A, const T *B, int64_t n, int R, double *out, double *part,
                  hipStream_t s);
template <typename T>
afn_status col_xr_launch(T *X, T *Rv, const T *Pv, const T *Q, const double *alpha, int64_t n,
                         int R, double *rr, double *part, hipStream_t s);
template <typename T>
afn_status col_p_launch(T *Pv, const T *Z, const double *beta, int64_t n, int R, hipStream_t s);
afn_status col_alpha_launch(const double *rho, const double *pq, const int *active, double *alpha,
                            int R, int *bad, hipStream_t s);
afn_status col_beta_launch(double *rho, const double *rho_new, const int *active, double *beta,
                           int R, hipStream_t s);
afn_status col_converged_launch(const double *rr, const double *bnorm2, const double *tol,
                                int *active, int *count, int R, int *bad, hipStream_t s);
template <typename T>
afn_status gather_rows(const double *X, int64_t ld, const int32_t *perm, int64_t n, int R,
                       const double *scale, T *Y, hipStream_t s);
afn_status scatter_rows(const double *Y, const int32_t *perm, int64_t n, int R, double *X,
                        int64_t ld, hipStream_t s);
afn_status scatter_rows_f32(const float *Y, int64_t n, int R, double *X, int64_t ld,
                            hipStream_t s);
afn_status sub_rows_launch(const double *B, const double *Y, double *Rr, int64_t total,
                           hipStream_t s);
// Block solve (R <= 64, d <= 8, FP32 copies present); see block.hip.  Its
// workspace for R columns is carved at setup: block_workspace_bytes bytes.
size_t block_workspace_bytes(int64_t n, int d, int64_t k, int R);
afn_status block_refine_solve(afn_handle *h, const double *B, int64_t ld, double *Xout, int R,
                              double tol, int maxit, hipStream_t s, int *iters, int *outer,
                              double *relres_max, int *conv_all, int *col_ok);
afn_status scale_to_f32_launch(const double *r, const double *inv, float *r32, int64_t n, int R,
                               hipStream_t s);
afn_status axpy_cols_f32_launch(const double *a, const float *e32, double *x, int64_t n, int R,
                                hipStream_t s);

}  // namespace afn

// ------------------------------------------------------------------ handle
struct afn_handle {
    int device = 0;
    int64_t n = 0, nr = 0;
    int d = 0, k = 0, w = 0;
    double l = 1.0, mu = 0.0;
    int kind = AFN_KERNEL_GAUSSIAN;   // afn_kernel
    afn::DevArena arena;
    double *Xp = nullptr;       // n x d, block order (landmarks first)
    int32_t *perm = nullptr;    // n: block position -> original index
    double *L = nullptr;        // k x k column-major lower
    double *Linv = nullptr;     // k x k column-major lower
    double *Dinv = nullptr;     // inverses of the 64 x 64 diagonal blocks of L
    double *V = nullptr;        // k x nr column-major: V = L^{-1} K12
    int32_t *cols = nullptr;    // nr x w padded pattern rows (ascending, diagonal last)
    double *gval = nullptr;     // nr x w padded values of G
    int64_t *tptr = nullptr;    // CSR of G^T: nr + 1
    int32_t *trow = nullptr;    // nnz
    double *tval = nullptr;     // nnz
    int64_t nnz = 0;
    int *flags = nullptr;       // device status flags
    double *work = nullptr;     // PCG / apply workspace
    int64_t work_doubles = 0;
    int64_t work_rhs = 0;       // right-hand sides the workspace is sized for
    double *Xs64 = nullptr;     // points pre-scaled for the symmetric tile kernel (d <= 8),
                                // in the spatial order kperm, with per-tile boxes box64
    int32_t *kperm = nullptr;   // packed position -> block index
    double *box64 = nullptr;
    float *box32 = nullptr;
    int precision = AFN_FP64;   // AFN_FP32: inner PCG in FP32 inside FP64 refinement
    float *Xs32 = nullptr;      // FP32 copies for the inner solve
    float *Linv32 = nullptr;
    float *V32 = nullptr;
    float *gval32 = nullptr;
    float *tval32 = nullptr;
    float *work32 = nullptr;
    afn::bf16_t *Linv16 = nullptr;   // AFN_BF16: the inner apply's factors in BF16
    afn::bf16_t *V16 = nullptr;
    afn::bf16_t *gval16 = nullptr;
    afn::bf16_t *tval16 = nullptr;
    afn::bf16_t *W16 = nullptr;
    // Nystrom preconditioner (method == AFN_METHOD_NYSTROM): W = [L^T | V]
    // (k x n column-major, V = L^{-1} K12 with L = chol(K11 + nu I)) and the
    // inverse Rginv of the lower Cholesky factor of W W^T + mu I
    int method = AFN_METHOD_AFN;
    double *W = nullptr;
    double *Rginv = nullptr;
    float *W32 = nullptr;
    float *Rginv32 = nullptr;
    void *mrhs_ws = nullptr;    // workspace of block solves (carved at setup)
    int nrhs_block = 0;         // columns it holds (0: no block solves)
    hipStream_t block_stream = nullptr;  // stream of the graph-captured block solve
    hipEvent_t block_ev = nullptr;
    void *ws_owned = nullptr;   // the workspace, when the library allocated it
    bool active = false;        // a step-wise solve (afn_pcg_state) is started
    double *host_sc = nullptr;  // pinned host copy of PCG scalars
    hipEvent_t kmv_ev[2] = {nullptr, nullptr};  // timing of the matvec tile kernel
    hipEvent_t chk_ev = nullptr;                // the PCG residual check's host copy
    hipEvent_t end_ev = nullptr;                // a step-wise solve moving to another stream
    int32_t *rorder = nullptr;                  // spatial order of the non-landmark rows (d <= 10)
    afn_setup_info info{};
};
