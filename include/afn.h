/*
 * afn.h -- C-ABI of libafn: AFN-preconditioned conjugate gradients for
 * regularized kernel systems on AMD Instinct MI355X (gfx950).
 *
 * Method: "An Adaptive Factorized Nystrom Preconditioner for Regularized
 * Kernel Matrices" (Zhao, Xu, Huang, Chow, Xi; arXiv 2304.05460).
 * Problem (Eq. (1.1)): solve (K + mu I) a = b with the Gaussian kernel
 *   K_ij = exp(-||x_i - x_j||^2 / l^2)                      (Eq. (1.2)),
 * or the Matern-3/2 kernel of Section 5 (afn_kernel).
 *
 * Conventions shared by every entry point:
 *  - Pointers named *_dev are DEVICE pointers (e.g. from contiguous torch
 *    tensors on the current HIP device); pointers named *_host are host
 *    pointers.  The caller owns every buffer it passes; the library never
 *    frees or retains caller buffers beyond the call.
 *  - Points X are FP64, row-major n x d (point i at X[i*d .. i*d+d-1]).
 *    Vectors are FP64 column-major n x nrhs with leading dimension ld >= n.
 *    Every vector crosses the boundary in the ORIGINAL point order; the
 *    landmark-first ordering is internal.
 *  - 'stream' is a hipStream_t (NULL = the default stream).  Work is
 *    stream-ordered.  kernel_matvec and afn_apply return without waiting;
 *    afn_setup and afn_pcg_solve synchronize the stream before returning,
 *    because they take host decisions (landmark count, convergence).
 *  - Every function returns an afn_status; failures never throw across the
 *    boundary.  afn_last_error() returns a thread-local message describing
 *    the last failure on the calling thread.  On failure, outputs other than
 *    those documented are unspecified.
 *  - A handle may be used by one host thread at a time, and its calls must
 *    not overlap on the device: they share the handle's workspace (use one
 *    stream per handle, or synchronize between calls on different streams).
 *    Different handles are independent.
 *  - Device memory: a handle lives in one workspace that the caller passes
 *    to afn_setup (afn_workspace_size bytes); setup and solves allocate no
 *    device memory of their own.  kernel_matvec keeps a per-device scratch
 *    area that it grows on demand; kernel_matvec_noalloc uses a static one.
 */
#ifndef AFN_H
#define AFN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum afn_status {
    AFN_OK = 0,
    AFN_EINVAL = 1,        /* invalid argument (sizes, l <= 0, mu < 0, ...)            */
    AFN_ENOMEM = 2,        /* device allocation failed                                 */
    AFN_ENOTSPD = 3,       /* a Cholesky pivot of K11 + mu I or of an FSAI block <= 0  */
    AFN_ENOCONV = 4,       /* PCG reached maxit; x holds the last iterate, info valid  */
    AFN_EBREAKDOWN = 5,    /* PCG breakdown: p'Ap <= 0 or a NaN appeared               */
    AFN_ESTAGNATION = 6,   /* iterative refinement stopped reducing the residual       */
    AFN_EDEVICE = 7        /* a HIP runtime call failed                                */
} afn_status;

/* Arithmetic.  kernel_matvec: AFN_FP64 = FP64 tiles; AFN_FP32 = distances,
 * kernel values and per-workgroup sums in FP32 (partials added in FP64,
 * vectors FP64 at the boundary).  afn_setup: AFN_FP32 makes afn_pcg_solve use
 * iterative refinement: the residual b - (K + mu I) x and the solution are
 * FP64, each correction comes from an inner PCG whose operator, preconditioner
 * apply and vectors are FP32 and whose scalar recurrences are FP64; the
 * factors are built in FP64 (L = chol(K11 + mu I) in FP64) and rounded.  If
 * an inner PCG breaks down (p'Ap <= 0 in FP32), or the refinement stops
 * halving the residual, or the inner products exceed 4 maxit, the solve
 * continues with textbook FP64 PCG from the current x (at most maxit more
 * products), so a mixed solve fails only where the FP64 solve would.
 * afn_setup with AFN_BF16: the same refinement, with the factors of the inner
 * apply stored in BF16 (V = L^{-1} K12, L^{-1}, G, G^T, or the Nystrom
 * W = L^{-1} K[S, :]) and widened to FP32 on load, sums in FP32; the Nystrom
 * W W^T + mu I is formed (in FP64) from the BF16-rounded W and its inverse
 * factor kept in FP32, so the inner preconditioner stays symmetric positive
 * definite.  Several right-hand sides are solved one at a time.  AFN_BF16 is
 * not a kernel_matvec precision (the operator of the inner solves is FP32). */
typedef enum afn_precision {
    AFN_FP64 = 0,
    AFN_FP32 = 1,
    AFN_BF16 = 2
} afn_precision;

/* Preconditioner (Algorithm 5).  AFN_METHOD_AFN: the AFN factorization
 * (Algorithm 2).  AFN_METHOD_NYSTROM: the column-sampling Nystrom
 * preconditioner M = K_nys + mu I on the same FPS landmarks, applied by the
 * Sherman-Morrison-Woodbury identity (Section 2) -- with
 * B = K[:, S] chol(K_SS + nu I)^{-T} (nu = eps ||K[:, S]||_F, the stabilizing
 * shift of the randomized Nystrom construction) it computes
 * M^{-1} r = (r - B (B^T B + mu I)^{-1} B^T r) / mu, which equals
 * U (Lambda + mu I)^{-1} U^T r + (r - U U^T r) / mu for the thin SVD
 * B = U Sigma V^T up to the shift (Lambda = Sigma^2 - nu; relative
 * difference <= nu / mu).  Needs mu > 0.  AFN_METHOD_AUTO: Algorithm 5's
 * choice -- Nystrom when the rank (the estimate of Algorithm 4, or k when
 * given) is below 2000, AFN otherwise. */
typedef enum afn_method {
    AFN_METHOD_AFN = 0,
    AFN_METHOD_NYSTROM = 1,
    AFN_METHOD_AUTO = 2
} afn_method;

/* Kernel function (Section 5), r = ||x - y||:
 *   AFN_KERNEL_GAUSSIAN   exp(-r^2 / l^2)                       (Eq. (1.2))
 *   AFN_KERNEL_MATERN32   (1 + sqrt(3) r / l) exp(-sqrt(3) r / l). */
typedef enum afn_kernel {
    AFN_KERNEL_GAUSSIAN = 0,
    AFN_KERNEL_MATERN32 = 1
} afn_kernel;

/* Landmark selection (Algorithm 2): AFN_LANDMARKS_AUTO = farthest point
 * sampling (Algorithm 6) for d <= 10 and uniform sampling above;
 * AFN_LANDMARKS_FPS / AFN_LANDMARKS_UNIFORM force one of them.  Uniform
 * sampling takes the first k entries of the splitmix64 partial Fisher-Yates
 * shuffle of 0..n-1 seeded with seed + 1 (k <= 4096), in that order. */
typedef enum afn_landmarks {
    AFN_LANDMARKS_AUTO = 0,
    AFN_LANDMARKS_FPS = 1,
    AFN_LANDMARKS_UNIFORM = 2
} afn_landmarks;

/* Construction parameters (Algorithm 2, Algorithm 4, Algorithm 5). */
typedef struct afn_params {
    int32_t k;          /* landmark count; -1 = estimate it (Algorithm 4)         */
    int32_t k_max;      /* cap on the estimated count (Section 3.2: e.g. 2000)     */
    int32_t w;          /* FSAI nonzeros per row incl. the diagonal, 1 <= w <= 128 */
    int32_t m;          /* rank-estimation subsample size; 0 = min(n, 2000)        */
    int32_t precision;  /* afn_precision of the PCG solve (FP32, BF16 need d <= 8) */
    int32_t method;     /* afn_method                                              */
    uint64_t seed;      /* seed of the rank-estimation subsample (splitmix64)      */
    int32_t landmarks;  /* afn_landmarks                                           */
    int32_t kernel;     /* afn_kernel                                              */
    int32_t nrhs_max;   /* widest block solve to provision (AFN_FP32, d <= 8):
                           >= 2 carves a block workspace for min(nrhs_max, 64)
                           columns; 0 or 1: several columns are solved one at a
                           time                                                    */
    int32_t reserved;   /* zero                                                    */
} afn_params;

/* Facts about a constructed preconditioner. */
typedef struct afn_setup_info {
    int64_t n;
    int32_t d;
    int32_t k;               /* landmarks used                                     */
    int32_t w;
    int32_t rank_r;          /* Algorithm 4: Nystrom rank on the subsample, -1 if k given */
    int64_t rank_k_est;      /* Algorithm 4: floor(r n / m), -1 if k given         */
    int32_t rank_eig_branch; /* 1 if the eigenvalue count replaced k_est           */
    int32_t rank_eig_count;  /* that count, -1 if not computed                     */
    int64_t nnz_g;           /* nonzeros of the FSAI factor G (0 for Nystrom)      */
    double ms_rank, ms_fps, ms_chol, ms_knn, ms_v, ms_fsai, ms_total;  /* phase times;
                                Nystrom: ms_fsai = forming and factoring B^T B + mu I */
    int32_t method;          /* afn_method built: AFN_METHOD_AFN or _NYSTROM       */
    int32_t landmarks;       /* AFN_LANDMARKS_FPS or _UNIFORM, as used             */
    double nu;               /* Nystrom stabilizing shift (0 for AFN)              */
    double kmv_kept_f64;     /* fraction of tile pairs the pruned kernel matvec   */
    double kmv_kept_f32;     /* evaluates with FP64 / FP32 tiles (1 if not pruned) */
    double kmv_far_f64;      /* fraction of tile pairs whose FP64 values are all
                                below 2^-46 and take the FP32 exponential (d <= 4;
                                0 otherwise)                                       */
    int64_t ws_bytes;        /* workspace size (afn_workspace_size)                 */
    int64_t ws_bytes_used;   /* bytes of it the setup carved                        */
} afn_setup_info;

/* Result of a PCG solve. */
typedef struct afn_solve_info {
    int32_t iterations;        /* products with K + mu I (per right-hand side: max) */
    int32_t converged;         /* 1 if every right-hand side met tol                */
    double relres;             /* recurrence residual ||r|| / ||b|| (max over rhs)   */
    double relres_true;        /* ||b - (K + mu I) x|| / ||b|| recomputed in FP64    */
    double ms_solve;
    double ms_matvec;          /* summed device time of the PCG operator's tile kernel
                                  (FP64, or FP32 for the inner solves of a mixed solve),
                                  from HIP events recorded around each of its launches */
    int32_t matvec_launches;   /* launches timed in ms_matvec                        */
    int32_t outer_iterations;  /* refinement steps of a mixed solve; 0 for FP64      */
    int32_t fp64_iterations;   /* mixed solve: FP64 PCG products after the FP32
                                  corrections broke down or stalled (max over rhs)  */
    int32_t grouped_units;     /* step-wise solve: units of work it advanced inside
                                  grouped launches shared with other solves
                                  (afn_pcg_step_many); 0 for afn_pcg_solve         */
} afn_solve_info;

typedef struct afn_handle afn_handle;

/* y = (K + mu I) v  (Eq. (1.1)), K evaluated on the fly from X (Eq. (1.2)).
 * X_dev: n x d FP64 row-major.  v_dev, y_dev: n x nrhs FP64 column-major,
 * leading dimension ld >= n; y must not alias v.  precision: afn_precision.
 * Asynchronous on 'stream'.  Uses a library-owned per-device workspace
 * (grown on demand, kept until the process ends): calls on one device that
 * overlap in time, from several threads or streams, race on it.  The handle
 * functions below use only per-handle memory and may run concurrently on
 * different handles and streams.  Errors: EINVAL (n < 1, d < 1 or d > 64,
 * l <= 0, mu < 0, nrhs < 1, ld < n), ENOMEM, EDEVICE. */
afn_status kernel_matvec(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                         const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld,
                         int32_t precision, void *stream);

/* kernel_matvec with the kernel function chosen (afn_kernel); kernel_matvec
 * is kernel_matvec_ex with AFN_KERNEL_GAUSSIAN.  Errors as kernel_matvec,
 * and EINVAL for an unknown kernel. */
afn_status kernel_matvec_ex(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                            const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld,
                            int32_t precision, int32_t kernel, void *stream);

/* kernel_matvec_ex for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, bit for bit, with the scratch
 * (spatial order, packed points, tile boxes, partial sums) in a static
 * 192 MiB device array that each device holds until the process ends.  No
 * device memory is allocated or freed by the call.  The scratch needed grows
 * with n (n = 1e5 at d = 3 fits with one column, n = 6000 with up to 64
 * columns: the many-column partial sums are larger); a call that would
 * need more is rejected on the host with EINVAL before any device work.
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (several threads or streams) race on it.  Errors as
 * kernel_matvec_ex, and EDEVICE if the array's address cannot be taken. */
afn_status kernel_matvec_noalloc(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                                 const double *v_dev, double *y_dev, int32_t nrhs, int64_t ld,
                                 int32_t precision, int32_t kernel, void *stream);

/* Device memory, in bytes, that afn_setup carves from its workspace for n
 * points in d dimensions with these parameters: the handle's persistent
 * buffers (points, permutation, L, L^{-1}, V = L^{-1} K12, the pattern, G,
 * G^T, their FP32 copies, packed points, PCG vectors, the block-solve
 * workspace of params->nrhs_max columns) plus every temporary of the
 * construction (rank estimation, FPS, orderings, transposes), which are
 * carved from the same workspace and not reused.  An adaptive landmark count
 * (k = -1) is priced at min(k_max, n), the most Algorithm 4 can return.
 * Host-only (no device call); a serving loop admits requests by this number.
 * Errors: EINVAL (as afn_setup). */
afn_status afn_workspace_size(int64_t n, int32_t d, const afn_params *params, size_t *bytes);

/* Construct the preconditioner.  AFN (Algorithm 2): landmarks by farthest
 * point sampling (Algorithm 6) -- k from params or estimated (Algorithm 4) --,
 * L = chol(K11 + mu I), and the FSAI factor G of the Schur complement
 * K22 + mu I - K12^T (K11 + mu I)^{-1} K12 (Algorithm 1) on the pattern of
 * the w-1 nearest earlier-numbered points (Section 3.1).  Nystrom and the
 * Algorithm 5 choice: see afn_method (w is then unused).
 * ws_dev: caller-owned device workspace of ws_bytes >= afn_workspace_size
 * bytes, 256-byte aligned; every device buffer of the handle and of its
 * solves lives in it, the library allocates no device memory, and the
 * workspace must stay allocated until afn_destroy.  ws_dev = NULL: the
 * library allocates one block of afn_workspace_size bytes itself and frees it
 * in afn_destroy.  The library copies what it needs from X_dev.  Synchronizes
 * 'stream'.  Errors: EINVAL (n < 1, d < 1 or d > 64, l <= 0, mu < 0, k < -1
 * or k > n, w < 1 or w > 64, unknown method, Nystrom with mu = 0, a
 * misaligned ws_dev), ENOMEM (ws_bytes below afn_workspace_size, or the
 * library's own allocation failed), ENOTSPD, EDEVICE.  *out is NULL on
 * failure. */
afn_status afn_setup(const double *X_dev, int64_t n, int32_t d, double l, double mu,
                     const afn_params *params, void *ws_dev, size_t ws_bytes, void *stream,
                     afn_handle **out);

/* z = M^{-1} r (Algorithm 3) for nrhs columns:
 *   s2 = G^T G (r2 - K12^T (K11 + mu I)^{-1} r1),
 *   s1 = (K11 + mu I)^{-1} (r1 - K12 s2).
 * r_dev, z_dev: n x nrhs FP64 column-major, leading dimension ld >= n, no
 * aliasing.  Asynchronous.  Errors: EINVAL, EDEVICE. */
afn_status afn_apply(afn_handle *h, const double *r_dev, double *z_dev, int32_t nrhs,
                     int64_t ld, void *stream);

/* Preconditioned CG from x0 = 0 (Algorithm 5, AFN branch) for each of nrhs
 * right-hand sides, stopping when ||r|| / ||b|| <= tol (Section 5 stopping
 * rule) or after maxit products with K + mu I.  A handle set up with
 * precision AFN_FP32 solves by iterative refinement instead: the FP64
 * residual ||b - (K + mu I) x|| / ||b|| is the stopping test, each inner FP32
 * PCG runs at most maxit iterations and stops at the relative residual its
 * step needs (half of tol over the current FP64 residual), but at 3e-2 at
 * the lowest, and the FP64 PCG described under
 * afn_precision takes over when the FP32 corrections stop working (the
 * status is then that of the FP64 PCG).  On a handle whose setup
 * provisioned a block workspace (AFN_FP32, d <= 8, params.nrhs_max >= 2) the
 * right-hand sides go through the block solver nrhs_max (at most 64) at a
 * time, on a stream the handle owns, ordered after 'stream'; a column it
 * leaves above tol is solved again on its own.  Otherwise the columns are
 * solved one at a time.  No device memory is allocated.  b_dev, x_dev: n x nrhs FP64
 * column-major, leading dimension ld.  info_host may be NULL.  Synchronizes.
 * Errors: EINVAL (tol <= 0, maxit < 1, nrhs < 1, ld < n), ENOCONV (x holds
 * the last iterate, info valid), EBREAKDOWN, ESTAGNATION, EDEVICE. */
afn_status afn_pcg_solve(afn_handle *h, const double *b_dev, double *x_dev, int32_t nrhs,
                         int64_t ld, double tol, int32_t maxit, afn_solve_info *info_host,
                         void *stream);

/* Setup facts (landmark count, rank-estimation outcome, phase timings). */
afn_status afn_get_info(const afn_handle *h, afn_setup_info *info_host);

/* Landmark indices (original numbering, FPS selection order) into idx_host
 * (capacity cap >= k).  *k_out = k.  Synchronous. */
afn_status afn_get_landmarks(const afn_handle *h, int32_t *idx_host, int64_t cap, int64_t *k_out);

/* FSAI sparsity pattern in CSR over the non-landmark points, numbered
 * 0..n-k-1 in ascending original index: rowptr_host (n-k+1 entries),
 * cols_host (capacity cap >= nnz; columns ascending, the diagonal last) and,
 * if vals_host is not NULL, the values of G (capacity cap).  *nnz_out = nnz. */
afn_status afn_get_fsai(const afn_handle *h, int64_t *rowptr_host, int32_t *cols_host,
                        double *vals_host, int64_t cap, int64_t *nnz_out);

/* The Cholesky factor L of K11 + mu I, k x k column-major (lower triangle;
 * the strict upper triangle is written as zero) into L_host with leading
 * dimension ld >= k.  Synchronous. */
afn_status afn_get_cholesky(const afn_handle *h, double *L_host, int64_t ld);

/* The same number as afn_workspace_size (kept for admission code). */
afn_status afn_footprint_bytes(int64_t n, int32_t d, const afn_params *params, size_t *bytes);

/* ---- Step-wise PCG (Algorithm 5's solve, advanced from outside) -------------
 * For a serving loop that advances many solves together: afn_pcg_begin
 * starts the solve of one right-hand side on a handle, afn_pcg_step_many
 * advances several started solves (on different handles) by a number of
 * iterations each, with one host wait per iteration for all of them, and
 * afn_pcg_query reports progress.  The iterates, stopping tests and results
 * are those of afn_pcg_solve with nrhs = 1 on the same handle, bit for bit
 * (FP64 PCG, or the iterative refinement of an AFN_FP32 handle with its FP64
 * fallback).  A state lives in its handle's workspace: one started solve per
 * handle at a time. */
typedef struct afn_pcg_state afn_pcg_state;

/* Start solving (K + mu I) x = b from x0 = 0 (b_dev, x_dev: n FP64 device
 * vectors in the original point order, not aliasing; both must stay
 * allocated until the solve is done).  Queues work on 'stream' and returns
 * without waiting.  Errors: EINVAL (tol <= 0, maxit < 1, a solve already
 * started on h), EDEVICE. */
afn_status afn_pcg_begin(afn_handle *h, const double *b_dev, double *x_dev, double tol, int32_t maxit,
                         void *stream, afn_pcg_state **out);

/* Advance each unfinished state in states[0..count) by up to 'iters'
 * products with K + mu I.  Every state keeps one unit of work in flight (an
 * iteration, or a refinement step's residual norm); the host polls their
 * events and takes each stopping decision as soon as that state's unit is
 * done, then queues its next one, so solves of different sizes advance at
 * their own pace.  The call returns when every state has finished or taken
 * 'iters' products, or, earlier, at the end of the first polling pass in
 * which a state finished (so the caller can release it and start another);
 * units still in flight stay with their states for the next call.  stream
 * NULL: each state's work goes on the stream it was begun on, so solves
 * overlap on the device; otherwise all of it goes on 'stream' (ordered after
 * the begin streams; pass the same value on every call for a state).  A state
 * that finishes writes x_dev and its info.
 *
 * Continuous batching (Algorithm 5's solve for many requests at once): the
 * units due in one polling pass are queued together; the inner FP32/BF16
 * iterations of like mixed-precision solves -- same d, kernel, precision,
 * method and pattern width, n within a factor of 2 -- run as ONE ragged
 * launch per kernel over all of them (a table of per-solve arguments and
 * block offsets passed as the kernel argument, at most 16 solves per launch;
 * no device memory of its own), on the stream of the first of them.  An inner
 * iteration that is due while a like solve's is in flight waits for it, so
 * like solves stay aligned.  Each solve's arithmetic is that of its own
 * launches: results are bitwise those of afn_pcg_solve.  info.grouped_units
 * counts the units a solve advanced in grouped launches.
 *
 * Errors: EINVAL (a NULL state, count < 1, iters < 1, two states on one
 * handle), EDEVICE; the outcome of each solve is read by afn_pcg_query. */
afn_status afn_pcg_step_many(afn_pcg_state *const *states, int32_t count, int32_t iters, void *stream);

/* Grouped launches in afn_pcg_step_many on (1, the default unless the
 * environment variable AFN_NO_GROUP=1 is set at load) or off (0: every unit
 * queued on its own; the results are the same bits).  Process-wide; takes
 * effect at the next afn_pcg_step_many call. */
void afn_group_config(int32_t on);

/* *done = 1 once the solve has finished; info_host (may be NULL) then holds
 * the result, and the return value is the solve's status (OK, ENOCONV,
 * EBREAKDOWN, ESTAGNATION).  Before that: *done = 0, AFN_OK, info_host
 * holds the iterations so far. */
afn_status afn_pcg_query(const afn_pcg_state *st, int32_t *done, afn_solve_info *info_host);

/* Release a state (finished or not), waiting for a unit it has in flight;
 * its handle can start another solve. */
void afn_pcg_end(afn_pcg_state *st);

/* Release the handle and its device memory.  NULL is allowed.  Work the
 * caller queued with afn_apply on the handle must be complete. */
void afn_destroy(afn_handle *h);

/* ---- Autotuner of launch shapes ---------------------------------------------
 * Tunables with a few candidates each, all computing the same result up to
 * the order of the sums: the tile kernel of the kernel matvec for d = 5..8
 * with tile boxes (MFMA distance contraction or plain differences), the
 * split count of the split-K GEMMs (the batched apply of block solves, the
 * Nystrom W W^T, the high-dimension FSAI columns) and the split count of the
 * GEMVs of the apply.  Modes: AFN_TUNE_OFF (default: the built-in
 * heuristics), AFN_TUNE_ON (the first call that meets a new shape class, on
 * a stream that is not recording a graph, times every candidate on its own
 * buffers -- one warm-up and three timed runs each -- and keeps the fastest
 * for the process), AFN_TUNE_FORCE (candidate 'index' of every tunable,
 * clamped to its count: for tests that every candidate agrees).  Decisions are
 * keyed by tunable, shape class and device (architecture and CU count).
 * cache_path (may be NULL): decisions are read from it now and the whole
 * table is written to it after each new decision, one "key choice" line each.
 * Process-wide; calls that overlap with it are not allowed.  Errors: EINVAL. */
typedef enum afn_tune_mode {
    AFN_TUNE_OFF = 0,
    AFN_TUNE_ON = 1,
    AFN_TUNE_FORCE = 2
} afn_tune_mode;
afn_status afn_tune_config(int32_t mode, int32_t index, const char *cache_path);

/* The decisions so far as text, one line per shape class: key, chosen
 * candidate and the measured milliseconds of each candidate (none for those
 * read from a cache file).  Writes at most cap - 1 characters and a NUL;
 * *len = the full length.  Errors: EINVAL. */
afn_status afn_tune_report(char *buf_host, int64_t cap, int64_t *len);

/* Static description of a status code. */
const char *afn_status_string(afn_status s);

/* Thread-local message of the last failure on this thread ("" if none). */
const char *afn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* AFN_H */
