/*
 * skltlt -- pivoted LTL^T factorization of skew-symmetric matrices and their
 * Pfaffians on AMD Instinct MI355X (gfx950).  C ABI of libskltlt.so.
 *
 * Paper: "Performant Tridiagonal Factorization of Skew-Symmetric Matrices",
 * arXiv 2411.09859.  The operation is the one of Sec. 3.2 (Specification):
 * for a skew-symmetric X (X = -X^T, Sec. 2.2) compute a unit lower
 * triangular L whose first column is e_0 and a skew-symmetric tridiagonal T
 * with P X P^T = L T L^T, overwriting X.  P comes from symmetric partial
 * pivoting (Sec. 3.7).  The Pfaffian follows from Sec. 1 and Sec. 2.2:
 * Pf(X) = det(P) * Pf(T) = det(P) * prod_i T[2i][2i+1].
 *
 * Conventions shared by every call:
 *   - Matrices are fp64, column-major, 0-based, leading dimension lda >= n.
 *   - Only the STRICT LOWER triangle of A is read or written; the diagonal
 *     and the upper triangle are never touched (the implicit structure of
 *     Sec. 2.4: unstored skew entries are neither read nor referenced).
 *   - Output layout in place (Sec. 4.1, "Storage details"): A[j+1][j] = t[j]
 *     (the subdiagonal of T; T[j][j+1] = -t[j]) and A[i][j] = L[i][j+1] for
 *     i >= j+2 (L shifted one column left; its unit diagonal and its first
 *     column e_0 are implicit).
 *   - ipiv is absolute and 0-based: ipiv[0] = 0 (the first pivot is never
 *     computed, caption of Fig. 5), and for r >= 1 ipiv[r] >= r is the row
 *     exchanged with row r (rows AND columns, P(pi) of Sec. 3.7.1) before
 *     column r of L was formed.  The permutation is P = P_{n-1} ... P_1 with
 *     P_r the transposition (r, ipiv[r]); (P A P^T)[i][j] = A[q[i]][q[j]]
 *     where q is the identity with those transpositions applied in order.
 *   - Pivot choice: largest magnitude in the column (iamax, Sec. 3.7.1),
 *     first index on ties.  A column with no non-zero candidate gives
 *     t = 0, a zero column of L and no exchange; this is not an error.
 *   - Pointers marked (device) are device pointers (hipMalloc or any device
 *     allocation of the current device); (host) are host pointers.
 *   - stream is a hipStream_t passed as void* (NULL: the null stream).  Work
 *     is enqueued asynchronously; buffers must stay alive until the stream
 *     has passed it.  The library allocates nothing on these paths and keeps
 *     no pointer after a call returns.
 *   - Every call returns a skltlt_status.  Argument errors are reported
 *     before anything is enqueued; a failed launch returns SKLTLT_EDEVICE.
 *     Inputs with NaN or Inf are outside the contract (as in LAPACK).
 *   - Calls on distinct streams with distinct buffers are independent; two
 *     calls may not share a workspace while both are in flight.
 *   - Concurrency: the panel kernels' workgroups wait for one another and
 *     must be resident together.  Panels of at most 16 workgroups (matrices
 *     up to order 2049 at panel width 256, the last panels of larger ones)
 *     are ordinary launches, so factorizations on different streams overlap;
 *     each of the first seven streams a process uses gets its own XCD for
 *     them.  Larger panels are cooperative launches, which the runtime runs
 *     one at a time across streams.  Up to seven streams factoring at once
 *     are guaranteed to make progress; beyond that a starved panel ends
 *     after its bounded waits with NaN in t (and the Pfaffian) rather than
 *     hanging.
 */
#ifndef SKLTLT_H
#define SKLTLT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SKLTLT_OK = 0,
    SKLTLT_EINVAL = -1,  /* bad argument (size, pointer, workspace, enum)    */
    SKLTLT_ENOMEM = -2,  /* reserved: the library itself never allocates     */
    SKLTLT_EDEVICE = -3, /* a HIP call or kernel launch failed               */
    SKLTLT_ENOTSUP = -4  /* size or option outside what the library supports */
} skltlt_status;

typedef enum {
    SKLTLT_FP64 = 0,        /* every step in fp64                                */
    SKLTLT_FP32_UPDATE = 1  /* trailing rank-2k update in fp32 MFMA with fp32
                               accumulation added to the fp64 matrix; pivot
                               search, panel, t and Pfaffian stay fp64        */
} skltlt_precision;

/* Human-readable name of a status code (static string, never NULL). */
const char *skltlt_status_string(int status);

/* Block size the library picks for order n when block_size = 0. */
int skltlt_default_block_size(int n);

/* Bytes of device workspace that skltlt_factor / skltlt_pfaffian need for
 * (n, block_size, precision).  *bytes (host) receives the size; the same
 * value is valid for every n' <= n with the same block size.
 * Returns SKLTLT_EINVAL for n < 0, block_size < 0 or an unknown precision,
 * SKLTLT_ENOTSUP if n is beyond the supported range for that block size. */
int skltlt_workspace_size(int n, int block_size, int precision, size_t *bytes);

/* Blocked pivoted LTL^T (Sec. 3.6.3 fused right-looking blocked algorithm,
 * with the pivoted left-looking panel of Sec. 3.7.3 and the trailing update
 * cast as a skew rank-2k update via Theorem "TandS" of Sec. 2.2 and
 * Sec. 3.6.5 "Forming W after the panel factorization").
 *   n           order (n >= 0).
 *   A (device)  n x n, lda >= max(1, n); in: strict lower triangle of the
 *               skew matrix; out: t and L in the layout described above.
 *   t (device)  n-1 doubles (may be NULL when n <= 1): T[j+1][j].
 *   ipiv (device) n ints (may be NULL when n == 0).
 *   block_size  columns per panel; 0 = skltlt_default_block_size(n).
 *   precision   skltlt_precision.
 *   work (device), work_bytes: at least skltlt_workspace_size(...) bytes,
 *               256-byte aligned; contents on entry are irrelevant.
 * In exact arithmetic the result equals the unblocked algorithm's (the
 * blocked variants establish the same postcondition, Sec. 3.6). */
int skltlt_factor(int n, double *A, int lda, double *t, int *ipiv,
                  int block_size, int precision, void *work,
                  size_t work_bytes, void *stream);

/* skltlt_factor followed, on the same stream, by the Pfaffian read off T
 * and P: log_abs_pf (device, 1 double) = log|Pf(A)| and sign (device, 1 int)
 * in {-1, 0, +1}, with Pf(A) = sign * exp(log_abs_pf).  Odd n, or a zero
 * t[2i], gives sign 0 and log_abs_pf = -inf (Pf = 0 exactly). */
int skltlt_pfaffian(int n, double *A, int lda, double *t, int *ipiv,
                    double *log_abs_pf, int *sign, int block_size,
                    int precision, void *work, size_t work_bytes,
                    void *stream);

/* The unpivoted factorization A = L T L^T (P = I): the blocked fused
 * algorithm of Sec. 3.6.3 without the pivoting of Sec. 3.7, for inputs known
 * to need none (e.g. matrices assembled from well-conditioned factors); on
 * other inputs it may divide by small or zero t (no error is raised: a zero
 * t[k] gives a zero column of L, as in the pivoted algorithm).  Without
 * exchanges each panel's dependent steps involve only its top rows: one
 * workgroup runs them and every other row follows independently.
 * Arguments, layout, workspace and errors as for skltlt_factor, with
 * ipiv[i] = i on return (so the result can be passed to skltlt_solve);
 * block_size 0 means 128, and widths above 128 are reduced to 128. */
int skltlt_factor_nopiv(int n, double *A, int lda, double *t, int *ipiv,
                        int block_size, int precision, void *work,
                        size_t work_bytes, void *stream);

/* skltlt_factor_nopiv followed by the Pfaffian, Pf(A) = prod_i (-t[2i]);
 * arguments as for skltlt_pfaffian. */
int skltlt_pfaffian_nopiv(int n, double *A, int lda, double *t, int *ipiv,
                          double *log_abs_pf, int *sign, int block_size,
                          int precision, void *work, size_t work_bytes,
                          void *stream);

/* Bytes of device workspace for skltlt_factor_left / skltlt_pfaffian_left
 * (the factorization's workspace plus the accumulated operands of the
 * left-looking update, 2 * n * ~n doubles). */
int skltlt_left_workspace_size(int n, int block_size, size_t *bytes);

/* The unpivoted factorization by the blocked left-looking algorithm
 * (Variant 3, Sec. 3.6.4, from Invariant 3 of Sec. 3.4): when a panel is
 * reached, all earlier panels' skew rank-2k terms are applied to its
 * columns only (skew_tridiag_gemm, Sec. 3.6.6), then the panel is factored
 * as in skltlt_factor_nopiv; nothing right of the panel is touched.  Same
 * result as skltlt_factor_nopiv in exact arithmetic (the split of the
 * update's sum over workgroups uses floating-point atomics, so the last bits
 * may differ between runs).  Arguments as for skltlt_factor_nopiv (ipiv[i] = i
 * on return); precision must be SKLTLT_FP64 (SKLTLT_ENOTSUP otherwise);
 * work_bytes >= skltlt_left_workspace_size(n, block_size). */
int skltlt_factor_left(int n, double *A, int lda, double *t, int *ipiv,
                       int block_size, int precision, void *work,
                       size_t work_bytes, void *stream);

/* skltlt_factor_left followed by the Pfaffian (as skltlt_pfaffian_nopiv). */
int skltlt_pfaffian_left(int n, double *A, int lda, double *t, int *ipiv,
                         double *log_abs_pf, int *sign, int block_size,
                         int precision, void *work, size_t work_bytes,
                         void *stream);

/* Pfaffian only, by the "partial" reduction (Wimmer's algorithm: the
 * two-step algorithm of Sec. 3.5.2 with the second Gauss transform of each
 * pair and its tau skipped, Sec. 3.5.2 Notes; blocked with accumulated
 * rank-2k updates, Sec. 3.6.5 Note).  Per pair of columns (k, k+1), k even:
 * the pivot search and symmetric exchange on column k only (Sec. 3.7),
 * tau_k = X[k+1][k], l = X[k+2:, k] / tau_k, c = X[k+2:, k+1], and the
 * Schur complement X[k+2:, k+2:] += l c^T - c l^T.  Pf(A) = det(P) *
 * prod_k (-tau_k) over the even k: the same value as skltlt_pfaffian in
 * exact arithmetic, with half the pivot steps.
 *   A (device)  read only (strict lower triangle, lda >= max(1, n)); no L
 *               is formed.
 *   t (device)  n-1 doubles: t[k] = tau_k for even k, 0 for odd k.
 *   ipiv (device) n ints: ipiv[0] = 0, ipiv[k+1] = pivot row of step k for
 *               even k, ipiv[k+2] = k+2 (no exchange) for the odd steps.
 *   log_abs_pf, sign (device): as for skltlt_pfaffian.
 *   block_size  0 = skltlt_default_block_size(n); an odd width is rounded
 *               down to even (1 to 2).
 *   precision, work, work_bytes, stream: as for skltlt_pfaffian (the same
 *               workspace size).
 * Errors as for skltlt_pfaffian. */
int skltlt_pfaffian_partial(int n, const double *A, int lda, double *t,
                            int *ipiv, double *log_abs_pf, int *sign,
                            int block_size, int precision, void *work,
                            size_t work_bytes, void *stream);

/* Largest order handled by skltlt_batched. */
int skltlt_batched_max_n(void);

/* Tuning hook (for the autotuner, not for concurrent use): persistent
 * workgroups per CU of the following skltlt_batched calls, 1 .. 4, or 0 for
 * the tuned table's choice (by the batch's largest order).  Process-wide;
 * SKLTLT_EINVAL outside 0 .. 4. */
int skltlt_tune_batched_wgpc(int wgpc);

/* Tuning hook (for measurements, not for concurrent use): the trailing
 * update of skltlt_factor / skltlt_pfaffian takes 64 x 64 tiles instead of
 * 128 x 128 when its trailing block has fewer than `tiles` 128-tiles (lower
 * triangle, diagonal included); 0 never, negative restores the default (the
 * device's CU count).  Both tilings give bit-identical results.
 * Process-wide; always SKLTLT_OK. */
int skltlt_tune_skr2k_small_tiles(int tiles);

/* Bytes of device workspace for skltlt_batched with `batch` matrices: the
 * work-queue counter and the processing order (4 bytes per matrix). */
int skltlt_batched_workspace_size(int batch, size_t *bytes);

/* Many independent small factorizations and Pfaffians in one persistent
 * kernel launch: each workgroup takes the next matrix from a queue and runs
 * the fused blocked algorithm of Sec. 3.6.3 on it with a small block size
 * (the two-step case b = 2 is Sec. 3.5.2), the panel's rows of L in the
 * workgroup's LDS and the trailing matrix in the caller's buffer.  The
 * queue hands out the largest matrices first (a counting sort by n[i] on the
 * device, in the same stream, ahead of the persistent launch).  No host
 * synchronization, no host staging: all descriptors are device arrays, so
 * the call can be captured in a hipGraph.
 *   batch        number of matrices (>= 0).
 *   n (device)   batch orders, each in [0, max_n].
 *   A (device)   batch device pointers, each to an n[i] x n[i] matrix with
 *                leading dimension lda[i] (device array lda), same in/out
 *                layout as skltlt_factor.
 *   t, ipiv (device) batch device pointers (n[i]-1 doubles, n[i] ints).
 *   log_abs_pf, sign (device) arrays of batch entries, or both NULL to skip
 *                the Pfaffians.
 *   info (device) batch ints or NULL: 0 = done, -1 = entry rejected
 *                (n[i] < 0, n[i] > max_n, lda[i] < max(1, n[i]), or a
 *                matrix spanning 2 GiB or more: (n[i]-1) lda[i] + n[i]
 *                doubles >= 2^31 - 1 bytes); a
 *                rejected entry's matrix, t and ipiv are not touched, and
 *                its log_abs_pf / sign (when given) are set to NaN / 0.
 *   max_n (host) upper bound of the n[i], at most skltlt_batched_max_n().
 *   block_size   0 = the autotuned choice for each n[i], else the panel
 *                width, at most 16 (SKLTLT_ENOTSUP above).
 *   precision    SKLTLT_FP64 (SKLTLT_FP32_UPDATE returns SKLTLT_ENOTSUP).
 *   work (device), work_bytes: skltlt_batched_workspace_size bytes.
 * Each matrix's result depends only on that matrix and on (max_n,
 * block_size), never on the other members of the batch or their order. */
int skltlt_batched(int batch, const int *n, double *const *A, const int *lda,
                   double *const *t, int *const *ipiv, double *log_abs_pf,
                   int *sign, int *info, int max_n, int block_size,
                   int precision, void *work, size_t work_bytes,
                   void *stream);

/* ---- Allocation-free batched call ---------------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  skltlt_batched with the same arguments minus work/work_bytes:
 * the queue counter and processing order live in a static device array of
 * 256 + 4 * skltlt_batched_noalloc_max_batch() bytes (1 MiB + 256 B), one per
 * device, which the process holds until it ends; its device address is
 * looked up once per device on the first call made with that device
 * current.  The call allocates nothing and clears what must start at zero
 * with a kernel (no memset), so it can be captured in a hipGraph.
 * Every call on a device shares that device's array: two calls that overlap
 * in time on one device (different streams or threads, not ordered by the
 * caller) race on it and may both produce wrong results.  Calls on one
 * stream, or ordered by events, are safe.
 * Returns SKLTLT_ENOTSUP for batch > skltlt_batched_noalloc_max_batch();
 * other arguments, results and errors as for skltlt_batched. */
int skltlt_batched_noalloc_max_batch(void);
int skltlt_batched_noalloc(int batch, const int *n, double *const *A,
                           const int *lda, double *const *t,
                           int *const *ipiv, double *log_abs_pf, int *sign,
                           int *info, int max_n, int block_size,
                           int precision, void *stream);

/* Text of the HIP error behind the most recent SKLTLT_EDEVICE returned in
 * the calling thread ("" if none).  Static storage, never NULL. */
const char *skltlt_last_device_error(void);

/* ---- Solving with the factors ------------------------------------------
 * Solve A X = B for a skew-symmetric A factored by skltlt_factor or
 * skltlt_pfaffian (the factorization serves to solve skew-symmetric systems,
 * Sec. 1): with P A P^T = L T L^T,
 *     X = P^T L^{-T} T^{-1} L^{-1} P B,
 * i.e. permute the rows of B by P, solve with the unit lower L, solve the
 * skew tridiagonal T (two first-order recurrences: odd unknowns from the
 * even rows, even unknowns from the odd rows), solve with L^T, undo P.
 *   n      order; must be even (an odd-order skew matrix is singular)
 *   nrhs   number of right-hand sides, >= 1
 *   LT     (device) the factored matrix exactly as the factorization left
 *          it (L below the subdiagonal, t on it), leading dimension lda >= n
 *   t      (device) the n-1 entries t of the factorization
 *   ipiv   (device) its n pivots
 *   B      (device) n x nrhs, column-major, ldb >= n; overwritten by X
 *   work   (device) skltlt_solve_workspace_size(n, nrhs) bytes, 256-byte
 *          aligned
 * T is singular exactly when some t[2i] = 0 (then Pf(A) = 0): X then holds
 * non-finite values.  Check the Pfaffian's sign first when that matters.
 * Returns SKLTLT_EINVAL for n < 0, odd n, nrhs < 1, lda or ldb < n, NULL
 * pointers or a short or misaligned workspace.  n = 0 does nothing. */
int skltlt_solve_workspace_size(int n, int nrhs, size_t *bytes);
int skltlt_solve(int n, int nrhs, const double *LT, int lda, const double *t,
                 const int *ipiv, double *B, int ldb, void *work, size_t work_bytes,
                 void *stream);

/* ---- Instrumentation ---------------------------------------------------
 * Per-kernel timing for measurement tools.  While enabled, every kernel the
 * library enqueues is bracketed by a pair of HIP events recorded on the same
 * stream as the kernel; the events are created by skltlt_timing_enable (not
 * on the factorization path).  Kernel classes: */
typedef enum {
    SKLTLT_K_PANEL = 0,    /* pivoted left-looking panel                      */
    SKLTLT_K_SKR2K = 1,    /* skew rank-2k trailing update (MFMA)            */
    SKLTLT_K_FINALIZE = 2, /* deferred row exchanges of earlier L columns    */
    SKLTLT_K_PFAFFIAN = 3, /* log|Pf| and sign                               */
    SKLTLT_K_BATCHED = 4,  /* batched persistent kernel                      */
    SKLTLT_K_OTHER = 5,    /* small fills                                    */
    SKLTLT_K_SOLVE = 6,    /* skltlt_solve's kernels                         */
    SKLTLT_K_COUNT = 7
} skltlt_kernel_class;

/* Start recording; max_launches bounds the number of bracketed launches
 * (launches beyond it are not timed).  Returns SKLTLT_EDEVICE if the events
 * cannot be created.  Not thread-safe with concurrent library calls. */
int skltlt_timing_enable(int max_launches);

/* Stop recording (events are kept until the next enable). */
int skltlt_timing_disable(void);

/* Destroys the events skltlt_timing_enable created (recording stops), so
 * that a measurement tool can release them before the HIP runtime is torn
 * down at process exit. */
int skltlt_timing_release(void);

/* Synchronizes the recorded events and returns, for one kernel class, the
 * summed duration in milliseconds and the number of timed launches (host
 * outputs).  Also returns the per-launch algorithmic flop count summed over
 * the timed launches of that class in *flops (0 for classes without one). */
int skltlt_timing_read(int kernel_class, double *total_ms, int *launches, double *flops);

#ifdef __cplusplus
}
#endif
#endif /* SKLTLT_H */
