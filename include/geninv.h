/*
 * libgeninv -- Moore-Penrose inverse by full-rank Cholesky factorization on
 * AMD Instinct MI355X (gfx950).
 *
 * Method (P. Courrieu, "Fast Computation of Moore-Penrose Inverse Matrices",
 * Section 2 and Appendix):
 *   A = G'G                      Gram matrix, Eq. (1)
 *   tol = 1e-9 * min{A_kk > 0}   Appendix (or a caller-supplied tol > 0)
 *   A = L L'                     full-rank Cholesky: column k of A is kept only
 *                                when its updated pivot is strictly above tol;
 *                                L is n x r, r = rank (Section 2, Eq. (1))
 *   M = (L'L)^-1                 Theorem 1
 *   Y = G^+ = L M M L' G'        Theorem 1
 *   W = G^+ F                    least-squares use, Section 1
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major (element (i,j) of X at X[i + j*ldx]), with
 *   ld >= max(1, rows).  Unless stated otherwise, matrix pointers are DEVICE
 *   pointers owned by the caller; the library never frees them.
 * - Every call enqueues its kernels on the context's stream and returns
 *   without waiting, except where a HOST output pointer is passed (then the
 *   call waits for the stream before writing it) and, by default, once in
 *   the middle of the whole-method calls to learn the rank
 *   (geninv_set_host_sync).
 * - The return value is a geninv_status code.  Nothing aborts or prints.
 *   Argument errors are detected on the host before anything is enqueued.
 *   Errors found on the device (non-finite data, a non-SPD L'L) are written
 *   to a device status word; calls that synchronize return them, and
 *   geninv_sync_status() returns them for asynchronous calls.
 * - A workspace grows on demand inside the context (device memory owned by
 *   the library, freed by geninv_destroy).  Calls on one context must not
 *   overlap on different host threads.
 * - m or n == 0 is valid: r = 0 and nothing is written.  A Gram matrix with
 *   no positive diagonal entry (e.g. G = 0) gives r = 0 and Y = 0, as the
 *   paper's minimum over an empty set makes every pivot test fail.
 */
#ifndef GENINV_H
#define GENINV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct geninv_ctx geninv_ctx;

typedef enum {
    GENINV_OK = 0,
    GENINV_EINVAL = -1,      /* bad argument (sizes, leading dimensions, null pointers) */
    GENINV_ENOMEM = -2,      /* device workspace allocation failed */
    GENINV_EHIP = -3,        /* a HIP runtime call failed */
    GENINV_ENONFINITE = -4,  /* G (or its Gram matrix) holds Inf/NaN; r is set to 0 */
    GENINV_ENOTSPD = -5,     /* L'L lost positive definiteness in the inverse */
    GENINV_ENOTSUP = -6,     /* valid request that the library does not support */
    GENINV_EACCURACY = -7,   /* mixed form: outputs written, but the error estimate exceeds the target */
    GENINV_ESCRATCH = -8     /* allocation-free call: the problem needs more than the fixed scratch area */
} geninv_status;

/* Arithmetic of a whole-method call (geninv_mixed, geninv_workspace_bytes). */
typedef enum {
    GENINV_FP64 = 0,         /* every product in float64 (geninv_dgeninv, geninv_dlstsq) */
    GENINV_MIXED_BF16 = 1,   /* Gram and chain products from 8-bit slices on the bfloat16 matrix cores */
    GENINV_MIXED_INT8 = 2    /* Gram and chain products from int8 residues modulo coprime moduli */
} geninv_precision;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL selects the legacy default stream).  *ctx receives the
 * handle.  Returns EINVAL for a null ctx or bad device, EHIP on runtime errors. */
int geninv_create(geninv_ctx **ctx, int device, void *hip_stream);

/* Wait for the context's stream, free its workspace and the handle. NULL is a no-op. */
int geninv_destroy(geninv_ctx *ctx);

/* Switch the stream later calls enqueue on (same device). */
int geninv_set_stream(geninv_ctx *ctx, void *hip_stream);

/* Cap on the context's workspace in bytes (0, the default, means none; the
 * environment variable GENINV_WORKSPACE_LIMIT sets it when the context is
 * created).  A call that needs a larger workspace returns GENINV_ENOMEM
 * before anything is enqueued and leaves its outputs untouched; the context
 * stays usable.  This is the hook through which tests force an allocation
 * failure; callers can also use it to bound the library's device memory.
 * EINVAL for a null ctx. */
int geninv_set_workspace_limit(geninv_ctx *ctx, size_t bytes);

/* Debug aids.  GENINV_DEBUG_POISON: every workspace the context allocates
 * from then on is filled with a quiet-NaN pattern before its first use (the
 * environment variable GENINV_DEBUG=1 sets it when the context is created),
 * so a step that reads memory no earlier step of its call wrote shows up as
 * NaN in the results.  geninv_debug_poison fills the current workspace with
 * that pattern now (on the context's stream), e.g. between two calls to
 * check that a call does not depend on what an earlier one left behind.
 * EINVAL for a null ctx or unknown flags. */
enum { GENINV_DEBUG_POISON = 1 };
int geninv_set_debug(geninv_ctx *ctx, int flags);
int geninv_debug_poison(geninv_ctx *ctx);

/* Whether a call reads the rank back to the host once its full-rank Cholesky
 * factorization is done (enable != 0, the default) or not (enable == 0).
 * On: one stream synchronization inside geninv_dgeninv, geninv_dlstsq and
 * geninv_mixed, after which every later launch (the (L'L)^-1 steps, the
 * chain products) is sized for the actual rank r.  Off: no host
 * synchronization inside those calls (e.g. for stream capture or host-side
 * overlap); the later kernels are then launched for the bound min(m, n) and
 * read r from device memory, which costs idle launches when r is well below
 * that bound.  Results are the same either way.  EINVAL for a null ctx. */
int geninv_set_host_sync(geninv_ctx *ctx, int enable);

/* Wait for the stream and return the device-side status of the calls made
 * since the last geninv_sync_status() (GENINV_OK, ENONFINITE or ENOTSPD);
 * the device status word is cleared. */
int geninv_sync_status(geninv_ctx *ctx);

/* Human-readable text for a status code (static storage). */
const char *geninv_strerror(int status);

/* Library version as 10000*major + 100*minor + patch. */
int geninv_version(void);

/* Device workspace (bytes) a call needs for an m x n problem: with
 * precision GENINV_FP64, geninv_dgeninv (k = 0) or geninv_dlstsq with k
 * right-hand sides (the digit and step arguments are ignored); with
 * GENINV_MIXED_BF16 or GENINV_MIXED_INT8, geninv_mixed with those
 * gram_digits, chain_digits and ns_steps (k ignored).  0 for invalid
 * arguments.  Calls grow the context's workspace to this size on first use. */
size_t geninv_workspace_bytes(int m, int n, int k, int precision, int gram_digits, int chain_digits, int ns_steps);

/* ---- whole method, float64 --------------------------------------------- */

/* Y = G^+ (Theorem 1; Appendix).
 *   G    m x n, ldg >= m (device, read only)
 *   tol  pivot threshold; <= 0 selects the paper's default 1e-9 * min positive A_kk
 *   Y    n x m, ldy >= n (device, written)
 *   rank HOST int* or NULL.  If non-NULL the call waits for the stream, writes
 *        r, and returns any device-side error status.
 *   piv  DEVICE int[max(1, min(m,n))] or NULL: piv[c] = 0-based index of the
 *        column of A (of G when m >= n, of G' otherwise) behind column c of L,
 *        for c < r.  Increasing.
 * When m < n the method factors A = G G' and forms Y = G' L M M L' (the
 * Appendix's transpose branch). */
int geninv_dgeninv(geninv_ctx *ctx, int m, int n, const double *G, int ldg, double tol,
                   double *Y, int ldy, int *rank, int *piv);

/* W = G^+ F, the minimum-norm least-squares solution of min ||G W - F|| (Section 1).
 *   F m x k (ldf >= m), W n x k (ldw >= n); rank as in geninv_dgeninv.
 * Evaluated as W = L (M (M (L' (G' F)))) without forming Y; when m < n the
 * Appendix's transpose branch factors G G' and evaluates
 * W = G' (L (M (M (L' F)))).  k <= 4096 (ENOTSUP above). */
int geninv_dlstsq(geninv_ctx *ctx, int m, int n, int k, const double *G, int ldg,
                  const double *F, int ldf, double tol, double *W, int ldw, int *rank);

/* The same least-squares solve for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops): every scratch
 * buffer of the call (Gram matrix, factor, inverse, split-K partials, rank
 * and pivots) lives in a fixed device array of geninv_noalloc_capacity()
 * bytes (256 MiB) that the library holds on each device until the process
 * ends; the call makes no hipMalloc, hipFree or other allocation (its event
 * timers are off for the call).  Problems whose workspace
 * (geninv_workspace_bytes(m, n, k, GENINV_FP64, 0, 0, 0)) exceeds it return
 * GENINV_ESCRATCH before anything is enqueued: in float64 with k <= 64 that
 * is about n = min(m, n) <= 1400.  Arguments, results and synchronization
 * as geninv_dlstsq (the rank read-back by default; see
 * geninv_set_host_sync).  Every call on one device uses the same array and
 * keeps the last call's contents: calls that overlap on one device (on
 * different streams or host threads, with any context) race.  Nothing in
 * the array needs to start at zero: each call writes every part it reads. */
int geninv_dlstsq_noalloc(geninv_ctx *ctx, int m, int n, int k, const double *G, int ldg, const double *F, int ldf,
                          double tol, double *W, int ldw, int *rank);
size_t geninv_noalloc_capacity(void);

/* ---- individual steps, float64 (same kernels as the whole method) ------- */

/* A = G'G, Eq. (1).  G m x n (ldg >= m), A n x n (lda >= n).  Writes the lower
 * triangle (diagonal included) when full == 0, the whole matrix otherwise. */
int geninv_dgram(geninv_ctx *ctx, int m, int n, const double *G, int ldg, double *A, int lda,
                 int full);

/* Full-rank Cholesky of the symmetric PSD A (n x n, lower triangle read,
 * not modified), Appendix loop:
 *   tol   <= 0 selects 1e-9 * min positive A_kk
 *   L     n x n (ldl >= n, device): columns 0..r-1 receive the factor, every
 *         other entry of the n x n block is set to zero; column c is zero above
 *         row piv[c]
 *   piv   DEVICE int[n] or NULL (as in geninv_dgeninv)
 *   d     DEVICE double[n] or NULL: d[k] = updated pivot value of column k
 *         before the test against tol (diagnostics for parity checks)
 *   tol_used  DEVICE double* or NULL: the threshold actually applied
 *         (+Inf when A has no positive diagonal)
 *   rank  HOST int* or NULL (waits), as in geninv_dgeninv. */
int geninv_dfrchol(geninv_ctx *ctx, int n, const double *A, int lda, double tol, double *L,
                   int ldl, int *piv, double *d, double *tol_used, int *rank);

/* M = B^-1 for symmetric positive definite B (r x r, ldb >= r, not
 * modified; the symmetric block sweep reads the lower triangle and the
 * diagonal 64 x 64 blocks in full); M r x r, ldm >= r, written in full and
 * exactly symmetric (Theorem 1: B = L'L).  A non-positive pivot block sets
 * the device status to ENOTSPD. */
int geninv_dspdinv(geninv_ctx *ctx, int r, const double *B, int ldb, double *M, int ldm);

/* The same inverse by Newton-Schulz iteration X <- X (2I - B X) on the
 * float64 matrix cores, X_0 = I / ||B||_F: the parallel alternative to the
 * sequential sweep (Section 2 cites O(log r) parallel time for such
 * inverses).  Each step forms the residual ||I - B X||_F / sqrt(r) of the
 * current X (one device-to-host read); the iteration stops when it no longer
 * falls (about cond(B) u) or after max_iter steps, and M receives the iterate
 * with the smallest residual.  *iters and *resid (HOST, optional) report the
 * number of residual evaluations and that residual.  Convergence takes about
 * log2(cond(B) sqrt(r)) + 6 steps of two r^3 products each.  ENOTSPD if ||B|| = 0,
 * ENONFINITE on a non-finite residual. */
int geninv_dspdinv_ns(geninv_ctx *ctx, int r, const double *B, int ldb, double *M, int ldm, int max_iter,
                      int *iters, double *resid);

/* Y = L M M L' G' (Theorem 1) for given factors: L n x r (ldl >= n),
 * M r x r symmetric (ldm >= r), G m x n (ldg >= m), Y n x m (ldy >= n). */
int geninv_dchain(geninv_ctx *ctx, int m, int n, int r, const double *L, int ldl,
                  const double *M, int ldm, const double *G, int ldg, double *Y, int ldy);

/* C = alpha * op(A) op(B) + beta * C with the library's float64 MFMA GEMM
 * (the contraction every step above is built from).  op(X) = X or X'
 * (transX = 0 / 1); C is M x N (ldc >= M).  Products with few output tiles
 * and a long K are split over K into the context's workspace (which may
 * grow) and summed in a fixed order; with A not transposed, N <= 16 and
 * K >= 1024 (right-hand sides such as W = Y F) a bandwidth-bound
 * row-per-thread kernel is used instead of MFMA tiles.  Used by the
 * benchmark for W and exposed for parity testing. */
int geninv_dgemm(geninv_ctx *ctx, int transA, int transB, int M, int N, int K, double alpha,
                 const double *A, int lda, const double *B, int ldb, double beta, double *C,
                 int ldc);

/* ---- incremental least squares ---------------------------------------------- */

/* Incremental learning (Section 4): when basis functions (columns of G) are
 * added to a network, the Gram matrix A = G'G and G'F grow by rows instead of
 * being formed again.  This call appends the rows of p new columns:
 *   A[n_old + i, j] = G(:, n_old + i)' G(:, j)    for every j < n_old + p
 *   B[n_old + i, q] = G(:, n_old + i)' F(:, q)    for q < k
 * (the new diagonal block is written in full, i.e. with its symmetric upper
 * part).  G is m x (n_old + p) with the old columns first (ldg >= m), F is
 * m x k (ldf >= m); A (lda >= n_old + p) and B (ldb >= n_old + p) keep the
 * rows of earlier calls, which are not read.  n_old = 0 forms both from
 * scratch.  Cost O(m (n_old + p) p) instead of O(m (n_old + p)^2).  All
 * pointers DEVICE memory; p = 0 returns at once. */
int geninv_inc_gram(geninv_ctx *ctx, int m, int n_old, int p, int k, const double *G, int ldg,
                    const double *F, int ldf, double *A, int lda, double *B, int ldb);

/* W = G^+ F (n x k, ldw >= n) from the lower triangle of the Gram matrix A
 * (n x n, lda >= n) and B = G'F (n x k, ldb >= n), e.g. as geninv_inc_gram
 * leaves them: the method from the tolerance on (Section 2, Eq. (1) - (4);
 * the Appendix after its Gram product), G itself is not needed.  A and B
 * are read only.  tol and rank as in geninv_dgeninv. */
int geninv_dlstsq_gram(geninv_ctx *ctx, int n, int k, const double *A, int lda, const double *B, int ldb,
                       double tol, double *W, int ldw, int *rank);

/* Incremental full-rank Cholesky (Section 4: basis functions added to a
 * network, rank deficiency allowed).  A is the Gram matrix of the n_old + p
 * columns seen so far (lower triangle and the new rows, as geninv_inc_gram
 * leaves it; lda >= n_old + p).  L (ldl >= n_old + p), piv and dvals
 * (int / double [n_old + p]) and M (ldm >= n_old + p) hold the factor of the
 * first n_old columns from the previous call: L's kept columns, their pivot
 * rows, every column's updated pivot value and M = (L'L)^-1 (r x r).
 * *rank_io (HOST) is that factor's rank r on entry and the new rank on
 * return; *tol_io (HOST) the threshold it used (written, not read, when
 * n_old = 0).  tol <= 0 selects the paper's default for all n_old + p
 * columns.
 * The earlier columns' factor does not change when columns are appended (the
 * Appendix loop is left to right), so the call computes only: the new rows
 * of L from the triangular system L_P X = B_P with the earlier pivot rows
 * L_P = L(piv, :) and B_P(c, i) = A(n_old + i, piv[c]) (blocked, MFMA
 * products); the full-rank Cholesky of the new columns' Schur complement
 * A_new - X'X with the same strict test; and M by a block update
 * (Woodbury for L_old'L_old + X X', then the Schur complement of the new
 * kept columns), O(r^2 p) instead of O(r^3); when the appended rows
 * dominate (trace of I + X' M_old X above 2 p + 64, where the update would
 * lose accuracy) M is formed directly from the extended L instead.  When
 * the default threshold
 * falls (a new column with a smaller diagonal) so far that an earlier
 * decision would change, the call refactors all n_old + p columns instead.
 * n_old = 0 factors from scratch.  Synchronizes (reads the new rank). */
int geninv_inc_factor(geninv_ctx *ctx, int n_old, int p, const double *A, int lda, double tol, double *L, int ldl,
                      int *piv, double *dvals, double *M, int ldm, int *rank_io, double *tol_io);

/* W = L (M (M (L' B))) (n x k, ldw >= n) for a factor L (n x r, ldl >= n)
 * and M = (L'L)^-1 (r x r, ldm >= r), e.g. from geninv_inc_factor, and
 * B = G'F (n x k, ldb >= n): the method's least-squares weights from the
 * factors (Theorem 1 with Section 1's W = G^+ F). */
int geninv_factored_lstsq(geninv_ctx *ctx, int n, int r, int k, const double *L, int ldl, const double *M, int ldm,
                          const double *B, int ldb, double *W, int ldw);

/* ---- mixed precision: error-free split products on bfloat16 matrix cores - */

/* Y = G^+ (Theorem 1) with the two dense products (the Gram matrix and
 * Y = P G', P = L M M L') on reduced-precision matrix cores, everything the
 * method decides in float64: the tolerance, the pivot decisions, the
 * Cholesky factor, (L'L)^-1, K = L M and P = K K'.  When m < n the Appendix's
 * transpose branch factors G G' and forms Y = G' P.
 *   precision  GENINV_MIXED_BF16: every column of G (every row of P and of G
 *              in the chain) is scaled by a power of two and cut into 8-bit
 *              integer slices (the error-free splitting of Ozaki, Ogita,
 *              Oishi and Rump); slice pairs are exact bfloat16 products with
 *              exact float32 class sums moved into float64 totals.  The Gram
 *              matrix takes every pair (the exactly rounded Gram matrix of
 *              the 8*digits-bit representation of G: a truncated pair set
 *              would not be the Gram matrix of any matrix); the chain the
 *              pairs t + u <= digits.  digits 1..4.
 *              GENINV_MIXED_INT8: every row/column is scaled by a power of
 *              two and rounded to an integer of beta bits; the integer
 *              product is formed exactly from int8 matrix products modulo
 *              `digits` pairwise coprime moduli <= 255 (Ozaki, Uchino and
 *              Imamura's modular scheme) and the Chinese remainder theorem,
 *              then rounded once to float64.  beta is the largest bit count
 *              (<= 52) the moduli allow for the product's depth K
 *              (K 2^(2 beta) < prod p / 2): 16 moduli give beta = 52 up to
 *              K = 2^17, i.e. float64 accuracy.  digits 1..16 (EINVAL when
 *              too few moduli leave no bits for this K).
 *   gram_digits   slices or moduli of the Gram matrix
 *   chain_digits  slices or moduli of Y = P G'; 0 evaluates it in float64
 *   ns_steps   0..16 Newton-Schulz steps X <- X (2I - G X), in the factored
 *              form P <- 2P - P (L L') P (X = P G') with float64 products:
 *              L L' is the Gram matrix of the columns the factorization
 *              kept, whose pseudoinverse P is the method's fixed point, so
 *              the steps remove the rounding of (L'L)^-1, K and P; a step is
 *              taken only while its correction ||P L L' P - P||_F / ||P||_F
 *              falls (each step reads one number back to the host).
 *   target     > 0: return GENINV_EACCURACY (outputs still written) when the
 *              error estimate exceeds it; <= 0: no check
 *   err_est    HOST double* or NULL.  When non-NULL or target > 0 the call
 *              estimates the relative change the engine makes to Y against
 *              the float64 form on the same G, from 16 random sign probes V
 *              and float64 products that use the caller's G (one host
 *              synchronization):
 *                resA  = ||A_e V - G'(G V)|| / ||G'(G V)||, the engine's
 *                        Gram matrix A_e against float64 products;
 *                kappa = max_k A_kk / (smallest accepted pivot), how much
 *                        the factorization amplifies a relative Gram error;
 *                resY  = ||Y V' - P (G' V')|| / ||P (G' V')||, the engine's
 *                        chain product against float64 products on the
 *                        same P (0 for a float64 chain);
 *              err_est = kappa resA + resY (a first-order estimate; the
 *              Frobenius norms come from the probes, relative spread about
 *              1 / sqrt(32)).
 * Other arguments as in geninv_dgeninv. */
int geninv_mixed(geninv_ctx *ctx, int m, int n, const double *G, int ldg, double tol, int precision,
                 int gram_digits, int chain_digits, int ns_steps, double target, double *Y, int ldy, int *rank,
                 int *piv, double *err_est);

/* C = op(A) op(B) (M x N, ldc >= M) on the int8 engine with `moduli`
 * moduli, exactly as geninv_mixed forms its products with
 * GENINV_MIXED_INT8: op(A) = A' when transA (A is K x M), A otherwise
 * (M x K); op(B) likewise.  lower != 0 (M == N) writes only the lower
 * triangle, diagonal included.  The product of the integer representations
 * is exact; the result is that product rounded to float64 (error about
 * 2 u |C| beyond the representation error).  For parity testing and as a
 * float64-accurate product at moduli = 16.  EINVAL when the moduli leave no
 * bits for this K. */
int geninv_mgemm(geninv_ctx *ctx, int transA, int transB, int M, int N, int K, const double *A, int lda,
                 const double *B, int ldb, int moduli, int lower, double *C, int ldc);

/* The slicing step on its own, for parity testing.  transposed == 0: column
 * exponents e[cols] and planes[t][i + j*ldp] = slice t of X(i, j) (ldp >= rows,
 * rows rows..ldp-1 zero).  transposed != 0: row exponents e[rows] and
 * planes[t][k + i*ldp] = slice t of X(i, k) (ldp >= cols, columns cols..ldp-1
 * zero).  planes: DEVICE bfloat16 array of slices*ldp*(cols or rows) elements,
 * 16-byte aligned, with ldp a multiple of 8 (EINVAL otherwise); e: DEVICE int
 * array. */
int geninv_bslice(geninv_ctx *ctx, int rows, int cols, const double *X, int ldx, int slices,
                  int transposed, void *planes, int ldp, int *e);

/* Lower triangle of the sliced Gram matrix G_s'G_s (n x n, lda >= n) exactly
 * as geninv_mixed forms it (slices 1..4), for parity testing. */
int geninv_bgram(geninv_ctx *ctx, int m, int n, const double *G, int ldg, int slices, double *A, int lda);

/* Y = P G' (n x m, ldy >= n) for P n x k (ldp >= n) and G m x k (ldg >= m),
 * exactly as geninv_mixed forms its chain product: rows of P and of G sliced
 * (slices 1..4), the pairs t + u <= slices multiplied, float64 totals.  For
 * parity testing.  k = 0 gives Y = 0. */
int geninv_bchain(geninv_ctx *ctx, int n, int m, int k, const double *P, int ldp, const double *G, int ldg,
                  int slices, double *Y, int ldy);

/* ---- batched least squares ---------------------------------------------- */

/* A plan solves `batch` independent small problems W_b = G_b^+ F_b (Section 1)
 * in one persistent launch: each workgroup takes problems from a device work
 * queue, largest first, and runs the whole method on one problem (Gram matrix
 * and G'F with float64 accumulation, tol, full-rank Cholesky, (L'L)^-1,
 * W = L M M L' G'F).
 *   m, n, ldg, ldf, ldw   HOST int[batch]; 1 <= min(m_b, n_b) <= 256 (m_b < n_b
 *                         takes the Appendix's transpose branch, in a second
 *                         persistent launch after the tall problems': G_b G_b'
 *                         is factored and W_b = G_b' L M M L' F_b)
 *   G, F                  HOST arrays of DEVICE pointers: G_b m_b x n_b and
 *                         F_b m_b x k, float32, column-major
 *   W                     HOST array of DEVICE pointers: W_b n_b x k, float64
 *   k                     1..16 right-hand sides (the same for every problem)
 *   tol                   <= 0: the paper's default per problem
 *   rank                  DEVICE int[batch]: r_b, written by every run
 * The pointers are fixed for the plan's lifetime; inputs may change between
 * runs.  The plan keeps its own device copies of the descriptors. */
typedef struct geninv_batch_plan geninv_batch_plan;
int geninv_batch_plan_create(geninv_ctx *ctx, geninv_batch_plan **plan, int batch, const int *m,
                             const int *n, int k, const float *const *G, const int *ldg,
                             const float *const *F, const int *ldf, double *const *W,
                             const int *ldw, double tol, int *rank);
int geninv_batch_plan_destroy(geninv_batch_plan *plan);

/* Enqueue one solve of every problem on the context stream.  use_graph != 0
 * captures the launch into a HIP graph on first use (on a non-default
 * stream) and replays it afterwards.  When the stream is already being
 * captured by the caller, or the plan's own capture or instantiation fails,
 * the run launches directly instead (same work; inside a caller's capture
 * the launches join the caller's graph) and the plan counts it:
 * geninv_batch_plan_graph_fallbacks returns that count (EINVAL for a null
 * plan). */
int geninv_batch_plan_run(geninv_batch_plan *plan, int use_graph);
int geninv_batch_plan_graph_fallbacks(const geninv_batch_plan *plan);

/* Autotuner: times each launch configuration (LDS threshold below which a
 * problem's Gram matrix and L'L live in LDS; workgroups per compute unit)
 * `reps` times and keeps the fastest.  cache_path (or NULL): a text file of
 * tuned configurations, one line "key nl grid ms" per batch, the key naming
 * the library version, the device and the batch's shapes; an entry for this
 * batch is applied without timing (*from_cache = 1), otherwise the result is
 * stored there (through a temporary file and a rename).  Unparsable or
 * inapplicable lines are ignored and a missing, unreadable or unwritable file
 * only means tuning (the plan keeps working with the tuned or default
 * configuration).  Outputs may be NULL.  Synchronizes. */
int geninv_batch_plan_autotune(geninv_batch_plan *plan, int reps, const char *cache_path, int *best_nl,
                               int *best_grid, double *best_ms, int *from_cache);

/* One-shot form of the batched solve, with the arguments of
 * geninv_batch_plan_create: builds a plan with the default launch
 * configuration, runs it once (no graph) and destroys it, which synchronizes
 * the context stream.  status (HOST int, optional) receives the device
 * status word as geninv_sync_status() returns it (0, or GENINV_ENONFINITE
 * for non-finite data).  For repeated solves of one problem set keep a plan:
 * it orders the problems and uploads their descriptors once. */
int geninv_lstsq_batched(geninv_ctx *ctx, int batch, const int *m, const int *n, int k,
                         const float *const *G, const int *ldg, const float *const *F,
                         const int *ldf, double tol, double *const *W, const int *ldw, int *rank,
                         int *status);

/* Optional per-problem pivot output: piv is a HOST array of `batch` DEVICE
 * pointers (int[min(m_b, n_b)] each, or NULL entries), or NULL to switch
 * the output off.  Each run then writes the 0-based indices of the r_b
 * columns problem b kept (rows of G_b in the transpose branch), increasing
 * (as geninv_dgeninv's piv).  Synchronizes the stream;
 * a graph captured earlier keeps reading the descriptors, so it follows. */
int geninv_batch_plan_set_pivots(geninv_batch_plan *plan, int *const *piv);

/* Set or read the launch configuration directly: LDS threshold nl, grid
 * workgroups (<= 1024).  EINVAL for a configuration whose LDS does not fit
 * a compute unit. */
int geninv_batch_plan_config(geninv_batch_plan *plan, int nl, int grid);
int geninv_batch_plan_get_config(geninv_batch_plan *plan, int *nl, int *grid);

/* ---- event timers ------------------------------------------------------- */

/* Per-kernel-class HIP event timers on the context stream, for profiling.
 * Classes are numbered 0 .. geninv_prof_classes()-1 and named by
 * geninv_prof_name() ("gram", "panel_factor", "chain_y", ...).  When bit k of
 * `mask` is set, every launch of class k is bracketed by two events;
 * geninv_prof_enable() also clears the totals.  Timers add two event
 * records per bracketed launch and nothing else. */
int geninv_prof_classes(void);
const char *geninv_prof_name(int cls);
int geninv_prof_enable(geninv_ctx *ctx, unsigned mask);

/* Wait for the recorded events and return the totals of class `cls` since
 * the last geninv_prof_enable(): summed milliseconds, number of bracketed
 * launches, and the algorithmic flops of those launches where the library
 * knows them on the host (0 for launches sized by the device-side rank).
 * Any output pointer may be NULL. */
int geninv_prof_read(geninv_ctx *ctx, int cls, double *total_ms, long *launches, double *flops);

#ifdef __cplusplus
}
#endif

#endif /* GENINV_H */
