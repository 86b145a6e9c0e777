/*
 * tsnmf.h - C ABI of libtsnmf: single-pass tall-and-skinny QR (R factor only),
 * Gaussian projection, and the n x n steps of near-separable NMF on MI355X.
 *
 * Method: Benson, Lee, Rajwa, Gleich, "Scalable methods for nonnegative matrix
 * factorizations of near-separable tall-and-skinny matrices".  For X (m x n,
 * m >> n, X >= 0) the extreme columns of X are those of the n x n factor R of
 * the thin QR X = QR (Sec. 2.2), H is found by NNLS on R (Sec. 2.4), the
 * column l1 norms D are accumulated in the same pass so that X D^{-1} can be
 * handled as R D^{-1} (Sec. 3.3), and G^T X with Gaussian G is the alternative
 * projection (Sec. 2.3, Sec. 3.2 / Algorithm 1).
 *
 * Conventions shared by every call
 *   - Matrix/vector arguments are DEVICE pointers owned by the caller, except
 *     where a comment says "host".  The library never frees or keeps them
 *     beyond the completion of the work it enqueued.
 *   - Every compute call is stream-ordered and asynchronous: it enqueues work on
 *     `stream` (NULL = the null stream) and returns; results are valid once the
 *     stream has reached that point.
 *   - Return value: 0 on success; -i if the i-th argument is invalid (checked on
 *     the host before anything is enqueued); a positive TSNMF_ERR_* code for a
 *     runtime failure (for TSNMF_ERR_HIP, tsnmf_last_hip_error() gives the HIP
 *     error code).
 *   - Numerical outcomes (early stop, iteration caps) are reported through
 *     optional device `info` outputs, never through host synchronisation.
 *   - NaN or Inf in the input propagates into the outputs; it is not trapped.
 *   - Outputs are column-major; index sets are 0-based int32.
 *   - The library keeps one grow-only device workspace per device.  It is
 *     allocated on first use (or by tsnmf_reserve); a call made while `stream`
 *     is being captured into a graph returns TSNMF_ERR_CAPTURE instead of
 *     allocating, so reserve before capturing.  When a later call (or a
 *     larger reserve) grows the workspace, the old buffer is retired, not
 *     freed: graphs captured earlier keep naming it in their kernel
 *     arguments and stay valid to replay.  tsnmf_workspace_release() frees
 *     the retired buffers once no such graph will be replayed.
 *   - Calls that share the workspace must not run concurrently on different
 *     streams of the same device.
 */
#ifndef TSNMF_H
#define TSNMF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- flags ---------------------------------------------------------------- */
#define TSNMF_F64          0x1u   /* input elements are IEEE binary64            */
#define TSNMF_F32          0x2u   /* input elements are IEEE binary32            */
#define TSNMF_BF16         0x4u   /* input elements are bfloat16                 */
#define TSNMF_DTYPE_MASK   0x7u
#define TSNMF_ROW_MAJOR    0x00u  /* X(i, j) at X[i * ld + j], ld >= n           */
#define TSNMF_COL_MAJOR    0x10u  /* X(i, j) at X[i + j * ld], ld >= m           */
#define TSNMF_LEAF_F64     0x20u  /* TSQR: factor row blocks in FP64 (default for
                                     F64 input; for F32 input the values are
                                     widened exactly and the whole path is FP64) */
#define TSNMF_GP_MFMA_BF16 0x100u /* projection on matrix cores: G and X rounded
                                     to bfloat16 (nearest-even), FP32 accumulate */
#define TSNMF_GP_SIMD_F32  0x200u /* projection on the vector ALUs in FP32       */

/* ---- status codes ----------------------------------------------------------- */
#define TSNMF_OK               0
#define TSNMF_ERR_HIP          1  /* a HIP runtime call failed                   */
#define TSNMF_ERR_NOMEM        2  /* workspace allocation failed                 */
#define TSNMF_ERR_CAPTURE      3  /* workspace too small while stream capturing   */
#define TSNMF_ERR_UNSUPPORTED  4  /* shape outside the supported range            */

#define TSNMF_MAX_N 256           /* largest column count of the TSQR / GP paths */
#define TSNMF_MAX_BATCH_N 128     /* largest column count of the batched TSQR    */

/* ---- thin QR, R factor only ------------------------------------------------- */

/*
 * tsnmf_tsqr_r: R factor of the thin QR of X, and the l1 column sums of X, in
 * one pass over X (Sec. 3.1 "TSQR and R-SVD": only R is formed, Q^T is applied
 * implicitly; Sec. 3.3 "Column normalization": the column norms are
 * accumulated in the same pass).
 *
 *   X       device, m x n, dtype and layout from `flags` (TSNMF_F32 or
 *           TSNMF_F64; TSNMF_ROW_MAJOR or TSNMF_COL_MAJOR; TSNMF_LEAF_F64
 *           optional).  Read exactly once.
 *   m, n    1 <= n <= TSNMF_MAX_N, m >= 1.  (m < n is accepted: R is then the
 *           n x n factor of X padded with zero rows.)
 *   ld      leading dimension in elements (>= n row-major, >= m column-major).
 *   R       device, n x n FP64, column-major (ldR = n), output: upper
 *           triangular with R(i, i) >= 0 and exact zeros below the diagonal, so
 *           that R^T R = X^T X.  Unique when X has full column rank.
 *   colsum  device FP64[n] or NULL; output colsum[j] = sum_i |X(i, j)|.
 *
 * Row blocks are factored by Householder reflections in the input precision
 * (FP32 for F32 input unless TSNMF_LEAF_F64), one wave (n <= 32) or one
 * workgroup (n > 32) keeping a running FP64 R for its contiguous slab of rows
 * (the leaf).  The leaf factors are then combined by a tree of FP64 QR
 * factorisations of stacked factors (groups of several factors per node), in
 * a second launch that climbs all levels by ticket.  The result is
 * deterministic for a given (m, n, flags, configuration).
 * The launch geometry is the library default, or the entry of the loaded
 * autotune table (tsnmf_tune_load) that matches the call.
 * Errors: -1 X NULL, -2 m < 1, -3 n < 1, -4 ld too small, -5 flags, -6 R NULL,
 * TSNMF_ERR_UNSUPPORTED for n > TSNMF_MAX_N.
 */
int tsnmf_tsqr_r(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags,
                 double* R, double* colsum, hipStream_t stream);

/*
 * tsnmf_tsqr_r_noalloc: tsnmf_tsqr_r for callers that cannot allocate device
 * memory (code under graph capture that has not reserved, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and error
 * codes; it calls no hipMalloc, hipFree or allocating routine.  Its tickets
 * and tree nodes live in a fixed 32 MiB scratch array that the library holds
 * on every device it runs on until the process ends; when the default slabs
 * would need a larger tree, the slabs are lengthened (fewer leaves) until the
 * tree fits, so R equals tsnmf_tsqr_r's up to rounding.  A shape whose tree
 * still cannot fit returns TSNMF_ERR_UNSUPPORTED (not reachable for
 * n <= TSNMF_MAX_N).  All calls on one device share that array: calls that
 * overlap on one device (other streams, other threads) race and must not be
 * made.  The first call on a device clears the array's ticket area on
 * `stream`.
 */
int tsnmf_tsqr_r_noalloc(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags,
                         double* R, double* colsum, hipStream_t stream);

/* Launch geometry of the TSQR path.  Zero fields mean "library default". */
typedef struct tsnmf_tsqr_config {
    int64_t leaf_rows;      /* rows per slab (the TSQR leaf); a slab that is not
                               a whole number of row blocks ends in a partial
                               block, padded with zero rows                     */
    int32_t tree_arity;     /* slab factors merged per tree node, 2..64 (2 = a
                               binary tree); n <= 32 only, capped at the most
                               stacked rows one workgroup pass holds; the wider
                               path merges 4 per node.  0 = library default.
                               Other values: -8 from tsnmf_tsqr_r_ex.        */
    int32_t rows_per_lane;  /* reserved, must be 0: the row block height is fixed
                               per width when the library is compiled        */
    int32_t wy_panel;       /* trailing update of FP32 row blocks with 33..64
                               columns (Sec. 3.1: any grouping of the
                               Householder steps gives the same R): 16 =
                               blocked compact-WY update on the matrix cores
                               with 16-column panels; 0 (library default) or
                               1 = unblocked (each step updates every trailing
                               column on the vector ALUs).  Other widths and
                               FP64 row blocks are unblocked.  Other values:
                               -8.                                            */
    int32_t reserved;       /* must be 0                                      */
} tsnmf_tsqr_config;

/* As tsnmf_tsqr_r with an explicit configuration (`cfg` is a host pointer or
   NULL: the library default, without the autotune table).  Every
   configuration gives the same R up to rounding. */
int tsnmf_tsqr_r_ex(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags,
                    double* R, double* colsum, const tsnmf_tsqr_config* cfg,
                    hipStream_t stream);

/*
 * tsnmf_tsqr_r_kron: tsnmf_tsqr_r of X = A (x) A without X in memory.  The
 * flow-cytometry matrix of Sec. 5.2 is this Kronecker product of a p x 5
 * matrix of cell measurements with itself (all pairs of cells); here each
 * row block of X is formed in registers from the rows of A it needs, so only
 * A (p x q, a few MB) is read, and X (p^2 x q^2) never exists.
 *   A       device FP32, p x q, row-major (lda >= q); row i p + i' of X holds
 *           A(i, a) A(i', b) in column a q + b, each product rounded to FP32
 *           once (the bytes an explicit FP32 X would hold).
 *   p       1 <= p <= 2^31;  q  1..5 (n = q^2 <= 25)
 *   R       device FP64 n x n column-major output (diag >= 0, R^T R = X^T X;
 *           in exact arithmetic R = R_A (x) R_A)
 *   colsum  device FP64[n] or NULL: l1 column sums of X
 * Same row blocks, slabs and tree as tsnmf_tsqr_r on the explicit X with
 * ld = n and the library default, so both give the same R.
 * Errors: -1 A NULL, -2 p, -3 q, -4 lda < q, -5 R NULL.
 */
int tsnmf_tsqr_r_kron(const float* A, int64_t p, int32_t q, int64_t lda, double* R, double* colsum,
                      hipStream_t stream);

/* ---- batched thin QR ---------------------------------------------------------- */

#define TSNMF_MAX_BATCH 4096

/*
 * tsnmf_tsqr_r_batched: R factors and l1 column sums of `batch` independent
 * tall-and-skinny matrices of uneven shape in one persistent launch.  The
 * paper has no batching; each matrix is treated as in tsnmf_tsqr_r (row
 * splits as the independent map tasks of Sec. 3.5, FP64 reduction of their
 * stacked R factors), and all matrices share one device work list.
 *   batch   number of matrices, 1..TSNMF_MAX_BATCH (host value).
 *   X       device array of `batch` device pointers, FP32 row-major matrices.
 *   m, n, ld  device arrays of `batch` int64: rows, columns, leading
 *           dimension of each matrix (1 <= n <= TSNMF_MAX_BATCH_N, m >= 1,
 *           ld >= n).
 *   flags   TSNMF_F32 (row-major); FP32 row blocks, FP64 R and trees.
 *   R       device array of `batch` device pointers to n x n FP64
 *           column-major outputs (diag(R) >= 0, R^T R = X^T X).
 *   colsum  device array of `batch` device pointers to FP64[n] outputs (an
 *           entry may be NULL), or NULL for no column sums.
 * The arrays are read on the device when the work runs, so a captured graph
 * may be replayed with new pointers and shapes in the same arrays.  A matrix
 * whose entry is invalid (NULL X or R, n outside 1..TSNMF_MAX_BATCH_N, m < 1,
 * or ld < n) is skipped; its R and column sums are set to NaN when R is not
 * NULL and n is in range.  Matrices are scheduled largest-first by m n^2.
 * Workspace: outside capture the call reads m, n and ld back (a host
 * synchronisation on `stream`) and grows its own device workspace as needed;
 * while capturing it uses what tsnmf_reserve_batched (or an earlier call)
 * provided and returns TSNMF_ERR_CAPTURE if that cannot hold `batch`
 * matrices.  With less tree storage than the default slabs need, the device
 * doubles every slab until the trees fit (fewer, longer slabs; same result
 * up to rounding).  Calls must not overlap on one device.
 * Returns -1 (batch), -2 (X), -3 (m), -4 (n), -5 (ld), -6 (flags), -7 (R).
 */
int tsnmf_tsqr_r_batched(int32_t batch, const void* const* X, const int64_t* m, const int64_t* n,
                         const int64_t* ld, uint32_t flags, double* const* R, double* const* colsum,
                         hipStream_t stream);

/*
 * tsnmf_tsqr_r_batched_ex: tsnmf_tsqr_r_batched with an explicit slab height
 * per width class.  The classes are 0: n = 16 with ld = 16, 1: n = 32 with
 * ld = 32 (one wave per slab), 2: other n <= 64, 3: n <= 128; a class's slab
 * is its default height times 2^slab_shift[c] (0..8; longer slabs mean fewer
 * tree leaves and fewer, longer work items).  cfg = NULL is the library
 * default, or the "batch" line of the loaded autotune table, which
 * tsnmf_tsqr_r_batched applies too.  Only the work split changes, so R
 * equals the default's up to rounding.  reserved must be 0.
 * Returns as tsnmf_tsqr_r_batched, and -8 for an invalid cfg.
 */
typedef struct tsnmf_batch_config {
    int32_t slab_shift[4];
    int32_t reserved[4];
} tsnmf_batch_config;
int tsnmf_tsqr_r_batched_ex(int32_t batch, const void* const* X, const int64_t* m, const int64_t* n,
                            const int64_t* ld, uint32_t flags, double* const* R, double* const* colsum,
                            const tsnmf_batch_config* cfg, hipStream_t stream);

/* Reserve the batched workspace for up to `max_batch` matrices with at most
   `max_rows` rows in total, at the default slab heights for any widths, so
   that tsnmf_tsqr_r_batched can be captured into a graph.  Host call,
   synchronous.  Returns -1 (max_batch outside 1..TSNMF_MAX_BATCH), -2
   (max_rows < 0). */
int tsnmf_reserve_batched(int32_t max_batch, int64_t max_rows);

/* ---- Gaussian projection -------------------------------------------------------- */

/*
 * tsnmf_gauss_proj: Y = G^T X with G (m x k) i.i.d. N(0, 1), generated on the
 * fly and never stored (Sec. 2.3; Sec. 3.2 Algorithm 1: each data row x_i
 * contributes the outer product g_i x_i^T, partial sums are combined, then
 * summed across workers).
 *   X        device, m x n, TSNMF_F32 or TSNMF_BF16, row-major (ld >= n).
 *   k        number of projected rows, multiple of 4, 4 <= k <= 4096.
 *   seed     64-bit key of the generator.
 *   row_offset  global index of X's first row (lets row shards of one matrix
 *            use the rows of G they would use unsharded).
 *   Y        device FP32, k x n column-major (ldY = k), output.
 *   colsum   device FP64[n] or NULL: l1 column sums of X in the same pass.
 *   flags    dtype | TSNMF_GP_MFMA_BF16 or TSNMF_GP_SIMD_F32 (BF16 input
 *            requires MFMA; F32 input defaults to SIMD).
 * G(i, l) is a fixed function of (seed, row_offset + i, l): Philox4x32-10
 * (Salmon et al., SC'11) with key (seed mod 2^32, seed >> 32) and counter
 * (i mod 2^32, i >> 32, l / 4, 0) gives x0..x3; u_a = ((x_a >> 8) + 1) 2^-24;
 * (G(i,4q), G(i,4q+1)) = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1) and
 * likewise (x2, x3) for columns 4q+2, 4q+3.  Independent of launch geometry.
 */
int tsnmf_gauss_proj(const void* X, int64_t m, int64_t n, int64_t ld, uint32_t flags,
                     int32_t k, uint64_t seed, int64_t row_offset, float* Y,
                     double* colsum, hipStream_t stream);

/*
 * tsnmf_gauss_colsum: s = G^T 1, i.e. s[l] = sum_{i < m} G(row_offset + i, l)
 * for the G of tsnmf_gauss_proj (the projection of a column of ones), computed
 * without reading any X.  It draws the normals exactly as the matrix-core
 * projection does (same launch shape and generation loop), so its time is the
 * cost of generating G alone; s also checks the generator's first moment
 * (E s[l] = 0, Var s[l] = m).
 *   m           rows of G (>= 1);  k  multiple of 4, 4 <= k <= 4096
 *   seed, row_offset  as in tsnmf_gauss_proj
 *   s           device FP32[k] output (FP32 sums per lane, FP64 across workgroups)
 * Errors: -1 m, -2 k, -4 row_offset < 0, -5 s NULL.
 */
int tsnmf_gauss_colsum(int64_t m, int32_t k, uint64_t seed, int64_t row_offset, float* s,
                       hipStream_t stream);

/* ---- n x n steps (FP64, one workgroup each) --------------------------------------- */

/*
 * tsnmf_select_spa: Successive Projection Algorithm (Sec. 2.1) on
 * M diag(1/colscale): r times pick j* = argmax_j ||Z(:, j)||_2^2 over columns
 * not yet picked (ties -> smallest j), then Z <- Z - u (u^T Z) with
 * u = Z(:, j*) / ||Z(:, j*)||.  Z starts as M diag(1/colscale).
 *   M         device FP64, p x n column-major (ldm >= p), p in 1..4096 (R,
 *             or the k x n projection G^T X of Sec. 2.3), n in 1..256
 *   colscale  device FP64[n] or NULL (no scaling); e.g. the colsum of tsnmf_tsqr_r
 *   r         1..n picks
 *   K         device int32[r] output, in selection order
 *   score     device FP64[r] or NULL: the winning ||Z(:, j*)||^2 of each pick
 *   info      device int32[1] output: number of columns picked (< r if the best
 *             score reached exactly 0 first; remaining K entries are -1)
 * Errors: -1 M NULL, -2 p, -3 n out of range, -4 ldm < p, -6 r outside 1..n,
 * -7 K NULL, -9 info NULL.
 */
int tsnmf_select_spa(const double* M, int32_t p, int32_t n, int32_t ldm,
                     const double* colscale, int32_t r, int32_t* K, double* score,
                     int32_t* info, hipStream_t stream);

/*
 * tsnmf_select_xray: greedy XRAY (Sec. 2.1): r times pick
 * j* = argmax_j ||Res^T M(:, j)||_2 / ||M(:, j)||_2 over unpicked nonzero
 * columns, then Res = M - M(:, K) H with H the NNLS fit of every column of M on
 * the picked columns (Lawson-Hanson, as tsnmf_nnls).  Res starts as M.
 *   M, p, n, ldm as in tsnmf_select_spa but p <= 256;  r in 1..min(n, 64)
 *   K     device int32[r] output in selection order (-1 past an early stop)
 *   info  device int32[1] output: number picked
 */
int tsnmf_select_xray(const double* M, int32_t p, int32_t n, int32_t ldm, int32_t r,
                      int32_t* K, int32_t* info, hipStream_t stream);

/*
 * tsnmf_select_gp: Gaussian-projection selection (Sec. 2.3): for each row l of
 * Y diag(1/colscale) the indices of the minimum and the maximum entries are
 * added to K (ties -> smallest j); the distinct indices are ranked by how many
 * rows chose them (descending), then by index, and the first r are returned.
 *   Y         device FP32, k x n column-major (ldy >= k), e.g. tsnmf_gauss_proj
 *   colscale  device FP64[n] or NULL
 *   K         device int32[r] output (-1 past the number found)
 *   counts    device int32[n] or NULL: selection count of every column
 *   info      device int32[1] output: number of indices returned
 */
int tsnmf_select_gp(const float* Y, int32_t k, int32_t n, int32_t ldy, const double* colscale,
                    int32_t r, int32_t* K, int32_t* counts, int32_t* info, hipStream_t stream);

/*
 * tsnmf_nnls: H(:, i) = argmin_{y >= 0} ||M(:, K) y - M(:, i)||_2^2 for every
 * column i (Sec. 2.4; with M = R this equals the fit on X itself), by the
 * Lawson-Hanson active-set method in FP64 (at most 3 r outer iterations).
 *   M, p, n, ldm  device FP64 p x n column-major
 *   K, r          device int32[r] column indices, 1 <= r <= min(n, 64)
 *   H             device FP64 r x n column-major (ldh >= r) output
 *   resid2        device FP64[n] or NULL: ||M(:, K) H(:, i) - M(:, i)||^2
 *   info          device int32[n] or NULL: 1 where the iteration cap was hit
 */
int tsnmf_nnls(const double* M, int32_t p, int32_t n, int32_t ldm, const int32_t* K, int32_t r,
               double* H, int32_t ldh, double* resid2, int32_t* info, hipStream_t stream);

/*
 * tsnmf_residual: relative residual ||M - M(:, K) H||_F^2 / ||M||_F^2 (Sec. 4's
 * error measure; Sec. 2.4 shows it can be computed from R instead of X).
 *   relerr  device FP64[1] output (0 when M = 0)
 */
int tsnmf_residual(const double* M, int32_t p, int32_t n, int32_t ldm, const int32_t* K,
                   int32_t r, const double* H, int32_t ldh, double* relerr, hipStream_t stream);

/*
 * tsnmf_rsvd: SVD of the n x n factor R = U diag(S) V^T (Sec. 3.1, "TSQR and
 * R-SVD": with X = QR, X = (QU) diag(S) V^T, so S and V are the singular
 * values and right singular vectors of X).  FP64 one-sided Jacobi on one
 * workgroup, which determines small singular values to high relative
 * accuracy.
 *   R     device FP64 n x n column-major (ldr >= n), 1 <= n <= 256
 *   S     device FP64[n] output, descending
 *   V     device FP64 n x n column-major output (ldv >= n)
 *   U     device FP64 n x n column-major output (ldu >= n) or NULL; columns of
 *         zero singular values are zero
 *   info  device int32[1] or NULL: Jacobi sweeps used, -1 if not converged in 40
 * Each pair (u_i, v_i) is signed so that the largest-magnitude entry of v_i
 * is positive.  Errors: -1 R, -2 n, -3 ldr, -4 S, -5 V, -6 ldv, -8 ldu.
 */
int tsnmf_rsvd(const double* R, int32_t n, int32_t ldr, double* S, double* V, int32_t ldv, double* U,
               int32_t ldu, int32_t* info, hipStream_t stream);

/*
 * tsnmf_rank_sweep: residuals of the separable fit for every rank 1..rmax in
 * the reduced space (Sec. 2.2, Sec. 2.4: the selection, the NNLS fit and the
 * residual are the same on R as on X, so a whole residual curve costs n x n
 * work).  K = SPA's rmax picks on R diag(1/colscale) (in order; the first r
 * are SPA's picks for r); for each r, H_r = NNLS(R(:, K[:r]), R) and
 * resid[r-1] = ||R - R(:, K[:r]) H_r||_F^2 / ||R||_F^2.
 *   R, p, n, ldr  device FP64 p x n column-major, p, n in 1..256
 *   colscale      device FP64[n] or NULL (as tsnmf_select_spa)
 *   rmax          1..min(n, 64)
 *   K             device int32[rmax] output
 *   H             device FP64 rmax x n (ldh >= rmax): work space; on return
 *                 H_rmax in its first rmax rows
 *   resid         device FP64[rmax] output
 *   info          device int32[1] output: SPA's picks (< rmax if the residual
 *                 reached 0 first; resid is NaN past it)
 * Errors: -1 R, -2 p, -3 n, -4 ldr, -6 rmax, -7 K, -8 H, -9 ldh, -10 resid,
 * -11 info.
 */
int tsnmf_rank_sweep(const double* R, int32_t p, int32_t n, int32_t ldr, const double* colscale,
                     int32_t rmax, int32_t* K, double* H, int32_t ldh, double* resid, int32_t* info,
                     hipStream_t stream);

/* ---- one pass over a matrix delivered in row blocks -------------------------------- */

/*
 * A tsnmf_onepass_t holds the state of one pass over a tall matrix X whose
 * rows arrive in consecutive blocks, possibly from host memory and in total
 * larger than device memory (Sec. 4 and Sec. 5.1 work on 286 GB and 2 TB
 * matrices read from disk; the method reads the data once, Sec. 3.3 and
 * Sec. 3.5).  For every block it computes, in the same pass over the block:
 * the block's R factor and column sums (as tsnmf_tsqr_r) and, when k > 0, the
 * block's share of G^T X with the rows of G that the block's global row
 * indices select (as tsnmf_gauss_proj with row_offset = rows pushed before),
 * so TSQR and the projection read the data once together (Sec. 3.5: the
 * projection cannot give H in the projected space, so R is computed in the
 * same pass).  The device state is the running FP64 R (the block's R and the
 * running R are merged by an FP64 QR of the two stacked factors: one more
 * node of the reduction tree), the FP64 column sums and FP64 G^T X: O(n^2 +
 * k n) doubles whatever the number of rows, a complete resumable state
 * (tsnmf_onepass_save / _load).
 *
 * tsnmf_onepass_create: new state for n columns.
 *   n       1..TSNMF_MAX_N.
 *   flags   TSNMF_F32 or TSNMF_F64 | TSNMF_ROW_MAJOR or TSNMF_COL_MAJOR
 *           [| TSNMF_LEAF_F64] [| TSNMF_GP_MFMA_BF16 or TSNMF_GP_SIMD_F32];
 *           with k > 0 the input must be TSNMF_F32, TSNMF_ROW_MAJOR.
 *   k       0 (no projection) or as tsnmf_gauss_proj (multiple of 4, 4..4096).
 *   seed    key of the projection's generator.
 *   out     host pointer that receives the handle.
 * Allocates the state and two 64 MiB device blocks for host input.  Host call.
 * Errors: -1 n, -2 flags, -3 k, -5 out; TSNMF_ERR_NOMEM, TSNMF_ERR_HIP.
 */
typedef struct tsnmf_onepass_s* tsnmf_onepass_t;
int tsnmf_onepass_create(int32_t n, uint32_t flags, int32_t k, uint64_t seed, tsnmf_onepass_t* out);

/*
 * tsnmf_onepass_push: the next `rows` rows of X, in device memory (dtype and
 * layout of the create flags; ld >= n row-major, >= rows column-major).
 * Enqueued on `stream`; the block must stay valid until the stream reaches
 * the end of the call's work.  Pushes to one state must be ordered (one
 * stream, or synchronised streams); the library workspace is shared as in
 * tsnmf_tsqr_r.  Errors: -1 state, -2 X, -3 rows < 1, -4 ld.
 */
int tsnmf_onepass_push(tsnmf_onepass_t p, const void* X, int64_t rows, int64_t ld, hipStream_t stream);

/*
 * tsnmf_onepass_push_host: the next `rows` rows of X in HOST memory
 * (row-major only, ld >= n), e.g. a memory-mapped file.  The rows go to the
 * device in blocks of tsnmf_onepass_block_rows() rows through two device
 * buffers: the copy of one block (on a copy stream of the library) overlaps
 * the work on the previous one (on `stream`).  Pinned host memory (allocated
 * by hipHostMalloc) is copied by DMA directly, or, for a state without
 * projection (k = 0), read by the leaf kernels over the host link with no
 * copy at all (the call then waits for `stream`); pageable memory is first
 * copied by host threads into pinned staging buffers.  Returns when every
 * row has been copied or read (X may then be reused); the remaining work
 * completes on `stream`.  The result equals that of tsnmf_onepass_push
 * called with the same blocks.  Errors: -1 state, -2 X, -3 rows < 1, -4 ld,
 * TSNMF_ERR_UNSUPPORTED for a column-major state.
 */
int tsnmf_onepass_push_host(tsnmf_onepass_t p, const void* X, int64_t rows, int64_t ld, hipStream_t stream);

/* Rows per device block of tsnmf_onepass_push_host (host value), and rows
   pushed so far.  Errors: -1 state, -2 out. */
int tsnmf_onepass_block_rows(tsnmf_onepass_t p, int64_t* rows);
int tsnmf_onepass_rows(tsnmf_onepass_t p, int64_t* rows);

/*
 * tsnmf_onepass_result: results over all rows pushed so far (the state is
 * unchanged; more rows may follow).
 *   R       device FP64 n x n column-major output (diag >= 0, R^T R = X^T X)
 *   colsum  device FP64[n] output or NULL
 *   Y       device FP32 k x n column-major output (G^T X) or NULL
 * Before any push, R, colsum and Y are zero.  Errors: -1 state, -2 R.
 */
int tsnmf_onepass_result(tsnmf_onepass_t p, double* R, double* colsum, float* Y, hipStream_t stream);

/*
 * Resumable state: tsnmf_onepass_state_bytes gives the size of the saved
 * state; tsnmf_onepass_save writes it to HOST memory `host` (a header with n,
 * k, flags, seed and the rows pushed, then R, the column sums and G^T X in
 * FP64) after waiting for `stream`; tsnmf_onepass_load restores it into a
 * state created with the same n, flags, k and seed (else -2), after which
 * pushes continue exactly where the saved pass stopped.  Errors: -1 state,
 * -2 host buffer or mismatching header, -3 (bytes) too small.
 */
int tsnmf_onepass_state_bytes(tsnmf_onepass_t p, size_t* bytes);
int tsnmf_onepass_save(tsnmf_onepass_t p, void* host, size_t bytes, hipStream_t stream);
int tsnmf_onepass_load(tsnmf_onepass_t p, const void* host, size_t bytes, hipStream_t stream);

/* Frees the state (waits for its pending work).  Errors: -1 state. */
int tsnmf_onepass_destroy(tsnmf_onepass_t p);

/* ---- housekeeping ------------------------------------------------------------------- */

/* Grow the current device's workspace so that TSQR calls with m <= max_m and
   n <= max_n (any dtype, layout, leaf precision and row stride, default
   geometry or a tuned entry; an explicit tsnmf_tsqr_config.leaf_rows that
   makes more than 2048 slabs may need more), and projections with
   k <= max_k, need no allocation (required before graph capture).  Host
   call, synchronous. */
int tsnmf_reserve(int64_t max_m, int32_t max_n, int32_t max_k);

/* Load the autotune table (host path of a text file written by the library's
   autotuner; NULL clears the table).  Each line
       tsqr <f32|f64> <row|col> <leaf f32|f64> <ld==n 1|0> <n> <floor(log2 m)> <leaf_rows> <tree_arity>
   gives the launch geometry (as tsnmf_tsqr_config) that tsnmf_tsqr_r applies
   to calls with that input dtype, layout, row-block precision, contiguity,
   width and row-count bucket; '#' starts a comment.  Calls without an entry
   use the library default.  Returns 0, or -1 if the file cannot be read or a
   line is malformed (the previous table is then kept).  Host call. */
int tsnmf_tune_load(const char* path);

/* Free the workspace buffers that growth has retired on the current device
   (single-call and batched), after waiting for the device.  Graphs captured
   before that growth must not be replayed afterwards.  Host call. */
int tsnmf_workspace_release(void);

/* Profiling aid.  While enabled, TSQR and projection calls record HIP
   events on their stream around their main kernel ("stage 0": the leaf /
   projection kernel; for the batched call the persistent kernel, trees
   included) and, with on = 1, also around the rest of the call ("stage 1":
   reduction tree and finalisation; for the batched call the device planner).
   on = 2 records stage 0 only (two events per call, the least intrusive);
   on = 0 stops recording.
   tsnmf_profile_query waits for the recorded events (host synchronisation),
   returns the summed elapsed milliseconds and the number of calls of a
   stage, and clears that stage.  Not for graph capture. */
int tsnmf_profile_enable(int on);
int tsnmf_profile_query(int stage, double* total_ms, int64_t* calls);

/* Human-readable text of a return code (static storage). */
const char* tsnmf_status_string(int status);

/* HIP error code of the most recent TSNMF_ERR_HIP on the calling thread. */
int tsnmf_last_hip_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int tsnmf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSNMF_H */
