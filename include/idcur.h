/*
 * idcur.h -- C ABI of the MI355X (gfx950) interpolative-decomposition / CUR
 * library (libidcur.so).
 *
 * The operations follow Voronin & Martinsson, "Efficient Algorithms for CUR and
 * Interpolative Matrix Decompositions":
 *   idcur_id_col        column ID  A ~ A(:, J(1:k)) [I_k T] P*      (Section 2.3, Algorithm 1)
 *   idcur_id_row        row ID     A ~ W A(I(1:k), :)                (remark closing Section 2.3)
 *   idcur_id_two_sided  two-sided  A ~ W A(I(1:k), J(1:k)) V*        (Section 2.4, Algorithm 2)
 *   idcur_cur           CUR-ID     A ~ C U R                         (Section 3, Algorithm 3)
 * each deterministic (k steps of column-pivoted QR on A itself) or randomized
 * (Section 5: Y = Omega A with an (k+p) x m Gaussian Omega, eq. (Y=OmegaA), then
 * q orthonormalised power steps, Section 5.3, then k CPQR steps on Y).
 *
 * Conventions shared by every entry point
 *   - All matrices are ROW-MAJOR with an explicit leading dimension (elements
 *     between consecutive rows). A is m x n.
 *   - Every array argument is a DEVICE pointer owned by the caller, except
 *     where marked "host". The library never allocates or frees caller memory.
 *   - Scratch memory is a caller-provided device workspace whose size comes from
 *     idcur_workspace_bytes() for the same (op, dtype, m, n, opts).
 *   - Indices are 0-based int32. J (length n) and I (length m) are full
 *     permutations with the skeleton first: J[0..k-1] are the selected columns.
 *   - Work is enqueued on the context's stream; calls return before the device
 *     finishes. Argument errors are returned synchronously (nothing is enqueued).
 *     Conditions found on the device (rank cap, non-finite data, a grid wait
 *     that exceeded its spin limit) are written to a device status word that
 *     idcur_sync_status() reads after synchronising the stream.
 *   - Outputs are undefined when a call returns an error.
 */
#ifndef IDCUR_H
#define IDCUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct idcur_ctx idcur_ctx;

typedef enum {
  IDCUR_OK = 0,
  IDCUR_EINVAL = -1,      /* invalid argument (sizes, rank, leading dimension, null pointer) */
  IDCUR_EDTYPE = -2,      /* unsupported dtype / precision combination */
  IDCUR_EWORKSPACE = -3,  /* workspace missing or smaller than idcur_workspace_bytes() */
  IDCUR_EHIP = -4,        /* a HIP runtime call failed (message in idcur_last_error) */
  IDCUR_ERANKCAP = -5,    /* device: tolerance not met within the rank cap */
  IDCUR_ENONFINITE = -6,  /* device: NaN or Inf met in the column norms */
  IDCUR_ETIMEOUT = -7     /* device: a grid-wide wait exceeded its spin limit */
} idcur_status;

typedef enum { IDCUR_F64 = 0, IDCUR_F32 = 1 } idcur_dtype;

/* Input precision of the sketch and power-step GEMMs (accumulation is FP32).
 * BF16 / FP16 need IDCUR_F32 data (IDCUR_EDTYPE otherwise): A and the thin operand
 * (Omega, or the orthonormal basis of a power step) are rounded to nearest even in
 * 16 bits as the matrix cores read them, products are accumulated in FP32 and
 * split-K partial sums in FP64. FP16 first multiplies A by 2^(15-e), where
 * max|A| lies in [2^(e-1), 2^e), so that A's entries stay clear of the FP16
 * subnormal range, and divides the FP32 result by the same power of two. Every
 * later step (orthonormalisation, CPQR, T, row ID, U) runs as in NATIVE. */
typedef enum { IDCUR_PREC_NATIVE = 0, IDCUR_PREC_BF16 = 1, IDCUR_PREC_FP16 = 2 } idcur_prec;

/* How the CPQR keeps the trailing column norms between pivots: downdated
 * (nu^2 -= s^2, recomputed from the data when the downdate has cancelled) or
 * recomputed exactly at every step. */
typedef enum { IDCUR_NORMS_DOWNDATE = 0, IDCUR_NORMS_EXACT = 1 } idcur_norms;

typedef enum {
  IDCUR_OP_ID_COL = 0,
  IDCUR_OP_ID_ROW = 1,
  IDCUR_OP_TWO_SIDED = 2,
  IDCUR_OP_CUR = 3,
  IDCUR_OP_SKETCH = 4,      /* idcur_sketch of A (the sketch an ID_COL call takes)  */
  IDCUR_OP_SKETCH_ROW = 5   /* idcur_sketch of A^T (the sketch an ID_ROW call takes) */
} idcur_op;

/* Kind of sketch matrix (Section 5): i.i.d. Gaussian (Section 5.1), or the
 * subsampled randomized Hadamard transform, the real counterpart of the
 * structured sketch of Section 5.2 (eq. (def_srft)): the unitary DFT replaced by
 * the orthonormal Walsh-Hadamard matrix of order m' (the smallest power of two
 * >= the sketched dimension M, the matrix extended by zero rows), the random
 * unit-modulus diagonal by random signs, so that
 *   Omega(r, i) = l^(-1/2) (-1)^popcount(rows[r] & i) sign_i,  r < l, i < M.
 * The structured sketch needs q = 0, NATIVE precision, no omega, l <= 512, and
 * its random inputs from the caller: srht_rows (device int32[l], distinct values
 * in [0, m'); values out of range are reported as IDCUR_EINVAL by
 * idcur_sync_status) and srht_signs (device int8[M]: -1 where negative, else
 * +1). M is m for the column ID, two-sided ID, CUR and IDCUR_OP_SKETCH, and n for
 * the row ID and IDCUR_OP_SKETCH_ROW. */
typedef enum { IDCUR_SKETCH_GAUSSIAN = 0, IDCUR_SKETCH_SRHT = 1 } idcur_sketch_kind;

typedef struct {
  int32_t k;          /* > 0: fixed rank, k < min(m, n), k <= 4096. 0: tolerance mode. */
  int32_t kmax;       /* rank cap in tolerance mode (ignored when k > 0), <= 4096; the
                         sketch width k + p (kmax + p) is also at most 4096.           */
  double tol;         /* tolerance mode: smallest k with |Y_res|_F <= tol |Y|_F
                         (Section 3: continue the QR until |E| is below a threshold). */
  double rank_tol;    /* stop early (exact rank deficiency, Section 2.3) when the
                         largest remaining column norm <= rank_tol * largest initial
                         norm; 0 selects 10 sqrt(l) u with a fixed rank and sqrt(l) u
                         in tolerance mode, u the unit roundoff of dtype        */
  int32_t p;          /* oversampling (Section 5.1); < 0: deterministic, Y = A.         */
  int32_t q;          /* orthonormalised power steps (Section 5.3), >= 0.               */
  uint64_t seed;      /* Philox4x32-10 key for Omega when omega == NULL.                */
  const void* omega;  /* optional device Omega, l x m row-major (l = k+p, or kmax+p),
                         leading dimension m, same dtype as A; NULL: generated.        */
  int32_t prec;       /* idcur_prec of the sketch GEMMs.                                 */
  int32_t norms;      /* idcur_norms.                                                    */
  int32_t sketch;     /* idcur_sketch_kind (default Gaussian).                           */
  const int8_t* srht_signs;   /* structured sketch: device int8[M] signs (see above).     */
  const int32_t* srht_rows;   /* structured sketch: device int32[l] sampled rows.         */
  int32_t u_correct;  /* idcur_cur only: 0 solves U R = V* (Section 4.3, eq. (cur_ur_sys));
                         1 solves U R = V* + C^+ E, E = A - C V* the column-ID error
                         (eq. (cur_ur_sys2)), which in exact arithmetic gives the
                         U minimising |A - C U R|_F for the chosen C and R.        */
  double t_reg;       /* 0: T = S11^{-1} S12 (Section 2.3, eq. (S11T=S12)). In (0, 1): the
                         stabilized T of Section 4.1 (eq. (lsqr_for_T) with a Tikhonov
                         term), T = argmin |S11 U - S12|_F^2 + lam^2 |U|_F^2 with
                         lam = t_reg max_j |S11(:, j)|_2 (= t_reg |S11(1, 1)| for the
                         pivoted QR), for every interpolation matrix the call forms
                         (column ID, row ID, both IDs of a two-sided ID or CUR).
                         Solved as the least-squares problem [S11; lam I] U =
                         [S12; 0] through an FP64 Cholesky QR taken twice, with an
                         error of about u / t_reg relative to |T| (u = 2^-53), so
                         t_reg should exceed about 1e-8. Other values:
                         IDCUR_EINVAL.                                             */
  double t_svd;       /* 0: as t_reg says. In (0, 1): the truncated-SVD T of Section 4.1
                         (the stabilized pseudo-inverse of S11 in eq. (lsqr_for_T)):
                         with S11 = U D V^T, the terms whose singular value is below
                         t_svd times the largest are dropped and T = V D^-1 U^T S12
                         over the rest, for every interpolation matrix the call forms.
                         The SVD is taken by one-sided Jacobi rotations in FP64 (at
                         most 16 sweeps). Excludes t_reg > 0 (IDCUR_EINVAL); other
                         values: IDCUR_EINVAL. This build switches the path off:
                         any t_svd > 0 returns IDCUR_EINVAL.                         */
} idcur_opts;

/* Fill *opts with defaults: k = 0, kmax = 0, tol = 0, rank_tol = 0, p = -1
 * (deterministic), q = 0, seed = 0, omega = NULL, NATIVE precision, downdated norms,
 * Gaussian sketch (srht_signs = srht_rows = NULL), u_correct = 0, t_reg = 0,
 * t_svd = 0. */
void idcur_opts_default(idcur_opts* opts /* host */);

/* Create a context bound to `stream` (a hipStream_t, borrowed, may be NULL for the
 * null stream). Allocates the context's small device status block on the current
 * device. Returns IDCUR_EHIP if that fails. */
idcur_status idcur_create(idcur_ctx** ctx /* host out */, void* stream);
idcur_status idcur_set_stream(idcur_ctx* ctx, void* stream);
idcur_status idcur_destroy(idcur_ctx* ctx);

/* Message for the last error returned by a call on this context (host string,
 * valid until the next call on the context). */
const char* idcur_last_error(const idcur_ctx* ctx);

/* Synchronise the context's stream, read and clear the device status word.
 * Returns IDCUR_OK or one of the device conditions (ERANKCAP, ENONFINITE, ETIMEOUT). */
idcur_status idcur_sync_status(idcur_ctx* ctx);

/* Per-stage GPU timers for measurement. With timing enabled, every later call on
 * this context records a pair of HIP events on the context's stream around each
 * stage: "omega", "pack", "sketch_gemm" (the sketch / power-step GEMM kernels
 * alone, without their split-K reduction), "orth", "cpqr", "trsm", "gather",
 * "row_id", "u_solve", "error", "backward", "batched", "srht" (the structured
 * sketch kernels), "spmm" (the sparse sketch kernels). Enabling (or disabling)
 * synchronises the stream and clears the accumulated marks. idcur_timing_read
 * synchronises and returns the summed elapsed milliseconds and the number of
 * marks of one stage (host outputs). */
idcur_status idcur_timing_enable(idcur_ctx* ctx, int32_t enable);
idcur_status idcur_timing_read(idcur_ctx* ctx, const char* stage, double* total_ms /* host */,
                               int32_t* count /* host */);

/* Workspace size in bytes for one call of `op` (idcur_op) with these arguments. */
idcur_status idcur_workspace_bytes(idcur_ctx* ctx, int32_t op, int32_t dtype, int64_t m, int64_t n,
                                   const idcur_opts* opts /* host */, size_t* bytes /* host out */);

/* Column ID (Section 2.3 eq. (S11T=S12), (column_approx_id2); Algorithm 1, or
 * Algorithm 4 with the power scheme of Section 5.3 when opts->p >= 0).
 *   A      m x n, leading dimension lda >= n.
 *   k_out  device int32[1]: the rank produced (k, or less on exact rank
 *          deficiency, or the tolerance-mode rank).
 *   J      device int32[n]: column permutation, skeleton first.
 *   T      device, dtype of A: k_out x (n - k_out) interpolation matrix, row r at
 *          T + r*ldt; ldt >= n - k (fixed rank) or >= n (tolerance mode, where the
 *          caller sizes T as kmax x n). Columns t >= ldt are never written: when
 *          exact rank deficiency makes k_out < k, pass ldt >= n - k_out (ldt = n
 *          always suffices) to receive all of T.
 * V* = [I T] P* is not formed: V*(:, J[s]) = e_s, V*(:, J[k+t]) = T(:, t). */
idcur_status idcur_id_col(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                          const idcur_opts* opts, void* ws, size_t ws_bytes,
                          int32_t* k_out, int32_t* J, void* T, int64_t ldt);

/* idcur_id_col without a workspace, for callers that cannot allocate device
 * memory (code under stream capture into a graph, serving loops, harnesses that
 * forbid allocation): the scratch memory is a fixed 64 MiB device array inside
 * the library, one per GPU, held until the process ends; the call itself
 * allocates nothing (no device or event allocation; stage timers are not taken).
 * Arguments, outputs and results are those of idcur_id_col on the same inputs.
 * Returns IDCUR_EWORKSPACE, with the size in idcur_last_error, when
 * idcur_workspace_bytes(IDCUR_OP_ID_COL, ...) exceeds 64 MiB (an FP32
 * 2400 x 1600, k = 100, p = 10, q = 1 column ID needs 28 MB and fits; the FP32
 * 20000 x 10000, k = 200 one needs 339 MB and is refused). Every call on one
 * GPU uses the same array and leaves its contents behind: calls that overlap on
 * one GPU (different streams or threads) race and must be serialised by the
 * caller. */
idcur_status idcur_id_col_noalloc(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                                  const idcur_opts* opts, int32_t* k_out, int32_t* J, void* T, int64_t ldt);

/* Column ID of a sparse A (Algorithm 4 with q = 0; the sparse matrices of
 * Sections 1 and 3 that motivate the ID and CUR) in compressed sparse column
 * form: the entries of column j are p = colptr[j] .. colptr[j+1] - 1, stored at
 * rows rowidx[p] with values vals[p] (any order within a column; repeated rows
 * add up). The sketch Y = Omega A (l = k + p rows, Omega as for idcur_id_col:
 * opts->omega l x m row-major, or drawn from opts->seed) reads each stored entry
 * once; the CPQR and T then run on Y as in idcur_id_col, so the outputs (k_out, J,
 * T, ldt) have the same meaning. Requires p >= 0 and k (kmax) + p < m, q = 0, the
 * Gaussian sketch and NATIVE precision; t_reg applies as usual.
 *   colptr  device int64[n + 1], nondecreasing, 0 <= colptr[j] <= nnz.
 *   rowidx  device int32[nnz], each in [0, m).   vals  device, dtype, [nnz].
 * Index values out of range are skipped and raise IDCUR_EINVAL from
 * idcur_sync_status. All buffers are the caller's; the workspace is sized by
 * idcur_id_col_csc_workspace_bytes for the same (dtype, m, n, nnz, opts). */
idcur_status idcur_id_col_csc_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz,
                                              const idcur_opts* opts /* host */, size_t* bytes /* host out */);
idcur_status idcur_id_col_csc(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                              const int32_t* rowidx, const void* vals, const idcur_opts* opts /* host */, void* ws,
                              size_t ws_bytes, int32_t* k_out, int32_t* J, void* T, int64_t ldt);

/* CUR-ID of a sparse A in compressed sparse column form (Algorithm 3 on the
 * sparse column ID above; Section 1 and Section 3 motivate the CUR by sparse
 * matrices, whose C and R are sparse): C = A(:, J(1:k)) and R = A(I(1:k), :) are
 * gathered from the stored entries into dense blocks (repeated rows of a column
 * add up), the row ID of C and U = V* R^+ follow as in idcur_cur. Arguments as in
 * idcur_id_col_csc for A and the options (p >= 0, q = 0, Gaussian sketch, NATIVE
 * precision) and as in idcur_cur for the outputs: k_out device int32[2] (column
 * rank, rank of C), J int32[n], I int32[m], U (ldu >= k), optional C (m x k, ldc
 * >= k) and R (k x n, ldr >= n), all dtype. u_correct must be 0 (the corrected
 * system needs the dense A). The workspace comes from
 * idcur_cur_csc_workspace_bytes for the same (dtype, m, n, nnz, opts). */
idcur_status idcur_cur_csc_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz,
                                           const idcur_opts* opts /* host */, size_t* bytes /* host out */);
idcur_status idcur_cur_csc(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                           const int32_t* rowidx, const void* vals, const idcur_opts* opts, void* ws, size_t ws_bytes,
                           int32_t* k_out, int32_t* J, int32_t* I, void* U, int64_t ldu, void* C, int64_t ldc, void* R,
                           int64_t ldr);

/* Row ID (remark closing Section 2.3): the column ID of A^T, computed from A in
 * place (no transposed copy). I (device int32[m]) is the row permutation, Tr the
 * k_out x (m - k_out) row interpolation matrix (ldtr as ldt above with m for n);
 * W = P [I_k; Tr^T] with row I[r] of W equal to e_r^T for r < k_out.
 * With p >= 0 the sketch is Omega A^T, Omega of size l x n. */
idcur_status idcur_id_row(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                          const idcur_opts* opts, void* ws, size_t ws_bytes,
                          int32_t* k_out, int32_t* I, void* Tr, int64_t ldtr);

/* Two-sided ID (Section 2.4 eq. (boat), (two_sided_approx_id); Algorithm 2):
 * the column ID (J, T) of A, then a full-rank ID of C^T with C = A(:, J(1:k)),
 * giving I and Tr (k x (m - k)). k_out is device int32[2]: {column rank, rank of C}. */
idcur_status idcur_id_two_sided(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A,
                                int64_t lda, const idcur_opts* opts, void* ws, size_t ws_bytes,
                                int32_t* k_out, int32_t* J, void* T, int64_t ldt,
                                int32_t* I, void* Tr, int64_t ldtr);

/* CUR-ID (Section 3 eq. (choice_C_and_R), (defU); Algorithm 3):
 * C = A(:, J(1:k)) (m x k), R = A(I(1:k), :) (k x n), U = V* R^+ (k x k), U solving
 * U R = V* in the least-squares sense (Section 4.3) through a QR factorisation of
 * R^T. k_out as for the two-sided ID. C and R are optional (NULL: not written).
 * U has leading dimension ldu >= k (kmax in tolerance mode). */
idcur_status idcur_cur(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                       const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out,
                       int32_t* J, int32_t* I, void* U, int64_t ldu,
                       void* C, int64_t ldc, void* R, int64_t ldr);

/* The randomized sketch alone (Section 5.1, eq. (Y=OmegaA); power steps of
 * Section 5.3): the matrix Y whose k-step pivoted QR selects the skeleton.
 *   op = IDCUR_OP_SKETCH:      Y = Omega A   (l x n, Omega l x m),
 *   op = IDCUR_OP_SKETCH_ROW:  Y = Omega A^T (l x m, Omega l x n),
 * then opts->q times Y <- orth(orth(Y) B^T) B with B the sketched matrix (A or
 * A^T) and orth(.) an orthonormal basis of the row space (Cholesky QR with an FP64
 * Gram matrix). l = k + p (kmax + p in tolerance mode); requires p >= 0 and l
 * below the sketched dimension (m for SKETCH, n for SKETCH_ROW), else
 * IDCUR_EINVAL. Omega and the precision are taken from opts exactly as the ID
 * calls take them, so the same opts give the Y those calls factor.
 *   Yt   device, dtype: Y^T, row c at Yt + c*ldy (c < n, or c < m for
 *        SKETCH_ROW), ldy >= l.
 * Workspace from idcur_workspace_bytes with the same op. */
idcur_status idcur_sketch(idcur_ctx* ctx, int32_t op, int32_t dtype, int64_t m, int64_t n, const void* A,
                          int64_t lda, const idcur_opts* opts, void* ws, size_t ws_bytes, void* Yt, int64_t ldy);

/* Error measurement (the relative Frobenius errors reported with every result).
 * Both write out[0] = |A - C W|_F^2 and out[1] = |A|_F^2 (device doubles), with
 * FP64 matrix-core products and FP64 sums (a fixed reduction order):
 *   idcur_id_error   C = A(:, J(1:k)), W = V* = [I T] P*, so |A - C V*|_F is the
 *                    column-ID error of Section 2.3 eq. (id_error).
 *   idcur_cur_error  W = U R, the CUR-ID error |A - C U R|_F of Section 3.
 * k_out is the device rank array written by the decomposition call (k_out[0]:
 * column rank; k_out[1]: row rank for the CUR); kcap is the k (or kmax) that
 * sized those buffers. Workspace from idcur_error_workspace_bytes (which: 0 for
 * the ID error, 1 for the CUR error). */
idcur_status idcur_error_workspace_bytes(idcur_ctx* ctx, int32_t which, int32_t dtype, int64_t m, int64_t n,
                                         int32_t kcap, size_t* bytes /* host out */);
idcur_status idcur_id_error(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                            const int32_t* J, const void* T, int64_t ldt, const int32_t* k_out, int32_t kcap,
                            void* ws, size_t ws_bytes, double* out);
idcur_status idcur_cur_error(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                             const void* C, int64_t ldc, const void* U, int64_t ldu, const void* R, int64_t ldr,
                             const int32_t* k_out, int32_t kcap, void* ws, size_t ws_bytes, double* out);

/* Gradient of the column-ID reconstruction loss with the skeleton frozen
 * (the column ID of Section 2.3 / Algorithm 1, sketched as in Section 5.1):
 *   Y = Omega A (omega != NULL) or Y = A (omega == NULL),
 *   T = argmin_X |Y(:,J1) X - Y(:,J2)|_F  (= S11^{-1} S12, Section 4.1),
 *   L = |A(:,J2) - A(:,J1) T|_F^2,        J1 = J[0..k-1], J2 = J[k..n-1].
 * Writes dA = scale * dL/dA (m x n, row-major, ld ldda >= n; overwritten) with J
 * and Omega held fixed: the explicit terms 2E and -2 E T^T plus the path through
 * T (the derivative of the least-squares solution, M = (Y1^T Y1)^{-1} Tbar with
 * Tbar = -2 A(:,J1)^T E; Y1^T Y1 factored in FP64 on the device).
 *   A      m x n (ld lda), dtype.
 *   omega  l x m row-major (ld m), same dtype, or NULL; k <= l <= m.
 *   J      device int32[n], a permutation (e.g. from idcur_id_col); values out of
 *          range are reported as IDCUR_EINVAL by idcur_sync_status.
 *   k      rank, 0 < k < min(m, n), k <= 4096 (host value).
 *   T      k x (n-k) (ld ldt >= n-k), dtype: the interpolation matrix of that ID.
 * Workspace from idcur_id_col_backward_workspace_bytes(dtype, m, n, k, l,
 * sketched = omega != NULL). */
idcur_status idcur_id_col_backward_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int32_t k,
                                                   int32_t l, int32_t sketched, size_t* bytes /* host out */);
idcur_status idcur_id_col_backward(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                                   const void* omega, int32_t l, const int32_t* J, int32_t k, const void* T,
                                   int64_t ldt, double scale, void* dA, int64_t ldda, void* ws, size_t ws_bytes);

/* Batched adaptive-rank column ID: nblk independent FP32 blocks in one persistent
 * launch (Section 3's tolerance variant of the column ID of Section 2.3, on the
 * randomized sketch of Section 5.1 / Algorithm 4). For block b (m[b] x n[b],
 * row-major at A[b] with leading dimension lda[b]):
 *   Y = Omega(:l, :m_b) A_b with one Omega (l_cap x mmax, i.i.d. N(0,1), drawn
 *   from opts->seed as idcur_gaussian(rows = l_cap, cols = mmax, stream 0) would,
 *   or opts->omega: l_cap x mmax row-major FP32, ld mmax) shared by all blocks;
 *   column-pivoted Householder QR of Y with exact column norms.
 *   Tolerance mode (opts->k == 0): the rank is the smallest k with
 *   |Y_res|_F <= opts->tol |Y|_F, at most l - p steps; l starts at
 *   min(32, l_cap) and doubles up to l_cap = opts->kmax + opts->p when the
 *   tolerance is not met (a block that misses it at l_cap keeps l_cap - p steps
 *   and sets IDCUR_ERANKCAP in the device status). Fixed rank (opts->k > 0):
 *   l = k + p, k steps. Exact rank deficiency stops early: when the largest
 *   remaining column norm is <= opts->rank_tol times the largest initial column
 *   norm of Y (opts->rank_tol == 0 selects sqrt(l_cap) u32 in tolerance mode,
 *   u32 = 2^-24, so that the Frobenius rule decides unless pivots reach rounding
 *   level, and 10 sqrt(l_cap) u32 with a fixed rank).
 *   T = S11^{-1} S12 by FP64 back-substitution.
 * Limits: 1 <= n_b <= nmax <= 512, 1 <= m_b <= mmax, (k or kmax) + p <= 64,
 * p >= 1, q = 0, t_reg = t_svd = 0, NATIVE precision, dtype IDCUR_F32. A block outside its limits
 * gets k_out[b] = -1 and IDCUR_EINVAL from idcur_sync_status.
 * All arrays are DEVICE arrays of nblk entries: m, n (int32), A (pointers to
 * const float), lda (int64), and the outputs k_out (int32), J (pointers to
 * int32[n_b]: pivots first, then the other columns in increasing order), T
 * (pointers to float, k_out[b] x (n_b - k_out[b]) written with leading
 * dimension ldt[b] >= n_b; the caller sizes each T as (k or kmax) x n_b).
 * The call only enqueues kernels on the context's stream (no allocation, no
 * host synchronisation, no memset node), so it can be captured in a hipGraph.
 * Results do not depend on the launch variant. Workspace from
 * idcur_id_col_batched_workspace_bytes. */
idcur_status idcur_id_col_batched_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax,
                                                  int32_t nmax, const idcur_opts* opts, size_t* bytes /* host out */);
idcur_status idcur_id_col_batched(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax, int32_t nmax,
                                  const int32_t* m, const int32_t* n, const void* const* A, const int64_t* lda,
                                  const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out, int32_t* const* J,
                                  void* const* T, const int64_t* ldt);
/* Autotuner: runs the batched call once per launch variant (sketch prefetch
 * depth, workgroups per CU, largest-first ordering), times each with HIP events
 * on the context's stream (synchronising it), keeps the fastest for this size
 * class (nblk rounded up to a power of two, mmax, nmax, l_cap, mode) in the
 * context, and leaves that variant's results in the outputs. *variant (host)
 * receives the choice. Later idcur_id_col_batched calls of the same class use it. */
idcur_status idcur_id_col_batched_autotune(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax, int32_t nmax,
                                           const int32_t* m, const int32_t* n, const void* const* A,
                                           const int64_t* lda, const idcur_opts* opts, void* ws, size_t ws_bytes,
                                           int32_t* k_out, int32_t* const* J, void* const* T, const int64_t* ldt,
                                           int32_t* variant /* host out */);
/* Batched gradient of the reconstruction loss of fixed-rank column IDs, each
 * block's skeleton frozen: the adjoint of idcur_id_col_batched with opts->k > 0,
 * block by block the derivative that idcur_id_col_backward computes for one
 * matrix, in one persistent launch. For block b (m[b] x n[b] FP32, row-major at
 * A[b], ld lda[b]):
 *   Y_b = Omega(:l, :m_b) A_b,  l = opts->k + opts->p, Omega the l x mmax matrix
 *         the batched ID draws (from opts->seed, or opts->omega: l x mmax
 *         row-major FP32, ld mmax),
 *   T_b = argmin_X |Y_b(:,J1) X - Y_b(:,J2)|_F (Section 2.3 on the sketch of
 *         Section 5.1), J1 = J_b[0..k_b-1], J2 = the rest,
 *   L_b = |A_b(:,J2) - A_b(:,J1) T_b|_F^2,
 *   dA_b = scale * dL_b / dA_b with J_b and Omega held fixed (written to dA[b],
 *          m_b x n_b row-major, ld ldd[b] >= n_b; overwritten).
 * k (device int32[nblk]) holds each block's rank k_b, 0 <= k_b <= opts->k (the
 * forward call's k_out); J (pointers to int32[n_b], permutations) and T
 * (pointers to FP32 k_b x (n_b - k_b), ld ldt[b]) as idcur_id_col_batched writes
 * them. m, n, A, lda, mmax, nmax as there. Limits: n_b <= nmax <= 512,
 * m_b <= mmax, opts->k + opts->p <= 64, p >= 1, q = 0, NATIVE precision, dtype
 * IDCUR_F32, lda[b] >= n_b, ldt[b] >= n_b - k_b. The m x n products run on the
 * FP32 matrix cores (FP32 sums); Y1^T Y1, its Cholesky factor and inverse are
 * FP64. A block outside the limits,
 * or a J_b that is not a permutation of 0..n_b-1, is reported as IDCUR_EINVAL by
 * idcur_sync_status (that block's dA_b is then left unwritten or undefined); a
 * singular Y1^T Y1 as IDCUR_ENONFINITE. The call only enqueues kernels on the
 * context's stream (no allocation, no host synchronisation, no memset node).
 * Workspace from idcur_id_col_batched_backward_workspace_bytes. */
idcur_status idcur_id_col_batched_backward_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int32_t nblk,
                                                           int32_t mmax, int32_t nmax, const idcur_opts* opts,
                                                           size_t* bytes /* host out */);
idcur_status idcur_id_col_batched_backward(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax, int32_t nmax,
                                           const int32_t* m, const int32_t* n, const void* const* A,
                                           const int64_t* lda, const idcur_opts* opts, const int32_t* k,
                                           const int32_t* const* J, const void* const* T, const int64_t* ldt,
                                           double scale, void* const* dA, const int64_t* ldd, void* ws,
                                           size_t ws_bytes);
/* Force a launch variant (0 .. 7) for every later batched call on this context;
 * -1 returns to the tuned or default choice. */
idcur_status idcur_id_col_batched_set_variant(idcur_ctx* ctx, int32_t variant);

/* The Gaussian sketch matrix alone (Section 5.1: i.i.d. N(0,1) entries): writes
 * Omega(r, i), r < rows, i < cols, to out + r*ldo + i. Entry (r, i) is defined by
 * the Philox4x32-10 counter (f/4 mod 2^32, f/4 div 2^32, stream, 0), f = r*cols + i,
 * key (seed mod 2^32, seed div 2^32), and a Box-Muller transform of its four
 * words (u1 = (x+1)/2^32, u2 = x'/2^32). This is the matrix the ID calls draw
 * when opts->omega is NULL (stream 0). */
idcur_status idcur_gaussian(idcur_ctx* ctx, int32_t dtype, int64_t rows, int64_t cols, uint64_t seed,
                            uint64_t stream, void* out, int64_t ldo);

#ifdef __cplusplus
}
#endif

#endif /* IDCUR_H */
