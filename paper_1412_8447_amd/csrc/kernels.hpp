// Launch interfaces of the HIP kernels behind libidcur (host-callable).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>

namespace idcur {

// dtype codes match idcur_dtype: 0 = double, 1 = float.

// ---------------------------------------------------------------------------
// Column-pivoted QR (cpqr.hip)
// ---------------------------------------------------------------------------
struct CpqrArgs {
  const void* Y;          // element (i, c) at Y[i*rs + c*cs]
  int64_t rs, cs;
  int l_host;             // rows (upper bound when l_dev is set)
  const int* l_dev;       // optional device row count
  int n;                  // columns
  int kmax_host;          // step cap (upper bound when kmax_dev is set)
  const int* kmax_dev;    // optional device step cap
  double tol;             // > 0: tolerance mode (relative Frobenius)
  double rank_tol;        // relative pivot-norm threshold for exact rank deficiency
  int norms_exact;        // 1: exact norms every step; 0: downdate + recompute
  void* S;                // kmax_host x n (dtype), row r at S + r*ldS, by original column
  int64_t ldS;
  int* J;                 // n
  int* k_out;             // device scalar
  int* status;            // device status word
  void* gslab;            // global slab (n * lpad) when the slab does not fit LDS
  void* rec;              // exchange records
  void* cvals;            // exchanged candidate columns
  int* fin;               // final-exchange flags (G * 16 ints, zeroed)
  int lpad;               // set by cpqr_launch
  int cols_per_wg;        // set by cpqr_launch
  int lanes_per_col;      // set by cpqr_launch
  int nb;                 // blocked kernel: panel width (set by cpqr_launch)
  int rpw;                // blocked kernel, tall form: rows per workgroup
  int vch;                // blocked kernel, tall form: rows of v staged in LDS
};

struct CpqrPlan {
  int G;
  int cols_per_wg;
  int lpad;
  int lanes_per_col;
  int reg_cfg;        // >= 0: register-slab kernel configuration; -1: blocked or slab kernel
  int res_cfg;        // >= 0: on-chip-slab kernel configuration (registers and LDS); -1: not used
  int blk;            // blocked kernel: 1 short form, 2 tall form; 0: not used
  int nb, rpw, vch;   // blocked kernel geometry
  bool in_lds;
  size_t lds_bytes;
  size_t rec_bytes, cvals_bytes, fin_bytes, gslab_bytes;
};

CpqrPlan cpqr_plan(int dtype_size, int l, int n, int kmax, int num_cus);
hipError_t cpqr_launch(int dtype, const CpqrPlan& p, CpqrArgs a, hipStream_t stream);
// blocked kernel (cpqr_blk.hip): fills p and returns its form (1 short, 2 tall)
// or 0 when the shape does not fit; force 1 / 2 restricts it to one form
int cpqr_blk_plan(CpqrPlan& p, int esz, int l, int n, int kmax, int num_cus, int force);
hipError_t cpqr_blk_launch(int dtype, const CpqrPlan& p, CpqrArgs a, hipStream_t stream);
// register-slab variant (cpqr_reg.hip): configuration index or -1 when the
// shape does not fit; sets the grid size and the columns per workgroup
int cpqr_reg_pick(int dtype_size, int l, int n, int num_cus, int* G, int* cols_per_wg);
size_t cpqr_reg_lds_bytes(int cfg, int kmax_host, int cols_per_wg, int dtype_size);
size_t cpqr_reg_rec_bytes(int G);
size_t cpqr_reg_cvals_bytes(int cfg, int G, int dtype_size);
hipError_t cpqr_reg_launch(int dtype, int cfg, int G, CpqrArgs a, size_t lds_bytes, hipStream_t stream);
// on-chip-slab variant (cpqr_res.hip, FP32): configuration index or -1
int cpqr_res_pick(int dtype_size, int l, int n, int kmax_host, int num_cus, int* G, int* cols_per_wg);
bool cpqr_res_forced();
size_t cpqr_res_lds_bytes(int cfg, int kmax_host, int cols_per_wg);
size_t cpqr_res_cvals_bytes(int cfg, int G);
hipError_t cpqr_res_launch(int cfg, int G, CpqrArgs a, size_t lds_bytes, hipStream_t stream);

// ---------------------------------------------------------------------------
// MFMA GEMM (gemm.hip): C (M x N) = A (M x K) * B (K x N)
//   A(i, k) = A[i*sam + k*sak]   with either sak == 1 (K contiguous) or sam == 1
//   B(k, j) = B[k*sbk + j*sbn]   with either sbn == 1 (N contiguous) or sbk == 1
//   C(i, j) = C[i*ldc + j]
// in: 0 double, 1 float.  acc: 0 double (f64 MFMA), 1 float (f32 MFMA).
// Split-K partial sums go to `part` (splitk * M * N of acc type) and are
// reduced in a fixed order by a second kernel.
// ---------------------------------------------------------------------------
struct GemmDesc {
  int64_t M, N, K;
  const void* A; int64_t sam, sak;
  const void* B; int64_t sbk, sbn;
  void* C; int64_t ldc;
  int in_type;      // of A and B (unless a_type / b_type are set)
  int a_type = -1;  // overrides in_type for A when >= 0
  int b_type = -1;  // overrides in_type for B when >= 0
  int acc_type;
  int out_type;     // of C
  int splitk;       // >= 1
  double alpha;     // C = alpha * A B (+ beta C when beta != 0)
  double beta;
  const int* m_dev; // optional device bound on M (rows >= *m_dev are skipped)
  const int* n_dev; // optional device bound on N
  const int* k_dev; // optional device bound on K
  bool b_rows_padded = false;   // every row of B is allocated up to round_up(N, 4)
  // C = A A^T-like square result of which only the lower triangle is read: tiles
  // wholly above the diagonal are skipped and that part of C is left unspecified
  bool lower = false;
};
size_t gemm_part_bytes(const GemmDesc& d);
int gemm_pick_splitk(int64_t M, int64_t N, int64_t K, int num_cus, bool acc64, bool lower = false);
// Split count for this descriptor (the FP32 thin kernel has its own choice).
int gemm_pick_splitk_desc(const GemmDesc& d, int num_cus);
// FP32 thin-output kernel (gemm_thin.hip), used by gemm_launch when eligible.
bool thin_f32_eligible(const GemmDesc& d);
int thin_f32_pick_splitk(int64_t M, int64_t N, int64_t K, int num_cus);
hipError_t thin_f32_launch(const GemmDesc& d, int splitk, void* part, hipStream_t stream);
// ev0/ev1 (optional) bracket the GEMM kernel itself, not the split-K reduction.
hipError_t gemm_launch(const GemmDesc& d, void* part, hipStream_t stream, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);

// Residual norm: out = sum_{i<M, j<N} (X(i,j) - (C W)(i,j))^2 with C (M x K,
// row-major ldc, type c_type), W (K x N, double, row-major ldw), X (M x N, x_type).
// FP64 matrix-core products; `part` holds one partial per 64 x 256 tile.
size_t gemm_resid_part_bytes(int64_t M, int64_t N);
hipError_t gemm_resid_launch(int x_type, int64_t M, int64_t N, int64_t K, const void* C, int64_t ldc, int c_type,
                             const double* W, int64_t ldw, const void* X, int64_t ldx, const int* k_dev,
                             double* part, double* out, hipStream_t stream);

// ---------------------------------------------------------------------------
// 16-bit MFMA GEMM (gemm16.hip): C (M x N, FP32, row-major ldc) = A (M x K) * B
// (K x N) with A FP32 in memory (A(i, k) = A[i*sam + k*sak], sak == 1 or
// sam == 1) rounded to BF16 / FP16 after multiplication by scale[0], and B
// packed as 16-bit B^T: B(k, j) = B[j*ldb + k]. FP32 accumulation; the result is
// multiplied by scale[1] (scale NULL: no scaling). Split-K partials (splitk * M *
// N floats) are summed in split order in FP64.
// ---------------------------------------------------------------------------
struct Gemm16Desc {
  int64_t M, N, K;
  const float* A; int64_t sam, sak;
  const void* B; int64_t ldb;
  float* C; int64_t ldc;
  int fp16;             // 0: BF16, 1: FP16
  const float* scale;   // device {s, 1/s} or NULL
  int splitk;
  int b_chunked;        // B packed by pack16c_launch (required exactly when gemm16_wide holds)
};
// Whether gemm16_launch runs the wide kernel (256 < N <= 640 output columns,
// aligned operands) for this shape and A layout; its B is then packed
// chunk-major by pack16c_launch with gemm16_wide_npad(N) columns and
// gemm16_wide_kchunks(K) chunks of 8 k.
bool gemm16_wide(int64_t M, int64_t N, int64_t K, const float* A, int64_t sam, int64_t sak);
int64_t gemm16_wide_npad(int64_t N);
int64_t gemm16_wide_kchunks(int64_t K);
// Chunk-major 16-bit packing: the 16-byte word (c, j) = round16(in(j, 8c .. 8c + 7))
// at out[16 (c npad + j)] bytes, in(j, k) = in[j*sj + k*sk], zero outside
// rows x cols; npad columns, kchunks chunks.
hipError_t pack16c_launch(int fp16, int64_t rows, int64_t cols, const float* in, int64_t sj, int64_t sk, int64_t npad,
                          int64_t kchunks, void* out, hipStream_t stream);
int gemm16_pick_splitk(int64_t M, int64_t N, int64_t K, int num_cus);
size_t gemm16_part_bytes(const Gemm16Desc& d);
hipError_t gemm16_launch(const Gemm16Desc& d, void* part, hipStream_t stream, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// out(j, k) = round16(in(j, k)) (round to nearest even), in(j, k) = in[j*sj + k*sk],
// for j < rows, k < cols, zero up to rows_pad x cols_pad; out row-major ldo.
hipError_t pack16_launch(int fp16, int64_t rows, int64_t cols, const float* in, int64_t sj, int64_t sk,
                         int64_t rows_pad, int64_t cols_pad, void* out, int64_t ldo, hipStream_t stream);
// FP16 prescale of a rows x cols FP32 matrix (ld lda): scale = {2^(15-e), 2^(e-15)}
// with max|A| in [2^(e-1), 2^e) ({1, 1} for a zero or non-finite maximum).
// part: kScaleParts floats.
constexpr int kScaleParts = 1024;
hipError_t fp16_scale_launch(int64_t rows, int64_t cols, const float* A, int64_t lda, float* part, float* scale,
                             hipStream_t stream);

// ---------------------------------------------------------------------------
// Batched adaptive-rank column ID (batched.hip): one persistent launch over
// nblk independent FP32 blocks. All per-block arrays are device arrays.
// ---------------------------------------------------------------------------
struct BatchedArgs {
  int nblk;
  const int* m; const int* n;
  const float* const* A; const int64_t* lda;
  int* const* J; float* const* T; const int64_t* ldt;
  int* k_out;
  const float* omt;        // Omega^T: batched_mpad(mmax) x batched_ldom(lcap), zero outside
  int mmax, nmax, lcap, p, kfix;
  double tol, rank_tol;
  int* order;              // nblk ints of scratch for the processing order (or NULL)
  int* queue;              // one int of scratch (zeroed by the launch)
  int* status;
};
int batched_ldom(int lcap);
int batched_mpad(int mmax);
int batched_max_width();
int batched_max_sketch();
size_t batched_lds_bytes(int lcap, int nmax);
int batched_num_variants();
hipError_t batched_launch(const BatchedArgs& a, int variant, int num_cus, hipStream_t stream);

// Subsampled randomized Hadamard sketch (srht.hip): Y^T (nc x l, ld ldo) of the
// mr x nc view X, X(i, c) = X[i*xr + c*xc] with xr == 1 or xc == 1;
// Y(r, c) = l^(-1/2) sum_i (-1)^popcount(rows[r] & i) s_i X(i, c), s_i = -1 where
// signs[i] < 0, else +1. Out-of-range rows flag ST_BADINDEX (row 0 is used).
constexpr int kSrhtMaxRows = 512;
struct SrhtDesc {
  const void* X; int64_t xr, xc;
  int64_t mr, nc;
  const int8_t* signs;
  const int* rows; int l;
  void* Yt; int64_t ldo;
  int splits;
  int* status;
};
int srht_pick_splits(int64_t mr, int64_t nc, int num_cus);
size_t srht_part_bytes(const SrhtDesc& d, int esize);
hipError_t srht_launch(int dtype, const SrhtDesc& d, void* part, hipStream_t stream);

// Batched gradient of the column-ID reconstruction loss (batched_bwd.hip): one
// persistent launch, one workgroup per block, each workgroup with a slot of
// batched_bwd_slot_floats floats of scratch (slot = grid slots).
struct BatchedBwdArgs {
  int nblk;
  const int* m; const int* n; const int* k;
  const float* const* A; const int64_t* lda;
  const int* const* J; const float* const* T; const int64_t* ldt;
  float* const* dA; const int64_t* ldd;
  const float* omt; int ldom;   // Omega^T: round_up(mmax, 16) x ldom, zero past column l
  int mmax, nmax, l, kcap;
  double scale;
  float* slot;                  // grid * batched_bwd_slot_floats(kcap, l, nmax) floats
  int* queue;                   // one int of scratch (zeroed by the launch)
  int* status;
};
int batched_bwd_max_width();
int batched_bwd_max_sketch();
int64_t batched_bwd_slot_floats(int kcap, int l, int nmax);
int batched_bwd_grid(int nblk, int num_cus);
hipError_t batched_bwd_launch(const BatchedBwdArgs& a, int grid, hipStream_t stream);

// ---------------------------------------------------------------------------
// Cholesky factor and triangular inverse (chol.hip), FP64, c <= 256, one workgroup
// (larger c: the blocked driver in host.cpp).
//   mode 0: G = L L^T (G(i,j) = G[i*gr + j*gc], optional diagonal shift
//           shift_rel * max diag) -> L (row-major, zeros above) and X = L^{-1}
//   mode 1: G is a lower-triangular factor (strided view) -> X = G^{-1}
// A non-positive pivot is clamped and reported through `status`.
// ---------------------------------------------------------------------------
size_t chol_inv_lds_bytes(int c_host);
// keep_l = 0: mode 0 leaves L as the working matrix only (the factor is not
// stored; callers that need just the inverse save the stores).
hipError_t chol_inv_launch(int mode, const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, double* L,
                           int64_t ldl, double* X, int64_t ldx, double shift_rel, int* status, hipStream_t stream,
                           int keep_l = 1);
// Mode 1 on the diagonal blocks of order bsz (at most 256, the kernel's limit) of
// the lower factor F (c x c, row-major ld ldf), one workgroup each, at once:
// X's diagonal block p = the inverse of F's.
hipError_t chol_inv_diag_launch(const double* F, int64_t ldf, int c, int bsz, double* X, int64_t ldx, int* status,
                                hipStream_t stream);

// S11 = S(0:c, J(0:c)) into a dense c x c double matrix (row-major, ld c_host).
hipError_t gather_s11_launch(int dtype, const void* S, int64_t ldS, const int* J, int c_host,
                             const int* c_dev, double* out, hipStream_t stream);
// S12 = S(0:c, J(c:n)) into a dense c x (n - c) double matrix (ld ldo) with c read
// on the device; also writes n - c to *ncols_out (device int).
hipError_t gather_s12_launch(int dtype, const void* S, int64_t ldS, const int* J, int64_t n, int c_host,
                             const int* c_dev, double* out, int64_t ldo, int* ncols_out, hipStream_t stream);

// ---------------------------------------------------------------------------
// Miscellaneous (misc.hip)
// ---------------------------------------------------------------------------
// Gaussian matrix from Philox4x32-10: element (r, i) of a rows x cols matrix
// written to out[r*sor + i*soc].
hipError_t gaussian_launch(int dtype, int64_t rows, int64_t cols, uint64_t seed, uint64_t stream_id,
                           void* out, int64_t sor, int64_t soc, hipStream_t stream);
// out(r, c) = in(r, c) for an r x c matrix with strides (transpose when swapped).
hipError_t copy2d_launch(int dtype, int64_t rows, int64_t cols, const void* in, int64_t sir, int64_t sic,
                         void* out, int64_t sor, int64_t soc, hipStream_t stream);
// out(j, i) = (float) in(i, j) (in: rows x cols, ld ldi; out: cols x ldo with
// ldo >= rows, columns [rows, ldo) zeroed).
hipError_t f64_to_f32_t_launch(int64_t rows, int64_t cols, const double* in, int64_t ldi, float* out, int64_t ldo,
                               hipStream_t stream);
// Gather columns: out(i, s) = A(i, idx[s]) for s < k (k = *k_dev if set), row-major out.
hipError_t gather_cols_launch(int dtype, int64_t m, const void* A, int64_t lda, const int* idx, int k_host,
                              const int* k_dev, void* out, int64_t ldo, int out_type, hipStream_t stream);
// inv[idx[s]] = s: the inverse of a permutation of 0..n-1 (out-of-range
// entries flag ST_BADINDEX).
hipError_t invert_perm_launch(const int* idx, int64_t n, int* inv, int* status, hipStream_t stream);
// out(i, c) = alpha * in(i, p[c]) (+= when accumulate) for c < ncols; in has nin
// columns (p[c] outside [0, nin) flags ST_BADINDEX and reads column 0).
hipError_t gather_cols_scaled_launch(int dtype, int64_t m, const void* in, int64_t ldi, int64_t nin, const int* p,
                                     int64_t ncols, double alpha, int accumulate, void* out, int64_t ldo, int* status,
                                     hipStream_t stream);
// Gather rows: out(s, j) = A(idx[s], j) for s < k.
hipError_t gather_rows_launch(int dtype, int64_t n, const void* A, int64_t lda, const int* idx, int k_host,
                              const int* k_dev, void* out, int64_t ldo, int out_type, hipStream_t stream);
// Fill bytes with zero (a kernel, so it can live inside a captured graph).
hipError_t zero_launch(void* p, size_t bytes, hipStream_t stream);
// V = V*^T (n x kcap, double, row-major ldv) from (J, T): row J[s] is e_s for
// s < k, row J[k+t] is T(:, t)^T (Section 2.3, eq. (column_approx_id2)).
hipError_t build_v_launch(int dtype, const void* T, int64_t ldt, const int* J, int64_t n, int kcap, const int* k_dev,
                          double* V, int64_t ldv, hipStream_t stream);
// out(a, b) += Q(a, J[b]) for a < ka, b < kb (double), Q row-major ldq.
// W = V* (kcap x n, double, row-major ldw): column J[s] is e_s (s < k), column
// J[k+t] is T(:, t); rows >= k are zero.
hipError_t build_vstar_launch(int dtype, const void* T, int64_t ldt, const int* J, int64_t n, int kcap,
                              const int* k_dev, double* W, int64_t ldw, hipStream_t stream);
// out = sum of squares of the m x n matrix A (FP64 accumulation; part: 1024 doubles).
hipError_t sumsq_launch(int dtype, int64_t m, int64_t n, const void* A, int64_t lda, double* part, double* out,
                        hipStream_t stream);
// P (c_host x c_host, ld ldp) = G's active c x c block (c = min(*c_dev, c_host),
// G(i, j) = G[i*gr + j*gc]) padded with the identity; lower_only zeroes the upper
// triangle; *shift (device, optional) is added to the active diagonal.
hipError_t pad_square_launch(const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, int lower_only,
                             const double* shift, double* P, int64_t ldp, hipStream_t stream);
// *out = rel * max_i G(i, i) over the active diagonal.
hipError_t diag_shift_launch(const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, double rel,
                             double* out, hipStream_t stream);
hipError_t zero2d_launch(double* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t stream);
// Sketch of a sparse m x n matrix in compressed sparse column form:
// Y^T (n x l, row-major, ld ldo; columns l..ldo-1 zero) with
// Y^T(j, :) = sum over the entries p of column j (colptr[j] <= p < colptr[j+1])
// of vals[p] Omega(:, rowidx[p])^T, Omega^T given m x ldom row-major. splits > 1
// (a multiple of 4) takes spmm_part_bytes of partial rows in `part`. Column
// pointers outside [0, nnz] or decreasing, and row indices outside [0, m),
// set ST_BADINDEX (the offending entries are skipped).
struct SpmmDesc {
  int64_t m, n, nnz;
  const int64_t* colptr;
  const int* rowidx;
  const void* vals;
  const void* Omt; int64_t ldom;
  int l;
  void* Yt; int64_t ldo;
  int splits;
  int* status;
};
int spmm_pick_splits(int64_t n, int64_t nnz, int num_cus);
// C (m x kcap, row-major ldc, zero on entry) = the columns J[0:k] of a sparse
// matrix in compressed sparse column form, k = min(*k_dev, kcap); repeated rows
// add up; bad indices set ST_BADINDEX.
hipError_t csc_gather_cols_launch(int dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                                  const int* rowidx, const void* vals, const int* J, int kcap, const int* k_dev,
                                  void* C, int64_t ldc, int* status, hipStream_t stream);
// R (kcap x n, row-major ldr, zero on entry) = the rows I[0:k] of the same
// matrix; slot is an int[m] scratch array.
hipError_t csc_gather_rows_launch(int dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                                  const int* rowidx, const void* vals, const int* I, int kcap, const int* k_dev,
                                  int* slot, void* R, int64_t ldr, hipStream_t stream);
size_t spmm_part_bytes(const SpmmDesc& d, int esize);
hipError_t spmm_csc_launch(int dtype, const SpmmDesc& d, void* part, hipStream_t stream);
// Y += (*s) X, rows x cols row-major FP64, the weight a device scalar.
// Truncated-SVD interpolation matrix (jacobi.hip): one-sided Jacobi SVD of the
// kcap x kcap FP64 matrix W (columns contiguous, rows / columns past *k_dev
// ignored) with the rotations accumulated in V; rot holds jacobi_max_sweeps()
// counters. tsvd_scale scales row i of P by 1 / s_i^2 (0 below thr max s).
int jacobi_max_sweeps();
hipError_t jacobi_svd_launch(double* W, double* V, int kcap, const int* k_dev, int* rot, hipStream_t stream);
hipError_t tsvd_scale_launch(const double* W, int kcap, const int* k_dev, double thr, double* P, int64_t ldp,
                             int64_t ncols, const int* ncols_dev, double* sv, hipStream_t stream);
hipError_t axpy_dev_launch(const double* s, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t rows,
                           int64_t cols, hipStream_t stream);
hipError_t add_gathered_launch(const double* Q, int64_t ldq, const int* J, int ka_host, const int* ka_dev,
                               int kb_host, const int* kb_dev, double* out, int64_t ldo, hipStream_t stream);

}  // namespace idcur
