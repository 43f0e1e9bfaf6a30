// Host side of libidcur: the C ABI declared in include/idcur.h.
//
// Every entry point runs the same planner twice: once without a workspace to
// size it (idcur_workspace_bytes), once to carve the caller's workspace and
// enqueue the kernels on the context's stream. Argument checks happen before
// anything is enqueued.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/idcur.h"
#include "args.hpp"
#include "common.hpp"
#include "kernels.hpp"

#include <map>
#include <vector>

struct idcur_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cus = 256;
  int* dstatus = nullptr;
  // device address of the file-scope scratch array on this context's device
  // (the workspace of idcur_id_col_noalloc), set once at context creation
  void* noalloc_scratch = nullptr;
  std::string err;
  // per-stage timers (HIP events on the stream), enabled by idcur_timing_enable
  bool timing = false;
  struct Mark {
    std::string stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  // batched launch variant per (size class of the batch): from the autotuner,
  // or forced with idcur_id_col_batched_set_variant (>= 0)
  std::map<std::vector<int64_t>, int> batched_tuned;
  int batched_forced = -1;
  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void recycle() {
    for (auto& m : marks) {
      pool.push_back(m.a);
      pool.push_back(m.b);
    }
    marks.clear();
  }
};

namespace idcur {
namespace {

constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
static_assert(kSrhtMaxRowsArg == kSrhtMaxRows, "argument check and kernel agree on the sketch rows");
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53

struct Fail {
  idcur_status code;
};

[[noreturn]] void fail(idcur_ctx* ctx, idcur_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  throw Fail{code};
}

void hipcheck(idcur_ctx* ctx, hipError_t e, const char* what) {
  if (e != hipSuccess) fail(ctx, IDCUR_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Workspace carving: dry runs only count bytes.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool dry = true;
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = dry ? nullptr : base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  }
};

size_t esz(int dtype) { return dtype == IDCUR_F32 ? 4 : 8; }

// A logical matrix X (rows x cols) viewed inside A: X(i, c) = A[i*xr + c*xc].
struct View {
  const void* A;
  int64_t rows, cols, xr, xc;
};

struct Ctx {
  idcur_ctx* c;
  hipStream_t s;
  bool dry;
  Arena* ar;
  void check(hipError_t e, const char* what) const {
    if (!dry) hipcheck(c, e, what);
  }
};

// Brackets the launches of one stage with a pair of events when timing is on.
struct Stage {
  const Ctx& x;
  hipEvent_t a = nullptr, b = nullptr;
  const char* name;
  Stage(const Ctx& xx, const char* nm) : x(xx), name(nm) {
    if (x.dry || !x.c->timing) return;
    a = x.c->get_event();
    b = x.c->get_event();
    if (a && b) (void)hipEventRecord(a, x.s);
  }
  ~Stage() {
    if (!a || !b) return;
    (void)hipEventRecord(b, x.s);
    x.c->marks.push_back({name, a, b});
  }
};

// ---------------------------------------------------------------------------
// GEMM helper: C = A * B in the descriptor's layout, with split-K scratch.
// ---------------------------------------------------------------------------
void gemm(const Ctx& x, GemmDesc d, const char* stage = nullptr) {
  d.splitk = gemm_pick_splitk_desc(d, x.c->num_cus);
  void* part = x.ar->take(gemm_part_bytes(d));
  if (x.dry) return;
  hipEvent_t a = nullptr, b = nullptr;
  if (stage && x.c->timing) {
    a = x.c->get_event();
    b = x.c->get_event();
  }
  x.check(gemm_launch(d, part, x.s, a, b), "gemm");
  if (a && b) x.c->marks.push_back({stage, a, b});
}

// Cholesky factor and triangular inverse of any order. Up to kCholDirect the
// one-workgroup kernel does it all; above, a right-looking blocked form runs the
// same kernel on diagonal blocks of at most kCholDirect and FP64 matrix-core
// products for the rest:
//   mode 0:  L_pp X_pp = chol/inverse of P_pp;  L_rp = P_rp X_pp^T;
//            P_rr -= L_rp L_rp^T  (P = G, shifted, updated in place)
//   mode 1:  X_pp = inverse of the given factor's diagonal block;
// then, block row by block row, X(r, 0:o) = -X_rr (F(r, 0:o) X(0:o, 0:o)) with F
// the lower factor. A device order c_dev is handled by padding G with the
// identity, whose factor and inverse are the identity. Only the lower triangle
// of G is read (its Gram products compute no more).
constexpr int kCholDirect = 256;

void chol_inv(const Ctx& x, int mode, const double* G, int64_t gr, int64_t gc, int c, const int* c_dev, double* L,
              int64_t ldl, double* X, int64_t ldx, double shift_rel, const char* what, bool keep_l = true) {
  if (c <= kCholDirect) {
    if (!x.dry) x.check(chol_inv_launch(mode, G, gr, gc, c, c_dev, L, ldl, X, ldx, shift_rel, x.c->dstatus, x.s, keep_l), what);
    return;
  }
  const int nb = (int)ceil_div(c, kCholDirect);
  const int b = (int)std::min<int64_t>(kCholDirect, round_up(ceil_div(c, nb), 32));
  double* P = static_cast<double*>(x.ar->take((size_t)c * c * 8));
  double* W = static_cast<double*>(x.ar->take((size_t)c * c * 8));
  double* sh = (mode == 0 && shift_rel > 0.0) ? static_cast<double*>(x.ar->take(8)) : nullptr;
  if (!x.dry) {
    if (sh) x.check(diag_shift_launch(G, gr, gc, c, c_dev, shift_rel, sh, x.s), what);
    x.check(pad_square_launch(G, gr, gc, c, c_dev, 1, sh, P, c, x.s), what);
    if (mode == 0) x.check(zero2d_launch(L, c, c, ldl, x.s), what);
    x.check(zero2d_launch(X, c, c, ldx, x.s), what);
  }
  auto mm = [&](int64_t M, int64_t N, int64_t K, const double* Am, int64_t sam, int64_t sak, const double* Bm,
                int64_t sbk, int64_t sbn, double* Cm, int64_t ldc, double alpha, double beta) {
    GemmDesc g{};
    g.M = M; g.N = N; g.K = K;
    g.A = Am; g.sam = sam; g.sak = sak;
    g.B = Bm; g.sbk = sbk; g.sbn = sbn;
    g.C = Cm; g.ldc = ldc;
    g.in_type = 0; g.acc_type = 0; g.out_type = 0;
    g.alpha = alpha; g.beta = beta;
    gemm(x, g);
  };
  // mode 1: the diagonal blocks are independent, one workgroup each in one launch
  if (mode == 1 && !x.dry) x.check(chol_inv_diag_launch(P, c, c, b, X, ldx, x.c->dstatus, x.s), what);
  for (int p = 0; p < nb; ++p) {
    const int o = p * b, sp = std::min(b, c - o);
    if (mode == 0 && !x.dry)
      x.check(chol_inv_launch(mode, P + (int64_t)o * c + o, c, 1, sp, nullptr, L + (int64_t)o * ldl + o, ldl,
                              X + (int64_t)o * ldx + o, ldx, 0.0, x.c->dstatus, x.s),
              what);
    const int r = c - o - sp;
    if (mode == 0 && r > 0) {
      double* Lrp = L + (int64_t)(o + sp) * ldl + o;
      mm(r, sp, sp, P + (int64_t)(o + sp) * c + o, c, 1, X + (int64_t)o * ldx + o, 1, ldx, Lrp, ldl, 1.0, 0.0);
      mm(r, r, sp, Lrp, ldl, 1, Lrp, 1, ldl, P + (int64_t)(o + sp) * c + (o + sp), c, -1.0, 1.0);
    }
  }
  const double* F = mode == 0 ? L : P;
  const int64_t ldf = mode == 0 ? ldl : c;
  for (int p = 1; p < nb; ++p) {
    const int o = p * b, sp = std::min(b, c - o);
    mm(sp, o, o, F + (int64_t)o * ldf, ldf, 1, X, ldx, 1, W, o, 1.0, 0.0);
    mm(sp, o, sp, X + (int64_t)o * ldx + o, ldx, 1, W, o, 1, X + (int64_t)o * ldx, ldx, -1.0, 0.0);
  }
}

// Row-orthonormalise V (l x N), stored transposed as Vt (N x l, row-major),
// into Qt (same layout): Cholesky QR, G = V V^T + s I = L L^T, Q = L^{-1} V,
// with an FP64 Gram matrix, factor and inverse, and Q^T = V^T L^{-T} as one
// matrix-core product. The next power step only needs a well-conditioned basis
// of the row space (the pivoted QR is invariant to which basis), so one pass
// with a tiny shift s, which rules out breakdown, is enough.
// Q^T = orth(V^T): V^T and Q^T are N x l with leading dimension ld.
// With q32 (FP32 data whose basis is next rounded to 16 bits for a matrix-core
// product) the last product runs on the FP32 matrix cores with L^{-T} rounded to
// FP32: its error, a few FP32 units per entry, lies far below the 16-bit
// rounding that follows; Q stays in the row space of V either way.
void orth_rows(const Ctx& x, int dtype, const void* Vt, void* Qt, int64_t N, int l, int64_t ld, bool q32 = false) {
  double* G = static_cast<double*>(x.ar->take((size_t)l * l * 8));
  double* L = static_cast<double*>(x.ar->take((size_t)l * l * 8));
  double* Li = static_cast<double*>(x.ar->take((size_t)l * l * 8));
  GemmDesc g{};
  g.M = l; g.N = l; g.K = N;
  g.A = Vt; g.sam = 1; g.sak = ld;
  g.B = Vt; g.sbk = ld; g.sbn = 1;
  g.C = G; g.ldc = l;
  g.in_type = dtype; g.acc_type = 0; g.out_type = 0;
  g.alpha = 1.0; g.beta = 0.0;
  g.lower = true;   // the factorisation reads the lower triangle only
  gemm(x, g);
  chol_inv(x, 0, G, l, 1, l, nullptr, L, l, Li, l, 1e-14, "chol", false);   // only L^{-1} is used
  GemmDesc q{};   // Q^T = V^T L^{-T}
  q.M = N; q.N = l; q.K = l;
  q.A = Vt; q.sam = ld; q.sak = 1;
  q.B = Li; q.sbk = 1; q.sbn = l;
  q.C = Qt; q.ldc = ld;
  q.a_type = dtype; q.b_type = 0; q.acc_type = 0; q.out_type = dtype;
  q.alpha = 1.0; q.beta = 0.0;
  if (q32 && dtype == IDCUR_F32) {
    // B(kk, j) = L^{-1}(j, kk) as an l x ld FP32 row-major matrix
    float* Lt = static_cast<float*>(x.ar->take((size_t)l * ld * 4));
    if (!x.dry) x.check(f64_to_f32_t_launch(l, l, Li, l, Lt, ld, x.s), "L^{-T} to FP32");
    q.B = Lt; q.sbk = ld; q.sbn = 1;
    q.b_rows_padded = true;
    q.in_type = 1; q.b_type = 1; q.acc_type = 1;
  }
  gemm(x, q);
}

// T = S11^{-1} S12 for the rank-c pivoted QR held in S (rows by original column,
// ld ldS): S11 gathered and inverted (as the lower factor S11^T), S12 gathered,
// T = (S11^{-T})^T S12 as an FP64 matrix-core product written in T's dtype.
void interp_matrix(const Ctx& x, int dtype, const void* S, int64_t ldS, const int* J, int64_t n, int kcap,
                   const int* k_dev, void* T, int64_t ldt, double t_reg = 0.0, double t_svd = 0.0) {
  double* S11 = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* S11it = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* S12 = static_cast<double*>(x.ar->take((size_t)kcap * std::max<int64_t>(n - 1, 1) * 8));
  int* ncol = static_cast<int*>(x.ar->take(256));
  const int64_t ldo = std::max<int64_t>(n - 1, 1);
  if (!x.dry) {
    x.check(gather_s11_launch(dtype, S, ldS, J, kcap, k_dev, S11, x.s), "gather S11");
    x.check(gather_s12_launch(dtype, S, ldS, J, n, kcap, k_dev, S12, ldo, ncol, x.s), "gather S12");
    // view S11^T as lower: element (i, j) = S11[j][i]
  }
  auto mm = [&](int64_t M, int64_t N, const double* Am, int64_t sam, int64_t sak, const double* Bm, int64_t sbk,
                int64_t sbn, void* Cm, int64_t ldc, int ct, const int* nd, double beta = 0.0) {
    GemmDesc g{};
    g.M = M; g.N = N; g.K = kcap;
    g.A = Am; g.sam = sam; g.sak = sak;
    g.B = Bm; g.sbk = sbk; g.sbn = sbn;
    g.C = Cm; g.ldc = ldc;
    g.in_type = 0; g.acc_type = 0; g.out_type = ct;
    g.alpha = 1.0; g.beta = beta;
    g.m_dev = k_dev; g.k_dev = k_dev; g.n_dev = nd;
    gemm(x, g);
  };
  if (t_reg > 0.0) {
    // Tikhonov-stabilized T (Section 4.1, eq. (lsqr_for_T) with a regularization
    // term): T = argmin |S11 U - S12|^2 + lam^2 |U|^2, lam = t_reg times the
    // largest column norm of S11, the least-squares solution of M U = [S12; 0]
    // with M = [S11; lam I]. M = Q R by Cholesky QR twice (FP64), which keeps
    // the error at about u cond(M) <= u / t_reg instead of the normal
    // equations' u / t_reg^2:
    //   L1 L1^T = M^T M = S11^T S11 + lam^2 I,  Q1 = M L1^{-T}
    //   L2 L2^T = Q1^T Q1 = Qt^T Qt + lam^2 L1^{-1} L1^{-T},  Qt = S11 L1^{-T}
    //   Q = Q1 L2^{-T}, R = L2^T L1^T, T = R^{-1} Q^T [S12; 0]
    //     = L1^{-T} L2^{-T} (Qt L2^{-T})^T S12.
    double* G = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* L = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* L1i = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* L2i = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* Qt = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* Q = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* P = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* lam2 = static_cast<double*>(x.ar->take(256));
    double* W = static_cast<double*>(x.ar->take((size_t)kcap * ldo * 8));
    double* Z = static_cast<double*>(x.ar->take((size_t)kcap * ldo * 8));
    // G = S11^T S11 (A(i, kk) = S11[kk][i]); lam^2 = t_reg^2 max diag(G)
    mm(kcap, kcap, S11, 1, kcap, S11, kcap, 1, G, kcap, 0, k_dev);
    if (!x.dry) x.check(diag_shift_launch(G, kcap, 1, kcap, k_dev, t_reg * t_reg, lam2, x.s), "lam^2");
    chol_inv(x, 0, G, kcap, 1, kcap, k_dev, L, kcap, L1i, kcap, t_reg * t_reg, "chol(S11^T S11 + lam^2 I)", false);
    // Qt = S11 L1^{-T} (B(kk, j) = L1i[j][kk]); G = Qt^T Qt + lam^2 L1^{-1} L1^{-T}
    mm(kcap, kcap, S11, kcap, 1, L1i, 1, kcap, Qt, kcap, 0, k_dev);
    mm(kcap, kcap, Qt, 1, kcap, Qt, kcap, 1, G, kcap, 0, k_dev);
    mm(kcap, kcap, L1i, kcap, 1, L1i, 1, kcap, P, kcap, 0, k_dev);
    if (!x.dry) x.check(axpy_dev_launch(lam2, P, kcap, G, kcap, kcap, kcap, x.s), "Q1^T Q1");
    chol_inv(x, 0, G, kcap, 1, kcap, k_dev, L, kcap, L2i, kcap, 0.0, "chol(Q1^T Q1)", false);
    // Q = Qt L2^{-T}; W = Q^T S12; Z = L2^{-T} W; T = L1^{-T} Z
    mm(kcap, kcap, Qt, kcap, 1, L2i, 1, kcap, Q, kcap, 0, k_dev);
    mm(kcap, n - 1, Q, 1, kcap, S12, ldo, 1, W, ldo, 0, ncol);
    mm(kcap, n - 1, L2i, 1, kcap, W, ldo, 1, Z, ldo, 0, ncol);
    mm(kcap, std::min<int64_t>(n - 1, ldt), L1i, 1, kcap, Z, ldo, 1, T, ldt, dtype, ncol);
    return;
  }
  if (t_svd > 0.0) {
    // Truncated-SVD T (Section 4.1, the stabilized pseudo-inverse of S11 in eq.
    // (lsqr_for_T)): one-sided Jacobi on the columns of S11 (contiguous rows of
    // the buffer), W V = U diag(s); P = W^T S12 with row i scaled by 1 / s_i^2
    // (0 where s_i < t_svd max s); T = V P.
    double* V = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* P = static_cast<double*>(x.ar->take((size_t)kcap * ldo * 8));
    double* sv = static_cast<double*>(x.ar->take((size_t)kcap * 8));
    int* rot = static_cast<int*>(x.ar->take((size_t)jacobi_max_sweeps() * 4 + 256));
    if (!x.dry) x.check(jacobi_svd_launch(S11, V, kcap, k_dev, rot, x.s), "Jacobi SVD of S11");
    // P = W^T S12 (A(i, kk) = W(kk, i) = S11[i][kk])
    mm(kcap, n - 1, S11, kcap, 1, S12, ldo, 1, P, ldo, 0, ncol);
    if (!x.dry) x.check(tsvd_scale_launch(S11, kcap, k_dev, t_svd, P, ldo, n - 1, ncol, sv, x.s), "1 / s^2");
    // T = V P (A(i, kk) = V(i, kk) = V[kk][i])
    mm(kcap, std::min<int64_t>(n - 1, ldt), V, 1, kcap, P, ldo, 1, T, ldt, dtype, ncol);
    return;
  }
  chol_inv(x, 1, S11, 1, kcap, kcap, k_dev, nullptr, 0, S11it, kcap, 0.0, "S11 inverse");
  // T = S11^{-1} S12, A(i, kk) = S11it[kk][i]
  mm(kcap, std::min<int64_t>(n - 1, ldt), S11it, 1, kcap, S12, ldo, 1, T, ldt, dtype, ncol);
}

// Exact rank deficiency (Section 2.3), relative to the largest initial column
// norm: 10 sqrt(l) u with a fixed rank (a safe margin over the rounding noise of
// an l-row column), sqrt(l) u in tolerance mode, where the Frobenius rule
// already stops at noise level and a coarser test would stop ahead of it (FP32
// pivots of a few 1e-6 at tol = 1e-6 are well resolved).
double default_rank_tol(int dtype, int64_t l, bool tolmode) {
  return (tolmode ? 1.0 : 10.0) * std::sqrt((double)std::max<int64_t>(l, 1)) * (dtype == IDCUR_F32 ? kU32 : kU64);
}

// The sketch of the view X (Section 5.1, eq. (Y=OmegaA)) with q orthonormalised
// power steps (Section 5.3): Y^T (nc x l, row-major, ld round_up(l, 4)) in the
// workspace, or X itself when no sketch is taken (p < 0 or k + p >= rows).
// With a 16-bit precision the GEMMs round A and the thin operand to BF16 or FP16
// (FP16: A prescaled by a power of two, undone on the FP32 result).
struct SketchOut {
  const void* Y;
  int64_t rs, cs;   // Y(i, c) at Y[i*rs + c*cs]
  int l;
  bool sketched;
};

SketchOut sketch(const Ctx& x, int dtype, const View& X, const idcur_opts& o, int kcap, bool allow_sketch) {
  SketchOut r{X.A, X.xr, X.xc, (int)X.rows, false};
  const int64_t mr = X.rows, nc = X.cols;
  if (!(allow_sketch && o.p >= 0 && (int64_t)kcap + o.p < mr)) return r;
  const int l = kcap + o.p;
  // the thin sketch matrices are row-major with their width l padded to a
  // multiple of 4 elements, so that every row starts 16-byte aligned and the
  // GEMMs read them with vector loads
  const int64_t ll = round_up(l, 4);
  if (o.sketch == IDCUR_SKETCH_SRHT) {
    // the subsampled randomized Hadamard sketch (Section 5.2's structured
    // sketch, real form): one pass over X, no power steps
    void* Yt = x.ar->take((size_t)nc * ll * esz(dtype));
    SrhtDesc d{};
    d.X = X.A; d.xr = X.xr; d.xc = X.xc; d.mr = mr; d.nc = nc;
    d.signs = static_cast<const int8_t*>(o.srht_signs);
    d.rows = o.srht_rows; d.l = l;
    d.Yt = Yt; d.ldo = ll;
    d.splits = srht_pick_splits(mr, nc, x.c->num_cus);
    d.status = x.c->dstatus;
    void* part = x.ar->take(srht_part_bytes(d, (int)esz(dtype)));
    if (!x.dry) {
      Stage st(x, "srht");
      x.check(srht_launch(dtype, d, part, x.s), "structured sketch");
    }
    r.Y = Yt; r.rs = 1; r.cs = ll; r.l = l; r.sketched = true;
    return r;
  }
  const bool lowp = o.prec == IDCUR_PREC_BF16 || o.prec == IDCUR_PREC_FP16;
  const int fp16 = o.prec == IDCUR_PREC_FP16;
  void* Omt = (lowp && o.omega) ? nullptr : x.ar->take((size_t)mr * ll * esz(dtype));   // Omega^T, mr x l
  void* Yt = x.ar->take((size_t)nc * ll * esz(dtype));    // Y^T,     nc x l
  void* Zt = o.q > 0 ? x.ar->take((size_t)mr * ll * esz(dtype)) : nullptr;
  void* Qyt = o.q > 0 ? x.ar->take((size_t)nc * ll * esz(dtype)) : nullptr;   // orth(Y)^T
  void* Qzt = o.q > 0 ? x.ar->take((size_t)mr * ll * esz(dtype)) : nullptr;   // orth(Z)^T
  // 16-bit thin operand, packed as B^T (l x K, k contiguous), or chunk-major
  // (8 k of all padded columns at a time) for the wide kernel; the FP16 scale
  const int64_t ldb16 = round_up(std::max(mr, nc), 8);
  const size_t b16_bytes =
      std::max((size_t)l * ldb16 * 2,
               (size_t)gemm16_wide_npad(l) * gemm16_wide_kchunks(std::max(mr, nc)) * 16);
  void* B16 = lowp ? x.ar->take(b16_bytes) : nullptr;
  float* scale = (lowp && fp16) ? static_cast<float*>(x.ar->take(2 * sizeof(float))) : nullptr;
  float* spart = (lowp && fp16) ? static_cast<float*>(x.ar->take(kScaleParts * sizeof(float))) : nullptr;

  // Cm = X' * B16^T with X' (M x K) = X or X^T as (sam, sak) say; B16 packed
  // from src (the K x l thin operand, element (k, j) at src[j*sj + k*sk]) in the
  // layout of the kernel that gemm16_launch picks for this shape
  auto gemm_lp = [&](int64_t M, int64_t K, int64_t sam, int64_t sak, const void* src, int64_t sj, int64_t sk,
                     void* Cm) {
    const bool wide = gemm16_wide(M, l, K, static_cast<const float*>(X.A), sam, sak);
    if (!x.dry) {
      Stage st(x, "pack");
      const float* in = static_cast<const float*>(src);
      x.check(wide ? pack16c_launch(fp16, l, K, in, sj, sk, gemm16_wide_npad(l), gemm16_wide_kchunks(K), B16, x.s)
                   : pack16_launch(fp16, l, K, in, sj, sk, l, round_up(K, 8), B16, ldb16, x.s),
              "pack16");
    }
    Gemm16Desc g{};
    g.M = M; g.N = l; g.K = K;
    g.A = static_cast<const float*>(X.A); g.sam = sam; g.sak = sak;
    g.B = B16; g.ldb = ldb16;
    g.b_chunked = wide ? 1 : 0;
    g.C = static_cast<float*>(Cm); g.ldc = ll;
    g.fp16 = fp16; g.scale = scale;
    g.splitk = gemm16_pick_splitk(M, l, K, x.c->num_cus);
    void* part = x.ar->take(gemm16_part_bytes(g));
    if (x.dry) return;
    hipEvent_t a = nullptr, b = nullptr;
    if (x.c->timing) {
      a = x.c->get_event();
      b = x.c->get_event();
    }
    x.check(gemm16_launch(g, part, x.s, a, b), "gemm16");
    if (a && b) x.c->marks.push_back({"sketch_gemm", a, b});
  };
  auto mul_t = [&](const void* Bm) {   // Y^T = X^T * Bm   (Bm: mr x l, ld ll)
    if (lowp) {
      gemm_lp(nc, mr, X.xc, X.xr, Bm, 1, ll, Yt);
      return;
    }
    GemmDesc g{};
    g.M = nc; g.N = l; g.K = mr;
    g.A = X.A; g.sam = X.xc; g.sak = X.xr;
    g.B = Bm; g.sbk = ll; g.sbn = 1;
    g.C = Yt; g.ldc = ll;
    g.b_rows_padded = true;   // Bm is mr x ll
    g.in_type = dtype; g.acc_type = dtype == IDCUR_F32 ? 1 : 0; g.out_type = dtype;
    g.alpha = 1.0; g.beta = 0.0;
    gemm(x, g, "sketch_gemm");
  };
  {
    Stage st(x, "omega");
    if (!x.dry && fp16) {
      // power-of-two prescale from max |A| over the stored matrix
      const bool rowmaj = X.xc == 1;
      x.check(fp16_scale_launch(rowmaj ? X.rows : X.cols, rowmaj ? X.cols : X.rows, static_cast<const float*>(X.A),
                                rowmaj ? X.xr : X.xc, spart, scale, x.s),
              "fp16 scale");
    }
    if (!x.dry) {
      if (o.omega && lowp) {
        // packed with the first product below
      } else if (o.omega)
        x.check(copy2d_launch(dtype, l, mr, o.omega, mr, 1, Omt, 1, ll, x.s), "omega copy");
      else
        x.check(gaussian_launch(dtype, l, mr, o.seed, 0, Omt, 1, ll, x.s), "omega");
    }
  }
  if (o.omega && lowp)
    gemm_lp(nc, mr, X.xc, X.xr, o.omega, mr, 1, Yt);
  else
    mul_t(Omt);
  for (int it = 0; it < o.q; ++it) {
    {
      Stage st(x, "orth");
      orth_rows(x, dtype, Yt, Qyt, nc, l, ll, lowp);
    }
    if (lowp) {   // Z^T = X * orth(Y)^T
      gemm_lp(mr, nc, X.xr, X.xc, Qyt, 1, ll, Zt);
    } else {
      GemmDesc g{};
      g.M = mr; g.N = l; g.K = nc;
      g.A = X.A; g.sam = X.xr; g.sak = X.xc;
      g.B = Qyt; g.sbk = ll; g.sbn = 1;
      g.C = Zt; g.ldc = ll;
      g.b_rows_padded = true;   // Qyt is nc x ll
      g.in_type = dtype; g.acc_type = dtype == IDCUR_F32 ? 1 : 0; g.out_type = dtype;
      g.alpha = 1.0; g.beta = 0.0;
      gemm(x, g, "sketch_gemm");
    }
    {
      Stage st(x, "orth");
      orth_rows(x, dtype, Zt, Qzt, mr, l, ll, lowp);
    }
    mul_t(Qzt);
  }
  r.Y = Yt; r.rs = 1; r.cs = ll; r.l = l; r.sketched = true;
  return r;
}

// Column ID of the view X: J (cols), T (kcap x (cols-k), ldt), k_out (device).
// Returns the S buffer (kcap x cols, by original column) for later use.
struct ColId {
  void* S = nullptr;
  int kcap = 0;
};

ColId column_id(const Ctx& x, int dtype, const View& X, const idcur_opts& o, int* k_out, int* J, void* T,
                int64_t ldt, bool allow_sketch) {
  ColId r;
  const int64_t nc = X.cols;
  const int kcap = o.k > 0 ? o.k : o.kmax;
  r.kcap = kcap;
  const SketchOut sk = sketch(x, dtype, X, o, kcap, allow_sketch);
  const int l = sk.l;
  const void* Ymat = sk.Y;
  const int64_t yrs = sk.rs, ycs = sk.cs;

  // CPQR on Y (l x nc)
  const CpqrPlan pl = cpqr_plan((int)esz(dtype), l, (int)nc, kcap, x.c->num_cus);
  void* rec = x.ar->take(pl.rec_bytes + pl.fin_bytes);
  void* cvals = x.ar->take(pl.cvals_bytes);
  void* gslab = pl.gslab_bytes ? x.ar->take(pl.gslab_bytes) : nullptr;
  void* S = x.ar->take((size_t)std::max(kcap, 1) * nc * esz(dtype));
  r.S = S;
  if (!x.dry) {
    Stage st(x, "cpqr");
    x.check(zero_launch(rec, pl.rec_bytes + pl.fin_bytes, x.s), "zero");
    // column words carry only the publish index as their stamp: words left by an
    // earlier call in the same memory must not match, so they start at zero
    x.check(zero_launch(cvals, pl.cvals_bytes, x.s), "zero");
    CpqrArgs a{};
    a.Y = Ymat; a.rs = yrs; a.cs = ycs;
    a.l_host = l; a.l_dev = nullptr; a.n = (int)nc;
    a.kmax_host = kcap; a.kmax_dev = nullptr;
    a.tol = o.k > 0 ? 0.0 : o.tol;
    a.rank_tol = o.rank_tol > 0 ? o.rank_tol : default_rank_tol(dtype, l, o.k == 0);
    a.norms_exact = o.norms == IDCUR_NORMS_EXACT;
    a.S = S; a.ldS = nc; a.J = J; a.k_out = k_out; a.status = x.c->dstatus;
    a.gslab = gslab; a.rec = rec; a.cvals = cvals;
    a.fin = reinterpret_cast<int*>(static_cast<char*>(rec) + pl.rec_bytes);
    x.check(cpqr_launch(dtype, pl, a, x.s), "cpqr");
  }
  {
    Stage st(x, "trsm");
    interp_matrix(x, dtype, S, nc, J, nc, kcap, k_out, T, ldt, o.t_reg, o.t_svd);
  }
  return r;
}

// Row ID of C (m x kcap, row-major ld kcap) with rank k_dev: the full-rank ID of
// C^T, giving I (m) and, with want_tr, Tr (k x (m-k), ldtr); k_out_r receives
// its rank. The CUR needs only the row pivots (R = A(I(1:k), :) and U from the
// least-squares solve U R = V*), so it skips the interpolation matrix.
void row_id_of_c(const Ctx& x, int dtype, const void* C, int64_t ldc, int64_t m, int kcap, const int* k_dev, int* k_out_r, int* I,
                 bool want_tr, void* Tr, int64_t ldtr, double t_reg, double t_svd) {
  const CpqrPlan pl = cpqr_plan((int)esz(dtype), kcap, (int)m, kcap, x.c->num_cus);
  void* rec = x.ar->take(pl.rec_bytes + pl.fin_bytes);
  void* cvals = x.ar->take(pl.cvals_bytes);
  void* gslab = pl.gslab_bytes ? x.ar->take(pl.gslab_bytes) : nullptr;
  void* S = x.ar->take((size_t)std::max(kcap, 1) * m * esz(dtype));
  if (!x.dry) {
    Stage st(x, "row_id");
    x.check(zero_launch(rec, pl.rec_bytes + pl.fin_bytes, x.s), "zero");
    // column words carry only the publish index as their stamp: words left by an
    // earlier call in the same memory must not match, so they start at zero
    x.check(zero_launch(cvals, pl.cvals_bytes, x.s), "zero");
    CpqrArgs a{};
    a.Y = C; a.rs = 1; a.cs = ldc;
    a.l_host = kcap; a.l_dev = k_dev; a.n = (int)m;
    a.kmax_host = kcap; a.kmax_dev = k_dev;
    a.tol = 0.0;
    a.rank_tol = 0.0;   // a full-rank ID: stop only on an exactly zero pivot
    a.norms_exact = 0;
    a.S = S; a.ldS = m; a.J = I; a.k_out = k_out_r; a.status = x.c->dstatus;
    a.gslab = gslab; a.rec = rec; a.cvals = cvals;
    a.fin = reinterpret_cast<int*>(static_cast<char*>(rec) + pl.rec_bytes);
    Stage sk(x, "row_cpqr");   // the pivoted QR launch alone (inside the row_id stage)
    x.check(cpqr_launch(dtype, pl, a, x.s), "cpqr(row)");
  }
  if (!want_tr) return;
  Stage st(x, "row_id");
  interp_matrix(x, dtype, S, m, I, m, kcap, k_out_r, Tr, ldtr, t_reg, t_svd);
}

// U = argmin |U R - V*|_F through the QR of R^T (Cholesky QR twice, FP64):
// R^T = Q S_R with S_R = L2^T L1^T and Q^T = L2^{-1} Q1^T, so
// U^T = S_R^{-1} Q^T V = L1^{-T} L2^{-T} L2^{-1} (Q1^T V): Q itself is never
// formed; L2^{-1} is applied to the k x k product Q1^T V instead.
// Every step is a matrix-core product with the explicit triangular inverses.
// R: kr x n (row-major ldr), V* from (J, T); k = kout[0] columns, kr = kout[1].
// With `corr` (A, lda, m and C = A(:, J(1:k)), m x kcap ld kcap given) the right
// side is V* + C^+ E, E = A - C V* (the error-corrected system of Section 4.3,
// eq. (cur_ur_sys2)): with Gc = C^T C = Lc Lc^T,
//   (C^+ E)^T = (A^T C - V Gc) Gc^{-1} = (A^T C - V Gc) Lc^{-T} Lc^{-1},
// A^T C accumulated in FP64, so the difference keeps its digits when E is small.
void solve_u(const Ctx& x, int dtype, const void* R, int64_t ldr, int64_t n, int kcap, const int* kout, const int* J,
             const void* T, int64_t ldt, void* U, int64_t ldu, bool corr = false, const void* A = nullptr,
             int64_t lda = 0, int64_t m = 0, const void* C = nullptr, int64_t ldc = 0) {
  const int* k_dev = kout;
  const int* kr_dev = kout + 1;
  double* G = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* L1 = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* L1i = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* L2 = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* L2i = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* Q1t = static_cast<double*>(x.ar->take((size_t)kcap * n * 8));
  double* B1 = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* V = static_cast<double*>(x.ar->take((size_t)n * kcap * 8));
  double* Bls = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  double* Y1 = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
  auto prod = [&](int64_t M, int64_t N, int64_t K, const void* Am, int64_t sam, int64_t sak, int at, const void* Bm,
                  int64_t sbk, int64_t sbn, int bt, void* Cm, int64_t ldc, int ct, const int* md, const int* nd,
                  const int* kd, bool lower = false) {
    GemmDesc g{};
    g.lower = lower;
    g.M = M; g.N = N; g.K = K;
    g.A = Am; g.sam = sam; g.sak = sak; g.a_type = at;
    g.B = Bm; g.sbk = sbk; g.sbn = sbn; g.b_type = bt;
    g.C = Cm; g.ldc = ldc; g.out_type = ct;
    g.in_type = at; g.acc_type = 0; g.alpha = 1.0; g.beta = 0.0;
    g.m_dev = md; g.n_dev = nd; g.k_dev = kd;
    gemm(x, g);
  };
  // G1 = R R^T, L1 L1^T = G1
  prod(kcap, kcap, n, R, ldr, 1, dtype, R, 1, ldr, dtype, G, kcap, 0, kr_dev, kr_dev, nullptr, true);
  chol_inv(x, 0, G, kcap, 1, kcap, kr_dev, L1, kcap, L1i, kcap, 1e-15, "chol(R)", false);
  // Q1^T = L1^{-1} R
  prod(kcap, n, kcap, L1i, kcap, 1, 0, R, ldr, 1, dtype, Q1t, n, 0, kr_dev, nullptr, kr_dev);
  // G2 = Q1^T Q1, L2 L2^T = G2
  prod(kcap, kcap, n, Q1t, n, 1, 0, Q1t, 1, n, 0, G, kcap, 0, kr_dev, kr_dev, nullptr, true);
  chol_inv(x, 0, G, kcap, 1, kcap, kr_dev, L2, kcap, L2i, kcap, 0.0, "chol(Q1)", false);
  // Bls = Q^T V = L2^{-1} (Q1^T V) (kr x k)
  if (!x.dry) x.check(build_v_launch(dtype, T, ldt, J, n, kcap, k_dev, V, kcap, x.s), "build V");
  if (corr) {
    double* Gc = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* Lc = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* Lci = static_cast<double*>(x.ar->take((size_t)kcap * kcap * 8));
    double* Zt = static_cast<double*>(x.ar->take((size_t)n * kcap * 8));
    double* W1 = static_cast<double*>(x.ar->take((size_t)n * kcap * 8));
    // Gc = C^T C, its factor's inverse
    prod(kcap, kcap, m, C, 1, ldc, dtype, C, ldc, 1, dtype, Gc, kcap, 0, k_dev, k_dev, nullptr);
    chol_inv(x, 0, Gc, kcap, 1, kcap, k_dev, Lc, kcap, Lci, kcap, 0.0, "chol(C)", false);
    // Zt = A^T C (n x k), then Zt -= V Gc
    prod(n, kcap, m, A, 1, lda, dtype, C, ldc, 1, dtype, Zt, kcap, 0, nullptr, k_dev, nullptr);
    GemmDesc g{};
    g.M = n; g.N = kcap; g.K = kcap;
    g.A = V; g.sam = kcap; g.sak = 1; g.a_type = 0;
    g.B = Gc; g.sbk = kcap; g.sbn = 1; g.b_type = 0;
    g.C = Zt; g.ldc = kcap; g.out_type = 0;
    g.in_type = 0; g.acc_type = 0; g.alpha = -1.0; g.beta = 1.0;
    g.n_dev = k_dev; g.k_dev = k_dev;
    gemm(x, g);
    // W1 = Zt Lc^{-T} (B(kk, j) = Lci[j][kk]), then V += W1 Lc^{-1}
    prod(n, kcap, kcap, Zt, kcap, 1, 0, Lci, 1, kcap, 0, W1, kcap, 0, nullptr, k_dev, k_dev);
    GemmDesc h{};
    h.M = n; h.N = kcap; h.K = kcap;
    h.A = W1; h.sam = kcap; h.sak = 1; h.a_type = 0;
    h.B = Lci; h.sbk = kcap; h.sbn = 1; h.b_type = 0;
    h.C = V; h.ldc = kcap; h.out_type = 0;
    h.in_type = 0; h.acc_type = 0; h.alpha = 1.0; h.beta = 1.0;
    h.n_dev = k_dev; h.k_dev = k_dev;
    gemm(x, h);
  }
  prod(kcap, kcap, n, Q1t, n, 1, 0, V, kcap, 1, 0, B1, kcap, 0, kr_dev, k_dev, nullptr);
  prod(kcap, kcap, kcap, L2i, kcap, 1, 0, B1, kcap, 1, 0, Bls, kcap, 0, kr_dev, k_dev, kr_dev);
  // Y1 = L2^{-T} Bls  (A(i, kk) = L2i[kk][i])
  prod(kcap, kcap, kcap, L2i, 1, kcap, 0, Bls, kcap, 1, 0, Y1, kcap, 0, kr_dev, k_dev, kr_dev);
  // U = Y1^T L1^{-1}  (k x kr): A(i, kk) = Y1[kk][i]
  prod(kcap, kcap, kcap, Y1, 1, kcap, 0, L1i, kcap, 1, 0, U, ldu, dtype, k_dev, kr_dev, kr_dev);
}

void validate(idcur_ctx* ctx, int op, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
              const idcur_opts* opts) {
  if (!ctx) throw Fail{IDCUR_EINVAL};
  (void)A;
  const ArgCheck r = check_id_args(op, dtype, m, n, lda, opts);
  if (r.code != IDCUR_OK) fail(ctx, r.code, r.msg);
}

void execute(idcur_ctx* ctx, int op, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
             const idcur_opts& o, Arena& ar, const Outs& out) {
  Ctx x{ctx, ctx->stream, ar.dry, &ar};
  const int kcap = o.k > 0 ? o.k : o.kmax;
  View X{A, m, n, lda, 1};
  if (op == OP_SKETCH || op == OP_SKETCH_ROW) {
    const View V = op == OP_SKETCH ? X : View{A, n, m, 1, lda};
    const SketchOut s = sketch(x, dtype, V, o, kcap, true);
    if (!ar.dry)
      x.check(copy2d_launch(dtype, V.cols, s.l, s.Y, s.cs, s.rs, out.Yt, out.ldy, 1, x.s), "sketch out");
    return;
  }
  if (op == OP_ROW) {
    View Xt{A, n, m, 1, lda};
    column_id(x, dtype, Xt, o, out.k_out, out.I, out.Tr, out.ldtr, true);
    return;
  }
  // column ID (internal J/T buffers when the caller does not receive them)
  int* J = out.J;
  void* T = out.T;
  int64_t ldt = out.ldt;
  if (!T) {
    T = ar.take((size_t)kcap * n * esz(dtype));
    ldt = n;
  }
  column_id(x, dtype, X, o, out.k_out, J, T, ldt, true);
  if (op == OP_COL) return;
  // C = A(:, J(1:k)), gathered straight into the caller's C when a CUR call
  // returns one (the row ID and the U solve read it there)
  const bool c_out = op == OP_CUR && out.C;
  void* C = c_out ? out.C : ar.take((size_t)m * kcap * esz(dtype));
  const int64_t ldc = c_out ? out.ldc : kcap;
  if (!ar.dry) {
    Stage st(x, "gather");
    x.check(gather_cols_launch(dtype, m, A, lda, J, kcap, out.k_out, C, ldc, dtype, x.s), "gather C");
  }
  void* Tr = out.Tr;
  int64_t ldtr = out.ldtr;
  if (!Tr && op == OP_TWO) {
    Tr = ar.take((size_t)kcap * m * esz(dtype));
    ldtr = m;
  }
  row_id_of_c(x, dtype, C, ldc, m, kcap, out.k_out, out.k_out + 1, out.I, op == OP_TWO, Tr, ldtr, o.t_reg, o.t_svd);
  if (op == OP_TWO) return;
  // CUR: R = A(I(1:k), :), optional C output, then U
  void* R = out.R;
  int64_t ldr = out.ldr;
  if (!R) {
    R = ar.take((size_t)kcap * n * esz(dtype));
    ldr = n;
  }
  if (!ar.dry) {
    Stage st(x, "gather");
    x.check(gather_rows_launch(dtype, n, A, lda, out.I, kcap, out.k_out + 1, R, ldr, dtype, x.s), "gather R");
  }
  Stage st(x, "u_solve");
  solve_u(x, dtype, R, ldr, n, kcap, out.k_out, J, T, ldt, out.U, out.ldu, o.u_correct != 0, A, lda, m, C, ldc);
}

// Error measurement: out[0] = |A - C W|_F^2, out[1] = |A|_F^2 (device doubles).
// which == 0: ID error with C = A(:, J(1:k)), W = V*;  which == 1: CUR error, W = U R.
struct ErrArgs {
  int which;
  const int* J; const void* T; int64_t ldt;
  const void* C; int64_t ldc; const void* U; int64_t ldu; const void* R; int64_t ldr;
  const int* k_out; int kcap; double* out;
};

void run_error(const Ctx& x, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const ErrArgs& e) {
  const int kcap = e.kcap;
  double* W = static_cast<double*>(x.ar->take((size_t)kcap * n * 8));
  double* rpart = static_cast<double*>(x.ar->take(gemm_resid_part_bytes(m, n)));
  double* spart = static_cast<double*>(x.ar->take(1024 * 8));
  const void* C = e.C;
  int64_t ldc = e.ldc;
  if (e.which == 0) {
    void* Cw = x.ar->take((size_t)m * kcap * esz(dtype));
    if (!x.dry) {
      x.check(gather_cols_launch(dtype, m, A, lda, e.J, kcap, e.k_out, Cw, kcap, dtype, x.s), "gather C");
      x.check(build_vstar_launch(dtype, e.T, e.ldt, e.J, n, kcap, e.k_out, W, n, x.s), "build V*");
    }
    C = Cw;
    ldc = kcap;
  } else {
    GemmDesc g{};   // W = U R  (k x n), FP64
    g.M = kcap; g.N = n; g.K = kcap;
    g.A = e.U; g.sam = e.ldu; g.sak = 1;
    g.B = e.R; g.sbk = e.ldr; g.sbn = 1;
    g.C = W; g.ldc = n;
    g.in_type = dtype; g.acc_type = 0; g.out_type = 0;
    g.alpha = 1.0; g.beta = 0.0; g.m_dev = e.k_out; g.k_dev = e.k_out + 1;
    gemm(x, g);
  }
  if (x.dry) return;
  x.check(gemm_resid_launch(dtype, m, n, kcap, C, ldc, dtype, W, n, A, lda, e.k_out, rpart, e.out, x.s), "residual");
  x.check(sumsq_launch(dtype, m, n, A, lda, spart, e.out + 1, x.s), "norm of A");
}

idcur_status run_err(idcur_ctx* ctx, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const ErrArgs& e,
                     void* ws, size_t ws_bytes, size_t* bytes_only) {
  try {
    if (!ctx) return IDCUR_EINVAL;
    if (dtype != IDCUR_F32 && dtype != IDCUR_F64) fail(ctx, IDCUR_EDTYPE, "bad dtype");
    if (m <= 0 || n <= 0 || lda < n || e.kcap <= 0 || e.kcap >= std::min(m, n)) fail(ctx, IDCUR_EINVAL, "bad sizes");
    Arena dry;
    Ctx xd{ctx, ctx->stream, true, &dry};
    run_error(xd, dtype, m, n, A, lda, e);
    if (bytes_only) {
      *bytes_only = dry.off + 256;
      return IDCUR_OK;
    }
    if (!A || !e.k_out || !e.out) fail(ctx, IDCUR_EINVAL, "null pointer");
    if (e.which == 0 && (!e.J || !e.T || e.ldt < 1)) fail(ctx, IDCUR_EINVAL, "J and T are required");
    if (e.which == 1 && (!e.C || !e.U || !e.R || e.ldc < e.kcap || e.ldu < e.kcap || e.ldr < n))
      fail(ctx, IDCUR_EINVAL, "C, U and R are required");
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    Ctx x{ctx, ctx->stream, false, &ar};
    Stage st(x, "error");
    run_error(x, dtype, m, n, A, lda, e);
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

// ---------------------------------------------------------------------------
// Gradient of the column-ID reconstruction loss with the skeleton frozen
// (Section 2.3 / Algorithm 1, sketched as in Section 5.1):
//   Y = Omega A (or A),  T = argmin |Y(:,J1) X - Y(:,J2)|_F = S11^{-1} S12,
//   E = A(:,J2) - A(:,J1) T,  L = |E|_F^2.
// With Tbar = -2 C^T E (C = A(:,J1)) and M = (Y1^T Y1)^{-1} Tbar:
//   Abar(:,J2) = 2E,  Abar(:,J1) = -2 E T^T,
//   Ybar2 = Y1 M,  Ybar1 = (Y2 - Y1 T) M^T - Y1 M T^T,  Abar += Omega^T Ybar.
// Everything is formed with columns in J order (Aj = A(:,J), Gj the gradient)
// and permuted back at the end. Y1^T Y1 = S11^T S11 is factored by the FP64
// Cholesky kernel; the small products run in FP64, the m x n ones in the
// dtype with FP64 accumulation where a cancellation can occur.
// ---------------------------------------------------------------------------
struct BwdArgs {
  const void* omega = nullptr;   // l x m row-major (ld m), or null: Y = A
  int l = 0;
  const int* J = nullptr;
  int k = 0;
  const void* T = nullptr;
  int64_t ldt = 0;
  double scale = 1.0;
  void* dA = nullptr;
  int64_t ldda = 0;
};

void id_col_backward(const Ctx& x, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const BwdArgs& b) {
  const size_t es = esz(dtype);
  const int k = b.k;
  const int64_t n2 = n - k;
  const bool sk = b.omega != nullptr;
  const int l = b.l;
  const int64_t ll = round_up(std::max(l, 1), 4);
  int* Jinv = static_cast<int*>(x.ar->take((size_t)n * sizeof(int)));
  char* Aj = static_cast<char*>(x.ar->take((size_t)m * n * es));   // A(:, J)
  char* Gj = static_cast<char*>(x.ar->take((size_t)m * n * es));   // gradient, J order
  double* Tb = static_cast<double*>(x.ar->take((size_t)k * n2 * 8));
  double* Gr = static_cast<double*>(x.ar->take((size_t)k * k * 8));
  double* Lf = static_cast<double*>(x.ar->take((size_t)k * k * 8));
  double* Li = static_cast<double*>(x.ar->take((size_t)k * k * 8));
  double* W = static_cast<double*>(x.ar->take((size_t)k * n2 * 8));
  double* M = static_cast<double*>(x.ar->take((size_t)k * n2 * 8));
  double* TMt = static_cast<double*>(x.ar->take((size_t)k * k * 8));
  char* Yjt = sk ? static_cast<char*>(x.ar->take((size_t)n * ll * es)) : nullptr;    // Y^T, rows in J order
  char* Rt = sk ? static_cast<char*>(x.ar->take((size_t)n2 * ll * es)) : nullptr;    // (Y2 - Y1 T)^T
  double* Ybt = sk ? static_cast<double*>(x.ar->take((size_t)n * ll * 8)) : nullptr; // Ybar^T
  const int F64 = IDCUR_F64;
  auto mm = [&](int64_t Mr, int64_t Nc, int64_t K, const void* Am, int64_t sam, int64_t sak, int at, const void* Bm,
                int64_t sbk, int64_t sbn, int bt, void* Cm, int64_t ldc, int ct, double alpha, double beta, int acc) {
    GemmDesc g{};
    g.M = Mr; g.N = Nc; g.K = K;
    g.A = Am; g.sam = sam; g.sak = sak; g.a_type = at;
    g.B = Bm; g.sbk = sbk; g.sbn = sbn; g.b_type = bt;
    g.C = Cm; g.ldc = ldc; g.out_type = ct;
    g.in_type = at; g.acc_type = acc; g.alpha = alpha; g.beta = beta;
    gemm(x, g);
  };
  const int acc_d = dtype == IDCUR_F32 ? 1 : 0;   // accumulation in the dtype
  // C = Aj(:, 0:k), E2 = 2E lives in Gj(:, k:n), Y1^T = Yjt rows 0..k
  if (!x.dry) {
    x.check(gather_cols_scaled_launch(dtype, m, A, lda, n, b.J, n, 1.0, 0, Aj, n, x.c->dstatus, x.s), "gather A(:,J)");
    x.check(gather_cols_scaled_launch(dtype, m, A, lda, n, b.J + k, n2, 2.0, 0, Gj + k * es, n, x.c->dstatus, x.s),
            "gather A(:,J2)");
  }
  // E2 = 2 A(:,J2) - 2 C T
  mm(m, n2, k, Aj, n, 1, dtype, b.T, b.ldt, 1, dtype, Gj + k * es, n, dtype, -2.0, 1.0, 0);
  // Tbar = -C^T E2 (FP64)
  mm(k, n2, m, Aj, 1, n, dtype, Gj + k * es, n, 1, dtype, Tb, n2, F64, -1.0, 0.0, 0);
  // Gj(:, 0:k) = -E2 T^T
  mm(m, k, n2, Gj + k * es, n, 1, dtype, b.T, 1, b.ldt, dtype, Gj, n, dtype, -1.0, 0.0, acc_d);
  // Gram Y1^T Y1 = S11^T S11
  if (sk) {
    // Y^T = Aj^T Omega^T (n x l, ld ll)
    mm(n, l, m, Aj, 1, n, dtype, b.omega, 1, m, dtype, Yjt, ll, dtype, 1.0, 0.0, acc_d);
    mm(k, k, l, Yjt, ll, 1, dtype, Yjt, 1, ll, dtype, Gr, k, F64, 1.0, 0.0, 0);
  } else {
    mm(k, k, m, Aj, 1, n, dtype, Aj, n, 1, dtype, Gr, k, F64, 1.0, 0.0, 0);
  }
  chol_inv(x, 0, Gr, k, 1, k, nullptr, Lf, k, Li, k, 0.0, "chol(Y1^T Y1)", false);
  // M = Li^T (Li Tbar) = (Y1^T Y1)^{-1} Tbar;  TMt = T M^T
  mm(k, n2, k, Li, k, 1, F64, Tb, n2, 1, F64, W, n2, F64, 1.0, 0.0, 0);
  mm(k, n2, k, Li, 1, k, F64, W, n2, 1, F64, M, n2, F64, 1.0, 0.0, 0);
  mm(k, k, n2, b.T, b.ldt, 1, dtype, M, 1, n2, F64, TMt, k, F64, 1.0, 0.0, 0);
  if (sk) {
    // R^T = Y2^T - T^T Y1^T
    if (!x.dry) x.check(copy2d_launch(dtype, n2, l, Yjt + (size_t)k * ll * es, ll, 1, Rt, ll, 1, x.s), "copy Y2^T");
    mm(n2, l, k, b.T, 1, b.ldt, dtype, Yjt, ll, 1, dtype, Rt, ll, dtype, -1.0, 1.0, 0);
    // Ybar2^T = M^T Y1^T;  Ybar1^T = M R^T - (T M^T) Y1^T
    mm(n2, l, k, M, 1, n2, F64, Yjt, ll, 1, dtype, Ybt + (size_t)k * ll, ll, F64, 1.0, 0.0, 0);
    mm(k, l, n2, M, n2, 1, F64, Rt, ll, 1, dtype, Ybt, ll, F64, 1.0, 0.0, 0);
    mm(k, l, k, TMt, k, 1, F64, Yjt, ll, 1, dtype, Ybt, ll, F64, -1.0, 1.0, 0);
    // Gj += Omega^T Ybar
    mm(m, n, l, b.omega, 1, m, dtype, Ybt, 1, ll, F64, Gj, n, dtype, 1.0, 1.0, 0);
  } else {
    // Y = A: Y1 = C, Y2 - Y1 T = E.  Ybar1 = E M^T - C (T M^T)^T first (it reads E),
    // then Ybar2 = C M
    mm(m, k, n2, Gj + k * es, n, 1, dtype, M, 1, n2, F64, Gj, n, dtype, 0.5, 1.0, 0);
    mm(m, k, k, Aj, n, 1, dtype, TMt, 1, k, F64, Gj, n, dtype, -1.0, 1.0, 0);
    mm(m, n2, k, Aj, n, 1, dtype, M, n2, 1, F64, Gj + k * es, n, dtype, 1.0, 1.0, 0);
  }
  // dA(:, c) = scale * Gj(:, Jinv(c))
  if (!x.dry) {
    x.check(invert_perm_launch(b.J, n, Jinv, x.c->dstatus, x.s), "invert J");
    x.check(gather_cols_scaled_launch(dtype, m, Gj, n, n, Jinv, n, b.scale, 0, b.dA, b.ldda, x.c->dstatus, x.s),
            "scatter gradient");
  }
}

idcur_status run_bwd(idcur_ctx* ctx, int dtype, int64_t m, int64_t n, const void* A, int64_t lda, const BwdArgs& b,
                     void* ws, size_t ws_bytes, size_t* bytes_only) {
  try {
    if (!ctx) return IDCUR_EINVAL;
    if (dtype != IDCUR_F32 && dtype != IDCUR_F64) fail(ctx, IDCUR_EDTYPE, "bad dtype");
    if (m <= 0 || n <= 0 || lda < n) fail(ctx, IDCUR_EINVAL, "bad sizes");
    if (b.k <= 0 || b.k >= std::min(m, n) || b.k > kMaxRank)
      fail(ctx, IDCUR_EINVAL, "k must satisfy 0 < k < min(m, n), k <= 4096");
    if (b.omega && (b.l < b.k || b.l > m)) fail(ctx, IDCUR_EINVAL, "sketch rows l must satisfy k <= l <= m");
    Arena dry;
    Ctx xd{ctx, ctx->stream, true, &dry};
    id_col_backward(xd, dtype, m, n, A, lda, b);
    if (bytes_only) {
      *bytes_only = dry.off + 256;
      return IDCUR_OK;
    }
    if (!A || !b.J || !b.T || !b.dA) fail(ctx, IDCUR_EINVAL, "null pointer");
    if (b.ldt < n - b.k || b.ldda < n) fail(ctx, IDCUR_EINVAL, "ldt or ldda too small");
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    Ctx x{ctx, ctx->stream, false, &ar};
    Stage st(x, "backward");
    id_col_backward(x, dtype, m, n, A, lda, b);
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

// ---------------------------------------------------------------------------
// Batched adaptive-rank column ID (one persistent launch, batched.hip)
// ---------------------------------------------------------------------------
struct BatchedCall {
  int nblk, mmax, nmax;
  const int32_t* m; const int32_t* n; const void* const* A; const int64_t* lda;
  int32_t* k_out; int32_t* const* J; void* const* T; const int64_t* ldt;
};

void batched_validate(idcur_ctx* ctx, int dtype, const BatchedCall& c, const idcur_opts* o) {
  if (!ctx) throw Fail{IDCUR_EINVAL};
  const ArgCheck r = check_batched_args(dtype, c.nblk, c.mmax, c.nmax, o, batched_max_width(), batched_max_sketch());
  if (r.code != IDCUR_OK) fail(ctx, r.code, r.msg);
}

std::vector<int64_t> batched_key(const BatchedCall& c, const idcur_opts& o) {
  int lg = 0;
  while ((1 << lg) < c.nblk) ++lg;
  return {lg, c.mmax, c.nmax, (o.k > 0 ? o.k : o.kmax) + o.p, o.k > 0 ? 1 : 0};
}

// Carves the workspace and (unless dry) enqueues: Omega^T, then the launch.
void batched_run(const Ctx& x, const BatchedCall& c, const idcur_opts& o, int variant) {
  const int kcap = o.k > 0 ? o.k : o.kmax;
  const int lcap = kcap + o.p;
  const int ldom = batched_ldom(lcap), mpad = batched_mpad(c.mmax);
  float* omt = static_cast<float*>(x.ar->take((size_t)mpad * ldom * sizeof(float)));
  int* order = static_cast<int*>(x.ar->take((size_t)std::max(c.nblk, 1) * sizeof(int)));
  int* queue = static_cast<int*>(x.ar->take(256));
  if (x.dry || c.nblk == 0) return;
  Stage st(x, "batched");
  x.check(zero_launch(omt, (size_t)mpad * ldom * sizeof(float), x.s), "zero Omega");
  if (o.omega)
    x.check(copy2d_launch(IDCUR_F32, lcap, c.mmax, o.omega, c.mmax, 1, omt, 1, ldom, x.s), "Omega copy");
  else
    x.check(gaussian_launch(IDCUR_F32, lcap, c.mmax, o.seed, 0, omt, 1, ldom, x.s), "Omega");
  BatchedArgs a{};
  a.nblk = c.nblk;
  a.m = c.m; a.n = c.n;
  a.A = reinterpret_cast<const float* const*>(c.A); a.lda = c.lda;
  a.J = c.J; a.T = reinterpret_cast<float* const*>(c.T); a.ldt = c.ldt;
  a.k_out = c.k_out;
  a.omt = omt;
  a.mmax = c.mmax; a.nmax = c.nmax; a.lcap = lcap; a.p = o.p; a.kfix = o.k;
  a.tol = o.k > 0 ? 0.0 : o.tol;
  a.rank_tol = o.rank_tol > 0 ? o.rank_tol : default_rank_tol(IDCUR_F32, lcap, o.k == 0);
  a.order = order; a.queue = queue; a.status = x.c->dstatus;
  x.check(batched_launch(a, variant, x.c->num_cus, x.s), "batched launch");
}

int batched_default_variant() { return 2; }   // prefetch 1, two workgroups per CU, largest first

idcur_status run_batched(idcur_ctx* ctx, int dtype, const BatchedCall& c, const idcur_opts* opts, void* ws,
                         size_t ws_bytes, size_t* bytes_only, int tune, int* variant_out) {
  try {
    batched_validate(ctx, dtype, c, opts);
    Arena dry;
    Ctx xd{ctx, ctx->stream, true, &dry};
    batched_run(xd, c, *opts, 0);
    if (bytes_only) {
      *bytes_only = dry.off + 256;
      return IDCUR_OK;
    }
    if (c.nblk > 0 && (!c.m || !c.n || !c.A || !c.lda || !c.k_out || !c.J || !c.T || !c.ldt))
      fail(ctx, IDCUR_EINVAL, "null array");
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    hipcheck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    Ctx x{ctx, ctx->stream, false, &ar};
    const auto key = batched_key(c, *opts);
    if (!tune) {
      int v = ctx->batched_forced;
      if (v < 0) {
        auto it = ctx->batched_tuned.find(key);
        v = it != ctx->batched_tuned.end() ? it->second : batched_default_variant();
      }
      batched_run(x, c, *opts, v);
      if (variant_out) *variant_out = v;
      return IDCUR_OK;
    }
    // autotune: time every variant (two untimed launches, then three timed), keep
    // the fastest for this size class, and leave its results in the outputs
    hipEvent_t e0 = ctx->get_event(), e1 = ctx->get_event();
    if (!e0 || !e1) fail(ctx, IDCUR_EHIP, "event creation failed");
    int best = batched_default_variant();
    float best_ms = 0.0f;
    for (int v = 0; v < batched_num_variants(); ++v) {
      for (int r = 0; r < 2; ++r) {
        ar.off = 0;
        batched_run(x, c, *opts, v);
      }
      hipcheck(ctx, hipEventRecord(e0, ctx->stream), "event");
      for (int r = 0; r < 3; ++r) {
        ar.off = 0;
        batched_run(x, c, *opts, v);
      }
      hipcheck(ctx, hipEventRecord(e1, ctx->stream), "event");
      hipcheck(ctx, hipEventSynchronize(e1), "event sync");
      float ms = 0.0f;
      hipcheck(ctx, hipEventElapsedTime(&ms, e0, e1), "event time");
      if (v == 0 || ms < best_ms) { best_ms = ms; best = v; }
    }
    ctx->pool.push_back(e0);
    ctx->pool.push_back(e1);
    ctx->batched_tuned[key] = best;
    ar.off = 0;
    batched_run(x, c, *opts, best);
    if (variant_out) *variant_out = best;
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

// ---------------------------------------------------------------------------
// Batched gradient of the fixed-rank column IDs' reconstruction losses (one
// persistent launch, batched_bwd.hip)
// ---------------------------------------------------------------------------
struct BatchedBwdCall {
  int nblk, mmax, nmax;
  const int32_t* m; const int32_t* n; const void* const* A; const int64_t* lda;
  const int32_t* k; const int32_t* const* J; const void* const* T; const int64_t* ldt;
  double scale;
  void* const* dA; const int64_t* ldd;
};

void batched_bwd_run(const Ctx& x, const BatchedBwdCall& c, const idcur_opts& o) {
  const int l = o.k + o.p;
  const int ldom = batched_ldom(l);
  const int64_t mrows = round_up(std::max(c.mmax, 1), 16);
  const int grid = batched_bwd_grid(c.nblk, x.c->num_cus);
  float* omt = static_cast<float*>(x.ar->take((size_t)mrows * ldom * sizeof(float)));
  float* slot = static_cast<float*>(x.ar->take((size_t)grid * batched_bwd_slot_floats(o.k, l, c.nmax) * sizeof(float)));
  int* queue = static_cast<int*>(x.ar->take(256));
  if (x.dry || c.nblk == 0) return;
  Stage st(x, "backward");
  x.check(zero_launch(omt, (size_t)mrows * ldom * sizeof(float), x.s), "zero Omega");
  if (o.omega)
    x.check(copy2d_launch(IDCUR_F32, l, c.mmax, o.omega, c.mmax, 1, omt, 1, ldom, x.s), "Omega copy");
  else
    x.check(gaussian_launch(IDCUR_F32, l, c.mmax, o.seed, 0, omt, 1, ldom, x.s), "Omega");
  BatchedBwdArgs a{};
  a.nblk = c.nblk;
  a.m = c.m; a.n = c.n; a.k = c.k;
  a.A = reinterpret_cast<const float* const*>(c.A); a.lda = c.lda;
  a.J = c.J; a.T = reinterpret_cast<const float* const*>(c.T); a.ldt = c.ldt;
  a.dA = reinterpret_cast<float* const*>(c.dA); a.ldd = c.ldd;
  a.omt = omt; a.ldom = ldom;
  a.mmax = c.mmax; a.nmax = c.nmax; a.l = l; a.kcap = o.k;
  a.scale = c.scale;
  a.slot = slot; a.queue = queue; a.status = x.c->dstatus;
  x.check(batched_bwd_launch(a, grid, x.s), "batched backward launch");
}

idcur_status run_batched_bwd(idcur_ctx* ctx, int dtype, const BatchedBwdCall& c, const idcur_opts* o, void* ws,
                             size_t ws_bytes, size_t* bytes_only) {
  try {
    if (!ctx) return IDCUR_EINVAL;
    if (!o) fail(ctx, IDCUR_EINVAL, "opts is NULL");
    if (dtype != IDCUR_F32) fail(ctx, IDCUR_EDTYPE, "the batched backward takes FP32 blocks");
    if (o->prec != IDCUR_PREC_NATIVE) fail(ctx, IDCUR_EDTYPE, "the batched backward sketches in FP32");
    if (c.nblk < 0 || c.nblk > (1 << 20)) fail(ctx, IDCUR_EINVAL, "nblk must be in [0, 2^20]");
    if (c.mmax < 1 || c.mmax > (1 << 24)) fail(ctx, IDCUR_EINVAL, "mmax must be in [1, 2^24]");
    if (c.nmax < 1 || c.nmax > batched_bwd_max_width()) fail(ctx, IDCUR_EINVAL, "nmax must be in [1, 512]");
    if (o->k < 1) fail(ctx, IDCUR_EINVAL, "the batched backward differentiates fixed-rank IDs (k >= 1)");
    if (o->p < 1) fail(ctx, IDCUR_EINVAL, "the batched backward needs oversampling p >= 1");
    if (o->q != 0) fail(ctx, IDCUR_EINVAL, "the batched backward takes no power steps (q = 0)");
    if ((int64_t)o->k + o->p > batched_bwd_max_sketch()) fail(ctx, IDCUR_EINVAL, "k + p must be <= 64");
    if (!std::isfinite(c.scale)) fail(ctx, IDCUR_EINVAL, "scale must be finite");
    Arena dry;
    Ctx xd{ctx, ctx->stream, true, &dry};
    batched_bwd_run(xd, c, *o);
    if (bytes_only) {
      *bytes_only = dry.off + 256;
      return IDCUR_OK;
    }
    if (c.nblk > 0 && (!c.m || !c.n || !c.A || !c.lda || !c.k || !c.J || !c.T || !c.ldt || !c.dA || !c.ldd))
      fail(ctx, IDCUR_EINVAL, "null array");
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    hipcheck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    Ctx x{ctx, ctx->stream, false, &ar};
    batched_bwd_run(x, c, *o);
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

idcur_status run(idcur_ctx* ctx, int op, int dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                 const idcur_opts* opts, void* ws, size_t ws_bytes, const Outs& out) {
  try {
    validate(ctx, op, dtype, m, n, A, lda, opts);
    const ArgCheck r = check_id_outs(op, m, n, A, *opts, out);
    if (r.code != IDCUR_OK) fail(ctx, r.code, r.msg);
    Arena dry;
    execute(ctx, op, dtype, m, n, A, lda, *opts, dry, out);
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    hipcheck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    execute(ctx, op, dtype, m, n, A, lda, *opts, ar, out);
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

// Column ID of a sparse A (compressed sparse column form): the sketch
// Y = Omega A by spmm_csc_kernel (Section 5.1), then the same CPQR and T as the
// dense path on Y.
struct Csc {
  int64_t m, n, nnz;
  const int64_t* colptr;
  const int* rowidx;
  const void* vals;
};

void validate_csc(idcur_ctx* ctx, int dtype, const Csc& a, const idcur_opts* o) {
  validate(ctx, OP_COL, dtype, a.m, a.n, nullptr, std::max<int64_t>(a.n, 1), o);
  if (a.nnz < 0) fail(ctx, IDCUR_EINVAL, "nnz must be >= 0");
  if (a.n > 0x7fffffff) fail(ctx, IDCUR_EINVAL, "n must be below 2^31");
  const int kcap = o->k > 0 ? o->k : o->kmax;
  if (o->p < 0 || (int64_t)kcap + o->p >= a.m)
    fail(ctx, IDCUR_EINVAL, "the sparse column ID sketches: p >= 0 and k (kmax) + p < m");
  if (o->q != 0) fail(ctx, IDCUR_EINVAL, "the sparse column ID takes no power steps (q = 0)");
  if (o->sketch != IDCUR_SKETCH_GAUSSIAN) fail(ctx, IDCUR_EINVAL, "the sparse column ID takes the Gaussian sketch");
  if (o->prec != IDCUR_PREC_NATIVE) fail(ctx, IDCUR_EDTYPE, "the sparse column ID computes in the dtype");
}

void execute_csc(idcur_ctx* ctx, int dtype, const Csc& a, const idcur_opts& o, Arena& ar, const Outs& out) {
  Ctx x{ctx, ctx->stream, ar.dry, &ar};
  const int kcap = o.k > 0 ? o.k : o.kmax;
  const int l = kcap + o.p;
  const int64_t ll = round_up(l, 4);
  void* Omt = ar.take((size_t)a.m * ll * esz(dtype));
  void* Yt = ar.take((size_t)a.n * ll * esz(dtype));
  SpmmDesc d{};
  d.m = a.m; d.n = a.n; d.nnz = a.nnz;
  d.colptr = a.colptr; d.rowidx = a.rowidx; d.vals = a.vals;
  d.Omt = Omt; d.ldom = ll; d.l = l; d.Yt = Yt; d.ldo = ll;
  d.splits = spmm_pick_splits(a.n, a.nnz, x.c->num_cus);
  d.status = x.c->dstatus;
  void* part = d.splits > 1 ? ar.take(spmm_part_bytes(d, (int)esz(dtype))) : nullptr;
  if (!x.dry) {
    {
      Stage st(x, "omega");
      if (o.omega)
        x.check(copy2d_launch(dtype, l, a.m, o.omega, a.m, 1, Omt, 1, ll, x.s), "omega copy");
      else
        x.check(gaussian_launch(dtype, l, a.m, o.seed, 0, Omt, 1, ll, x.s), "omega");
    }
    Stage st(x, "spmm");
    x.check(spmm_csc_launch(dtype, d, part, x.s), "sparse sketch");
  }
  // Y (l x n) is the sketch: the dense column ID on it, without sketching again
  idcur_opts o2 = o;
  o2.p = -1;
  const View Y{Yt, l, a.n, 1, ll};
  column_id(x, dtype, Y, o2, out.k_out, out.J, out.T, out.ldt, false);
}

// CUR of a sparse A (Algorithm 3 on the sparse column ID): C = A(:, J(1:k)) and
// R = A(I(1:k), :) gathered from the compressed columns into dense blocks, the
// row ID of C and U = V* R^+ as on the dense path.
void execute_cur_csc(idcur_ctx* ctx, int dtype, const Csc& a, const idcur_opts& o, Arena& ar, const Outs& out) {
  Ctx x{ctx, ctx->stream, ar.dry, &ar};
  const int kcap = o.k > 0 ? o.k : o.kmax;
  const int64_t m = a.m, n = a.n;
  Outs oc;
  oc.k_out = out.k_out;
  oc.J = out.J;
  oc.T = ar.take((size_t)kcap * n * esz(dtype));
  oc.ldt = n;
  execute_csc(ctx, dtype, a, o, ar, oc);
  void* C = ar.take((size_t)m * kcap * esz(dtype));
  if (!ar.dry) {
    Stage st(x, "gather");
    x.check(zero_launch(C, (size_t)m * kcap * esz(dtype), x.s), "zero C");
    x.check(csc_gather_cols_launch(dtype, m, n, a.nnz, a.colptr, a.rowidx, a.vals, out.J, kcap, out.k_out, C, kcap,
                                   x.c->dstatus, x.s),
            "gather C");
  }
  row_id_of_c(x, dtype, C, kcap, m, kcap, out.k_out, out.k_out + 1, out.I, false, nullptr, 0, o.t_reg, o.t_svd);
  void* R = ar.take((size_t)kcap * n * esz(dtype));
  int* slot = static_cast<int*>(ar.take((size_t)m * sizeof(int)));
  if (!ar.dry) {
    Stage st(x, "gather");
    x.check(zero_launch(R, (size_t)kcap * n * esz(dtype), x.s), "zero R");
    x.check(csc_gather_rows_launch(dtype, m, n, a.nnz, a.colptr, a.rowidx, a.vals, out.I, kcap, out.k_out + 1, slot,
                                   R, n, x.s),
            "gather R");
    if (out.C) x.check(copy2d_launch(dtype, m, kcap, C, kcap, 1, out.C, out.ldc, 1, x.s), "C out");
    if (out.R) x.check(copy2d_launch(dtype, kcap, n, R, n, 1, out.R, out.ldr, 1, x.s), "R out");
  }
  Stage st(x, "u_solve");
  solve_u(x, dtype, R, n, n, kcap, out.k_out, out.J, oc.T, oc.ldt, out.U, out.ldu);
}

}  // namespace
}  // namespace idcur

using namespace idcur;

extern "C" {

void idcur_opts_default(idcur_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->p = -1;
  o->prec = IDCUR_PREC_NATIVE;
  o->norms = IDCUR_NORMS_DOWNDATE;
}

// Workspace of idcur_id_col_noalloc: a fixed device array, one copy per GPU the
// library runs on, held until the process ends. In host code the name stands for
// a host-side symbol, not a device address: hipGetSymbolAddress gives the device
// address, once per device, at context creation.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

idcur_status idcur_create(idcur_ctx** out, void* stream) {
  if (!out) return IDCUR_EINVAL;
  *out = nullptr;
  idcur_ctx* c = new idcur_ctx();
  c->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return IDCUR_EHIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) { delete c; return IDCUR_EHIP; }
  c->num_cus = prop.multiProcessorCount;
  if (hipMalloc(&c->dstatus, 64) != hipSuccess) { delete c; return IDCUR_EHIP; }
  if (hipMemset(c->dstatus, 0, 64) != hipSuccess) { (void)hipFree(c->dstatus); delete c; return IDCUR_EHIP; }
  if (hipGetSymbolAddress(&c->noalloc_scratch, HIP_SYMBOL(scratch)) != hipSuccess || !c->noalloc_scratch) {
    (void)hipFree(c->dstatus);
    delete c;
    return IDCUR_EHIP;
  }
  *out = c;
  return IDCUR_OK;
}

idcur_status idcur_set_stream(idcur_ctx* ctx, void* stream) {
  if (!ctx) return IDCUR_EINVAL;
  ctx->stream = static_cast<hipStream_t>(stream);
  return IDCUR_OK;
}

idcur_status idcur_destroy(idcur_ctx* ctx) {
  if (!ctx) return IDCUR_EINVAL;
  ctx->recycle();
  for (hipEvent_t e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->dstatus) (void)hipFree(ctx->dstatus);
  delete ctx;
  return IDCUR_OK;
}

const char* idcur_last_error(const idcur_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

idcur_status idcur_sync_status(idcur_ctx* ctx) {
  if (!ctx) return IDCUR_EINVAL;
  int st = 0;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) { ctx->err = "stream synchronisation failed"; return IDCUR_EHIP; }
  if (hipMemcpy(&st, ctx->dstatus, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return IDCUR_EHIP;
  if (hipMemset(ctx->dstatus, 0, sizeof(int)) != hipSuccess) return IDCUR_EHIP;
  if (st & ST_TIMEOUT) { ctx->err = "a grid-wide wait exceeded its spin limit"; return IDCUR_ETIMEOUT; }
  if (st & ST_NONFINITE) { ctx->err = "non-finite value or breakdown in a factorisation"; return IDCUR_ENONFINITE; }
  if (st & ST_BADINDEX) { ctx->err = "an index array held a value out of range"; return IDCUR_EINVAL; }
  if (st & ST_RANKCAP) { ctx->err = "tolerance not reached within the rank cap"; return IDCUR_ERANKCAP; }
  return IDCUR_OK;
}

idcur_status idcur_timing_enable(idcur_ctx* ctx, int32_t enable) {
  if (!ctx) return IDCUR_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) { ctx->err = "stream synchronisation failed"; return IDCUR_EHIP; }
  ctx->recycle();
  ctx->timing = enable != 0;
  return IDCUR_OK;
}

idcur_status idcur_timing_read(idcur_ctx* ctx, const char* stage, double* total_ms, int32_t* count) {
  if (!ctx || !stage || !total_ms || !count) return IDCUR_EINVAL;
  if (hipStreamSynchronize(ctx->stream) != hipSuccess) { ctx->err = "stream synchronisation failed"; return IDCUR_EHIP; }
  double tot = 0.0;
  int cnt = 0;
  for (auto& m : ctx->marks) {
    if (m.stage != stage) continue;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess) { ctx->err = "event timing failed"; return IDCUR_EHIP; }
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *count = cnt;
  return IDCUR_OK;
}

idcur_status idcur_workspace_bytes(idcur_ctx* ctx, int32_t op, int32_t dtype, int64_t m, int64_t n,
                                   const idcur_opts* opts, size_t* bytes) {
  try {
    if (!bytes) fail(ctx, IDCUR_EINVAL, "bytes is NULL");
    validate(ctx, op, dtype, m, n, nullptr, std::max<int64_t>(n, 1), opts);
    Arena dry;
    Outs out;
    out.ldt = out.ldtr = std::max(m, n);
    execute(ctx, op, dtype, m, n, nullptr, n, *opts, dry, out);
    *bytes = dry.off + 256;
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

idcur_status idcur_id_col_csc_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz,
                                              const idcur_opts* opts, size_t* bytes) {
  try {
    if (!bytes) fail(ctx, IDCUR_EINVAL, "bytes is NULL");
    const Csc a{m, n, nnz, nullptr, nullptr, nullptr};
    validate_csc(ctx, dtype, a, opts);
    Arena dry;
    Outs out;
    out.ldt = n;
    execute_csc(ctx, dtype, a, *opts, dry, out);
    *bytes = dry.off + 256;
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

idcur_status idcur_id_col_csc(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                              const int32_t* rowidx, const void* vals, const idcur_opts* opts, void* ws, size_t ws_bytes,
                              int32_t* k_out, int32_t* J, void* T, int64_t ldt) {
  try {
    const Csc a{m, n, nnz, colptr, rowidx, vals};
    validate_csc(ctx, dtype, a, opts);
    if (!colptr || (nnz > 0 && (!rowidx || !vals))) fail(ctx, IDCUR_EINVAL, "colptr, rowidx and vals are required");
    if (!k_out || !J || !T) fail(ctx, IDCUR_EINVAL, "k_out, J and T are required");
    const int kcap = opts->k > 0 ? opts->k : opts->kmax;
    if (ldt < (opts->k > 0 ? n - kcap : n)) fail(ctx, IDCUR_EINVAL, "ldt too small");
    Outs out;
    out.k_out = k_out; out.J = J; out.T = T; out.ldt = ldt;
    Arena dry;
    execute_csc(ctx, dtype, a, *opts, dry, out);
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    hipcheck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    execute_csc(ctx, dtype, a, *opts, ar, out);
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

idcur_status idcur_cur_csc_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz,
                                           const idcur_opts* opts, size_t* bytes) {
  try {
    if (!bytes) fail(ctx, IDCUR_EINVAL, "bytes is NULL");
    const Csc a{m, n, nnz, nullptr, nullptr, nullptr};
    validate_csc(ctx, dtype, a, opts);
    if (opts->u_correct) fail(ctx, IDCUR_EINVAL, "the sparse CUR solves the plain U system (u_correct = 0)");
    Arena dry;
    Outs out;
    execute_cur_csc(ctx, dtype, a, *opts, dry, out);
    *bytes = dry.off + 256;
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

idcur_status idcur_cur_csc(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                           const int32_t* rowidx, const void* vals, const idcur_opts* opts, void* ws, size_t ws_bytes,
                           int32_t* k_out, int32_t* J, int32_t* I, void* U, int64_t ldu, void* C, int64_t ldc, void* R,
                           int64_t ldr) {
  try {
    const Csc a{m, n, nnz, colptr, rowidx, vals};
    validate_csc(ctx, dtype, a, opts);
    if (opts->u_correct) fail(ctx, IDCUR_EINVAL, "the sparse CUR solves the plain U system (u_correct = 0)");
    if (!colptr || (nnz > 0 && (!rowidx || !vals))) fail(ctx, IDCUR_EINVAL, "colptr, rowidx and vals are required");
    if (!k_out || !J || !I || !U) fail(ctx, IDCUR_EINVAL, "k_out, J, I and U are required");
    const int kcap = opts->k > 0 ? opts->k : opts->kmax;
    if (ldu < kcap) fail(ctx, IDCUR_EINVAL, "ldu too small");
    if (C && ldc < kcap) fail(ctx, IDCUR_EINVAL, "ldc too small");
    if (R && ldr < n) fail(ctx, IDCUR_EINVAL, "ldr too small");
    Outs out;
    out.k_out = k_out; out.J = J; out.I = I; out.U = U; out.ldu = ldu; out.C = C; out.ldc = ldc; out.R = R; out.ldr = ldr;
    Arena dry;
    execute_cur_csc(ctx, dtype, a, *opts, dry, out);
    if (!ws || ws_bytes < dry.off) fail(ctx, IDCUR_EWORKSPACE, "workspace missing or too small");
    Arena ar;
    ar.dry = false;
    ar.base = static_cast<char*>(ws);
    ar.cap = ws_bytes;
    hipcheck(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    execute_cur_csc(ctx, dtype, a, *opts, ar, out);
    return IDCUR_OK;
  } catch (const Fail& f) {
    return f.code;
  }
}

idcur_status idcur_id_col(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                          const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out, int32_t* J, void* T,
                          int64_t ldt) {
  Outs o;
  o.k_out = k_out; o.J = J; o.T = T; o.ldt = ldt;
  return run(ctx, OP_COL, dtype, m, n, A, lda, opts, ws, ws_bytes, o);
}

idcur_status idcur_id_col_noalloc(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                                  const idcur_opts* opts, int32_t* k_out, int32_t* J, void* T, int64_t ldt) {
  if (!ctx) return IDCUR_EINVAL;
  if (!ctx->noalloc_scratch) {
    ctx->err = "no scratch address for this device";
    return IDCUR_EHIP;
  }
  size_t need = 0;
  const idcur_status st = idcur_workspace_bytes(ctx, IDCUR_OP_ID_COL, dtype, m, n, opts, &need);
  if (st != IDCUR_OK) return st;
  if (need > kNoAllocScratchBytes) {
    ctx->err = "problem needs " + std::to_string(need) + " bytes of workspace, above the " +
               std::to_string(kNoAllocScratchBytes) + "-byte scratch array of idcur_id_col_noalloc";
    return IDCUR_EWORKSPACE;
  }
  // stage timers would create events: none are taken in this call
  const bool timing = ctx->timing;
  ctx->timing = false;
  Outs o;
  o.k_out = k_out; o.J = J; o.T = T; o.ldt = ldt;
  const idcur_status r = run(ctx, OP_COL, dtype, m, n, A, lda, opts, ctx->noalloc_scratch, kNoAllocScratchBytes, o);
  ctx->timing = timing;
  return r;
}

idcur_status idcur_id_row(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                          const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out, int32_t* I, void* Tr,
                          int64_t ldtr) {
  Outs o;
  o.k_out = k_out; o.I = I; o.Tr = Tr; o.ldtr = ldtr;
  return run(ctx, OP_ROW, dtype, m, n, A, lda, opts, ws, ws_bytes, o);
}

idcur_status idcur_id_two_sided(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                                const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out, int32_t* J, void* T,
                                int64_t ldt, int32_t* I, void* Tr, int64_t ldtr) {
  Outs o;
  o.k_out = k_out; o.J = J; o.T = T; o.ldt = ldt; o.I = I; o.Tr = Tr; o.ldtr = ldtr;
  return run(ctx, OP_TWO, dtype, m, n, A, lda, opts, ws, ws_bytes, o);
}

idcur_status idcur_cur(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                       const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out, int32_t* J, int32_t* I,
                       void* U, int64_t ldu, void* C, int64_t ldc, void* R, int64_t ldr) {
  Outs o;
  o.k_out = k_out; o.J = J; o.I = I; o.U = U; o.ldu = ldu; o.C = C; o.ldc = ldc; o.R = R; o.ldr = ldr;
  return run(ctx, OP_CUR, dtype, m, n, A, lda, opts, ws, ws_bytes, o);
}

idcur_status idcur_sketch(idcur_ctx* ctx, int32_t op, int32_t dtype, int64_t m, int64_t n, const void* A,
                          int64_t lda, const idcur_opts* opts, void* ws, size_t ws_bytes, void* Yt, int64_t ldy) {
  if (op != IDCUR_OP_SKETCH && op != IDCUR_OP_SKETCH_ROW) {
    if (ctx) ctx->err = "op must be IDCUR_OP_SKETCH or IDCUR_OP_SKETCH_ROW";
    return IDCUR_EINVAL;
  }
  Outs o;
  o.Yt = Yt; o.ldy = ldy;
  return run(ctx, op, dtype, m, n, A, lda, opts, ws, ws_bytes, o);
}

idcur_status idcur_error_workspace_bytes(idcur_ctx* ctx, int32_t which, int32_t dtype, int64_t m, int64_t n,
                                         int32_t kcap, size_t* bytes) {
  if (!bytes || (which != 0 && which != 1)) return IDCUR_EINVAL;
  ErrArgs e{};
  e.which = which;
  e.kcap = kcap;
  return run_err(ctx, dtype, m, n, nullptr, n, e, nullptr, 0, bytes);
}

idcur_status idcur_id_error(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                            const int32_t* J, const void* T, int64_t ldt, const int32_t* k_out, int32_t kcap, void* ws,
                            size_t ws_bytes, double* out) {
  ErrArgs e{};
  e.which = 0; e.J = J; e.T = T; e.ldt = ldt; e.k_out = k_out; e.kcap = kcap; e.out = out;
  return run_err(ctx, dtype, m, n, A, lda, e, ws, ws_bytes, nullptr);
}

idcur_status idcur_cur_error(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                             const void* C, int64_t ldc, const void* U, int64_t ldu, const void* R, int64_t ldr,
                             const int32_t* k_out, int32_t kcap, void* ws, size_t ws_bytes, double* out) {
  ErrArgs e{};
  e.which = 1; e.C = C; e.ldc = ldc; e.U = U; e.ldu = ldu; e.R = R; e.ldr = ldr;
  e.k_out = k_out; e.kcap = kcap; e.out = out;
  return run_err(ctx, dtype, m, n, A, lda, e, ws, ws_bytes, nullptr);
}

idcur_status idcur_id_col_backward_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, int32_t k,
                                                   int32_t l, int32_t sketched, size_t* bytes) {
  if (!bytes) return IDCUR_EINVAL;
  idcur::BwdArgs b;
  b.k = k;
  b.l = l;
  static const char dummy = 0;
  b.omega = sketched ? &dummy : nullptr;
  return idcur::run_bwd(ctx, dtype, m, n, nullptr, n, b, nullptr, 0, bytes);
}

idcur_status idcur_id_col_backward(idcur_ctx* ctx, int32_t dtype, int64_t m, int64_t n, const void* A, int64_t lda,
                                   const void* omega, int32_t l, const int32_t* J, int32_t k, const void* T,
                                   int64_t ldt, double scale, void* dA, int64_t ldda, void* ws, size_t ws_bytes) {
  idcur::BwdArgs b;
  b.omega = omega; b.l = l; b.J = J; b.k = k; b.T = T; b.ldt = ldt; b.scale = scale; b.dA = dA; b.ldda = ldda;
  return idcur::run_bwd(ctx, dtype, m, n, A, lda, b, ws, ws_bytes, nullptr);
}

idcur_status idcur_id_col_batched_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax,
                                                  int32_t nmax, const idcur_opts* opts, size_t* bytes) {
  if (!bytes) return IDCUR_EINVAL;
  idcur::BatchedCall c{};
  c.nblk = nblk; c.mmax = mmax; c.nmax = nmax;
  return idcur::run_batched(ctx, dtype, c, opts, nullptr, 0, bytes, 0, nullptr);
}

static idcur::BatchedCall batched_call(int32_t nblk, int32_t mmax, int32_t nmax, const int32_t* m, const int32_t* n,
                                       const void* const* A, const int64_t* lda, int32_t* k_out, int32_t* const* J,
                                       void* const* T, const int64_t* ldt) {
  idcur::BatchedCall c{};
  c.nblk = nblk; c.mmax = mmax; c.nmax = nmax;
  c.m = m; c.n = n; c.A = A; c.lda = lda; c.k_out = k_out; c.J = J; c.T = T; c.ldt = ldt;
  return c;
}

idcur_status idcur_id_col_batched(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax, int32_t nmax,
                                  const int32_t* m, const int32_t* n, const void* const* A, const int64_t* lda,
                                  const idcur_opts* opts, void* ws, size_t ws_bytes, int32_t* k_out, int32_t* const* J,
                                  void* const* T, const int64_t* ldt) {
  return idcur::run_batched(ctx, dtype, batched_call(nblk, mmax, nmax, m, n, A, lda, k_out, J, T, ldt), opts, ws,
                            ws_bytes, nullptr, 0, nullptr);
}

idcur_status idcur_id_col_batched_autotune(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax, int32_t nmax,
                                           const int32_t* m, const int32_t* n, const void* const* A,
                                           const int64_t* lda, const idcur_opts* opts, void* ws, size_t ws_bytes,
                                           int32_t* k_out, int32_t* const* J, void* const* T, const int64_t* ldt,
                                           int32_t* variant) {
  int v = -1;
  const idcur_status st = idcur::run_batched(ctx, dtype, batched_call(nblk, mmax, nmax, m, n, A, lda, k_out, J, T, ldt),
                                             opts, ws, ws_bytes, nullptr, 1, &v);
  if (variant) *variant = v;
  return st;
}

idcur_status idcur_id_col_batched_backward_workspace_bytes(idcur_ctx* ctx, int32_t dtype, int32_t nblk,
                                                           int32_t mmax, int32_t nmax, const idcur_opts* opts,
                                                           size_t* bytes) {
  if (!bytes) return IDCUR_EINVAL;
  idcur::BatchedBwdCall c{};
  c.nblk = nblk; c.mmax = mmax; c.nmax = nmax; c.scale = 1.0;
  return idcur::run_batched_bwd(ctx, dtype, c, opts, nullptr, 0, bytes);
}

idcur_status idcur_id_col_batched_backward(idcur_ctx* ctx, int32_t dtype, int32_t nblk, int32_t mmax, int32_t nmax,
                                           const int32_t* m, const int32_t* n, const void* const* A,
                                           const int64_t* lda, const idcur_opts* opts, const int32_t* k,
                                           const int32_t* const* J, const void* const* T, const int64_t* ldt,
                                           double scale, void* const* dA, const int64_t* ldd, void* ws,
                                           size_t ws_bytes) {
  idcur::BatchedBwdCall c{};
  c.nblk = nblk; c.mmax = mmax; c.nmax = nmax;
  c.m = m; c.n = n; c.A = A; c.lda = lda; c.k = k; c.J = J; c.T = T; c.ldt = ldt;
  c.scale = scale; c.dA = dA; c.ldd = ldd;
  return idcur::run_batched_bwd(ctx, dtype, c, opts, ws, ws_bytes, nullptr);
}

idcur_status idcur_id_col_batched_set_variant(idcur_ctx* ctx, int32_t variant) {
  if (!ctx) return IDCUR_EINVAL;
  if (variant < -1 || variant >= idcur::batched_num_variants()) {
    ctx->err = "variant out of range";
    return IDCUR_EINVAL;
  }
  ctx->batched_forced = variant;
  return IDCUR_OK;
}

idcur_status idcur_gaussian(idcur_ctx* ctx, int32_t dtype, int64_t rows, int64_t cols, uint64_t seed, uint64_t stream,
                            void* out, int64_t ldo) {
  if (!ctx) return IDCUR_EINVAL;
  if (dtype != IDCUR_F32 && dtype != IDCUR_F64) { ctx->err = "bad dtype"; return IDCUR_EDTYPE; }
  if (rows < 0 || cols < 0 || ldo < cols || (!out && rows * cols > 0)) { ctx->err = "bad arguments"; return IDCUR_EINVAL; }
  hipError_t e = gaussian_launch(dtype, rows, cols, seed, stream, out, ldo, 1, ctx->stream);
  if (e != hipSuccess) { ctx->err = hipGetErrorString(e); return IDCUR_EHIP; }
  return IDCUR_OK;
}

}  // extern "C"
