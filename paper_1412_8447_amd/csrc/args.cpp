// Argument checks of the C ABI (no GPU calls; see args.hpp).
#include "args.hpp"

#include <algorithm>
#include <cmath>

namespace idcur {

namespace {
constexpr ArgCheck kOk{IDCUR_OK, nullptr};
constexpr ArgCheck inval(const char* m) { return ArgCheck{IDCUR_EINVAL, m}; }
constexpr ArgCheck dtype_err(const char* m) { return ArgCheck{IDCUR_EDTYPE, m}; }
}  // namespace

ArgCheck check_id_args(int op, int dtype, int64_t m, int64_t n, int64_t lda, const idcur_opts* opts) {
  if (!opts) return inval("opts is NULL");
  if (dtype != IDCUR_F32 && dtype != IDCUR_F64) return dtype_err("dtype must be IDCUR_F32 or IDCUR_F64");
  if (opts->prec != IDCUR_PREC_NATIVE && opts->prec != IDCUR_PREC_BF16 && opts->prec != IDCUR_PREC_FP16)
    return inval("unknown precision");
  if (opts->prec != IDCUR_PREC_NATIVE && dtype != IDCUR_F32) return dtype_err("BF16 / FP16 sketches take FP32 data");
  if (op < OP_COL || op > OP_SKETCH_ROW) return inval("unknown op");
  if (m <= 0 || n <= 0) return inval("m and n must be positive");
  if (m > (1LL << 30) || n > (1LL << 30)) return inval("m and n must be below 2^30");
  if (lda < n) return inval("lda must be >= n");
  const bool rowop = op == OP_ROW || op == OP_SKETCH_ROW;
  const int64_t mr = rowop ? n : m;   // rows of the sketched view
  const int64_t mn = std::min(m, n);
  if (opts->k < 0) return inval("k must be >= 0");
  if (opts->k > 0) {
    if (opts->k >= mn) return inval("k must be < min(m, n)");
  } else {
    if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) return inval("tolerance mode needs tol > 0");
    if (opts->kmax <= 0 || opts->kmax >= mn) return inval("tolerance mode needs 0 < kmax < min(m, n)");
  }
  const int kcap = opts->k > 0 ? opts->k : opts->kmax;
  if (opts->q < 0) return inval("q must be >= 0");
  if (kcap > kMaxRank || (opts->p >= 0 && (int64_t)kcap + opts->p > kMaxRank))
    return inval("k (kmax) and k + p must be <= 4096");
  if ((op == OP_SKETCH || op == OP_SKETCH_ROW) && !(opts->p >= 0 && (int64_t)kcap + opts->p < mr))
    return inval("a sketch needs p >= 0 and k + p below the sketched dimension");
  if (opts->rank_tol < 0 || !std::isfinite(opts->rank_tol)) return inval("rank_tol must be >= 0");
  if (opts->norms != IDCUR_NORMS_DOWNDATE && opts->norms != IDCUR_NORMS_EXACT) return inval("bad norms");
  if (opts->sketch != IDCUR_SKETCH_GAUSSIAN && opts->sketch != IDCUR_SKETCH_SRHT) return inval("unknown sketch kind");
  if (opts->u_correct != 0 && opts->u_correct != 1) return inval("u_correct must be 0 or 1");
  if (!(opts->t_reg >= 0.0 && opts->t_reg < 1.0)) return inval("t_reg must be in [0, 1)");
  if (!(opts->t_svd >= 0.0 && opts->t_svd < 1.0)) return inval("t_svd must be in [0, 1)");
  if (opts->t_reg > 0.0 && opts->t_svd > 0.0) return inval("t_reg and t_svd exclude each other");
  // the truncated-SVD path is switched off: a GPU run that included it ended
  // with a device fault whose cause is not shown
  if (opts->t_svd > 0.0) return inval("t_svd is switched off in this build");
  if (opts->sketch == IDCUR_SKETCH_SRHT && opts->p >= 0 && (int64_t)kcap + opts->p < mr) {
    if (opts->q != 0) return inval("the structured sketch takes no power steps (q = 0)");
    if (opts->prec != IDCUR_PREC_NATIVE) return dtype_err("the structured sketch runs in the native precision");
    if (opts->omega) return inval("omega and the structured sketch exclude each other");
    if (!opts->srht_rows || !opts->srht_signs) return inval("srht_rows and srht_signs are required");
    if ((int64_t)kcap + opts->p > kSrhtMaxRowsArg) return inval("k (kmax) + p must be <= 512 for the structured sketch");
  }
  return kOk;
}

ArgCheck check_id_outs(int op, int64_t m, int64_t n, const void* A, const idcur_opts& opts, const Outs& out) {
  if (!A) return inval("A is NULL");
  const int kcap = opts.k > 0 ? opts.k : opts.kmax;
  const int64_t nc = op == OP_ROW ? m : n;
  if (op == OP_SKETCH || op == OP_SKETCH_ROW) {
    if (!out.Yt) return inval("Yt is NULL");
    if (out.ldy < kcap + opts.p) return inval("ldy too small");
    return kOk;
  }
  if (!out.k_out) return inval("k_out is NULL");
  if (op == OP_ROW) {
    if (!out.I || !out.Tr) return inval("I and Tr are required");
    if (out.ldtr < (opts.k > 0 ? m - kcap : m)) return inval("ldtr too small");
    return kOk;
  }
  if (!out.J) return inval("J is required");
  if (op != OP_CUR) {
    if (!out.T) return inval("T is required");
    if (out.ldt < (opts.k > 0 ? nc - kcap : nc)) return inval("ldt too small");
  }
  if (op == OP_TWO) {
    if (!out.I || !out.Tr) return inval("I and Tr are required");
    if (out.ldtr < (opts.k > 0 ? m - kcap : m)) return inval("ldtr too small");
  }
  if (op == OP_CUR) {
    if (!out.I || !out.U) return inval("I and U are required");
    if (out.ldu < kcap) return inval("ldu too small");
    if (out.C && out.ldc < kcap) return inval("ldc too small");
    if (out.R && out.ldr < n) return inval("ldr too small");
  }
  return kOk;
}

ArgCheck check_batched_args(int dtype, int nblk, int mmax, int nmax, const idcur_opts* o, int max_width,
                            int max_sketch) {
  if (!o) return inval("opts is NULL");
  if (dtype != IDCUR_F32) return dtype_err("the batched ID takes FP32 blocks");
  if (o->prec != IDCUR_PREC_NATIVE) return dtype_err("the batched ID sketches in FP32");
  if (nblk < 0 || nblk > (1 << 20)) return inval("nblk must be in [0, 2^20]");
  if (mmax < 1 || mmax > (1 << 24)) return inval("mmax must be in [1, 2^24]");
  if (nmax < 1 || nmax > max_width) return inval("nmax must be in [1, 512]");
  if (o->p < 1) return inval("the batched ID needs oversampling p >= 1");
  if (o->q != 0) return inval("the batched ID takes no power steps (q = 0)");
  if (o->k < 0) return inval("k must be >= 0");
  if (o->k == 0) {
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return inval("tolerance mode needs tol > 0");
    if (o->kmax < 1) return inval("tolerance mode needs kmax >= 1");
  }
  const int kcap = o->k > 0 ? o->k : o->kmax;
  if ((int64_t)kcap + o->p > max_sketch) return inval("k (kmax) + p must be <= 64");
  if (o->rank_tol < 0 || !std::isfinite(o->rank_tol)) return inval("rank_tol must be >= 0");
  if (o->t_reg != 0.0 || o->t_svd != 0.0)
    return inval("the batched ID forms T by back-substitution (t_reg = t_svd = 0)");
  return kOk;
}

}  // namespace idcur
