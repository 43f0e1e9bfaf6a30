// Truncated column-pivoted Householder QR on an l x n matrix Y, as one
// persistent cooperative kernel (Section 2.2, eq. (trunc); the k CPQR steps of
// Algorithms 1 and 4).
//
// Design (gfx950):
//  * Columns are split into G contiguous ranges, one per workgroup (G <= #CUs,
//    all co-resident). A workgroup keeps its columns (its "slab") in LDS for the
//    whole factorisation when they fit, else in a global column-major copy.
//  * Every pivot step needs the global argmax of the remaining column norms.
//    Each workgroup publishes one candidate -- its best column's norm key, the
//    column's trailing values, its exact norm and the workgroup's sum of squared
//    norms -- in a record whose last word carries the step number. Thread t of
//    every workgroup polls record t, so the exchange doubles as the grid
//    barrier: one exchange per step, no atomic read-modify-write.
//  * After the exchange every workgroup holds identical inputs and reduces them
//    in the same order, so all of them take the same pivot, the same stopping
//    decision and the same Householder reflector, without a second round trip.
//  * The reflector is applied to the local columns (dot product, rank-1 update,
//    row j of S), then the norms are downdated (nu^2 -= s^2, recomputed in FP64
//    from the slab when the downdate has cancelled) or recomputed exactly.
//  * Pivots: largest norm, ties to the smallest column index. Householder sign:
//    alpha = -sgn(x0)|x|. Output S is written by original column index; J lists
//    the pivots, then the remaining columns in increasing order.
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace idcur {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

struct Rec {            // one candidate record (4 x 64-bit words)
  uint64_t key;         // bits of the (downdated or exact) norm, double
  uint64_t xnorm;       // bits of the exact norm of the candidate's trailing part
  uint64_t sumsq;       // bits of the workgroup's sum of squared active norms
  uint64_t tag;         // (publish index + 1) << 32 | column (0xffffffff: none)
};

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

template <typename T>
struct Slab {
  T* p;
  int ld;
  __device__ __forceinline__ T& at(int c, int i) const { return p[(size_t)c * ld + i]; }
};

// Block-wide reductions over kThreads threads; every workgroup runs the same
// instruction sequence, so identical inputs give bitwise identical results.
__device__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kWaves; ++i) s += scratch[i];
  return s;
}
__device__ ArgMax block_argmax(ArgMax a, double* sv, int* si) {
  a = wave_argmax(a);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) { sv[w] = a.v; si[w] = a.i; }
  __syncthreads();
  ArgMax b{sv[0], si[0]};
  for (int i = 1; i < kWaves; ++i)
    if (better(sv[i], si[i], b.v, b.i)) { b.v = sv[i]; b.i = si[i]; }
  return b;
}

// Argmax and sum in one pass (one pair of barriers).
__device__ ArgMax block_argmax_sum(ArgMax a, double& s, double* sv, int* si, double* ss) {
  a = wave_argmax(a);
  s = wave_sum(s);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) { sv[w] = a.v; si[w] = a.i; ss[w] = s; }
  __syncthreads();
  ArgMax b{sv[0], si[0]};
  double t = ss[0];
  for (int i = 1; i < kWaves; ++i) {
    if (better(sv[i], si[i], b.v, b.i)) { b.v = sv[i]; b.i = si[i]; }
    t += ss[i];
  }
  s = t;
  return b;
}

template <typename T, bool IN_LDS>
__global__ __launch_bounds__(kThreads) void cpqr_kernel(CpqrArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;

  const int l = a.l_dev ? min(*a.l_dev, a.l_host) : a.l_host;
  const int n = a.n;
  int kmax = a.kmax_dev ? min(*a.kmax_dev, a.kmax_host) : a.kmax_host;
  kmax = min(kmax, min(l, n));
  const int c0 = (int)(((int64_t)g * n) / G), c1 = (int)(((int64_t)(g + 1) * n) / G);
  const int ncl = c1 - c0;
  const int lpad = a.lpad;
  const T* Y = static_cast<const T*>(a.Y);

  // ---- LDS layout --------------------------------------------------------
  unsigned char* sp = smem;
  Slab<T> slab;
  slab.ld = lpad;
  if (IN_LDS) {
    slab.p = reinterpret_cast<T*>(sp);
    sp += (size_t)a.cols_per_wg * lpad * sizeof(T);
  } else {
    slab.p = static_cast<T*>(a.gslab) + (size_t)c0 * lpad;
  }
  T* v = reinterpret_cast<T*>(sp);                 sp += (size_t)lpad * sizeof(T);
  sp = smem + (((sp - smem) + 15) & ~(ptrdiff_t)15);   // offset arithmetic keeps LDS addressing
  double* nu = reinterpret_cast<double*>(sp);      sp += (size_t)a.cols_per_wg * sizeof(double);
  double* nuref = reinterpret_cast<double*>(sp);   sp += (size_t)a.cols_per_wg * sizeof(double);
  double* red = reinterpret_cast<double*>(sp);     sp += 16 * sizeof(double);
  int* act = reinterpret_cast<int*>(sp);           sp += (size_t)a.cols_per_wg * sizeof(int);
  int* redi = reinterpret_cast<int*>(sp);          sp += 16 * sizeof(int);
  int* win = reinterpret_cast<int*>(sp);           // kmax_host ints
  __shared__ int sh_flags[4];                      // stop flag, winner owner, ...
  __shared__ double sh_d[2];

  Rec* recs = reinterpret_cast<Rec*>(a.rec);      // [2][G]
  T* cvals = static_cast<T*>(a.cvals);             // [2][G][lpad]

  // Lanes per column in the update loops (a power of two).
  const int R = a.lanes_per_col;
  const int gpw = 64 / R;                          // column groups per wave
  const int gidx = lane / R, rgi = lane % R;
  const int per_pass = kWaves * gpw;
  const int npass = (ncl + per_pass - 1) / per_pass;
  const T* Ybase = Y;

  // ---- load the slab -------------------------------------------------------
  if (ncl > 0 && l > 0) {
    const int64_t tot = (int64_t)ncl * l;
    if (a.cs == 1) {
      for (int64_t e = tid; e < tot; e += kThreads) {
        const int i = (int)(e / ncl), c = (int)(e % ncl);
        slab.at(c, i) = Ybase[(int64_t)i * a.rs + (int64_t)(c0 + c)];
      }
    } else {
      for (int64_t e = tid; e < tot; e += kThreads) {
        const int c = (int)(e / l), i = (int)(e % l);
        slab.at(c, i) = Ybase[(int64_t)i * a.rs + (int64_t)(c0 + c) * a.cs];
      }
    }
  }
  for (int c = tid; c < a.cols_per_wg; c += kThreads) act[c] = (c < ncl) ? 1 : 0;
  __syncthreads();

  // ---- initial norms -------------------------------------------------------
  for (int pass = 0; pass < npass; ++pass) {
    const int cl = pass * per_pass + wv * gpw + gidx;
    const bool valid = cl < ncl;
    double ss = 0.0;
    if (valid)
      for (int i = rgi; i < l; i += R) { const double y = (double)slab.at(cl, i); ss += y * y; }
    ss = group_sum(ss, R);
    if (valid && rgi == 0) { nu[cl] = sqrt(ss); nuref[cl] = nu[cl]; }
  }
  __syncthreads();

  const double eps = (sizeof(T) == 4) ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  const double tol3z = sqrt(eps);
  double y0fro2 = 0.0, nu0 = 0.0;
  int j = 0;
  bool timed_out = false;

  // Publish this workgroup's candidate for publish index e (rows [rb, l)):
  // all data words first, one wait for their completion, then the tag.
  auto publish = [&](int e, int rb, bool norms_exact) {
    ArgMax best{-1.0, 0x7fffffff};
    double ssq = 0.0;
    for (int c = tid; c < ncl; c += kThreads) {
      if (act[c]) {
        ssq += nu[c] * nu[c];
        if (better(nu[c], c0 + c, best.v, best.i)) { best.v = nu[c]; best.i = c0 + c; }
      }
    }
    best = block_argmax_sum(best, ssq, red, redi, red + 8);
    const int par = e & 1;
    const int cb = best.i - c0;
    double xnorm = best.v;
    if (!norms_exact && best.i != 0x7fffffff) {
      // the key is a downdated norm: the reflector needs the exact one
      double xs = 0.0;
      for (int i = rb + tid; i < l; i += kThreads) {
        const double y = (double)slab.at(cb, i);
        xs += y * y;
      }
      xnorm = sqrt(block_sum(xs, red + 12));
    }
    T* dst = cvals + ((size_t)par * G + g) * lpad;
    if (best.i != 0x7fffffff)
      for (int i = rb + tid; i < l; i += kThreads) cstore(dst + (i - rb), slab.at(cb, i));
    Rec* r = recs + (size_t)par * G + g;
    if (tid == 0) {
      cstore(&r->key, dbits(best.v));
      cstore(&r->xnorm, dbits(xnorm));
      cstore(&r->sumsq, dbits(ssq));
    }
    wait_all_mem();
    __syncthreads();
    if (tid == 0) cstore(&r->tag, ((uint64_t)(e + 1) << 32) | (uint32_t)best.i);
  };

  publish(0, 0, true);

  while (true) {
    // ---- exchange: read every workgroup's record of publish index j ------
    const int par = j & 1;
    ArgMax cand{-2.0, 0x7fffffff};
    double ssq = 0.0;
    if (tid < G) {
      const Rec* r = recs + (size_t)par * G + tid;
      const uint64_t want = (uint64_t)(j + 1);
      long spins = 0;
      uint64_t tag = cload(&r->tag);
      while ((tag >> 32) != want) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) { timed_out = true; break; }
        tag = cload(&r->tag);
      }
      if (!timed_out) {
        cand.v = bitsd(cload(&r->key));
        cand.i = (int)(uint32_t)(tag & 0xffffffffu);
        ssq = bitsd(cload(&r->sumsq));
      }
    }
    if (tid == 0) sh_flags[0] = 0;
    __syncthreads();
    if (timed_out) sh_flags[0] = 1;
    // owner of the best candidate = the thread index that holds it
    double tot = ssq;
    const ArgMax w = block_argmax_sum(cand, tot, red, redi, red + 8);
    if (cand.i == w.i && tid < G && w.i != 0x7fffffff) sh_flags[1] = tid;
    __syncthreads();
    if (sh_flags[0]) {
      if (tid == 0) set_status(a.status, ST_TIMEOUT);
      break;
    }
    const int wowner = sh_flags[1];
    if (j == 0) { y0fro2 = tot; nu0 = w.v; }
    // stopping rules (identical in every workgroup)
    if (!(tot == tot) || !(w.v == w.v) || isinf(tot) || isinf(w.v)) {
      if (g == 0 && tid == 0) set_status(a.status, ST_NONFINITE);
      break;
    }
    if (a.tol > 0.0 && tot <= a.tol * a.tol * y0fro2) break;
    if (j >= kmax) {
      if (a.tol > 0.0 && g == 0 && tid == 0) set_status(a.status, ST_RANKCAP);
      break;
    }
    if (w.i == 0x7fffffff || w.v <= a.rank_tol * nu0) break;
    // winner's exact norm and trailing column, loaded together
    const Rec* wr = recs + (size_t)par * G + wowner;
    const T* src = cvals + ((size_t)par * G + wowner) * lpad;
    const int len = l - j;
    if (tid == 0) sh_d[0] = bitsd(cload(&wr->xnorm));
    for (int i = tid; i < len; i += kThreads) v[i] = cload(src + i);
    __syncthreads();
    const double xnorm = sh_d[0];
    if (!(xnorm > 0.0)) break;
    const double x0 = (double)v[0];
    const double alpha = (x0 >= 0.0) ? -xnorm : xnorm;
    const double tau = 1.0 / (xnorm * (xnorm + fabs(x0)));
    __syncthreads();
    if (tid == 0) {
      v[0] = (T)(x0 - alpha);
      win[j] = w.i;
    }
    if (w.i >= c0 && w.i < c1) {
      const int cw = w.i - c0;
      if (tid == 0) act[cw] = 0;
      for (int i = j + tid; i < l; i += kThreads) slab.at(cw, i) = (i == j) ? (T)alpha : (T)0;
    }
    __syncthreads();

    // ---- apply the reflector to the local active columns -----------------
    for (int pass = 0; pass < npass; ++pass) {
      const int cl = pass * per_pass + wv * gpw + gidx;
      const bool valid = cl < ncl && act[cl];
      double dot = 0.0;
      if (valid) {
        // unrolled so that several LDS reads are in flight (independent sums)
        double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
        int i = j + rgi;
        for (; i + 3 * R < l; i += 4 * R) {
          d0 += (double)v[i - j] * (double)slab.at(cl, i);
          d1 += (double)v[i + R - j] * (double)slab.at(cl, i + R);
          d2 += (double)v[i + 2 * R - j] * (double)slab.at(cl, i + 2 * R);
          d3 += (double)v[i + 3 * R - j] * (double)slab.at(cl, i + 3 * R);
        }
        for (; i < l; i += R) d0 += (double)v[i - j] * (double)slab.at(cl, i);
        dot = (d0 + d1) + (d2 + d3);
      }
      dot = group_sum(dot, R);
      const double wgt = tau * dot;
      double ss = 0.0, s_own = 0.0;
      if (valid) {
        int i = j + rgi;
        if (rgi == 0) {   // row j: the entry of S
          const T y = (T)((double)slab.at(cl, i) - wgt * (double)v[0]);
          slab.at(cl, i) = y;
          s_own = (double)y;
          i += R;
        }
        double s0 = 0.0, s1 = 0.0;
        for (; i + R < l; i += 2 * R) {
          const double a0 = (double)slab.at(cl, i), a1 = (double)slab.at(cl, i + R);
          const double b0 = (double)v[i - j], b1 = (double)v[i + R - j];
          const T y0 = (T)(a0 - wgt * b0), y1 = (T)(a1 - wgt * b1);
          slab.at(cl, i) = y0;
          slab.at(cl, i + R) = y1;
          s0 += (double)y0 * (double)y0;
          s1 += (double)y1 * (double)y1;
        }
        for (; i < l; i += R) {
          const T y = (T)((double)slab.at(cl, i) - wgt * (double)v[i - j]);
          slab.at(cl, i) = y;
          s0 += (double)y * (double)y;
        }
        if (a.norms_exact) ss = s0 + s1;
      }
      // row j of S for this column: held by the group's first lane
      const double s = __shfl(s_own, (lane / R) * R, 64);
      if (a.norms_exact) {
        ss = group_sum(ss, R);
        if (valid && rgi == 0) { nu[cl] = sqrt(ss); nuref[cl] = nu[cl]; }
      } else {
        // downdate nu^2 -= s^2; recompute when it has cancelled
        bool need = false;
        double t1 = 0.0;
        if (valid) {
          const double nc = nu[cl];
          if (nc > 0.0) {
            const double r = fabs(s) / nc;
            t1 = fmax(0.0, (1.0 + r) * (1.0 - r));
            const double q = nc / nuref[cl];
            need = (t1 * q * q) <= tol3z;
          }
        }
        if (__any(need)) {
          // each lane re-reads only the rows it has just written
          double rs = 0.0;
          if (need)
            for (int i = j + rgi; i < l; i += R)
              if (i > j) { const double y = (double)slab.at(cl, i); rs += y * y; }
          rs = group_sum(rs, R);
          if (need && rgi == 0) { nu[cl] = sqrt(rs); nuref[cl] = nu[cl]; }
        }
        if (valid && !need && rgi == 0) nu[cl] = nu[cl] * sqrt(t1);
      }
    }
    __syncthreads();
    ++j;
    if (a.tol <= 0.0 && j >= kmax) break;   // fixed rank: nothing left to decide
    publish(j, j, a.norms_exact != 0);
  }

  // ---- epilogue -------------------------------------------------------------
  const int kout = j;
  __syncthreads();
  // rows of S for the local columns, by original column index
  if (a.S) {
    T* S = static_cast<T*>(a.S);
    const int64_t tot = (int64_t)kout * ncl;
    for (int64_t e = tid; e < tot; e += kThreads) {
      const int r = (int)(e / ncl), c = (int)(e % ncl);
      S[(int64_t)r * a.ldS + c0 + c] = slab.at(c, r);
    }
  }
  // J: pivots first (workgroup 0), then unselected columns in increasing order
  if (tid == 0) {
    int sel = 0;
    for (int c = 0; c < ncl; ++c) sel += act[c] ? 0 : 1;
    sh_flags[2] = sel;
    cstore(a.fin + g * 16, sel + 1);
  }
  __syncthreads();
  int before = 0, ftmo = 0;
  if (tid == 0) sh_flags[3] = 0;
  __syncthreads();
  if (tid < g) {
    long spins = 0;
    int vfin = cload(a.fin + tid * 16);
    while (vfin == 0) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) { ftmo = 1; break; }
      vfin = cload(a.fin + tid * 16);
    }
    before = vfin > 0 ? vfin - 1 : 0;
  }
  if (ftmo) atomicOr(&sh_flags[3], 1);
  const double bsum = block_sum((double)before, red);
  if (sh_flags[3]) {
    // a count never arrived: the positions would be wrong, so leave J alone
    // and report the time-out
    if (tid == 0) set_status(a.status, ST_TIMEOUT);
  } else if (tid == 0) {
    int pos = kout + (c0 - (int)bsum);
    for (int c = 0; c < ncl; ++c)
      if (act[c]) {
        if (pos >= kout && pos < n) a.J[pos] = c0 + c;
        ++pos;
      }
  }
  if (g == 0) {
    for (int t = tid; t < kout; t += kThreads) a.J[t] = win[t];
    if (tid == 0) *a.k_out = kout;
  }
}

}  // namespace

template <typename T>
static size_t cpqr_lds_bytes(int cols_per_wg, int lpad, int kmax, bool in_lds) {
  size_t b = 0;
  if (in_lds) b += (size_t)cols_per_wg * lpad * sizeof(T);
  b += (size_t)lpad * sizeof(T);
  b = (b + 15) & ~(size_t)15;
  b += 2 * (size_t)cols_per_wg * sizeof(double) + 16 * sizeof(double);
  b += (size_t)cols_per_wg * sizeof(int) + 16 * sizeof(int);
  b += (size_t)kmax * sizeof(int);
  return b;
}

// Kernel choice: the register-slab kernel when the columns fit in the
// registers of at most one workgroup per CU, else (FP32) the on-chip-slab
// kernel when they fit in registers and LDS, else the blocked kernel (short
// form when its panel of reflectors fits in LDS, else tall), else the
// unblocked slab kernel below. IDCUR_CPQR_SLAB selects a kernel for testing:
// 1 the blocked kernel (its own form), 2 its tall form, 3 the unblocked one;
// IDCUR_CPQR_RESCFG=i the on-chip-slab kernel's configuration i.
CpqrPlan cpqr_plan(int dtype_size, int l, int n, int kmax, int num_cus) {
  CpqrPlan p{};
  p.reg_cfg = -1;
  p.res_cfg = -1;
  const char* fs = getenv("IDCUR_CPQR_SLAB");
  const int force = (fs && fs[0] >= '1' && fs[0] <= '3') ? fs[0] - '0' : 0;
  if (force == 0) {
    int G = 0, cpw = 0;
    const int cfg = cpqr_res_forced() ? -1 : cpqr_reg_pick(dtype_size, l, n, num_cus, &G, &cpw);
    if (cfg >= 0) {
      p.reg_cfg = cfg;
      p.G = G;
      p.cols_per_wg = cpw;
      p.lpad = (int)round_up(std::max(l, 1), 4);
      p.lanes_per_col = 0;
      p.in_lds = true;
      p.lds_bytes = cpqr_reg_lds_bytes(cfg, kmax, cpw, dtype_size);
      p.rec_bytes = cpqr_reg_rec_bytes(p.G);
      p.cvals_bytes = cpqr_reg_cvals_bytes(cfg, p.G, dtype_size);
      p.fin_bytes = (size_t)p.G * 16 * sizeof(int);
      p.gslab_bytes = 0;
      return p;
    }
    const int rcfg = cpqr_res_pick(dtype_size, l, n, kmax, num_cus, &G, &cpw);
    if (rcfg >= 0) {
      p.res_cfg = rcfg;
      p.G = G;
      p.cols_per_wg = cpw;
      p.lpad = (int)round_up(std::max(l, 1), 4);
      p.lanes_per_col = 0;
      p.in_lds = true;
      p.lds_bytes = cpqr_res_lds_bytes(rcfg, kmax, cpw);
      p.rec_bytes = cpqr_reg_rec_bytes(p.G);
      p.cvals_bytes = cpqr_res_cvals_bytes(rcfg, p.G);
      p.fin_bytes = (size_t)p.G * 16 * sizeof(int);
      p.gslab_bytes = 0;
      return p;
    }
  }
  if (force != 3) {
    CpqrPlan b = p;
    if (cpqr_blk_plan(b, dtype_size, l, n, kmax, num_cus, force == 2 ? 2 : 0) > 0) return b;
  }
  p.blk = 0;
  p.G = (int)std::max(1, std::min(num_cus, n));
  p.cols_per_wg = (int)ceil_div(n, p.G);
  p.lpad = (int)round_up(std::max(l, 1), 4) + (dtype_size == 4 ? 1 : 0);
  const size_t budget = 150 * 1024;
  const size_t need = dtype_size == 4 ? cpqr_lds_bytes<float>(p.cols_per_wg, p.lpad, kmax, true)
                                      : cpqr_lds_bytes<double>(p.cols_per_wg, p.lpad, kmax, true);
  p.in_lds = need <= budget;
  p.lds_bytes = p.in_lds ? need
                         : (dtype_size == 4 ? cpqr_lds_bytes<float>(p.cols_per_wg, p.lpad, kmax, false)
                                            : cpqr_lds_bytes<double>(p.cols_per_wg, p.lpad, kmax, false));
  // lanes per column: enough column groups to keep all lanes busy
  int R = 1;
  while (R < 64 && (int64_t)(kThreads / (R * 2)) >= p.cols_per_wg) R *= 2;
  while (R < 64 && l / R > 48) R *= 2;
  p.lanes_per_col = R;
  p.rec_bytes = 2 * (size_t)p.G * sizeof(Rec);
  p.cvals_bytes = 2 * (size_t)p.G * p.lpad * dtype_size;
  p.fin_bytes = (size_t)p.G * 16 * sizeof(int);
  p.gslab_bytes = p.in_lds ? 0 : (size_t)n * p.lpad * dtype_size;
  return p;
}

hipError_t cpqr_launch(int dtype, const CpqrPlan& p, CpqrArgs a, hipStream_t stream) {
  a.lpad = p.lpad;
  a.cols_per_wg = p.cols_per_wg;
  a.lanes_per_col = p.lanes_per_col;
  if (p.blk > 0) return cpqr_blk_launch(dtype, p, a, stream);
  if (p.res_cfg >= 0) {
    hipError_t e = zero_launch(a.cvals, p.cvals_bytes, stream);
    if (e != hipSuccess) return e;
    return cpqr_res_launch(p.res_cfg, p.G, a, p.lds_bytes, stream);
  }
  if (p.reg_cfg >= 0) {
    // exchanged words carry the publish index: clear what an earlier call left
    hipError_t e = zero_launch(a.cvals, p.cvals_bytes, stream);
    if (e != hipSuccess) return e;
    return cpqr_reg_launch(dtype, p.reg_cfg, p.G, a, p.lds_bytes, stream);
  }
  void* args[] = {&a};
  const void* fn;
  if (dtype == 0) fn = p.in_lds ? (const void*)cpqr_kernel<double, true> : (const void*)cpqr_kernel<double, false>;
  else fn = p.in_lds ? (const void*)cpqr_kernel<float, true> : (const void*)cpqr_kernel<float, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel(fn, dim3(p.G), dim3(kThreads), args, (unsigned)p.lds_bytes, stream);
}

}  // namespace idcur
