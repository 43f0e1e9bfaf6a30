#pragma once
// Truncated column-pivoted Householder QR with the column slab held in
// registers (Section 2.2, eq. (trunc); the k CPQR steps of Algorithms 1 and 4).
//
// One persistent cooperative launch; workgroup g owns a contiguous range of
// columns and keeps them in VGPRs for the whole factorisation:
//  * a column belongs to a group of R consecutive lanes; lane r of the group
//    holds rows r, r + R, r + 2R, ... (RPL slots, zero past the last row);
//  * a group holds NC columns, a workgroup NGR = 256/R groups, so NGR*NC
//    columns;
//  * per step a lane loads its rows of the winning column once (v), forms NC
//    dot products, sums them over the group (DPP row rotations, no LDS) and
//    updates its NC*RPL values in place; rows above the pivot row have v = 0
//    and are left untouched, which keeps the rows of S in place.
// Every group keeps its squared column norms redundantly on all of its lanes;
// keys, totals and thresholds are compared as squares (same order, no square
// roots or divisions on the per-column path).
//
// Exchange (one per step, the grid barrier included): each workgroup publishes
// its best column -- norm key, column index (and, in tolerance mode, its sum
// of squared norms) in a record, and the column's trailing values -- as 64-bit
// words that carry the publish index in their upper half. Thread t of every
// workgroup polls workgroup t's record until all of its words carry the
// expected index, so a writer never waits for its own stores. The winning
// column is then read once per workgroup (one word per thread, staged in LDS)
// together with its exact trailing norm, which the publisher formed after
// posting its record (while the readers were still waiting for the others).
// Every workgroup reduces the records in the same order and so takes the same
// pivot, stopping decision and reflector.
//
// The new row-j entries the norm downdates need come from lane j mod R of each
// group by a DPP row broadcast (v_readlane for R = 64).
//
// Pivots: largest norm, ties to the smallest column index. Householder sign:
// alpha = -sgn(x0)|x|. S is written by original column index; J lists the
// pivots, then the remaining columns in increasing order.
#include <utility>

#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace cr {

constexpr int kRT = 256;
constexpr int kRW = kRT / 64;
constexpr int kRecWords = 8;   // words per record (2 used, 4 in tolerance mode)
// Every record is written in kRep copies; workgroup g reads copy g % kRep (its
// XCD, with round-robin placement), so each hot line serves about G / kRep
// readers instead of G. (Copies of the candidate columns cost more to write than
// they saved.)
constexpr int kRep = 8;

__device__ __forceinline__ uint64_t stamp32(uint32_t s, uint32_t payload) { return ((uint64_t)s << 32) | payload; }

template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  return __hiloint2double(dpp_i<CTRL>(__double2hiint(x)), dpp_i<CTRL>(__double2loint(x)));
}
__device__ __forceinline__ double readlane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}

// DPP controls: rotate right within a row of 16 lanes, permute within quads
constexpr int kRor8 = 0x128, kRor4 = 0x124, kQuadX2 = 0x4E, kQuadX1 = 0xB1;

// Sum over each aligned row of 16 lanes. Partners always hold equal partial
// sums with swapped operands, so every lane of the row ends with the same bits.
__device__ __forceinline__ double sum16(double v) {
  v += dpp_d<kRor8>(v);
  v += dpp_d<kRor4>(v);
  v += dpp_d<kQuadX2>(v);
  v += dpp_d<kQuadX1>(v);
  return v;
}
// Sum over a group of R lanes (16 or 64); the same bits on every lane of the group.
template <int R>
__device__ __forceinline__ double gsum(double v) {
  v = sum16(v);
  if constexpr (R == 64) {
    const double r0 = readlane_d(v, 0), r1 = readlane_d(v, 16), r2 = readlane_d(v, 32), r3 = readlane_d(v, 48);
    v = (r0 + r1) + (r2 + r3);
  }
  return v;
}

// Every lane of each group of R lanes receives lane jr's value (jr uniform):
// a DPP row broadcast for R = 16 (one case per source lane, chosen by a scalar
// branch), v_readlane for R = 64.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, x)));
}
template <int R, int NC, typename T>
__device__ __forceinline__ void group_bcast(const T (&x)[NC], T (&r)[NC], int jr) {
  if constexpr (R == 64) {
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      if constexpr (sizeof(T) == 8) r[u] = readlane_d(x[u], jr);
      else r[u] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x[u]), jr));
    }
  } else {
    switch (jr) {
#define IDCUR_BCAST_CASE(n)                                                          \
  case n:                                                                            \
    _Pragma("unroll") for (int u = 0; u < NC; ++u) {                                 \
      if constexpr (sizeof(T) == 8) r[u] = dpp_d<0x150 + n>(x[u]);                   \
      else r[u] = dpp_f<0x150 + n>(x[u]);                                            \
    }                                                                                \
    break;
      IDCUR_BCAST_CASE(0) IDCUR_BCAST_CASE(1) IDCUR_BCAST_CASE(2) IDCUR_BCAST_CASE(3)
      IDCUR_BCAST_CASE(4) IDCUR_BCAST_CASE(5) IDCUR_BCAST_CASE(6) IDCUR_BCAST_CASE(7)
      IDCUR_BCAST_CASE(8) IDCUR_BCAST_CASE(9) IDCUR_BCAST_CASE(10) IDCUR_BCAST_CASE(11)
      IDCUR_BCAST_CASE(12) IDCUR_BCAST_CASE(13) IDCUR_BCAST_CASE(14) IDCUR_BCAST_CASE(15)
#undef IDCUR_BCAST_CASE
      default:
        break;
    }
  }
}

// candidate: value and column (the owning group or workgroup follows from the
// column: workgroups own contiguous column ranges, groups interleave in them)
struct Cand {
  double v;
  int i;
};
__device__ __forceinline__ void cand_merge(Cand& a, const Cand& b) {
  if (better(b.v, b.i, a.v, a.i)) a = b;
}
template <int CTRL>
__device__ __forceinline__ Cand cand_dpp(const Cand& a) {
  return Cand{dpp_d<CTRL>(a.v), dpp_i<CTRL>(a.i)};
}
__device__ __forceinline__ Cand cand_readlane(const Cand& a, int l) {
  return Cand{readlane_d(a.v, l), __builtin_amdgcn_readlane(a.i, l)};
}
// argmax over each row of 16 lanes; the merge is a total order, so every lane
// of the row ends with the same candidate
__device__ __forceinline__ void cand_row16(Cand& c) {
  cand_merge(c, cand_dpp<kRor8>(c));
  cand_merge(c, cand_dpp<kRor4>(c));
  cand_merge(c, cand_dpp<kQuadX2>(c));
  cand_merge(c, cand_dpp<kQuadX1>(c));
}
// plain sum over each row of 16 lanes (tolerance mode only)
__device__ __forceinline__ void sum_row16(double& s) {
  s += dpp_d<kRor8>(s);
  s += dpp_d<kRor4>(s);
  s += dpp_d<kQuadX2>(s);
  s += dpp_d<kQuadX1>(s);
}
// combine the four rows of the wave in a fixed order (uniform result)
__device__ __forceinline__ void cand_rows(Cand& c) {
  Cand b = cand_readlane(c, 0);
  cand_merge(b, cand_readlane(c, 16));
  cand_merge(b, cand_readlane(c, 32));
  cand_merge(b, cand_readlane(c, 48));
  c = b;
}
__device__ __forceinline__ void sum_rows(double& s) {
  const double s0 = readlane_d(s, 0), s1 = readlane_d(s, 16), s2 = readlane_d(s, 32), s3 = readlane_d(s, 48);
  s = (s0 + s1) + (s2 + s3);
}

// 64-bit words of a value of type T, each stamped with the publish index
template <typename T>
struct Words;
template <>
struct Words<float> {
  static constexpr int N = 1;
  __device__ static void put(uint64_t* w, uint32_t st, float x) { cstore(w, stamp32(st, __float_as_uint(x))); }
  // true when the word carries stamp st; x receives the value
  __device__ static bool get(const uint64_t* w, uint32_t st, float& x) {
    const uint64_t a = cload(w);
    x = __uint_as_float((uint32_t)a);
    return (uint32_t)(a >> 32) == st;
  }
};
template <>
struct Words<double> {
  static constexpr int N = 2;
  __device__ static void put(uint64_t* w, uint32_t st, double x) {
    cstore(w, stamp32(st, (uint32_t)__double2hiint(x)));
    cstore(w + 1, stamp32(st, (uint32_t)__double2loint(x)));
  }
  __device__ static bool get(const uint64_t* w, uint32_t st, double& x) {
    const uint64_t a = cload(w), b = cload(w + 1);
    x = __hiloint2double((int)(uint32_t)a, (int)(uint32_t)b);
    return (uint32_t)(a >> 32) == st && (uint32_t)(b >> 32) == st;
  }
};

// 16 bytes (two stamped words) read coherently across XCDs: a buffer load with
// the sc1 policy, marked volatile so that it is never hoisted out of a polling
// loop. One wide load per record (and per pair of column rows) instead of one
// per word: every workgroup reads every record, and the hot lines serve fewer
// requests.
typedef unsigned cr_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void cload16(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off, uint64_t& w0, uint64_t& w1) {
  const cr_u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)byte_off, 0, (int)(16u | 0x80000000u));
  w0 = ((uint64_t)v[1] << 32) | v[0];
  w1 = ((uint64_t)v[3] << 32) | v[2];
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
// Records: two (tolerance mode: four) words, each with the publish index in its
// top 16 bits: [s | v >> 16], [s | v & 0xffff | column], [s | tot >> 16],
// [s | tot & 0xffff].
__device__ __forceinline__ uint64_t rec_hi(uint32_t s16, uint64_t bits) { return ((uint64_t)s16 << 48) | (bits >> 16); }
__device__ __forceinline__ uint64_t rec_lo(uint32_t s16, uint64_t bits, uint32_t low) {
  return ((uint64_t)s16 << 48) | ((bits & 0xffffull) << 32) | low;
}
__device__ __forceinline__ uint64_t rec_bits(uint64_t hi, uint64_t lo) {
  return ((hi & 0xffffffffffffull) << 16) | ((lo >> 32) & 0xffffull);
}

// x where keep, else +0, without a branch (the compiler may otherwise move a
// load feeding a select into a conditional block with its own wait)
__device__ __forceinline__ float keep_or_zero(float x, bool keep) {
  return __uint_as_float(__float_as_uint(x) & (keep ? 0xffffffffu : 0u));
}
__device__ __forceinline__ double keep_or_zero(double x, bool keep) {
  return __longlong_as_double(__double_as_longlong(x) & (keep ? -1ll : 0ll));
}

template <typename T, int R, int RPL, int NC>
__global__ __launch_bounds__(kRT) void cpqr_reg_kernel(CpqrArgs a) {
  constexpr int NGR = kRT / R;    // column groups per workgroup
  constexpr int GPW = 64 / R;     // column groups per wave
  constexpr int WN = Words<T>::N;
  extern __shared__ __align__(16) unsigned char rsm[];
  // candidate reductions: publish (p_*) and exchange (x_*) use separate arrays,
  // so that a wave entering the next phase cannot overwrite entries another
  // wave is still reading
  __shared__ double p_v[kRW], p_s[kRW], x_v[kRW], x_s[kRW];
  __shared__ int p_i[kRW], x_i[kRW], x_t[kRW];
  __shared__ int s_vfail;   // a thread gave up waiting for the winning column
  __shared__ double s_xnorm;   // the winning column's exact trailing norm
  int* win = reinterpret_cast<int*>(rsm);   // kmax_host pivots
  int* act_s = win + a.kmax_host;           // cols_per_wg flags
  // the winning column by row (R * RPL entries; rows outside [j, l) unused)
  T* vbuf = reinterpret_cast<T*>(rsm + (((size_t)a.kmax_host + a.cols_per_wg) * sizeof(int) + 15) / 16 * 16);

  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int grp = tid / R, rgi = tid % R;
  const int l = a.l_dev ? min(*a.l_dev, a.l_host) : a.l_host;
  const int n = a.n;
  int kmax = a.kmax_dev ? min(*a.kmax_dev, a.kmax_host) : a.kmax_host;
  kmax = min(kmax, min(l, n));
  const int cpw = a.cols_per_wg;
  const int c0 = g * cpw, c1 = min(n, c0 + cpw);
  const T* Y = static_cast<const T*>(a.Y);
  uint64_t* recs = static_cast<uint64_t*>(a.rec);      // [2][G][kRecWords]
  // [2][G][CW]: the candidate column by row (R * RPL * WN words), then the exact
  // norm of its rows at or below the publish index (2 words)
  uint64_t* cvals = static_cast<uint64_t*>(a.cvals);
  constexpr int CW = R * RPL * WN + 2;
  const __amdgpu_buffer_rsrc_t rs_rec = buf_rsrc(a.rec), rs_cv = buf_rsrc(a.cvals);
  static_assert(R * RPL > 0, "");
  const bool exact = a.norms_exact != 0;
  const bool tolmode = a.tol > 0.0;
  const int nwords = tolmode ? 5 : 3;   // record words polled

  T y[NC][RPL];
  double nu2[NC], lim[NC];   // squared norm; recompute threshold tol3z * (squared norm at the last recompute)
  bool act[NC];
  int col[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    col[u] = c0 + u * NGR + grp;
    act[u] = col[u] < c1;
  }
  // ---- load the slab (clamped addresses, masked values) ------------------------
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int64_t cc = max(0, min(col[u], n - 1));
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = rgi + R * t;
      const T val = Y[(int64_t)max(0, min(row, l - 1)) * a.rs + cc * a.cs];
      y[u][t] = keep_or_zero(val, act[u] && row < l);
    }
  }
  // ---- initial norms -------------------------------------------------------------
  {
    double ss[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      ss[u] = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) ss[u] += (double)y[u][t] * (double)y[u][t];
    }
#pragma unroll
    for (int u = 0; u < NC; ++u) nu2[u] = gsum<R>(ss[u]);
  }

  if (tid == 0) s_vfail = 0;
  const double eps = (sizeof(T) == 4) ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  const double tol3z = sqrt(eps);
  double y0fro2 = 0.0, nu0sq = 0.0;
#pragma unroll
  for (int u = 0; u < NC; ++u) lim[u] = tol3z * nu2[u];
  int j = 0;

  // Publish this workgroup's candidate for publish index e (rows [e, l)).
  auto publish = [&](int e) {
    const uint32_t st = (uint32_t)(e + 1);
    // the group's best active column and the group's sum of squared norms
    Cand c{-1.0, 0x7fffffff};
    double ssq = 0.0;
    int bu = -1;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      if (act[u]) {
        ssq += nu2[u];
        if (better(nu2[u], col[u], c.v, c.i)) {
          c.v = nu2[u];
          c.i = col[u];
          bu = u;
        }
      }
    }
    T yb[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      yb[t] = (T)0;
#pragma unroll
      for (int u = 0; u < NC; ++u) yb[t] = (bu == u) ? y[u][t] : yb[t];
    }
    // across the groups of the wave, then across the waves
    if constexpr (GPW > 1) {
      cand_rows(c);
      if (tolmode) sum_rows(ssq);
    }
    if (lane == 0) {
      p_v[wv] = c.v;
      p_i[wv] = c.i;
      p_s[wv] = ssq;
    }
    __syncthreads();
    if (tid == 0) s_vfail = 0;   // read by every thread before this barrier, set only after the next one
    Cand b{p_v[0], p_i[0]};
    double tot = p_s[0];
#pragma unroll
    for (int w = 1; w < kRW; ++w) {
      cand_merge(b, Cand{p_v[w], p_i[w]});
      tot += p_s[w];
    }
    const int par = e & 1;
    const uint32_t s16 = st & 0xffffu;
    if (tid < kRep) {
      uint64_t* r = recs + (((size_t)par * kRep + tid) * G + g) * kRecWords;
      const uint64_t vb = (uint64_t)__double_as_longlong(b.v);
      cstore(r + 0, rec_hi(s16, vb));
      cstore(r + 1, rec_lo(s16, vb, (uint32_t)b.i));
      if (tolmode) {
        const uint64_t tb = (uint64_t)__double_as_longlong(tot);
        cstore(r + 2, rec_hi(s16, tb));
        cstore(r + 3, rec_lo(s16, tb, 0u));
      }
    }
    if (b.i != 0x7fffffff && grp == (b.i - c0) % NGR) {
      uint64_t* dst = cvals + ((size_t)par * G + g) * CW;
      // every slot, by row: readers take rows [e, l) only
#pragma unroll
      for (int t = 0; t < RPL; ++t) Words<T>::put(dst + (size_t)(rgi + R * t) * WN, st, yb[t]);
      // the exact norm of rows [e, l), formed exactly as a reader of the column
      // would form it (same lanes, same order), while the readers still wait
      // for the other records: it leaves the path after the exchange
      double xs = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = rgi + R * t;
        const T q = keep_or_zero(yb[t], row >= e && row < l);
        xs += (double)q * (double)q;
      }
      const double xn = sqrt(gsum<R>(xs));
      if (rgi == 0) Words<double>::put(dst + (size_t)R * RPL * WN, st, xn);
    }
  };

  publish(0);

  bool done = false;
  while (!done) {
    // ---- exchange: every workgroup's record of publish index j -------------------
    const int par = j & 1;
    const uint32_t st = (uint32_t)(j + 1);
    Cand c{-2.0, 0x7fffffff};
    double ssq = 0.0;
    int tmo = 0;
    if (tid < G) {
      const uint32_t off = (uint32_t)((((size_t)par * kRep + g % kRep) * G + tid) * kRecWords * sizeof(uint64_t));
      const uint64_t s16 = st & 0xffffu;
      long spins = 0;
      while (true) {
        uint64_t w0, w1, w2 = s16 << 48, w3 = s16 << 48;
        cload16(rs_rec, off, w0, w1);
        if (tolmode) cload16(rs_rec, off + 16, w2, w3);
        if ((w0 >> 48) == s16 && (w1 >> 48) == s16 && (w2 >> 48) == s16 && (w3 >> 48) == s16) {
          c.v = __longlong_as_double((long long)rec_bits(w0, w1));
          c.i = (int)(uint32_t)w1;
          ssq = tolmode ? __longlong_as_double((long long)rec_bits(w2, w3)) : 0.0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          tmo = 1;
          break;
        }
      }
    }
    cand_row16(c);
    cand_rows(c);
    if (tolmode) {
      sum_row16(ssq);
      sum_rows(ssq);
    }
    const int tmo_w = __any(tmo) ? 1 : 0;
    if (lane == 0) {
      x_v[wv] = c.v;
      x_i[wv] = c.i;
      x_s[wv] = ssq;
      x_t[wv] = tmo_w;
    }
    __syncthreads();
    Cand w{x_v[0], x_i[0]};
    double tot = x_s[0];
    int timed_out = x_t[0];
#pragma unroll
    for (int q = 1; q < kRW; ++q) {
      cand_merge(w, Cand{x_v[q], x_i[q]});
      tot += x_s[q];
      timed_out |= x_t[q];
    }
    if (j == 0) {
      y0fro2 = tot;
      nu0sq = w.v;
    }
    // stopping rules (identical in every workgroup)
    int stop = 0;
    if (timed_out) stop = ST_TIMEOUT;
    else if (!(tot == tot) || !(w.v == w.v) || isinf(tot) || isinf(w.v)) stop = ST_NONFINITE;
    else if (a.tol > 0.0 && tot <= a.tol * a.tol * y0fro2) stop = -1;
    else if (j >= kmax) stop = a.tol > 0.0 ? ST_RANKCAP : -1;
    else if (w.i == 0x7fffffff || w.v <= a.rank_tol * a.rank_tol * nu0sq) stop = -1;
    // ---- the winner's trailing column (rows j..l-1), once per workgroup ----------
    T v[RPL];
    double x0 = 0.0, xnorm = 0.0;
    if (stop == 0) {
      // the owner's slot, 16 bytes per load: two rows of a float column, one row
      // of a double column; the thread with the last index takes the norm
      const uint32_t slot = (uint32_t)(((size_t)par * G + w.i / cpw) * CW * sizeof(uint64_t));
      bool ok = true;
      auto fetch = [&](uint32_t byte_off, uint64_t& a0, uint64_t& a1) {
        long spins = 0;
        while (true) {
          cload16(rs_cv, byte_off, a0, a1);
          if ((uint32_t)(a0 >> 32) == st && (uint32_t)(a1 >> 32) == st) return;
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) {
            ok = false;
            return;
          }
        }
      };
      if (tid == kRT - 1) {
        uint64_t a0, a1;
        fetch(slot + (uint32_t)(R * RPL * WN) * 8u, a0, a1);
        s_xnorm = __hiloint2double((int)(uint32_t)a0, (int)(uint32_t)a1);
      }
      if constexpr (WN == 1) {
        for (int q = (j >> 1) + tid; 2 * q < l; q += kRT) {
          uint64_t a0, a1;
          fetch(slot + (uint32_t)(2 * q) * 8u, a0, a1);
          vbuf[2 * q] = __uint_as_float((uint32_t)a0);
          vbuf[2 * q + 1] = __uint_as_float((uint32_t)a1);
        }
      } else {
        for (int i = j + tid; i < l; i += kRT) {
          uint64_t a0, a1;
          fetch(slot + (uint32_t)(2 * i) * 8u, a0, a1);
          vbuf[i] = (T)__hiloint2double((int)(uint32_t)a0, (int)(uint32_t)a1);
        }
      }
      // every thread either has its words or has given up; agree on the outcome
      if (!ok) s_vfail = 1;
      __syncthreads();
      if (s_vfail) stop = ST_TIMEOUT;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int row = rgi + R * t;
        v[t] = keep_or_zero(vbuf[row], row >= j && row < l);
      }
      x0 = (double)vbuf[j];
      xnorm = s_xnorm;   // exact norm of the trailing column, formed by its publisher
      if (stop == 0 && !(xnorm > 0.0)) stop = -1;
    } else {
#pragma unroll
      for (int t = 0; t < RPL; ++t) v[t] = (T)0;
    }
    if (stop != 0) {
      if (stop > 0 && tid == 0 && (stop == ST_TIMEOUT || g == 0)) set_status(a.status, stop);
      done = true;
      continue;
    }
    const double alpha = (x0 >= 0.0) ? -xnorm : xnorm;
    const double tau = 1.0 / (xnorm * (xnorm + fabs(x0)));
    // pivot row j sits in slot jt of lane jr of every group
    const int jt = __builtin_amdgcn_readfirstlane(j / R), jr = __builtin_amdgcn_readfirstlane(j % R);
    const bool mj = rgi == jr, mg = rgi > jr;
#pragma unroll
    for (int t = 0; t < RPL; ++t)
      if (t == jt && mj) v[t] = (T)(x0 - alpha);
    if (tid == 0) win[j] = w.i;
    // the winner itself becomes (alpha, 0, ..., 0) below row j and leaves the active set
    if (w.i >= c0 && w.i < c1) {
      const int cl = w.i - c0;
      if (grp == cl % NGR) {
#pragma unroll
        for (int u = 0; u < NC; ++u) {
          if (u == cl / NGR) {
            act[u] = false;
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              const int row = rgi + R * t;
              y[u][t] = (row == j) ? (T)alpha : (row > j ? (T)0 : y[u][t]);
            }
          }
        }
      }
    }
    // ---- apply the reflector to the group's columns --------------------------------
    double dot[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) dot[u] = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const double vt = (double)v[t];
#pragma unroll
      for (int u = 0; u < NC; ++u) dot[u] = fma(vt, (double)y[u][t], dot[u]);
    }
    T mw[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const double d = gsum<R>(dot[u]);
      mw[u] = act[u] ? (T)(-tau * d) : (T)0;
    }
    double ss[NC];
    T sj[NC];   // each lane's slot-jt value (row jt R + rgi)
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      ss[u] = 0.0;
      sj[u] = (T)0;
    }
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const bool after = t > jt, at = t == jt;   // the same on every lane
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const T yn = fma(mw[u], v[t], y[u][t]);
        y[u][t] = yn;
        if (exact) {
          const double q = (double)yn;
          ss[u] += after ? q * q : 0.0;
        }
        sj[u] = at ? yn : sj[u];
      }
    }
    // squared norm below row j of column u, summed over the group
    auto below = [&](int u) {
      double q = (double)sj[u];
      double r = mg ? q * q : 0.0;
      if (exact) {
        r += ss[u];
      } else {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          // the empty asm keeps the compiler from computing these squares
          // ahead of the (rarely taken) recompute branch on every step
          T yt = y[u][t];
          asm volatile("" : "+v"(yt));
          const double qq = (double)yt;
          r += (t > jt) ? qq * qq : 0.0;
        }
      }
      return gsum<R>(r);
    };
    if (exact) {
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const double rs = below(u);
        if (act[u]) nu2[u] = rs;
      }
    } else {
      // downdate nu^2 -= s^2 with s the new row-j entry; recompute from the
      // column when the downdate has cancelled below tol3z of the norm^2 at
      // the last recompute
      bool need[NC];
      // the new row-j entry of every column, from lane jr of the group (the
      // value a group sum of it and zeros would give, up to the sign of zero)
      T sb[NC];
      group_bcast<R, NC>(sj, sb, jr);
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const double s = (double)sb[u];
        need[u] = false;
        if (act[u] && nu2[u] > 0.0) {
          const double nn = fmax(0.0, nu2[u] - s * s);
          need[u] = nn <= lim[u];
          nu2[u] = nn;
        }
      }
      // one wave vote per column slot: only the slots some group needs
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        if (__any(need[u])) {
          const double rs = below(u);
          if (need[u]) {
            nu2[u] = rs;
            lim[u] = tol3z * rs;
          }
        }
      }
    }
    ++j;
    done = a.tol <= 0.0 && j >= kmax;   // fixed rank: nothing left to decide
    if (!done) publish(j);
  }

  // ---- epilogue -------------------------------------------------------------------
  const int kout = j;
  if (a.S) {
    T* S = static_cast<T*>(a.S);
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      if (col[u] < c1) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int row = rgi + R * t;
          if (row < kout) S[(int64_t)row * a.ldS + col[u]] = y[u][t];
        }
      }
    }
  }
  if (rgi == 0) {
#pragma unroll
    for (int u = 0; u < NC; ++u) act_s[u * NGR + grp] = act[u] ? 1 : 0;
  }
  __syncthreads();
  const int ncl = max(0, c1 - c0);
  // J: pivots first (workgroup 0), then unselected columns in increasing order
  if (tid == 0) {
    int sel = 0;
    for (int cl = 0; cl < ncl; ++cl) sel += act_s[cl] ? 0 : 1;
    cstore(a.fin + g * 16, sel + 1);
  }
  int before = 0, ftmo = 0;
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
  const int ftmo_w = __any(ftmo) ? 1 : 0;
  // workgroup sum of `before` (integers: any order is exact)
  int bsum = before;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) bsum += __shfl_xor(bsum, o, 64);
  if (lane == 0) {
    x_t[wv] = bsum;
    p_i[wv] = ftmo_w;
  }
  __syncthreads();
  bsum = 0;
  int fin_tmo = 0;
  for (int q = 0; q < kRW; ++q) {
    bsum += x_t[q];
    fin_tmo |= p_i[q];
  }
  if (fin_tmo) {
    // a count never arrived: the positions would be wrong, so leave J alone
    // and report the time-out
    if (tid == 0) set_status(a.status, ST_TIMEOUT);
  } else if (tid == 0) {
    int pos = kout + (c0 - bsum);
    for (int cl = 0; cl < ncl; ++cl)
      if (act_s[cl]) {
        if (pos >= kout && pos < n) a.J[pos] = c0 + cl;
        ++pos;
      }
  }
  if (g == 0) {
    for (int t = tid; t < kout; t += kRT) a.J[t] = win[t];
    if (tid == 0) *a.k_out = kout;
  }
}

struct RegCfg {
  int R, RPL, NC;
};
// searched in order: the first entry that covers l, fits the register budget
// and needs at most one workgroup per compute unit is taken
constexpr RegCfg kRegCfgs[] = {{16, 8, 1}, {16, 16, 1}, {16, 8, 2}, {16, 13, 2}, {16, 14, 2}, {16, 16, 2},
                               {16, 8, 3}, {16, 13, 3}, {16, 14, 3}, {16, 16, 3},
                               {16, 8, 4}, {16, 13, 4}, {16, 14, 4}, {16, 16, 4},
                               {16, 8, 5}, {16, 13, 5}, {16, 14, 5}, {16, 16, 5},
                               {16, 8, 6}, {16, 13, 6}, {16, 14, 6}, {16, 16, 6}, {16, 16, 8},
                               {64, 16, 1}, {64, 16, 2}, {64, 16, 4}, {64, 16, 8},
                               {64, 32, 1}, {64, 32, 2}, {64, 32, 4},
                               // sketch heights up to 528 / 576 rows (e.g. 520 x 20000): the
                               // slab takes up to 180 registers per lane, part of it in AGPRs
                               {16, 33, 3}, {16, 33, 4}, {16, 33, 5},
                               {64, 9, 12}, {64, 9, 16}, {64, 9, 20}};
constexpr int kNumRegCfgs = sizeof(kRegCfgs) / sizeof(kRegCfgs[0]);
// slab registers per lane (4-byte units): FP32 slabs up to 180 (the compiler
// keeps the excess in AGPRs, no scratch), FP64 slabs up to 128
template <typename T>
constexpr int kRegSlabCap = sizeof(T) == 4 ? 180 : 128;

template <typename T, int I>
const void* reg_kernel_ptr() {
  constexpr RegCfg c = kRegCfgs[I];
  if constexpr (c.NC * c.RPL * (int)sizeof(T) / 4 > kRegSlabCap<T>) return nullptr;
  else return (const void*)cpqr_reg_kernel<T, c.R, c.RPL, c.NC>;
}

template <typename T, int... I>
const void* reg_kernel_lookup(int i, std::integer_sequence<int, I...>) {
  const void* p = nullptr;
  ((i == I ? (p = reg_kernel_ptr<T, I>(), 0) : 0), ...);
  return p;
}

}  // namespace cr
}  // namespace idcur
