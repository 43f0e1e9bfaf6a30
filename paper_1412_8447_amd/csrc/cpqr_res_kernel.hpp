#pragma once
// Truncated column-pivoted Householder QR with the column slab resident on chip,
// part in registers and part in LDS (Section 2.2, eq. (trunc); the k CPQR steps
// of Algorithms 1 and 4), for FP32 matrices of at most 16 RPL rows whose
// columns do not fit in registers alone: the 500 x 50000 transposed C of a
// rank-500 row ID is 100 MB, about four fifths of all register files.
//
// The algorithm, the exchange and the arithmetic are those of the register-slab
// kernel (cpqr_reg_kernel.hpp) with R = 16 lanes per column:
//  * a group of 16 lanes holds NC columns in registers and NL more in LDS, where
//    lane r of the group owns rows r, r + 16, ... of each (RPL slots); the LDS
//    slots are laid out thread-major, so that a wave reads 64 consecutive words
//    and no thread ever touches another's entries (no barrier guards them);
//  * slots wholly above the pivot row see a zero reflector and are skipped by a
//    scalar branch: the zero products they would add change no bit of the dot
//    products, norms or entries, so the results equal the register-slab
//    kernel's for the same matrix (the same pivots, S and J in fixed-rank mode);
//  * the reflector is read from LDS slot by slot instead of being held in
//    registers, the squared norms and recompute thresholds of the columns sit in
//    LDS (one entry per group and slot, written with the same bits by all of the
//    group's lanes), and the publishing group picks its candidate column by a
//    scalar branch on its slot.
#include "cpqr_reg_kernel.hpp"

namespace idcur {
namespace cr {

// NTH threads per workgroup (256: one wave per SIMD, the register slots may
// spill into AGPRs; 512: two waves per SIMD, so that one wave's LDS and
// exchange latencies overlap the other's arithmetic). EXACT: the exact-norm
// mode (norms recomputed every step), a template parameter so that the
// default mode carries no per-slot norm accumulators.
template <int NTH, int RPL, int NC, int NL, bool EXACT>
__global__ __launch_bounds__(NTH) void cpqr_res_kernel(CpqrArgs a) {
  using T = float;
  constexpr int R = 16;
  constexpr int NWV = NTH / 64;   // waves
  constexpr int NGR = NTH / R;   // column groups per workgroup
  constexpr int NT = NC + NL;    // column slots per group
  static_assert(NC > 0 && NL >= 0, "");
  extern __shared__ __align__(16) unsigned char rsm[];
  __shared__ double p_v[NWV], p_s[NWV], x_v[NWV], x_s[NWV];
  __shared__ int p_i[NWV], x_i[NWV], x_t[NWV];
  __shared__ int s_vfail;
  __shared__ double s_xnorm;
  // dynamic LDS, by byte offset: the winning column by row (R RPL words), the
  // squared norms and recompute thresholds by slot and group (NT x NGR doubles
  // each), the pivots (kmax_host), the column flags (cols_per_wg), then the LDS
  // slots of the slab (NL x RPL x NTH words, thread-major, from yoff). Every
  // access is a byte offset from rsm, so that it stays an LDS access with the
  // constant part in the instruction's offset field.
  constexpr uint32_t kNuOff = R * RPL * 4;
  constexpr uint32_t kLimOff = kNuOff + NT * NGR * 8;
  constexpr uint32_t kWinOff = kLimOff + NT * NGR * 8;
  auto f_at = [&](uint32_t off) -> float& { return *reinterpret_cast<float*>(rsm + off); };
  auto d_at = [&](uint32_t off) -> double& { return *reinterpret_cast<double*>(rsm + off); };
  int* win = reinterpret_cast<int*>(rsm + kWinOff);
  int* act_s = win + a.kmax_host;
  const uint32_t yoff = (kWinOff + 4u * (uint32_t)(a.kmax_host + a.cols_per_wg) + 15u) & ~15u;
  constexpr uint32_t kSlotBytes = RPL * NTH * 4;

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
  uint64_t* recs = static_cast<uint64_t*>(a.rec);   // [2][kRep][G][kRecWords]
  // [2][G][CW]: the candidate column by row, then the exact norm of its rows at
  // or below the publish index (2 words)
  uint64_t* cvals = static_cast<uint64_t*>(a.cvals);
  constexpr int CW = R * RPL + 2;
  const __amdgpu_buffer_rsrc_t rs_rec = buf_rsrc(a.rec), rs_cv = buf_rsrc(a.cvals);
  const bool tolmode = a.tol > 0.0;

  T y[NC][RPL];
  // this thread's entry of LDS slot 0; passed through an empty asm once per
  // step, so that the compiler forms each slot's address from it inside the
  // step instead of keeping RPL NL precomputed addresses live across the loop
  uint32_t ybase = yoff + 4u * (uint32_t)tid;
  // slot u, row slot t of this lane (u and t are constants once unrolled)
  auto yget = [&](int u, int t) -> T {
    if (u < NC) return y[u < NC ? u : 0][t];
    return f_at(ybase + (uint32_t)(u - NC) * kSlotBytes + (uint32_t)t * (NTH * 4));
  };
  auto yset = [&](int u, int t, T v) {
    if (u < NC) y[u < NC ? u : 0][t] = v;
    else f_at(ybase + (uint32_t)(u - NC) * kSlotBytes + (uint32_t)t * (NTH * 4)) = v;
  };

  // column of slot u; its squared norm, recompute threshold and active flag
  auto col = [&](int u) { return c0 + u * NGR + grp; };
  auto nu2 = [&](int u) -> double& { return d_at(kNuOff + 8u * (uint32_t)(u * NGR + grp)); };
  auto lim = [&](int u) -> double& { return d_at(kLimOff + 8u * (uint32_t)(u * NGR + grp)); };
  uint32_t actb = 0;
#pragma unroll
  for (int u = 0; u < NT; ++u) actb |= (col(u) < c1 ? 1u : 0u) << u;
  auto act = [&](int u) { return ((actb >> u) & 1u) != 0; };
  // ---- load the slab (clamped addresses, masked values) ------------------------
  // LDS slots first, one at a time (the empty asm with a memory clobber keeps
  // the compiler from issuing every load of the slab before the first store)
  auto load_slot = [&](int u) {
    const int64_t cc = max(0, min(col(u), n - 1));
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int row = rgi + R * t;
      const T val = Y[(int64_t)max(0, min(row, l - 1)) * a.rs + cc * a.cs];
      yset(u, t, keep_or_zero(val, act(u) && row < l));
    }
  };
#pragma unroll
  for (int u = NC; u < NT; ++u) {
    load_slot(u);
    asm volatile("" ::: "memory");
  }
#pragma unroll
  for (int u = 0; u < NC; ++u) load_slot(u);
  // ---- initial norms -------------------------------------------------------------
  const double eps = 5.9604644775390625e-08;
  const double tol3z = sqrt(eps);
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    double ss = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const double q = (double)yget(u, t);
      ss += q * q;
    }
    const double s2 = gsum<R>(ss);
    nu2(u) = s2;
    lim(u) = tol3z * s2;
    asm volatile("" ::: "memory");
  }

  // the staged winning column: rows at or past l stay zero (the slab holds
  // zeros there and publishers copy them), so reads of it need no row mask
  for (int r = tid; r < R * RPL; r += NTH) f_at(4u * (uint32_t)r) = 0.0f;
  if (tid == 0) s_vfail = 0;
  double y0fro2 = 0.0, nu0sq = 0.0;
  int j = 0;

  // Publish this workgroup's candidate for publish index e (rows [e, l)).
  auto publish = [&](int e) {
    const uint32_t st = (uint32_t)(e + 1);
    Cand c{-1.0, 0x7fffffff};
    double ssq = 0.0;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      if (act(u)) {
        const double v = nu2(u);
        ssq += v;
        if (better(v, col(u), c.v, c.i)) {
          c.v = v;
          c.i = col(u);
        }
      }
    }
    // across the four groups of the wave, then across the waves
    cand_rows(c);
    if (tolmode) sum_rows(ssq);
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
    for (int w = 1; w < NWV; ++w) {
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
    if (b.i != 0x7fffffff) {
      // the candidate is slot bu of group bg (the same on every thread)
      const int cl = b.i - c0;
      const int bu = __builtin_amdgcn_readfirstlane(cl / NGR);
      if (grp == cl % NGR) {
        T yb[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) yb[t] = (T)0;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (u == bu) {
#pragma unroll
            for (int t = 0; t < RPL; ++t) yb[t] = yget(u, t);
          }
        }
        uint64_t* dst = cvals + ((size_t)par * G + g) * CW;
        // every slot, by row: readers take rows [e, l) only
#pragma unroll
        for (int t = 0; t < RPL; ++t) Words<T>::put(dst + (size_t)(rgi + R * t), st, yb[t]);
        // the exact norm of rows [e, l), formed as a reader of the column would
        // form it, while the readers still wait for the other records (rows at
        // or past l hold zeros)
        const int et = __builtin_amdgcn_readfirstlane(e / R), er = __builtin_amdgcn_readfirstlane(e % R);
        const bool ein = rgi >= er;
        double xs = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const T q = keep_or_zero(yb[t], t > et || (t == et && ein));
          xs += (double)q * (double)q;
        }
        const double xn = sqrt(gsum<R>(xs));
        if (rgi == 0) Words<double>::put(dst + (size_t)R * RPL, st, xn);
      }
    }
  };

  publish(0);

  bool done = false;
  while (!done) {
    asm volatile("" : "+v"(ybase));
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
    for (int q = 1; q < NWV; ++q) {
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
    double x0 = 0.0, xnorm = 0.0;
    if (stop == 0) {
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
      if (tid == NTH - 1) {
        uint64_t a0, a1;
        fetch(slot + (uint32_t)(R * RPL) * 8u, a0, a1);
        s_xnorm = __hiloint2double((int)(uint32_t)a0, (int)(uint32_t)a1);
      }
      for (int q = (j >> 1) + tid; 2 * q < l; q += NTH) {
        uint64_t a0, a1;
        fetch(slot + (uint32_t)(2 * q) * 8u, a0, a1);
        f_at(8u * (uint32_t)q) = __uint_as_float((uint32_t)a0);
        f_at(8u * (uint32_t)q + 4u) = __uint_as_float((uint32_t)a1);
      }
      if (!ok) s_vfail = 1;
      __syncthreads();
      if (s_vfail) stop = ST_TIMEOUT;
      x0 = (double)f_at(4u * (uint32_t)j);
      xnorm = s_xnorm;   // exact norm of the trailing column, formed by its publisher
      if (stop == 0 && !(xnorm > 0.0)) stop = -1;
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
    // the reflector's entry in slot t of this lane: for t > jt the staged
    // column (rows below j); in slot jt, x0 - alpha at row j, the staged column
    // below it and zero above
    const T vjt = mj ? (T)(x0 - alpha) : (mg ? f_at(4u * (uint32_t)(rgi + R * jt)) : (T)0);
    // LDS addresses of slot t: the staged column's entry, the LDS column slots
    auto vaddr = [&](int t) { return 4u * (uint32_t)(rgi + R * t); };
    auto laddr = [&](int i, int t) { return ybase + (uint32_t)i * kSlotBytes + (uint32_t)t * (NTH * 4); };
    constexpr int NLA = NL > 0 ? NL : 1;
    // The two slot passes below load the reflector entry and the LDS columns of
    // slot t + 1 while slot t's products run (slot jt's come from a run-time
    // address before the first); the products keep their order.
    if (tid == 0) win[j] = w.i;
    // the winner itself becomes (alpha, 0, ..., 0) below row j and leaves the active set
    if (w.i >= c0 && w.i < c1) {
      const int cl = w.i - c0;
      const int wu = __builtin_amdgcn_readfirstlane(cl / NGR);
      if (grp == cl % NGR) {
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (u == wu) {
            actb &= ~(1u << u);
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
              if (t < jt) continue;
              if (t == jt) yset(u, t, mj ? (T)alpha : (mg ? (T)0 : yget(u, t)));
              else yset(u, t, (T)0);
            }
          }
        }
      }
    }
    // ---- apply the reflector to the group's columns --------------------------------
    double dot[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) dot[u] = 0.0;
    {
      T pv = vjt, pl[NLA];
#pragma unroll
      for (int i = 0; i < NL; ++i) pl[i] = f_at(laddr(i, jt));
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        if (t < jt) continue;
        const T cv = pv;
        T cl[NLA];
#pragma unroll
        for (int i = 0; i < NL; ++i) cl[i] = pl[i];
        if (t + 1 < RPL) {
          pv = f_at(vaddr(t + 1));
#pragma unroll
          for (int i = 0; i < NL; ++i) pl[i] = f_at(laddr(i, t + 1));
        }
        const double vt = (double)cv;
#pragma unroll
        for (int u = 0; u < NC; ++u) dot[u] = fma(vt, (double)y[u][t], dot[u]);
#pragma unroll
        for (int i = 0; i < NL; ++i) dot[NC + i] = fma(vt, (double)cl[i], dot[NC + i]);
      }
    }
    // the update pass reads the LDS slots again: without this the compiler keeps
    // the values the dot products loaded in registers until then
    asm volatile("" ::: "memory");
    T mw[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const double d = gsum<R>(dot[u]);
      mw[u] = act(u) ? (T)(-tau * d) : (T)0;
    }
    double ss[NT];
    T sj[NT];   // each lane's slot-jt value (row jt R + rgi)
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      ss[u] = 0.0;
      sj[u] = (T)0;
    }
    {
      T pv = vjt, pl[NLA];
#pragma unroll
      for (int i = 0; i < NL; ++i) pl[i] = f_at(laddr(i, jt));
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        if (t < jt) continue;
        const T vt = pv;
        T cl[NLA];
#pragma unroll
        for (int i = 0; i < NL; ++i) cl[i] = pl[i];
        if (t + 1 < RPL) {
          pv = f_at(vaddr(t + 1));
#pragma unroll
          for (int i = 0; i < NL; ++i) pl[i] = f_at(laddr(i, t + 1));
        }
        const bool at = t == jt, after = t > jt;   // the same on every lane
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          const T yo = u < NC ? y[u < NC ? u : 0][t] : cl[u < NC ? 0 : u - NC];
          const T yn = fmaf(mw[u], vt, yo);
          if (u < NC) y[u < NC ? u : 0][t] = yn;
          else f_at(laddr(u - NC, t)) = yn;
          if constexpr (EXACT) {
            const double q = (double)yn;
            ss[u] += after ? q * q : 0.0;
          }
          sj[u] = at ? yn : sj[u];
        }
      }
    }
    // squared norm below row j of column u, summed over the group
    auto below = [&](int u) {
      const double q = (double)sj[u];
      double r = mg ? q * q : 0.0;
      if constexpr (EXACT) {
        r += ss[u];
      } else {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          if (t <= jt) continue;
          // the empty asm keeps the compiler from computing these squares
          // ahead of the (rarely taken) recompute branch on every step
          T yt = yget(u, t);
          asm volatile("" : "+v"(yt));
          const double qq = (double)yt;
          r += qq * qq;
        }
      }
      return gsum<R>(r);
    };
    if constexpr (EXACT) {
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const double rs = below(u);
        if (act(u)) nu2(u) = rs;
      }
    } else {
      // downdate nu^2 -= s^2 with s the new row-j entry; recompute from the
      // column when the downdate has cancelled below tol3z of the norm^2 at
      // the last recompute
      bool need[NT];
      T sb[NT];
      group_bcast<R, NT>(sj, sb, jr);
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        const double s = (double)sb[u];
        need[u] = false;
        const double o = nu2(u);
        if (act(u) && o > 0.0) {
          const double nn = fmax(0.0, o - s * s);
          need[u] = nn <= lim(u);
          nu2(u) = nn;
        }
      }
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        if (__any(need[u])) {
          const double rs = below(u);
          if (need[u]) {
            nu2(u) = rs;
            lim(u) = tol3z * rs;
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
    for (int u = 0; u < NT; ++u) {
      if (col(u) < c1) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int row = rgi + R * t;
          if (row < kout) S[(int64_t)row * a.ldS + col(u)] = yget(u, t);
        }
      }
    }
  }
  if (rgi == 0) {
#pragma unroll
    for (int u = 0; u < NT; ++u) act_s[u * NGR + grp] = act(u) ? 1 : 0;
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
  for (int q = 0; q < NWV; ++q) {
    bsum += x_t[q];
    fin_tmo |= p_i[q];
  }
  if (fin_tmo) {
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
    for (int t = tid; t < kout; t += NTH) a.J[t] = win[t];
    if (tid == 0) *a.k_out = kout;
  }
}

struct ResCfg {
  int NTH, RPL, NC, NL;
};
// searched in order: the first entry that covers l and n with at most one
// workgroup per compute unit and fits LDS is taken. Two waves per SIMD (512
// threads, the register slots in plain VGPRs) measured 5.7 ms for the 499 steps
// of a 500 x 50000 slab against 7.2 ms with one wave per SIMD (9 register and
// 4 LDS slots per group, part of them in AGPRs).
constexpr ResCfg kResCfgs[] = {{512, 32, 5, 2}, {512, 33, 4, 2}};
constexpr int kNumResCfgs = sizeof(kResCfgs) / sizeof(kResCfgs[0]);

template <int I>
const void* res_kernel_ptr(bool exact) {
  constexpr ResCfg c = kResCfgs[I];
  return exact ? (const void*)cpqr_res_kernel<c.NTH, c.RPL, c.NC, c.NL, true>
               : (const void*)cpqr_res_kernel<c.NTH, c.RPL, c.NC, c.NL, false>;
}
template <int... I>
const void* res_kernel_lookup(int i, bool exact, std::integer_sequence<int, I...>) {
  const void* p = nullptr;
  ((i == I ? (p = res_kernel_ptr<I>(exact), 0) : 0), ...);
  return p;
}

}  // namespace cr
}  // namespace idcur
