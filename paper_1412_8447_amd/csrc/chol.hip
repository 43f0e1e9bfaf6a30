// Cholesky factor and triangular inverse of a small matrix (c <= 256), FP64.
//
// Serves the Cholesky-QR orthonormalisation of the sketch between power steps
// (orth in Section 5.3), the QR factorisation of R^T for the least-squares
// solve of U R = V* (Section 4.3), and the inverse of S11 from which T follows
// by a matrix product (Section 4.1, eq. (S11T=S12)).
//
//   mode 0:  G = L L^T  ->  L and X = L^{-1}
//   mode 1:  lower-triangular L given (strided view)  ->  X = L^{-1}
//
// One workgroup of 8 waves, right-looking over 32 x 32 tiles (T = ceil(c/32)
// tile rows, padded with the identity). For panel p, with D_p = L_pp^{-1}:
//   phase 2 (all waves, one tile each):
//       L_rp = A_rp D_p^T                (mode 0; mode 1 reads L_rp)   r > p
//       X_pc = D_p X_pc                  (X_pc accumulated so far)     c < p
//       X_pp = D_p
//   phase 3 (waves 1..7):
//       A_rs -= L_rp L_sp^T              (mode 0 trailing update)      p < s <= r
//       X_rc -= L_rp X_pc                                              r > p, c <= p
//   phase 3 (wave 0, look-ahead): update A_{p+1,p+1}, factor it and invert
//       its factor, so that D_{p+1} is ready when the barrier ends the phase.
// Tile products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64) with
// operands from LDS (the panel column L_.p and the panel row X_p.); the
// trailing tiles of A and X are accumulated in place in the output arrays
// (L2-resident). The diagonal tile is factored by one wave with its rows in
// registers (one row per lane, pivot columns broadcast with v_readlane) and
// inverted with a column per lane.
//
// f64 16x16x4 operand layout: lane L holds A(L%16, L/16) and B(L/16, L%16);
// result register t of lane L is C(L/16 + 4t, L%16).
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kCT = 512;             // 8 waves
constexpr int kWaves = kCT / 64;
constexpr int kTS = 32;              // tile edge
constexpr int kTL = kTS + 1;         // LDS row stride of a tile (doubles)
constexpr int kTile = kTS * kTL;     // doubles per LDS tile
constexpr int kMaxT = 8;
constexpr int kMaxC = kMaxT * kTS;

typedef double d4 __attribute__((ext_vector_type(4)));

struct CArgs {
  const double* G; int64_t gr, gc;   // mode 0: G(i,j) = G[i*gr + j*gc]; mode 1: the factor L
  int c_host; const int* c_dev;
  double* L; int64_t ldl;             // mode 0 output (lower, zeros above)
  double* X; int64_t ldx;             // inverse (lower, zeros above)
  double shift_rel;
  int mode;
  int keep_l;   // mode 0: store the factor to L (else L is only the working matrix)
  int* status;
  int bsz;      // mode 1 with a grid of several workgroups: workgroup p inverts the
                // diagonal block [p bsz, min((p + 1) bsz, c))^2 of G into X
};

// strided read-only view, padded with the identity outside [0, c)^2
struct View {
  const double* p;
  int64_t rs, cs;
  int c;
  __device__ __forceinline__ double at(int i, int j) const {
    const bool in = i < c && j < c;
    const double v = p[(int64_t)min(i, c - 1) * rs + (int64_t)min(j, c - 1) * cs];
    return in ? v : (i == j ? 1.0 : 0.0);
  }
};

// LDS (dynamic): every helper addresses it through `sm` with an offset, so
// that out-of-line helpers still compile to LDS instructions.
extern __shared__ __align__(16) double sm[];
constexpr int kPan = 0;                          // L(r, p), r = 1..kMaxT-1 at kPan + (r-1)*kTile
constexpr int kXrow = kPan + (kMaxT - 1) * kTile;    // X(p, c), c = 0..kMaxT-2
constexpr int kDbuf = kXrow + (kMaxT - 1) * kTile;   // D_p, double-buffered
constexpr int kDg = kDbuf + 2 * kTile;               // diagonal tile being factored
constexpr int kRinv = kDg + kTile;                   // reciprocals of its diagonal (32)
constexpr int kOnehot = kRinv + kTS;                 // 64 doubles: e_32
constexpr int kSmax = kOnehot + 64;                  // per-wave maxima (kWaves)
constexpr int kLdsDoubles = kSmax + kWaves;

struct Acc {
  d4 v[2][2];
};

__device__ __forceinline__ void acc_zero(Acc& a) {
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) a.v[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
}

// accumulator element (bi, bj, t) of lane L sits at tile row bi*16 + L/16 + 4t,
// column bj*16 + L%16
__device__ __forceinline__ void acc_load(Acc& a, const View& m, int i0, int j0) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) a.v[bi][bj][t] = m.at(i0 + bi * 16 + q + 4 * t, j0 + bj * 16 + r16);
}

__device__ __forceinline__ void acc_store(const Acc& a, double* M, int64_t ld, int i0, int j0, int c, bool lower_only) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = i0 + bi * 16 + q + 4 * t, j = j0 + bj * 16 + r16;
        if (i < c && j < c && (!lower_only || j <= i)) M[(int64_t)i * ld + j] = a.v[bi][bj][t];
      }
}

__device__ __forceinline__ void acc_to_lds(const Acc& a, int tile) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int t = 0; t < 4; ++t) sm[tile + (bi * 16 + q + 4 * t) * kTL + bj * 16 + r16] = a.v[bi][bj][t];
}

// one wave copies the tile at (i0, j0) of the view into LDS
__device__ __forceinline__ void tile_from_view(int tile, const View& m, int i0, int j0) {
  const int lane = threadIdx.x & 63;
  double v[kTS * kTS / 64];
#pragma unroll
  for (int t = 0; t < kTS * kTS / 64; ++t) {
    const int e = lane + 64 * t;
    v[t] = m.at(i0 + (e >> 5), j0 + (e & 31));
  }
#pragma unroll
  for (int t = 0; t < kTS * kTS / 64; ++t) {
    const int e = lane + 64 * t;
    sm[tile + (e >> 5) * kTL + (e & 31)] = v[t];
  }
}

// acc += sgn * A * B (NT = false: B[k][j]; NT = true: B given transposed, B[j][k])
template <bool NT>
__device__ __forceinline__ void tile_mma(Acc& acc, int A, int B, double sgn) {
  const int lane = threadIdx.x & 63, q = lane >> 4, r16 = lane & 15;
#pragma unroll
  for (int k0 = 0; k0 < kTS; k0 += 4) {
    const double a0 = sgn * sm[A + r16 * kTL + k0 + q];
    const double a1 = sgn * sm[A + (16 + r16) * kTL + k0 + q];
    const double b0 = NT ? sm[B + r16 * kTL + k0 + q] : sm[B + (k0 + q) * kTL + r16];
    const double b1 = NT ? sm[B + (16 + r16) * kTL + k0 + q] : sm[B + (k0 + q) * kTL + 16 + r16];
    acc.v[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc.v[0][0], 0, 0, 0);
    acc.v[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc.v[0][1], 0, 0, 0);
    acc.v[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc.v[1][0], 0, 0, 0);
    acc.v[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc.v[1][1], 0, 0, 0);
  }
}

// 1/sqrt(a) for a > 0: the hardware estimate refined by two Newton-Raphson
// steps y <- y + y (1 - a y^2) / 2 (each step doubles the correct bits)
__device__ __forceinline__ double rsqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-a * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// ---- work items (out of line: each computes its own lane indexing, so the
// compiler keeps none of it alive across the panel loop) ----------------------

// phase 2, mode 0: L(r, p) = A(r, p) D_p^T into LDS and L; mode 1: L(r, p) into LDS
__device__ __noinline__ void item_panel(View A, double* L, int64_t ldl, int r, int p, int D, bool m0, bool keep_l) {
  const int P = kPan + (r - 1) * kTile;
  tile_from_view(P, A, r * kTS, p * kTS);
  if (m0) {
    Acc acc;
    acc_zero(acc);
    tile_mma<true>(acc, P, D, 1.0);
    acc_to_lds(acc, P);
    if (keep_l) acc_store(acc, L, ldl, r * kTS, p * kTS, A.c, false);
  }
}

// phase 2: X(p, p) = D_p
__device__ __noinline__ void item_store_d(double* X, int64_t ldx, int p, int D, int c) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < kTS * kTS / 64; ++t) {
    const int e = lane + 64 * t;
    const int i = p * kTS + (e >> 5), j = p * kTS + (e & 31);
    if (i < c && j < c) X[(int64_t)i * ldx + j] = sm[D + (e >> 5) * kTL + (e & 31)];
  }
}

// phase 2: X(p, cc) = D_p X(p, cc) into LDS and X
__device__ __noinline__ void item_xrow(View XV, double* X, int64_t ldx, int p, int cc, int D) {
  const int Xr = kXrow + cc * kTile;
  tile_from_view(Xr, XV, p * kTS, cc * kTS);
  Acc acc;
  acc_zero(acc);
  tile_mma<false>(acc, D, Xr, 1.0);
  acc_to_lds(acc, Xr);
  acc_store(acc, X, ldx, p * kTS, cc * kTS, XV.c, false);
}

// phase 3 for one of the waves 1..kWaves-1: its share of the tiles
//   trailing (mode 0): A(r, s) -= L(r, p) L(s, p)^T, p+1 <= s <= r <= T-1,
//                      without (p+1, p+1), which wave 0 takes
//   X:                 X(r, cc) -= L(r, p) X(p, cc), r > p, cc <= p (X(p, p) = D_p)
// The accumulator tile of the next item is loaded while the current one is
// multiplied.
__device__ __noinline__ void phase3_items(View A, double* L, int64_t ldl, View XV, double* X, int64_t ldx, int p,
                                          int m, bool m0, int D, int w) {
  const int ntr = m0 ? m * (m + 1) / 2 - 1 : 0;
  const int n = ntr + m * (p + 1);
  const int step = kWaves - 1;
  struct Item {
    int r, s;
    bool tr;
  };
  auto decode = [&](int it) {
    Item t;
    if (it < ntr) {
      int e = it + 1, s = p + 1, len = m;
      while (e >= len) {
        e -= len;
        ++s;
        --len;
      }
      t.r = s + e;
      t.s = s;
      t.tr = true;
    } else {
      const int j = it - ntr;
      t.r = p + 1 + j / (p + 1);
      t.s = j % (p + 1);
      t.tr = false;
    }
    return t;
  };
  int it = w;
  if (it >= n) return;
  Item cur = decode(it);
  Acc acc;
  acc_load(acc, cur.tr ? A : XV, cur.r * kTS, cur.s * kTS);
  for (; it < n; it += step) {
    Acc nxt;
    Item ni = cur;
    const bool more = it + step < n;
    if (more) {
      ni = decode(it + step);
      acc_load(nxt, ni.tr ? A : XV, ni.r * kTS, ni.s * kTS);
    }
    if (cur.tr) {
      tile_mma<true>(acc, kPan + (cur.r - 1) * kTile, kPan + (cur.s - 1) * kTile, -1.0);
      acc_store(acc, L, ldl, cur.r * kTS, cur.s * kTS, A.c, cur.r == cur.s);
    } else {
      tile_mma<false>(acc, kPan + (cur.r - 1) * kTile, cur.s == p ? D : kXrow + cur.s * kTile, -1.0);
      acc_store(acc, X, ldx, cur.r * kTS, cur.s * kTS, XV.c, false);
    }
    if (more) {
      acc = nxt;
      cur = ni;
    }
  }
}

// ---- the diagonal tile, as a 2 x 2 block recursion on 16 x 16 blocks ---------
// Cholesky of a 16 x 16 block in registers: lane i (< 16) holds row i, pivot
// columns are broadcast with v_readlane (lanes 16..63 repeat lanes 0..15).
__device__ __forceinline__ void chol16(double (&r)[16], bool& bad) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    double akk = readlane_d(r[k], k);
    bad = bad || !(akk > 0.0);
    akk = (akk > 0.0) ? akk : 1e-300;
    const double inv = rsqrt_nr(akk);
    // row k's own entry becomes akk / sqrt(akk), the pivot; rows above k only
    // ever change entries above their diagonal
    const double lk = r[k] * inv;
    r[k] = lk;
#pragma unroll
    for (int j = k + 1; j < 16; ++j) r[j] = fma(-lk, readlane_d(r[k], j), r[j]);
  }
}

// X = L^{-1} for the lower-triangular 16 x 16 block of the tile at (o, o) of
// kDg, into the block (o, o) of out: lane i (< 16) forms column i by forward
// substitution from the unit vector (zeros above the diagonal), column-oriented:
// once x[t] is final it is subtracted from all later rows, so the dependent
// chain is two operations per row.
__device__ __forceinline__ void inv16(int o, int out) {
  const int lane = threadIdx.x & 63, i = lane & 15;
  if (lane < 16) sm[kRinv + o + i] = 1.0 / sm[kDg + (o + i) * kTL + o + i];
  double x[16];
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) x[ii] = sm[kOnehot + 32 + i - ii];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    x[t] *= sm[kRinv + o + t];
#pragma unroll
    for (int ii = t + 1; ii < 16; ++ii) x[ii] = fma(-sm[kDg + (o + ii) * kTL + o + t], x[t], x[ii]);
  }
  if (lane < 16) {
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) sm[out + (o + ii) * kTL + o + i] = x[ii];
  }
}

// One wave: diagonal tile q (after the update by panel q-1, whose L(q, q-1)
// sits in the panel buffer when upd is set). With the tile [A11 .; A21 A22] in
// 16 x 16 blocks:
//   mode 0:  L11 = chol(A11), X11 = L11^{-1}, L21 = A21 X11^T,
//            L22 = chol(A22 - L21 L21^T), X22 = L22^{-1};
//   mode 1:  the blocks of the given factor, X11 and X22 the same way;
//   both:    X21 = -X22 (L21 X11), so dout <- L_qq^{-1} = [X11 0; X21 X22].
// The 16 x 16 products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64,
// 4 k steps each); the serial chains are two 16-column eliminations and two
// 16-row substitutions instead of 32 + 32. L_qq goes to L (mode 0).
__device__ __noinline__ void item_diag(View A, double* L, int64_t ldl, int q, bool upd, int dout, bool m0,
                                       bool keep_l, int* status) {
  const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
  const int q0 = q * kTS;
  if (m0) {
    Acc acc;
    acc_load(acc, A, q0, q0);
    if (upd) tile_mma<true>(acc, kPan + (q - 1) * kTile, kPan + (q - 1) * kTile, -1.0);
    acc_to_lds(acc, kDg);
  } else {
    tile_from_view(kDg, A, q0, q0);
  }
  bool bad = false;
  if (m0) {
    double r[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) r[j] = sm[kDg + i * kTL + j];
    chol16(r, bad);
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < 16; ++j) sm[kDg + i * kTL + j] = r[j];
    }
  }
  inv16(0, dout);
  if (lane < 16) {
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) sm[dout + ii * kTL + 16 + i] = 0.0;   // X12 = 0
  }
  // f64 16x16x4 operands: lane L holds A(L%16, 4kk + L/16) and B(4kk + L/16, L%16);
  // result register t of lane L is C(L/16 + 4t, L%16)
  if (m0) {
    d4 c = d4{0.0, 0.0, 0.0, 0.0};   // L21 = A21 X11^T
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(sm[kDg + (16 + i) * kTL + 4 * kk + g], sm[dout + i * kTL + 4 * kk + g], c, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) sm[kDg + (16 + g + 4 * t) * kTL + i] = c[t];
    d4 s22;   // A22 - L21 L21^T
#pragma unroll
    for (int t = 0; t < 4; ++t) s22[t] = sm[kDg + (16 + g + 4 * t) * kTL + 16 + i];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const double l = sm[kDg + (16 + i) * kTL + 4 * kk + g];
      s22 = __builtin_amdgcn_mfma_f64_16x16x4f64(-l, l, s22, 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) sm[kDg + (16 + g + 4 * t) * kTL + 16 + i] = s22[t];
    double r[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) r[j] = sm[kDg + (16 + i) * kTL + 16 + j];
    chol16(r, bad);
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < 16; ++j) sm[kDg + (16 + i) * kTL + 16 + j] = r[j];
    }
  }
  inv16(16, dout);
  {
    d4 pm = d4{0.0, 0.0, 0.0, 0.0};   // P = L21 X11
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      pm = __builtin_amdgcn_mfma_f64_16x16x4f64(sm[kDg + (16 + i) * kTL + 4 * kk + g], sm[dout + (4 * kk + g) * kTL + i], pm, 0, 0, 0);
    // X21 = -X22 P: the B operand P(4kk + L/16, L%16) is result register kk of lane L
    d4 x21 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      x21 = __builtin_amdgcn_mfma_f64_16x16x4f64(-sm[dout + (16 + i) * kTL + 16 + 4 * kk + g], pm[kk], x21, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) sm[dout + (16 + g + 4 * t) * kTL + i] = x21[t];
  }
  if (bad && lane == 0) set_status(status, ST_NONFINITE);
  if (m0 && keep_l && lane < kTS && q0 + lane < A.c) {
#pragma unroll
    for (int j = 0; j < kTS; ++j)
      if (j <= lane) L[(int64_t)(q0 + lane) * ldl + q0 + j] = sm[kDg + lane * kTL + j];
  }
}

__global__ __launch_bounds__(kCT) void chol_inv_kernel(CArgs a) {
  if (gridDim.x > 1) {   // independent diagonal blocks (mode 1, no device order)
    const int o = (int)blockIdx.x * a.bsz;
    a.G += (int64_t)o * a.gr + (int64_t)o * a.gc;
    a.X += (int64_t)o * a.ldx + o;
    a.c_host = min(a.bsz, a.c_host - o);
  }
  const int c = a.c_dev ? min(*a.c_dev, a.c_host) : a.c_host;
  if (c <= 0) return;
  const int T = (c + kTS - 1) / kTS;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool m0 = a.mode == 0;
  double* L = a.L;
  double* X = a.X;
  if (tid < 64) sm[kOnehot + tid] = tid == 32 ? 1.0 : 0.0;

  // ---- setup: L = lower(G) + shift (mode 0), X = 0 ---------------------------
  if (m0) {
    double sh = 0.0;
    if (a.shift_rel > 0.0) {
      double mx = 0.0;
      for (int i = tid; i < c; i += kCT) mx = fmax(mx, a.G[(int64_t)i * a.gr + (int64_t)i * a.gc]);
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      if (lane == 0) sm[kSmax + wv] = mx;
      __syncthreads();
      mx = 0.0;
      for (int w = 0; w < kWaves; ++w) mx = fmax(mx, sm[kSmax + w]);
      sh = a.shift_rel * mx;
    }
    // sixteen loads in flight per thread before the stores (which the compiler
    // keeps behind the loads, not knowing that G and L never overlap)
    const int total = c * c;
    constexpr int kU = 16;
    for (int e0 = 0; e0 < total; e0 += kCT * kU) {
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = min(e0 + u * kCT + tid, total - 1);
        v[u] = a.G[(int64_t)(e / c) * a.gr + (int64_t)(e % c) * a.gc];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * kCT + tid;
        if (e < total) {
          const int i = e / c, j = e % c;
          L[(int64_t)i * a.ldl + j] = (j <= i) ? v[u] + (i == j ? sh : 0.0) : 0.0;
        }
      }
    }
  }
  for (int e = tid; e < c * c; e += kCT) X[(int64_t)(e / c) * a.ldx + e % c] = 0.0;
  __syncthreads();

  // the matrix being factored (mode 0: L, updated in place) or the given factor
  const View A = m0 ? View{L, a.ldl, 1, c} : View{a.G, a.gr, a.gc, c};
  const View XV{X, a.ldx, 1, c};

  // p = -1 only factors the first diagonal tile
  for (int p = -1; p < T; ++p) {
    const int m = T - 1 - p;   // tile rows below the panel
    const int D = kDbuf + (p & 1) * kTile;
    if (p >= 0) {
      // ---- phase 2 --------------------------------------------------------------
      for (int it = wv; it < T; it += kWaves) {
        if (it < m) item_panel(A, L, a.ldl, p + 1 + it, p, D, m0, a.keep_l != 0);
        else if (it == m) item_store_d(X, a.ldx, p, D, c);
        else item_xrow(XV, X, a.ldx, p, it - m - 1, D);
      }
      __syncthreads();
      if (m == 0) break;
    }
    // ---- phase 3 ----------------------------------------------------------------
    if (wv == 0) {
      item_diag(A, L, a.ldl, p + 1, p >= 0, kDbuf + ((p + 1) & 1) * kTile, m0, a.keep_l != 0, a.status);
    } else if (p >= 0) {
      phase3_items(A, L, a.ldl, XV, X, a.ldx, p, m, m0, D, wv - 1);
    }
    __syncthreads();
  }
}

}  // namespace

size_t chol_inv_lds_bytes(int c_host) {
  (void)c_host;
  return (size_t)kLdsDoubles * sizeof(double);
}

hipError_t chol_inv_launch(int mode, const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, double* L,
                           int64_t ldl, double* X, int64_t ldx, double shift_rel, int* status, hipStream_t stream,
                           int keep_l) {
  if (c_host <= 0) return hipSuccess;
  if (c_host > kMaxC) return hipErrorInvalidValue;
  if (mode == 0 && !L) return hipErrorInvalidValue;
  CArgs a{};
  a.G = G; a.gr = gr; a.gc = gc; a.c_host = c_host; a.c_dev = c_dev;
  a.L = L; a.ldl = ldl; a.X = X; a.ldx = ldx; a.shift_rel = shift_rel; a.mode = mode; a.status = status;
  a.keep_l = keep_l;
  const size_t lds = chol_inv_lds_bytes(c_host);
  hipError_t e = hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)chol_inv_kernel, dim3(1), dim3(kCT), args, lds, stream);
}

hipError_t chol_inv_diag_launch(const double* F, int64_t ldf, int c, int bsz, double* X, int64_t ldx, int* status,
                                hipStream_t stream) {
  if (c <= 0) return hipSuccess;
  if (bsz <= 0 || bsz > kMaxC) return hipErrorInvalidValue;
  CArgs a{};
  a.G = F; a.gr = ldf; a.gc = 1; a.c_host = c; a.c_dev = nullptr;
  a.L = nullptr; a.ldl = 0; a.X = X; a.ldx = ldx; a.shift_rel = 0.0; a.mode = 1; a.status = status;
  a.bsz = bsz;
  const size_t lds = chol_inv_lds_bytes(bsz);
  hipError_t e = hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)chol_inv_kernel, dim3((unsigned)ceil_div(c, bsz)), dim3(kCT), args, lds, stream);
}

}  // namespace idcur
