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
// One workgroup of 512 threads, right-looking over 32-column panels. For a
// panel with diagonal block D and rows below B:
//   mode 0 only: one wave factors D in LDS, the rows below become B D^{-T},
//                and the trailing lower triangle takes - B B^T;
//   both modes:  D^{-1} (one wave, a column per lane), then the elimination
//                applied to X: X_p <- D^{-1} X_p for the panel rows, and
//                X_below <- X_below - B X_p.
// Every inner operation is a block of independent multiply-adds over LDS
// operands; the only sequential chains are the 32 steps inside a diagonal
// block, each confined to a single wave.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kCT = 512;
constexpr int kNB = 32;
constexpr int kMaxC = 256;
constexpr int kLd = kNB + 1;   // padded row stride of the 32-wide LDS tiles

struct CArgs {
  const double* G; int64_t gr, gc;   // mode 0: G(i,j) = G[i*gr + j*gc]; mode 1: the factor L
  int c_host; const int* c_dev;
  double* L; int64_t ldl;             // mode 0 output (lower, zeros above)
  double* X; int64_t ldx;             // inverse (lower, zeros above)
  double shift_rel;
  int mode;
  int* status;
};

// sum_{t < 32, lo <= t <= hi} a[t*sa] * b[t*sb] with both operands read into
// registers first (all 64 LDS reads in flight), masked terms selected to zero.
__device__ __forceinline__ double dot32(const double* a, int sa, const double* b, int sb, int lo, int hi) {
  double x[kNB], y[kNB];
#pragma unroll
  for (int t = 0; t < kNB; ++t) {
    x[t] = a[t * sa];
    y[t] = b[t * sb];
  }
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < kNB; ++t) s += (t >= lo && t <= hi) ? x[t] * y[t] : 0.0;
  return s;
}
// same with the first operand already in registers
__device__ __forceinline__ double dot32r(const double (&x)[kNB], const double* b, int sb, int lo, int hi) {
  double y[kNB];
#pragma unroll
  for (int t = 0; t < kNB; ++t) y[t] = b[t * sb];
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < kNB; ++t) s += (t >= lo && t <= hi) ? x[t] * y[t] : 0.0;
  return s;
}

// Element-wise copy with B independent loads in flight per thread: load(e)
// must be safe for e = 0; store(e, v) is only called for e < total.
template <int B, class LoadF, class StoreF>
__device__ __forceinline__ void batched(int total, LoadF load, StoreF store) {
  for (int e0 = 0; e0 < total; e0 += kCT * B) {
    double v[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int e = e0 + q * kCT + (int)threadIdx.x;
      v[q] = load(e < total ? e : 0);
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int e = e0 + q * kCT + (int)threadIdx.x;
      if (e < total) store(e, v[q]);
    }
  }
}

__global__ __launch_bounds__(kCT) void chol_inv_kernel(CArgs a) {
  extern __shared__ __align__(16) double sm[];
  double* D = sm;                          // kNB x kLd   diagonal block (factored)
  double* Di = D + kNB * kLd;              // kNB x kLd   its inverse
  double* Pb = Di + kNB * kLd;             // c_host x kLd rows below the block (the factor's panel)
  double* Xp = Pb + (size_t)a.c_host * kLd;// kNB x (c_host+1) panel rows of X
  __shared__ double smax[kCT / 64];
  const int c = a.c_dev ? min(*a.c_dev, a.c_host) : a.c_host;
  const int ldxp = a.c_host + 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* L = a.L;
  double* X = a.X;

  // ---- setup: L = lower(G) (+ shift), X = I --------------------------------
  double sh = 0.0;
  if (a.mode == 0 && a.shift_rel > 0.0) {
    double mx = 0.0;
    for (int i = tid; i < c; i += kCT) mx = fmax(mx, a.G[(int64_t)i * a.gr + (int64_t)i * a.gc]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) smax[wv] = mx;
    __syncthreads();
    mx = 0.0;
    for (int w = 0; w < kCT / 64; ++w) mx = fmax(mx, smax[w]);
    sh = a.shift_rel * mx;
  }
  if (a.mode == 0)
    batched<8>(c * c,
               [&](int e) { const int i = e / c, j = e % c; return a.G[(int64_t)i * a.gr + (int64_t)j * a.gc]; },
               [&](int e, double v) {
                 const int i = e / c, j = e % c;
                 L[(int64_t)i * a.ldl + j] = (j <= i) ? v + (i == j ? sh : 0.0) : 0.0;
               });
  for (int e = tid; e < c * c; e += kCT) X[(int64_t)(e / c) * a.ldx + e % c] = (e / c == e % c) ? 1.0 : 0.0;
  __syncthreads();
  // the factor being eliminated: L (mode 0, updated in place) or the input view
  auto fel = [&](int i, int j) -> double {
    return a.mode == 0 ? L[(int64_t)i * a.ldl + j] : a.G[(int64_t)i * a.gr + (int64_t)j * a.gc];
  };

  for (int p0 = 0; p0 < c; p0 += kNB) {
    const int nb = min(kNB, c - p0);
    const int p1 = p0 + nb;
    const int nr = c - p1;
    // ---- (a) diagonal block to LDS -----------------------------------------
    batched<2>(kNB * kNB,
               [&](int e) { const int i = min(e / kNB, nb - 1), j = min(e % kNB, nb - 1); return fel(p0 + i, p0 + j); },
               [&](int e, double v) {
                 const int i = e / kNB, j = e % kNB;
                 D[i * kLd + j] = (i < nb && j < nb && j <= i) ? v : (i == j ? 1.0 : 0.0);
               });
    __syncthreads();
    // ---- (b) mode 0: factor D in place (wave 0, row `lane`) -------------------
    // (loads are unconditional and results selected, so that the LDS reads of
    // one step are issued together instead of one masked branch per term)
    if (a.mode == 0 && wv == 0 && lane < kNB) {
      for (int j = 0; j < nb; ++j) {
        if (lane == j) {
          double d = D[j * kLd + j];
          if (!(d > 0.0)) {
            set_status(a.status, ST_NONFINITE);
            d = 1e-300;
          }
          D[j * kLd + j] = sqrt(d);
        }
        const double djj = D[j * kLd + j];
        const bool below = lane > j && lane < nb;
        const double lraw = D[lane * kLd + j];
        const double lij = below ? lraw / djj : 0.0;
        if (below) D[lane * kLd + j] = lij;
        double dk[kNB], cur[kNB];
#pragma unroll
        for (int k = 1; k < kNB; ++k) {
          dk[k] = D[k * kLd + j];
          cur[k] = D[lane * kLd + k];
        }
#pragma unroll
        for (int k = 1; k < kNB; ++k)
          D[lane * kLd + k] = (k > j && k <= lane && below) ? cur[k] - lij * dk[k] : cur[k];
      }
    }
    __syncthreads();
    // ---- (c) Di = D^{-1} (wave 0, column `lane`) ------------------------------
    if (wv == 0 && lane < kNB) {
      const int j = lane;
      for (int i = 0; i < kNB; ++i) {
        double v;
        if (i < j) v = 0.0;
        else if (i == j) v = 1.0 / D[i * kLd + i];
        else {
          const double s = dot32(D + i * kLd, 1, Di + j, kLd, j, i - 1);
          v = -s / D[i * kLd + i];
        }
        Di[i * kLd + j] = v;
      }
    }
    __syncthreads();
    if (a.mode == 0) {
      for (int e = tid; e < nb * kNB; e += kCT) {
        const int i = e / kNB, j = e % kNB;
        if (j <= i) L[(int64_t)(p0 + i) * a.ldl + p0 + j] = D[i * kLd + j];
      }
    }
    // ---- (d) rows below: Pb = B (mode 1) or B D^{-T} (mode 0) ----------------
    // stage B into Pb
    batched<8>(nr * kNB,
               [&](int e) { return fel(p1 + e / kNB, p0 + min(e % kNB, nb - 1)); },
               [&](int e, double v) { Pb[(e / kNB) * kLd + e % kNB] = (e % kNB < nb) ? v : 0.0; });
    __syncthreads();
    if (a.mode == 0) {
      // out(r, j) = sum_{t <= j} B(r, t) Di(j, t), in place along row r with j
      // descending (out(r, j) only reads entries t <= j, still unchanged)
      for (int r = tid; r < nr; r += kCT) {
        double row[kNB];
#pragma unroll
        for (int t = 0; t < kNB; ++t) row[t] = Pb[r * kLd + t];
        for (int j = nb - 1; j >= 0; --j) {
          const double s = dot32r(row, Di + j * kLd, 1, 0, j);
          Pb[r * kLd + j] = s;
          L[(int64_t)(p1 + r) * a.ldl + p0 + j] = s;
        }
      }
      __syncthreads();
      // trailing lower triangle: L(i, l) -= sum_t Pb(i, t) Pb(l, t), p1 <= l <= i
      const int64_t ntri = (int64_t)nr * (nr + 1) / 2;
      for (int64_t e0 = 0; e0 < ntri; e0 += (int64_t)kCT * 4) {
        int ii[4], ll[4];
        double cur[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t e = e0 + (int64_t)q * kCT + tid;
          const int64_t ec = e < ntri ? e : 0;
          int i = (int)((sqrt(8.0 * (double)ec + 1.0) - 1.0) * 0.5);
          while ((int64_t)i * (i + 1) / 2 > ec) --i;
          while ((int64_t)(i + 1) * (i + 2) / 2 <= ec) ++i;
          ii[q] = i;
          ll[q] = (int)(ec - (int64_t)i * (i + 1) / 2);
          cur[q] = L[(int64_t)(p1 + ii[q]) * a.ldl + p1 + ll[q]];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t e = e0 + (int64_t)q * kCT + tid;
          const double s = dot32(Pb + ii[q] * kLd, 1, Pb + ll[q] * kLd, 1, 0, kNB - 1);
          if (e < ntri) L[(int64_t)(p1 + ii[q]) * a.ldl + p1 + ll[q]] = cur[q] - s;
        }
      }
    }
    __syncthreads();
    // ---- (e) elimination applied to X ----------------------------------------
    // stage X[p0:p1, 0:p1] (rows not yet final) into Xp
    batched<8>(nb * p1, [&](int e) { return X[(int64_t)(p0 + e / p1) * a.ldx + e % p1]; },
               [&](int e, double v) { Xp[(e / p1) * ldxp + e % p1] = v; });
    __syncthreads();
    // Xp <- Di Xp, in place down each column with rows descending (row i only
    // reads rows t <= i, still unchanged)
    for (int col = tid; col < p1; col += kCT) {
      double xc[kNB];
#pragma unroll
      for (int t = 0; t < kNB; ++t) xc[t] = Xp[t * ldxp + col];
      for (int i = nb - 1; i >= 0; --i) {
        const double s = dot32r(xc, Di + i * kLd, 1, 0, i);
        Xp[i * ldxp + col] = s;
        X[(int64_t)(p0 + i) * a.ldx + col] = s;
      }
    }
    __syncthreads();
    // rows below: X[p1+r, col] -= sum_t Pb(r, t) Xp(t, col), col < p1
    batched<8>(nr * p1, [&](int e) { return X[(int64_t)(p1 + e / p1) * a.ldx + e % p1]; },
               [&](int e, double v) {
                 const int r = e / p1, col = e % p1;
                 X[(int64_t)(p1 + r) * a.ldx + col] = v - dot32(Pb + r * kLd, 1, Xp + col, ldxp, 0, kNB - 1);
               });
    __syncthreads();
  }
}

}  // namespace

size_t chol_inv_lds_bytes(int c_host) {
  return ((size_t)2 * kNB * kLd + (size_t)c_host * kLd + (size_t)kNB * (c_host + 1)) * sizeof(double);
}

hipError_t chol_inv_launch(int mode, const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, double* L,
                           int64_t ldl, double* X, int64_t ldx, double shift_rel, int* status, hipStream_t stream) {
  if (c_host <= 0) return hipSuccess;
  if (c_host > kMaxC) return hipErrorInvalidValue;
  CArgs a{};
  a.G = G; a.gr = gr; a.gc = gc; a.c_host = c_host; a.c_dev = c_dev;
  a.L = L; a.ldl = ldl; a.X = X; a.ldx = ldx; a.shift_rel = shift_rel; a.mode = mode; a.status = status;
  const size_t lds = chol_inv_lds_bytes(c_host);
  hipError_t e = hipFuncSetAttribute((const void*)chol_inv_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)chol_inv_kernel, dim3(1), dim3(kCT), args, lds, stream);
}

}  // namespace idcur
