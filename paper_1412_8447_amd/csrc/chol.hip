// Cholesky factorisation G = L L^T of a small SPD matrix (c <= 544), FP64.
//
// Serves the Cholesky-QR orthonormalisation of the sketch between power steps
// (orth in Section 5.3) and the QR factorisation of R^T used to solve
// U R = V* in the least-squares sense (Section 4.3).
//
// One workgroup, right-looking by 32-column panels:
//   (a) the 32 x 32 diagonal block is factored by one wave, one row per lane,
//       entirely in registers (column broadcasts by lane shuffles);
//   (b) the rows below solve against that block (one row per thread), and the
//       resulting panel is kept in LDS;
//   (c) the trailing lower triangle, held in the output buffer (L2 resident),
//       is updated with the panel's outer product read from LDS.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kCT = 256;
constexpr int kNB = 32;
constexpr int kMaxC = 544;

__global__ __launch_bounds__(kCT) void chol_kernel(const double* G, int64_t ldg, int c_host, const int* c_dev,
                                                   double* L, int64_t ldl, double shift_rel, int* status) {
  extern __shared__ __align__(16) double sm[];
  double* Ld = sm;                         // kNB x (kNB+1)
  double* Ps = sm + kNB * (kNB + 1);       // (c_host) x kNB panel rows
  __shared__ double smax[kCT / 64];
  const int c = c_dev ? min(*c_dev, c_host) : c_host;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  // shift relative to the largest diagonal entry
  double mx = 0.0;
  for (int i = tid; i < c; i += kCT) mx = fmax(mx, G[(int64_t)i * ldg + i]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) smax[wv] = mx;
  __syncthreads();
  mx = 0.0;
  for (int w = 0; w < kCT / 64; ++w) mx = fmax(mx, smax[w]);
  const double sh = shift_rel * mx;
  // L <- lower(G) (+ shift on the diagonal), zeros above
  for (int64_t e = tid; e < (int64_t)c * c; e += kCT) {
    const int i = (int)(e / c), j = (int)(e % c);
    double v = 0.0;
    if (j <= i) v = G[(int64_t)i * ldg + j] + (i == j ? sh : 0.0);
    L[(int64_t)i * ldl + j] = v;
  }
  __syncthreads();

  for (int p0 = 0; p0 < c; p0 += kNB) {
    const int nb = min(kNB, c - p0);
    const int p1 = p0 + nb;
    const int nr = c - p1;
    // (a) diagonal block, wave 0, row `lane` of the block
    if (wv == 0) {
      double a[kNB];
      const bool own = lane < nb;
#pragma unroll
      for (int k = 0; k < kNB; ++k) a[k] = (own && k <= lane && k < nb) ? L[(int64_t)(p0 + lane) * ldl + p0 + k] : 0.0;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (j < nb) {
          double d = __shfl(a[j], j, 64);
          if (!(d > 0.0)) {
            if (lane == 0) set_status(status, ST_NONFINITE);
            d = 1e-300;
          }
          const double s = sqrt(d);
          if (lane == j) a[j] = s;
          else if (lane > j) a[j] /= s;
#pragma unroll
          for (int k = j + 1; k < kNB; ++k) {
            const double lkj = __shfl(a[j], k, 64);
            if (lane >= k && lane > j && k < nb) a[k] -= a[j] * lkj;
          }
        }
      }
      if (own) {
#pragma unroll
        for (int k = 0; k < kNB; ++k) {
          if (k <= lane && k < nb) {
            Ld[lane * (kNB + 1) + k] = a[k];
            L[(int64_t)(p0 + lane) * ldl + p0 + k] = a[k];
          }
        }
      }
    }
    __syncthreads();
    // (b) panel rows below: x L_D^T = row  (forward substitution along the row)
    for (int r = tid; r < nr; r += kCT) {
      double x[kNB];
#pragma unroll
      for (int k = 0; k < kNB; ++k) x[k] = (k < nb) ? L[(int64_t)(p1 + r) * ldl + p0 + k] : 0.0;
#pragma unroll
      for (int j = 0; j < kNB; ++j) {
        if (j < nb) {
          double s = x[j];
#pragma unroll
          for (int i = 0; i < j; ++i) s -= x[i] * Ld[j * (kNB + 1) + i];
          x[j] = s / Ld[j * (kNB + 1) + j];
        }
      }
#pragma unroll
      for (int k = 0; k < kNB; ++k) {
        if (k < nb) {
          Ps[r * kNB + k] = x[k];
          L[(int64_t)(p1 + r) * ldl + p0 + k] = x[k];
        }
      }
    }
    __syncthreads();
    // (c) trailing update of the lower triangle
    for (int64_t e = tid; e < (int64_t)nr * nr; e += kCT) {
      const int i = (int)(e / nr), j = (int)(e % nr);
      if (j <= i) {
        double s = 0.0;
        for (int k = 0; k < nb; ++k) s += Ps[i * kNB + k] * Ps[j * kNB + k];
        L[(int64_t)(p1 + i) * ldl + p1 + j] -= s;
      }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t chol_launch(const double* G, int64_t ldg, int c_host, const int* c_dev, double* L, int64_t ldl,
                       double shift_rel, int* status, hipStream_t stream) {
  if (c_host <= 0) return hipSuccess;
  if (c_host > kMaxC) return hipErrorInvalidValue;
  const size_t lds = ((size_t)kNB * (kNB + 1) + (size_t)c_host * kNB) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void*)chol_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(kCT), lds, stream, G, ldg, c_host, c_dev, L, ldl, shift_rel, status);
  return hipGetLastError();
}

}  // namespace idcur
