// Truncated-SVD interpolation matrix (Section 4.1: the stabilized pseudo-inverse
// of S11 in eq. (lsqr_for_T)). The SVD of the k x k factor S11 is taken by
// one-sided (Hestenes) Jacobi rotations in FP64: columns of W = S11 are rotated
// in pairs until all are orthogonal, so that W V = U diag(s) with V the
// accumulated rotations and s_i the column norms. Then
//
//   T = V diag(1 / s_i) U^T S12 = V diag(keep_i / s_i^2) (W V)^T S12,
//
// keep_i = [s_i >= thr max s], the terms with small singular values dropped.
//
// One launch per round of a sweep: the round-robin (circle) ordering pairs every
// column once per round and every two columns once per sweep, the pairs of a
// round are independent, and one wave rotates one pair. A sweep in which no
// pair needed a rotation ends the iteration: later launches return at once.
// The S11 factor of a column-pivoted QR is graded, on which one-sided Jacobi
// converges in a few sweeps.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kJacBT = 256;   // four waves, one pair each

// V = I on the kcap x kcap block (column-major, columns contiguous)
__global__ __launch_bounds__(256) void jacobi_init_kernel(double* V, int kcap, int* rot, int nsweeps) {
  const int64_t total = (int64_t)kcap * kcap;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    V[e] = (e / kcap == e % kcap) ? 1.0 : 0.0;
  if (blockIdx.x == 0)
    for (int s = threadIdx.x; s < nsweeps; s += blockDim.x) rot[s] = 0;
}

// One round of one sweep: pair `pair` of round `round` in the circle ordering of
// kp = kcap rounded up to even columns (index kp - 1 stays fixed, the others
// turn); pairs with a column at or past the device rank k are idle.
__global__ __launch_bounds__(kJacBT) void jacobi_round_kernel(double* W, double* V, int kcap, const int* k_dev,
                                                              int round, int sweep, int* rot) {
  if (sweep > 0 && rot[sweep - 1] == 0) return;   // the previous sweep rotated nothing
  const int kp = kcap + (kcap & 1);
  const int pair = blockIdx.x * (kJacBT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (pair >= kp / 2) return;
  int p, q;
  if (pair == 0) {
    p = round;
    q = kp - 1;
  } else {
    p = (round + pair) % (kp - 1);
    q = (round - pair + kp - 1) % (kp - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  const int k = k_dev ? min(*k_dev, kcap) : kcap;
  if (q >= k) return;
  double* wp = W + (size_t)p * kcap;
  double* wq = W + (size_t)q * kcap;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int i = lane; i < k; i += 64) {
    const double x = wp[i], y = wq[i];
    a = fma(x, x, a);
    b = fma(y, y, b);
    c = fma(x, y, c);
  }
  // the butterfly leaves the same bits on every lane: the decision is uniform
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const double tol = sqrt((double)k) * 1.1102230246251565e-16;
  if (!(fabs(c) > tol * sqrt(a * b))) return;
  if (lane == 0) atomicAdd(&rot[sweep], 1);
  // the rotation that makes the two columns orthogonal (smaller root of
  // t^2 + 2 zeta t - 1 = 0, zeta = (b - a) / (2c))
  const double zeta = (b - a) / (2.0 * c);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
  for (int i = lane; i < k; i += 64) {
    const double x = wp[i], y = wq[i];
    wp[i] = cs * x - sn * y;
    wq[i] = sn * x + cs * y;
  }
  double* vp = V + (size_t)p * kcap;
  double* vq = V + (size_t)q * kcap;
  for (int i = lane; i < k; i += 64) {
    const double x = vp[i], y = vq[i];
    vp[i] = cs * x - sn * y;
    vq[i] = sn * x + cs * y;
  }
}

// s_i = |W(:, i)|, then row i of P (k x ncols, ld ldp) scaled by 1 / s_i^2 where
// s_i >= thr max s, zeroed elsewhere. One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void tsvd_scale_kernel(const double* W, int kcap, const int* k_dev, double thr,
                                                          double* P, int64_t ldp, int64_t ncols,
                                                          const int* ncols_dev, double* sv) {
  __shared__ double red[16];
  const int k = k_dev ? min(*k_dev, kcap) : kcap;
  const int64_t nc = ncols_dev ? min((int64_t)*ncols_dev, ncols) : ncols;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // column norms, one wave per column
  for (int i = wv; i < k; i += 16) {
    double s = 0.0;
    for (int r = lane; r < k; r += 64) s = fma(W[(size_t)i * kcap + r], W[(size_t)i * kcap + r], s);
    s = wave_sum(s);
    if (lane == 0) sv[i] = sqrt(s);
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = threadIdx.x; i < k; i += 1024) mx = fmax(mx, sv[i]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) red[wv] = mx;
  __syncthreads();
  mx = 0.0;
  for (int w = 0; w < 16; ++w) mx = fmax(mx, red[w]);
  const double cut = thr * mx;
  for (int i = wv; i < k; i += 16) {
    const double s = sv[i];
    const double f = (s > 0.0 && s >= cut) ? 1.0 / (s * s) : 0.0;
    for (int64_t c = lane; c < nc; c += 64) P[(size_t)i * ldp + c] *= f;
  }
}

}  // namespace

int jacobi_max_sweeps() { return 16; }

hipError_t jacobi_svd_launch(double* W, double* V, int kcap, const int* k_dev, int* rot, hipStream_t stream) {
  if (kcap <= 0) return hipSuccess;
  const int ns = jacobi_max_sweeps();
  const int64_t nb = ceil_div((int64_t)kcap * kcap, 256);
  const unsigned gi = (unsigned)(nb < 4096 ? nb : 4096);
  hipLaunchKernelGGL(jacobi_init_kernel, dim3(gi), dim3(256), 0, stream, V, kcap, rot, ns);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (kcap < 2) return hipSuccess;
  const int kp = kcap + (kcap & 1);
  const unsigned grid = (unsigned)ceil_div(kp / 2, kJacBT / 64);
  for (int s = 0; s < ns; ++s)
    for (int r = 0; r < kp - 1; ++r) {
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(grid), dim3(kJacBT), 0, stream, W, V, kcap, k_dev, r, s, rot);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t tsvd_scale_launch(const double* W, int kcap, const int* k_dev, double thr, double* P, int64_t ldp,
                             int64_t ncols, const int* ncols_dev, double* sv, hipStream_t stream) {
  if (kcap <= 0) return hipSuccess;
  hipLaunchKernelGGL(tsvd_scale_kernel, dim3(1), dim3(1024), 0, stream, W, kcap, k_dev, thr, P, ldp, ncols,
                     ncols_dev, sv);
  return hipGetLastError();
}

}  // namespace idcur
