// Triangular solves with many right-hand sides, in FP64.
//
// Used for the interpolation matrix T = S11^{-1} S12 (Section 4.1: S11 is upper
// triangular and T follows by a backwards solve, one column of S12 at a time),
// for the row-interpolation matrix of the two-sided ID, and for applying the
// inverse Cholesky factors of the orthonormalisation and of the least-squares
// solve for U.
//
// Each workgroup owns NB right-hand-side columns, held in LDS as FP64 for the
// whole solve; the triangle is staged through LDS 16 columns at a time, so the
// k sequential elimination steps only touch LDS and cost one barrier each.
// Every column is solved by plain substitution in the natural order.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kBS = 16;   // triangle columns staged per block

struct TArgs {
  const double* tri; int64_t ldt; int upper, trans;
  int c_host; const int* c_dev;
  int64_t ncol_host; int ncol_sub_c; const int* ncol_dev;
  const void* B; int b_type; int64_t sbr, sbc; const int* col_idx; int col_idx_off_c;
  void* X; int x_type; int64_t sxr, sxc; int64_t xcol_lim;
  int NB;
};

__device__ __forceinline__ double ld_any(const void* p, int type, int64_t off) {
  return type == 1 ? (double)static_cast<const float*>(p)[off] : static_cast<const double*>(p)[off];
}
__device__ __forceinline__ void st_any(void* p, int type, int64_t off, double v) {
  if (type == 1) static_cast<float*>(p)[off] = (float)v;
  else static_cast<double*>(p)[off] = v;
}

__global__ __launch_bounds__(256) void trsm_kernel(TArgs a) {
  extern __shared__ __align__(16) double sm[];
  const int c = a.c_dev ? min(*a.c_dev, a.c_host) : a.c_host;
  const int64_t ncol = a.ncol_dev ? min((int64_t)*a.ncol_dev, a.ncol_host) : (a.ncol_sub_c ? a.ncol_host - c : a.ncol_host);
  const int NB = a.NB;
  const int64_t col0 = (int64_t)blockIdx.x * NB;
  if (col0 >= ncol || c <= 0) return;
  const int tid = threadIdx.x;
  const int cc = tid % NB, rg = tid / NB, RG = 256 / NB;
  const int ncc = (int)min((int64_t)NB, ncol - col0);
  double* Xs = sm;                         // c x NB
  double* Tb = sm + (size_t)a.c_host * NB; // kBS x c_host
  const int idx_off = a.col_idx_off_c ? c : 0;

  // load the right-hand sides
  for (int e = tid; e < c * NB; e += 256) {
    const int r = e / NB, q = e % NB;
    double v = 0.0;
    if (q < ncc) {
      const int64_t col = col0 + q;
      const int64_t bc = a.col_idx ? (int64_t)a.col_idx[idx_off + col] : col;
      v = ld_any(a.B, a.b_type, (int64_t)r * a.sbr + bc * a.sbc);
    }
    Xs[r * NB + q] = v;
  }

  // op(T)(r, i): upper/lower as given, transposed on request
  auto tel = [&](int r, int i) -> double {
    return a.trans ? a.tri[(int64_t)i * a.ldt + r] : a.tri[(int64_t)r * a.ldt + i];
  };
  const bool up = a.upper;   // the effective triangle is upper <=> upper (trans flips roles below)
  // For op(T) = T^T of a lower T the system is upper, and vice versa.
  const bool eff_upper = a.trans ? !up : up;

  const int nblk = (c + kBS - 1) / kBS;
  for (int b = 0; b < nblk; ++b) {
    // block of step indices, in elimination order
    const int i0 = eff_upper ? max(0, c - (b + 1) * kBS) : b * kBS;
    const int i1 = eff_upper ? c - b * kBS : min(c, (b + 1) * kBS);
    __syncthreads();
    // stage op(T)(r, i) for i in [i0, i1), all r
    const int w = i1 - i0;
    for (int e = tid; e < w * c; e += 256) {
      int ii, r;
      if (a.trans) { ii = e / c; r = e % c; }      // contiguous in r
      else { r = e / w; ii = e % w; }               // contiguous in i
      Tb[ii * a.c_host + r] = tel(r, i0 + ii);
    }
    __syncthreads();
    for (int s = 0; s < w; ++s) {
      const int ii = eff_upper ? (w - 1 - s) : s;
      const int i = i0 + ii;
      const double* tc = Tb + (size_t)ii * a.c_host;
      const double xi = Xs[i * NB + cc] / tc[i];
      if (rg == 0 && cc < ncc && (a.xcol_lim <= 0 || col0 + cc < a.xcol_lim)) st_any(a.X, a.x_type, (int64_t)i * a.sxr + (col0 + cc) * a.sxc, xi);
      if (eff_upper) {
        for (int r = rg; r < i; r += RG) Xs[r * NB + cc] -= tc[r] * xi;
      } else {
        for (int r = i + 1 + rg; r < c; r += RG) Xs[r * NB + cc] -= tc[r] * xi;
      }
      __syncthreads();
    }
  }
}

}  // namespace

hipError_t trsm_launch(const TrsmDesc& d, hipStream_t stream) {
  if (d.ncol_host <= 0 || d.c_host <= 0) return hipSuccess;
  TArgs a{};
  a.tri = d.tri; a.ldt = d.ldt; a.upper = d.upper; a.trans = d.trans;
  a.c_host = d.c_host; a.c_dev = d.c_dev;
  a.ncol_host = d.ncol_host; a.ncol_sub_c = d.ncol_sub_c; a.ncol_dev = d.ncol_dev;
  a.B = d.B; a.b_type = d.b_type; a.sbr = d.sbr; a.sbc = d.sbc; a.col_idx = d.col_idx;
  a.col_idx_off_c = d.col_idx_off_c;
  a.X = d.X; a.x_type = d.x_type; a.sxr = d.sxr; a.sxc = d.sxc; a.xcol_lim = d.xcol_lim;
  a.NB = d.c_host <= 300 ? 32 : 16;
  const size_t lds = ((size_t)d.c_host * a.NB + (size_t)kBS * d.c_host) * sizeof(double);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)trsm_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)ceil_div(d.ncol_host, a.NB);
  hipLaunchKernelGGL(trsm_kernel, dim3(grid), dim3(256), lds, stream, a);
  return hipGetLastError();
}

namespace {
template <typename T>
__global__ void gather_s11_kernel(const T* S, int64_t ldS, const int* J, int c_host, const int* c_dev, double* out) {
  const int c = c_dev ? min(*c_dev, c_host) : c_host;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)c * c; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / c), s = (int)(e % c);
    out[(int64_t)r * c_host + s] = (double)S[(int64_t)r * ldS + J[s]];
  }
}
}  // namespace

hipError_t gather_s11_launch(int dtype, const void* S, int64_t ldS, const int* J, int c_host, const int* c_dev,
                             double* out, hipStream_t stream) {
  if (c_host <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div((int64_t)c_host * c_host, 256), 1024);
  if (dtype == 1)
    hipLaunchKernelGGL(gather_s11_kernel<float>, dim3(grid), dim3(256), 0, stream, static_cast<const float*>(S), ldS, J,
                       c_host, c_dev, out);
  else
    hipLaunchKernelGGL(gather_s11_kernel<double>, dim3(grid), dim3(256), 0, stream, static_cast<const double*>(S), ldS,
                       J, c_host, c_dev, out);
  return hipGetLastError();
}

}  // namespace idcur
