// Small bandwidth kernels: the Gaussian sketch matrix (Philox4x32-10 +
// Box-Muller), strided copies, the gathers C = A(:, J(1:k)) and
// R = A(I(1:k), :) of the CUR-ID (Section 3, eq. (choice_C_and_R)), and a
// zero fill.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4x32 Philox bijection,
// multipliers 0xD2511F53 / 0xCD9E8D57, key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint2 key) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { key.x += 0x9E3779B9u; key.y += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * ctr.x, hi0 = __umulhi(0xD2511F53u, ctr.x);
    const uint32_t lo1 = 0xCD9E8D57u * ctr.z, hi1 = __umulhi(0xCD9E8D57u, ctr.z);
    ctr = make_uint4(hi1 ^ ctr.y ^ key.x, lo1, hi0 ^ ctr.w ^ key.y, lo0);
  }
  return ctr;
}

// Counter g yields elements 4g .. 4g+3 of the row-major rows x cols matrix. With
// colmajor (cols % 4 == 0, out column-major: sor == 1) consecutive threads take
// the same four columns of consecutive rows, so that the stores coalesce; the
// values are the same either way.
template <typename T>
__global__ void gaussian_kernel(int64_t rows, int64_t cols, uint64_t seed, uint64_t sid, T* out, int64_t sor,
                                int64_t soc, int colmajor) {
  const int64_t total = rows * cols;
  const int64_t ngroups = (total + 3) / 4;
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ngroups; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = colmajor ? (e % rows) * (cols / 4) + e / rows : e;
    const uint4 x = philox4x32_10(make_uint4((uint32_t)g, (uint32_t)(g >> 32), (uint32_t)sid, 0u), key);
    const uint32_t w[4] = {x.x, x.y, x.z, x.w};
    double z[4];
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
      const double u1 = ((double)w[2 * pr] + 1.0) * 2.3283064365386963e-10;   // 2^-32
      const double u2 = (double)w[2 * pr + 1] * 2.3283064365386963e-10;
      const double rho = sqrt(-2.0 * log(u1));
      const double th = (2.0 * 3.141592653589793) * u2;
      z[2 * pr] = rho * cos(th);
      z[2 * pr + 1] = rho * sin(th);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t f = g * 4 + q;
      if (f < total) {
        const int64_t r = f / cols, i = f % cols;
        out[r * sor + i * soc] = (T)z[q];
      }
    }
  }
}

// out(j, i) = (float) in(i, j) for i < rows, j < cols; out is cols x ldo
// (row-major) and its columns [rows, ldo) are zeroed.
__global__ void f64_to_f32_t_kernel(int64_t rows, int64_t cols, const double* in, int64_t ldi, float* out,
                                    int64_t ldo) {
  const int64_t total = cols * ldo;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / ldo, i = e % ldo;
    out[e] = i < rows ? (float)in[i * ldi + j] : 0.0f;
  }
}

template <typename T>
__global__ void copy2d_kernel(int64_t rows, int64_t cols, const T* in, int64_t sir, int64_t sic, T* out, int64_t sor,
                              int64_t soc) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    out[r * sor + c * soc] = in[r * sir + c * sic];
  }
}

// out(r, c) = in(r, c) with in's rows and out's columns contiguous (a
// transpose): 32 x 32 tiles through LDS, so reads and writes are both coalesced.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(int64_t rows, int64_t cols, const T* in, int64_t sir, T* out,
                                                        int64_t soc) {
  __shared__ T tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int64_t r = r0 + ty + k, c = c0 + tx;
    if (r < rows && c < cols) tile[ty + k][tx] = in[r * sir + c];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; k += 8) {
    const int64_t c = c0 + ty + k, r = r0 + tx;
    if (r < rows && c < cols) out[r + c * soc] = tile[tx][ty + k];
  }
}

template <typename T, typename TO>
__global__ void gather_cols_kernel(int64_t m, const T* A, int64_t lda, const int* idx, int k_host, const int* k_dev,
                                   TO* out, int64_t ldo) {
  const int k = k_dev ? min(*k_dev, k_host) : k_host;
  const int64_t total = m * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k, s = e % k;
    out[i * ldo + s] = (TO)A[i * lda + idx[s]];
  }
}

template <typename T, typename TO>
__global__ void gather_rows_kernel(int64_t n, const T* A, int64_t lda, const int* idx, int k_host, const int* k_dev,
                                   TO* out, int64_t ldo) {
  const int k = k_dev ? min(*k_dev, k_host) : k_host;
  const int64_t total = (int64_t)k * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / n, j = e % n;
    out[s * ldo + j] = (TO)A[(int64_t)idx[s] * lda + j];
  }
}

__global__ void fill_int_kernel(int* p, int64_t n, int v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

// inv[idx[s]] = s for s < n (idx a permutation of 0..n-1); out-of-range
// entries are skipped and flagged.
__global__ void invert_perm_kernel(const int* idx, int64_t n, int* inv, int* status) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    const int c = idx[s];
    if (c < 0 || c >= n) {
      set_status(status, ST_BADINDEX);
      continue;
    }
    inv[c] = (int)s;
  }
}

// out(i, c) = alpha * in(i, p[c]) (+ out(i, c) when accumulate), c < ncols; an
// out-of-range p[c] reads column 0 and is flagged.
template <typename T>
__global__ void gather_cols_scaled_kernel(int64_t m, const T* in, int64_t ldi, int64_t nin, const int* p, int64_t ncols,
                                          double alpha, int accumulate, T* out, int64_t ldo, int* status) {
  const int64_t total = m * ncols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / ncols, c = e % ncols;
    int s = p[c];
    if (s < 0 || s >= nin) {
      set_status(status, ST_BADINDEX);
      s = 0;
    }
    const double v = alpha * (double)in[i * ldi + s];
    T* o = out + i * ldo + c;
    *o = accumulate ? (T)((double)*o + v) : (T)v;
  }
}

__global__ void zero_kernel(uint32_t* p, size_t nwords) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < nwords; e += (size_t)gridDim.x * blockDim.x) p[e] = 0u;
}

// P (c_host x c_host, row-major ldp) = the active c x c block of G (c = min(*c_dev,
// c_host)), identity outside it; lower_only zeroes the part above the diagonal;
// *shift (when given) is added to the active diagonal.
__global__ void pad_square_kernel(const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev,
                                  int lower_only, const double* shift, double* P, int64_t ldp) {
  const int c = c_dev ? min(*c_dev, c_host) : c_host;
  const double sh = shift ? *shift : 0.0;
  const int64_t total = (int64_t)c_host * c_host;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / c_host), j = (int)(e % c_host);
    double v;
    if (i < c && j < c) v = (lower_only && j > i) ? 0.0 : G[(int64_t)i * gr + (int64_t)j * gc] + (i == j ? sh : 0.0);
    else v = i == j ? 1.0 : 0.0;
    P[(int64_t)i * ldp + j] = v;
  }
}

// *out = rel * max_i G(i, i) over the active diagonal (one workgroup).
__global__ __launch_bounds__(256) void diag_shift_kernel(const double* G, int64_t gr, int64_t gc, int c_host,
                                                         const int* c_dev, double rel, double* out) {
  __shared__ double ws[4];
  const int c = c_dev ? min(*c_dev, c_host) : c_host;
  double mx = 0.0;
  for (int i = threadIdx.x; i < c; i += 256) mx = fmax(mx, G[(int64_t)i * gr + (int64_t)i * gc]);
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) *out = rel * fmax(fmax(ws[0], ws[1]), fmax(ws[2], ws[3]));
}

// Y += (*s) X over rows x cols (row-major, leading dimensions ldx, ldy): an
// update whose weight was computed on the device.
__global__ void axpy_dev_kernel(const double* s, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t rows,
                                int64_t cols) {
  const double w = *s;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e % cols;
    Y[i * ldy + j] += w * X[i * ldx + j];
  }
}

__global__ void zero2d_kernel(double* p, int64_t rows, int64_t cols, int64_t ld) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    p[(e / cols) * ld + e % cols] = 0.0;
}

__global__ void add_gathered_kernel(const double* Q, int64_t ldq, const int* J, int ka_host, const int* ka_dev,
                                    int kb_host, const int* kb_dev, double* out, int64_t ldo) {
  const int ka = ka_dev ? min(*ka_dev, ka_host) : ka_host;
  const int kb = kb_dev ? min(*kb_dev, kb_host) : kb_host;
  const int64_t total = (int64_t)ka * kb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / kb, b = e % kb;
    out[a * ldo + b] += Q[a * ldq + J[b]];
  }
}

// V (n x kcap, ld ldv): row J[p] is e_p for p < k and column p - k of T for
// p >= k (zeros past k): the rows of [I_k; T^T] in the order J. 64 x 64 tiles of
// (r, p) pass through LDS, so that T is read along p and V written along r,
// both coalesced.
template <typename T>
__global__ __launch_bounds__(256) void build_v_kernel(const T* Tm, int64_t ldt, const int* J, int64_t n, int kcap,
                                                      const int* k_dev, double* V, int64_t ldv) {
  __shared__ double tile[64][65];
  const int k = k_dev ? min(*k_dev, kcap) : kcap;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int r0 = (int)blockIdx.y * 64;
  const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
  for (int i = hi; i < 64; i += 4) {
    const int r = r0 + i;
    const int64_t p = p0 + lo;
    double v = 0.0;
    if (r < kcap && p < n) {
      if (p < k) v = (r == p) ? 1.0 : 0.0;
      else if (r < k) v = (double)Tm[(int64_t)r * ldt + (p - k)];
    }
    tile[i][lo] = v;
  }
  __syncthreads();
  for (int i = hi; i < 64; i += 4) {
    const int64_t p = p0 + i;
    const int r = r0 + lo;
    if (p < n && r < kcap) V[(int64_t)J[p] * ldv + r] = tile[lo][i];
  }
}

template <typename T>
__global__ void build_vstar_kernel(const T* Tm, int64_t ldt, const int* J, int64_t n, int kcap, const int* k_dev,
                                   double* W, int64_t ldw) {
  const int k = k_dev ? min(*k_dev, kcap) : kcap;
  const int64_t total = (int64_t)kcap * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, p = e % n;
    double v = 0.0;
    if (r < k) v = (p < k) ? ((r == p) ? 1.0 : 0.0) : (double)Tm[r * ldt + (p - k)];
    W[r * ldw + J[p]] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void sumsq_kernel(int64_t m, int64_t n, const T* A, int64_t lda, double* part) {
  __shared__ double ws[4];
  double s = 0.0;
  const int64_t total = m * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)A[(e / n) * lda + e % n];
    s += v * v;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

__global__ __launch_bounds__(256) void sum1024(const double* part, double* out) {
  __shared__ double ws[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < 1024; i += 256) s += part[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

template <typename T>
__global__ void gather_s11_kernel(const T* S, int64_t ldS, const int* J, int c_host, const int* c_dev, double* out) {
  const int c = c_dev ? min(*c_dev, c_host) : c_host;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)c * c; e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / c), s = (int)(e % c);
    out[(int64_t)r * c_host + s] = (double)S[(int64_t)r * ldS + J[s]];
  }
}

template <typename T>
__global__ void gather_s12_kernel(const T* S, int64_t ldS, const int* J, int64_t n, int c_host, const int* c_dev,
                                  double* out, int64_t ldo, int* ncols_out) {
  const int c = c_dev ? min(*c_dev, c_host) : c_host;
  const int64_t nc = n - c;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ncols_out = (int)nc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)c * nc; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / nc, t = e % nc;
    out[r * ldo + t] = (double)S[r * ldS + J[c + t]];
  }
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 8192)); }

}  // namespace

hipError_t gaussian_launch(int dtype, int64_t rows, int64_t cols, uint64_t seed, uint64_t sid, void* out, int64_t sor,
                           int64_t soc, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const unsigned g = grid_for(ceil_div(rows * cols, 4));
  const int colmajor = sor == 1 && soc != 1 && cols % 4 == 0 && rows > 1;
  if (dtype == 1)
    hipLaunchKernelGGL(gaussian_kernel<float>, dim3(g), dim3(256), 0, stream, rows, cols, seed, sid,
                       static_cast<float*>(out), sor, soc, colmajor);
  else
    hipLaunchKernelGGL(gaussian_kernel<double>, dim3(g), dim3(256), 0, stream, rows, cols, seed, sid,
                       static_cast<double*>(out), sor, soc, colmajor);
  return hipGetLastError();
}

hipError_t copy2d_launch(int dtype, int64_t rows, int64_t cols, const void* in, int64_t sir, int64_t sic, void* out,
                         int64_t sor, int64_t soc, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int64_t gx = ceil_div(cols, 32), gy = ceil_div(rows, 32);
  if (sic == 1 && sor == 1 && rows > 1 && cols > 1 && gx <= 0x7fffffff && gy <= 65535) {
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (dtype == 1)
      hipLaunchKernelGGL(transpose_kernel<float>, grid, dim3(256), 0, stream, rows, cols,
                         static_cast<const float*>(in), sir, static_cast<float*>(out), soc);
    else
      hipLaunchKernelGGL(transpose_kernel<double>, grid, dim3(256), 0, stream, rows, cols,
                         static_cast<const double*>(in), sir, static_cast<double*>(out), soc);
    return hipGetLastError();
  }
  const unsigned g = grid_for(rows * cols);
  if (dtype == 1)
    hipLaunchKernelGGL(copy2d_kernel<float>, dim3(g), dim3(256), 0, stream, rows, cols, static_cast<const float*>(in), sir,
                       sic, static_cast<float*>(out), sor, soc);
  else
    hipLaunchKernelGGL(copy2d_kernel<double>, dim3(g), dim3(256), 0, stream, rows, cols, static_cast<const double*>(in),
                       sir, sic, static_cast<double*>(out), sor, soc);
  return hipGetLastError();
}

hipError_t f64_to_f32_t_launch(int64_t rows, int64_t cols, const double* in, int64_t ldi, float* out, int64_t ldo,
                               hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (ldo < rows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f64_to_f32_t_kernel, dim3(grid_for(cols * ldo)), dim3(256), 0, stream, rows, cols, in, ldi, out,
                     ldo);
  return hipGetLastError();
}

hipError_t invert_perm_launch(const int* idx, int64_t n, int* inv, int* status, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  // entries no index points to stay -1 (then flagged by the gathers that read them)
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n)), dim3(256), 0, stream, inv, n, -1);
  hipLaunchKernelGGL(invert_perm_kernel, dim3(grid_for(n)), dim3(256), 0, stream, idx, n, inv, status);
  return hipGetLastError();
}

hipError_t gather_cols_scaled_launch(int dtype, int64_t m, const void* in, int64_t ldi, int64_t nin, const int* p,
                                     int64_t ncols, double alpha, int accumulate, void* out, int64_t ldo, int* status,
                                     hipStream_t stream) {
  if (m <= 0 || ncols <= 0) return hipSuccess;
  const unsigned g = grid_for(m * ncols);
  if (dtype == 1)
    hipLaunchKernelGGL(gather_cols_scaled_kernel<float>, dim3(g), dim3(256), 0, stream, m, static_cast<const float*>(in),
                       ldi, nin, p, ncols, alpha, accumulate, static_cast<float*>(out), ldo, status);
  else
    hipLaunchKernelGGL(gather_cols_scaled_kernel<double>, dim3(g), dim3(256), 0, stream, m,
                       static_cast<const double*>(in), ldi, nin, p, ncols, alpha, accumulate, static_cast<double*>(out),
                       ldo, status);
  return hipGetLastError();
}

hipError_t gather_cols_launch(int dtype, int64_t m, const void* A, int64_t lda, const int* idx, int k_host,
                              const int* k_dev, void* out, int64_t ldo, int out_type, hipStream_t stream) {
  if (m <= 0 || k_host <= 0) return hipSuccess;
  const unsigned g = grid_for(m * k_host);
  if (dtype == 1 && out_type == 1)
    hipLaunchKernelGGL((gather_cols_kernel<float, float>), dim3(g), dim3(256), 0, stream, m, static_cast<const float*>(A), lda,
                       idx, k_host, k_dev, static_cast<float*>(out), ldo);
  else if (dtype == 1 && out_type == 0)
    hipLaunchKernelGGL((gather_cols_kernel<float, double>), dim3(g), dim3(256), 0, stream, m, static_cast<const float*>(A),
                       lda, idx, k_host, k_dev, static_cast<double*>(out), ldo);
  else if (dtype == 0 && out_type == 0)
    hipLaunchKernelGGL((gather_cols_kernel<double, double>), dim3(g), dim3(256), 0, stream, m,
                       static_cast<const double*>(A), lda, idx, k_host, k_dev, static_cast<double*>(out), ldo);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t gather_rows_launch(int dtype, int64_t n, const void* A, int64_t lda, const int* idx, int k_host,
                              const int* k_dev, void* out, int64_t ldo, int out_type, hipStream_t stream) {
  if (n <= 0 || k_host <= 0) return hipSuccess;
  const unsigned g = grid_for(n * k_host);
  if (dtype == 1 && out_type == 1)
    hipLaunchKernelGGL((gather_rows_kernel<float, float>), dim3(g), dim3(256), 0, stream, n, static_cast<const float*>(A), lda,
                       idx, k_host, k_dev, static_cast<float*>(out), ldo);
  else if (dtype == 1 && out_type == 0)
    hipLaunchKernelGGL((gather_rows_kernel<float, double>), dim3(g), dim3(256), 0, stream, n, static_cast<const float*>(A),
                       lda, idx, k_host, k_dev, static_cast<double*>(out), ldo);
  else if (dtype == 0 && out_type == 0)
    hipLaunchKernelGGL((gather_rows_kernel<double, double>), dim3(g), dim3(256), 0, stream, n,
                       static_cast<const double*>(A), lda, idx, k_host, k_dev, static_cast<double*>(out), ldo);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t zero_launch(void* p, size_t bytes, hipStream_t stream) {
  if (bytes == 0) return hipSuccess;
  const size_t nw = bytes / 4;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for((int64_t)nw)), dim3(256), 0, stream, static_cast<uint32_t*>(p), nw);
  return hipGetLastError();
}

hipError_t build_v_launch(int dtype, const void* T, int64_t ldt, const int* J, int64_t n, int kcap, const int* k_dev,
                          double* V, int64_t ldv, hipStream_t stream) {
  if (n <= 0 || kcap <= 0) return hipSuccess;
  if (ldv < kcap || ceil_div(n, 64) > 0x7fffffff || ceil_div(kcap, 64) > 65535) return hipErrorInvalidValue;
  const dim3 g((unsigned)ceil_div(n, 64), (unsigned)ceil_div(kcap, 64));
  if (dtype == 1)
    hipLaunchKernelGGL(build_v_kernel<float>, g, dim3(256), 0, stream, static_cast<const float*>(T), ldt, J, n, kcap,
                       k_dev, V, ldv);
  else
    hipLaunchKernelGGL(build_v_kernel<double>, g, dim3(256), 0, stream, static_cast<const double*>(T), ldt, J, n,
                       kcap, k_dev, V, ldv);
  return hipGetLastError();
}

hipError_t gather_s11_launch(int dtype, const void* S, int64_t ldS, const int* J, int c_host, const int* c_dev,
                             double* out, hipStream_t stream) {
  if (c_host <= 0) return hipSuccess;
  const unsigned g = grid_for((int64_t)c_host * c_host);
  if (dtype == 1)
    hipLaunchKernelGGL(gather_s11_kernel<float>, dim3(g), dim3(256), 0, stream, static_cast<const float*>(S), ldS, J,
                       c_host, c_dev, out);
  else
    hipLaunchKernelGGL(gather_s11_kernel<double>, dim3(g), dim3(256), 0, stream, static_cast<const double*>(S), ldS, J,
                       c_host, c_dev, out);
  return hipGetLastError();
}

hipError_t gather_s12_launch(int dtype, const void* S, int64_t ldS, const int* J, int64_t n, int c_host,
                             const int* c_dev, double* out, int64_t ldo, int* ncols_out, hipStream_t stream) {
  const unsigned g = grid_for((int64_t)c_host * n);
  if (dtype == 1)
    hipLaunchKernelGGL(gather_s12_kernel<float>, dim3(g), dim3(256), 0, stream, static_cast<const float*>(S), ldS, J, n,
                       c_host, c_dev, out, ldo, ncols_out);
  else
    hipLaunchKernelGGL(gather_s12_kernel<double>, dim3(g), dim3(256), 0, stream, static_cast<const double*>(S), ldS, J,
                       n, c_host, c_dev, out, ldo, ncols_out);
  return hipGetLastError();
}

hipError_t build_vstar_launch(int dtype, const void* T, int64_t ldt, const int* J, int64_t n, int kcap,
                              const int* k_dev, double* W, int64_t ldw, hipStream_t stream) {
  if (n <= 0 || kcap <= 0) return hipSuccess;
  const unsigned g = grid_for((int64_t)kcap * n);
  if (dtype == 1)
    hipLaunchKernelGGL(build_vstar_kernel<float>, dim3(g), dim3(256), 0, stream, static_cast<const float*>(T), ldt, J, n,
                       kcap, k_dev, W, ldw);
  else
    hipLaunchKernelGGL(build_vstar_kernel<double>, dim3(g), dim3(256), 0, stream, static_cast<const double*>(T), ldt, J,
                       n, kcap, k_dev, W, ldw);
  return hipGetLastError();
}

hipError_t sumsq_launch(int dtype, int64_t m, int64_t n, const void* A, int64_t lda, double* part, double* out,
                        hipStream_t stream) {
  if (dtype == 1)
    hipLaunchKernelGGL(sumsq_kernel<float>, dim3(1024), dim3(256), 0, stream, m, n, static_cast<const float*>(A), lda, part);
  else
    hipLaunchKernelGGL(sumsq_kernel<double>, dim3(1024), dim3(256), 0, stream, m, n, static_cast<const double*>(A), lda,
                       part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum1024, dim3(1), dim3(256), 0, stream, part, out);
  return hipGetLastError();
}

hipError_t pad_square_launch(const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, int lower_only,
                             const double* shift, double* P, int64_t ldp, hipStream_t stream) {
  if (c_host <= 0) return hipSuccess;
  hipLaunchKernelGGL(pad_square_kernel, dim3(grid_for((int64_t)c_host * c_host)), dim3(256), 0, stream, G, gr, gc,
                     c_host, c_dev, lower_only, shift, P, ldp);
  return hipGetLastError();
}

hipError_t diag_shift_launch(const double* G, int64_t gr, int64_t gc, int c_host, const int* c_dev, double rel,
                             double* out, hipStream_t stream) {
  hipLaunchKernelGGL(diag_shift_kernel, dim3(1), dim3(256), 0, stream, G, gr, gc, c_host, c_dev, rel, out);
  return hipGetLastError();
}

hipError_t axpy_dev_launch(const double* s, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t rows,
                           int64_t cols, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_dev_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, stream, s, X, ldx, Y, ldy, rows, cols);
  return hipGetLastError();
}

hipError_t zero2d_launch(double* p, int64_t rows, int64_t cols, int64_t ld, hipStream_t stream) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero2d_kernel, dim3(grid_for(rows * cols)), dim3(256), 0, stream, p, rows, cols, ld);
  return hipGetLastError();
}

hipError_t add_gathered_launch(const double* Q, int64_t ldq, const int* J, int ka_host, const int* ka_dev, int kb_host,
                               const int* kb_dev, double* out, int64_t ldo, hipStream_t stream) {
  if (ka_host <= 0 || kb_host <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_gathered_kernel, dim3(grid_for((int64_t)ka_host * kb_host)), dim3(256), 0, stream, Q, ldq, J,
                     ka_host, ka_dev, kb_host, kb_dev, out, ldo);
  return hipGetLastError();
}

}  // namespace idcur
