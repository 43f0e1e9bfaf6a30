// Host side of the 16-bit sketch GEMM (kernel in gemm16_kernel.hpp), the packing
// of the thin operand into 16-bit B^T, the FP16 prescale factor, and the fixed-
// order split-K reduction. BF16 instantiations live here, FP16 ones in
// gemm16_f16.hip.
#include "gemm16_kernel.hpp"
#include "gemm16w_kernel.hpp"

#include <cmath>

namespace idcur {
namespace g16 {
hipError_t launch_bf16(int nt, const Args& a, bool akc, hipStream_t s) { return launch_h<false>(nt, a, akc, s); }
hipError_t launch_wide_bf16(const Args& a, bool akc, int cb, hipStream_t s) { return launch_wide<false>(a, akc, cb, s); }
}  // namespace g16

namespace {

using g16::BK;
using g16::BM;

// Columns per workgroup (16 * nt) and column tiles: the 16-column blocks of N are
// spread evenly over the fewest tiles of at most 16 blocks.
void pick_cols(int64_t N, int* nt, int* gy) {
  const int64_t t = std::max<int64_t>(1, ceil_div(N, 16));
  const int64_t y = ceil_div(t, 16);
  int64_t per = ceil_div(t, y);
  per += per & 1;
  *nt = (int)std::max<int64_t>(2, per);
  *gy = (int)y;
}

// Sum of the split-K partials in split order (FP64), written as FP32.
__global__ __launch_bounds__(256) void reduce16_kernel(const float* part, int splitk, int64_t M, int64_t N, float* C,
                                                       int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splitk; ++z) s += (double)part[(int64_t)z * total + e];
    C[(e / N) * ldc + e % N] = (float)s;
  }
}

// out(j, k) = round16(in(j, k)), in(j, k) = in[j*sj + k*sk], for j < rows,
// k < cols; zero for rows <= j < rows_pad or cols <= k < cols_pad. 64 x 64 tiles
// through LDS so that both the strided read and the row-major write coalesce.
template <bool H>
__global__ __launch_bounds__(256) void pack16_kernel(int64_t rows, int64_t cols, const float* in, int64_t sj,
                                                     int64_t sk, int64_t rows_pad, int64_t cols_pad, uint16_t* out,
                                                     int64_t ldo) {
  __shared__ float t[64][65];
  const int64_t j0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    int jj, kk;
    if (sk == 1) { jj = idx >> 6; kk = idx & 63; }
    else { kk = idx >> 6; jj = idx & 63; }
    const int64_t j = j0 + jj, k = k0 + kk;
    t[jj][kk] = (j < rows && k < cols) ? in[j * sj + k * sk] : 0.0f;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int jj = idx >> 6, kk = idx & 63;
    const int64_t j = j0 + jj, k = k0 + kk;
    if (j < rows_pad && k < cols_pad) {
      uint16_t b;
      if constexpr (H) b = __builtin_bit_cast(uint16_t, (_Float16)t[jj][kk]);
      else b = __builtin_bit_cast(uint16_t, (__bf16)t[jj][kk]);
      out[j * ldo + k] = b;
    }
  }
}

// Chunk-major packing for the wide kernel: thread w writes the 16-byte word of
// chunk c = w / npad, column j = w % npad (eight consecutive k rounded to 16
// bits, the same rounding as pack16_kernel).
template <bool H>
__global__ __launch_bounds__(256) void pack16c_kernel(int64_t rows, int64_t cols, const float* in, int64_t sj,
                                                      int64_t sk, int64_t npad, int64_t words, g16::u32x4* out) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= words) return;
  const int64_t j = w % npad, c = w / npad;
  float f[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = 8 * c + e;
    f[e] = (j < rows && k < cols) ? in[j * sj + k * sk] : 0.0f;
  }
  out[w] = g16::pack8<H>(f, 1.0f);
}

// Per-block maximum of |A| over a rows x cols row-major matrix (ld lda).
__global__ __launch_bounds__(256) void amax_kernel(int64_t rows, int64_t cols, const float* A, int64_t lda,
                                                   float* part) {
  __shared__ float ws[4];
  float mx = 0.0f;
  const bool vec = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const float* row = A + r * lda;
    if (vec) {
      const int64_t c4 = cols / 4;
      for (int64_t c = threadIdx.x; c < c4; c += 256) {
        const float4 v = reinterpret_cast<const float4*>(row)[c];
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        // a NaN makes fmaxf return the other operand; flag it through +inf
        if (v.x != v.x || v.y != v.y || v.z != v.z || v.w != v.w) mx = INFINITY;
      }
      for (int64_t c = 4 * c4 + threadIdx.x; c < cols; c += 256) {
        const float v = row[c];
        mx = (v != v) ? INFINITY : fmaxf(mx, fabsf(v));
      }
    } else {
      for (int64_t c = threadIdx.x; c < cols; c += 256) {
        const float v = row[c];
        mx = (v != v) ? INFINITY : fmaxf(mx, fabsf(v));
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(ws[0], ws[1]), fmaxf(ws[2], ws[3]));
}

// scale = {2^(15-e), 2^(e-15)} with max|A| in [2^(e-1), 2^e): the largest entry
// lands in [2^14, 2^15), inside the FP16 range with a factor 2 of headroom.
// A zero or non-finite maximum leaves the data unscaled.
__global__ void scale_kernel(const float* part, int nparts, float* scale) {
  __shared__ float ws[4];
  float mx = 0.0f;
  for (int i = threadIdx.x; i < nparts; i += 256) mx = fmaxf(mx, part[i]);
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float a = fmaxf(fmaxf(ws[0], ws[1]), fmaxf(ws[2], ws[3]));
    float s = 1.0f;
    if (a > 0.0f && a <= 3.402823466e38f) {
      int e = 0;
      (void)frexpf(a, &e);
      const int sh = min(max(15 - e, -126), 127);
      s = ldexpf(1.0f, sh);
    }
    scale[0] = s;
    scale[1] = 1.0f / s;
  }
}

}  // namespace

// The wide form (gemm16w_kernel.hpp) covers 256 < N <= 576 in one column tile
// of 80-row stripes, one workgroup per CU, when the operands admit whole
// vectors: K a multiple of 8 (>= 8), A rows 16-byte aligned (k contiguous) or
// 8-byte aligned with M even (row index contiguous), B rows 16-byte aligned.
// the wide kernel reads A in 16-byte vectors when k is contiguous, in single
// words across rows otherwise; B (chunk-major, from pack16c_launch) always in
// 16-byte vectors
bool gemm16_wide(int64_t M, int64_t N, int64_t K, const float* A, int64_t sam, int64_t sak) {
  if (sak != 1 && sam != 1) return false;
  const bool akc = sak == 1;
  const bool avec = !akc || ((uintptr_t)A % 16 == 0 && sam % 4 == 0);
  // the kernel's 32-bit byte offsets within a stripe (k contiguous: 80 rows of
  // sam) or within a k-step (row index contiguous: 32 k of sak, plus M rows)
  const bool off32 = akc ? (int64_t)g16::WBM * sam * 4 < (1LL << 31) : (32 * sak + M) * 4 < (1LL << 31);
  return g16::wide_cb(N) > 0 && avec && off32 && K >= 8 && K % 8 == 0 && M >= 1;
}
int64_t gemm16_wide_npad(int64_t N) { return 16 * g16::WNW * (int64_t)g16::wide_cb(N); }
// every chunk of K, rounded up to a k-step, and one more k-step: a step that
// starts inside K reads its four chunks without clamping
int64_t gemm16_wide_kchunks(int64_t K) { return round_up(ceil_div(std::max<int64_t>(K, 1), 8), 4) + 4; }

int gemm16_pick_splitk(int64_t M, int64_t N, int64_t K, int num_cus) {
  if (g16::wide_cb(N) > 0 && K >= 8 && K % 8 == 0) {
    // one workgroup per CU. With at least half the CUs busy, the split of 1 to 4
    // with the fewest rounds of workgroups per unit of work, taken only when it
    // saves more than 5% (the partial sums cost a pass over C): 625 stripes on
    // 256 CUs run 3 rounds unsplit, 2.5 with K split in two
    const int64_t stripes = ceil_div(M, g16::WBM);
    if (2 * stripes >= num_cus) {
      int best = 1;
      double bv = (double)ceil_div(stripes, num_cus);
      for (int s = 2; s <= 4; ++s) {
        if (K / s < 4096) break;
        const double v = (double)ceil_div(stripes * s, num_cus) / s;
        if (v < 0.95 * bv) {
          bv = v;
          best = s;
        }
      }
      return best;
    }
    int64_t s = num_cus / stripes;
    s = std::min<int64_t>(s, std::max<int64_t>(1, K / 1024));
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
  }
  int nt, gy;
  pick_cols(N, &nt, &gy);
  const int64_t stripes = ceil_div(M, BM) * gy;
  const int64_t slots = 2 * (int64_t)num_cus;   // two workgroups per CU
  if (stripes >= slots) return 1;
  int64_t s = slots / stripes;
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / 256));
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

size_t gemm16_part_bytes(const Gemm16Desc& d) {
  if (d.splitk <= 1) return 0;
  return (size_t)d.splitk * d.M * d.N * sizeof(float);
}

hipError_t gemm16_launch(const Gemm16Desc& d, void* part, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.sak != 1 && d.sam != 1) return hipErrorInvalidValue;
  int nt, gy;
  pick_cols(d.N, &nt, &gy);
  const int splitk = std::max(1, d.splitk);
  const bool akc = d.sak == 1;
  g16::Args a{};
  a.M = d.M; a.N = d.N; a.K = d.K;
  a.A = d.A; a.sam = d.sam; a.sak = d.sak;
  a.B = static_cast<const uint16_t*>(d.B); a.ldb = d.ldb;
  a.kps = round_up(ceil_div(std::max<int64_t>(d.K, 1), splitk), BK);
  a.direct = splitk == 1;
  a.out = a.direct ? d.C : static_cast<float*>(part);
  a.ldo = a.direct ? d.ldc : d.N;
  a.scale = d.scale;
  const bool avec = akc ? ((uintptr_t)d.A % 16 == 0 && d.sam % 4 == 0) : ((uintptr_t)d.A % 8 == 0 && d.sak % 2 == 0);
  const bool bvec = (uintptr_t)d.B % 16 == 0 && d.ldb % 8 == 0;
  a.vec = avec && bvec;
  a.gx = (int)ceil_div(d.M, BM); a.gy = gy; a.gz = splitk;
  if (ev0) (void)hipEventRecord(ev0, stream);
  hipError_t e;
  const bool wide = gemm16_wide(d.M, d.N, d.K, d.A, d.sam, d.sak);
  if (wide != (d.b_chunked != 0)) return hipErrorInvalidValue;   // B packed for the other kernel
  if (wide) {
    a.gx = (int)ceil_div(d.M, g16::WBM);
    a.gy = 1;
    a.ldb = gemm16_wide_npad(d.N);
    a.kc8max = gemm16_wide_kchunks(d.K) - 4;
    const int cb = g16::wide_cb(d.N);
    e = d.fp16 ? g16::launch_wide_fp16(a, akc, cb, stream) : g16::launch_wide_bf16(a, akc, cb, stream);
  } else {
    e = d.fp16 ? g16::launch_fp16(nt, a, akc, stream) : g16::launch_bf16(nt, a, akc, stream);
  }
  if (ev1) (void)hipEventRecord(ev1, stream);
  if (e != hipSuccess || splitk == 1) return e;
  const int64_t total = d.M * d.N;
  const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
  hipLaunchKernelGGL(reduce16_kernel, dim3(blocks), dim3(256), 0, stream, static_cast<const float*>(part), splitk, d.M,
                     d.N, d.C, d.ldc);
  return hipGetLastError();
}

hipError_t pack16c_launch(int fp16, int64_t rows, int64_t cols, const float* in, int64_t sj, int64_t sk, int64_t npad,
                          int64_t kchunks, void* out, hipStream_t stream) {
  const int64_t words = npad * kchunks;
  if (words <= 0) return hipSuccess;
  const unsigned grid = (unsigned)ceil_div(words, 256);
  if (fp16)
    hipLaunchKernelGGL(pack16c_kernel<true>, dim3(grid), dim3(256), 0, stream, rows, cols, in, sj, sk, npad, words,
                       static_cast<g16::u32x4*>(out));
  else
    hipLaunchKernelGGL(pack16c_kernel<false>, dim3(grid), dim3(256), 0, stream, rows, cols, in, sj, sk, npad, words,
                       static_cast<g16::u32x4*>(out));
  return hipGetLastError();
}

hipError_t pack16_launch(int fp16, int64_t rows, int64_t cols, const float* in, int64_t sj, int64_t sk,
                         int64_t rows_pad, int64_t cols_pad, void* out, int64_t ldo, hipStream_t stream) {
  if (rows_pad <= 0 || cols_pad <= 0) return hipSuccess;
  const dim3 grid((unsigned)ceil_div(cols_pad, 64), (unsigned)ceil_div(rows_pad, 64));
  if (fp16)
    hipLaunchKernelGGL(pack16_kernel<true>, grid, dim3(256), 0, stream, rows, cols, in, sj, sk, rows_pad, cols_pad,
                       static_cast<uint16_t*>(out), ldo);
  else
    hipLaunchKernelGGL(pack16_kernel<false>, grid, dim3(256), 0, stream, rows, cols, in, sj, sk, rows_pad, cols_pad,
                       static_cast<uint16_t*>(out), ldo);
  return hipGetLastError();
}

hipError_t fp16_scale_launch(int64_t rows, int64_t cols, const float* A, int64_t lda, float* part, float* scale,
                             hipStream_t stream) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(rows, kScaleParts));
  hipLaunchKernelGGL(amax_kernel, dim3(nb), dim3(256), 0, stream, rows, cols, A, lda, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(256), 0, stream, part, nb, scale);
  return hipGetLastError();
}

}  // namespace idcur
