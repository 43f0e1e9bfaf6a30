// Host dispatch of the FP32 thin-output GEMM (kernel in gemm_thin_kernel.hpp).
// Eligibility (else the general kernel runs): FP32 in, FP32 accumulation and
// output, B contiguous along N with every row readable up to round_up(N, 4), A
// contiguous along M or K with that extent a multiple of 4, 16-byte aligned
// bases and 4-aligned strides, no device-side bounds.
#include "gemm_thin_kernel.hpp"

namespace idcur {

using namespace gt;

bool thin_f32_eligible(const GemmDesc& d) {
  const int ta = d.a_type >= 0 ? d.a_type : d.in_type, tb = d.b_type >= 0 ? d.b_type : d.in_type;
  if (ta != 1 || tb != 1 || d.acc_type != 1 || d.out_type != 1) return false;
  if (d.m_dev || d.n_dev || d.k_dev) return false;
  if (d.sbn != 1 || d.sbk % 4 != 0 || (uintptr_t)d.B % 16 != 0 || !d.b_rows_padded) return false;
  if (d.sbk < round_up(d.N, 4)) return false;
  if ((uintptr_t)d.A % 16 != 0) return false;
  if (d.sak == 1) return d.sam % 4 == 0 && d.K % 4 == 0;
  if (d.sam == 1) return d.sak % 4 == 0 && d.M % 4 == 0;
  return false;
}

int thin_f32_nt(int64_t N) {
  const int64_t t = ceil_div(N, 16);
  return t <= 8 ? 8 : (t <= 14 ? 14 : 16);
}

// Split count: the smallest with at least 4.5 workgroups per CU (about 1.5
// rounds of the 3 resident per CU) and 256 K per split. Measured on the
// 20000 x 10000 (x 210 columns) sketch and power products, the kernel time is
// flat from there on while the partial sums grow with the split count.
int thin_f32_pick_splitk(int64_t M, int64_t N, int64_t K, int num_cus) {
  const int nt = thin_f32_nt(N);
  const int64_t tiles = ceil_div(M, BM) * ceil_div(N, 16 * nt);
  int s = 1;
  while (2 * tiles * s < 9LL * std::max(num_cus, 1) && K / (s + 1) >= 256 && s < 64) ++s;
  return s;
}

template <int NT, int OCC, int BK, int WR>
static void launch_v(bool akc, dim3 grid, const KArgs& k, hipStream_t stream) {
  if (akc) hipLaunchKernelGGL((thin_f32_kernel<NT, true, OCC, BK, WR>), grid, dim3(256), 0, stream, k);
  else hipLaunchKernelGGL((thin_f32_kernel<NT, false, OCC, BK, WR>), grid, dim3(256), 0, stream, k);
}

hipError_t thin_f32_launch(const GemmDesc& d, int splitk, void* part, hipStream_t stream) {
  const int nt = thin_f32_nt(d.N);
  KArgs k{};
  k.M = d.M; k.N = d.N; k.K = d.K;
  k.A = d.A; k.sam = d.sam; k.sak = d.sak;
  k.B = d.B; k.sbk = d.sbk; k.sbn = 1;
  k.kps = round_up(ceil_div(std::max<int64_t>(d.K, 1), splitk), 16);
  k.direct = splitk == 1;
  k.out = k.direct ? d.C : part;
  k.ldo = k.direct ? d.ldc : d.N;
  k.out_type = 1;
  k.alpha = d.alpha; k.beta = d.beta;
  k.gx = (int)ceil_div(d.M, BM); k.gy = (int)ceil_div(d.N, 16 * nt); k.gz = splitk;
  const dim3 grid(gk::xcd_grid(k));
  const bool akc = d.sak == 1;
  // 2 x 2 wave split, 16-deep stages (the fastest of the measured variants)
  if (nt == 8) launch_v<8, 4, 16, 32>(akc, grid, k, stream);
  else if (nt == 14) launch_v<14, 3, 16, 32>(akc, grid, k, stream);
  else launch_v<16, 3, 16, 32>(akc, grid, k, stream);
  return hipGetLastError();
}

}  // namespace idcur
