// Thin-output MFMA GEMM: C (M x N) = A (M x K) * B (K x N) with N small
// (the sketch width l = k + p, or a Gram matrix), M and K large.
//
// This is the sketch Y = Omega A of Section 5.1 (eq. (Y=OmegaA)), the power
// steps orth(Y) A^T / orth(Y) A of Section 5.3, and the Gram matrices of the
// Cholesky-based orthonormalisation. One workgroup owns a 64-row stripe of C
// and ALL of N (up to 16*NT columns), so the big operand A streams from HBM
// exactly once per pass; the thin operand B is re-read from L2. K is split
// over grid.z when there are too few stripes to fill the 256 CUs; the split
// partial sums are reduced in a fixed order (deterministic results).
//
// Matrix cores: v_mfma_f32_16x16x4f32 (FP32) or v_mfma_f64_16x16x4f64 (FP64).
// Operand layout per 16x16x4 block: lane L holds A(L%16, L/16) and B(L/16, L%16).
// Result layout: FP32 -> row 4*(L/16) + r, FP64 -> row L/16 + 4*r, column L%16.
#include "gemm_kernel.hpp"

namespace idcur {
using namespace gk;
namespace {

int pick_nt(int64_t N, bool acc64) {
  const int64_t t = ceil_div(N, 16);
  if (t <= 2) return 2;
  // FP64 accumulation: 64-column tiles. Wider tiles need 200-400 registers, one
  // wave per SIMD and fewer workgroups; measured on the FP64 products of the CUR
  // step (Gram matrices, bases, T = S11^-1 S12) 64 columns were 1.2-2x faster
  if (t <= 4 || acc64) return 4;
  if (t <= 8) return 8;
  if (t <= 14) return 14;
  return 16;
}

__global__ __launch_bounds__(256) void sum_partials(const double* part, int64_t n, double* out) {
  // one workgroup; fixed assignment and order -> deterministic
  __shared__ double ws[4];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += 256) s += part[e];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

}  // namespace

size_t gemm_resid_part_bytes(int64_t M, int64_t N) {
  return (size_t)ceil_div(M, BM) * ceil_div(N, 256) * sizeof(double);
}

hipError_t gemm_resid_launch(int x_type, int64_t M, int64_t N, int64_t K, const void* Cm, int64_t ldc, int c_type,
                             const double* W, int64_t ldw, const void* X, int64_t ldx, const int* k_dev,
                             double* part, double* out, hipStream_t stream) {
  if (M <= 0 || N <= 0) return hipSuccess;
  KArgs k{};
  k.M = M; k.N = N; k.K = K;
  k.A = Cm; k.sam = ldc; k.sak = 1;
  k.B = W; k.sbk = ldw; k.sbn = 1;
  k.kps = round_up(std::max<int64_t>(K, 1), BK);
  k.direct = 1; k.alpha = 1.0;
  k.vec_a = 0; k.vec_b = ((uintptr_t)W % 32 == 0) && (ldw % 4 == 0);
  k.X = X; k.ldx = ldx; k.x_type = x_type; k.rpart = part;
  k.k_dev = k_dev;
  k.gx = (int)ceil_div(M, BM); k.gy = (int)ceil_div(N, 256); k.gz = 1;
  dim3 grid(xcd_grid(k));
  if (c_type == 1)
    hipLaunchKernelGGL((gemm_kernel<float, double, double, 16, true, true, true>), grid, dim3(256), 0, stream, k);
  else
    hipLaunchKernelGGL((gemm_kernel<double, double, double, 16, true, true, true>), grid, dim3(256), 0, stream, k);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, stream, part, (int64_t)k.gx * k.gy, out);
  return hipGetLastError();
}

size_t gemm_part_bytes(const GemmDesc& d) {
  if (d.splitk <= 1) return 0;
  return (size_t)d.splitk * d.M * d.N * (d.acc_type == 1 ? 4 : 8);
}

int gemm_pick_splitk(int64_t M, int64_t N, int64_t K, int num_cus, bool acc64, bool lower) {
  const int64_t gx = ceil_div(M, BM), bn = 16 * pick_nt(N, acc64), gy = ceil_div(N, bn);
  int64_t stripes = gx * gy;
  if (lower) {   // tiles that meet the lower triangle
    stripes = 0;
    for (int64_t y = 0; y < gy; ++y) stripes += std::max<int64_t>(0, gx - (y * bn) / BM);
  }
  int s = 1;
  // aim for at least 4 workgroups per CU, keep >= 256 K per split
  while (stripes * s < 4 * num_cus && K / (2 * s) >= 256 && s < 64) s *= 2;
  return s;
}

int gemm_pick_splitk_desc(const GemmDesc& d, int num_cus) {
  if (thin_f32_eligible(d)) return thin_f32_pick_splitk(d.M, d.N, d.K, num_cus);
  return gemm_pick_splitk(d.M, d.N, d.K, num_cus, d.acc_type == 0, d.lower && d.M == d.N);
}

hipError_t gemm_launch(const GemmDesc& d, void* part, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (thin_f32_eligible(d)) {
    const int splitk = std::max(1, d.splitk);
    if (ev0) (void)hipEventRecord(ev0, stream);
    hipError_t e = thin_f32_launch(d, splitk, part, stream);
    if (ev1) (void)hipEventRecord(ev1, stream);
    if (e != hipSuccess || splitk == 1) return e;
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(d.M * d.N, 256), 4096);
    hipLaunchKernelGGL(splitk_reduce<float>, dim3(blocks), dim3(256), 0, stream, static_cast<const float*>(part),
                       splitk, d.M, d.N, d.C, d.ldc, 1, d.alpha, d.beta, d.m_dev, d.n_dev);
    return hipGetLastError();
  }
  const bool akc = (d.sak == 1);
  const bool bnc = (d.sbn == 1);
  const int nt = pick_nt(d.N, d.acc_type == 0);
  const int bn = 16 * nt;
  const int splitk = std::max(1, d.splitk);
  KArgs k{};
  k.M = d.M; k.N = d.N; k.K = d.K;
  k.A = d.A; k.sam = d.sam; k.sak = d.sak;
  k.B = d.B; k.sbk = d.sbk; k.sbn = d.sbn;
  k.kps = round_up(ceil_div(std::max<int64_t>(d.K, 1), splitk), BK);
  k.direct = splitk == 1;
  k.out = k.direct ? d.C : part;
  k.ldo = k.direct ? d.ldc : d.N;
  k.out_type = d.out_type;
  k.alpha = d.alpha; k.beta = d.beta;
  k.m_dev = d.m_dev; k.n_dev = d.n_dev; k.k_dev = d.k_dev;
  k.lower = d.lower && d.M == d.N;
  const int ta_ = d.a_type >= 0 ? d.a_type : d.in_type, tb_ = d.b_type >= 0 ? d.b_type : d.in_type;
  auto aligned = [&](const void* p, int64_t other_stride, int t) {
    return ((uintptr_t)p % (4 * (t == 1 ? 4 : 8)) == 0) && (other_stride % 4 == 0);
  };
  k.vec_a = aligned(d.A, akc ? d.sam : d.sak, ta_);
  k.vec_b = aligned(d.B, bnc ? d.sbk : d.sbn, tb_);
  k.gx = (int)ceil_div(d.M, BM); k.gy = (int)ceil_div(d.N, bn); k.gz = splitk;
  dim3 grid(xcd_grid(k));
  hipError_t e;
  if (ev0) (void)hipEventRecord(ev0, stream);
  const int ta = d.a_type >= 0 ? d.a_type : d.in_type, tb = d.b_type >= 0 ? d.b_type : d.in_type;
  if (ta == 1 && tb == 1 && d.acc_type == 1) e = launch_f32(nt, k, grid, akc, bnc, stream);
  else if (ta == 1 && tb == 1 && d.acc_type == 0) e = launch_f32_f64acc(nt, k, grid, akc, bnc, stream);
  else if (ta == 0 && tb == 0 && d.acc_type == 0) e = launch_f64(nt, k, grid, akc, bnc, stream);
  else if (ta == 1 && tb == 0 && d.acc_type == 0) e = launch_f32_f64(nt, k, grid, akc, bnc, stream);
  else if (ta == 0 && tb == 1 && d.acc_type == 0) e = launch_f64_f32(nt, k, grid, akc, bnc, stream);
  else return hipErrorInvalidValue;
  if (ev1) (void)hipEventRecord(ev1, stream);
  if (e != hipSuccess || splitk == 1) return e;
  const int64_t total = d.M * d.N;
  const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(total, 256), 4096);
  if (d.acc_type == 1)
    hipLaunchKernelGGL(splitk_reduce<float>, dim3(blocks), dim3(256), 0, stream, static_cast<const float*>(part),
                       splitk, d.M, d.N, d.C, d.ldc, d.out_type, d.alpha, d.beta, d.m_dev, d.n_dev);
  else
    hipLaunchKernelGGL(splitk_reduce<double>, dim3(blocks), dim3(256), 0, stream, static_cast<const double*>(part),
                       splitk, d.M, d.N, d.C, d.ldc, d.out_type, d.alpha, d.beta, d.m_dev, d.n_dev);
  return hipGetLastError();
}

}  // namespace idcur
