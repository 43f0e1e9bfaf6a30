// FP32 thin-output GEMM kernel on the FP32 matrix cores (templates; the host
// dispatch is in gemm_thin.hip): C (M x N) = A (M x K) B (K x N) with N up to
// 16*NT per column tile, M and K large: the sketch Y = Omega A of Section 5.1
// and the power-step products of Section 5.3 in single precision.
//
// Same tiling as the general kernel (a 64-row stripe of C and all 16*NT columns
// of a column tile per workgroup, K split over the grid, XCD-contiguous tile
// ranges), built for throughput on 4-aligned operands:
//  * every global load is an unconditional 16-byte load from a clamped
//    address; K entries past the end of the split are cleared by a bit mask
//    when the stage is written to LDS (using the loaded values any earlier
//    would make the wave wait for them at once). Rows of A past M and columns
//    of B past N only feed outputs that are never stored, so they are clamped,
//    not cleared;
//  * LDS row strides are 16 or 48 words mod 64, so the 4 k-rows that one MFMA
//    operand read touches fall on 4 different groups of 16 banks;
//  * the operands of the next 4-deep k step are read from LDS before the MFMAs
//    of the current one are issued;
//  * the wave tile is WR rows x (16*NT*WR/64) columns: WR = 16 gives each of
//    the 4 waves all the columns (1 A and NT B operand reads for NT MFMAs per
//    k step), WR = 32 a 2 x 2 split (2 A and NT/2 B reads for NT MFMAs).
#pragma once
#include "gemm_kernel.hpp"

namespace idcur {
namespace gt {

using gk::KArgs;
using gk::f32x4;

constexpr int BM = 64;
constexpr int SA = 80;   // A stage tile As[k][m]: 64 + 16, k-rows 16 banks apart

__host__ __device__ constexpr int sb_stride(int bn) {
  // smallest stride >= bn that is 16 or 48 mod 64
  return (bn % 64 <= 16) ? bn - bn % 64 + 16 : (bn % 64 <= 48 ? bn - bn % 64 + 48 : bn - bn % 64 + 80);
}

typedef const __attribute__((address_space(1))) f32x4 gf32x4;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// global (not flat) 16-byte load
__device__ __forceinline__ f32x4 ldg4(const float* p) { return *(gf32x4*)p; }

__device__ __forceinline__ f32x4 keep4(f32x4 v, unsigned m0, unsigned m1, unsigned m2, unsigned m3) {
  const u32x4 m = {m0, m1, m2, m3};
  return __builtin_bit_cast(f32x4, __builtin_bit_cast(u32x4, v) & m);
}

template <int NT, bool A_KC, int OCC, int BK, int WR>
__global__ __launch_bounds__(256, OCC) void thin_f32_kernel(KArgs p) {
  constexpr int BN = 16 * NT;
  constexpr int SB = sb_stride(BN);
  constexpr int RT = WR / 16;                // row tiles per wave
  constexpr int WM = BM / WR;                // waves along M
  constexpr int WN = 4 / WM;                 // waves along N
  constexpr int CT = NT / WN;                // column tiles per wave
  static_assert(NT % WN == 0, "column tiles must split evenly over the waves");
  constexpr int NQA = BM * BK / 4;           // A quads per stage
  constexpr int AQ = (NQA + 255) / 256;      // per thread
  constexpr int NQ = BN * BK / 4;            // B quads per stage
  constexpr int BQ = (NQ + 255) / 256;       // per thread
  __shared__ float As[2][BK * SA];
  __shared__ float Bs[2][BK * SB];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wv % WM, wn = wv / WM;
  const int64_t W = gk::tiles_total(p), per = (W + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= W) return;
  const int bx = (int)(tile % p.gx), by = (int)((tile / p.gx) % p.gy), bz = (int)(tile / ((int64_t)p.gx * p.gy));
  const int64_t M = p.M, N = p.N;
  const int64_t m0 = (int64_t)bx * BM, n0 = (int64_t)by * BN;
  const int64_t kb = (int64_t)bz * p.kps;
  const int64_t ke = min(p.K, kb + p.kps);
  const float* A = static_cast<const float*>(p.A);
  const float* B = static_cast<const float*>(p.B);

  // A quad j of this thread, q = tid + 256 j:
  //   A_KC:  A(m0 + q % 64, k0 + 4 (q / 64) .. +3)     (transposed into As[k][m])
  //   else:  A(m0 + 4 (q % 16) .. +3, k0 + q / 16)
  auto a_m = [&](int j) { const int q = min(tid + 256 * j, NQA - 1); return A_KC ? q % 64 : 4 * (q % 16); };
  auto a_k = [&](int j) { const int q = min(tid + 256 * j, NQA - 1); return A_KC ? 4 * (q / 64) : q / 16; };
  // B quad j: row q / (BN/4), column quad q % (BN/4) of the stage
  auto b_k = [&](int j) { return min(tid + 256 * j, NQ - 1) / (BN / 4); };
  auto b_n = [&](int j) { return (min(tid + 256 * j, NQ - 1) % (BN / 4)) * 4; };

  f32x4 ra[AQ];
  f32x4 rb[BQ];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < AQ; ++j) {
      const int64_t gi = m0 + a_m(j);
      const int64_t gic = gi < M ? gi : 0;
      const int64_t k = k0 + a_k(j);
      const int64_t kc = k < ke ? k : kb;
      ra[j] = ldg4(A_KC ? A + gic * p.sam + kc : A + kc * p.sak + gic);
    }
#pragma unroll
    for (int j = 0; j < BQ; ++j) {
      const int64_t gj = n0 + b_n(j);
      const int64_t k = k0 + b_k(j);
      rb[j] = ldg4(B + (k < ke ? k : kb) * p.sbk + (gj < N ? gj : 0));
    }
  };
  auto sstore = [&](int buf, int64_t k0) {
    float* as = As[buf];
#pragma unroll
    for (int j = 0; j < AQ; ++j) {
      if (j + 1 < AQ || NQA % 256 == 0 || tid + 256 * j < NQA) {
        const int am = a_m(j), ak = a_k(j);
        const int64_t k = k0 + ak;
        if (A_KC) {
          const f32x4 v = keep4(ra[j], k < ke ? ~0u : 0u, k + 1 < ke ? ~0u : 0u, k + 2 < ke ? ~0u : 0u,
                                k + 3 < ke ? ~0u : 0u);
          as[(ak + 0) * SA + am] = v[0];
          as[(ak + 1) * SA + am] = v[1];
          as[(ak + 2) * SA + am] = v[2];
          as[(ak + 3) * SA + am] = v[3];
        } else {
          const unsigned msk = k < ke ? ~0u : 0u;
          *reinterpret_cast<f32x4*>(as + ak * SA + am) = keep4(ra[j], msk, msk, msk, msk);
        }
      }
    }
    float* bs = Bs[buf];
#pragma unroll
    for (int j = 0; j < BQ; ++j) {
      if (j + 1 < BQ || NQ % 256 == 0 || tid + 256 * j < NQ) {
        const int r = b_k(j);
        const unsigned msk = k0 + r < ke ? ~0u : 0u;
        *reinterpret_cast<f32x4*>(bs + r * SB + b_n(j)) = keep4(rb[j], msk, msk, msk, msk);
      }
    }
  };

  f32x4 acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int g = lane >> 4, c = lane & 15;
  const int64_t ntile = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (ntile > 0) {
    gload(kb);
    sstore(0, kb);
    __syncthreads();
    for (int64_t it = 0; it < ntile; ++it) {
      const int buf = (int)(it & 1);
      if (it + 1 < ntile) gload(kb + (it + 1) * BK);
      // MFMA operands of lane L at k step kk: A(m = WR wm + 16 i + L%16, k = 4 kk + L/16),
      // B(k = 4 kk + L/16, n = 16 (CT wn + t) + L%16)
      const float* as = As[buf] + g * SA + WR * wm + c;
      const float* bs = Bs[buf] + g * SB + 16 * CT * wn + c;
      float av[2][RT];
      float bv[2][CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) av[0][i] = as[16 * i];
#pragma unroll
      for (int t = 0; t < CT; ++t) bv[0][t] = bs[t * 16];
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int cur = kk & 1, nxt = cur ^ 1;
        if (kk + 1 < BK / 4) {
#pragma unroll
          for (int i = 0; i < RT; ++i) av[nxt][i] = as[(kk + 1) * 4 * SA + 16 * i];
#pragma unroll
          for (int t = 0; t < CT; ++t) bv[nxt][t] = bs[(kk + 1) * 4 * SB + t * 16];
        }
        // keep the next step's operand reads ahead of this step's MFMAs
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int t = 0; t < CT; ++t)
            acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[cur][i], bv[cur][t], acc[i][t], 0, 0, 0);
      }
      if (it + 1 < ntile) sstore(buf ^ 1, kb + (it + 1) * BK);
      __syncthreads();
    }
  }

  // epilogue: FP32 16x16x4 result layout, row 4*(L/16) + r, column L%16
#pragma unroll
  for (int i = 0; i < RT; ++i) {
#pragma unroll
    for (int t = 0; t < CT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = m0 + WR * wm + 16 * i + 4 * g + r;
        const int64_t gj = n0 + 16 * (CT * wn + t) + c;
        if (gi < M && gj < N) {
          const float v = acc[i][t][r];
          if (p.direct) {
            float* C = static_cast<float*>(p.out) + gi * p.ldo + gj;
            const double o = p.beta != 0.0 ? p.beta * (double)*C : 0.0;
            *C = (float)(p.alpha * (double)v + o);
          } else {
            static_cast<float*>(p.out)[((int64_t)bz * M + gi) * N + gj] = v;
          }
        }
      }
    }
  }
}

}  // namespace gt
}  // namespace idcur
