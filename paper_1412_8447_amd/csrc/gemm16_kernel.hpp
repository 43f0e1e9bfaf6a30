// Thin-output GEMM on the 16-bit matrix cores: C (M x N, FP32) = A (M x K, FP32
// in memory, rounded to BF16 or FP16 on the way in) * B (K x N, 16-bit,
// pre-packed), FP32 accumulation. This is the low-precision form of the sketch
// Y = Omega A (Section 5.1) and of the power steps of Section 5.3.
//
// Matrix core: v_mfma_f32_16x16x32_{bf16,f16}. Per 16x16x32 block, lane L holds
// A(L%16, 8*(L/16) + e) and B(8*(L/16) + e, L%16) for e = 0..7 (eight consecutive
// k in one 128-bit register quad), and receives C(4*(L/16) + r, L%16), r = 0..3.
//
// Workgroup tile: 128 rows x 16*NT columns, k-steps of 32. The four waves split
// it 2 x 2 (64 rows x 8*NT columns each: 4 x NT/2 accumulator blocks).
//   * A (FP32, the big operand, read from HBM once per pass) is loaded with
//     vector loads, scaled (FP16 prescaling), rounded to 16 bits in registers
//     and written to LDS as rows of 32 k (one 16-byte chunk per 8 k). When A is
//     stored with k contiguous, a thread loads 8 consecutive k of a row; when it
//     is stored with the row index contiguous, a thread loads 8 k-rows of 2
//     adjacent rows (coalesced along the rows) and transposes in registers.
//   * B is stored packed as B^T (N x K, k contiguous, 16-bit), so its chunks go
//     to LDS unchanged.
//   * LDS rows are 80 bytes (64 + 16 padding): the 16 rows read by one operand
//     load then start in 16 distinct bank quads.
// Double-buffered LDS with a register prefetch of the next k-step; one barrier
// per k-step. K is split over the grid when there are too few row stripes to
// occupy every CU; partial sums are reduced in a fixed order (deterministic).
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace g16 {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128;
constexpr int BK = 32;
constexpr int RS = 5;   // LDS row stride in 16-byte chunks (4 data + 1 pad)

struct Args {
  int64_t M, N, K;
  const float* A; int64_t sam, sak;
  const uint16_t* B; int64_t ldb;   // B(k, j) = B[j*ldb + k]; wide kernel: chunk-major, ldb = padded columns
  int64_t kc8max;                   // wide kernel: last chunk index a k-step may start at
  float* out; int64_t ldo;          // C (direct) or partials (ld N)
  int64_t kps;                      // K per split (multiple of BK)
  int direct;
  const float* scale;               // {s, 1/s} or NULL
  int vec;                          // aligned vector loads allowed for A and B
  int gx, gy, gz;
};

__host__ __device__ inline int64_t tiles_total(const Args& p) { return (int64_t)p.gx * p.gy * p.gz; }

// 8 values rounded to the 16-bit format; FP16 values are scaled by s first
// (BF16 has FP32's exponent range and is never scaled)
template <bool H>
__device__ __forceinline__ u32x4 pack8(const float (&f)[8], float s) {
  if constexpr (H) {
    f16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (_Float16)(f[e] * s);
    return __builtin_bit_cast(u32x4, v);
  } else {
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)f[e];
    return __builtin_bit_cast(u32x4, v);
  }
}

template <bool H>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
  if constexpr (H)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

template <bool H, int NT, bool A_KC, int D>
__global__ __launch_bounds__(256, 2) void gemm16_kernel(Args p) {
  constexpr int BN = 16 * NT;
  constexpr int HN = NT / 2;                    // column blocks per wave
  constexpr int BQ = (BN * 4 + 255) / 256;      // B chunks per thread
  __shared__ u32x4 As[2][BM * RS];
  __shared__ u32x4 Bs[2][BN * RS];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;
  const int64_t W = tiles_total(p), per = (W + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= W) return;
  // column tiles of one row stripe are adjacent (same XCD, dispatched together),
  // so the stripe of A they all read comes from HBM once and from L2 after that
  const int by = (int)(tile % p.gy), bx = (int)((tile / p.gy) % p.gx), bz = (int)(tile / ((int64_t)p.gx * p.gy));
  const int64_t m0 = (int64_t)bx * BM, n0 = (int64_t)by * BN;
  const int64_t kb = (int64_t)bz * p.kps, ke = min(p.K, kb + p.kps);
  const float s_in = p.scale ? p.scale[0] : 1.0f;
  const float s_out = p.scale ? p.scale[1] : 1.0f;

  // D k-steps in registers: the loads of D k-steps are in flight while the
  // matrix cores work on the k-step in LDS (a load takes microseconds under
  // full-chip traffic, a k-step's products a few hundred cycles)
  float fas[D][16];
  u32x4 rbs[D][BQ];

  // ---- global -> registers (one k-step) -----------------------------------
  auto gload = [&](int64_t k0, float (&fa)[16], u32x4 (&rb)[BQ]) {
    const bool full = p.vec && (k0 + BK <= ke) && (m0 + BM <= p.M);
    if (A_KC) {
      // thread: rows r0 and r0 + 64, k = k0 + 8g .. +7
      const int r0 = tid >> 2, g = tid & 3;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t gi = m0 + r0 + 64 * h, gk = k0 + 8 * g;
        const float* src = p.A + gi * p.sam + gk;
        if (full) {
          const float4 u = *reinterpret_cast<const float4*>(src);
          const float4 v = *reinterpret_cast<const float4*>(src + 4);
          fa[8 * h + 0] = u.x; fa[8 * h + 1] = u.y; fa[8 * h + 2] = u.z; fa[8 * h + 3] = u.w;
          fa[8 * h + 4] = v.x; fa[8 * h + 5] = v.y; fa[8 * h + 6] = v.z; fa[8 * h + 7] = v.w;
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) fa[8 * h + e] = (gi < p.M && gk + e < ke) ? src[e] : 0.0f;
        }
      }
    } else {
      // thread: rows 2c, 2c + 1 (c = lane), k = k0 + 8*wave .. +7
      const int64_t gi = m0 + 2 * lane;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t gk = k0 + 8 * wv + e;
        const float* src = p.A + gk * p.sak + gi;
        if (full) {
          const float2 u = *reinterpret_cast<const float2*>(src);
          fa[e] = u.x; fa[8 + e] = u.y;
        } else {
          const bool kv = gk < ke;
          fa[e] = (kv && gi < p.M) ? src[0] : 0.0f;
          fa[8 + e] = (kv && gi + 1 < p.M) ? src[1] : 0.0f;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < BQ; ++r) {
      const int q = tid + 256 * r;
      if (q < BN * 4) {
        const int64_t gj = n0 + (q >> 2), gk = k0 + 8 * (q & 3);
        const uint16_t* src = p.B + gj * p.ldb + gk;
        if (gj < p.N && p.vec && gk + 8 <= ke) {
          rb[r] = *reinterpret_cast<const u32x4*>(src);
        } else {
          uint32_t w[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t lo = (gj < p.N && gk + 2 * e < ke) ? src[2 * e] : 0u;
            const uint32_t hi = (gj < p.N && gk + 2 * e + 1 < ke) ? src[2 * e + 1] : 0u;
            w[e] = lo | (hi << 16);
          }
          rb[r] = u32x4{w[0], w[1], w[2], w[3]};
        }
      }
    }
  };
  // ---- registers -> LDS ------------------------------------------------------
  auto sstore = [&](int buf, const float (&fa)[16], const u32x4 (&rb)[BQ]) {
    if (A_KC) {
      const int r0 = tid >> 2, g = tid & 3;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float f[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = fa[8 * h + e];
        As[buf][(r0 + 64 * h) * RS + g] = pack8<H>(f, s_in);
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float f[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = fa[8 * h + e];
        As[buf][(2 * lane + h) * RS + wv] = pack8<H>(f, s_in);
      }
    }
#pragma unroll
    for (int r = 0; r < BQ; ++r) {
      const int q = tid + 256 * r;
      if (q < BN * 4) Bs[buf][(q >> 2) * RS + (q & 3)] = rb[r];
    }
  };

  f32x4 acc[4][HN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < HN; ++c) acc[i][c] = f32x4{0, 0, 0, 0};

  const int64_t nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    // k-step s is loaded into register stage s % D; k-step t is in LDS buffer
    // t % 2 while it is multiplied. After the products of step t, step t + 1
    // goes from its stage to LDS and step t + 1 + D is loaded into that stage.
#pragma unroll
    for (int s = 0; s < D; ++s)
      if (s < nk) gload(kb + s * BK, fas[s], rbs[s]);
    sstore(0, fas[0], rbs[0]);
    if (D < nk) gload(kb + D * BK, fas[0], rbs[0]);
    __syncthreads();
    for (int64_t t0 = 0; t0 < nk; t0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int64_t it = t0 + d;
        if (it >= nk) break;
        const int buf = (int)(it & 1);
        const u32x4* as = As[buf];
        const u32x4* bs = Bs[buf];
        u32x4 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = as[(wm * 64 + i * 16 + (lane & 15)) * RS + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < HN; ++c) {
          const u32x4 b = bs[(wn * HN * 16 + c * 16 + (lane & 15)) * RS + (lane >> 4)];
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][c] = mfma16<H>(a[i], b, acc[i][c]);
        }
        const int sn = (d + 1) % D;   // stage of k-step it + 1 (constant once unrolled)
        if (it + 1 < nk) sstore(buf ^ 1, fas[sn], rbs[sn]);
        if (it + 1 + D < nk) gload(kb + (it + 1 + D) * BK, fas[sn], rbs[sn]);
        __syncthreads();
      }
    }
  }

  // ---- epilogue ---------------------------------------------------------------
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int c = 0; c < HN; ++c) {
      const int64_t gj = n0 + wn * HN * 16 + c * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + r;
        if (gi < p.M && gj < p.N) {
          const float v = acc[i][c][r] * s_out;
          if (p.direct) p.out[gi * p.ldo + gj] = v;
          else p.out[((int64_t)bz * p.M + gi) * p.N + gj] = v;
        }
      }
    }
  }
}

// register stages of the k-step prefetch: three where the registers allow it
// (two waves per SIMD, 256 registers each), one for the widest tiles (more
// stages there spill)
constexpr int prefetch_stages(int nt) { return nt >= 14 ? 1 : 3; }

template <bool H, int NT>
hipError_t launch_nt(const Args& a, bool akc, hipStream_t s) {
  const unsigned grid = (unsigned)(8 * ((tiles_total(a) + 7) / 8));
  if (akc) hipLaunchKernelGGL((gemm16_kernel<H, NT, true, prefetch_stages(NT)>), dim3(grid), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((gemm16_kernel<H, NT, false, prefetch_stages(NT)>), dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <bool H>
hipError_t launch_h(int nt, const Args& a, bool akc, hipStream_t s) {
  switch (nt) {
    case 2: return launch_nt<H, 2>(a, akc, s);
    case 4: return launch_nt<H, 4>(a, akc, s);
    case 6: return launch_nt<H, 6>(a, akc, s);
    case 8: return launch_nt<H, 8>(a, akc, s);
    case 10: return launch_nt<H, 10>(a, akc, s);
    case 12: return launch_nt<H, 12>(a, akc, s);
    case 14: return launch_nt<H, 14>(a, akc, s);
    default: return launch_nt<H, 16>(a, akc, s);
  }
}

hipError_t launch_bf16(int nt, const Args& a, bool akc, hipStream_t s);
hipError_t launch_fp16(int nt, const Args& a, bool akc, hipStream_t s);

}  // namespace g16
}  // namespace idcur
