// Wide form of the 16-bit thin-output GEMM (gemm16_kernel.hpp) for 256 < N <=
// 640 output columns, the sketch width of rank-500 decompositions (Section 5.1;
// the power steps of Section 5.3): one workgroup computes an 80-row stripe of C
// over all columns, so that its stripe of A (FP32, the big operand) is fetched
// from memory once. With column tiles of at most 256, the same launch would
// fetch every stripe of A once per tile.
//
// Eight waves split the columns (CB blocks of 16 each) and share the 80 rows
// (five row blocks), two waves per SIMD, so that one wave's loads are in flight
// while the other's products run; the B stage of all columns fills most of LDS,
// so the kernel runs one workgroup per CU. Every global load
// is unconditional, from a clamped address inside the operand: rows of A past M
// and columns of B past N only feed outputs that are never stored, and 8-k
// chunks past the end of the K split are cleared (by select) before they reach
// LDS. Nothing in the k loop depends on the step count (steps past the end read
// cleared chunks), so the D register stages of the prefetch stay in flight
// together. Requires K % 8 == 0, aligned rows (16 bytes for A with k
// contiguous, 8 bytes and M even for A with the row index contiguous, 16 bytes
// for the packed B) and K >= 8.
#pragma once
#include "gemm16_kernel.hpp"

namespace idcur {
namespace g16 {

constexpr int WRB = 5;          // row blocks of 16 in a stripe
constexpr int WBM = 16 * WRB;   // stripe height

constexpr int WNW = 8;            // waves
constexpr int WNT = 64 * WNW;     // threads

template <bool H, bool A_KC, int CB, int D>
__global__ __launch_bounds__(WNT, 1) void gemm16w_kernel(Args p) {
  constexpr int BN = 16 * WNW * CB;                            // WNW waves x CB blocks x 16 columns
  constexpr int FA = A_KC ? 8 : 16;                            // floats per A chunk
  constexpr int NCA = A_KC ? WBM * 4 : (WBM / 2) * 4;          // A chunks per k-step
  constexpr int CA = (NCA + WNT - 1) / WNT;                    // per thread
  static_assert((BN * 4) % WNT == 0 && BN * 4 / WNT == CB, "B chunks split evenly");
  __shared__ u32x4 As[2][WBM * RS];
  __shared__ u32x4 Bs[2][BN * RS];

  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t W = (int64_t)p.gx * p.gz, per = (W + 7) / 8;
  // tile ranges contiguous per XCD: the stripes running together on one XCD
  // read the same k-range of B, which L2 then serves
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= W) return;
  const int bx = (int)(tile % p.gx), bz = (int)(tile / p.gx);
  const int64_t m0 = (int64_t)bx * WBM;
  const int64_t kb = (int64_t)bz * p.kps, ke = min(p.K, kb + p.kps);
  const float s_in = p.scale ? p.scale[0] : 1.0f;
  const float s_out = p.scale ? p.scale[1] : 1.0f;
  const int64_t mlast = A_KC ? p.M - 1 : p.M - 2;   // last row (pair) of A

  // A chunk c of this thread (q = min(tid + 512 c, NCA - 1)):
  //   A_KC:  row q / 4, k = 8 (q % 4) .. +7
  //   else:  rows 2 (q % 40), +1, k = 8 (q / 40) .. +7
  auto a_row = [&](int c) {
    const int q = min(tid + WNT * c, NCA - 1);
    return A_KC ? q >> 2 : 2 * (q % (WBM / 2));
  };
  auto a_kg = [&](int c) {
    const int q = min(tid + WNT * c, NCA - 1);
    return A_KC ? (q & 3) : q / (WBM / 2);
  };

  float fas[D][CA][FA];
  u32x4 rbs[D][CB];

  auto gload = [&](int64_t k0, float (&fa)[CA][FA], u32x4 (&rb)[CB]) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int64_t gi = min(m0 + a_row(c), mlast);
      const int64_t kc = min(k0 + 8 * a_kg(c), ke - 8);
      // A is read once: non-temporal loads, so that its stream does not push
      // the thin operand B (read by every stripe) out of L2
      typedef float nf4 __attribute__((ext_vector_type(4)));
      typedef float nf2 __attribute__((ext_vector_type(2)));
      if (A_KC) {
        const float* src = p.A + gi * p.sam + kc;
        const nf4 u = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(src));
        const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(src + 4));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          fa[c][e] = u[e];
          fa[c][4 + e] = v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const nf2 u = __builtin_nontemporal_load(reinterpret_cast<const nf2*>(p.A + (kc + e) * p.sak + gi));
          fa[c][e] = u[0];
          fa[c][8 + e] = u[1];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = tid + WNT * c;
      const int64_t gj = min((int64_t)(q >> 2), p.N - 1);
      const int64_t kc = min(k0 + 8 * (q & 3), ke - 8);
      rb[c] = *reinterpret_cast<const u32x4*>(p.B + gj * p.ldb + kc);
    }
  };
  auto sstore = [&](int buf, int64_t k0, const float (&fa)[CA][FA], const u32x4 (&rb)[CB]) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      if (c + 1 < CA || NCA % WNT == 0 || tid + WNT * c < NCA) {
        const bool kv = k0 + 8 * a_kg(c) < ke;   // whole chunk in the split (K % 8 == 0)
        const int r = a_row(c), g = a_kg(c);
        float f[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) f[e] = kv ? fa[c][e] : 0.0f;
        As[buf][r * RS + g] = pack8<H>(f, s_in);
        if (!A_KC) {
#pragma unroll
          for (int e = 0; e < 8; ++e) f[e] = kv ? fa[c][8 + e] : 0.0f;
          As[buf][(r + 1) * RS + g] = pack8<H>(f, s_in);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = tid + WNT * c;
      const bool kv = k0 + 8 * (q & 3) < ke;
      Bs[buf][(q >> 2) * RS + (q & 3)] = kv ? rb[c] : u32x4{0u, 0u, 0u, 0u};
    }
  };

  f32x4 acc[WRB][CB];
#pragma unroll
  for (int i = 0; i < WRB; ++i)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[i][c] = f32x4{0, 0, 0, 0};

  const int64_t nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    // k-step s in register stage s % D; k-step t in LDS buffer t % 2 while it
    // is multiplied; after the products of step t, step t + 1 goes to LDS and
    // step t + 1 + D is loaded into its stage
#pragma unroll
    for (int s = 0; s < D; ++s) gload(kb + s * BK, fas[s], rbs[s]);
    sstore(0, kb, fas[0], rbs[0]);
    gload(kb + D * BK, fas[0], rbs[0]);
    __syncthreads();
    for (int64_t t0 = 0; t0 < nk; t0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int64_t it = t0 + d;
        const int buf = (int)(it & 1);
        const u32x4* as = As[buf];
        const u32x4* bs = Bs[buf];
        u32x4 a[WRB];
#pragma unroll
        for (int i = 0; i < WRB; ++i) a[i] = as[(i * 16 + (lane & 15)) * RS + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < CB; ++c) {
          const u32x4 b = bs[((wv * CB + c) * 16 + (lane & 15)) * RS + (lane >> 4)];
#pragma unroll
          for (int i = 0; i < WRB; ++i) acc[i][c] = mfma16<H>(a[i], b, acc[i][c]);
        }
        const int sn = (d + 1) % D;   // stage of k-step it + 1 (constant once unrolled)
        sstore(buf ^ 1, kb + (it + 1) * BK, fas[sn], rbs[sn]);
        gload(kb + (it + 1 + D) * BK, fas[sn], rbs[sn]);
        __syncthreads();
      }
    }
  }

  // ---- epilogue (C block layout: row 4 (L / 16) + r, column L % 16) -----------------
#pragma unroll
  for (int i = 0; i < WRB; ++i) {
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int64_t gj = (int64_t)(wv * CB + c) * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = m0 + i * 16 + 4 * (lane >> 4) + r;
        if (gi < p.M && gj < p.N) {
          const float v = acc[i][c][r] * s_out;
          if (p.direct) p.out[gi * p.ldo + gj] = v;
          else p.out[((int64_t)bz * p.M + gi) * p.N + gj] = v;
        }
      }
    }
  }
}

// register stages of the prefetch
constexpr int kWideStages = 2;

// column blocks per wave for N columns (BN = 128 CB >= N), or 0 when the wide
// form does not apply
inline int wide_cb(int64_t N) { return N > 256 && N <= 384 ? 3 : (N > 384 && N <= 640 ? 5 : 0); }

template <bool H>
hipError_t launch_wide(const Args& a, bool akc, int cb, hipStream_t s) {
  const unsigned grid = (unsigned)(8 * (((int64_t)a.gx * a.gz + 7) / 8));
  if (cb == 3) {
    if (akc) hipLaunchKernelGGL((gemm16w_kernel<H, true, 3, kWideStages>), dim3(grid), dim3(WNT), 0, s, a);
    else hipLaunchKernelGGL((gemm16w_kernel<H, false, 3, kWideStages>), dim3(grid), dim3(WNT), 0, s, a);
  } else {
    if (akc) hipLaunchKernelGGL((gemm16w_kernel<H, true, 5, kWideStages>), dim3(grid), dim3(WNT), 0, s, a);
    else hipLaunchKernelGGL((gemm16w_kernel<H, false, 5, kWideStages>), dim3(grid), dim3(WNT), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_wide_bf16(const Args& a, bool akc, int cb, hipStream_t s);
hipError_t launch_wide_fp16(const Args& a, bool akc, int cb, hipStream_t s);

}  // namespace g16
}  // namespace idcur
