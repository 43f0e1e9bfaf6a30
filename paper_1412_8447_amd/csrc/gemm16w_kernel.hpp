// Wide form of the 16-bit thin-output GEMM (gemm16_kernel.hpp) for 256 < N <=
// 640 output columns, the sketch width of rank-500 decompositions (Section 5.1;
// the power steps of Section 5.3): one workgroup computes an 80-row stripe of C
// over all columns, so that its stripe of A (FP32, the big operand) is fetched
// from memory once. With column tiles of at most 256, the same launch would
// fetch every stripe of A once per tile.
//
// Eight waves split the columns (CB blocks of 16 each) and share the 80 rows
// (five row blocks), two waves per SIMD, so that one wave's loads are in flight
// while the other's products run. A, shared by all waves, is rounded to 16 bits
// on its way into LDS. The thin operand B goes straight from memory into the
// matrix-core operand registers: each wave multiplies only its own column
// blocks, so B gains nothing from LDS. B is packed chunk-major (8 consecutive k
// of all padded columns, then the next 8), so lane L of a wave loads B(k0 + 8
// (L / 16) .. +7, column 16 c + L % 16), the operand layout of
// v_mfma_f32_16x16x32, as one 16-byte load at a fixed offset from a base that
// only the k-step moves: no per-lane address arithmetic. B fragments of step t
// sit in register stage t % 2 and are reloaded with step t + 2 as soon as step
// t's products are issued. (With B staged through LDS as well, a 50000x20000
// launch took 2.90 / 2.80 ms for A^T B / A B against 2.33 / 2.60 ms.)
//
// Every global load is unconditional, from a clamped address inside the
// operand: rows of A past M and columns of B past N only feed outputs that are
// never stored, and 8-k chunks of A past the end of the K split are cleared (by
// select) before they reach LDS. B needs no clearing or clamping of columns:
// its padded columns are zero, its chunks past the end of the split meet those
// cleared A chunks (B is finite: the packed sketching matrix or basis), and
// the chunk index is clamped so that no read passes the packed buffer. Nothing
// in the k loop depends on the step count (steps past the end read cleared
// chunks), so the register stages of the prefetch stay in flight together.
// Requires K % 8 == 0, aligned rows (16 bytes for A with k contiguous and for
// the packed B) and K >= 8.
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
  // A chunks: one row, 8 consecutive k (WBM rows x 4 chunks per k-step)
  constexpr int NCA = WBM * 4;
  constexpr int CA = (NCA + WNT - 1) / WNT;
  __shared__ u32x4 As[2][WBM * RS];

  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t W = (int64_t)p.gx * p.gz, per = (W + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= W) return;
  const int bx = (int)(tile % p.gx), bz = (int)(tile / p.gx);
  const int64_t m0 = (int64_t)bx * WBM;
  const int64_t kb = (int64_t)bz * p.kps, ke = min(p.K, kb + p.kps);
  const float s_in = p.scale ? p.scale[0] : 1.0f;
  const float s_out = p.scale ? p.scale[1] : 1.0f;
  const int64_t mlast = p.M - 1;

  // chunk q of a k-step: with k contiguous, four threads read a row's 32 k
  // (128 bytes); with the row index contiguous, 80 threads read one k across
  // the stripe's 80 rows, for each of their 8 k
  auto a_row = [&](int c) {
    const int q = min(tid + WNT * c, NCA - 1);
    return A_KC ? q >> 2 : q % WBM;
  };
  auto a_kg = [&](int c) {
    const int q = min(tid + WNT * c, NCA - 1);
    return A_KC ? (q & 3) : q / WBM;
  };
  // B chunk-major: the 16-byte word (chunk c of 8 k, column j) at byte
  // 16 (c ldb + j), ldb = 128 CB padded columns, zeros past N and past K. This
  // lane's word of a k-step: chunk k0 / 8 + L / 16, column 16 (CB wv + c) + L % 16,
  // at a fixed byte offset from the step's (uniform) base; the column blocks
  // are 256 bytes apart
  const uint32_t boff = (uint32_t)(16 * ((lane >> 4) * p.ldb + wv * CB * 16 + (lane & 15)));

  float fas[D][CA][8];
  u32x4 rbs[2][CB];

  static_assert(CA == 1, "one A chunk per thread and k-step");
  // A addresses: a uniform base per k-step (scalar arithmetic) plus this lane's
  // 32-bit byte offset, so that the loads need no per-lane 64-bit arithmetic.
  // The lane's chunk starts at kc = min(k0 + 8 g, ke - 8) (clamped, like every
  // chunk past the end of the split, to end at ke). The step's base row is
  // kbase = max(min(k0, ke - 32), 0) <= kc, so the offset kc - kbase lies in
  // [0, 24]: the unsigned 32-bit byte offsets never wrap.
  const int g0 = a_kg(0);
  const int64_t gi0 = min(m0 + a_row(0), mlast);
  auto kbase = [&](int64_t k0) { return max<int64_t>(min(k0, ke - 32), 0); };
  auto aload = [&](int64_t k0, float (&fa)[CA][8]) {
    const int64_t kb0 = kbase(k0);
    // kc - kbase = min(8 g + (k0 - kbase), ke - 8 - kbase), both bounds uniform
    const int ko = min(8 * g0 + (int)min<int64_t>(k0 - kb0, 1 << 20), (int)(ke - 8 - kb0));
    typedef float nf4 __attribute__((ext_vector_type(4)));
    if constexpr (A_KC) {
      // (row gi0, kc .. kc + 7): base A + m0 sam + kbase, offset (gi0 - m0) sam + ko
      const char* base = reinterpret_cast<const char*>(p.A + m0 * p.sam + kb0);
      const uint32_t off = (uint32_t)(4 * ((int)(gi0 - m0) * (int)p.sam + ko));
      const nf4 u = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(base + off));
      const nf4 v = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(base + off + 16));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        fa[0][e] = u[e];
        fa[0][4 + e] = v[e];
      }
    } else {
      // (kc + e, row gi0): base A + (kbase + e) sak, offset ko sak + gi0
      const uint32_t off = (uint32_t)(4 * (ko * (int)p.sak + (int)gi0));
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const char* base = reinterpret_cast<const char*>(p.A + (kb0 + e) * p.sak);
        fa[0][e] = __builtin_nontemporal_load(reinterpret_cast<const float*>(base + off));
      }
    }
  };
  auto bload = [&](int64_t k0, u32x4 (&rb)[CB]) {
    // steps past the end of K read the last chunks (their A is cleared)
    const int64_t c8 = min(k0 >> 3, p.kc8max);
    const char* base = reinterpret_cast<const char*>(p.B) + c8 * p.ldb * 16;
#pragma unroll
    for (int c = 0; c < CB; ++c) rb[c] = *reinterpret_cast<const u32x4*>(base + boff + 256 * c);
  };
  auto astore = [&](int buf, int64_t k0, const float (&fa)[CA][8]) {
    if (NCA % WNT == 0 || tid < NCA) {
      // the whole chunk lies in the split (K % 8 == 0)
      const bool kv = 8 * g0 < (int)min<int64_t>(ke - k0, (int64_t)(1 << 30));
      const u32x4 v = pack8<H>(fa[0], s_in);
      As[buf][a_row(0) * RS + g0] = kv ? v : u32x4{0u, 0u, 0u, 0u};
    }
  };

  f32x4 acc[WRB][CB];
#pragma unroll
  for (int i = 0; i < WRB; ++i)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[i][c] = f32x4{0, 0, 0, 0};

  const int64_t nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    // A: step s in register stage s % D, LDS buffer s % 2 while multiplied;
    // B: step s in register stage s % 2
#pragma unroll
    for (int s = 0; s < D; ++s) aload(kb + s * BK, fas[s]);
    bload(kb, rbs[0]);
    bload(kb + BK, rbs[1]);
    astore(0, kb, fas[0]);
    aload(kb + D * BK, fas[0]);
    __syncthreads();
    constexpr int P = D % 2 == 0 ? D : 2 * D;   // unrolled period (a multiple of 2 and D)
    for (int64_t t0 = 0; t0 < nk; t0 += P) {
#pragma unroll
      for (int d = 0; d < P; ++d) {
        const int64_t it = t0 + d;
        const int buf = d & 1;
        const u32x4* as = As[buf];
        u32x4 a[WRB];
#pragma unroll
        for (int i = 0; i < WRB; ++i) a[i] = as[(i * 16 + (lane & 15)) * RS + (lane >> 4)];
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
          for (int i = 0; i < WRB; ++i) acc[i][c] = mfma16<H>(a[i], rbs[buf][c], acc[i][c]);
        bload(kb + (it + 2) * BK, rbs[buf]);
        const int sn = (d + 1) % D;
        astore(buf ^ 1, kb + (it + 1) * BK, fas[sn]);
        aload(kb + (it + 1 + D) * BK, fas[sn]);
        __syncthreads();
      }
    }
  }

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

// register stages of A's prefetch (four measured the same as two)
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
