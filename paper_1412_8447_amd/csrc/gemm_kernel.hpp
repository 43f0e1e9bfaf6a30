// Thin-output MFMA GEMM kernel template (see gemm.hip for the design notes).
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace gk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64;
constexpr int BK = 16;

template <typename TAcc> struct AccVec;
template <> struct AccVec<float> { using type = f32x4; };
template <> struct AccVec<double> { using type = f64x4; };

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS row strides chosen so that the 4 k-rows touched by one MFMA operand read
// start on different bank groups.
template <typename TAcc>
__host__ __device__ constexpr int lds_stride(int w) {
  return sizeof(TAcc) == 4 ? (w + ((16 - (w % 64)) % 64 + 64) % 64) : (w + ((16 - (w % 32)) % 32 + 32) % 32);
}

struct KArgs {
  int64_t M, N, K;
  const void* A; int64_t sam, sak;
  const void* B; int64_t sbk, sbn;
  void* out; int64_t ldo;      // C (direct) or partial buffer (ld = N)
  int64_t kps;                 // K per split (multiple of BK)
  int direct;                  // 1: write C with alpha/beta/out_type
  int out_type;
  double alpha, beta;
  int vec_a, vec_b;            // 4-wide vector loads allowed
  const int* m_dev; const int* n_dev;
  // residual mode: accumulate sum (X - A*B)^2 over the tile instead of storing
  const void* X; int64_t ldx; int x_type; double* rpart;
  const int* k_dev;            // optional device bound on K
  int gx, gy, gz;              // tile grid: row stripes, column tiles, K splits
  int lower;                   // skip tiles wholly above the diagonal (square C)
};

// Tiles are numbered t = x + gx*(y + gy*z) (z = K split). The launch is 1-D with
// 8*ceil(W/8) workgroups, and workgroup `lin` takes tile (lin % 8)*ceil(W/8) +
// lin / 8. Workgroups are handed to the 8 XCDs round-robin by `lin`, so each XCD
// gets one contiguous range of tiles: the tiles of one K split, whose slice of
// the thin operand then stays in that XCD's L2 instead of being re-read from the
// Infinity Cache by every XCD.
__host__ __device__ inline int64_t tiles_total(const KArgs& p) { return (int64_t)p.gx * p.gy * p.gz; }
__host__ inline unsigned xcd_grid(const KArgs& p) { return (unsigned)(8 * ((tiles_total(p) + 7) / 8)); }

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

template <typename T>
__device__ __forceinline__ void load4(const T* base, int64_t off, int nvalid, bool vec, T (&r)[4]) {
  if (vec && nvalid >= 4) {
    const typename V4<T>::type q = *reinterpret_cast<const typename V4<T>::type*>(base + off);
    r[0] = q.x; r[1] = q.y; r[2] = q.z; r[3] = q.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = (e < nvalid) ? base[off + e] : (T)0;
  }
}

template <typename TA, typename TB, typename TAcc, int NT, bool A_KC, bool B_NC, bool RESID = false>
__global__ __launch_bounds__(256) void gemm_kernel(KArgs p) {
  constexpr int BN = 16 * NT;
  constexpr int SA = lds_stride<TAcc>(BM);
  constexpr int SB = lds_stride<TAcc>(BN);
  constexpr int BQ = (BN * BK / 4 + 255) / 256;   // B quads per thread
  __shared__ TAcc As[2][BK * SA];
  __shared__ TAcc Bs[2][BK * SB];

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t W = tiles_total(p), per = (W + 7) / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= W) return;
  const int bx = (int)(tile % p.gx), by = (int)((tile / p.gx) % p.gy), bz = (int)(tile / ((int64_t)p.gx * p.gy));
  const int64_t Mb = p.m_dev ? min((int64_t)*p.m_dev, p.M) : p.M;
  const int64_t Nb = p.n_dev ? min((int64_t)*p.n_dev, p.N) : p.N;
  const int64_t m0 = (int64_t)bx * BM;
  const int64_t n0 = (int64_t)by * BN;
  if (m0 >= Mb || n0 >= Nb) {
    if (RESID && threadIdx.x == 0) p.rpart[(int64_t)by * p.gx + bx] = 0.0;
    return;
  }
  if (!RESID && p.lower && n0 >= m0 + BM) return;
  const int64_t Kb = p.k_dev ? min((int64_t)*p.k_dev, p.K) : p.K;
  const int64_t kb = (int64_t)bz * p.kps;
  const int64_t ke = min(Kb, kb + p.kps);
  const TA* A = static_cast<const TA*>(p.A);
  const TB* B = static_cast<const TB*>(p.B);

  TA ra[4];
  TB rb[BQ][4];

  auto gload = [&](int64_t k0) {
    // A tile: BM x BK
    if (A_KC) {
      // a wave takes one k-quad of 64 rows: its transposing LDS stores below
      // then hit 64 consecutive words (no bank conflicts)
      const int row = tid & 63, kq = (tid >> 6) * 4;
      const int64_t gi = m0 + row, gk = k0 + kq;
      const int nv = (gi < Mb) ? (int)max((int64_t)0, min((int64_t)4, ke - gk)) : 0;
      load4(A, gi * p.sam + gk, nv, p.vec_a, ra);
    } else {
      const int kr = tid >> 4, iq = (tid & 15) * 4;
      const int64_t gk = k0 + kr, gi = m0 + iq;
      const int nv = (gk < ke) ? (int)max((int64_t)0, min((int64_t)4, Mb - gi)) : 0;
      load4(A, gk * p.sak + gi, nv, p.vec_a, ra);
    }
    // B tile: BK x BN
#pragma unroll
    for (int qq = 0; qq < BQ; ++qq) {
      const int q = tid + qq * 256;
      if (q < BN * BK / 4) {
        if (B_NC) {
          const int kr = q / (BN / 4), jq = (q % (BN / 4)) * 4;
          const int64_t gk = k0 + kr, gj = n0 + jq;
          const int nv = (gk < ke) ? (int)max((int64_t)0, min((int64_t)4, Nb - gj)) : 0;
          load4(B, gk * p.sbk + gj, nv, p.vec_b, rb[qq]);
        } else {
          const int jc = q >> 2, kq = (q & 3) * 4;
          const int64_t gj = n0 + jc, gk = k0 + kq;
          const int nv = (gj < Nb) ? (int)max((int64_t)0, min((int64_t)4, ke - gk)) : 0;
          load4(B, gj * p.sbn + gk, nv, p.vec_b, rb[qq]);
        }
      }
    }
  };
  auto sstore = [&](int buf) {
    TAcc* as = As[buf];
    TAcc* bs = Bs[buf];
    if (A_KC) {
      const int row = tid & 63, kq = (tid >> 6) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) as[(kq + e) * SA + row] = (TAcc)ra[e];
    } else {
      const int kr = tid >> 4, iq = (tid & 15) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) as[kr * SA + iq + e] = (TAcc)ra[e];
    }
#pragma unroll
    for (int qq = 0; qq < BQ; ++qq) {
      const int q = tid + qq * 256;
      if (q < BN * BK / 4) {
        if (B_NC) {
          const int kr = q / (BN / 4), jq = (q % (BN / 4)) * 4;
#pragma unroll
          for (int e = 0; e < 4; ++e) bs[kr * SB + jq + e] = (TAcc)rb[qq][e];
        } else {
          const int jc = q >> 2, kq = (q & 3) * 4;
#pragma unroll
          for (int e = 0; e < 4; ++e) bs[(kq + e) * SB + jc] = (TAcc)rb[qq][e];
        }
      }
    }
  };

  using AV = typename AccVec<TAcc>::type;
  AV acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = AV{0, 0, 0, 0};

  const int64_t ntile = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (ntile > 0) {
    gload(kb);
    sstore(0);
    __syncthreads();
    for (int64_t it = 0; it < ntile; ++it) {
      const int buf = (int)(it & 1);
      if (it + 1 < ntile) gload(kb + (it + 1) * BK);
      // operands of the next 4-deep k step are read before this step's MFMAs
      // issue (a scheduling barrier keeps them apart), so LDS latency overlaps
      // the matrix cores instead of stalling every pair of MFMAs
      const TAcc* as = As[buf] + (lane >> 4) * SA + wv * 16 + (lane & 15);
      const TAcc* bs = Bs[buf] + (lane >> 4) * SB + (lane & 15);
      TAcc av[2];
      TAcc bv[2][NT];
      av[0] = as[0];
#pragma unroll
      for (int t = 0; t < NT; ++t) bv[0][t] = bs[t * 16];
#pragma unroll
      for (int kq = 0; kq < BK / 4; ++kq) {
        const int cur = kq & 1, nxt = cur ^ 1;
        if (kq + 1 < BK / 4) {
          av[nxt] = as[(kq + 1) * 4 * SA];
#pragma unroll
          for (int t = 0; t < NT; ++t) bv[nxt][t] = bs[(kq + 1) * 4 * SB + t * 16];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma(av[cur], bv[cur][t], acc[t]);
      }
      if (it + 1 < ntile) sstore(buf ^ 1);
      __syncthreads();
    }
  }

  if (RESID) {
    // sum of squared residuals of this tile, reduced in a fixed order
    __shared__ double wsum[4];
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = (sizeof(TAcc) == 4) ? (4 * (lane >> 4) + r) : ((lane >> 4) + 4 * r);
        const int64_t gi = m0 + wv * 16 + rl;
        const int64_t gj = n0 + t * 16 + (lane & 15);
        if (gi < Mb && gj < Nb) {
          const double x = p.x_type == 1 ? (double)static_cast<const float*>(p.X)[gi * p.ldx + gj]
                                         : static_cast<const double*>(p.X)[gi * p.ldx + gj];
          const double d = x - p.alpha * (double)acc[t][r];
          s += d * d;
        }
      }
    }
    s = wave_sum(s);
    if (lane == 0) wsum[wv] = s;
    __syncthreads();
    if (tid == 0) p.rpart[(int64_t)by * p.gx + bx] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
    return;
  }
  // epilogue
#pragma unroll
  for (int t = 0; t < NT; ++t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rl = (sizeof(TAcc) == 4) ? (4 * (lane >> 4) + r) : ((lane >> 4) + 4 * r);
      const int64_t gi = m0 + wv * 16 + rl;
      const int64_t gj = n0 + t * 16 + (lane & 15);
      if (gi < Mb && gj < Nb) {
        const TAcc v = acc[t][r];
        if (p.direct) {
          if (p.out_type == 1) {
            float* C = static_cast<float*>(p.out) + gi * p.ldo + gj;
            const double o = p.beta != 0.0 ? p.beta * (double)*C : 0.0;
            *C = (float)(p.alpha * (double)v + o);
          } else {
            double* C = static_cast<double*>(p.out) + gi * p.ldo + gj;
            const double o = p.beta != 0.0 ? p.beta * *C : 0.0;
            *C = p.alpha * (double)v + o;
          }
        } else {
          TAcc* P = static_cast<TAcc*>(p.out) + ((int64_t)bz * p.M + gi) * p.N + gj;
          *P = v;
        }
      }
    }
  }
}

template <typename TAcc>
__global__ __launch_bounds__(256) void splitk_reduce(const TAcc* part, int splitk, int64_t M, int64_t N,
                                                     void* C, int64_t ldc, int out_type, double alpha,
                                                     double beta, const int* m_dev, const int* n_dev) {
  const int64_t Mb = m_dev ? min((int64_t)*m_dev, M) : M;
  const int64_t Nb = n_dev ? min((int64_t)*n_dev, N) : N;
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / N, j = e % N;
    if (i >= Mb || j >= Nb) continue;
    // the partial sums in split order, eight loads in flight at a time
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= splitk; z += 8) {
      TAcc v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * total + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += (double)v[u];
    }
    for (; z < splitk; ++z) s += (double)part[(int64_t)z * total + e];
    if (out_type == 1) {
      float* c = static_cast<float*>(C) + i * ldc + j;
      *c = (float)(alpha * s + (beta != 0.0 ? beta * (double)*c : 0.0));
    } else {
      double* c = static_cast<double*>(C) + i * ldc + j;
      *c = alpha * s + (beta != 0.0 ? beta * *c : 0.0);
    }
  }
}


template <typename TA, typename TB, typename TAcc, int NT>
hipError_t launch_nt(const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s) {
  if (akc && bnc) hipLaunchKernelGGL((gemm_kernel<TA, TB, TAcc, NT, true, true>), grid, dim3(256), 0, s, k);
  else if (akc && !bnc) hipLaunchKernelGGL((gemm_kernel<TA, TB, TAcc, NT, true, false>), grid, dim3(256), 0, s, k);
  else if (!akc && bnc) hipLaunchKernelGGL((gemm_kernel<TA, TB, TAcc, NT, false, true>), grid, dim3(256), 0, s, k);
  else hipLaunchKernelGGL((gemm_kernel<TA, TB, TAcc, NT, false, false>), grid, dim3(256), 0, s, k);
  return hipGetLastError();
}

template <typename TA, typename TB, typename TAcc>
hipError_t launch_types(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s) {
  switch (nt) {
    case 2: return launch_nt<TA, TB, TAcc, 2>(k, grid, akc, bnc, s);
    case 4: return launch_nt<TA, TB, TAcc, 4>(k, grid, akc, bnc, s);
    case 8: return launch_nt<TA, TB, TAcc, 8>(k, grid, akc, bnc, s);
    case 14: return launch_nt<TA, TB, TAcc, 14>(k, grid, akc, bnc, s);
    default: return launch_nt<TA, TB, TAcc, 16>(k, grid, akc, bnc, s);
  }
}

// One translation unit per type combination (parallel compilation).
hipError_t launch_f32(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s);        // f32 f32 -> f32 acc
hipError_t launch_f32_f64acc(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s); // f32 f32 -> f64 acc
hipError_t launch_f64(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s);        // f64 f64
hipError_t launch_f32_f64(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s);    // f32 x f64
hipError_t launch_f64_f32(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s);    // f64 x f32

}  // namespace gk
}  // namespace idcur
