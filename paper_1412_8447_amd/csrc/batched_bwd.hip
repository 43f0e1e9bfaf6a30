// Batched gradient of the column-ID reconstruction loss with the skeleton
// frozen. For many independent FP32 blocks A_b (m_b x n_b, n_b <= 512) one
// persistent launch computes dA_b = scale * dL_b / dA_b, where
//   Y_b = Omega(:l, :m_b) A_b   (the Gaussian sketch of Section 5.1),
//   T_b = S11^{-1} S12          (the column ID of Section 2.3 on Y_b, as the
//                                fixed-rank batched ID returns it, J_b frozen),
//   E_b = A_b(:,J2) - A_b(:,J1) T_b,   L_b = |E_b|_F^2.
// The derivative through the least-squares T is the one of the single-matrix
// adjoint (Tbar = -2 C^T E, M = (Y1^T Y1)^{-1} Tbar, Ybar2 = Y1 M,
// Ybar1 = (Y2 - Y1 T) M^T - Y1 M T^T, Abar += Omega^T Ybar), rearranged so that
// every block is read in its own column order. With V* = [I T] P^T (k x n:
// column J[s] is e_s, column J[k+t] is T(:, t), Section 2.3):
//   Et = A - C V*     (zero on the skeleton columns, E on the others),
//   Mt = (Y1^T Y1)^{-1} (-2 C^T Et)         (zero on the skeleton columns),
//   Yh = Y1 Mt on the other columns, Ybar1 = (Y - Y1 V*) Mt^T - Y1 (Mt V*^T)
//        on column J[s] (its column s),
//   G  = 2 Et - 2 (Et V*^T) placed at columns J[s] + Omega^T Yh.
//
// One workgroup (4 waves) per block, blocks taken from an atomic counter:
//   pass 1  16-row stripes: Et tiles (K = k), -2 C^T Et and Y = Omega A on the
//           FP32 matrix cores, each element of A loaded once for both
//           reductions. The stripe's rows are assigned to the k steps of the
//           reductions in the order the Et tile's result registers hold them
//           (register r of lane L is row 4 (L / 16) + r), so Et and A feed the
//           next products straight from registers;
//   middle  Y1^T Y1 in FP64, its Cholesky factor and the factor's inverse (one
//           wave, a row or a column per lane), (Y1^T Y1)^{-1} Tbar on the FP64
//           matrix cores, and the l x n and k x k products that form Yh;
//   pass 2  per stripe: Et again (to LDS), Et V*^T (K = n, fixed-order sum of
//           the four waves' parts), then G (K = l), scaled and stored.
// The per-block k x n and l x n intermediates live in a per-workgroup slot of
// the workspace (L2-resident). Every reduction has a fixed order, so results do
// not depend on which workgroup takes a block.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kT = 256;          // threads per workgroup
constexpr int kNmax = 512;       // largest block width
constexpr int kPmax = 64;        // largest rank / sketch rows, padded to 16
constexpr int CS = kPmax + 1;    // LDS row stride of the float k-wide arrays
constexpr int DS = kPmax + 1;    // LDS row stride of the FP64 k x k arrays
constexpr int kESmax = kNmax + 4;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) float gfloat;

// LDS map (bytes): J and its inverse, the C stripe, then one region used by
// pass 2 (Et stripe, the waves' Et V*^T parts) or by the middle phase (Y1,
// the FP64 Gram / Cholesky factor / inverse Gram, the factor's inverse, later
// reused for Mt V*^T).
constexpr int kOffJ = 0;
constexpr int kOffJinv = kOffJ + kNmax * 4;
constexpr int kOffC = kOffJinv + kNmax * 4;
constexpr int kOffU = kOffC + 16 * CS * 4;
constexpr int kOffEst = kOffU;
constexpr int kOffWp = kOffEst + 16 * kESmax * 4;
constexpr int kOffY1 = kOffU;
constexpr int kOffL = kOffY1 + kPmax * CS * 4;
constexpr int kOffLi = kOffL + kPmax * DS * 8;
constexpr int kEndP2 = kOffWp + 4 * 16 * CS * 4;
constexpr int kEndMid = kOffLi + kPmax * DS * 8;
constexpr int kLdsBytes = kEndP2 > kEndMid ? kEndP2 : kEndMid;
static_assert(kOffU % 16 == 0 && kOffL % 8 == 0 && kOffLi % 8 == 0, "LDS alignment");

struct BBArgs {
  int nblk;
  const int* m; const int* n; const int* k;
  const float* const* A; const int64_t* lda;
  const int* const* J; const float* const* T; const int64_t* ldt;
  float* const* dA; const int64_t* ldd;
  const float* omt; int ldom;     // Omega^T: rows up to round_up(mmax, 16), zero past column l
  int mmax, nmax, l, kcap;
  double scale;
  float* slot; int64_t slot_stride; int ldn, kcp, lcp;
  int* queue; int* status;
};

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// A(i, c) of the block, or 0 outside it; the load itself is always issued (at a
// clamped in-range address) and its value masked.
__device__ __forceinline__ float load_or_zero(const float* A, int64_t lda, int i, int c, int m, int n) {
  const bool ok = i < m && c < n;
  const float v = *(gfloat*)(A + (ok ? (int64_t)i * lda + c : 0));
  return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) & (ok ? ~0u : 0u));
}

__device__ __forceinline__ void gather_c_stripe(float* Cst, const float* A, int64_t lda, const int* Jl, int i0,
                                                int m, int k, int kp) {
  for (int e = threadIdx.x; e < 16 * kp; e += kT) {
    const int ii = e / kp, q = e - (e / kp) * kp;
    const int i = i0 + ii;
    Cst[ii * CS + q] = (i < m && q < k) ? A[(int64_t)i * lda + Jl[q]] : 0.0f;
  }
}

__global__ __launch_bounds__(kT, 1) void batched_bwd_kernel(BBArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  int* Jl = reinterpret_cast<int*>(lds + kOffJ);
  int* Jinv = reinterpret_cast<int*>(lds + kOffJinv);
  float* Cst = reinterpret_cast<float*>(lds + kOffC);
  float* Est = reinterpret_cast<float*>(lds + kOffEst);
  float* Wp = reinterpret_cast<float*>(lds + kOffWp);
  float* Y1s = reinterpret_cast<float*>(lds + kOffY1);
  double* Ls = reinterpret_cast<double*>(lds + kOffL);
  double* Lis = reinterpret_cast<double*>(lds + kOffLi);
  float* K2s = reinterpret_cast<float*>(lds + kOffLi);
  __shared__ int sblk;
  __shared__ int sbad;

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, cl = lane & 15;
  const int ldn = a.ldn;
  float* Vs = a.slot + (int64_t)blockIdx.x * a.slot_stride;   // V*      kcp x ldn
  float* Tb = Vs + (int64_t)a.kcp * ldn;                     // Tbar    kcp x ldn
  float* Ms = Tb + (int64_t)a.kcp * ldn;                     // Mt      kcp x ldn
  float* Ys = Ms + (int64_t)a.kcp * ldn;                     // Y       lcp x ldn
  float* Rs = Ys + (int64_t)a.lcp * ldn;                     // Y - Y1 V*
  float* Yb = Rs + (int64_t)a.lcp * ldn;                     // Yh
  const int l = a.l, lp = (l + 15) & ~15, nlt = lp / 16;
  const int ldom = a.ldom;

  for (;;) {
    if (tid == 0) {
      sblk = atomicAdd(a.queue, 1);
      sbad = 0;
    }
    __syncthreads();
    const int b = sblk;
    if (b >= a.nblk) break;
    const int m = a.m[b], n = a.n[b], k = a.k[b];
    if (m < 1 || n < 1 || m > a.mmax || n > a.nmax || k < 0 || k > a.kcap || k > n || a.lda[b] < n ||
        a.ldd[b] < n || a.ldt[b] < n - k) {
      if (tid == 0) set_status(a.status, ST_BADINDEX);
      __syncthreads();   // every thread has read sblk before it changes
      continue;
    }
    const float* Ab = a.A[b];
    const int64_t lda = a.lda[b];
    const int* Jg = a.J[b];
    const float* Tg = a.T[b];
    const int64_t ldt = a.ldt[b];
    const int kp = (k + 15) & ~15, nkt = kp / 16;
    const int NT = (n + 15) / 16;
    const int ncol = NT * 16;

    // ---- J, its inverse, and V* in the slot ------------------------------------
    for (int c = tid; c < n; c += kT) Jinv[c] = -1;
    __syncthreads();
    for (int p = tid; p < n; p += kT) {
      int c = Jg[p];
      if (c < 0 || c >= n) {
        sbad = 1;
        c = c < 0 ? 0 : n - 1;
      }
      Jl[p] = c;
      Jinv[c] = p;
    }
    __syncthreads();
    for (int c = tid; c < n; c += kT)
      if (Jinv[c] < 0) sbad = 1;   // J repeats a column
    for (int e = tid; e < kp * ncol; e += kT) {
      const int q = e / ncol, c = e - (e / ncol) * ncol;
      float v = 0.0f;
      if (q < k && c < n) {
        const int pos = Jinv[c];
        v = pos < 0 ? 0.0f : (pos < k ? (pos == q ? 1.0f : 0.0f) : Tg[(int64_t)q * ldt + (pos - k)]);
      }
      Vs[(int64_t)q * ldn + c] = v;
    }
    __syncthreads();
    if (tid == 0 && sbad) set_status(a.status, ST_BADINDEX);

    // ---- pass 1: Tbar = -2 C^T Et and Y = Omega A ---------------------------------
    for (int c0 = 0; c0 < ncol; c0 += 128) {   // 8 column tiles per group, 2 per wave
      f32x4 tb[2][4], yy[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          tb[j][t] = f32x4{0.f, 0.f, 0.f, 0.f};
          yy[j][t] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      for (int i0 = 0; i0 < m; i0 += 16) {
        __syncthreads();
        gather_c_stripe(Cst, Ab, lda, Jl, i0, m, k, kp);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int c = c0 + 32 * w + 16 * j + cl;
          if (c0 + 32 * w + 16 * j < ncol) {
            float a4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a4[r] = load_or_zero(Ab, lda, i0 + 4 * g + r, c, m, n);
            f32x4 e = f32x4{a4[0], a4[1], a4[2], a4[3]};
            for (int s = 0; s < kp / 4; ++s)
              e = mfma4(-Cst[cl * CS + 4 * s + g], Vs[(int64_t)(4 * s + g) * ldn + c], e);
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (t < nkt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) tb[j][t] = mfma4(Cst[(4 * g + r) * CS + 16 * t + cl], e[r], tb[j][t]);
              }
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (t < nlt) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  yy[j][t] = mfma4(a.omt[(int64_t)(i0 + 4 * g + r) * ldom + 16 * t + cl], a4[r], yy[j][t]);
              }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int c = c0 + 32 * w + 16 * j + cl;
        if (c0 + 32 * w + 16 * j < ncol) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (t < nkt) {
#pragma unroll
              for (int r = 0; r < 4; ++r) Tb[(int64_t)(16 * t + 4 * g + r) * ldn + c] = -2.0f * tb[j][t][r];
            }
            if (t < nlt) {
#pragma unroll
              for (int r = 0; r < 4; ++r) Ys[(int64_t)(16 * t + 4 * g + r) * ldn + c] = yy[j][t][r];
            }
          }
        }
      }
    }
    __syncthreads();

    // ---- middle: Gram, Cholesky, inverse, Mt, Yh -----------------------------------
    for (int e = tid; e < lp * kp; e += kT) {
      const int r = e / kp, p = e - (e / kp) * kp;
      Y1s[r * CS + p] = p < k ? Ys[(int64_t)r * ldn + Jl[p]] : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += kT) {
      const int p = e / k, q = e - (e / k) * k;
      double s = 0.0;
      for (int r = 0; r < lp; ++r) s += (double)Y1s[r * CS + p] * (double)Y1s[r * CS + q];
      Ls[p * DS + q] = s;
    }
    __syncthreads();
    if (w == 0) {
      // Cholesky Y1^T Y1 = L L^T, row `lane` of L (left-looking: step j forms column j)
      bool bad = false;
      for (int j = 0; j < k; ++j) {
        double s = 0.0;
        if (lane >= j && lane < k) {
          s = Ls[lane * DS + j];
          for (int q = 0; q < j; ++q) s -= Ls[lane * DS + q] * Ls[j * DS + q];
        }
        const double d = __shfl(s, j, 64);
        const bool ok = d > 0.0 && __builtin_isfinite(d);
        bad = bad || !ok;
        const double rd = sqrt(ok ? d : 1.0);
        if (lane == j) Ls[j * DS + j] = rd;
        else if (lane > j && lane < k) Ls[lane * DS + j] = s / rd;
      }
      if (bad && lane == 0) set_status(a.status, ST_NONFINITE);
      // X = L^{-1}, column `lane` (zero above the diagonal)
      for (int i = 0; i < k; ++i) {
        double s = i == lane ? 1.0 : 0.0;
        for (int q = 0; q < i; ++q) s -= Ls[i * DS + q] * Lis[q * DS + lane];
        Lis[i * DS + lane] = s / Ls[i * DS + i];
      }
    }
    __syncthreads();
    // (Y1^T Y1)^{-1} = X^T X (kp x kp, zero past k) over the factor's place
    for (int e = tid; e < kp * kp; e += kT) {
      const int p = e / kp, q = e - (e / kp) * kp;
      double s = 0.0;
      if (p < k && q < k)
        for (int i = p > q ? p : q; i < k; ++i) s += Lis[i * DS + p] * Lis[i * DS + q];
      Ls[p * DS + q] = s;
    }
    __syncthreads();
    // Mt = (Y1^T Y1)^{-1} Tbar on the FP64 matrix cores; result register t of
    // lane L is row L/16 + 4t, column L%16 of the tile
    for (int t = w; t < nkt * NT; t += 4) {
      const int ta = t / NT, ct = t - (t / NT) * NT;
      const int c = ct * 16 + cl;
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
      for (int s = 0; s < kp / 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ls[(16 * ta + cl) * DS + 4 * s + g],
                                                   (double)Tb[(int64_t)(4 * s + g) * ldn + c], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ms[(int64_t)(16 * ta + g + 4 * r) * ldn + c] = (float)acc[r];
    }
    __syncthreads();
    // R = Y - Y1 V* and Yh = Y1 Mt (l x n, K = k); K2 = Mt V*^T (k x k, K = n)
    for (int t = w; t < nlt * NT + nkt * nkt; t += 4) {
      if (t < nlt * NT) {
        const int lt = t / NT, ct = t - (t / NT) * NT;
        const int c = ct * 16 + cl;
        f32x4 racc, yacc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int r = 0; r < 4; ++r) racc[r] = Ys[(int64_t)(16 * lt + 4 * g + r) * ldn + c];
        for (int s = 0; s < kp / 4; ++s) {
          const float y1 = Y1s[(16 * lt + cl) * CS + 4 * s + g];
          racc = mfma4(-y1, Vs[(int64_t)(4 * s + g) * ldn + c], racc);
          yacc = mfma4(y1, Ms[(int64_t)(4 * s + g) * ldn + c], yacc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          Rs[(int64_t)(16 * lt + 4 * g + r) * ldn + c] = racc[r];
          Yb[(int64_t)(16 * lt + 4 * g + r) * ldn + c] = yacc[r];
        }
      } else {
        const int u = t - nlt * NT, ta = u / nkt, tq = u - (u / nkt) * nkt;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int s = 0; s < ncol / 4; ++s)
          acc = mfma4(Ms[(int64_t)(16 * ta + cl) * ldn + 4 * s + g], Vs[(int64_t)(16 * tq + cl) * ldn + 4 * s + g], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) K2s[(16 * ta + 4 * g + r) * CS + 16 * tq + cl] = acc[r];
      }
    }
    __syncthreads();
    // Ybar1 = R Mt^T - Y1 K2 (l x k), placed at columns J[s] of Yh
    for (int t = w; t < nlt * nkt; t += 4) {
      const int lt = t / nkt, kt = t - (t / nkt) * nkt;
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int s = 0; s < ncol / 4; ++s)
        acc = mfma4(Rs[(int64_t)(16 * lt + cl) * ldn + 4 * s + g], Ms[(int64_t)(16 * kt + cl) * ldn + 4 * s + g], acc);
      for (int s = 0; s < kp / 4; ++s)
        acc = mfma4(-Y1s[(16 * lt + cl) * CS + 4 * s + g], K2s[(4 * s + g) * CS + 16 * kt + cl], acc);
      const int p = 16 * kt + cl;
      if (p < k) {
        const int c = Jl[p];
#pragma unroll
        for (int r = 0; r < 4; ++r) Yb[(int64_t)(16 * lt + 4 * g + r) * ldn + c] = acc[r];
      }
    }

    // ---- pass 2: G = 2 Et | -2 (Et V*^T) + Omega^T Yh, stripe by stripe -------------
    float* dAb = a.dA[b];
    const int64_t ldd = a.ldd[b];
    const int ES = ldn + 4;
    const float scale = (float)a.scale;
    for (int i0 = 0; i0 < m; i0 += 16) {
      __syncthreads();
      gather_c_stripe(Cst, Ab, lda, Jl, i0, m, k, kp);
      __syncthreads();
      for (int ct = w; ct < NT; ct += 4) {
        const int c = ct * 16 + cl;
        f32x4 e;
#pragma unroll
        for (int r = 0; r < 4; ++r) e[r] = load_or_zero(Ab, lda, i0 + 4 * g + r, c, m, n);
        for (int s = 0; s < kp / 4; ++s)
          e = mfma4(-Cst[cl * CS + 4 * s + g], Vs[(int64_t)(4 * s + g) * ldn + c], e);
#pragma unroll
        for (int r = 0; r < 4; ++r) Est[(4 * g + r) * ES + c] = e[r];
      }
      __syncthreads();
      f32x4 wp[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) wp[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int ct = w; ct < NT; ct += 4) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int cc = ct * 16 + 4 * s + g;
          const float ev = Est[cl * ES + cc];
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (t < nkt) wp[t] = mfma4(ev, Vs[(int64_t)(16 * t + cl) * ldn + cc], wp[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < nkt) {
#pragma unroll
          for (int r = 0; r < 4; ++r) Wp[(16 * w + 4 * g + r) * CS + 16 * t + cl] = wp[t][r];
        }
      __syncthreads();
      for (int ct = w; ct < NT; ct += 4) {
        const int c = ct * 16 + cl;
        const int pos = c < n ? Jinv[c] : -1;
        f32x4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 4 * g + r;
          float v = 0.0f;
          if (pos >= k) {
            v = 2.0f * Est[row * ES + c];
          } else if (pos >= 0) {
            const float s4 = ((Wp[row * CS + pos] + Wp[(16 + row) * CS + pos]) + Wp[(32 + row) * CS + pos]) +
                             Wp[(48 + row) * CS + pos];
            v = -2.0f * s4;
          }
          acc[r] = v;
        }
        for (int s = 0; s < lp / 4; ++s)
          acc = mfma4(a.omt[(int64_t)(i0 + cl) * ldom + 4 * s + g], Yb[(int64_t)(4 * s + g) * ldn + c], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + 4 * g + r;
          if (i < m && c < n) dAb[(int64_t)i * ldd + c] = scale * acc[r];
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace

size_t batched_bwd_lds_bytes() { return (size_t)kLdsBytes; }
int batched_bwd_max_width() { return kNmax; }
int batched_bwd_max_sketch() { return kPmax; }

// Floats of one workgroup's slot: V*, Tbar, Mt (kcp rows each) and Y, Y - Y1 V*,
// Yh (lcp rows each), ldn = round_up(nmax, 16) columns.
int64_t batched_bwd_slot_floats(int kcap, int l, int nmax) {
  const int64_t ldn = round_up(std::max(nmax, 1), 16);
  return (3 * round_up(std::max(kcap, 1), 16) + 3 * round_up(l, 16)) * ldn;
}

int batched_bwd_grid(int nblk, int num_cus) { return std::max(1, std::min(nblk, std::max(num_cus, 1))); }

hipError_t batched_bwd_launch(const BatchedBwdArgs& ba, int grid, hipStream_t stream) {
  if (ba.nblk <= 0) return hipSuccess;
  if (ba.nmax > kNmax || ba.l > kPmax || ba.l < 1 || ba.kcap > kPmax || ba.kcap < 0) return hipErrorInvalidValue;
  BBArgs a{};
  a.nblk = ba.nblk;
  a.m = ba.m; a.n = ba.n; a.k = ba.k;
  a.A = ba.A; a.lda = ba.lda; a.J = ba.J; a.T = ba.T; a.ldt = ba.ldt;
  a.dA = ba.dA; a.ldd = ba.ldd;
  a.omt = ba.omt; a.ldom = ba.ldom;
  a.mmax = ba.mmax; a.nmax = ba.nmax; a.l = ba.l; a.kcap = ba.kcap;
  a.scale = ba.scale;
  a.ldn = (int)round_up(std::max(ba.nmax, 1), 16);
  a.kcp = (int)round_up(std::max(ba.kcap, 1), 16);
  a.lcp = (int)round_up(ba.l, 16);
  a.slot = ba.slot;
  a.slot_stride = batched_bwd_slot_floats(ba.kcap, ba.l, ba.nmax);
  a.queue = ba.queue; a.status = ba.status;
  hipError_t e = zero_launch(ba.queue, sizeof(int), stream);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)batched_bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel((const void*)batched_bwd_kernel, dim3(grid), dim3(kT), args, kLdsBytes, stream);
}

}  // namespace idcur
