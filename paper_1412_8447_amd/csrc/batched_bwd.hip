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
//   middle  Y1^T Y1 in FP64, its Cholesky factor and the factor's inverse in
//           one wave's registers (a row, then a column, per lane),
//           (Y1^T Y1)^{-1} Tbar on the FP64 matrix cores, and the l x n and
//           k x k products that form Yh;
//   pass 2  per stripe: Et again (in LDS, over the stripe's A), Et V*^T (K = n,
//           fixed-order sum of the waves' parts), then G (K = l), scaled and
//           stored.
// Both passes load the next stripe's A elements, gathered skeleton columns and
// Omega^T rows while the current stripe is multiplied. V* and Yh, the operands
// every stripe reads, stay in LDS when they fit (else in the workgroup's slot
// of the workspace, like the other per-block intermediates). Every reduction
// has a fixed order, so results do not depend on which workgroup takes a block.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kT = 256;          // threads per workgroup
constexpr int kW = kT / 64;      // waves
constexpr int kNmax = 512;       // largest block width
constexpr int kPmax = 64;        // largest rank / sketch rows, padded to 16
constexpr int kTPW = kNmax / 16 / kW;   // most pass-2 column tiles per wave
constexpr int kLdsCap = 160 * 1024;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) float gfloat;

// LDS map (bytes), for padded rank KP, padded sketch rows LP and row length
// ldn: J and its inverse, two C stripes, then one region used either by pass 2
// (two A / Et stripes, the waves' Et V*^T parts) or by the middle phase (Y1, the FP64
// factor / inverse Gram, the factor's inverse, later Mt V*^T), then (when they
// fit) V* and Yh.
struct LdsMap {
  int jl, jinv, cst, est, wp, y1, lf, li, vs, yb, total;
  int CS, ES, VS, YS;
};
__host__ __device__ inline int r16(int x) { return (x + 15) & ~15; }
__host__ __device__ inline LdsMap lds_map(int KP, int LP, int ldn, bool vl) {
  LdsMap mp{};
  mp.CS = KP + 1;
  mp.ES = ldn + 4;
  mp.VS = vl ? ((ldn + 63) & ~63) + 20 : ldn;
  mp.YS = vl ? ((ldn + 63) & ~63) + 16 : ldn;
  int off = 0;
  mp.jl = off; off += ldn * 4;
  mp.jinv = off; off += ldn * 4;
  mp.cst = off; off = r16(off + 2 * 16 * mp.CS * 4);
  const int u = off;
  mp.est = u;
  mp.wp = r16(u + 2 * 16 * mp.ES * 4);
  const int e2 = mp.wp + kW * 16 * mp.CS * 4;
  mp.y1 = u;
  mp.lf = r16(u + LP * mp.CS * 4);
  mp.li = mp.lf + KP * (KP + 1) * 8;
  const int e3 = mp.li + KP * (KP + 1) * 8;
  off = r16(e2 > e3 ? e2 : e3);
  mp.vs = off;
  mp.yb = off;
  if (vl) {
    off += KP * mp.VS * 4;
    mp.yb = off;
    off += LP * mp.YS * 4;
  }
  mp.total = off;
  return mp;
}

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

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// The 16 x KP stripe C(i0:i0+16, :) = A(i0:i0+16, J[0:k]) (zero past m and k),
// CG elements per thread: loaded to registers, then stored to LDS.
template <int KP>
struct CStripe {
  static constexpr int CG = (16 * KP + kT - 1) / kT;
  float v[CG];
  __device__ __forceinline__ void load(const float* A, int64_t lda, const int* Jl, int i0, int m, int k) {
#pragma unroll
    for (int u = 0; u < CG; ++u) {
      const int e = threadIdx.x + kT * u;
      const int ii = e / KP, q = e % KP;
      const bool ok = e < 16 * KP && i0 + ii < m && q < k;
      const float x = *(gfloat*)(A + (ok ? (int64_t)(i0 + ii) * lda + Jl[q] : 0));
      v[u] = __builtin_bit_cast(float, __builtin_bit_cast(unsigned, x) & (ok ? ~0u : 0u));
    }
  }
  __device__ __forceinline__ void store(float* Cb, int CS) const {
#pragma unroll
    for (int u = 0; u < CG; ++u) {
      const int e = threadIdx.x + kT * u;
      if (e < 16 * KP) Cb[(e / KP) * CS + e % KP] = v[u];
    }
  }
};

// KP = the rank cap rounded up to 16, LP = l rounded up to 16: every product's
// depth is a compile-time constant, so each chain of matrix-core steps and the
// loads that feed it are unrolled and issued together. A block of smaller rank
// k_b runs with zero rows past k_b in V*, C, Tbar and Mt. VL: V* and Yh in LDS.
template <int KP, int LP, bool VL>
__global__ __launch_bounds__(kT, 1) void batched_bwd_kernel(BBArgs a) {
  constexpr int nkt = KP / 16, nlt = LP / 16;
  // pass-1 column tiles per wave and column group: about 64 accumulator registers
  constexpr int kCPW = 16 / (nkt + nlt) < 1 ? 1 : (16 / (nkt + nlt) > 4 ? 4 : 16 / (nkt + nlt));
  extern __shared__ __align__(16) unsigned char lds[];
  const int ldn = a.ldn;
  const LdsMap mp = lds_map(KP, LP, ldn, VL);
  const int CS = mp.CS, ES = mp.ES, VS = mp.VS, YS = mp.YS;
  constexpr int DS = KP + 1;
  int* Jl = reinterpret_cast<int*>(lds + mp.jl);
  int* Jinv = reinterpret_cast<int*>(lds + mp.jinv);
  float* Cst = reinterpret_cast<float*>(lds + mp.cst);
  float* Est = reinterpret_cast<float*>(lds + mp.est);
  float* Wp = reinterpret_cast<float*>(lds + mp.wp);
  float* Y1s = reinterpret_cast<float*>(lds + mp.y1);
  double* Ls = reinterpret_cast<double*>(lds + mp.lf);
  double* Lis = reinterpret_cast<double*>(lds + mp.li);
  float* K2s = reinterpret_cast<float*>(lds + mp.li);
  __shared__ int sblk;
  __shared__ int sbad;

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, cl = lane & 15;
  float* slot = a.slot + (int64_t)blockIdx.x * a.slot_stride;
  float* Tb = slot + (int64_t)a.kcp * ldn;                   // Tbar    kcp x ldn
  float* Ms = Tb + (int64_t)a.kcp * ldn;                     // Mt      kcp x ldn
  float* Ys = Ms + (int64_t)a.kcp * ldn;                     // Y       lcp x ldn
  float* Rs = Ys + (int64_t)a.lcp * ldn;                     // Y - Y1 V*
  float* Vs = VL ? reinterpret_cast<float*>(lds + mp.vs) : slot;                            // V*
  float* Yb = VL ? reinterpret_cast<float*>(lds + mp.yb) : Rs + (int64_t)a.lcp * ldn;       // Yh
  const int ldom = a.ldom;
  const float* omt = a.omt;

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
    const int NT = (n + 15) / 16;
    const int ncol = NT * 16;

    // ---- J, its inverse, and V* ------------------------------------------------
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
    // V*: zero, then column J[s] = e_s (s < k) and column J[k+t] = T(:, t), T read
    // along its rows
    for (int e = tid; e < KP * ncol; e += kT) Vs[(e / ncol) * VS + e % ncol] = 0.0f;
    __syncthreads();
    for (int p = tid; p < k; p += kT) Vs[p * VS + Jl[p]] = 1.0f;
    for (int e = tid; e < k * (n - k); e += kT) {
      const int q = e / (n - k), t = e - (e / (n - k)) * (n - k);
      Vs[q * VS + Jl[k + t]] = Tg[(int64_t)q * ldt + t];
    }
    __syncthreads();
    if (tid == 0 && sbad) set_status(a.status, ST_BADINDEX);

    // ---- pass 1: Tbar = -2 C^T Et and Y = Omega A, kCPW column tiles per wave -----
    for (int c0 = 0; c0 < ncol; c0 += 16 * kCPW * kW) {
      f32x4 tb[kCPW][nkt], yy[kCPW][nlt];
#pragma unroll
      for (int j = 0; j < kCPW; ++j) {
#pragma unroll
        for (int t = 0; t < nkt; ++t) tb[j][t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < nlt; ++t) yy[j][t] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      CStripe<KP> cs;
      float av[kCPW][4], an[kCPW][4], ov[nlt][4], on[nlt][4];
      cs.load(Ab, lda, Jl, 0, m, k);
#pragma unroll
      for (int j = 0; j < kCPW; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) av[j][r] = load_or_zero(Ab, lda, 4 * g + r, c0 + 16 * (kCPW * w + j) + cl, m, n);
#pragma unroll
      for (int t = 0; t < nlt; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) ov[t][r] = omt[(4 * g + r) * ldom + 16 * t + cl];
      __syncthreads();
      cs.store(Cst, CS);
      __syncthreads();
      int buf = 0;
      for (int i0 = 0; i0 < m; i0 += 16) {
        const bool more = i0 + 16 < m;
        if (more) {   // next stripe, in flight during this one
          cs.load(Ab, lda, Jl, i0 + 16, m, k);
#pragma unroll
          for (int j = 0; j < kCPW; ++j)
            if (c0 + 16 * (kCPW * w + j) < ncol) {   // uniform per wave
#pragma unroll
              for (int r = 0; r < 4; ++r)
                an[j][r] = load_or_zero(Ab, lda, i0 + 16 + 4 * g + r, c0 + 16 * (kCPW * w + j) + cl, m, n);
            }
#pragma unroll
          for (int t = 0; t < nlt; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) on[t][r] = omt[(i0 + 16 + 4 * g + r) * ldom + 16 * t + cl];
        }
        const float* Cc = Cst + buf * 16 * CS;
#pragma unroll
        for (int j = 0; j < kCPW; ++j) {
          const int c = c0 + 16 * (kCPW * w + j) + cl;
          if (c0 + 16 * (kCPW * w + j) < ncol) {   // uniform per wave
            f32x4 e = f32x4{av[j][0], av[j][1], av[j][2], av[j][3]};
#pragma unroll
            for (int s = 0; s < KP / 4; ++s) e = mfma4(-Cc[cl * CS + 4 * s + g], Vs[(4 * s + g) * VS + c], e);
#pragma unroll
            for (int t = 0; t < nkt; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r) tb[j][t] = mfma4(Cc[(4 * g + r) * CS + 16 * t + cl], e[r], tb[j][t]);
#pragma unroll
            for (int t = 0; t < nlt; ++t)
#pragma unroll
              for (int r = 0; r < 4; ++r) yy[j][t] = mfma4(ov[t][r], av[j][r], yy[j][t]);
          }
        }
        if (more) {
          cs.store(Cst + (buf ^ 1) * 16 * CS, CS);
#pragma unroll
          for (int j = 0; j < kCPW; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) av[j][r] = an[j][r];
#pragma unroll
          for (int t = 0; t < nlt; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) ov[t][r] = on[t][r];
        }
        __syncthreads();
        buf ^= 1;
      }
#pragma unroll
      for (int j = 0; j < kCPW; ++j) {
        const int c = c0 + 16 * (kCPW * w + j) + cl;
        if (c0 + 16 * (kCPW * w + j) < ncol) {
#pragma unroll
          for (int t = 0; t < nkt; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) Tb[(int64_t)(16 * t + 4 * g + r) * ldn + c] = -2.0f * tb[j][t][r];
#pragma unroll
          for (int t = 0; t < nlt; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) Ys[(int64_t)(16 * t + 4 * g + r) * ldn + c] = yy[j][t][r];
        }
      }
    }
    __syncthreads();

    // ---- middle: Gram, Cholesky, inverse, Mt, Yh -----------------------------------
    for (int e = tid; e < LP * KP; e += kT) {
      const int r = e / KP, p = e % KP;
      Y1s[r * CS + p] = p < k ? Ys[(int64_t)r * ldn + Jl[p]] : 0.0f;
    }
    __syncthreads();
    for (int e = tid; e < KP * KP; e += kT) {
      const int p = e / KP, q = e % KP;
      double s = 0.0;
      if (p < k && q < k) {
#pragma unroll 8
        for (int r = 0; r < LP; ++r) s += (double)Y1s[r * CS + p] * (double)Y1s[r * CS + q];
      } else {
        s = p == q ? 1.0 : 0.0;   // the padded Gram matrix is diag(Y1^T Y1, I)
      }
      Ls[p * DS + q] = s;
    }
    __syncthreads();
    if (w == 0) {
      // the padded Gram matrix diag(Y1^T Y1, I) -> its Cholesky factor L in Ls
      // and X = L^{-1} in Lis: in registers for KP <= 32, in LDS above (the
      // register form of order 48 or 64 does not fit beside the rest)
      if constexpr (KP <= 32) {
      // Cholesky of the padded Gram matrix in registers: lane i holds row i
      // (lanes past KP hold zeros). Step j divides column j by the root of the
      // diagonal (lane j's own entry becomes that root) and passes the column
      // through LDS (one wave's LDS accesses complete in program order); every
      // lane then updates its whole row. Entries right of a lane's diagonal
      // only ever combine with each other and are dropped at the end.
      const int i = lane;
      // an offset the compiler cannot see to be zero and uniform: the broadcast
      // LDS reads below stay vector loads instead of being hoisted as scalars
      int zo = 0;
      asm volatile("" : "+v"(zo));
      double* col = Lis + zo;   // broadcast buffer; the inverse is written after
      double row[KP];
#pragma unroll
      for (int q = 0; q < KP; ++q) row[q] = i < KP ? Ls[(i < KP ? i : 0) * DS + q] : 0.0;
      bool bad = false;
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        const double d = readlane_f64(row[j], j);
        const bool ok = d > 0.0 && __builtin_isfinite(d);
        bad = bad || !ok;
        const double inv = 1.0 / sqrt(ok ? d : 1.0);
        row[j] *= inv;
        col[i] = row[j];
#pragma unroll
        for (int q = j + 1; q < KP; ++q) row[q] -= row[j] * col[q];
      }
      if (bad && lane == 0) set_status(a.status, ST_NONFINITE);
      if (i < KP) {
#pragma unroll
        for (int q = 0; q < KP; ++q) Ls[i * DS + q] = q <= i ? row[q] : 0.0;
      }
      // X = L^{-1} in registers, lane c holds column c: row j of X is final
      // once divided by L(j,j), then every later row r subtracts L(r,j) X(j,c)
      const int c = lane;
      double x[KP];
#pragma unroll
      for (int r = 0; r < KP; ++r) x[r] = r == c ? 1.0 : 0.0;
      const double* Lz = Ls + zo;
#pragma unroll
      for (int j = 0; j < KP; ++j) {
        const double xj = x[j] / Lz[j * DS + j];
        x[j] = xj;
#pragma unroll
        for (int r = j + 1; r < KP; ++r) x[r] -= Lz[r * DS + j] * xj;
      }
      if (c < KP) {
#pragma unroll
        for (int r = 0; r < KP; ++r) Lis[r * DS + c] = x[r];
      }
      } else {
      // Cholesky in place in LDS (right-looking, lane i owns row i): step j
      // scales column j, then row i subtracts L(i,j) L(q,j) for j < q <= i.
      // One wave's LDS accesses complete in program order, so a lane reads
      // what another lane wrote earlier.
      bool bad = false;
      const int i = lane;
      for (int j = 0; j < KP; ++j) {
        const double d = Ls[j * DS + j];
        const bool ok = d > 0.0 && __builtin_isfinite(d);
        bad = bad || !ok;
        const double rd = sqrt(ok ? d : 1.0);
        const double inv = 1.0 / rd;
        double lij = 0.0;
        if (i > j && i < KP) {
          lij = Ls[i * DS + j] * inv;
          Ls[i * DS + j] = lij;
        }
        if (i == j) Ls[j * DS + j] = rd;
        if (i > j && i < KP)
          for (int q = j + 1; q <= i; ++q) Ls[i * DS + q] -= lij * Ls[q * DS + j];
      }
      if (bad && lane == 0) set_status(a.status, ST_NONFINITE);
      if (i < KP)
        for (int q = i + 1; q < KP; ++q) Ls[i * DS + q] = 0.0;
      // X = L^{-1} (right-looking, lane c owns column c)
      const int c = lane;
      if (c < KP) {
        for (int r = 0; r < KP; ++r) Lis[r * DS + c] = r == c ? 1.0 : 0.0;
        for (int j = 0; j < KP; ++j) {
          const double xj = Lis[j * DS + c] / Ls[j * DS + j];
          Lis[j * DS + c] = xj;
          for (int r = j + 1; r < KP; ++r) Lis[r * DS + c] -= Ls[r * DS + j] * xj;
        }
      }
      }
    }
    __syncthreads();
    // (Y1^T Y1)^{-1} = X^T X (KP x KP, zero past k) over the factor's place
    for (int e = tid; e < KP * KP; e += kT) {
      const int p = e / KP, q = e % KP;
      double s = 0.0;
      if (p < k && q < k)
        for (int r = p > q ? p : q; r < k; ++r) s += Lis[r * DS + p] * Lis[r * DS + q];
      Ls[p * DS + q] = s;
    }
    __syncthreads();
    // Mt = (Y1^T Y1)^{-1} Tbar on the FP64 matrix cores; result register t of
    // lane L is row L/16 + 4t, column L%16 of the tile
#pragma unroll 2
    for (int t = w; t < nkt * NT; t += kW) {
      const int ta = t / NT, ct = t - (t / NT) * NT;
      const int c = ct * 16 + cl;
      f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KP / 4; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ls[(16 * ta + cl) * DS + 4 * s + g],
                                                   (double)Tb[(int64_t)(4 * s + g) * ldn + c], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) Ms[(int64_t)(16 * ta + g + 4 * r) * ldn + c] = (float)acc[r];
    }
    __syncthreads();
    // R = Y - Y1 V* and Yh = Y1 Mt (l x n, K = k); K2 = Mt V*^T (k x k, K = n)
#pragma unroll 2
    for (int t = w; t < nlt * NT; t += kW) {
      const int lt = t / NT, ct = t - (t / NT) * NT;
      const int c = ct * 16 + cl;
      f32x4 racc, yacc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) racc[r] = Ys[(int64_t)(16 * lt + 4 * g + r) * ldn + c];
#pragma unroll
      for (int s = 0; s < KP / 4; ++s) {
        const float y1 = Y1s[(16 * lt + cl) * CS + 4 * s + g];
        racc = mfma4(-y1, Vs[(4 * s + g) * VS + c], racc);
        yacc = mfma4(y1, Ms[(int64_t)(4 * s + g) * ldn + c], yacc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Rs[(int64_t)(16 * lt + 4 * g + r) * ldn + c] = racc[r];
        Yb[(16 * lt + 4 * g + r) * YS + c] = yacc[r];
      }
    }
    for (int u = w; u < nkt * nkt; u += kW) {
      const int ta = u / nkt, tq = u - (u / nkt) * nkt;
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 16
      for (int s = 0; s < ncol / 4; ++s)
        acc = mfma4(Ms[(int64_t)(16 * ta + cl) * ldn + 4 * s + g], Vs[(16 * tq + cl) * VS + 4 * s + g], acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) K2s[(16 * ta + 4 * g + r) * CS + 16 * tq + cl] = acc[r];
    }
    __syncthreads();
    // Ybar1 = R Mt^T - Y1 K2 (l x k), placed at columns J[s] of Yh
    for (int t = w; t < nlt * nkt; t += kW) {
      const int lt = t / nkt, kt = t - (t / nkt) * nkt;
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 16
      for (int s = 0; s < ncol / 4; ++s)
        acc = mfma4(Rs[(int64_t)(16 * lt + cl) * ldn + 4 * s + g], Ms[(int64_t)(16 * kt + cl) * ldn + 4 * s + g], acc);
#pragma unroll
      for (int s = 0; s < KP / 4; ++s)
        acc = mfma4(-Y1s[(16 * lt + cl) * CS + 4 * s + g], K2s[(4 * s + g) * CS + 16 * kt + cl], acc);
      const int p = 16 * kt + cl;
      if (p < k) {
        const int c = Jl[p];
#pragma unroll
        for (int r = 0; r < 4; ++r) Yb[(16 * lt + 4 * g + r) * YS + c] = acc[r];
      }
    }
    __syncthreads();

    // ---- pass 2: G = 2 Et | -2 (Et V*^T) + Omega^T Yh, stripe by stripe -------------
    // Wave w owns column tiles w, w + kW, ...; its columns of the two stripe
    // buffers (A of the next stripe, then Et in place of A) are its own.
    {
      float* dAb = a.dA[b];
      const int64_t ldd = a.ldd[b];
      const float scale = (float)a.scale;
      CStripe<KP> cs;
      float an[kTPW][4], ov[LP / 4], on[LP / 4];
      cs.load(Ab, lda, Jl, 0, m, k);
#pragma unroll
      for (int j = 0; j < kTPW; ++j)
        if (w + kW * j < NT) {   // uniform per wave
#pragma unroll
          for (int r = 0; r < 4; ++r) an[j][r] = load_or_zero(Ab, lda, 4 * g + r, (w + kW * j) * 16 + cl, m, n);
        }
#pragma unroll
      for (int s = 0; s < LP / 4; ++s) ov[s] = omt[cl * ldom + 4 * s + g];
      cs.store(Cst, CS);   // the middle phase ended with a barrier; buffer 0 is free
#pragma unroll
      for (int j = 0; j < kTPW; ++j)
        if (w + kW * j < NT) {
#pragma unroll
          for (int r = 0; r < 4; ++r) Est[(4 * g + r) * ES + (w + kW * j) * 16 + cl] = an[j][r];
        }
      __syncthreads();
      int buf = 0;
      for (int i0 = 0; i0 < m; i0 += 16) {
        const bool more = i0 + 16 < m;
        float* Ec = Est + buf * 16 * ES;
        if (more) {   // next stripe, in flight during this one
          cs.load(Ab, lda, Jl, i0 + 16, m, k);
#pragma unroll
          for (int j = 0; j < kTPW; ++j)
            if (w + kW * j < NT) {   // uniform per wave
#pragma unroll
              for (int r = 0; r < 4; ++r)
                an[j][r] = load_or_zero(Ab, lda, i0 + 16 + 4 * g + r, (w + kW * j) * 16 + cl, m, n);
            }
#pragma unroll
          for (int s = 0; s < LP / 4; ++s) on[s] = omt[(i0 + 16 + cl) * ldom + 4 * s + g];
        }
        const float* Cc = Cst + buf * 16 * CS;
#pragma unroll 1
        for (int ct = w; ct < NT; ct += kW) {   // Et = A - C V*, in place
          const int c = ct * 16 + cl;
          f32x4 e;
#pragma unroll
          for (int r = 0; r < 4; ++r) e[r] = Ec[(4 * g + r) * ES + c];
#pragma unroll
          for (int s = 0; s < KP / 4; ++s) e = mfma4(-Cc[cl * CS + 4 * s + g], Vs[(4 * s + g) * VS + c], e);
#pragma unroll
          for (int r = 0; r < 4; ++r) Ec[(4 * g + r) * ES + c] = e[r];
        }
        // this wave's part of Et V*^T over its own column tiles
        f32x4 wp[nkt];
#pragma unroll
        for (int t = 0; t < nkt; ++t) wp[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
        for (int ct = w; ct < NT; ct += kW) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int cc = ct * 16 + 4 * s + g;
            const float ev = Ec[cl * ES + cc];
#pragma unroll
            for (int t = 0; t < nkt; ++t) wp[t] = mfma4(ev, Vs[(16 * t + cl) * VS + cc], wp[t]);
          }
        }
#pragma unroll
        for (int t = 0; t < nkt; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) Wp[(16 * w + 4 * g + r) * CS + 16 * t + cl] = wp[t][r];
        __syncthreads();
#pragma unroll 1
        for (int ct = w; ct < NT; ct += kW) {
          const int c = ct * 16 + cl;
          const int pos = c < n ? Jinv[c] : -1;
          f32x4 acc;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 4 * g + r;
            float v = 0.0f;
            if (pos >= k) {
              v = 2.0f * Ec[row * ES + c];
            } else if (pos >= 0) {
              float s4 = Wp[row * CS + pos];
#pragma unroll
              for (int q = 1; q < kW; ++q) s4 += Wp[(16 * q + row) * CS + pos];
              v = -2.0f * s4;
            }
            acc[r] = v;
          }
#pragma unroll
          for (int s = 0; s < LP / 4; ++s) acc = mfma4(ov[s], Yb[(4 * s + g) * YS + c], acc);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = i0 + 4 * g + r;
            if (i < m && c < n) dAb[(int64_t)i * ldd + c] = scale * acc[r];
          }
        }
        if (more) {   // the next stripe's operands, loaded a whole stripe ago
          cs.store(Cst + (buf ^ 1) * 16 * CS, CS);
          float* En = Est + (buf ^ 1) * 16 * ES;
#pragma unroll
          for (int j = 0; j < kTPW; ++j)
            if (w + kW * j < NT) {
#pragma unroll
              for (int r = 0; r < 4; ++r) En[(4 * g + r) * ES + (w + kW * j) * 16 + cl] = an[j][r];
            }
#pragma unroll
          for (int s = 0; s < LP / 4; ++s) ov[s] = on[s];
        }
        __syncthreads();
        buf ^= 1;
      }
    }
  }
}

// Instances with LP >= KP only (l = k + p > k).
template <int KP, int LP>
const void* kernel_if(bool vl) {
  if constexpr (LP >= KP)
    return vl ? (const void*)batched_bwd_kernel<KP, LP, true> : (const void*)batched_bwd_kernel<KP, LP, false>;
  else
    return nullptr;
}
template <int KP>
const void* kernel_kp(int lcp, bool vl) {
  switch (lcp) {
    case 16: return kernel_if<KP, 16>(vl);
    case 32: return kernel_if<KP, 32>(vl);
    case 48: return kernel_if<KP, 48>(vl);
    case 64: return kernel_if<KP, 64>(vl);
    default: return nullptr;
  }
}
const void* kernel_for(int kcp, int lcp, bool vl) {
  switch (kcp) {
    case 16: return kernel_kp<16>(lcp, vl);
    case 32: return kernel_kp<32>(lcp, vl);
    case 48: return kernel_kp<48>(lcp, vl);
    case 64: return kernel_kp<64>(lcp, vl);
    default: return nullptr;
  }
}

// V* and Yh in LDS when the whole map fits.
bool use_lds_operands(int kcp, int lcp, int ldn) { return lds_map(kcp, lcp, ldn, true).total + 64 <= kLdsCap; }

}  // namespace

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
  const bool vl = use_lds_operands(a.kcp, a.lcp, a.ldn);
  const void* fn = kernel_for(a.kcp, a.lcp, vl);
  if (!fn) return hipErrorInvalidValue;
  const int lds = lds_map(a.kcp, a.lcp, a.ldn, vl).total;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3(grid), dim3(kT), args, lds, stream);
}

}  // namespace idcur
