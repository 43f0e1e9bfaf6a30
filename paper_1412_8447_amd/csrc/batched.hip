// Batched adaptive-rank column ID: many independent blocks A_b (m_b x n_b, FP32,
// n_b <= 512) compressed in one persistent launch. Per block, one workgroup
// runs the tolerance variant of Section 3 on the randomized sketch of Section
// 5.1 (Algorithm 4):
//
//   1. Y = Omega(:l, :m_b) A_b on the FP32 matrix cores (v_mfma_f32_16x16x4f32,
//      FP32 sums over 16-k chunks added in FP64), written straight into LDS
//      (column-major, odd column stride);
//   2. column-pivoted Householder QR of Y with each thread's two columns in
//      registers (columns stay in place; a pivot list records the order), the
//      pivot column shared through LDS, every wave forming the reflector itself,
//      and the column norms recomputed exactly after every update; before each step the residual
//      |Y_res|_F is compared with tol |Y|_F; at most l - p steps are taken;
//      when the tolerance is not met, l doubles (up to l_cap = kmax + p) and
//      the block is sketched and factored again;
//   3. T = S11^{-1} S12 by back-substitution in FP64 registers (Section 4.1),
//      written with J = [pivots, the other columns in increasing order].
//
// One Omega (l_cap x m_max, stored transposed) serves every block. Workgroups
// take blocks from an atomic counter, in the order of a one-workgroup counting
// sort by m_b n_b (largest first) so the last blocks to start are the smallest.
// Results do not depend on which workgroup takes a block or on the launch
// shape: every reduction inside a block has a fixed order.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kBT = 256;        // threads per workgroup
constexpr int kBL0 = 32;        // first sketch width
constexpr int kBLmax = 64;      // largest sketch width
constexpr int kBNmax = 512;     // largest block width

typedef float f32x4 __attribute__((ext_vector_type(4)));

struct BArgs {
  int nblk;
  const int* m; const int* n;
  const float* const* A; const int64_t* lda;
  int* const* J; float* const* T; const int64_t* ldt;
  int* k_out;
  const float* omt; int ldom;      // Omega^T: mpad x ldom, zero outside l_cap x m_max
  int mmax, nmax, lcap, p, kfix;   // kfix > 0: fixed rank k, l = k + p
  double tol, rank_tol;
  const int* order;                // processing order, or NULL
  int* queue;                      // block counter, zero at launch
  int* status;
  int ldy;                         // LDS column stride of Y (odd)
};

// ---- block-wide reductions (256 threads, fixed order) ------------------------
struct Best {
  double v;
  int o;   // original column index (tie-break)
  int pos; // position in the factorisation
};
__device__ __forceinline__ bool beats(const Best& a, const Best& b) {
  return a.v > b.v || (a.v == b.v && a.o < b.o);
}

__device__ Best block_best_sum(Best b, double& s, Best* sb, double* ss) {
  for (int o = 32; o > 0; o >>= 1) {
    Best c{__shfl_xor(b.v, o, 64), __shfl_xor(b.o, o, 64), __shfl_xor(b.pos, o, 64)};
    if (beats(c, b)) b = c;
    s += __shfl_xor(s, o, 64);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) { sb[w] = b; ss[w] = s; }
  __syncthreads();
  Best r = sb[0];
  double t = ss[0];
#pragma unroll
  for (int i = 1; i < kBT / 64; ++i) {
    if (beats(sb[i], r)) r = sb[i];
    t += ss[i];
  }
  s = t;
  return r;
}

// ---- 1. sketch: rows r0 .. r0 + 16 RT - 1 of Y = Omega A (LDS, Y(i, c) at
// Ys[c*LDY + i]). The 16-column tiles are spread over the waves, four per wave
// and pass (tiles w + 4t + 16g for pass g). Products are summed on the matrix
// cores in FP32 over chunks of 16 consecutive k (four 16x16x4 steps) and the
// chunks are added in FP64: at the tolerances this path serves (1e-6 on smooth
// kernels, about 16 u32) FP32 sums over all m_b terms would put rounding noise
// of the tolerance's own size into Y. The next chunk's operands are loaded
// while the current chunk is multiplied (two register buffers); rows and
// columns past the block are read at a clamped in-range address and zeroed.
template <int RT>
struct Chunk {
  float av[4][RT];
  float bv[4][4];
};

// A load whose result is always used (so the compiler cannot sink it into a
// branch on the validity test, which serialises the loads behind full waits),
// from the global address space, zeroed by a bit mask when out of range.
typedef const __attribute__((address_space(1))) float gfloat;
__device__ __forceinline__ float ld_keep(const float* p, unsigned keep) {
  const float v = *(gfloat*)p;
  return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, v) & keep);
}

template <int RT>
__device__ __forceinline__ void load_chunk(Chunk<RT>& ch, const BArgs& a, const float* __restrict__ A, int64_t lda,
                                           int m, int c, int kq, int ocol, const int (&jt)[4], const bool (&jv)[4]) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int k = 16 * c + 4 * st + kq;
    const unsigned kk = k < m ? ~0u : 0u;
    const int kc = k < m ? k : m - 1;
    const float* orow = a.omt + (int64_t)kc * a.ldom + ocol;
    const float* arow = A + (int64_t)kc * lda;
#pragma unroll
    for (int r = 0; r < RT; ++r) ch.av[st][r] = ld_keep(orow + r * 16, kk);
#pragma unroll
    for (int t = 0; t < 4; ++t) ch.bv[st][t] = ld_keep(arow + jt[t], kk & (jv[t] ? ~0u : 0u));
  }
}

template <int RT>
__device__ __forceinline__ void mul_chunk(const Chunk<RT>& ch, double (&tot)[RT][4][4], int ntile) {
  f32x4 acc[RT][4];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[r][t] = f32x4{0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < 4; ++st)
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < ntile)
#pragma unroll
        for (int r = 0; r < RT; ++r)
          acc[r][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ch.av[st][r], ch.bv[st][t], acc[r][t], 0, 0, 0);
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) tot[r][t][q] += (double)acc[r][t][q];
}

template <int RT, int LDY>
__device__ __forceinline__ void sketch_rows(const BArgs& a, const float* __restrict__ A, int64_t lda, int m, int n,
                                            int r0, float* Ys) {
  // the wave index is uniform within a wave: say so, so that the tile guards
  // below are scalar branches and not masked lanes with full waits
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int kq = lane >> 4, col = lane & 15;
  const int ctn = (n + 15) >> 4;
  const int nch = (m + 15) >> 4;
  for (int g = 0; g < 2; ++g) {
    if (wv + 16 * g >= ctn) break;   // this wave has no tile in this pass
    // tiles of this wave in this pass: t < ntile (wave-uniform)
    const int ntile = min(4, (ctn - (wv + 16 * g) + 3) >> 2);
    int jt[4];
    bool jv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = (wv + 4 * t + 16 * g) * 16 + col;
      jv[t] = j < n;
      jt[t] = jv[t] ? j : n - 1;
    }
    double tot[RT][4][4];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) tot[r][t][q] = 0.0;
    Chunk<RT> c0, c1;
    load_chunk<RT>(c0, a, A, lda, m, 0, kq, r0 + col, jt, jv);
    for (int c = 0; c < nch; c += 2) {
      if (c + 1 < nch) load_chunk<RT>(c1, a, A, lda, m, c + 1, kq, r0 + col, jt, jv);
      mul_chunk<RT>(c0, tot, ntile);
      if (c + 1 >= nch) break;
      if (c + 2 < nch) load_chunk<RT>(c0, a, A, lda, m, c + 2, kq, r0 + col, jt, jv);
      mul_chunk<RT>(c1, tot, ntile);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < ntile && jv[t])
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) Ys[jt[t] * LDY + r0 + r * 16 + 4 * kq + q] = (float)tot[r][t][q];
    }
  }
}

// Rows 0 .. l-1 (rounded up to 16) in passes of at most 32 rows.
template <int PF, int LDY>
__device__ __forceinline__ void sketch_any(const BArgs& a, const float* A, int64_t lda, int m, int n, int l, float* Ys) {
  for (int r0 = 0; r0 < l; r0 += 32) {
    if (l - r0 > 16) sketch_rows<2, LDY>(a, A, lda, m, n, r0, Ys);
    else sketch_rows<1, LDY>(a, A, lda, m, n, r0, Ys);
  }
}

// ---- 3. T = S11^{-1} S12 (Section 4.1) -----------------------------------------
// S11 is copied into an identity-padded KP x KP square Sp (column-major,
// Sp[i*KP + q] = S(q, i)) with FP64 reciprocals of its diagonal, KP = 16, 32 or
// 64 >= k, so every column's back-substitution runs over KP rows with no
// per-row conditions: padded rows only ever meet zeros above the diagonal.
// The right-hand side sits in 32 FP64 registers (static indices); with KP = 64
// the lower 32 rows are solved and stored first, then folded into the upper 32.
// Solutions overwrite the column in LDS, and T is written from there.
template <int KP, int LDY>
__device__ __forceinline__ void solve_rows(const float* Sp, const double* dinv, int base, double (&r)[32]) {
  constexpr int R = KP < 32 ? KP : 32;
#pragma unroll
  for (int i = R - 1; i >= 0; --i) {
    const double ti = r[i] * dinv[base + i];
    r[i] = ti;
#pragma unroll
    for (int q = 0; q < i; ++q) r[q] -= (double)Sp[(base + i) * KP + base + q] * ti;
  }
}

template <int KP, int LDY>
__device__ __forceinline__ void solve_columns(float* Ys, const float* Sp, const double* dinv, const int* ord, int n) {
  constexpr int R = KP < 32 ? KP : 32;
  for (int c = threadIdx.x; c < n; c += kBT) {
    if (ord[c] >= 0) continue;   // a selected column
    float* y = Ys + c * LDY;
    double r[32];
    if (KP == 64) {
#pragma unroll
      for (int i = 0; i < 32; ++i) r[i] = (double)y[32 + i];
      solve_rows<KP, LDY>(Sp, dinv, 32, r);
#pragma unroll
      for (int i = 0; i < 32; ++i) y[32 + i] = (float)r[i];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) r[i] = (double)y[i];
    if (KP == 64) {
      for (int i = 32; i < 64; ++i) {
        const double ti = (double)y[i];
#pragma unroll
        for (int q = 0; q < 32; ++q) r[q] -= (double)Sp[i * KP + q] * ti;
      }
    }
    solve_rows<KP, LDY>(Sp, dinv, 0, r);
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = (float)r[i];
  }
}

template <int PF, int LDY>
__global__ __launch_bounds__(kBT, (LDY < 64 ? 2 : 1)) void batched_id_kernel(BArgs a) {
  constexpr int LR = LDY - 1;   // rows kept per column (>= the sketch width)
  // every region at a compile-time offset, the small ones first: unrolled accesses
  // then fold their constant offsets (< 64 KiB) into the LDS instructions
  extern __shared__ __align__(16) unsigned char bsm[];
  constexpr int kSpBytes = LR * LR * (int)sizeof(float);
  float* Sp = reinterpret_cast<float*>(bsm);
  int* ord = reinterpret_cast<int*>(bsm + kSpBytes);    // pivot step of a column, -1 if unselected
  int* cpos = ord + kBNmax;                               // column of the tc-th unselected column
  float* Ys = reinterpret_cast<float*>(bsm + kSpBytes + 2 * kBNmax * sizeof(int));
  __shared__ float xcol[kBLmax];
  __shared__ int piv[kBLmax];
  __shared__ double dinv[kBLmax];
  __shared__ Best sb[kBT / 64];
  __shared__ double ss[kBT / 64];
  __shared__ int sblk;
  const int tid = threadIdx.x, lane = tid & 63;
  // rows of Y beyond a block's sketch width are read (and multiplied by zeros)
  // by the padded back-substitution: keep them finite
  for (int e = tid; e < kBNmax * LDY; e += kBT) Ys[e] = 0.0f;

  for (;;) {
    if (tid == 0) sblk = atomicAdd(a.queue, 1);
    __syncthreads();
    const int slot = sblk;
    __syncthreads();
    if (slot >= a.nblk) break;
    const int b = a.order ? a.order[slot] : slot;
    const int m = a.m[b], n = a.n[b];
    if (m < 1 || m > a.mmax || n < 1 || n > a.nmax) {
      if (tid == 0) {
        a.k_out[b] = -1;
        set_status(a.status, ST_BADINDEX);
      }
      continue;
    }
    const float* A = a.A[b];
    const int64_t lda = a.lda[b];
    const bool tolmode = a.kfix <= 0;
    const int lcap = a.lcap;
    int l = tolmode ? min(kBL0, lcap) : lcap;
    int k = 0;
    bool met = false;
    // this thread's columns c = tid and tid + 256, kept in registers through the
    // pivoted QR; columns never move (the pivot list records the order)
    float y[2][LR];
    for (;;) {
      // ---- sketch ----------------------------------------------------------------
      sketch_any<PF, LDY>(a, A, lda, m, n, l, Ys);
      __syncthreads();
      double nu[2];   // squared trailing norm of a candidate column, -1 once selected or absent
      Best b0{-1.0, 0x7fffffff, 0};
      double y0 = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int c = tid + q * kBT;
        const bool own = c < n;
        double sq = 0.0;
#pragma unroll
        for (int i = 0; i < LR; ++i) {
          y[q][i] = (own && i < l) ? Ys[(own ? c : 0) * LDY + i] : 0.0f;
          sq += (double)y[q][i] * (double)y[q][i];
        }
        nu[q] = own ? sq : -1.0;
        if (own) {
          y0 += sq;
          Best cb{sq, c, c};
          if (beats(cb, b0)) b0 = cb;
        }
      }
      b0 = block_best_sum(b0, y0, sb, ss);
      const double nu0max = b0.v;
      const int cap = min(tolmode ? l - a.p : a.kfix, n);
      // ---- pivoted QR ------------------------------------------------------------
      int j = 0;
      met = !tolmode;
      for (;;) {
        Best bb{-1.0, 0x7fffffff, 0};
        double rs = 0.0;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (nu[q] >= 0.0) {
            rs += nu[q];
            const int c = tid + q * kBT;
            Best cb{nu[q], c, c};
            if (beats(cb, bb)) bb = cb;
          }
        }
        bb = block_best_sum(bb, rs, sb, ss);
        if (tolmode && rs <= a.tol * a.tol * y0) { met = true; break; }
        if (j >= cap) break;
        if (bb.v <= a.rank_tol * a.rank_tol * nu0max) { met = true; break; }
        const int P = bb.pos;
        // the pivot's owner publishes the column and takes it out of the candidates
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (P == tid + q * kBT) {
#pragma unroll
            for (int i = 0; i < LR; ++i) xcol[i] = y[q][i];
            nu[q] = -1.0;
          }
        }
        if (tid == 0) piv[j] = P;
        __syncthreads();
        // every wave forms the reflector of rows j..l-1 itself (lane = row)
        const double xd = (lane < LR && lane >= j) ? (double)xcol[lane < LR ? lane : 0] : 0.0;
        double s2 = xd * xd;
        for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
        const double x0 = __shfl(xd, j, 64);
        const double normx = sqrt(s2);
        const double alpha = x0 >= 0.0 ? -normx : normx;
        const float vf = (float)(lane == j ? x0 - alpha : xd);
        double vv = (double)vf * (double)vf;
        for (int o = 32; o > 0; o >>= 1) vv += __shfl_xor(vv, o, 64);
        const double beta = vv > 0.0 ? 2.0 / vv : 0.0;
        float v[LR];
#pragma unroll
        for (int i = 0; i < LR; ++i)
          v[i] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, vf), i));
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (nu[q] >= 0.0) {
            double w = 0.0;
#pragma unroll
            for (int i = 0; i < LR; ++i) w += (double)v[i] * (double)y[q][i];
            w *= beta;
            double sq = 0.0;
#pragma unroll
            for (int i = 0; i < LR; ++i) {
              y[q][i] = (float)((double)y[q][i] - w * (double)v[i]);
              sq += i > j ? (double)y[q][i] * (double)y[q][i] : 0.0;
            }
            nu[q] = sq;
          } else if (P == tid + q * kBT) {
            // the pivot column becomes column j of S: alpha on the diagonal, zeros below
#pragma unroll
            for (int i = 0; i < LR; ++i) y[q][i] = i < j ? y[q][i] : (i == j ? (float)alpha : 0.0f);
          }
        }
        ++j;
      }
      k = j;
      if (met || !tolmode || l >= lcap) break;
      l = min(2 * l, lcap);
      __syncthreads();
    }
    if (!met && tid == 0) set_status(a.status, ST_RANKCAP);
    // columns back to LDS (rows 0..k-1 hold S, the rest the residual)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int c = tid + q * kBT;
      if (c < n) {
#pragma unroll
        for (int i = 0; i < LR; ++i) Ys[c * LDY + i] = y[q][i];
        ord[c] = -1;
      }
    }
    __syncthreads();
    if (tid < k) ord[piv[tid]] = tid;
    // ---- T = S11^{-1} S12, written with J = [pivots, the rest ascending] ----------
    const int KP = k <= 16 ? 16 : (k <= 32 ? 32 : 64);
    for (int e = tid; e < KP * KP; e += kBT) {
      const int i = e / KP, q = e % KP;
      Sp[e] = i < k ? (q <= i ? Ys[piv[i] * LDY + q] : 0.0f) : (q == i ? 1.0f : 0.0f);
    }
    for (int i = tid; i < KP; i += kBT) dinv[i] = i < k ? 1.0 / (double)Ys[piv[i] * LDY + i] : 1.0;
    __syncthreads();
    int* J = a.J[b];
    for (int c = tid; c < n; c += kBT) {
      if (ord[c] >= 0) {
        J[ord[c]] = c;
      } else {
        int below = 0;
        for (int q = 0; q < k; ++q) below += piv[q] < c ? 1 : 0;
        const int tc = c - below;   // rank among the unselected columns
        J[k + tc] = c;
        cpos[tc] = c;
      }
    }
    if (k > 0) {
      if (KP == 16) solve_columns<16, LDY>(Ys, Sp, dinv, ord, n);
      else if (KP == 32) solve_columns<32, LDY>(Ys, Sp, dinv, ord, n);
      else solve_columns<64, LDY>(Ys, Sp, dinv, ord, n);
    }
    __syncthreads();
    {
      float* T = a.T[b];
      const int64_t ldt = a.ldt[b];
      const int nt = n - k;
      for (int e = tid; e < k * nt; e += kBT) {
        const int i = e / nt, tc = e % nt;
        T[(int64_t)i * ldt + tc] = Ys[cpos[tc] * LDY + i];
      }
    }
    if (tid == 0) a.k_out[b] = k;
    __syncthreads();
  }
}

// Processing order: block indices by size class m_b n_b / 1024 (0 .. 256 for
// blocks up to 512 x 512), largest class first, by a counting sort in one
// workgroup. The order inside a class (set by LDS atomics) only changes which
// workgroup takes a block when, never a block's result.
constexpr int kClasses = 257;
__global__ __launch_bounds__(1024) void batch_order_kernel(const int* m, const int* n, int nblk, int* order) {
  __shared__ int cnt[kClasses];
  __shared__ int start[kClasses];
  for (int c = threadIdx.x; c < kClasses; c += 1024) cnt[c] = 0;
  __syncthreads();
  auto cls = [&](int i) {
    const long long w = (long long)max(m[i], 0) * (long long)max(n[i], 0);
    return (int)min(w >> 10, (long long)(kClasses - 1));
  };
  for (int i = threadIdx.x; i < nblk; i += 1024) atomicAdd(&cnt[cls(i)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {   // exclusive scan from the largest class down
    int run = 0;
    for (int c = kClasses - 1; c >= 0; --c) {
      start[c] = run;
      run += cnt[c];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nblk; i += 1024) order[atomicAdd(&start[cls(i)], 1)] = i;
}

template <int PF>
const void* kernel_pf(int ldy) {
  switch (ldy) {
    case 17: return (const void*)batched_id_kernel<PF, 17>;
    case 33: return (const void*)batched_id_kernel<PF, 33>;
    default: return (const void*)batched_id_kernel<PF, 65>;
  }
}
const void* kernel_for(int pf, int ldy) { return pf == 0 ? kernel_pf<1>(ldy) : kernel_pf<2>(ldy); }

}  // namespace

// Rows of the LDS copy of Y (and columns of the stored Omega^T): 16, 32 or 64, so
// that the padded back-substitution (order 16, 32 or 64 >= k) stays inside a column.
int batched_ldom(int lcap) { return lcap <= 16 ? 16 : (lcap <= 32 ? 32 : 64); }
int batched_mpad(int mmax) { return (int)round_up(std::max(mmax, 1), 4); }
int batched_max_width() { return kBNmax; }
int batched_max_sketch() { return kBLmax; }

size_t batched_lds_bytes(int lcap, int nmax) {
  (void)nmax;
  const int ldom = batched_ldom(lcap);
  const int ldy = ldom + 1;
  return (size_t)ldom * ldom * sizeof(float) + 2 * (size_t)kBNmax * sizeof(int) + (size_t)kBNmax * ldy * sizeof(float);
}

// Variant v: sketch prefetch depth PF = 1 + v % 2 (16-k chunks of loads issued together);
// workgroups per CU = 1 + (v / 2) % 2 (when LDS allows two); largest-first
// processing order when v / 4 == 0. Results do not depend on the variant.
int batched_num_variants() { return 8; }

hipError_t batched_launch(const BatchedArgs& ba, int variant, int num_cus, hipStream_t stream) {
  if (ba.nblk <= 0) return hipSuccess;
  if (ba.nblk > (1 << 20) || ba.nmax > kBNmax || ba.lcap > kBLmax || ba.lcap < 1) return hipErrorInvalidValue;
  BArgs a{};
  a.nblk = ba.nblk;
  a.m = ba.m; a.n = ba.n; a.A = ba.A; a.lda = ba.lda; a.J = ba.J; a.T = ba.T; a.ldt = ba.ldt; a.k_out = ba.k_out;
  a.omt = ba.omt; a.ldom = batched_ldom(ba.lcap);
  a.mmax = ba.mmax; a.nmax = ba.nmax; a.lcap = ba.lcap; a.p = ba.p; a.kfix = ba.kfix;
  a.tol = ba.tol; a.rank_tol = ba.rank_tol;
  a.queue = ba.queue; a.status = ba.status;
  a.ldy = a.ldom + 1;
  const int pf = variant % 2, occ_pick = (variant / 2) % 2, lpt = (variant / 4) == 0;
  hipError_t e = zero_launch(ba.queue, sizeof(int), stream);
  if (e != hipSuccess) return e;
  a.order = nullptr;
  if (lpt && ba.order) {
    hipLaunchKernelGGL(batch_order_kernel, dim3(1), dim3(1024), 0, stream, ba.m, ba.n, ba.nblk, ba.order);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    a.order = ba.order;
  }
  const size_t lds = batched_lds_bytes(ba.lcap, ba.nmax);
  const int per_cu = (occ_pick == 1 && 2 * lds <= 160 * 1024) ? 2 : 1;
  const int grid = std::max(1, std::min(ba.nblk, per_cu * num_cus));
  const void* fn = kernel_for(pf, a.ldy);
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3(grid), dim3(kBT), args, lds, stream);
}

}  // namespace idcur
