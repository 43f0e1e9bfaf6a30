// Blocked truncated column-pivoted Householder QR for slabs that do not fit in
// registers (Section 2.2, eq. (trunc); the k CPQR steps of Algorithms 1 and 4,
// and of the row ID on C^T that completes a CUR).
//
// One persistent cooperative launch of G <= #CUs workgroups (512 threads).
// Workgroup g owns the columns [c0, c1) of a global column-major copy of Y (the
// slab, rows padded to a multiple of 32) and updates only those. Reflectors are
// applied in panels of nb (<= 32) steps, in the compact form that LAPACK's
// blocked pivoted QR uses: with Y0 the trailing matrix at the panel start, V the
// panel's reflectors and F (n x nb) the accumulated products,
//     Y = Y0 - V F^T,   f_i = tau_i (Y0^T v_i - F (V^T v_i)),
// so a step reads Y0 once (one matrix-vector product over the local columns)
// and writes nothing but the new row of S; the trailing matrix is brought up to
// date once per panel by a rank-nb update on the matrix cores
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64). Norms are downdated
// (nu^2 -= s^2); when a downdate has cancelled, the owning workgroup brings that
// column alone up to date (Y0(:, c) -= V F(c, :)^T, F(c, :) = 0 -- the panel's
// formulas stay valid) and recomputes its norm in FP64 before it publishes its
// next candidate, so pivots always come from valid norms.
//
// Two forms, fixed per launch:
//  * short (V fits in LDS, e.g. the 500 x 50000 C^T of a rank-500 CUR): every
//    workgroup reads the winning column of Y0 and forms the reflector, V^T v
//    and its copy of V itself -- one exchange per step;
//  * tall (Y = A of the deterministic comparator, thousands of rows): the rows
//    are split over the workgroups as well; workgroup g forms rows [r0, r1) of
//    the updated pivot column and its parts of |v|^2 and V^T v, which a second
//    exchange sums; V lives in a global buffer that the flush reads.
//
// Exchange records carry the publish index in their tag word; a writer waits for
// its data stores before storing the tag, and thread t of every workgroup polls
// workgroup t's tag (the grid barrier). Every workgroup reduces the records in
// the same order, so all take the same pivot, stopping decision and reflector.
// Records, v and V are written and read with device-coherent (sc1) accesses. A
// workgroup reads and writes its own slab columns with ordinary accesses and,
// after loading them and after each panel update, writes its XCD's L2 back
// before it next publishes; other workgroups read a winning column with
// device-coherent loads.
//
// Pivots: largest norm, ties to the smallest column index. Householder sign:
// alpha = -sgn(x0)|x|. S is written by original column index; J lists the
// pivots, then the remaining columns in increasing order.
#include <cstdlib>

#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace cb {

constexpr int kBT = 512;
constexpr int kBW = kBT / 64;
constexpr int kNBMax = 32;
constexpr int kW1 = 40;   // words per step record: key, sumsq, (unused), tag, F[0:nb]
constexpr int kW2 = 40;   // words per row record (tall): ssq, tag, w'[0:nb]

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint64_t dbits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double bitsd(uint64_t b) { return __longlong_as_double((long long)b); }

// buffer resource over [base, base + bytes): loads past the end return zero and
// stores past it are dropped
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr int kSC1 = 16;   // device-coherent cache policy
constexpr int kOWN = 0;    // default policy: a workgroup's own slab columns
// an offset past every resource used here (all are below 2^31 bytes), also
// after adding the 16 bytes of a second load
constexpr uint32_t kOOB = 0x80000000u;

// four consecutive elements (16 or 32 bytes), device-coherent
template <typename T>
struct Quad;
template <>
struct Quad<float> {
  using acc = f32x4;
  __device__ static void load(__amdgpu_buffer_rsrc_t rs, uint32_t off, double (&x)[4]) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kOWN);
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = (double)__uint_as_float(v[e]);
  }
  __device__ static void load_raw(__amdgpu_buffer_rsrc_t rs, uint32_t off, float (&x)[4]) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kOWN);
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = __uint_as_float(v[e]);
  }
  __device__ static acc load_acc(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kOWN);
    return acc{__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3])};
  }
  __device__ static void store_acc(__amdgpu_buffer_rsrc_t rs, uint32_t off, acc a) {
    const u32x4 v{__float_as_uint(a[0]), __float_as_uint(a[1]), __float_as_uint(a[2]), __float_as_uint(a[3])};
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, kOWN);
  }
  __device__ static void store(__amdgpu_buffer_rsrc_t rs, uint32_t off, const float (&x)[4]) {
    const u32x4 v{__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]), __float_as_uint(x[3])};
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, kOWN);
  }
  __device__ static f32x4 mfma(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // the 16 x 16 accumulator tile: lane L holds rows 4 (L / 16) + r, r = 0..3,
  // of column L % 16 (one 16-byte access); e0 = element index of the tile's
  // row 0 in this lane's column, or kOOB for a column outside the slab
  __device__ static acc tile_load(__amdgpu_buffer_rsrc_t rs, uint32_t e0, int kq) {
    return load_acc(rs, e0 == kOOB ? kOOB : (e0 + 4u * kq) * 4u);
  }
  __device__ static void tile_store(__amdgpu_buffer_rsrc_t rs, uint32_t e0, int kq, acc a) {
    store_acc(rs, e0 == kOOB ? kOOB : (e0 + 4u * kq) * 4u, a);
  }
};
template <>
struct Quad<double> {
  using acc = f64x4;
  __device__ static void load(__amdgpu_buffer_rsrc_t rs, uint32_t off, double (&x)[4]) {
    const u32x4 v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kOWN);
    const u32x4 v1 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16u), 0, kOWN);
    x[0] = __hiloint2double((int)v0[1], (int)v0[0]);
    x[1] = __hiloint2double((int)v0[3], (int)v0[2]);
    x[2] = __hiloint2double((int)v1[1], (int)v1[0]);
    x[3] = __hiloint2double((int)v1[3], (int)v1[2]);
  }
  __device__ static void load_raw(__amdgpu_buffer_rsrc_t rs, uint32_t off, double (&x)[4]) { load(rs, off, x); }
  __device__ static acc load_acc(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    double x[4];
    load(rs, off, x);
    return acc{x[0], x[1], x[2], x[3]};
  }
  __device__ static void store2(__amdgpu_buffer_rsrc_t rs, uint32_t off, double a, double b) {
    const u32x4 v{(unsigned)__double2loint(a), (unsigned)__double2hiint(a), (unsigned)__double2loint(b),
                  (unsigned)__double2hiint(b)};
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)off, 0, kOWN);
  }
  __device__ static void store_acc(__amdgpu_buffer_rsrc_t rs, uint32_t off, acc a) {
    store2(rs, off, a[0], a[1]);
    store2(rs, off + 16u, a[2], a[3]);
  }
  __device__ static void store(__amdgpu_buffer_rsrc_t rs, uint32_t off, const double (&x)[4]) {
    store2(rs, off, x[0], x[1]);
    store2(rs, off + 16u, x[2], x[3]);
  }
  __device__ static f64x4 mfma(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // the FP64 accumulator tile: lane L holds rows L / 16 + 4 r, r = 0..3, of
  // column L % 16 (four 8-byte accesses)
  __device__ static double ld8(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, kOWN);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(off + 4u), 0, kOWN);
    return __hiloint2double((int)hi, (int)lo);
  }
  __device__ static void st8(__amdgpu_buffer_rsrc_t rs, uint32_t off, double x) {
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)__double2loint(x), rs, (int)off, 0, kOWN);
    __builtin_amdgcn_raw_buffer_store_b32((unsigned)__double2hiint(x), rs, (int)(off + 4u), 0, kOWN);
  }
  __device__ static acc tile_load(__amdgpu_buffer_rsrc_t rs, uint32_t e0, int kq) {
    acc a;
#pragma unroll
    for (int r = 0; r < 4; ++r) a[r] = ld8(rs, e0 == kOOB ? kOOB : (e0 + kq + 4u * r) * 8u);
    return a;
  }
  __device__ static void tile_store(__amdgpu_buffer_rsrc_t rs, uint32_t e0, int kq, acc a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) st8(rs, e0 == kOOB ? kOOB : (e0 + kq + 4u * r) * 8u, a[r]);
  }
};

// four consecutive elements written by other workgroups (device-coherent)
template <typename T>
__device__ __forceinline__ void load4_sc1(__amdgpu_buffer_rsrc_t rs, uint32_t off, double (&x)[4]) {
  if constexpr (sizeof(T) == 4) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kSC1);
#pragma unroll
    for (int e = 0; e < 4; ++e) x[e] = (double)__uint_as_float(v[e]);
  } else {
    const u32x4 v0 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, kSC1);
    const u32x4 v1 = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16u), 0, kSC1);
    x[0] = __hiloint2double((int)v0[1], (int)v0[0]);
    x[1] = __hiloint2double((int)v0[3], (int)v0[2]);
    x[2] = __hiloint2double((int)v1[1], (int)v1[0]);
    x[3] = __hiloint2double((int)v1[3], (int)v1[2]);
  }
}
template <typename T>
__device__ __forceinline__ T load1_sc1(__amdgpu_buffer_rsrc_t rs, uint32_t idx) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(idx * 4u), 0, kSC1));
  } else {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(idx * 8u), 0, kSC1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, (int)(idx * 8u + 4u), 0, kSC1);
    return __hiloint2double((int)hi, (int)lo);
  }
}

// Make this workgroup's slab stores visible to the other XCDs: every thread
// waits for its stores, then one thread writes the XCD's L2 back (agent-scope
// release). Readers in other workgroups use device-coherent loads, and no
// 128-byte line holds data of two workgroups (columns start on 128-byte
// boundaries), so they never see a stale copy.
__device__ __forceinline__ void publish_slab() {
  wait_all_mem();
  __syncthreads();
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}

// ---------------------------------------------------------------------------
// Block reductions over kBT threads (fixed order: identical inputs give
// identical bits in every workgroup).
// ---------------------------------------------------------------------------
__device__ double bsum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kBW; ++i) s += red[i];
  return s;
}
// argmax and sum in one pass
__device__ ArgMax bargmax_sum(ArgMax a, double& s, int& flag, double* rv, int* ri, double* rs, int* rf) {
  a = wave_argmax(a);
  s = wave_sum(s);
  const int f = __any(flag) ? 1 : 0;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) { rv[w] = a.v; ri[w] = a.i; rs[w] = s; rf[w] = f; }
  __syncthreads();
  ArgMax b{rv[0], ri[0]};
  double t = rs[0];
  int ff = rf[0];
#pragma unroll
  for (int i = 1; i < kBW; ++i) {
    if (better(rv[i], ri[i], b.v, b.i)) { b.v = rv[i]; b.i = ri[i]; }
    t += rs[i];
    ff |= rf[i];
  }
  s = t;
  flag = ff;
  return b;
}

template <typename T, bool TALL>
__global__ __launch_bounds__(kBT) void cpqr_blk_kernel(CpqrArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;

  const int l = a.l_dev ? min(*a.l_dev, a.l_host) : a.l_host;
  const int n = a.n;
  int kmax = a.kmax_dev ? min(*a.kmax_dev, a.kmax_host) : a.kmax_host;
  kmax = min(kmax, min(l, n));
  const int c0 = (int)(((int64_t)g * n) / G), c1 = (int)(((int64_t)(g + 1) * n) / G);
  const int ncl = c1 - c0;
  const int lpad = a.lpad;          // multiple of 32, >= l_host
  const int cpw = a.cols_per_wg;    // >= ncl, multiple of 16
  const int nb = a.nb;              // panel width (<= kNBMax)
  const int nbp = ((nb + 3) & ~3) + 1;   // F row stride (odd; entries past nb stay zero)
  const int R = a.lanes_per_col;    // lanes per column in the sweeps (16 or 64)
  const int r0 = TALL ? (int)(((int64_t)g * l) / G) : 0;
  const int r1 = TALL ? (int)(((int64_t)(g + 1) * l) / G) : 0;
  const int rpw = a.rpw;            // >= r1 - r0 (tall)
  const int vch = a.vch;            // rows of v staged in LDS per pass (tall)
  T* slab = static_cast<T*>(a.gslab);
  const __amdgpu_buffer_rsrc_t rs_wg =
      rsrc(slab + (size_t)c0 * lpad, (uint32_t)((size_t)ncl * lpad * sizeof(T)));
  uint64_t* rec1 = static_cast<uint64_t*>(a.rec);                 // [2][G][kW1]
  uint64_t* rec2 = rec1 + (size_t)2 * G * kW1;                     // [2][G][kW2] (tall)
  T* vglob = static_cast<T*>(a.cvals);                             // lpad (tall)
  T* Vglob = vglob + lpad;                                         // nb x lpad (tall)

  // ---- LDS -----------------------------------------------------------------------
  unsigned char* sp = smem;
  T* Vl = reinterpret_cast<T*>(sp);   // short: nb x lpad; tall: nb x rpw (own rows)
  sp += (size_t)nb * (TALL ? rpw : lpad) * sizeof(T);
  sp = smem + (((sp - smem) + 15) & ~(ptrdiff_t)15);   // offset arithmetic keeps LDS addressing
  // v of the current step in FP64 (its T values, exact): short lpad rows, tall
  // vch rows at a time
  double* vd = reinterpret_cast<double*>(sp);
  double* vloc = vd;
  sp += (size_t)(TALL ? vch : lpad) * 8;
  T* F = reinterpret_cast<T*>(sp);     sp += (size_t)cpw * nbp * sizeof(T);
  sp = smem + (((sp - smem) + 15) & ~(ptrdiff_t)15);   // offset arithmetic keeps LDS addressing
  double* nu2 = reinterpret_cast<double*>(sp);    sp += (size_t)cpw * 8;
  double* lim = reinterpret_cast<double*>(sp);    sp += (size_t)cpw * 8;
  double* dots = reinterpret_cast<double*>(sp);   sp += (size_t)cpw * 8;
  double* salpha = reinterpret_cast<double*>(sp); sp += (size_t)cpw * 8;
  double* y0j = reinterpret_cast<double*>(sp);    sp += (size_t)cpw * 8;   // Y0(j, c) from the sweep
  double* wv_ = reinterpret_cast<double*>(sp);    sp += kNBMax * 8;   // V^T v
  double* Vj = reinterpret_cast<double*>(sp);     sp += kNBMax * 8;   // row j of V
  double* Fp = reinterpret_cast<double*>(sp);     sp += kNBMax * 8;   // the winner's F row
  double* rd = reinterpret_cast<double*>(sp);     sp += 4 * kBW * 8;
  int* sel = reinterpret_cast<int*>(sp);          sp += (size_t)cpw * 4;   // -1 active, else its step
  int* need = reinterpret_cast<int*>(sp);         sp += (size_t)cpw * 4;
  int* flist = reinterpret_cast<int*>(sp);        sp += (size_t)cpw * 4;   // columns to refresh
  double* rfl = reinterpret_cast<double*>(sp);    sp += 8 * kBW * 8;       // their partial sums
  int* ri = reinterpret_cast<int*>(sp);           sp += 2 * kBW * 4;
  int* win = reinterpret_cast<int*>(sp);          // kmax_host
  __shared__ int sh[4];
  __shared__ double shd[4];

  const double eps = (sizeof(T) == 4) ? 5.9604644775390625e-08 : 1.1102230246251565e-16;
  const double tol3z = sqrt(eps);
  const bool tolmode = a.tol > 0.0;
  const int gpw = 64 / R, rgi = lane % R, gidx = lane / R;
  const int groups = kBW * gpw;

  // ---- load the slab (rows past l zero) -------------------------------------------------
  const T* Y = static_cast<const T*>(a.Y);
  if (a.cs == 1 && a.rs != 1) {
    // row-major source: tiles of 16 rows through LDS (the F region), so that both
    // the reads (along a row) and the slab writes (16 rows of a column) are wide
    T* tile = F;   // cpw x nbp, rt rows at a time
    const int rt = ((nbp - 1) / 4) * 4;
    for (int rb = 0; rb < lpad; rb += rt) {
      for (int e = tid; e < rt * cpw; e += kBT) {
        const int rr = e / cpw, cc = e % cpw;
        const int row = rb + rr;
        tile[cc * nbp + rr] = (row < l && cc < ncl) ? Y[(int64_t)row * a.rs + (int64_t)(c0 + cc)] : (T)0;
      }
      __syncthreads();
      for (int e = tid; e < (rt / 4) * cpw; e += kBT) {
        const int cc = e / (rt / 4), qd = e % (rt / 4);
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = tile[cc * nbp + 4 * qd + u];
        const bool in = cc < ncl && rb + 4 * qd < lpad;
        const uint32_t off = in ? (uint32_t)(((size_t)cc * lpad + rb + 4 * qd) * sizeof(T)) : kOOB;
        Quad<T>::store(rs_wg, off, x);
      }
      __syncthreads();
    }
  } else {
    const int nq = lpad / 4;
    for (int64_t e = tid; e < (int64_t)ncl * nq; e += kBT) {
      const int cc = (int)(e / nq), qd = (int)(e % nq);
      T x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int row = 4 * qd + u;
        x[u] = row < l ? Y[(int64_t)row * a.rs + (int64_t)(c0 + cc) * a.cs] : (T)0;
      }
      Quad<T>::store(rs_wg, (uint32_t)(((size_t)cc * lpad + 4 * qd) * sizeof(T)), x);
    }
  }
  for (int c = tid; c < cpw; c += kBT) {
    sel[c] = c < ncl ? -1 : -2;
    need[c] = 0;
    dots[c] = 0.0;
  }
  for (int e = tid; e < cpw * nbp; e += kBT) F[e] = (T)0;
  publish_slab();
  __syncthreads();

  // squared norms of rows [rb, l) of the local columns (all active ones, or the
  // flagged ones), group-parallel, FP64
  auto norms = [&](int rb, bool all) {
    const int q0 = rb >> 2, nq = lpad >> 2;
    for (int cb = 0; cb < ncl; cb += groups) {
      const int cl = cb + wv * gpw + gidx;
      const bool doit = cl < ncl && sel[cl] == -1 && (all || need[cl]);
      if (!__any(doit)) continue;
      double ss = 0.0;
      for (int qd = q0 + rgi; qd < nq; qd += R) {
        double x[4];
        Quad<T>::load(rs_wg, doit ? (uint32_t)(((size_t)cl * lpad + 4 * qd) * sizeof(T)) : kOOB, x);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int row = 4 * qd + u;
          ss += (row >= rb) ? x[u] * x[u] : 0.0;
        }
      }
      ss = group_sum(ss, R);
      if (doit && rgi == 0) {
        nu2[cl] = ss;
        lim[cl] = tol3z * ss;
        need[cl] = 0;
      }
    }
  };
  norms(0, true);
  __syncthreads();

  // Bring the trailing rows [j, l) of the local columns up to date with the
  // panel's ib reflectors: Y -= V F^T on the matrix cores, 16 x 16 tiles. Rows
  // above j (rows of S) and past l see a zero V operand and keep their bits.
  auto flush = [&](int ib, int j) {
    if (ib > 0) {
      const int nks = (ib + 3) >> 2;
      const int kq = lane >> 4, li = lane & 15;
      const __amdgpu_buffer_rsrc_t rs_V = rsrc(Vglob, (uint32_t)((size_t)nb * lpad * sizeof(T)));
      const int ntc = cpw >> 4;
      // the V operand of row tile rt (16 rows x ib), zero outside rows [j, l)
      auto vload = [&](int rt, T (&av)[kNBMax / 4]) {
        const int r = rt * 16 + li;
#pragma unroll
        for (int ks = 0; ks < kNBMax / 4; ++ks) {
          const int s = 4 * ks + kq;
          T x = (T)0;
          if (ks < nks && s < ib && r >= j && r < l && rt < (lpad >> 4)) {
            if constexpr (TALL) x = -load1_sc1<T>(rs_V, (uint32_t)(s * lpad + r));
            else x = -Vl[(size_t)s * lpad + r];
          }
          av[ks] = x;
        }
      };
      T av[kNBMax / 4], avn[kNBMax / 4];
      int rt = (j >> 4) + wv;
      vload(rt, av);
      const int nrt = lpad >> 4;
      if (ntc <= 4) {
        // at most 64 columns: a row tile is one group of four column tiles, and
        // the next row tile's slab tiles (and V operand) load while this one's
        // products run; tiles past the last row tile read zero, stores drop
        auto tiles = [&](int r, typename Quad<T>::acc (&acc)[4], uint32_t (&e0)[4]) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int cl = u * 16 + li;
            e0[u] = (r < nrt && u < ntc && cl < ncl) ? (uint32_t)((size_t)cl * lpad + r * 16) : kOOB;
            acc[u] = Quad<T>::tile_load(rs_wg, e0[u], kq);
          }
        };
        typename Quad<T>::acc acc[4], accn[4];
        uint32_t e0[4], e0n[4];
        tiles(rt, acc, e0);
        for (; rt < nrt; rt += kBW) {
          vload(rt + kBW, avn);
          tiles(rt + kBW, accn, e0n);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (u < ntc) {
              const int cl = u * 16 + li;
#pragma unroll
              for (int ks = 0; ks < kNBMax / 4; ++ks)
                if (ks < nks) acc[u] = Quad<T>::mfma(av[ks], F[cl * nbp + 4 * ks + kq], acc[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            Quad<T>::tile_store(rs_wg, e0[u], kq, acc[u]);
            acc[u] = accn[u];
            e0[u] = e0n[u];
          }
#pragma unroll
          for (int ks = 0; ks < kNBMax / 4; ++ks) av[ks] = avn[ks];
        }
      } else
      for (; rt < nrt; rt += kBW) {
        vload(rt + kBW, avn);   // the next row tile's operand, in flight during this one
        // four column tiles at a time: their loads in flight together
        for (int ct0 = 0; ct0 < ntc; ct0 += 4) {
          typename Quad<T>::acc acc[4];
          uint32_t e0[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int cl = (ct0 + u) * 16 + li;
            e0[u] = (ct0 + u < ntc && cl < ncl) ? (uint32_t)((size_t)cl * lpad + rt * 16) : kOOB;
            acc[u] = Quad<T>::tile_load(rs_wg, e0[u], kq);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (ct0 + u < ntc) {
              const int cl = (ct0 + u) * 16 + li;
#pragma unroll
              for (int ks = 0; ks < kNBMax / 4; ++ks)
                if (ks < nks) acc[u] = Quad<T>::mfma(av[ks], F[cl * nbp + 4 * ks + kq], acc[u]);
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) Quad<T>::tile_store(rs_wg, e0[u], kq, acc[u]);
        }
#pragma unroll
        for (int ks = 0; ks < kNBMax / 4; ++ks) av[ks] = avn[ks];
      }
      publish_slab();
      __syncthreads();
    }
    norms(j, a.norms_exact != 0);
    for (int e = tid; e < cpw * nbp; e += kBT) F[e] = (T)0;
    wait_all_mem();
    __syncthreads();
  };

  // Columns whose downdated norm cancelled: bring their trailing rows [j, l) up
  // to date with the panel's ib reflectors (Y0(:, c) -= V F(c, :)^T, then F(c, :)
  // = 0, which keeps every later formula of the panel valid for them), recompute
  // their norms in FP64 and write the slab back for the other workgroups. Local
  // to the workgroup: no other workgroup waits for it.
  auto refresh = [&](int ib, int j) {
    constexpr int NF = 4;
    if (tid == 0) sh[3] = 0;
    __syncthreads();
    for (int c = tid; c < ncl; c += kBT)
      if (need[c] && sel[c] == -1) flist[atomicAdd(&sh[3], 1)] = c;
    __syncthreads();
    const int nflag = sh[3];
    if (nflag == 0) return;
    const __amdgpu_buffer_rsrc_t rs_V = rsrc(Vglob, (uint32_t)((size_t)nb * lpad * sizeof(T)));
    for (int f0 = 0; f0 < nflag; f0 += NF) {
      const int nf = min(NF, nflag - f0);
      double ss[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) ss[f] = 0.0;
      // four consecutive rows per thread: V(r..r+3, s) is one 16-byte load
      for (int qd = (j >> 2) + tid; 4 * qd < l; qd += kBT) {
        double y[NF][4];
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) {
            const int r = 4 * qd + e2;
            y[f][e2] = (f < nf && r >= j && r < l) ? (double)slab[(size_t)(c0 + flist[f0 + f]) * lpad + r] : 0.0;
          }
        for (int sb = 0; sb < ib; sb += 4) {
          double vr[4][4];
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            if (sb + s2 < ib) {
              if constexpr (TALL) {
                load4_sc1<T>(rs_V, (uint32_t)(((sb + s2) * lpad + 4 * qd) * sizeof(T)), vr[s2]);
              } else {
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) vr[s2][e2] = (double)Vl[(size_t)(sb + s2) * lpad + 4 * qd + e2];
              }
            } else {
#pragma unroll
              for (int e2 = 0; e2 < 4; ++e2) vr[s2][e2] = 0.0;
            }
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            if (f < nf) {
              const T* fc = F + flist[f0 + f] * nbp + sb;
#pragma unroll
              for (int s2 = 0; s2 < 4; ++s2) {
                const double fv = (sb + s2 < ib) ? (double)fc[s2] : 0.0;
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) y[f][e2] -= vr[s2][e2] * fv;
              }
            }
          }
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          if (f < nf) {
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
              const int r = 4 * qd + e2;
              if (r >= j && r < l) {
                const T yt = (T)y[f][e2];
                slab[(size_t)(c0 + flist[f0 + f]) * lpad + r] = yt;
                ss[f] += (double)yt * (double)yt;
              }
            }
          }
        }
      }
      // per-column sums in a fixed order: waves, then the waves' partials
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const double w = wave_sum(ss[f]);
        if (lane == 0) rfl[wv * NF + f] = w;
      }
      __syncthreads();
      if (tid < nf) {
        double t = 0.0;
        for (int w2 = 0; w2 < kBW; ++w2) t += rfl[w2 * NF + tid];
        const int c = flist[f0 + tid];
        nu2[c] = t;
        lim[c] = tol3z * t;
        need[c] = 0;
      }
      __syncthreads();
    }
    for (int q = tid; q < nflag * nbp; q += kBT) F[flist[q / nbp] * nbp + q % nbp] = (T)0;
    publish_slab();
    __syncthreads();
  };

  // Publish this workgroup's candidate for publish index e: the best active
  // column's squared norm and index, the sum of the active squared norms and
  // the candidate's F row (panel entries [0, i)).
  auto publish = [&](int e, int i) {
    ArgMax best{-1.0, 0x7fffffff};
    double ssq = 0.0;
    int flag = 0;
    for (int c = tid; c < ncl; c += kBT) {
      if (sel[c] == -1) {
        ssq += nu2[c];
        if (better(nu2[c], c0 + c, best.v, best.i)) { best.v = nu2[c]; best.i = c0 + c; }
      }
    }
    best = bargmax_sum(best, ssq, flag, rd, ri, rd + kBW, ri + kBW);
    uint64_t* r = rec1 + ((size_t)(e & 1) * G + g) * kW1;
    if (tid < i && best.i != 0x7fffffff) cstore(r + 4 + tid, dbits((double)F[(best.i - c0) * nbp + tid]));
    if (tid == 0) {
      cstore(r + 0, dbits(best.v));
      cstore(r + 1, dbits(ssq));
    }
    wait_all_mem();
    __syncthreads();
    if (tid == 0) cstore(r + 3, ((uint64_t)(e + 1) << 32) | (uint32_t)best.i);
  };

  double y0fro2 = 0.0, nu0sq = 0.0;
  int j = 0, i = 0, e = 0;
  int stop = 0;
  publish(0, 0);

  while (true) {
    // ---- exchange 1: every workgroup's candidate ------------------------------------
    ArgMax cand{-2.0, 0x7fffffff};
    double tot = 0.0;
    if (tid == 0) sh[0] = 0;
    int flag = 0, tmo = 0;
    if (tid < G) {
      const uint64_t* r = rec1 + ((size_t)(e & 1) * G + tid) * kW1;
      const uint64_t want = (uint64_t)(e + 1);
      long spins = 0;
      uint64_t tag = cload(r + 3);
      while ((tag >> 32) != want) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) { tmo = 1; break; }
        tag = cload(r + 3);
      }
      if (!tmo) {
        cand.v = bitsd(cload(r + 0));
        cand.i = (int)(uint32_t)(tag & 0xffffffffu);
        tot = bitsd(cload(r + 1));
      }
    }
    if (tid == 0) sh[1] = 0;
    int any_tmo = tmo;
    {
      int fl = flag;
      const ArgMax w0 = bargmax_sum(cand, tot, fl, rd, ri, rd + kBW, ri + kBW);
      flag = fl;
      // the owner of the winning column is the workgroup whose record held it
      if (tid < G && cand.i == w0.i && w0.i != 0x7fffffff) sh[0] = tid;
      cand = w0;
    }
    // time-outs: any thread of the workgroup
    {
      const int t = __any(any_tmo) ? 1 : 0;
      if (lane == 0 && t) atomicOr(&sh[1], 1);
      __syncthreads();
      any_tmo = sh[1];
    }
    const ArgMax w = cand;
    if (any_tmo) stop = ST_TIMEOUT;
    else {
      if (e == 0) { y0fro2 = tot; nu0sq = w.v; }
      if (!(tot == tot) || !(w.v == w.v) || isinf(tot) || isinf(w.v)) stop = ST_NONFINITE;
      else if (tolmode && tot <= a.tol * a.tol * y0fro2) stop = -1;
      else if (j >= kmax) stop = tolmode ? ST_RANKCAP : -1;
      else if (w.i == 0x7fffffff || w.v <= a.rank_tol * a.rank_tol * nu0sq) stop = -1;
    }
    if (stop != 0) {
      if (stop > 0 && tid == 0 && (stop == ST_TIMEOUT || g == 0)) set_status(a.status, stop);
      break;
    }
    const int p = w.i;
    const int owner = sh[0];
    // the winner's F row
    if (tid < i) Fp[tid] = bitsd(cload(rec1 + ((size_t)(e & 1) * G + owner) * kW1 + 4 + tid));
    __syncthreads();
    const __amdgpu_buffer_rsrc_t rs_p = rsrc(slab + (size_t)p * lpad, (uint32_t)((size_t)l * sizeof(T)));

    double xnorm, yj;
    if constexpr (!TALL) {
      // ---- short: every workgroup forms the reflector and V^T v itself -------------
      T* vi = Vl + (size_t)i * lpad;
      double ss = 0.0;
      for (int r = tid; r < lpad; r += kBT) {
        T yt = (T)0;
        if (r >= j && r < l) {
          double y = (double)load1_sc1<T>(rs_p, (uint32_t)r);
          for (int s = 0; s < i; ++s) y -= (double)Vl[(size_t)s * lpad + r] * Fp[s];
          yt = (T)y;
          ss += (double)yt * (double)yt;
        }
        vi[r] = yt;
      }
      ss = bsum(ss, rd);   // ends with barriers: vi is complete
      xnorm = sqrt(ss);
      yj = (double)vi[j];
    } else {
      // ---- tall: rows [r0, r1) of the pivot column here, sums by exchange 2 ----------
      double ss = 0.0;
      const int r = r0 + tid;
      T yt = (T)0;
      if (tid < r1 - r0) {
        if (r >= j) {
          double y = (double)load1_sc1<T>(rs_p, (uint32_t)r);
          for (int s = 0; s < i; ++s) y -= (double)Vl[(size_t)s * rpw + tid] * Fp[s];
          yt = (T)y;
          ss = (double)yt * (double)yt;
          cstore(vglob + r, yt);
          cstore(Vglob + (size_t)i * lpad + r, yt);
        }
        Vl[(size_t)i * rpw + tid] = yt;
      }
      ss = bsum(ss, rd);   // barriers: Vl column i complete
      // this workgroup's part of V^T y over its rows at or below j
      uint64_t* rr = rec2 + ((size_t)(j & 1) * G + g) * kW2;
      for (int s = wv; s < i; s += kBW) {
        double acc = 0.0;
        for (int t = lane; t < r1 - r0; t += 64)
          if (r0 + t >= j) acc += (double)Vl[(size_t)s * rpw + t] * (double)Vl[(size_t)i * rpw + t];
        acc = wave_sum(acc);
        if (lane == 0) cstore(rr + 2 + s, dbits(acc));
      }
      if (tid == 0) cstore(rr + 0, dbits(ss));
      wait_all_mem();
      __syncthreads();
      if (tid == 0) cstore(rr + 1, (uint64_t)(j + 1) << 32);
      // exchange 2
      double part = 0.0;
      int t2 = 0;
      if (tid < G) {
        const uint64_t* q = rec2 + ((size_t)(j & 1) * G + tid) * kW2;
        long spins = 0;
        uint64_t tag = cload(q + 1);
        while ((tag >> 32) != (uint64_t)(j + 1)) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) { t2 = 1; break; }
          tag = cload(q + 1);
        }
        if (!t2) part = bitsd(cload(q + 0));
      }
      if (tid == 0) sh[1] = 0;
      __syncthreads();
      if (__any(t2) && lane == 0) atomicOr(&sh[1], 1);
      const double ssq = bsum(part, rd);
      if (sh[1]) {
        if (tid == 0) set_status(a.status, ST_TIMEOUT);
        stop = ST_TIMEOUT;
        break;
      }
      // w'[s] summed over the workgroups in a fixed order
      for (int s = wv; s < i; s += kBW) {
        double acc = 0.0;
        for (int t = lane; t < G; t += 64) acc += bitsd(cload(rec2 + ((size_t)(j & 1) * G + t) * kW2 + 2 + s));
        acc = wave_sum(acc);
        if (lane == 0) wv_[s] = acc;
      }
      if (tid < i) Vj[tid] = (double)cload(Vglob + (size_t)tid * lpad + j);
      if (tid == kBT - 1) shd[0] = (double)cload(vglob + j);
      __syncthreads();
      xnorm = sqrt(ssq);
      yj = shd[0];
    }
    if (!(xnorm > 0.0)) { stop = -1; break; }
    const double alpha = (yj >= 0.0) ? -xnorm : xnorm;
    const double tau = 1.0 / (xnorm * (xnorm + fabs(yj)));
    const T vjT = (T)(yj - alpha);
    const double vj = (double)vjT;
    if constexpr (!TALL) {
      __syncthreads();
      if (tid == 0) Vl[(size_t)i * lpad + j] = vjT;
      __syncthreads();
      // w = V(:, 0:i)^T v over rows [j, l), row j of V
      for (int s = wv; s < i; s += kBW) {
        double acc = 0.0;
        for (int r = j + lane; r < l; r += 64)
          acc += (double)Vl[(size_t)s * lpad + r] * (double)Vl[(size_t)i * lpad + r];
        acc = wave_sum(acc);
        if (lane == 0) wv_[s] = acc;
      }
      if (tid < i) Vj[tid] = (double)Vl[(size_t)tid * lpad + j];
      // v in FP64 for the sweep (rows above j are zero)
      for (int r = tid; r < lpad; r += kBT) vd[r] = (double)Vl[(size_t)i * lpad + r];
    } else {
      // v differs from y only in row j
      if (tid < i) wv_[tid] += Vj[tid] * (vj - yj);
      if (j >= r0 && j < r1 && tid == 0) Vl[(size_t)i * rpw + (j - r0)] = vjT;
    }
    if (tid == 0) {
      Vj[i] = vj;
      win[j] = p;
    }
    // the winner leaves the active set: S(j, p) = alpha, zeros below
    if (p >= c0 && p < c1 && tid == 0) {
      const int cl = p - c0;
      sel[cl] = j;
      salpha[cl] = alpha;
      need[cl] = 0;
    }
    __syncthreads();
    if (p >= c0 && p < c1)
      for (int s = tid; s < nbp; s += kBT) F[(p - c0) * nbp + s] = (T)0;

    // ---- Y0^T v over the local active columns (rows [j, l)) --------------------------
    const int j4 = j & ~3;
    const int nq = lpad >> 2;
    // dots[c] += sum over row quads [qa, qb) of Y0(rows, c) v(rows) for the local
    // active columns. A lane walks a fixed sequence of (pass, quad) units -- pass
    // = a set of one column per group of R lanes, quads rgi, rgi + R, ... of it --
    // and keeps U loads in flight; a pass's group sum is taken when its last unit
    // is consumed (the same unit index on every lane). The lane holding row j
    // keeps Y0(j, c) for the new row of S.
    auto sweep = [&](const double* vsrc, int vbase, int qa, int qb) {
      constexpr int U = sizeof(T) == 4 ? 8 : 4;
      const int qpl = (qb - qa + R - 1) / R;
      if (qpl <= 0) return;
      const int npass = (ncl + groups - 1) / groups;
      const int total = npass * qpl;
      const int qj = j >> 2, jr = j & 3;
      const int gcol = wv * gpw + gidx;
      // (pass, quad) of the next unit to load and to consume, advanced by one per
      // unit (the same sequence on every lane of a wave), and whether the load
      // side's current column is active
      int lps = 0, lt = 0, cps = 0, ct = 0;
      bool lact = false;
      double dot = 0.0;
      for (int u0 = 0; u0 < total; u0 += U) {
        T x[U][4];
#pragma unroll
        for (int v = 0; v < U; ++v) {
          const int cl = lps * groups + gcol;
          if (lt == 0) lact = cl < ncl && sel[min(cl, cpw - 1)] == -1;
          const int qd = qa + rgi + R * lt;
          const bool ok = u0 + v < total && lact && qd < qb;
          Quad<T>::load_raw(rs_wg, ok ? (uint32_t)(((size_t)cl * lpad + 4 * qd) * sizeof(T)) : kOOB, x[v]);
          if (++lt == qpl) { lt = 0; ++lps; }
        }
#pragma unroll
        for (int v = 0; v < U; ++v) {
          if (u0 + v >= total) continue;   // the same on every lane (the tail of the last batch)
          const int cl = cps * groups + gcol;
          const int qd = qa + rgi + R * ct;
          const double* vq = vsrc + 4 * min(qd, qb - 1) - vbase;   // x is zero past qb
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) dot = fma((double)x[v][e2], vq[e2], dot);
          if (qd == qj && cl < ncl) {
            const T xj = jr == 0 ? x[v][0] : (jr == 1 ? x[v][1] : (jr == 2 ? x[v][2] : x[v][3]));
            y0j[cl] = (double)xj;
          }
          if (ct == qpl - 1) {
            const double d = group_sum(dot, R);
            if (rgi == 0 && cl < ncl && sel[cl] == -1) dots[cl] += d;
            dot = 0.0;
          }
          if (++ct == qpl) { ct = 0; ++cps; }
        }
      }
    };
    if constexpr (!TALL) {
      // rows below j of column i are zero, so the sweep may start at the quad of j
      sweep(vd, 0, j4 >> 2, nq);
    } else {
      const __amdgpu_buffer_rsrc_t rs_v = rsrc(vglob, (uint32_t)((size_t)lpad * sizeof(T)));
      // v was stored by every workgroup with device-coherent stores: read it the same way
      for (int cs = j4; cs < lpad; cs += vch) {
        const int ce = min(lpad, cs + vch);
        for (int qd = (cs >> 2) + tid; qd < (ce >> 2); qd += kBT) {
          double x[4];
          load4_sc1<T>(rs_v, (uint32_t)(4 * qd * sizeof(T)), x);
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) {
            const int r = 4 * qd + e2;
            vloc[r - cs] = (r < j || r >= l) ? 0.0 : (r == j ? vj : x[e2]);
          }
        }
        __syncthreads();
        sweep(vloc, cs, cs >> 2, ce >> 2);
        __syncthreads();
      }
    }
    __syncthreads();

    // ---- per column: F(c, i), the new row j of S, the norm downdate ------------------
    for (int cl = tid; cl < ncl; cl += kBT) {
      if (sel[cl] != -1) continue;
      const T* fr = F + cl * nbp;
      double corr = 0.0, sr = 0.0;
      for (int s = 0; s < i; ++s) {
        const double fs = (double)fr[s];
        corr = fma(fs, wv_[s], corr);
        sr = fma(fs, Vj[s], sr);
      }
      const T fT = (T)(tau * (dots[cl] - corr));
      F[cl * nbp + i] = fT;
      dots[cl] = 0.0;
      const T sT = (T)(y0j[cl] - sr - vj * (double)fT);
      slab[(size_t)(c0 + cl) * lpad + j] = sT;   // a row of S: read back by this workgroup only
      const double s = (double)sT;
      const double nc = nu2[cl];
      if (nc > 0.0) {
        const double nn = fmax(0.0, nc - s * s);
        if (nn <= lim[cl]) need[cl] = 1;
        nu2[cl] = nn;
      }
    }
    __syncthreads();
    ++j;
    ++i;
    if (!tolmode && j >= kmax) break;   // fixed rank: nothing left to decide
    refresh(i, j);
    if (i == nb) {
      flush(i, j);
      i = 0;
    }
    ++e;
    publish(e, i);
  }

  // ---- epilogue ------------------------------------------------------------------------
  const int kout = j;
  __syncthreads();
  if (a.S) {
    T* S = static_cast<T*>(a.S);
    for (int64_t q = tid; q < (int64_t)kout * ncl; q += kBT) {
      const int r = (int)(q / ncl), cl = (int)(q % ncl);
      const int st = sel[cl];
      T v;
      if (st == -1 || r < st) v = slab[(size_t)(c0 + cl) * lpad + r];
      else v = (r == st) ? (T)salpha[cl] : (T)0;
      S[(int64_t)r * a.ldS + c0 + cl] = v;
    }
  }
  // J: pivots first (workgroup 0), then the unselected columns in increasing
  // order; a workgroup learns how many columns before its range were selected
  // from the others' counts
  if (tid == 0) {
    int nsel = 0;
    for (int cl = 0; cl < ncl; ++cl) nsel += sel[cl] >= 0 ? 1 : 0;
    cstore(a.fin + g * 16, nsel + 1);
    sh[2] = 0;
  }
  __syncthreads();
  int before = 0, ftmo = 0;
  if (tid < g) {
    long spins = 0;
    int vfin = cload(a.fin + tid * 16);
    while (vfin == 0) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) { ftmo = 1; break; }
      vfin = cload(a.fin + tid * 16);
    }
    before = vfin > 0 ? vfin - 1 : 0;
  }
  if (__any(ftmo) && lane == 0) atomicOr(&sh[2], 1);
  const double bs = bsum((double)before, rd);
  if (sh[2]) {
    // a count never arrived: the positions would be wrong, so leave J alone and
    // report the time-out
    if (tid == 0) set_status(a.status, ST_TIMEOUT);
  } else if (tid == 0) {
    int pos = kout + (c0 - (int)bs);
    for (int cl = 0; cl < ncl; ++cl)
      if (sel[cl] == -1) {
        if (pos >= kout && pos < n) a.J[pos] = c0 + cl;
        ++pos;
      }
  }
  if (g == 0) {
    for (int t = tid; t < kout; t += kBT) a.J[t] = win[t];
    if (tid == 0) *a.k_out = kout;
  }
}

}  // namespace cb

using namespace cb;

// LDS bytes of one workgroup
static size_t blk_lds_bytes(bool tall, int esz, int lpad, int nb, int cpw, int rpw, int vch, int kmax) {
  size_t b = (size_t)nb * (tall ? rpw : lpad) * esz;
  b = (b + 15) & ~(size_t)15;
  b += (size_t)(tall ? vch : lpad) * 8;
  b += (size_t)cpw * (((nb + 3) & ~3) + 1) * esz;
  b = (b + 15) & ~(size_t)15;
  b += (size_t)cpw * 8 * 5 + 3 * kNBMax * 8 + 4 * kBW * 8;
  b += (size_t)cpw * 4 * 3 + 8 * kBW * 8 + 2 * kBW * 4 + (size_t)kmax * 4;
  return b;
}

// Plan of the blocked kernel: 1 short, 2 tall, 0 when the shape does not fit.
// force: 0 free choice, 1 short only, 2 tall only.
int cpqr_blk_plan(CpqrPlan& p, int esz, int l, int n, int kmax, int num_cus, int force) {
  const size_t budget = 152 * 1024;
  const int G = std::max(1, std::min(num_cus, n));
  const int cpw = (int)round_up(ceil_div(n, G), 16);
  // columns start on 128-byte lines (see publish_slab)
  const int lpad = (int)round_up(std::max(l, 1), 32);
  if ((size_t)cpw * lpad * esz >= ((size_t)1 << 31)) return 0;
  if ((size_t)lpad * esz >= ((size_t)1 << 31)) return 0;
  p.G = G;
  p.cols_per_wg = cpw;
  p.lpad = lpad;
  p.lanes_per_col = lpad > 2048 ? 64 : 16;
  p.reg_cfg = -1;
  p.in_lds = false;
  p.fin_bytes = (size_t)G * 16 * sizeof(int);
  p.gslab_bytes = (size_t)n * lpad * esz + 256;
  if (force != 2) {
    for (int nb : {32, 16, 8}) {
      const size_t lds = blk_lds_bytes(false, esz, lpad, nb, cpw, 0, 0, kmax);
      if (lds <= budget) {
        p.blk = 1;
        p.nb = nb;
        p.rpw = 0;
        p.vch = 0;
        p.lds_bytes = lds;
        p.rec_bytes = (size_t)2 * G * kW1 * 8;
        p.cvals_bytes = 0;
        return 1;
      }
    }
    if (force == 1) return 0;
  }
  const int rpw = (int)round_up(ceil_div(l, G), 4);
  if (rpw > kBT) return 0;
  const int nb = 32;
  const size_t base = blk_lds_bytes(true, esz, lpad, nb, cpw, rpw, 0, kmax);
  if (base + 4096 * (size_t)8 > budget) return 0;
  int vch = (int)std::min<size_t>((size_t)lpad, ((budget - base) / 8) / 16 * 16);
  vch = std::max(16, vch / 16 * 16);
  p.blk = 2;
  p.nb = nb;
  p.rpw = rpw;
  p.vch = vch;
  p.lds_bytes = blk_lds_bytes(true, esz, lpad, nb, cpw, rpw, vch, kmax);
  p.rec_bytes = (size_t)2 * G * (kW1 + kW2) * 8;
  p.cvals_bytes = (size_t)lpad * (1 + nb) * esz;
  return 2;
}

hipError_t cpqr_blk_launch(int dtype, const CpqrPlan& p, CpqrArgs a, hipStream_t stream) {
  a.lpad = p.lpad;
  a.cols_per_wg = p.cols_per_wg;
  a.lanes_per_col = p.lanes_per_col;
  a.nb = p.nb;
  a.rpw = p.rpw;
  a.vch = p.vch;
  if (a.norms_exact) a.nb = 1;   // exact norms every step: flush and recompute after each reflector
  const bool tall = p.blk == 2;
  const void* fn;
  if (dtype == 0) fn = tall ? (const void*)cpqr_blk_kernel<double, true> : (const void*)cpqr_blk_kernel<double, false>;
  else fn = tall ? (const void*)cpqr_blk_kernel<float, true> : (const void*)cpqr_blk_kernel<float, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds_bytes);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(p.G), dim3(kBT), args, (unsigned)p.lds_bytes, stream);
}

}  // namespace idcur
