// Subsampled randomized Hadamard sketch: the real counterpart of the structured
// sketch of Section 5.2, eq. (def_srft) (unitary DFT -> orthonormal
// Walsh-Hadamard of order m', random unit-modulus diagonal -> random signs).
// For the mr x nc view X it writes Y^T (nc x l) with
//   Y(r, c) = l^(-1/2) sum_{i < mr} (-1)^popcount(s_r & i) d_i X(i, c),
// s_r the sampled rows (distinct, < m' = the smallest power of two >= mr),
// d_i = +-1. With i = 256 i1 + i2 and s = 256 s1 + s2 the sign factors into
// (-1)^popcount(s1 & i1) (-1)^popcount(s2 & i2): each 256-row block of X is
// transformed by the length-256 Walsh-Hadamard transform (eight butterfly
// stages: four on a thread's 16 rows in registers, four more after one
// exchange through LDS), and every sampled row takes entry s2 of the
// transformed block with sign (-1)^popcount(s1 & i1). X is read once, with 8
// additions and l / 256 signed additions per element. Row blocks are split
// over the grid; the split partial sums are added in split order by a second
// kernel.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

constexpr int kSB = 256;                      // rows per block
constexpr int kSBL = 8;                       // log2(kSB)
constexpr int kSC = 16;                       // columns per workgroup
constexpr int kST = 256;                      // threads
constexpr int kSG = kST / kSC;                // row groups (16)
static_assert(kST == kSB, "a thread per block row");

template <typename T>
struct SArgs {
  const T* X; int64_t xr, xc;
  int64_t mr, nc;
  const int8_t* signs;
  const int* rows; int l;
  T* out; int64_t ldo;     // split s writes rows s*nc .. (s+1)*nc - 1 (ld ldo)
  int64_t nblk, bps;       // row blocks, blocks per split
  int64_t mp;              // padded order
  double scale;            // l^(-1/2)
  int* status;
};

template <typename T>
__device__ __forceinline__ T load_or_zero(const T* X, int64_t off, bool ok) {
  const T v = X[ok ? off : 0];
  return ok ? v : T(0);
}

// Loads through a buffer descriptor: offsets at or past the descriptor's byte
// count read as zero, which takes the place of per-element bounds selects and
// 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T rsrc_load(const T* base, int64_t nrec_bytes, uint32_t byte_off) {
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)nrec_bytes, 0x00020000);
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)byte_off, 0, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)byte_off, 0, 0));
  }
}

// LAY 0: X(i, c) = X[i*xr + c] (rows along memory) with pointer loads; LAY 3:
// the same through one descriptor per block (the block's rows below mr; a
// block's bytes, 257 xr sizeof(T), below 2^31); LAY 1: X(i, c) = X[i + c*xc]
// with pointer loads; LAY 2: the same through one descriptor per column (a
// column's bytes, mr * sizeof(T) plus one block, below 2^31).
// kSJ: sampled rows per thread (l <= kSG kSJ).
template <typename T, int LAY, int kSJ>
__global__ __launch_bounds__(kST) void srht_kernel(SArgs<T> a) {
  constexpr bool XC1 = LAY == 0 || LAY == 3;
  // one sampled row's term for the current block: the byte offset of its
  // entry s2 in buf (column 0) and its sign (-1)^popcount(s1 & i1)
  struct Tap {
    int off;
    float sgn;
  };
  __shared__ T buf[kSB][kSC + 1];
  __shared__ Tap tap_s[kSG * kSJ];    // the sampled rows' terms, rebuilt per block
  __shared__ float sgn_s[2][kSB];     // the signs of a block's rows (two blocks in flight)
  const int tid = threadIdx.x, c = tid % kSC, g = tid / kSC;
  // XCD-aware order: the 8 XCDs take workgroups round-robin, so XCD x gets the
  // contiguous column-block range x*per .. (x+1)*per - 1 and neighbouring blocks
  // (which share the 128-byte lines a row straddles) meet in the same L2
  const int64_t per = gridDim.x / 8;   // gridDim.x is a multiple of 8
  const int64_t cb = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (cb >= ceil_div(a.nc, kSC)) return;   // whole workgroup, before any barrier
  const int64_t c0 = cb * kSC;
  const int64_t b0 = (int64_t)blockIdx.y * a.bps;
  const int64_t b1 = min(a.nblk, b0 + a.bps);

  // the sampled rows this thread keeps the terms of (r = tid + kST h; thread
  // g, c accumulates rows r = g + kSG j); rows past l get sign 0
  constexpr int kSH = (kSG * kSJ + kST - 1) / kST;
  unsigned s_hi[kSH];
  int s_off[kSH];
  bool s_on[kSH];
  bool bad = false;
#pragma unroll
  for (int h = 0; h < kSH; ++h) {
    const int r = tid + kST * h;
    int s = r < a.l ? a.rows[r] : 0;
    if (s < 0 || s >= a.mp) {
      bad = true;
      s = 0;
    }
    s_hi[h] = (unsigned)s >> kSBL;
    s_off[h] = (s & (kSB - 1)) * (kSC + 1) * (int)sizeof(T);
    s_on[h] = r < a.l;
  }
  if (bad) set_status(a.status, ST_BADINDEX);
  const char* col_base = reinterpret_cast<const char*>(&buf[0][c]);
  T acc[kSJ];
#pragma unroll
  for (int j = 0; j < kSJ; ++j) acc[j] = T(0);

  // coalesced loads of one 256 x 16 block: XC1 -> thread (g, c) takes rows
  // 16 g .. 16 g + 15 of column c; else thread t takes row t of the 16 columns
  T ld[16];
  int8_t sg = 0;
  // LAY 3: load q of a block reads row 16 g + q through a descriptor based at
  // block row q, at the lane's byte offset (16 g xr + c) sizeof(T), which is
  // below the descriptor's count exactly when the row is below mr; columns past
  // nc take an offset past every count, so they read zero
  const uint32_t lane_off = c0 + c < a.nc ? (uint32_t)((16 * g * a.xr + c) * (int64_t)sizeof(T)) : 0x80000000u;
  auto load_block = [&](int64_t i1) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      if constexpr (LAY == 3) {
        const int64_t r0 = i1 * kSB + q;   // the descriptor's first row
        const int64_t nrec = r0 < a.mr ? min(a.mr - r0, (int64_t)kSB) * a.xr * (int64_t)sizeof(T) : 0;
        ld[q] = rsrc_load(a.X + r0 * a.xr + c0, nrec, lane_off);
      } else if constexpr (LAY == 0) {
        const int64_t i = i1 * kSB + 16 * g + q, cc = c0 + c;
        ld[q] = load_or_zero(a.X, i * a.xr + cc, i < a.mr && cc < a.nc);
      } else if constexpr (LAY == 1) {
        const int64_t i = i1 * kSB + tid, cc = c0 + q;
        ld[q] = load_or_zero(a.X, i + cc * a.xc, i < a.mr && cc < a.nc);
      } else {
        const int64_t cc = c0 + q;
        ld[q] = rsrc_load(a.X + cc * a.xc, cc < a.nc ? a.mr * (int64_t)sizeof(T) : 0,
                         (uint32_t)((i1 * kSB + tid) * (int64_t)sizeof(T)));
      }
    }
    {
      const int64_t i = i1 * kSB + tid;   // kST == kSB
      sg = a.signs[i < a.mr ? i : 0];
    }
  };
  // XC1: the loaded rows are the ones the thread transforms first, so they stay
  // in registers, and the row signs go to LDS for them; else thread t holds
  // row t of every column, applies its sign and stores the block to LDS
  auto store_block = [&](int sb) {
    const float sgf = sg < 0 ? -1.0f : 1.0f;
    if constexpr (XC1) {
      sgn_s[sb][tid] = sgf;
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) buf[tid][q] = (T)sgf * ld[q];   // exact, branch-free
    }
  };

  if (b0 < b1) load_block(b0);
  int sb = 0;
  for (int64_t i1 = b0; i1 < b1; ++i1, sb ^= 1) {
    store_block(sb);
    const unsigned i1u = (unsigned)i1;
#pragma unroll
    for (int h = 0; h < kSH; ++h) {
      const int r = tid + kST * h;
      if (r < kSG * kSJ) {
        const float sg1 = (__builtin_popcount(s_hi[h] & i1u) & 1) ? -1.0f : 1.0f;
        tap_s[r] = Tap{s_off[h], s_on[h] ? sg1 : 0.0f};
      }
    }
    __syncthreads();
    // stages 1, 2, 4, 8: a thread's 16 consecutive rows of column c, signed
    T v[16];
    if constexpr (XC1) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = (T)sgn_s[sb][16 * g + q] * ld[q];   // exact
    }
    if (i1 + 1 < b1) load_block(i1 + 1);   // in flight during this block
    if constexpr (!XC1) {
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = buf[16 * g + q][c];
    }
#pragma unroll
    for (int h = 1; h < 16; h *= 2)
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if ((q & h) == 0) {
          const T x0 = v[q], x1 = v[q + h];
          v[q] = x0 + x1;
          v[q + h] = x0 - x1;
        }
#pragma unroll
    for (int q = 0; q < 16; ++q) buf[16 * g + q][c] = v[q];
    __syncthreads();
    // stages 16, 32, 64, 128: rows g + 16 u (u < 16) of column c
    {
      T u[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) u[q] = buf[g + 16 * q][c];
#pragma unroll
      for (int h = 1; h < 16; h *= 2)
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if ((q & h) == 0) {
            const T x0 = u[q], x1 = u[q + h];
            u[q] = x0 + x1;
            u[q + h] = x0 - x1;
          }
#pragma unroll
      for (int q = 0; q < 16; ++q) buf[g + 16 * q][c] = u[q];
    }
    __syncthreads();
    // each sampled row takes its signed entry of the transformed block (rows
    // past l add zero times row 0: no branches, so the LDS reads issue together)
#pragma unroll
    for (int j = 0; j < kSJ; ++j) {
      const Tap e = tap_s[g + kSG * j];
      const T z = *reinterpret_cast<const T*>(col_base + e.off);
      acc[j] = fma((T)e.sgn, z, acc[j]);
    }
    __syncthreads();
  }
  const int64_t cc = c0 + c;
  if (cc < a.nc) {
    T* o = a.out + ((int64_t)blockIdx.y * a.nc + cc) * a.ldo;
#pragma unroll
    for (int j = 0; j < kSJ; ++j) {
      const int r = g + kSG * j;
      if (r < a.l) o[r] = (T)(a.scale * (double)acc[j]);
    }
  }
}

// Y^T(c, r) = sum over splits s (in order) of part[s](c, r).
template <typename T>
__global__ void srht_reduce_kernel(const T* part, int splits, int64_t nc, int l, int64_t ldo, T* Yt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nc * l) return;
  const int64_t c = e / l, r = e % l;
  double s = 0.0;
  for (int q = 0; q < splits; ++q) s += (double)part[((int64_t)q * nc + c) * ldo + r];
  Yt[c * ldo + r] = (T)s;
}

template <typename T>
hipError_t launch_t(const SrhtDesc& d, void* part, hipStream_t stream) {
  SArgs<T> a{};
  a.X = static_cast<const T*>(d.X); a.xr = d.xr; a.xc = d.xc;
  a.mr = d.mr; a.nc = d.nc;
  a.signs = d.signs; a.rows = d.rows; a.l = d.l;
  a.ldo = d.ldo;
  a.nblk = ceil_div(d.mr, kSB);
  a.bps = ceil_div(a.nblk, d.splits);
  int64_t mp = 1;
  while (mp < d.mr) mp *= 2;
  a.mp = mp;
  a.scale = 1.0 / std::sqrt((double)std::max(d.l, 1));
  a.status = d.status;
  a.out = d.splits > 1 ? static_cast<T*>(part) : static_cast<T*>(d.Yt);
  // x: column blocks rounded up to a multiple of 8 (the XCD-aware order skips
  // the indices past the last block)
  const dim3 grid((unsigned)round_up(ceil_div(d.nc, kSC), 8), (unsigned)d.splits);
  const bool wide = d.l > kSG * 16;
  // column descriptors hold a column's bytes (plus a block of slack for the
  // offsets past mr) in 31 bits
  const bool bufok = (d.mr + kSB) * (int64_t)sizeof(T) < ((int64_t)1 << 31);
  // row-major: a block's bytes (and the offsets of the columns past nc, from
  // 2^31 up) in 32 bits
  const bool rbufok = (kSB + 1) * d.xr * (int64_t)sizeof(T) < ((int64_t)1 << 31) && d.xr >= d.nc;
  if (d.xc == 1 && rbufok) {
    if (wide) hipLaunchKernelGGL((srht_kernel<T, 3, 32>), grid, dim3(kST), 0, stream, a);
    else hipLaunchKernelGGL((srht_kernel<T, 3, 16>), grid, dim3(kST), 0, stream, a);
  } else if (d.xc == 1) {
    if (wide) hipLaunchKernelGGL((srht_kernel<T, 0, 32>), grid, dim3(kST), 0, stream, a);
    else hipLaunchKernelGGL((srht_kernel<T, 0, 16>), grid, dim3(kST), 0, stream, a);
  } else if (bufok) {
    if (wide) hipLaunchKernelGGL((srht_kernel<T, 2, 32>), grid, dim3(kST), 0, stream, a);
    else hipLaunchKernelGGL((srht_kernel<T, 2, 16>), grid, dim3(kST), 0, stream, a);
  } else {
    if (wide) hipLaunchKernelGGL((srht_kernel<T, 1, 32>), grid, dim3(kST), 0, stream, a);
    else hipLaunchKernelGGL((srht_kernel<T, 1, 16>), grid, dim3(kST), 0, stream, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || d.splits == 1) return e;
  const int64_t tot = d.nc * d.l;
  hipLaunchKernelGGL((srht_reduce_kernel<T>), dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, stream,
                     static_cast<const T*>(part), d.splits, d.nc, d.l, d.ldo, static_cast<T*>(d.Yt));
  return hipGetLastError();
}

}  // namespace

// Splits of the row blocks: about four workgroups per CU over the column
// blocks, each split at least 8 blocks (2048 rows) deep.
int srht_pick_splits(int64_t mr, int64_t nc, int num_cus) {
  const int64_t cb = ceil_div(nc, kSC), nblk = ceil_div(mr, kSB);
  int64_t s = ceil_div(4LL * std::max(num_cus, 1), cb);
  s = std::min<int64_t>(s, std::max<int64_t>(1, nblk / 8));
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

size_t srht_part_bytes(const SrhtDesc& d, int esize) {
  return d.splits > 1 ? (size_t)d.splits * d.nc * d.ldo * esize : 0;
}

hipError_t srht_launch(int dtype, const SrhtDesc& d, void* part, hipStream_t stream) {
  if (d.l < 1 || d.l > kSrhtMaxRows || d.splits < 1 || (d.xc != 1 && d.xr != 1)) return hipErrorInvalidValue;
  if (d.mr <= 0 || d.nc <= 0) return hipSuccess;
  return dtype == 0 ? launch_t<double>(d, part, stream) : launch_t<float>(d, part, stream);
}

}  // namespace idcur
