// Sketch of a sparse matrix in compressed sparse column form (Section 5.1, eq.
// (Y=OmegaA), for the sparse matrices that motivate the ID and CUR): for each
// column j, Y^T(j, :) = sum over the stored A(i, j) of A(i, j) Omega(:, i)^T.
// Omega^T is stored m x ldom row-major, so every stored entry reads one
// contiguous row of it: a wave takes a column (or a split of its entries) and
// its 64 lanes read consecutive elements of each row, 64 R sketch rows at a
// time, eight rows in flight. Splits of a column's entries write partial rows that a second kernel
// adds in split order, so the result does not depend on scheduling.
#include "common.hpp"
#include "kernels.hpp"

namespace idcur {
namespace {

template <typename T>
struct SpArgs {
  int64_t m, n, nnz;
  const int64_t* colptr;
  const int* rowidx;
  const T* vals;
  const T* Omt; int64_t ldom;
  int l;
  T* out; int64_t ldo;   // split s writes rows s*n .. (s+1)*n - 1 (ld ldo)
  int splits;
  int* status;
};

template <typename T, int R>
__global__ __launch_bounds__(256) void spmm_csc_kernel(SpArgs<T> a) {
  const int lane = threadIdx.x & 63;
  const int wpg = blockDim.x >> 6;                       // waves per workgroup
  const int s = blockIdx.y * wpg + (threadIdx.x >> 6);   // this wave's split
  const int64_t j = blockIdx.x;
  if (s >= a.splits) return;   // whole wave; the kernel has no barrier
  int64_t p0 = a.colptr[j], p1 = a.colptr[j + 1];
  if (p0 < 0 || p1 > a.nnz || p0 > p1) {
    if (lane == 0) set_status(a.status, ST_BADINDEX);
    p0 = p1 = 0;
  }
  const int64_t len = p1 - p0;
  const int64_t q0 = p0 + len * s / a.splits, q1 = p0 + len * (s + 1) / a.splits;
  T* o = a.out + ((int64_t)s * a.n + j) * a.ldo;
  // 64 entries at a time: lane t loads entry t (coalesced), then their row
  // indices and values are broadcast one by one and eight rows of Omega^T are
  // in flight together; entries are added in storage order.
  bool bad = false;
  for (int c0 = 0; c0 < a.ldo; c0 += 64 * R) {
    T acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = T(0);
    for (int64_t pb = q0; pb < q1; pb += 64) {
      const int64_t pp = pb + lane;
      const bool in = pp < q1;
      int iv = in ? a.rowidx[pp] : 0;
      T vv = in ? a.vals[pp] : T(0);
      if (iv < 0 || iv >= a.m) {   // skipped and reported
        bad = true;
        iv = 0;
        vv = T(0);
      }
      const int cnt = (int)min<int64_t>(64, q1 - pb);   // the same for every lane
      for (int u0 = 0; u0 < cnt; u0 += 8) {
        T x[8][R];
        T w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {   // entries past cnt carry value 0 and row 0
          const int i = __shfl(iv, u0 + u, 64);
          w[u] = __shfl(vv, u0 + u, 64);
          const T* om = a.Omt + (int64_t)i * a.ldom;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int c = c0 + lane + 64 * r;
            x[u][r] = c < a.l ? om[c] : T(0);
          }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] += w[u] * x[u][r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int c = c0 + lane + 64 * r;
      if (c < a.ldo) o[c] = c < a.l ? acc[r] : T(0);
    }
  }
  if (bad) set_status(a.status, ST_BADINDEX);
}

// Y^T(j, c) = sum over splits s (in order) of part[s](j, c).
template <typename T>
__global__ void spmm_reduce_kernel(const T* part, int splits, int64_t n, int64_t ldo, T* Yt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * ldo) return;
  T acc = T(0);
  for (int q = 0; q < splits; ++q) acc += part[(int64_t)q * n * ldo + e];
  Yt[e] = acc;
}

template <typename T>
hipError_t launch_t(const SpmmDesc& d, void* part, hipStream_t stream) {
  SpArgs<T> a{};
  a.m = d.m; a.n = d.n; a.nnz = d.nnz;
  a.colptr = d.colptr; a.rowidx = d.rowidx; a.vals = static_cast<const T*>(d.vals);
  a.Omt = static_cast<const T*>(d.Omt); a.ldom = d.ldom;
  a.l = d.l; a.ldo = d.ldo; a.splits = d.splits; a.status = d.status;
  a.out = d.splits > 1 ? static_cast<T*>(part) : static_cast<T*>(d.Yt);
  const int wpg = d.splits >= 4 ? 4 : 1;
  const dim3 grid((unsigned)d.n, (unsigned)ceil_div(d.splits, wpg));
  const dim3 block(64 * wpg);
  if (d.l <= 64) hipLaunchKernelGGL((spmm_csc_kernel<T, 1>), grid, block, 0, stream, a);
  else if (d.l <= 128) hipLaunchKernelGGL((spmm_csc_kernel<T, 2>), grid, block, 0, stream, a);
  else hipLaunchKernelGGL((spmm_csc_kernel<T, 4>), grid, block, 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || d.splits == 1) return e;
  const int64_t tot = d.n * d.ldo;
  hipLaunchKernelGGL((spmm_reduce_kernel<T>), dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, stream,
                     static_cast<const T*>(part), d.splits, d.n, d.ldo, static_cast<T*>(d.Yt));
  return hipGetLastError();
}

// C (m x kcap, row-major ldc, zero on entry) = A(:, J[0:k]) for a matrix in
// compressed sparse column form: column s of C receives the stored entries of
// column J[s]. Workgroup (s, y) scatters slice y of the entries; repeated rows
// add up (in a scheduling-dependent order when a column repeats a row three or
// more times). k = min(*k_dev, kcap).
template <typename T>
__global__ __launch_bounds__(256) void csc_gather_cols_kernel(int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                                                            const int* rowidx, const T* vals, const int* J, int kcap,
                                                            const int* k_dev, T* C, int64_t ldc, int* status) {
  const int s = blockIdx.x;
  const int k = min(*k_dev, kcap);
  if (s >= k) return;
  const int j = J[s];
  if (j < 0 || j >= n) {
    if (threadIdx.x == 0) set_status(status, ST_BADINDEX);
    return;
  }
  int64_t p0 = colptr[j], p1 = colptr[j + 1];
  if (p0 < 0 || p1 > nnz || p0 > p1) {
    if (threadIdx.x == 0) set_status(status, ST_BADINDEX);
    return;
  }
  const int64_t len = p1 - p0;
  const int64_t q0 = p0 + len * blockIdx.y / gridDim.y, q1 = p0 + len * (blockIdx.y + 1) / gridDim.y;
  for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const int i = rowidx[q];
    if (i < 0 || i >= m) {
      set_status(status, ST_BADINDEX);
      continue;
    }
    atomicAdd(&C[(int64_t)i * ldc + s], vals[q]);
  }
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int* p, int64_t n, int v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}
hipError_t fill_i32_launch(int* p, int64_t n, int v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 4096)), dim3(256), 0, stream,
                     p, n, v);
  return hipGetLastError();
}

// slot[i] = s for the selected rows i = I[s], s < min(*k_dev, kcap) (slot is -1
// everywhere else on entry).
__global__ __launch_bounds__(256) void csc_row_slots_kernel(int64_t m, const int* I, int kcap, const int* k_dev,
                                                          int* slot) {
  const int k = min(*k_dev, kcap);
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < k; s += gridDim.x * blockDim.x) {
    const int i = I[s];
    if (i >= 0 && i < m) slot[i] = s;
  }
}

// R (kcap x n, row-major ldr, zero on entry) = A(I[0:k], :): every stored entry
// whose row is selected goes to its slot's row. Workgroup j reads column j's
// entries once.
template <typename T>
__global__ __launch_bounds__(256) void csc_gather_rows_kernel(int64_t m, int64_t nnz, const int64_t* colptr,
                                                            const int* rowidx, const T* vals, const int* slot, T* R,
                                                            int64_t ldr) {
  const int64_t j = blockIdx.x;
  int64_t p0 = colptr[j], p1 = colptr[j + 1];
  if (p0 < 0 || p1 > nnz || p0 > p1) return;   // reported by the sketch
  for (int64_t q = p0 + threadIdx.x; q < p1; q += blockDim.x) {
    const int i = rowidx[q];
    if (i < 0 || i >= m) continue;
    const int sl = slot[i];
    if (sl >= 0) atomicAdd(&R[(int64_t)sl * ldr + j], vals[q]);
  }
}

}  // namespace

hipError_t csc_gather_cols_launch(int dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                                  const int* rowidx, const void* vals, const int* J, int kcap, const int* k_dev,
                                  void* C, int64_t ldc, int* status, hipStream_t stream) {
  if (kcap <= 0) return hipSuccess;
  const int64_t per = std::max<int64_t>(1, nnz / std::max<int64_t>(n, 1));
  const unsigned ys = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, per / 2048));
  const dim3 grid((unsigned)kcap, ys);
  if (dtype == 0)
    hipLaunchKernelGGL(csc_gather_cols_kernel<double>, grid, dim3(256), 0, stream, m, n, nnz, colptr, rowidx,
                       static_cast<const double*>(vals), J, kcap, k_dev, static_cast<double*>(C), ldc, status);
  else
    hipLaunchKernelGGL(csc_gather_cols_kernel<float>, grid, dim3(256), 0, stream, m, n, nnz, colptr, rowidx,
                       static_cast<const float*>(vals), J, kcap, k_dev, static_cast<float*>(C), ldc, status);
  return hipGetLastError();
}

hipError_t csc_gather_rows_launch(int dtype, int64_t m, int64_t n, int64_t nnz, const int64_t* colptr,
                                  const int* rowidx, const void* vals, const int* I, int kcap, const int* k_dev,
                                  int* slot, void* R, int64_t ldr, hipStream_t stream) {
  if (kcap <= 0 || n <= 0) return hipSuccess;
  hipError_t e = fill_i32_launch(slot, m, -1, stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(csc_row_slots_kernel, dim3((unsigned)ceil_div(kcap, 256)), dim3(256), 0, stream, m, I, kcap,
                     k_dev, slot);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == 0)
    hipLaunchKernelGGL(csc_gather_rows_kernel<double>, dim3((unsigned)n), dim3(256), 0, stream, m, nnz, colptr,
                       rowidx, static_cast<const double*>(vals), slot, static_cast<double*>(R), ldr);
  else
    hipLaunchKernelGGL(csc_gather_rows_kernel<float>, dim3((unsigned)n), dim3(256), 0, stream, m, nnz, colptr,
                       rowidx, static_cast<const float*>(vals), slot, static_cast<float*>(R), ldr);
  return hipGetLastError();
}

// Splits of each column's entries: enough waves to fill the chip (32 per CU)
// over few columns, each split about 64 entries or more; 1 when the columns
// alone fill it.
int spmm_pick_splits(int64_t n, int64_t nnz, int num_cus) {
  const int64_t want = ceil_div(32LL * std::max(num_cus, 1), std::max<int64_t>(n, 1));
  const int64_t most = std::max<int64_t>(1, nnz / (64 * std::max<int64_t>(n, 1)));
  int64_t s = std::min(want, most);
  if (s <= 1) return 1;
  s = std::min<int64_t>(round_up(s, 4), 256);
  return (int)s;
}

size_t spmm_part_bytes(const SpmmDesc& d, int esize) {
  return d.splits > 1 ? (size_t)d.splits * d.n * d.ldo * esize : 0;
}

hipError_t spmm_csc_launch(int dtype, const SpmmDesc& d, void* part, hipStream_t stream) {
  if (d.l < 1 || d.ldo < d.l || d.ldom < d.l || d.splits < 1 || (d.splits > 1 && d.splits % 4)) return hipErrorInvalidValue;
  if (d.n <= 0) return hipSuccess;
  if (d.n > 0x7fffffff) return hipErrorInvalidValue;
  return dtype == 0 ? launch_t<double>(d, part, stream) : launch_t<float>(d, part, stream);
}

}  // namespace idcur
