// Host side of the on-chip-slab CPQR (kernel in cpqr_res_kernel.hpp; FP32 only).
#include <cstdlib>

#include "cpqr_res_kernel.hpp"

namespace idcur {
using namespace cr;

namespace {
// LDS per workgroup on gfx950, less the kernel's static arrays
constexpr size_t kResLdsCap = 160 * 1024 - 256;
}  // namespace

size_t cpqr_res_lds_bytes(int cfg, int kmax_host, int cols_per_wg) {
  // the winning column, the norms and thresholds, the pivots and column flags
  // (padded to 16 bytes), then the LDS slots of the slab
  const ResCfg c = kResCfgs[cfg];
  const size_t head = (size_t)16 * c.RPL * sizeof(float) + 2 * (size_t)(c.NC + c.NL) * (c.NTH / 16) * sizeof(double) +
                      ((size_t)kmax_host + (size_t)cols_per_wg) * sizeof(int);
  return (head + 15) / 16 * 16 + (size_t)c.NL * c.RPL * c.NTH * sizeof(float);
}

// IDCUR_CPQR_RESCFG=i restricts the search to table entry i (tests run it on
// shapes the register-slab kernel also covers, to compare the two).
int cpqr_res_pick(int dtype_size, int l, int n, int kmax_host, int num_cus, int* G, int* cols_per_wg) {
  if (dtype_size != 4) return -1;
  const char* force = getenv("IDCUR_CPQR_RESCFG");
  const int forced = force ? atoi(force) : -1;
  for (int i = 0; i < kNumResCfgs; ++i) {
    const ResCfg c = kResCfgs[i];
    if (forced >= 0 && i != forced) continue;
    if (16 * c.RPL < l) continue;
    const int cp = (c.NTH / 16) * (c.NC + c.NL);
    const int64_t g = ceil_div(n, cp);
    if (g > num_cus || g < 1) continue;
    if (cpqr_res_lds_bytes(i, kmax_host, cp) > kResLdsCap) continue;
    *G = (int)g;
    *cols_per_wg = cp;
    return i;
  }
  return -1;
}

bool cpqr_res_forced() { return getenv("IDCUR_CPQR_RESCFG") != nullptr; }

size_t cpqr_res_cvals_bytes(int cfg, int G) {
  const ResCfg c = kResCfgs[cfg];
  return 2 * (size_t)G * ((size_t)16 * c.RPL + 2) * sizeof(uint64_t);
}

hipError_t cpqr_res_launch(int cfg, int G, CpqrArgs a, size_t lds_bytes, hipStream_t stream) {
  if (cfg < 0 || cfg >= kNumResCfgs) return hipErrorInvalidValue;
  const void* fn = res_kernel_lookup(cfg, a.norms_exact != 0, std::make_integer_sequence<int, kNumResCfgs>{});
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(kResCfgs[cfg].NTH), args, (unsigned)lds_bytes, stream);
}

}  // namespace idcur
