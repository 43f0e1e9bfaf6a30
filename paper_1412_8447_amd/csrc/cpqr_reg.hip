// Host side of the register-slab CPQR (kernel in cpqr_reg_kernel.hpp; the FP32
// and FP64 instantiations are compiled in cpqr_reg_f32.hip and cpqr_reg_f64.hip).
#include <cstdlib>

#include "cpqr_reg_kernel.hpp"

namespace idcur {
using namespace cr;

const void* cpqr_reg_fn_f32(int cfg);
const void* cpqr_reg_fn_f64(int cfg);

// IDCUR_CPQR_REGCFG=i restricts the search to table entry i, so that a test
// can run every configuration on a matrix it covers; an entry that does not fit
// then leaves the choice to the other kernels.
int cpqr_reg_pick(int dtype_size, int l, int n, int num_cus, int* G, int* cols_per_wg) {
  const char* force = getenv("IDCUR_CPQR_REGCFG");
  const int forced = force ? atoi(force) : -1;
  for (int i = 0; i < kNumRegCfgs; ++i) {
    const RegCfg c = kRegCfgs[i];
    if (forced >= 0 && i != forced) continue;
    if (c.R * c.RPL < l) continue;
    if (c.NC * c.RPL * dtype_size / 4 > (dtype_size == 4 ? kRegSlabCap<float> : kRegSlabCap<double>)) continue;
    const int cp = (kRT / c.R) * c.NC;
    const int64_t g = ceil_div(n, cp);
    if (g > num_cus || g < 1) continue;
    *G = (int)g;
    *cols_per_wg = cp;
    return i;
  }
  return -1;
}

size_t cpqr_reg_lds_bytes(int cfg, int kmax_host, int cols_per_wg, int dtype_size) {
  const RegCfg c = kRegCfgs[cfg];
  return ((size_t)kmax_host + (size_t)cols_per_wg) * sizeof(int) / 16 * 16 + 16 + (size_t)c.R * c.RPL * dtype_size;
}

size_t cpqr_reg_rec_bytes(int G) { return 2 * (size_t)kRep * G * kRecWords * sizeof(uint64_t); }
size_t cpqr_reg_cvals_bytes(int cfg, int G, int dtype_size) {
  const RegCfg c = kRegCfgs[cfg];
  return 2 * (size_t)G * ((size_t)c.R * c.RPL * (dtype_size / 4) + 2) * sizeof(uint64_t);
}

hipError_t cpqr_reg_launch(int dtype, int cfg, int G, CpqrArgs a, size_t lds_bytes, hipStream_t stream) {
  if (cfg < 0 || cfg >= kNumRegCfgs) return hipErrorInvalidValue;
  const void* fn = dtype == 0 ? cpqr_reg_fn_f64(cfg) : cpqr_reg_fn_f32(cfg);
  if (!fn) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(G), dim3(kRT), args, (unsigned)lds_bytes, stream);
}

}  // namespace idcur
