// float instantiations of the register-slab CPQR kernel.
#include "cpqr_reg_kernel.hpp"

namespace idcur {
const void* cpqr_reg_fn_f32(int cfg) {
  return cr::reg_kernel_lookup<float>(cfg, std::make_integer_sequence<int, cr::kNumRegCfgs>{});
}
}  // namespace idcur
