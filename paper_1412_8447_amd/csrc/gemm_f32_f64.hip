// GEMM instantiations: A float, B double, accumulation double.
#include "gemm_kernel.hpp"

namespace idcur {
namespace gk {
hipError_t launch_f32_f64(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s) {
  return launch_types<float, double, double>(nt, k, grid, akc, bnc, s);
}
}  // namespace gk
}  // namespace idcur
