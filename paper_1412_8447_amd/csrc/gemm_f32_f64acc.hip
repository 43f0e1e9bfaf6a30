// GEMM instantiations: A float, B float, accumulation double.
#include "gemm_kernel.hpp"

namespace idcur {
namespace gk {
hipError_t launch_f32_f64acc(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s) {
  return launch_types<float, float, double>(nt, k, grid, akc, bnc, s);
}
}  // namespace gk
}  // namespace idcur
