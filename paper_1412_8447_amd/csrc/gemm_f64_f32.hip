// GEMM instantiations: A double, B float, accumulation double.
#include "gemm_kernel.hpp"

namespace idcur {
namespace gk {
hipError_t launch_f64_f32(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s) {
  return launch_types<double, float, double>(nt, k, grid, akc, bnc, s);
}
}  // namespace gk
}  // namespace idcur
