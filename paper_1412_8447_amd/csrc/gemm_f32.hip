// GEMM instantiations: A float, B float, accumulation float.
#include "gemm_kernel.hpp"

namespace idcur {
namespace gk {
hipError_t launch_f32(int nt, const KArgs& k, dim3 grid, bool akc, bool bnc, hipStream_t s) {
  return launch_types<float, float, float>(nt, k, grid, akc, bnc, s);
}
}  // namespace gk
}  // namespace idcur
