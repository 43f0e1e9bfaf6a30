// 16-bit sketch GEMM instantiations with FP16 operands.
#include "gemm16_kernel.hpp"
#include "gemm16w_kernel.hpp"

namespace idcur {
namespace g16 {
hipError_t launch_fp16(int nt, const Args& a, bool akc, hipStream_t s) { return launch_h<true>(nt, a, akc, s); }
hipError_t launch_wide_fp16(const Args& a, bool akc, int cb, hipStream_t s) { return launch_wide<true>(a, akc, cb, s); }
}  // namespace g16
}  // namespace idcur
