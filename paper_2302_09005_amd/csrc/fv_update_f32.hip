// The update kernels' float32 instances (kernels in fv_update_kernels.hpp).
// This translation unit is compiled with the scheduler that favours
// instruction-level parallelism: the float march has registers to spare at
// four waves per SIMD (123 of 128 with it, 100 without), and on 4096 patches
// of 8^3 the pipelined step runs about 3 % faster.  The float64 instances keep
// the default schedule, which holds them at 126 registers; with this one they
// need 148 and lose a wave per SIMD.
#include "fv_update_kernels.hpp"

namespace fvk {

FV_INSTANTIATE(float)
#undef FV_INSTANTIATE

}  // namespace fvk
