// The update kernels' float64 instances and the launch helpers that are not
// templates (the kernels themselves are in fv_update_kernels.hpp; the float32
// instances are built in fv_update_f32.hip with an instruction schedule of
// their own).
#include "fv_update_kernels.hpp"

namespace fvk {

int64_t update_workgroups(int dim, int p, int64_t n) {
#define FV_CASE(DD, PP) \
  if (dim == DD && p == PP) return (n + Geo<DD, PP>::PPW - 1) / Geo<DD, PP>::PPW;
  FV_CASE(2, 4)
  FV_CASE(2, 8)
  FV_CASE(2, 16)
  FV_CASE(2, 17)
  FV_CASE(2, 32)
  FV_CASE(3, 4)
  FV_CASE(3, 8)
  FV_CASE(3, 16)
#undef FV_CASE
  return 0;
}

bool update_supported(int dim, int p) {
  if (dim == 2) return p == 4 || p == 8 || p == 16 || p == 17 || p == 32;
  if (dim == 3) return p == 4 || p == 8 || p == 16;
  return false;
}

int mixed_patches_per_unit(int p) {
  // one 16^3 patch per workgroup; one 8^3 patch, or four 4^3 patches, per wave
  return p == 16 ? MixedGeo<16>::PPW
       : p == 8  ? (kMixedNT / 64) * MixedGeo<8>::PPW
       : p == 4  ? (kMixedNT / 64) * MixedGeo<4>::PPW
                 : 0;
}

template int launch_step_halo<double>(const fv_patch*, int64_t, const int64_t*, const double*,
                                      int64_t, double*, int64_t, int, int, double,
                                      const double*, double*, const CflOut&, hipStream_t);

FV_INSTANTIATE(double)
#undef FV_INSTANTIATE

}  // namespace fvk
