// Face-halo fill between patches (the engine's consistency step of Section 2
// of arXiv 2302.09005): every face-halo volume takes the facing interior
// volume of its neighbour, or (transmissive boundary, neighbour -1) the
// patch's own boundary volume.  One thread per halo value; the innermost
// thread index runs along the first tangential axis, which is contiguous in
// memory for y- and z-faces.  Edge and corner halo volumes are not touched.
//
// The x-face values are strided (one volume per row of p + 2), so every one
// of them costs a whole memory sector, and a row holds the values that two
// different patches need (the +x halo of one neighbour, the -x halo of the
// other).  Workgroups are handed to the XCDs in contiguous ranges, so that
// the workgroups of neighbouring patches share an L2 and the second reader
// of a row finds it there.
#include "fv_internal.hpp"

namespace fvk {

namespace {

template <int D, int P>
__global__ void __launch_bounds__(256)
fill_halo_kernel(const fv_patch* __restrict__ patches, int64_t n,
                 const int64_t* __restrict__ neighbours, double* __restrict__ q, int64_t q_len,
                 int which) {
  constexpr int S = D + 2;
  constexpr int W = P + 2;
  constexpr int FACE = ipow(P, D - 1);
  constexpr int64_t VIN = ipow(W, D);
  const int64_t total = n * (2 * D) * S * FACE;
  // workgroup w runs on XCD w mod 8: give each XCD a contiguous range
  const int64_t nwg = gridDim.x, w = blockIdx.x;
  const int64_t xq = nwg / 8, xr = nwg % 8, xc = w % 8;
  const int64_t wgi = xc * xq + (xc < xr ? xc : xr) + w / 8;
  const int64_t i = wgi * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int64_t rest = i;
  const int t1 = (int)(rest % P);
  rest /= P;
  int t2 = 0;
  if (D == 3) {
    t2 = (int)(rest % P);
    rest /= P;
  }
  const int m = (int)(rest % S);
  rest /= S;
  const int f = (int)(rest % (2 * D));
  const int64_t b = rest / (2 * D);
  const int ax = f >> 1, side = f & 1;
  const int64_t nb = neighbours[b * (2 * D) + f];
  if (nb < -1 || nb >= n) return;
  const int64_t src = nb >= 0 ? nb : b;
  const int64_t od = which == FV_OFFSETS_OUT ? patches[b].q_out : patches[b].q_in;
  const int64_t os = which == FV_OFFSETS_OUT ? patches[src].q_out : patches[src].q_in;
  const int64_t lim = q_len - S * VIN;
  if (od < 0 || od > lim || os < 0 || os > lim) return;
  if (patches[b].p != P || patches[src].p != P) return;
  const int dst_c = side ? P + 1 : 0;
  const int src_c = nb >= 0 ? (side ? 1 : P) : (side ? P : 1);
  int cd[3], cs[3];
  const int tang[2] = {t1 + 1, t2 + 1};
  int k = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      cd[a] = cs[a] = 0;
    } else if (a == ax) {
      cd[a] = dst_c;
      cs[a] = src_c;
    } else {
      cd[a] = cs[a] = tang[k++];
    }
  }
  const int64_t id = cd[0] + (int64_t)W * cd[1] + (int64_t)W * W * cd[2];
  const int64_t is = cs[0] + (int64_t)W * cs[1] + (int64_t)W * W * cs[2];
  q[od + (int64_t)m * VIN + id] = q[os + (int64_t)m * VIN + is];
}

template <int D, int P>
void launch_h(const fv_patch* patches, int64_t n, const int64_t* nbr, double* q, int64_t q_len,
              int which, hipStream_t st) {
  const int64_t total = n * (2 * D) * (D + 2) * ipow(P, D - 1);
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL((fill_halo_kernel<D, P>), dim3((unsigned)blocks), dim3(256), 0, st, patches,
                     n, nbr, q, q_len, which);
}

}  // namespace

int launch_fill_halo_f64(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                         double* q, int64_t q_len, int which, int dim, int p, hipStream_t st) {
#define FV_CASE(DD, PP)                                                      \
  if (dim == DD && p == PP) {                                                \
    launch_h<DD, PP>(patches, n, neighbours, q, q_len, which, st);           \
    return 0;                                                                \
  }
  FV_CASE(2, 4)
  FV_CASE(2, 8)
  FV_CASE(2, 16)
  FV_CASE(2, 17)
  FV_CASE(2, 32)
  FV_CASE(3, 4)
  FV_CASE(3, 8)
  FV_CASE(3, 16)
#undef FV_CASE
  return FV_EUNSUPPORTED;
}

}  // namespace fvk
