// Largest-eigenvalue reductions (Algorithm 1 last step; Section 4 of
// arXiv 2302.09005) and the global CFL time step.
//
//  * patch_max_kernel: one workgroup per patch; every lane decodes volumes of
//    the patch interior (coalesced unknown-major reads), takes
//    max_j(|u_j| + c), and the workgroup reduces with wave shuffles and LDS.
//  * reduce_cfl_kernel: one workgroup folds the per-patch maxima (NaN wins)
//    and the smallest volume width into Lambda and
//    dt = cfl * min dx / (dim * Lambda).  A single workgroup keeps the result
//    deterministic and needs no atomics.
#include "fv_euler.hpp"
#include "fv_internal.hpp"

namespace fvk {

namespace {

constexpr int kRedThreads = 256;

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = nanmax_pos(v, T(__shfl_xor(v, o, 64)));
  return v;
}

template <typename T, int D, int P>
__global__ void __launch_bounds__(kRedThreads)
patch_max_kernel(const fv_patch* __restrict__ patches, int64_t n, const T* __restrict__ q,
                 int64_t q_len, int q_halo, int which, T gamma,
                 double* __restrict__ per_patch) {
  constexpr int S = D + 2;
  __shared__ double red[kRedThreads / 64];
  const int64_t b = blockIdx.x;
  if (b >= n) return;
  const fv_patch pd = patches[b];
  const int64_t off = which == FV_OFFSETS_OUT ? pd.q_out : pd.q_in;
  const int w = q_halo ? P + 2 : P;
  const int o = q_halo ? 1 : 0;
  const int64_t vol = q_halo ? (int64_t)ipow(P + 2, D) : (int64_t)ipow(P, D);
  const bool ok = pd.p == P && off >= 0 && off <= q_len - S * vol;
  T lam = T(0);
  if (ok) {
    const T* blk = q + off;
    for (int i = threadIdx.x; i < ipow(P, D); i += kRedThreads) {
      const int x = i % P;
      const int y = (i / P) % P;
      const int z = D == 3 ? i / (P * P) : 0;
      const int64_t idx = (x + o) + (int64_t)w * (y + o) + (D == 3 ? (int64_t)w * w * (z + o) : 0);
      T qv[S];
#pragma unroll
      for (int m = 0; m < S; ++m) qv[m] = blk[(int64_t)m * vol + idx];
      const Prim<T> wv = decode<T, D>(qv, gamma);
      lam = nanmax_pos(lam, max_wave_speed<T, D>(qv, wv));
    }
  }
  double lamd = wave_max(double(lam));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lamd;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 1; i < kRedThreads / 64; ++i) lamd = nanmax_pos(lamd, red[i]);
    per_patch[b] = ok ? lamd : __builtin_nan("");
  }
}

// Conserved totals in FP64 whatever the state's precision: one workgroup per
// patch sums its interior volumes per unknown (fixed order: strided partial
// sums, then a fixed shuffle tree), then one workgroup sums the patches in a
// fixed order.  Deterministic for a given batch.
template <typename T, int D, int P>
__global__ void __launch_bounds__(kRedThreads)
patch_totals_kernel(const fv_patch* __restrict__ patches, int64_t n, const T* __restrict__ q,
                    int64_t q_len, int q_halo, int which, double* __restrict__ per_patch) {
  constexpr int S = D + 2;
  __shared__ double red[S][kRedThreads / 64];
  const int64_t b = blockIdx.x;
  if (b >= n) return;
  const fv_patch pd = patches[b];
  const int64_t off = which == FV_OFFSETS_OUT ? pd.q_out : pd.q_in;
  const int w = q_halo ? P + 2 : P;
  const int o = q_halo ? 1 : 0;
  const int64_t vol = q_halo ? (int64_t)ipow(P + 2, D) : (int64_t)ipow(P, D);
  const bool ok = pd.p == P && off >= 0 && off <= q_len - S * vol;
  double acc[S];
#pragma unroll
  for (int m = 0; m < S; ++m) acc[m] = 0.0;
  if (ok) {
    const T* blk = q + off;
    for (int i = threadIdx.x; i < ipow(P, D); i += kRedThreads) {
      const int x = i % P;
      const int y = (i / P) % P;
      const int z = D == 3 ? i / (P * P) : 0;
      const int64_t idx = (x + o) + (int64_t)w * (y + o) + (D == 3 ? (int64_t)w * w * (z + o) : 0);
#pragma unroll
      for (int m = 0; m < S; ++m) acc[m] += double(blk[(int64_t)m * vol + idx]);
    }
  }
#pragma unroll
  for (int m = 0; m < S; ++m) {
    double v = acc[m];
#pragma unroll
    for (int off2 = 32; off2 > 0; off2 >>= 1) v += __shfl_xor(v, off2, 64);
    if ((threadIdx.x & 63) == 0) red[m][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int m = 0; m < S; ++m) {
      double v = red[m][0];
      for (int i = 1; i < kRedThreads / 64; ++i) v += red[m][i];
      per_patch[b * S + m] = ok ? v : __builtin_nan("");
    }
  }
}

__global__ void __launch_bounds__(1024)
sum_patches_kernel(const double* __restrict__ per_patch, int64_t n, int s,
                   double* __restrict__ totals) {
  __shared__ double red[16];
  for (int m = 0; m < s; ++m) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += blockDim.x) v += per_patch[b * s + m];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = red[0];
      for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t += red[i];
      totals[m] = t;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024)
reduce_cfl_kernel(const fv_patch* __restrict__ patches, int64_t n,
                  const double* __restrict__ per_patch, int dim, double cfl,
                  double* __restrict__ lambda_out, double* __restrict__ dt_out) {
  __shared__ double rl[16], rh[16];
  constexpr int U = 4;  // patches per thread and round: their loads are issued together
  double lam = 0.0, h = __builtin_inf();
  for (int64_t b0 = threadIdx.x; b0 < n; b0 += (int64_t)U * blockDim.x) {
    double lv[U], hv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t b = b0 + (int64_t)u * blockDim.x;
      lv[u] = 0.0;
      hv[u] = __builtin_inf();
      if (b < n) {
        lv[u] = per_patch[b];
        const double* dx = patches[b].dx;
        hv[u] = fmin(dx[0], dx[1]);
        if (dim == 3) hv[u] = fmin(hv[u], dx[2]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      lam = nanmax_pos(lam, lv[u]);
      h = fmin(h, hv[u]);
    }
  }
  lam = wave_max(lam);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) h = fmin(h, __shfl_xor(h, o, 64));
  if ((threadIdx.x & 63) == 0) {
    rl[threadIdx.x >> 6] = lam;
    rh[threadIdx.x >> 6] = h;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      lam = nanmax_pos(lam, rl[i]);
      h = fmin(h, rh[i]);
    }
    if (lambda_out) *lambda_out = lam;
    if (dt_out) *dt_out = cfl * h / ((double)dim * lam);
  }
}

template <typename T, int D, int P>
void launch_pm(const fv_patch* patches, int64_t n, const T* q, int64_t q_len, int q_halo,
               int which, double gamma, double* per_patch, hipStream_t st) {
  hipLaunchKernelGGL((patch_max_kernel<T, D, P>), dim3((unsigned)n), dim3(kRedThreads), 0, st,
                     patches, n, q, q_len, q_halo, which, T(gamma), per_patch);
}

template <typename T, int D, int P>
void launch_tot(const fv_patch* patches, int64_t n, const T* q, int64_t q_len, int q_halo,
                int which, double* per_patch, hipStream_t st) {
  hipLaunchKernelGGL((patch_totals_kernel<T, D, P>), dim3((unsigned)n), dim3(kRedThreads), 0, st,
                     patches, n, q, q_len, q_halo, which, per_patch);
}

// Local time steps: one thread per patch, dt = cfl * min dx / (dim * lambda).
__global__ void __launch_bounds__(256)
local_dt_kernel(fv_patch* __restrict__ patches, int64_t n, const double* __restrict__ per_patch,
                int dim, double cfl) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= n) return;
  double h = patches[b].dx[0];
  for (int j = 1; j < dim; ++j) h = fmin(h, patches[b].dx[j]);
  patches[b].dt = cfl * h / ((double)dim * per_patch[b]);
}

}  // namespace

int launch_local_dt(fv_patch* patches, int64_t n, const double* per_patch, int dim, double cfl,
                    hipStream_t st) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks == 0) return 0;
  hipLaunchKernelGGL(local_dt_kernel, dim3((unsigned)blocks), dim3(256), 0, st, patches, n,
                     per_patch, dim, cfl);
  return 0;
}

template <typename T>
int launch_patch_max(const fv_patch* patches, int64_t n, const T* q, int64_t q_len, int q_halo,
                     int which, int dim, int p, double gamma, double* per_patch, hipStream_t st) {
#define FV_CASE(DD, PP)                                                                 \
  if (dim == DD && p == PP) {                                                           \
    launch_pm<T, DD, PP>(patches, n, q, q_len, q_halo, which, gamma, per_patch, st);    \
    return 0;                                                                           \
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

template <typename T>
int launch_totals(const fv_patch* patches, int64_t n, const T* q, int64_t q_len, int q_halo,
                  int which, int dim, int p, double* per_patch, double* totals, hipStream_t st) {
  int rc = FV_EUNSUPPORTED;
#define FV_CASE(DD, PP)                                                           \
  if (dim == DD && p == PP) {                                                     \
    launch_tot<T, DD, PP>(patches, n, q, q_len, q_halo, which, per_patch, st);    \
    rc = 0;                                                                       \
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
  if (rc == 0 && totals)
    hipLaunchKernelGGL(sum_patches_kernel, dim3(1), dim3(1024), 0, st, per_patch, n, dim + 2,
                       totals);
  return rc;
}

template int launch_patch_max<double>(const fv_patch*, int64_t, const double*, int64_t, int, int,
                                      int, int, double, double*, hipStream_t);
template int launch_patch_max<float>(const fv_patch*, int64_t, const float*, int64_t, int, int,
                                     int, int, double, double*, hipStream_t);
template int launch_totals<double>(const fv_patch*, int64_t, const double*, int64_t, int, int,
                                   int, int, double*, double*, hipStream_t);
template int launch_totals<float>(const fv_patch*, int64_t, const float*, int64_t, int, int, int,
                                  int, double*, double*, hipStream_t);

int launch_reduce_cfl(const fv_patch* patches, int64_t n, const double* per_patch, int dim,
                      double cfl, double* lambda_out, double* dt_out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_cfl_kernel, dim3(1), dim3(1024), 0, st, patches, n, per_patch, dim,
                     cfl, lambda_out, dt_out);
  return 0;
}

}  // namespace fvk
