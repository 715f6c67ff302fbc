// Learned face-flux correction, 2-D Euler: training-data and training kernels.
//
// Training data come from runs on a grid r times finer than the one the
// correction serves (r = 4): the fine state is coarse-grained conservatively
// (r x r averages), the fine Rusanov fluxes through the r fine faces that
// make up each coarse face are averaged over those faces and over the r fine
// steps of one coarse step, and the target of a coarse face is that average
// minus the coarse Rusanov flux, in the face frame (rho, j_n, j_t, E).  The
// network (16 -> 64 -> 64 -> 4, tanh) is trained in float32 by minibatch
// Adam on the mean-squared error of normalised targets; every reduction runs
// in a fixed order, so training is deterministic.
//
// Grids here are regular patch grids: npx x npy patches of p x p volumes,
// compact blocks [4][p][p] back to back in patch-lexicographic order (x
// fastest).  Boundaries: periodic or transmissive (zero gradient).
#include <math.h>

#include "fv_euler.hpp"
#include "fv_internal.hpp"

namespace fvk {

namespace {

constexpr int kS2 = 4;  // unknowns in 2-D

struct Grid2 {
  int npx, npy, p, bc;  // bc: 0 periodic, 1 transmissive
  __device__ int nx() const { return npx * p; }
  __device__ int ny() const { return npy * p; }
  // element index of unknown m of volume (gx, gy), boundary applied
  __device__ int64_t at(int gx, int gy, int m) const {
    const int NX = nx(), NY = ny();
    if (bc == 0) {
      gx = (gx % NX + NX) % NX;
      gy = (gy % NY + NY) % NY;
    } else {
      gx = gx < 0 ? 0 : (gx >= NX ? NX - 1 : gx);
      gy = gy < 0 ? 0 : (gy >= NY ? NY - 1 : gy);
    }
    const int px = gx / p, py = gy / p;
    const int64_t patch = (int64_t)py * npx + px;
    return patch * kS2 * p * p + (int64_t)m * p * p + (int64_t)(gy - py * p) * p + (gx - px * p);
  }
  __device__ void load(const double* q, int gx, int gy, double (&v)[kS2]) const {
#pragma unroll
    for (int m = 0; m < kS2; ++m) v[m] = q[at(gx, gy, m)];
  }
};

// Rusanov flux across a face with normal along axis k, in grid axes.
__device__ void face_flux(const double (&L)[kS2], const double (&R)[kS2], int k, double gamma,
                          double (&F)[kS2]) {
  const Prim<double> wl = decode<double, 2>(L, gamma);
  const Prim<double> wr = decode<double, 2>(R, gamma);
  if (k == 0) {
    rusanov<double, 2, 0>(L, wl, R, wr, F);
  } else {
    rusanov<double, 2, 1>(L, wl, R, wr, F);
  }
#pragma unroll
  for (int m = 0; m < kS2; ++m) F[m] *= 0.5;  // rusanov gives 2F
}

// acc += weight * (mean over the r fine faces of each coarse face of the fine
// Rusanov flux).  One thread per coarse face: x faces [ncy][ncx + 1], then y
// faces [ncy + 1][ncx].
__global__ void __launch_bounds__(256)
face_flux_accumulate_kernel(const double* __restrict__ qf, Grid2 g, int r, double gamma,
                            double weight, double* __restrict__ accx, double* __restrict__ accy) {
  const int ncx = g.nx() / r, ncy = g.ny() / r;
  const int64_t nxf = (int64_t)ncy * (ncx + 1), nyf = (int64_t)(ncy + 1) * ncx;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxf + nyf) return;
  const bool xdir = t < nxf;
  const int64_t f = xdir ? t : t - nxf;
  const int cols = xdir ? ncx + 1 : ncx;
  const int I = (int)(f % cols), J = (int)(f / cols);
  double sum[kS2] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < r; ++s) {
    double L[kS2], R[kS2], F[kS2];
    if (xdir) {
      g.load(qf, r * I - 1, r * J + s, L);
      g.load(qf, r * I, r * J + s, R);
    } else {
      g.load(qf, r * I + s, r * J - 1, L);
      g.load(qf, r * I + s, r * J, R);
    }
    face_flux(L, R, xdir ? 0 : 1, gamma, F);
#pragma unroll
    for (int m = 0; m < kS2; ++m) sum[m] += F[m];
  }
  double* acc = xdir ? accx : accy;
  const int64_t plane = xdir ? nxf : nyf;
#pragma unroll
  for (int m = 0; m < kS2; ++m) acc[m * plane + f] += weight * (sum[m] / r);
}

// Coarse volume = mean of its r x r fine volumes (row-major sum).  The coarse
// grid is a regular patch grid of the same p with npx / r x npy / r patches.
__global__ void __launch_bounds__(256)
coarse_grain_kernel(const double* __restrict__ qf, Grid2 g, int r, double* __restrict__ qc) {
  const Grid2 c{g.npx / r, g.npy / r, g.p, g.bc};
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nvol = (int64_t)c.nx() * c.ny();
  if (t >= nvol) return;
  const int I = (int)(t % c.nx()), J = (int)(t / c.nx());
#pragma unroll
  for (int m = 0; m < kS2; ++m) {
    double s = 0.0;
    for (int b = 0; b < r; ++b)
      for (int a = 0; a < r; ++a) s += qf[g.at(r * I + a, r * J + b, m)];
    qc[c.at(I, J, m)] = s / (double)(r * r);
  }
}

// Samples of every coarse face (x faces then y faces, row-major): features =
// the 4-volume stencil in the face frame, target = face-frame difference
// between the accumulated reference flux and the coarse Rusanov flux,
// indicator = |rho_R - rho_L| / min(rho_L, rho_R).
__global__ void __launch_bounds__(256)
face_samples_kernel(const double* __restrict__ qc, Grid2 g, double gamma,
                    const double* __restrict__ accx, const double* __restrict__ accy,
                    float* __restrict__ feats, float* __restrict__ targ, float* __restrict__ ind) {
  const int ncx = g.nx(), ncy = g.ny();
  const int64_t nxf = (int64_t)ncy * (ncx + 1), nyf = (int64_t)(ncy + 1) * ncx;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxf + nyf) return;
  const bool xdir = t < nxf;
  const int64_t f = xdir ? t : t - nxf;
  const int cols = xdir ? ncx + 1 : ncx;
  const int I = (int)(f % cols), J = (int)(f / cols);
  const int k = xdir ? 0 : 1;
  double v[4][kS2];
  for (int o = 0; o < 4; ++o) {
    if (xdir) g.load(qc, I - 2 + o, J, v[o]);
    else g.load(qc, I, J - 2 + o, v[o]);
  }
  const int tn = 1 + k, tt = 2 - k;  // face-frame components
  for (int o = 0; o < 4; ++o) {
    feats[t * 16 + 4 * o + 0] = (float)v[o][0];
    feats[t * 16 + 4 * o + 1] = (float)v[o][tn];
    feats[t * 16 + 4 * o + 2] = (float)v[o][tt];
    feats[t * 16 + 4 * o + 3] = (float)v[o][3];
  }
  double F[kS2];
  face_flux(v[1], v[2], k, gamma, F);
  const double* acc = xdir ? accx : accy;
  const int64_t plane = xdir ? nxf : nyf;
  double d[kS2];
#pragma unroll
  for (int m = 0; m < kS2; ++m) d[m] = acc[m * plane + f] - F[m];
  targ[t * 4 + 0] = (float)d[0];
  targ[t * 4 + 1] = (float)d[tn];
  targ[t * 4 + 2] = (float)d[tt];
  targ[t * 4 + 3] = (float)d[3];
  ind[t] = (float)(fabs(v[2][0] - v[1][0]) / fmin(v[1][0], v[2][0]));
}

// Per-column mean and spread of x[n][cols] (one workgroup per column, fixed
// order, float64 sums).  mode 0: out_scale = 1 / std (feature normalisation);
// mode 1: out_scale = std (target de-normalisation).  std is floored at
// 1e-12 of the column's largest magnitude (and 1e-30).
__global__ void __launch_bounds__(256)
column_stats_kernel(const float* __restrict__ x, int64_t x_rows, int64_t n, int cols, int mode,
                    const int64_t* __restrict__ rows, float* __restrict__ out_mean,
                    float* __restrict__ out_scale) {
  __shared__ double red[256];
  __shared__ double red2[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0, mx = 0.0;
  for (int64_t i = t; i < n; i += 256) {
    const int64_t r = rows ? rows[i] : i;
    const double v = (r >= 0 && r < x_rows) ? x[r * cols + c] : 0.0;
    s += v;
    mx = fmax(mx, fabs(v));
  }
  red[t] = s;
  red2[t] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      red[t] += red[t + w];
      red2[t] = fmax(red2[t], red2[t + w]);
    }
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  const double amax = red2[0];
  __syncthreads();
  double q = 0.0;
  for (int64_t i = t; i < n; i += 256) {
    const int64_t r = rows ? rows[i] : i;
    const double v = ((r >= 0 && r < x_rows) ? x[r * cols + c] : 0.0) - mean;
    q += v * v;
  }
  red[t] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) {
    double sd = sqrt(red[0] / (double)n);
    sd = fmax(sd, fmax(1e-12 * amax, 1e-30));
    out_mean[c] = (float)mean;
    out_scale[c] = (float)(mode == 0 ? 1.0 / sd : sd);
  }
}

// ---------------------------------------------------------------------------
// Training.  Blob offsets (float32 words) of the parameter layout.
// ---------------------------------------------------------------------------
constexpr int kNF = 16, kNH = 64, kNO = 4;
constexpr int kXM = 0, kXS = 16, kW1 = 32, kB1 = kW1 + kNH * kNF, kW2 = kB1 + kNH,
              kB2 = kW2 + kNH * kNH, kW3 = kB2 + kNH, kB3 = kW3 + kNO * kNH, kYS = kB3 + kNO,
              kYM = kYS + kNO, kBlob = kYM + kNO;
static_assert(kBlob == 5548, "parameter blob layout");
constexpr int kTrain0 = kW1, kTrainN = kYS - kW1;  // trained words: W1 .. b3
static_assert(kTrainN == FV_MLP_TRAINED_WORDS, "trained words");
// workspace, field-major: field f of sample b at f * batch + b; fields x_hat[16],
// h1[64], h2[64], d1[64], d2[64], dout[4], loss (the last batch words: the
// per-sample mean squared error)
constexpr int kWs = kNF + 4 * kNH + kNO + 1;

// Forward and backward of one sample per 64-thread workgroup (float32).
__global__ void __launch_bounds__(64)
mlp_sample_kernel(const float* __restrict__ blob, const float* __restrict__ feats,
                  const float* __restrict__ targ, int64_t n_rows,
                  const int64_t* __restrict__ idx, int batch, float* __restrict__ ws) {
  __shared__ float xs[kNF], h1[kNH], h2[kNH], d2[kNH], dout[kNO];
  const int b = blockIdx.x, j = threadIdx.x;
  // a row index outside the data contributes nothing (zero residual)
  const int64_t row0 = idx[b];
  const bool valid = row0 >= 0 && row0 < n_rows;
  const int64_t row = valid ? row0 : 0;
  float* w = ws + b;  // field f at w[f * batch]
  if (j < kNF) {
    const float xh = (feats[row * kNF + j] - blob[kXM + j]) * blob[kXS + j];
    xs[j] = xh;
    w[(int64_t)j * batch] = xh;
  }
  __syncthreads();
  float a = blob[kB1 + j];
  for (int k = 0; k < kNF; ++k) a = fmaf(blob[kW1 + j * kNF + k], xs[k], a);
  const float v1 = tanhf(a);
  h1[j] = v1;
  __syncthreads();
  a = blob[kB2 + j];
  for (int k = 0; k < kNH; ++k) a = fmaf(blob[kW2 + j * kNH + k], h1[k], a);
  const float v2 = tanhf(a);
  h2[j] = v2;
  __syncthreads();
  if (j < kNO) {
    float o = blob[kB3 + j];
    for (int k = 0; k < kNH; ++k) o = fmaf(blob[kW3 + j * kNH + k], h2[k], o);
    const float y = (targ[row * kNO + j] - blob[kYM + j]) / blob[kYS + j];
    const float e = valid ? o - y : 0.0f;
    dout[j] = 2.0f * e / (float)(batch * kNO);
    w[(int64_t)(kNF + 4 * kNH + j) * batch] = dout[j];
    xs[j] = e * e;  // per-output squared error (xs no longer needed)
  }
  __syncthreads();
  if (j == 0) w[(int64_t)(kNF + 4 * kNH + kNO) * batch] = (xs[0] + xs[1] + xs[2] + xs[3]) / (float)kNO;
  float g = 0.0f;
  for (int m = 0; m < kNO; ++m) g = fmaf(dout[m], blob[kW3 + m * kNH + j], g);
  const float dd2 = g * (1.0f - v2 * v2);
  d2[j] = dd2;
  __syncthreads();
  g = 0.0f;
  for (int i = 0; i < kNH; ++i) g = fmaf(d2[i], blob[kW2 + i * kNH + j], g);
  const float dd1 = g * (1.0f - v1 * v1);
  w[(int64_t)(kNF + j) * batch] = v1;
  w[(int64_t)(kNF + kNH + j) * batch] = v2;
  w[(int64_t)(kNF + 2 * kNH + j) * batch] = dd1;
  w[(int64_t)(kNF + 3 * kNH + j) * batch] = dd2;
}

// Gradient of one trained word per wave and its Adam step (Kingma and Ba,
// 2015; beta1 0.9, beta2 0.999, eps 1e-8).  Lane i sums the samples i, i + 64,
// ... in order, then a fixed butterfly across the wave adds the 64 partial
// sums: the same order on every call, so training is deterministic.
constexpr int kAdamWaves = 4;  // words per 256-thread workgroup
__global__ void __launch_bounds__(64 * kAdamWaves)
mlp_adam_kernel(float* __restrict__ blob, float* __restrict__ adam, int step, float lr,
                const float* __restrict__ ws, int batch, float* __restrict__ grad_out) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * kAdamWaves + (threadIdx.x >> 6);  // the same in the whole wave
  if (t >= kTrainN) return;
  const int word = kTrain0 + t;
  // which parameter: (source a, source b) offsets inside a sample's workspace
  int oa, ob;  // g = sum_b ws[oa] * ws[ob] (ob < 0: factor 1)
  if (word < kB1) {
    const int jj = (word - kW1) / kNF, k = (word - kW1) % kNF;
    oa = kNF + 2 * kNH + jj;  // d1[j]
    ob = k;                   // x_hat[k]
  } else if (word < kW2) {
    oa = kNF + 2 * kNH + (word - kB1);
    ob = -1;
  } else if (word < kB2) {
    const int i = (word - kW2) / kNH, k = (word - kW2) % kNH;
    oa = kNF + 3 * kNH + i;  // d2[i]
    ob = kNF + k;            // h1[k]
  } else if (word < kW3) {
    oa = kNF + 3 * kNH + (word - kB2);
    ob = -1;
  } else if (word < kB3) {
    const int m = (word - kW3) / kNH, k = (word - kW3) % kNH;
    oa = kNF + 4 * kNH + m;  // dout[m]
    ob = kNF + kNH + k;      // h2[k]
  } else {
    oa = kNF + 4 * kNH + (word - kB3);
    ob = -1;
  }
  // field-major workspace: the lanes read consecutive samples
  const float* wa = ws + (int64_t)oa * batch;
  const float* wb = ob < 0 ? nullptr : ws + (int64_t)ob * batch;
  float g = 0.0f;
  for (int b = lane; b < batch; b += 64) g = fmaf(wa[b], wb ? wb[b] : 1.0f, g);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o, 64);
  if (lane != 0) return;
  if (grad_out) grad_out[t] = g;
  float* m = adam;
  float* v = adam + kTrainN;
  const float mt = 0.9f * m[t] + 0.1f * g;
  const float vt = 0.999f * v[t] + 0.001f * g * g;
  m[t] = mt;
  v[t] = vt;
  const float mh = mt / (1.0f - powf(0.9f, (float)step));
  const float vh = vt / (1.0f - powf(0.999f, (float)step));
  blob[word] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

}  // namespace

int launch_face_flux_accumulate(const double* qf, int npx, int npy, int p, int r, int bc,
                                double gamma, double weight, double* accx, double* accy,
                                hipStream_t st) {
  const Grid2 g{npx, npy, p, bc};
  const int64_t ncx = (int64_t)npx * p / r, ncy = (int64_t)npy * p / r;
  const int64_t n = ncy * (ncx + 1) + (ncy + 1) * ncx;
  hipLaunchKernelGGL(face_flux_accumulate_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     st, qf, g, r, gamma, weight, accx, accy);
  return 0;
}

int launch_coarse_grain(const double* qf, int npx, int npy, int p, int r, double* qc,
                        hipStream_t st) {
  const Grid2 g{npx, npy, p, 0};
  const int64_t n = (int64_t)(npx / r) * p * (int64_t)(npy / r) * p;
  hipLaunchKernelGGL(coarse_grain_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, qf,
                     g, r, qc);
  return 0;
}

int launch_face_samples(const double* qc, int npx, int npy, int p, int bc, double gamma,
                        const double* accx, const double* accy, float* feats, float* targ,
                        float* ind, hipStream_t st) {
  const Grid2 g{npx, npy, p, bc};
  const int64_t ncx = (int64_t)npx * p, ncy = (int64_t)npy * p;
  const int64_t n = ncy * (ncx + 1) + (ncy + 1) * ncx;
  hipLaunchKernelGGL(face_samples_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, qc,
                     g, gamma, accx, accy, feats, targ, ind);
  return 0;
}

int launch_column_stats(const float* x, int64_t x_rows, int64_t n, int cols, int mode,
                        const int64_t* rows, float* mean, float* scale, hipStream_t st) {
  hipLaunchKernelGGL(column_stats_kernel, dim3(cols), dim3(256), 0, st, x, x_rows, n, cols, mode,
                     rows, mean, scale);
  return 0;
}

int mlp_blob_words() { return kBlob; }
int mlp_trained_words() { return kTrainN; }
int mlp_workspace_words(int batch) { return batch * kWs; }

int launch_mlp_train_step(float* blob, float* adam, int step, float lr, const float* feats,
                          const float* targ, int64_t n_rows, const int64_t* idx, int batch,
                          float* ws, float* grad_out, hipStream_t st) {
  hipLaunchKernelGGL(mlp_sample_kernel, dim3(batch), dim3(64), 0, st, blob, feats, targ, n_rows,
                     idx, batch, ws);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kTrainN + kAdamWaves - 1) / kAdamWaves),
                     dim3(64 * kAdamWaves), 0, st, blob, adam, step, lr, ws, batch, grad_out);
  return 0;
}

}  // namespace fvk
