// Learned face-flux correction, 2-D Euler: inference.  The per-face network
// (16 -> 64 -> 64 -> 4, tanh) runs on the matrix cores: one wave evaluates 64
// faces at a time, as two tiles of 32 faces, with three bfloat16 products per
// tile and float32 sums (v_mfma_f32_32x32x16_bf16; layer 1 is 2
// instructions per tile, layer 2 2 x 4, layer 3 4 with the four outputs
// padded to 32 rows).  The fused update keeps a patch of 16 x 16 volumes and
// its two-volume face halo in LDS, evaluates all 544 faces (Rusanov flux in
// float64 plus the correction), then updates every volume from its four face
// fluxes.
#include <hip/hip_ext.h>
#include <math.h>

#include <atomic>

#include "fv_euler.hpp"
#include "fv_internal.hpp"

namespace fvk {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kNF = 16, kNH = 64, kNO = 4;
constexpr int kXM = 0, kXS = 16, kW1 = 32, kB1 = kW1 + kNH * kNF, kW2 = kB1 + kNH,
              kB2 = kW2 + kNH * kNH, kW3 = kB2 + kNH, kB3 = kW3 + kNO * kNH, kYS = kB3 + kNO,
              kYM = kYS + kNO;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// Two float32 values as a pair of bfloat16 (round to nearest even, the
// hardware conversion; NaN stays NaN).
__device__ __forceinline__ bf16x2 to_bf16x2(float a, float b) {
  const floatx2 v = {a, b};
  return __builtin_convertvector(v, bf16x2);
}
__device__ __forceinline__ bf16x8 to_bf16x8(const float* v) {
  bf16x8 f;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const bf16x2 p = to_bf16x2(v[e], v[e + 1]);
    f[e] = p[0];
    f[e + 1] = p[1];
  }
  return f;
}

// tanh(x) = 1 - 2 / (exp(2x) + 1) from the hardware base-2 exponential and
// reciprocal, the last step one fused multiply-add (a few ulp of float32 away
// from the correctly rounded value for |tanh x| >= 1/2, a few 1e-8 absolute
// below; the result is rounded to bfloat16 next, 2^-9 relative).  Five
// instructions, two of them transcendental.  +-inf and large |x| give +-1,
// NaN stays NaN.
__device__ __forceinline__ float tanh_fast(float x) {
  const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);  // 2 / ln 2
  return __builtin_fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

// Matrix-core lane layout of the 32 x 32 x 16 product (wave64), lane
// l = 32 h + j: the lane holds A[j][8 h + e] and B[8 h + e][j] for e = 0..7,
// and accumulator register r holds C[8 (r / 4) + 4 h + r % 4][j].
//
// The network runs transposed, H^T = W X^T: units are rows, the 32 faces of a
// tile are columns, so face j stays in lanes j and 32 + j throughout.  The
// accumulator registers r = 8 q + e (e = 0..7) of the unit tile mt hold the
// units 32 mt + 16 q + 8 (e / 4) + 4 h + e % 4 of face j, which is the B
// operand of the next layer's k-step s = 2 mt + q once that layer's weight
// columns are taken in the order unit_of(s, h, e).  So the hidden layers
// never leave the registers.
__device__ __forceinline__ int unit_of(int s, int h, int e) {
  return 16 * s + 8 * (e >> 2) + 4 * h + (e & 3);
}

struct MlpFrags {
  bf16x8 w1[2];      // [unit tile]: W1[32 mt + j][8 h + e]
  bf16x8 w2[2][4];   // [unit tile][k step]: W2[32 mt + j][unit_of(s, h, e)]
  bf16x8 w3[4];      // [k step]: W3[j][unit_of(s, h, e)], rows j >= 4 zero
};

__device__ MlpFrags load_frags(const float* __restrict__ blob, int l) {
  MlpFrags F;
  const int j = l & 31, h = l >> 5;
  float v[8];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = blob[kW1 + (32 * mt + j) * kNF + 8 * h + e];
    F.w1[mt] = to_bf16x8(v);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = blob[kW2 + (32 * mt + j) * kNH + unit_of(ks, h, e)];
      F.w2[mt][ks] = to_bf16x8(v);
    }
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = j < kNO ? blob[kW3 + j * kNH + unit_of(ks, h, e)] : 0.0f;
    F.w3[ks] = to_bf16x8(v);
  }
  return F;
}

// The fragments of all 64 lanes as one table [14][64] of bfloat16 x 8 (w1[2],
// w2[2][4], w3[4]), built once per workgroup by all its threads (each lane
// fragment from 8 blob words), then read back by every wave: 896 fragment
// builds per workgroup instead of 14 per lane of every wave.
constexpr int kFrags = 14;
__device__ void stage_frags(const float* __restrict__ blob, bf16x8* table, int tid, int nthreads) {
  for (int i = tid; i < kFrags * 64; i += nthreads) {
    const int f = i >> 6, lane = i & 63;
    const int j = lane & 31, h = lane >> 5;
    float v[8];
    if (f < 2) {
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = blob[kW1 + (32 * f + j) * kNF + 8 * h + e];
    } else if (f < 10) {
      const int mt = (f - 2) >> 2, ks = (f - 2) & 3;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = blob[kW2 + (32 * mt + j) * kNH + unit_of(ks, h, e)];
    } else {
      const int ks = f - 10;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = j < kNO ? blob[kW3 + j * kNH + unit_of(ks, h, e)] : 0.0f;
    }
    table[i] = to_bf16x8(v);
  }
}

__device__ MlpFrags frags_from_table(const bf16x8* table, int l) {
  MlpFrags F;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    F.w1[mt] = table[mt * 64 + l];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) F.w2[mt][ks] = table[(2 + mt * 4 + ks) * 64 + l];
  }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) F.w3[ks] = table[(10 + ks) * 64 + l];
  return F;
}

// Biases in accumulator order, [unit tile][h][register]: a layer starts its
// sums from them.  One copy per workgroup, filled by fill_bias.
struct MlpBias {
  float b1[2][2][16];
  float b2[2][2][16];
  float b3[2][16];
};

__device__ void fill_bias(const float* __restrict__ blob, MlpBias& b, int tid, int nthreads) {
  for (int i = tid; i < 64; i += nthreads) {
    const int mt = i >> 5, h = (i >> 4) & 1, r = i & 15;
    const int u = 32 * mt + 8 * (r >> 2) + 4 * h + (r & 3);
    b.b1[mt][h][r] = blob[kB1 + u];
    b.b2[mt][h][r] = blob[kB2 + u];
    if (mt == 0) b.b3[h][r] = (h == 0 && r < kNO) ? blob[kB3 + r] : 0.0f;
  }
}

// Per-wave LDS of the network: the bfloat16 features of the 64 faces (the
// layer-1 operand of both tiles).  A face's 4 outputs are written over its
// first 16 bytes of features once its tile's layer-1 product has read them.
struct MlpLds {
  alignas(16) bf16x8 x[64][2];   // [face][feature / 8]
};
__device__ __forceinline__ float* mlp_out(MlpLds& s, int face) {
  return reinterpret_cast<float*>(&s.x[face][0]);
}

// tanh of an accumulator tile, packed as the two k-step operands of the next
// layer.
__device__ __forceinline__ void tanh_pack(const floatx16& c, bf16x8& k0, bf16x8& k1) {
  float t[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) t[r] = tanh_fast(c[r]);
  k0 = to_bf16x8(t);
  k1 = to_bf16x8(t + 8);
}

// The network on the 64 faces of this wave: lane l holds the normalised
// features xh[16] of face l and receives its outputs o[4].  Wave-local: the
// LDS traffic of one wave is ordered, so no workgroup barrier is needed.
// tiles: 2, or 1 when faces 32..63 are not needed (their o values are then
// meaningless); the same on every lane of the wave.
__device__ void mlp64(const MlpFrags& F, const MlpBias& B, MlpLds& s, int l,
                      const float (&xh)[kNF], float (&o)[kNO], int tiles = 2) {
  const int j = l & 31, h = l >> 5;
  s.x[l][0] = to_bf16x8(xh);
  s.x[l][1] = to_bf16x8(xh + 8);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    if (t >= tiles) break;
    const bf16x8 xt = s.x[32 * t + j][h];  // X^T tile: features 8 h + e of face 32 t + j
    bf16x8 h1[4], h2[4];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      floatx16 c = *reinterpret_cast<const floatx16*>(B.b1[mt][h]);
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.w1[mt], xt, c, 0, 0, 0);
      tanh_pack(c, h1[2 * mt], h1[2 * mt + 1]);
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      floatx16 c = *reinterpret_cast<const floatx16*>(B.b2[mt][h]);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.w2[mt][ks], h1[ks], c, 0, 0, 0);
      tanh_pack(c, h2[2 * mt], h2[2 * mt + 1]);
    }
    floatx16 c = *reinterpret_cast<const floatx16*>(B.b3[h]);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(F.w3[ks], h2[ks], c, 0, 0, 0);
    // rows 0..3 = the outputs of face 32 t + j, over its features (read by
    // this tile's layer-1 product above, in program order; the fence keeps
    // the compiler from moving the store above that read)
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (h == 0) {
      float* op = mlp_out(s, 32 * t + j);
#pragma unroll
      for (int m = 0; m < kNO; ++m) op[m] = c[m];
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  {
    const float* op = mlp_out(s, l);
#pragma unroll
    for (int m = 0; m < kNO; ++m) o[m] = op[m];
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Network outputs for raw feature rows (one wave per 64 rows).
__global__ void __launch_bounds__(64)
mlp_forward_kernel(const float* __restrict__ blob, const float* __restrict__ feats, int64_t n,
                   float* __restrict__ out) {
  __shared__ MlpLds s;
  __shared__ MlpBias bias;
  const int l = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * 64 + l;
  fill_bias(blob, bias, l, 64);
  __syncthreads();
  const MlpFrags F = load_frags(blob, l);
  const int64_t rr = row < n ? row : n - 1;
  float xh[kNF], o[kNO];
#pragma unroll
  for (int k = 0; k < kNF; ++k) xh[k] = (feats[rr * kNF + k] - blob[kXM + k]) * blob[kXS + k];
  mlp64(F, bias, s, l, xh, o);
  if (row < n) {
#pragma unroll
    for (int m = 0; m < kNO; ++m) out[row * kNO + m] = o[m];
  }
}

// ---------------------------------------------------------------------------
// Fused update of 2-D patches of 16 x 16 volumes with corrected fluxes.
// ---------------------------------------------------------------------------
constexpr int kP = 16, kH = 2, kW = kP + 2 * kH;  // volumes per axis with the halo
constexpr int kNXF = (kP + 1) * kP;              // x faces (= y faces) per patch
constexpr int kNFACE = 2 * kNXF;                 // 544
constexpr int kVolThreads = kP * kP;  // one thread per volume in the update
// Workgroup size: NTH threads (4 or 8 waves) share the 9 face batches.  Eight
// waves shorten a patch's face phase (at most 1.5 batches per wave instead of
// 2.5) for small launches; four waves fit three workgroups per CU for large
// ones.
template <int NTH>
struct PatchLds {
  double q[4][kW][kW];        // state with a two-volume face halo (corners unused)
  union {
    struct {
      double fx[4][kP][kP + 1];   // x-face fluxes [m][y][face x]
      double fy[4][kP + 1][kP];   // y-face fluxes [m][face y][x]
    };
    bf16x8 frags[kFrags * 64];  // network fragments, read by every wave before any flux
  };
  double red[NTH / 64];
  MlpBias bias;
  MlpLds mlp[NTH / 64];
};

// Four-wave workgroups: 39 KB of LDS lets four of them share a CU, and at
// most 128 registers per thread lets their 16 waves be resident together
// (4 per SIMD instead of 3).  Eight-wave workgroups run one per CU.
template <int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(NTH == 256 ? 4 : 2)))
learned_update_kernel(const fv_patch* __restrict__ patches, int64_t n,
                      const int64_t* __restrict__ neighbours, const double* __restrict__ qin,
                      int64_t qin_len, double* __restrict__ qout, int64_t qout_len,
                      double gamma, const double* __restrict__ dt_dev,
                      const float* __restrict__ blob, double threshold,
                      double* __restrict__ max_eig) {
  __shared__ PatchLds<NTH> s;
  const int tid = threadIdx.x, wave = tid >> 6, l = tid & 63;
  const int64_t b = blockIdx.x;
  constexpr int64_t blk = 4 * kP * kP;
  // descriptor and neighbour checks (the same in every thread)
  const fv_patch pd = patches[b];
  bool ok = pd.p == kP && pd.q_in >= 0 && pd.q_in <= qin_len - blk && pd.q_out >= 0 &&
            pd.q_out <= qout_len - blk;
  // the neighbour row, then the neighbours' descriptors, each as one batch
  // of independent loads (an index outside [0, n) reads the own descriptor
  // and is judged below, without branches)
  int64_t nbi[4], nq[4], nbo[4];
  int np[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) nbi[f] = neighbours[b * 4 + f];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int64_t c = (nbi[f] >= 0 && nbi[f] < n) ? nbi[f] : b;
    nq[f] = patches[c].q_in;
    np[f] = patches[c].p;
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int64_t nb = nbi[f];
    const bool inr = (nb >= 0) & (nb < n);
    const bool good = (np[f] == kP) & (nq[f] >= 0) & (nq[f] <= qin_len - blk);
    nbo[f] = (inr & good) ? nq[f] : -1;
    ok = ok & (inr ? good : nb == -1);
  }
  if (!ok) {
    if (tid == 0 && max_eig) max_eig[b] = __builtin_nan("");
    return;  // uniform: the whole workgroup leaves
  }
  const double dt = dt_dev ? *dt_dev : pd.dt;
  const double rx = dt / pd.dx[0], ry = dt / pd.dx[1];

  // ---- state and face halo into LDS --------------------------------------
  if (tid < kVolThreads) {
    const int x = tid & 15, y = tid >> 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) s.q[m][y + kH][x + kH] = qin[pd.q_in + m * kP * kP + y * kP + x];
  }
  if (tid < 128) {
    // halo volume: side (-x, +x, -y, +y) and 32 per side (2 layers x 16)
    const int side = tid >> 5, t = tid & 31, layer = t >> 4, pos = t & 15;
    int hx, hy, sx, sy;  // LDS coordinates and source coordinates in the source block
    int64_t src = pd.q_in;
    if (side == 0) {        // x = -2 + layer
      hx = layer; hy = pos + kH;
      sx = nbo[0] >= 0 ? kP - 2 + layer : 0; sy = pos;
      if (nbo[0] >= 0) src = nbo[0];
    } else if (side == 1) { // x = 16 + layer
      hx = kP + kH + layer; hy = pos + kH;
      sx = nbo[1] >= 0 ? layer : kP - 1; sy = pos;
      if (nbo[1] >= 0) src = nbo[1];
    } else if (side == 2) { // y = -2 + layer
      hx = pos + kH; hy = layer;
      sx = pos; sy = nbo[2] >= 0 ? kP - 2 + layer : 0;
      if (nbo[2] >= 0) src = nbo[2];
    } else {                // y = 16 + layer
      hx = pos + kH; hy = kP + kH + layer;
      sx = pos; sy = nbo[3] >= 0 ? layer : kP - 1;
      if (nbo[3] >= 0) src = nbo[3];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) s.q[m][hy][hx] = qin[src + m * kP * kP + sy * kP + sx];
  }
  fill_bias(blob, s.bias, tid, NTH);
  stage_frags(blob, s.frags, tid, NTH);
  __syncthreads();
  const MlpFrags F = frags_from_table(s.frags, l);
  __syncthreads();  // the flux buffers reuse the fragment table

  // ---- faces: 9 batches of 64 over the NTH / 64 waves ---------------------
  for (int batch = wave; batch * 64 < kNFACE; batch += NTH / 64) {
    const int f = batch * 64 + l;
    const bool real = f < kNFACE;
    const int ff = real ? f : kNFACE - 1;
    const bool xdir = ff < kNXF;
    const int g = xdir ? ff : ff - kNXF;
    // face between volumes (i-1) and i along the normal; (fi, fj) in LDS
    int I, J;
    if (xdir) { I = g % (kP + 1); J = g / (kP + 1); }
    else { I = g % kP; J = g / kP; }
    double v[4][4];  // stencil volumes -2..+1, grid-axis components
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const int cx = xdir ? I - 2 + o + kH : I + kH;
      const int cy = xdir ? J + kH : J - 2 + o + kH;
#pragma unroll
      for (int m = 0; m < 4; ++m) v[o][m] = s.q[m][cy][cx];
    }
    float xh[kNF];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      const double fr[4] = {v[o][0], xdir ? v[o][1] : v[o][2], xdir ? v[o][2] : v[o][1], v[o][3]};
#pragma unroll
      for (int c = 0; c < 4; ++c)
        xh[4 * o + c] = ((float)fr[c] - blob[kXM + 4 * o + c]) * blob[kXS + 4 * o + c];
    }
    float out[kNO];
    // the last batch holds 544 - 8 * 64 = 32 faces: one tile of the network
    mlp64(F, s.bias, s.mlp[wave], l, xh, out, (batch + 1) * 64 <= kNFACE ? 2 : 1);
    // plain flux of the face, grid axes
    double Fr[4];
    {
      const Prim<double> wl = decode<double, 2>(v[1], gamma);
      const Prim<double> wr = decode<double, 2>(v[2], gamma);
      if (xdir) rusanov<double, 2, 0>(v[1], wl, v[2], wr, Fr);
      else rusanov<double, 2, 1>(v[1], wl, v[2], wr, Fr);
    }
    const double ind = fabs(v[2][0] - v[1][0]) / fmin(v[1][0], v[2][0]);
    const bool corr = !(ind > threshold);
    double dfr[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) dfr[c] = corr ? (double)(out[c] * blob[kYS + c] + blob[kYM + c]) : 0.0;
    const double dF[4] = {dfr[0], xdir ? dfr[1] : dfr[2], xdir ? dfr[2] : dfr[1], dfr[3]};
    if (real) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double flux = 0.5 * Fr[m] + dF[m];  // rusanov gives 2F
        if (xdir) s.fx[m][J][I] = flux;
        else s.fy[m][J][I] = flux;
      }
    }
  }
  __syncthreads();

  // ---- update, new-state maximum ----------------------------------------
  double lam = 0.0;  // threads past the volumes contribute nothing
  if (tid < kVolThreads) {
    const int x = tid & 15, y = tid >> 4;
    double qn[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      double v = s.q[m][y + kH][x + kH] - rx * (s.fx[m][y][x + 1] - s.fx[m][y][x]);
      v = v - ry * (s.fy[m][y + 1][x] - s.fy[m][y][x]);
      qn[m] = v;
      qout[pd.q_out + m * kP * kP + y * kP + x] = v;
    }
    const Prim<double> wn = decode<double, 2>(qn, gamma);
    lam = max_wave_speed<double, 2>(qn, wn);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) lam = nanmax_pos(lam, __shfl_xor(lam, o, 64));
  if (l == 0) s.red[wave] = lam;
  __syncthreads();
  if (tid == 0 && max_eig) {
    double mx = s.red[0];
    for (int w = 1; w < NTH / 64; ++w) mx = nanmax_pos(mx, s.red[w]);
    max_eig[b] = mx;
  }
}

}  // namespace

int launch_mlp_forward(const float* blob, const float* feats, int64_t n, float* out,
                       hipStream_t st) {
  const int64_t blocks = (n + 63) / 64;
  if (blocks == 0) return 0;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(64), 0, st, blob, feats, n,
                     out);
  return 0;
}

int launch_update_learned_2d(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                             const double* qin, int64_t qin_len, double* qout, int64_t qout_len,
                             double gamma, const double* dt_dev, const float* blob,
                             double threshold, double* max_eig, hipStream_t st) {
  if (n == 0) return 0;
  const LaunchEvents& ev = launch_events();
  // eight waves per patch while every patch has a CU of its own
  const int cus = device_cu_count();
  if (n <= cus)
    hipExtLaunchKernelGGL(learned_update_kernel<512>, dim3((unsigned)n), dim3(512), 0, st,
                          ev.start, ev.stop, 0, patches, n, neighbours, qin, qin_len, qout,
                          qout_len, gamma, dt_dev, blob, threshold, max_eig);
  else
    hipExtLaunchKernelGGL(learned_update_kernel<256>, dim3((unsigned)n), dim3(256), 0, st,
                          ev.start, ev.stop, 0, patches, n, neighbours, qin, qin_len, qout,
                          qout_len, gamma, dt_dev, blob, threshold, max_eig);
  return 0;
}

}  // namespace fvk
