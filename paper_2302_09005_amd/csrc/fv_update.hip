// Plane-marching batched patch update for gfx950 (Section 2 eqs. (3)-(5) and
// Algorithm 1 of arXiv 2302.09005).
//
// Mapping.  A patch of P^D volumes is swept along its last axis ("marching
// axis": z in 3-D, y in 2-D).  Lane l of the patch owns the column of volumes
// at in-plane position l and walks it plane by plane, so every global load
// and store is a whole plane of one unknown: contiguous rows of P elements,
// unit stride across lanes (coalesced SoA traffic).  A 3-D 8^3 patch is one
// wave64; smaller cross-sections pack several patches into one wave, larger
// ones span several waves of one workgroup.
//
// Per plane:
//   A. each lane publishes its volume (q, 1/rho, p, c) to LDS; lanes
//      l < RING also load, decode and publish one face-halo volume of the
//      plane ("ring"), so halo volumes are decoded once;
//   B. each lane computes the in-plane faces on its low side; lanes
//      l < NEXTRA compute the faces on the patch's high boundary;
//   C. the face fluxes go to LDS (the plane buffer is reused);
//   D. each lane reads the flux of its high-side faces (computed by the
//      neighbouring lane), computes the marching-axis face above its volume
//      in registers (the one below is carried from the previous plane),
//      applies the explicit Euler update in axis order x, y, z, stores it and
//      folds max_j(|u_j| + c) of the new state into a running maximum.
// Every face flux is therefore evaluated exactly once.  The next plane's
// volume and ring loads are issued one plane ahead, before the LDS phases,
// so HBM latency overlaps the arithmetic of the current plane.
//
// The per-patch maximum is reduced across the patch's lanes with wave
// shuffles (and LDS across waves when a patch spans several waves).
#include "fv_euler.hpp"
#include "fv_internal.hpp"

namespace fvk {

namespace {

template <typename T, int D, int P>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, Geo<D, P>::NT)))
fv_update_kernel(const fv_patch* __restrict__ patches, int64_t n,
                 const T* __restrict__ qin, int64_t qin_len,
                 T* __restrict__ qout, int64_t qout_len, int out_halo, T gamma,
                 const double* __restrict__ dt_dev, double* __restrict__ max_eig) {
  using G = Geo<D, P>;
  constexpr int S = G::S;
  constexpr int K = D - 1;  // marching axis
  constexpr int W = G::W;
  constexpr int LANES = G::LANES;
  constexpr int NCELL = G::NCELL;
  constexpr int NF = G::NF;

  __shared__ T lds[G::PPW * G::SLOT];
  __shared__ T red[G::NT / 64];

  const int tid = threadIdx.x;
  const int slot = tid / LANES;
  const int l = tid - slot * LANES;
  const int64_t b = (int64_t)blockIdx.x * G::PPW + slot;
  const bool in_range = (slot < G::PPW) && (b < n);
  const int x = l % P;
  const int y = (D == 3) ? l / P : 0;

  // ---- descriptor and device-side bounds check --------------------------
  int64_t off_in = 0, off_out = 0;
  T r[3] = {T(0), T(0), T(0)};
  bool ok = false;
  if (in_range) {
    const fv_patch pd = patches[b];
    off_in = pd.q_in;
    off_out = pd.q_out;
    const int64_t blk_in = (int64_t)S * G::VIN;
    const int64_t blk_out = out_halo ? (int64_t)S * G::VIN : (int64_t)S * G::VOUT;
    ok = pd.p == P && off_in >= 0 && off_in <= qin_len - blk_in && off_out >= 0 &&
         off_out <= qout_len - blk_out;
    const double dt = dt_dev ? *dt_dev : pd.dt;
#pragma unroll
    for (int j = 0; j < D; ++j) r[j] = T(dt / pd.dx[j]);
  }
  T* cell = lds + (ok ? slot * G::SLOT : 0);  // plane buffer [NV][NCELL]
  T* face = cell;                             // face buffer [D-1][S][NF], same storage

  // own column (halo'd in-plane index), ring volume, output column
  const int in_col = (x + 1) + (D == 3 ? (y + 1) * W : 0);
  const bool has_ring = l < G::RING;
  int ring_col = 0;
  if (D == 3) {
    const int q4 = l / P, rr = l - q4 * P;
    ring_col = q4 == 0 ? (rr + 1) * W
             : q4 == 1 ? (P + 1) + (rr + 1) * W
             : q4 == 2 ? (rr + 1)
                       : (rr + 1) + (P + 1) * W;
  } else {
    ring_col = l == 0 ? 0 : P + 1;
  }
  const T* col = qin + off_in + in_col;
  const T* ring = qin + off_in + ring_col;
  const int64_t ostride = out_halo ? G::SM : G::SMO;
  const int64_t ocomp = out_halo ? G::VIN : G::VOUT;
  T* outp = qout + off_out +
            (out_halo ? (int64_t)in_col + G::SM : (int64_t)x + (D == 3 ? y * P : 0));

  // ---- prologue: planes -1 and 0, first marching-axis face ---------------
  T qlo[S], qc[S], qnx[S], rraw[S];
#pragma unroll
  for (int m = 0; m < S; ++m) {
    qlo[m] = T(0);
    qc[m] = T(1);
    qnx[m] = T(1);
    rraw[m] = T(1);
  }
  if (ok) {
#pragma unroll
    for (int m = 0; m < S; ++m) {
      qlo[m] = col[(int64_t)m * G::VIN];
      qc[m] = col[(int64_t)m * G::VIN + G::SM];
      qnx[m] = col[(int64_t)m * G::VIN + 2 * G::SM];
      if (has_ring) rraw[m] = ring[(int64_t)m * G::VIN + G::SM];
    }
  }
  Prim<T> wc = decode<T, D>(qc, gamma);
  T Flo[S];
  {
    const Prim<T> wlo = decode<T, D>(qlo, gamma);
    rusanov<T, D, K>(qlo, wlo, qc, wc, Flo);
  }
  T lam = T(0);

  for (int pl = 0; pl < P; ++pl) {
    // prefetch: ring of plane pl+1 and own volume of plane pl+2
    T rnext[S], qnn[S];
#pragma unroll
    for (int m = 0; m < S; ++m) {
      rnext[m] = rraw[m];
      qnn[m] = qnx[m];
    }
    if (ok) {
      if (has_ring && pl + 1 < P) {
#pragma unroll
        for (int m = 0; m < S; ++m) rnext[m] = ring[(int64_t)m * G::VIN + (int64_t)(pl + 2) * G::SM];
      }
      if (pl + 3 <= P + 1) {
#pragma unroll
        for (int m = 0; m < S; ++m) qnn[m] = col[(int64_t)m * G::VIN + (int64_t)(pl + 3) * G::SM];
      }
    }

    // A. publish own and ring volumes of this plane
    if (ok) {
#pragma unroll
      for (int m = 0; m < S; ++m) cell[m * NCELL + l] = qc[m];
      cell[(S + 0) * NCELL + l] = wc.ir;
      cell[(S + 1) * NCELL + l] = wc.p;
      cell[(S + 2) * NCELL + l] = wc.c;
      if (has_ring) {
        const Prim<T> wr = decode<T, D>(rraw, gamma);
#pragma unroll
        for (int m = 0; m < S; ++m) cell[m * NCELL + LANES + l] = rraw[m];
        cell[(S + 0) * NCELL + LANES + l] = wr.ir;
        cell[(S + 1) * NCELL + LANES + l] = wr.p;
        cell[(S + 2) * NCELL + LANES + l] = wr.c;
      }
    }
    __syncthreads();

    // B. in-plane faces on the low side of each volume, plus the high boundary
    T Fl0[S], Fl1[S], Fx[S];
    if (ok) {
      {
        const int nb = x > 0 ? l - 1 : LANES + (D == 3 ? y : 0);
        T qn[S];
#pragma unroll
        for (int m = 0; m < S; ++m) qn[m] = cell[m * NCELL + nb];
        const Prim<T> wn{cell[(S + 0) * NCELL + nb], cell[(S + 1) * NCELL + nb],
                         cell[(S + 2) * NCELL + nb]};
        rusanov<T, D, 0>(qn, wn, qc, wc, Fl0);
      }
      if constexpr (D == 3) {
        const int nb = y > 0 ? l - P : LANES + 2 * P + x;
        T qn[S];
#pragma unroll
        for (int m = 0; m < S; ++m) qn[m] = cell[m * NCELL + nb];
        const Prim<T> wn{cell[(S + 0) * NCELL + nb], cell[(S + 1) * NCELL + nb],
                         cell[(S + 2) * NCELL + nb]};
        rusanov<T, D, 1>(qn, wn, qc, wc, Fl1);
      }
      if (l < G::NEXTRA) {
        // high-boundary face: interior volume at coordinate P-1 against the ring
        const bool ydir = (D == 3) && l >= P;
        const int t = ydir ? l - P : l;
        const int lc = D == 3 ? (ydir ? (P - 1) * P + t : t * P + (P - 1)) : P - 1;
        const int rc = D == 3 ? (ydir ? LANES + 3 * P + t : LANES + P + t) : LANES + 1;
        T qa[S], qb[S];
#pragma unroll
        for (int m = 0; m < S; ++m) {
          qa[m] = cell[m * NCELL + lc];
          qb[m] = cell[m * NCELL + rc];
        }
        const Prim<T> wa{cell[(S + 0) * NCELL + lc], cell[(S + 1) * NCELL + lc],
                         cell[(S + 2) * NCELL + lc]};
        const Prim<T> wb{cell[(S + 0) * NCELL + rc], cell[(S + 1) * NCELL + rc],
                         cell[(S + 2) * NCELL + rc]};
        if (ydir) {
          if constexpr (D == 3) rusanov<T, D, 1>(qa, wa, qb, wb, Fx);
        } else {
          rusanov<T, D, 0>(qa, wa, qb, wb, Fx);
        }
      }
    }
    __syncthreads();

    // C. publish face fluxes: face[k][m][line * (P+1) + position along k]
    if (ok) {
#pragma unroll
      for (int m = 0; m < S; ++m) face[m * NF + y * (P + 1) + x] = Fl0[m];
      if constexpr (D == 3) {
#pragma unroll
        for (int m = 0; m < S; ++m) face[(S + m) * NF + x * (P + 1) + y] = Fl1[m];
      }
      if (l < G::NEXTRA) {
        const bool ydir = (D == 3) && l >= P;
        const int t = ydir ? l - P : l;
        const int base = (ydir ? S * NF : 0) + t * (P + 1) + P;
#pragma unroll
        for (int m = 0; m < S; ++m) face[base + m * NF] = Fx[m];
      }
    }
    __syncthreads();

    // D. high-side faces, marching-axis face, update, store, running maximum
    if (ok) {
      T Fr0[S], Fr1[S];
#pragma unroll
      for (int m = 0; m < S; ++m) {
        Fr0[m] = face[m * NF + y * (P + 1) + x + 1];
        if constexpr (D == 3) Fr1[m] = face[(S + m) * NF + x * (P + 1) + y + 1];
      }
      const Prim<T> wu = decode<T, D>(qnx, gamma);
      T Fhi[S];
      rusanov<T, D, K>(qc, wc, qnx, wu, Fhi);
      T qn[S];
#pragma unroll
      for (int m = 0; m < S; ++m) {
        T v = fma(-r[0], Fr0[m] - Fl0[m], qc[m]);
        if constexpr (D == 3) v = fma(-r[1], Fr1[m] - Fl1[m], v);
        qn[m] = fma(-r[K], Fhi[m] - Flo[m], v);
        outp[(int64_t)m * ocomp + (int64_t)pl * ostride] = qn[m];
      }
      const Prim<T> wn = decode<T, D>(qn, gamma);
      lam = nanmax(lam, max_wave_speed<T, D>(qn, wn));
#pragma unroll
      for (int m = 0; m < S; ++m) {
        qc[m] = qnx[m];
        Flo[m] = Fhi[m];
      }
      wc = wu;
    }
#pragma unroll
    for (int m = 0; m < S; ++m) {
      qnx[m] = qnn[m];
      rraw[m] = rnext[m];
    }
    __syncthreads();
  }

  // ---- per-patch maximum: shuffles within the patch's lanes ---------------
  constexpr bool pow2 = (LANES & (LANES - 1)) == 0;
  if constexpr (pow2) {
    constexpr int seg = LANES < 64 ? LANES : 64;
#pragma unroll
    for (int o = seg / 2; o > 0; o >>= 1) lam = nanmax(lam, T(__shfl_xor(lam, o, 64)));
    if constexpr (LANES > 64) {
      if ((tid & 63) == 0) red[tid >> 6] = lam;
      __syncthreads();
      if (tid == 0) {
#pragma unroll
        for (int w = 1; w < LANES / 64; ++w) lam = nanmax(lam, red[w]);
      }
    }
  } else {
    // odd cross-sections (e.g. 17 lanes): gather through LDS
    lds[tid < G::PPW * G::SLOT ? tid : 0] = lam;
    __syncthreads();
    if (in_range && l == 0) {
      for (int i = 1; i < LANES; ++i) lam = nanmax(lam, lds[slot * LANES + i]);
    }
  }
  if (in_range && l == 0 && max_eig) {
    max_eig[b] = ok ? double(lam) : __builtin_nan("");
  }
}

template <typename T, int D, int P>
int launch(const fv_patch* patches, int64_t n, const T* qin, int64_t qin_len, T* qout,
           int64_t qout_len, int out_halo, T gamma, const double* dt_dev, double* max_eig,
           hipStream_t st) {
  using G = Geo<D, P>;
  static_assert(G::PPW * G::LANES <= G::NT, "workgroup too small");
  static_assert(G::LANES % G::PPW == 0 || G::LANES < 64, "bad packing");
  const int64_t blocks = (n + G::PPW - 1) / G::PPW;
  hipLaunchKernelGGL((fv_update_kernel<T, D, P>), dim3((unsigned)blocks), dim3(G::NT), 0, st,
                     patches, n, qin, qin_len, qout, qout_len, out_halo, gamma, dt_dev, max_eig);
  return 0;
}

}  // namespace

bool update_supported(int dim, int p) {
  if (dim == 2) return p == 4 || p == 8 || p == 16 || p == 17 || p == 32;
  if (dim == 3) return p == 4 || p == 8 || p == 16;
  return false;
}

int launch_update_f64(const fv_patch* patches, int64_t n, const double* qin, int64_t qin_len,
                      double* qout, int64_t qout_len, int out_halo, int dim, int p,
                      double gamma, const double* dt_dev, double* max_eig, hipStream_t st) {
#define FV_CASE(DD, PP)                                                                   \
  if (dim == DD && p == PP)                                                               \
    return launch<double, DD, PP>(patches, n, qin, qin_len, qout, qout_len, out_halo, gamma, \
                                  dt_dev, max_eig, st);
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
