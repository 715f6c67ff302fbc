// Plane-marching batched patch update for gfx950 (Section 2 eqs. (3)-(5) and
// Algorithm 1 of arXiv 2302.09005).
//
// Mapping.  A patch of P^D volumes is swept along its last axis ("marching
// axis": z in 3-D, y in 2-D).  Lane l of the patch owns the column of volumes
// at in-plane position l and walks it plane by plane, so every global load
// and store is a whole plane of one unknown: contiguous rows of P elements,
// unit stride across lanes (coalesced SoA traffic).  A 3-D 8^3 patch is one
// wave64; smaller cross-sections pack several patches into one wave, larger
// ones span several waves of one workgroup.  A patch may also be marched in
// chunks of planes side by side (2-D 16^2, 17^2 and 32^2 patches: 4, 3 and 2
// chunks, each a lane group of one wave), each chunk recomputing the face
// below its first plane; the results do not depend on the split.
//
// Per plane:
//   A. each lane publishes its volume (q, 1/rho, p, c) to LDS; lanes
//      l < RING also publish one face-halo volume of the plane ("ring"), so
//      halo volumes are decoded once;
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
// Two sources for the face halo, one kernel body:
//   * HALO (the paper's interface): every patch block carries its own halo
//     layer, [s][(P+2)^D]; the halo is read from the block itself.
//   * GATHER: blocks are compact, [s][P^D], and each face-halo volume is read
//     directly from the facing interior volume of the neighbouring patch (or,
//     at a transmissive boundary, from the patch's own boundary volume).  This
//     fuses the halo exchange into the tile gather: the multi-step loop needs
//     no separate halo-fill pass and no halo storage.  Results are identical.
//
// The per-patch maximum is reduced across the patch's lanes with wave
// shuffles (and LDS across waves or chunks).  Launches that write more than
// 128 MB store the new state with non-temporal stores (a second instance of
// each kernel; same values).
#pragma once

#include <hip/hip_ext.h>

#include <atomic>

#include "fv_euler.hpp"
#include "fv_internal.hpp"


namespace fvk {

namespace {

// IEEE bit pattern of +inf: for positive doubles, kInfBits - bits(h) is
// positive and decreases as h grows, so an integer max of it is a min of h.
constexpr unsigned long long kInfBits = 0x7ff0000000000000ull;

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double v) {
  return __longlong_as_double(uni((int64_t)__double_as_longlong(v)));
}
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Orders the LDS accesses of a workgroup's threads at a phase boundary.  A
// workgroup of one wave needs no barrier and no wait: the LDS performs the
// accesses of one wave in program order, so it is enough that the compiler
// keeps them in order (a wavefront-scope fence).
template <int NT>
__device__ __forceinline__ void phase_sync() {
  if constexpr (NT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Per-workgroup outputs of the update body for the caller's epilogue.
struct BodyOut {
  double lam;    // maximum of the new state of this thread's patch (NaN if skipped)
  double hmin;   // smallest volume width of that patch
  bool in_range; // this thread's slot holds a patch
  bool lead;     // this thread carries its patch's results (lam valid here)
  int slot;      // slot of this thread in the workgroup
  double dt;     // pipelined step: the time step taken (every thread)
  double lprev;  // pipelined step: Lambda it was computed from (NaN with a given dt)
};

// The update of the (up to PPW) patches of one workgroup of NTW threads, each
// marched in ZS chunks.  b: the patch of this thread's slot (-1: none).
// lds: PPW * ZS * SLOT elements, red: Geo::NRED elements, both shared by the
// body's NTW threads, whose index in the body is tid.  MODE:
// see StepMode (kLocalDt needs a writable descriptor array and cfl).  NTS:
// write the new state with non-temporal stores (the same values).  PUSH
// (halo'd input and output blocks): the halo exchange of the new state is
// fused into the update, the other way round from GATHER: every boundary
// volume of the new state is also stored into the face halo that reads it,
// the facing halo slot of the neighbour's output block (the neighbour must
// name this patch across the opposite face), or at a transmissive face the
// adjacent halo slot of the own block.
template <typename T, int D, int P, int NTW, int ZS, bool GATHER, int MODE, bool NTS,
          bool PUSH = false>
__device__ __forceinline__ BodyOut update_body(
    const fv_patch* __restrict__ patches, int64_t n, const int64_t* __restrict__ neighbours,
    const T* __restrict__ qin, int64_t qin_len, T* __restrict__ qout, int64_t qout_len,
    int out_halo, T gamma, const double* __restrict__ dt_dev, double* __restrict__ max_eig,
    double cfl, int64_t b, T* __restrict__ lds, T* __restrict__ red, int tid,
    const unsigned long long* __restrict__ prev_slots = nullptr, bool prio = false) {
  using G = Geo<D, P, NTW, ZS>;
  constexpr int S = G::S;
  constexpr int PC = G::PC;  // planes of a chunk (the last chunk may have fewer)
  constexpr bool UNEVEN = P % ZS != 0;
  constexpr int K = D - 1;  // marching axis
  constexpr int W = G::W;
  constexpr int LANES = G::LANES;
  constexpr int NCELL = G::CST;  // stride of one value in the plane buffer
  constexpr int NF = G::FST;     // stride of one value in the face buffer
  // strides of the input blocks: component, marching-axis plane
  constexpr int CS = GATHER ? G::VOUT : G::VIN;
  constexpr int PS = GATHER ? G::SMO : G::SM;

  const int slot = G::PPW == 1 ? 0 : tid / G::TPP;
  const int tp = G::PPW == 1 ? tid : tid - slot * G::TPP;  // thread within the patch
  const int chunk = ZS == 1 ? 0 : tp / LANES;
  const int l = ZS == 1 ? tp : tp - chunk * LANES;
  const int p0 = chunk * PC;  // first plane of the chunk
  // planes of this chunk (PC, or fewer for the last chunk of an uneven split)
  const int nrows = UNEVEN ? (P - p0 < PC ? P - p0 : PC) : PC;
  // threads past the workgroup's patches (a lone patch of fewer threads than
  // the workgroup, e.g. 3 chunks of 17 lanes in a wave) take no part
  const bool in_patch = G::PPW * G::TPP == G::NT || tid < G::PPW * G::TPP;
  const bool in_range = in_patch && (G::PPW == 1 || slot < G::PPW) && b >= 0 && b < n;
  const bool lead = in_range && l == 0 && chunk == 0;  // writes the patch results
  const int x = l % P;
  const int y = (D == 3) ? l / P : 0;
  const bool has_ring = l < G::RING;
  // ring volume of this lane: quadrant (= the face it lies across) and
  // position along it
  const int q4 = D == 3 ? l / P : l;
  const int rr = D == 3 ? l - q4 * P : 0;

  // ---- descriptor, sources, device-side bounds checks -------------------
  const int64_t blk_in = (int64_t)S * (GATHER ? G::VOUT : G::VIN);
  const int64_t blk_out = out_halo ? (int64_t)S * G::VIN : (int64_t)S * G::VOUT;
  int64_t off_in = 0, off_out = 0;
  int64_t lo_base = 0, hi_base = 0, ring_src = 0;  // element offsets (GATHER)
  // PUSH: element distance from a boundary volume's own output slot to the
  // halo slot that receives it, per face (-x, +x, -y, +y[, -z, +z])
  int64_t pshift[2 * D];
#pragma unroll
  for (int f = 0; f < 2 * D; ++f) pshift[f] = 0;
  T r[3] = {T(0), T(0), T(0)};
  double hmin = __builtin_inf();
  double dt_used = 0.0, t_used = 0.0;
  bool ok = false;
  // the device time step, loaded alongside the descriptor rather than after it
  const bool dev_dt = MODE != kLocalDt && dt_dev != nullptr;
  const double dt_d = dev_dt ? *dt_dev : 0.0;
  // Pipelined step: the slot maxima the previous launch folded, one slot per
  // lane, loaded before the descriptor (so they have arrived when the
  // descriptor has).  The previous launch has completed, so its atomics are
  // visible to ordinary loads, which the workgroups of an XCD then serve from
  // that XCD's L2 (device-scope loads of every workgroup would all go to the
  // same few lines in memory).
  constexpr bool PIPE = MODE == kPipelinedCfl;
  unsigned long long pL = 0, pH = 0;
  if constexpr (PIPE) {
    const int sl = tid & 63;
    if (prev_slots && sl < kPipeSlots) {
      pL = prev_slots[(size_t)kCflSlot * sl + kCflWord];
      pH = prev_slots[(size_t)kCflSlot * sl + 2 * kCflWord];
    }
  }
  double lprev = __builtin_nan("");
  // dt = cfl * min dx / (D * Lambda) over the previous launch's maxima,
  // exactly as the fused step computes it at its end.  The slots sit in
  // lanes 0 .. kPipeSlots-1, which are active wherever this runs (a patch's
  // lanes start at lane 0), so they are folded among themselves and lane 0's
  // result is given to the whole wave: lanes past a patch's last thread (17^2
  // patches use 51 of 64) may be inactive here.
  static_assert(kPipeSlots <= 64 && (kPipeSlots & (kPipeSlots - 1)) == 0, "slot fold");
  auto pipe_dt = [&]() -> double {
    if (!prev_slots) return dt_d;
#pragma unroll
    for (int o = kPipeSlots / 2; o > 0; o >>= 1) {
      pL = max(pL, (unsigned long long)__shfl_xor(pL, o, 64));
      pH = max(pH, (unsigned long long)__shfl_xor(pH, o, 64));
    }
    pL = (unsigned long long)uni((int64_t)pL);
    pH = (unsigned long long)uni((int64_t)pH);
    lprev = __longlong_as_double((long long)pL);
    const double h = __longlong_as_double((long long)(kInfBits - pH));
    return cfl * h / ((double)D * lprev);
  };
  // a one-wave, one-patch workgroup is converged inside the patch's checks
  // (the patch is the same in every lane): the time step is taken there, where
  // the other modes take theirs
  constexpr bool PIPE_IN = PIPE && G::PPW == 1 && G::NT == 64;
  static_assert(!PIPE_IN || G::TPP >= kPipeSlots, "the slot lanes are inside the patch");
  // GATHER: the chunk's first two own planes, loaded as soon as the own
  // descriptor has been checked, while the neighbours' descriptors are still
  // on their way (for chunks whose march is fully unrolled; in the others the
  // early values would stay live across the loop)
  constexpr bool HOIST = GATHER && PC <= 8;
  T qpre0[S], qpre1[S];
#pragma unroll
  for (int m = 0; m < S; ++m) qpre0[m] = qpre1[m] = T(1);
  if (in_range) {
    // The neighbour table row (loaded with the descriptor), then the
    // neighbours' descriptors as one batch of independent loads (an index
    // outside [0, n) reads the own descriptor instead and is judged below):
    // two memory round trips before the first plane can be loaded, whatever
    // the number of faces.
    int64_t nbi[2 * D];
    if constexpr (GATHER || PUSH) {
#pragma unroll
      for (int f = 0; f < 2 * D; ++f) nbi[f] = neighbours[b * 2 * D + f];
    }
    const fv_patch pd = patches[b];
    off_in = pd.q_in;
    off_out = pd.q_out;
    ok = pd.p == P && off_in >= 0 && off_in <= qin_len - blk_in && off_out >= 0 &&
         off_out <= qout_len - blk_out;
    if constexpr (HOIST) {
      if (ok) {
        const T* g0 = qin + off_in + (x + (D == 3 ? y * P : 0)) + (int64_t)p0 * PS;
#pragma unroll
        for (int m = 0; m < S; ++m) qpre0[m] = g0[(int64_t)m * CS];
        if (nrows >= 2) {
#pragma unroll
          for (int m = 0; m < S; ++m) qpre1[m] = g0[(int64_t)m * CS + PS];
        }
      }
    }
    double dt = dev_dt ? dt_d : pd.dt;
    if constexpr (PIPE_IN) dt = pipe_dt();
    dt_used = dt;
    t_used = pd.t;
    if constexpr (!PIPE || PIPE_IN) {
#pragma unroll
      for (int j = 0; j < D; ++j) r[j] = T(dt / pd.dx[j]) * T(0.5);  // rusanov gives 2F
    }
    hmin = pd.dx[0];
#pragma unroll
    for (int j = 1; j < D; ++j) hmin = fmin(hmin, pd.dx[j]);
    if constexpr (GATHER) {
      // face order -x, +x, -y, +y[, -z, +z]; -1 = transmissive
      int64_t nq[2 * D];
      int np[2 * D];
#pragma unroll
      for (int f = 0; f < 2 * D; ++f) {
        const int64_t c = (nbi[f] >= 0 && nbi[f] < n) ? nbi[f] : b;
        nq[f] = patches[c].q_in;
        np[f] = patches[c].p;
      }
      // judged without branches, so that the loads above are not sunk into
      // a chain of conditional ones
      int64_t nbo[2 * D];
#pragma unroll
      for (int f = 0; f < 2 * D; ++f) {
        const int64_t nb = nbi[f];
        const bool inr = (nb >= 0) & (nb < n);
        const bool good = (np[f] == P) & (nq[f] >= 0) & (nq[f] <= qin_len - blk_in);
        nbo[f] = (inr & good) ? nq[f] : -1;
        ok = ok & (inr ? good : nb == -1);
      }
      constexpr int fl = 2 * K, fh = 2 * K + 1;  // marching-axis faces
      constexpr int last = (P - 1) * G::SMO;
      // block bases of the two marching-axis halo planes (plane offset included)
      lo_base = nbo[fl] >= 0 ? nbo[fl] + last : off_in;
      hi_base = nbo[fh] >= 0 ? nbo[fh] : off_in + last;
      if (has_ring) {
        // the facing volume of the neighbour, or the own boundary volume
        const bool hasnb = nbo[q4] >= 0;
        int idx;
        if (D == 3) {
          idx = q4 == 0 ? (hasnb ? P - 1 : 0) + P * rr
              : q4 == 1 ? (hasnb ? 0 : P - 1) + P * rr
              : q4 == 2 ? rr + P * (hasnb ? P - 1 : 0)
                        : rr + P * (hasnb ? 0 : P - 1);
        } else {
          idx = q4 == 0 ? (hasnb ? P - 1 : 0) : (hasnb ? 0 : P - 1);
        }
        ring_src = (hasnb ? nbo[q4] : off_in) + idx;
      } else {
        ring_src = off_in + x + (D == 3 ? y * P : 0);  // own column, never used
      }
    }
    if constexpr (PUSH) {
      // The neighbours' output offsets, sizes and back references, each as
      // one batch of independent loads (as for the gather above).  Along the
      // face axis a boundary volume sits at halo'd coordinate 1 (low face)
      // or P (high face); it lands at P+1 or 0 of the neighbour's block, or
      // at 0 or P+1 of the own block (transmissive).
      int64_t nq[2 * D], back[2 * D];
      int np[2 * D];
#pragma unroll
      for (int f = 0; f < 2 * D; ++f) {
        const int64_t c = (nbi[f] >= 0 && nbi[f] < n) ? nbi[f] : b;
        nq[f] = patches[c].q_out;
        np[f] = patches[c].p;
        back[f] = neighbours[c * 2 * D + (f ^ 1)];
      }
#pragma unroll
      for (int f = 0; f < 2 * D; ++f) {
        const int64_t nb = nbi[f];
        const int64_t astride = f < 2 ? 1 : f < 4 ? W : (int64_t)W * W;
        const bool hi = f & 1;
        const bool inr = (nb >= 0) & (nb < n);
        const bool good = (np[f] == P) & (nq[f] >= 0) & (nq[f] <= qout_len - blk_out) &
                          (back[f] == b);
        pshift[f] = inr ? (nq[f] - off_out) + (hi ? -P : P) * astride
                        : (hi ? astride : -astride);
        ok = ok & (inr ? good : nb == -1);
      }
    }
  }
  if constexpr (PIPE && !PIPE_IN) {
    // several patches or waves per workgroup: the time step once the wave
    // has left the patches' checks
    const double dtp = pipe_dt();
    dt_used = dtp;
    // the volume widths read again (cached) rather than kept live through
    // the neighbour checks
    const fv_patch* pr = patches + (in_range ? b : 0);
#pragma unroll
    for (int j = 0; j < D; ++j) r[j] = T(dtp / pr->dx[j]) * T(0.5);  // rusanov gives 2F
  }
  if constexpr (G::PPW == 1) {
    // one patch per workgroup: every lane read the same descriptor, so its
    // values live in scalar registers
    ok = __builtin_amdgcn_readfirstlane((int)ok) != 0;
    off_in = uni(off_in);
    off_out = uni(off_out);
    lo_base = uni(lo_base);
    hi_base = uni(hi_base);
#pragma unroll
    for (int j = 0; j < 3; ++j) r[j] = uni(r[j]);
    if constexpr (PUSH) {
#pragma unroll
      for (int f = 0; f < 2 * D; ++f) pshift[f] = uni(pshift[f]);
    }
    hmin = uni(hmin);
    dt_used = uni(dt_used);
    t_used = uni(t_used);
    if constexpr (PIPE) lprev = uni(lprev);
  }
  // plane buffer [NV][NCELL]
  T* cell = lds + (ok && in_patch ? (slot * ZS + chunk) * G::SLOT : 0);
  T* face = cell;                             // face buffers, same storage

  // in-plane element index of the own column (compact and halo'd) and of
  // the ring volume inside the own halo'd block
  const int col_c = x + (D == 3 ? y * P : 0);
  const int col_h = (x + 1) + (D == 3 ? (y + 1) * W : 0);
  int ring_h;
  if (D == 3) {
    ring_h = q4 == 0 ? (rr + 1) * W
           : q4 == 1 ? (P + 1) + (rr + 1) * W
           : q4 == 2 ? (rr + 1)
                     : (rr + 1) + (P + 1) * W;
  } else {
    ring_h = l == 0 ? 0 : P + 1;
  }
  const int col_in = GATHER ? col_c : col_h;
  const int col_out = out_halo ? col_h + G::SM : col_c;
  const int64_t ostride = out_halo ? G::SM : G::SMO;
  const int64_t ocomp = out_halo ? G::VIN : G::VOUT;

  // the chunk's own planes p0 .. p0+nrows-1 (storage plane j = 1 + plane in a
  // halo'd block, = plane in a compact one), the plane below and the plane
  // above it (halo planes, or planes of the neighbouring chunks)
  const int64_t jin = GATHER ? p0 : p0 + 1;
  const T* gin = qin + off_in + col_in + jin * PS;
  const T* glo = (GATHER && chunk == 0) ? qin + lo_base + col_c : gin - PS;
  const T* ghi =
      (GATHER && chunk == ZS - 1) ? qin + hi_base + col_c : gin + (int64_t)nrows * PS;
  const T* gring = (GATHER ? qin + ring_src : qin + off_in + ring_h + PS) + (int64_t)p0 * PS;
  T* gout = qout + off_out + col_out + (int64_t)p0 * ostride;

  // unknown m of the own column at chunk storage plane j in [0, nrows+1] (0
  // and nrows+1: the planes below and above the chunk)
  auto ld_own = [&](int j, int m) -> T {
    if (j == 0) return glo[(int64_t)m * CS];
    if (j == nrows + 1) return ghi[(int64_t)m * CS];
    return gin[(int64_t)m * CS + (int64_t)(j - 1) * PS];
  };
  // unknown m of the ring volume at chunk plane j in [1, nrows]
  auto ld_ring = [&](int j, int m) -> T { return gring[(int64_t)m * CS + (int64_t)(j - 1) * PS]; };
  // NTS: streaming (non-temporal) stores, for outputs too large to stay in
  // the caches until the next step reads them
  auto st_out = [&](int pl, int m, T v, int64_t shift = 0) {
    T* dst = gout + (int64_t)m * ocomp + (int64_t)pl * ostride + shift;
    if constexpr (NTS) __builtin_nontemporal_store(v, dst);
    else *dst = v;
  };

  // a patch that failed its checks skips all work (its max_eig becomes NaN)
  const bool act = ok && in_patch;
  T lam = T(0);
  // UNI: the workgroup marches one patch with all its threads, so act is the
  // same in every thread and the whole march below is run or skipped; inside
  // it nothing is conditional, and no register holds a default for a skipped
  // load.  Otherwise every load, LDS access and update is guarded by the
  // thread's own act.  UNI only for float state: with float64 state the
  // scheduler's freedom in the branch-free march costs registers (3-D 8^3:
  // 126 -> 204, two waves per SIMD instead of four); float state has room.
  constexpr bool UNI = sizeof(T) == 4 && G::PPW == 1 && G::TPP == G::NT && !UNEVEN;
  if (!UNI || act) {
  // ---- prologue: planes -1 and 0, first marching-axis face ---------------
  T qlo[S], qc[S], qnx[S], rraw[S];
  if constexpr (!UNI) {
#pragma unroll
    for (int m = 0; m < S; ++m) {
      qlo[m] = T(0);
      qc[m] = T(1);
      qnx[m] = T(1);
      rraw[m] = T(1);
    }
  }
  if (UNI || act) {
#pragma unroll
    for (int m = 0; m < S; ++m) {
      qlo[m] = ld_own(0, m);
      qc[m] = HOIST ? qpre0[m] : ld_own(1, m);
      rraw[m] = ld_ring(1, m);  // lanes without a ring volume read their own column
    }
  }
  Prim<T> wc = decode<T, D>(qc, gamma);
  T Flo[S];
  {
    const Prim<T> wlo = decode<T, D>(qlo, gamma);
    rusanov<T, D, K>(qlo, wlo, qc, wc, Flo);
  }

  // face buffers: x-faces [y][x] for the low face of every volume followed by
  // the high-boundary faces [y]; y-faces [y][x] for y in [0, P] (the last row
  // is the high boundary).  Every lane's low and high faces then sit at
  // consecutive addresses across lanes (no LDS bank conflicts).
  constexpr int FX_EXTRA = LANES;
  const int fx_lo = l;
  const int fx_hi = x < P - 1 ? l + 1 : FX_EXTRA + (D == 3 ? y : 0);
  const int fy_lo = l;
  const int fy_hi = l + P;

  // fully unrolled for small patches so that the rolling registers are
  // renamed instead of copied
  constexpr int UNROLL = PC <= 8 ? PC : 2;
#pragma unroll UNROLL
  for (int pl = 0; pl < PC; ++pl) {
    if (prio) {
      // Issue priority falls from 3 to 0 as the march advances, so the waves
      // that share a SIMD progress together: with the hardware's oldest-first
      // arbitration alone, some race ahead and the last one marches alone at
      // the end with nothing to hide its latency.  (Only when every
      // workgroup of the launch is resident at once; the host decides.)
      const int lv = (4 * pl) / PC;
      if (pl == 0 || lv != (4 * (pl - 1)) / PC) {
        switch (lv) {
          case 0: __builtin_amdgcn_s_setprio(3); break;
          case 1: __builtin_amdgcn_s_setprio(2); break;
          case 2: __builtin_amdgcn_s_setprio(1); break;
          default: __builtin_amdgcn_s_setprio(0); break;
        }
      }
    }
    // the last chunk of an uneven split idles through its missing planes
    const bool live = !UNEVEN || pl < nrows;
    const bool run = UNI || (act && live);
    // loads for the next plane: its own volumes (needed for the
    // marching-axis face in D) and its ring (needed in the next A)
    T rnext[S];
#pragma unroll
    for (int m = 0; m < S; ++m) {
      rnext[m] = rraw[m];
      if constexpr (!UNI) qnx[m] = qc[m];
    }
    if (run) {
      if (pl + 1 < nrows) {
#pragma unroll
        for (int m = 0; m < S; ++m) rnext[m] = ld_ring(pl + 2, m);
      }
#pragma unroll
      for (int m = 0; m < S; ++m)
        qnx[m] = (HOIST && pl == 0 && nrows >= 2) ? qpre1[m] : ld_own(pl + 2, m);
    }
    // A. publish own and ring volumes of this plane
    if (run) {
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
    phase_sync<G::NT>();

    // B. in-plane faces on the low side of each volume, plus the high boundary.
    // The boundary faces come first: their operands (two volumes from LDS)
    // are then live while no other face result is, which keeps the body at
    // 4 waves per SIMD for 3-D 8^3 FP64 (126 VGPRs; 168 the other way round).
    T Fl0[S], Fl1[S], Fx[S];
    if (run) {
      if (l < G::NEXTRA) {
        // high-boundary face: interior volume at coordinate P-1 against the
        // ring.  A y face reads its two in-plane momenta swapped, so that one
        // x-direction flux serves both directions (the same operations on the
        // same values: bit-identical to a y-direction flux).
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
    }
    phase_sync<G::NT>();

    // C. publish face fluxes: face[k][m][index]
    if (run) {
#pragma unroll
      for (int m = 0; m < S; ++m) face[m * NF + fx_lo] = Fl0[m];
      if constexpr (D == 3) {
#pragma unroll
        for (int m = 0; m < S; ++m) face[(S + m) * NF + fy_lo] = Fl1[m];
      }
      if (l < G::NEXTRA) {
        const bool ydir = (D == 3) && l >= P;
        const int t = ydir ? l - P : l;
        const int base = ydir ? S * NF + P * P + t : FX_EXTRA + t;
#pragma unroll
        for (int m = 0; m < S; ++m) face[base + m * NF] = Fx[m];
      }
    }
    phase_sync<G::NT>();

    // D. high-side faces, marching-axis face, update, store, running maximum.
    // The x and y terms of the update are applied first, so the in-plane face
    // fluxes are dead before the marching-axis face is evaluated (same
    // operations in the same order as one expression per unknown).
    if (run) {
      T v[S];
#pragma unroll
      for (int m = 0; m < S; ++m) {
        v[m] = fma(-r[0], face[m * NF + fx_hi] - Fl0[m], qc[m]);
        if constexpr (D == 3) v[m] = fma(-r[1], face[(S + m) * NF + fy_hi] - Fl1[m], v[m]);
      }
      const Prim<T> wu = decode<T, D>(qnx, gamma);
      T Fhi[S];
      rusanov<T, D, K>(qc, wc, qnx, wu, Fhi);
      T qn[S];
#pragma unroll
      for (int m = 0; m < S; ++m) {
        qn[m] = fma(-r[K], Fhi[m] - Flo[m], v[m]);
        st_out(pl, m, qn[m]);
      }
      if constexpr (PUSH) {
        // boundary volumes of the new state into the face halos that read them
        auto push = [&](int f) {
#pragma unroll
          for (int m = 0; m < S; ++m) st_out(pl, m, qn[m], pshift[f]);
        };
        if (x == 0) push(0);
        if (x == P - 1) push(1);
        if constexpr (D == 3) {
          if (y == 0) push(2);
          if (y == P - 1) push(3);
        }
        if (p0 + pl == 0) push(2 * K);
        if (p0 + pl == P - 1) push(2 * K + 1);
      }
      const Prim<T> wn = decode<T, D>(qn, gamma);
      lam = nanmax_pos(lam, max_wave_speed<T, D>(qn, wn));
#pragma unroll
      for (int m = 0; m < S; ++m) {
        qc[m] = qnx[m];
        Flo[m] = Fhi[m];
      }
      wc = wu;
    }
#pragma unroll
    for (int m = 0; m < S; ++m) rraw[m] = rnext[m];
    phase_sync<G::NT>();
  }
  }  // the march

  // ---- per-patch maximum: shuffles within the patch's lanes ---------------
  constexpr bool pow2 = (LANES & (LANES - 1)) == 0;
  if constexpr (pow2) {
    constexpr int seg = LANES < 64 ? LANES : 64;
#pragma unroll
    for (int o = seg / 2; o > 0; o >>= 1) lam = nanmax_pos(lam, T(__shfl_xor(lam, o, 64)));
    if constexpr (LANES > 64) {
      if ((tid & 63) == 0) red[tid >> 6] = lam;
      phase_sync<G::NT>();
      if (tid == 0) {
#pragma unroll
        for (int w = 1; w < LANES / 64; ++w) lam = nanmax_pos(lam, red[w]);
      }
    } else if constexpr (ZS > 1) {
      // fold the chunks of each patch (whole waves, or lane groups of one)
      if (l == 0 && in_patch) red[slot * ZS + chunk] = lam;
      phase_sync<G::NT>();
      if (lead) {
#pragma unroll
        for (int c = 1; c < ZS; ++c) lam = nanmax_pos(lam, red[slot * ZS + c]);
      }
    }
  } else {
    // odd cross-sections (e.g. 17 lanes): gather the lanes of every chunk
    // of the patch through LDS
    lds[tid < G::PPW * G::SLOT ? tid : 0] = lam;
    phase_sync<G::NT>();
    if (lead) {
      for (int i = 1; i < G::TPP; ++i) lam = nanmax_pos(lam, lds[slot * G::TPP + i]);
    }
  }
  const double lam_b = ok ? double(lam) : __builtin_nan("");
  if (lead && max_eig) max_eig[b] = lam_b;
  if constexpr (MODE == kLocalDt) {
    // local time stepping: this patch moves to t + dt and takes its own
    // next CFL step from the new state
    if (lead && ok) {
      fv_patch* pw = const_cast<fv_patch*>(patches) + b;
      pw->t = t_used + dt_used;
      pw->dt = cfl * hmin / ((double)D * lam_b);
    }
  }
  return BodyOut{lam_b, hmin, in_range, lead, slot, dt_used, lprev};

}

// Workgroup w of a launch runs on XCD w mod 8 (round-robin dispatch over the
// eight XCDs, each with its own L2).  Hand each XCD a contiguous range of
// launch items instead, so that neighbouring patches, whose face layers a
// patch reads, are updated on the same XCD at about the same time and meet
// in its L2.
__device__ __forceinline__ int64_t xcd_contiguous(int64_t w, int64_t nwg) {
  constexpr int64_t kXcd = 8;
  const int64_t q = nwg / kXcd, r = nwg % kXcd;
  const int64_t x = w % kXcd, k = w / kXcd;
  return x * q + (x < r ? x : r) + k;
}

template <typename T, int D, int P, bool GATHER, int MODE, bool NTS, bool PUSH>
__global__ void __attribute__((amdgpu_flat_work_group_size(1, Geo<D, P>::NT)))
fv_update_kernel(const fv_patch* __restrict__ patches, int64_t n,
                 const int64_t* __restrict__ neighbours,
                 const T* __restrict__ qin, int64_t qin_len,
                 T* __restrict__ qout, int64_t qout_len, int out_halo, T gamma,
                 const double* __restrict__ dt_dev, double* __restrict__ max_eig,
                 CflOut cflo, const int64_t* __restrict__ order, int64_t order_base,
                 int64_t count, int prio) {
  using G = Geo<D, P>;
  __shared__ T lds[G::PPW * G::CHUNKS * G::SLOT];
  __shared__ T red[G::NRED];
  const int tid = threadIdx.x;
  const int slot = G::PPW == 1 ? 0 : tid / G::TPP;
  // the patch of this thread's slot: launch item i is patch i, or the
  // patch order[order_base + i] when the launch covers a sorted range
  const int64_t wgi = xcd_contiguous(blockIdx.x, gridDim.x);
  const int64_t i = wgi * G::PPW + slot;
  int64_t b = -1;
  if (slot < G::PPW && i < count) b = order ? order[order_base + i] : i;
  constexpr int BMODE = MODE == kLocalDt ? kLocalDt : MODE == kPipelinedCfl ? kPipelinedCfl : kPlain;
  const unsigned long long* prev =
      MODE == kPipelinedCfl && !dt_dev
          ? cflo.ws + (size_t)kCflSlot * kPipeSlots * (unsigned)((cflo.phase + 2) % 3)
          : nullptr;
  const BodyOut bo = update_body<T, D, P, 64, G::CHUNKS, GATHER, BMODE, NTS, PUSH>(
      patches, n, neighbours, qin, qin_len, qout, qout_len, out_halo, gamma, dt_dev, max_eig,
      cflo.cfl, b, lds, red, tid, prev, prio != 0);
  const double lam_b = bo.lam;
  const double hmin = bo.hmin;
  const bool lead = bo.lead;
  if constexpr (MODE == kPipelinedCfl) {
    // Pipelined CFL step: fold this patch's maximum and smallest width into
    // slot (workgroup mod kPipeSlots) of set `phase` (atomic maxima of IEEE
    // bit patterns, as below; nothing waits for them: the next launch reads
    // the set after this one has completed).  Workgroup 0 clears the set the
    // previous launch read, which the next launch folds into, and reports
    // the step.
    unsigned long long* gw =
        cflo.ws + (size_t)kCflSlot * (kPipeSlots * (unsigned)cflo.phase + blockIdx.x % kPipeSlots);
    if (lead) {
      __hip_atomic_fetch_max(&gw[kCflWord], (unsigned long long)__double_as_longlong(lam_b),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_max(&gw[2 * kCflWord],
                             kInfBits - (unsigned long long)__double_as_longlong(hmin),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
      unsigned long long* sc =
          cflo.ws + (size_t)kCflSlot * kPipeSlots * (unsigned)((cflo.phase + 1) % 3);
      if (tid < kPipeSlots) {
        __hip_atomic_store(&sc[(size_t)kCflSlot * tid + kCflWord], 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&sc[(size_t)kCflSlot * tid + 2 * kCflWord], 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
      if (tid == 0) {
        if (cflo.dt_used) *cflo.dt_used = bo.dt;
        if (cflo.lambda_out && !dt_dev) *cflo.lambda_out = bo.lprev;
      }
    }
  }
  if constexpr (MODE == kGlobalCfl) {
    // Fused CFL step.  Patch maxima and smallest volume widths are folded
    // with device-scope atomic maxima of IEEE bit patterns (values >= 0 or
    // NaN, so integer order is numeric order with NaN on top, and the result
    // does not depend on the order of arrival).  Same-address atomics
    // serialize, so the workgroups fold into the slots of their group
    // (kCflGroup consecutive ones) and count their arrival there; the last of
    // a group counts the group's arrival at the top, and the last group to
    // arrive reads (and clears) every group's slots, one group per lane, and
    // computes the next time step: four dependent atomic round trips from
    // the last workgroup's fold to the time step.  Ordering without fences:
    // the maxima are returning atomics whose results feed the arrival
    // increment, so a fold is counted only after it has been performed, and
    // each later step is issued only after the count before it returned.
    __shared__ unsigned long long dep_s[G::PPW];
    __shared__ int last;  // this workgroup is the last of the launch to arrive
    const unsigned nwg = gridDim.x;
    const unsigned grp = blockIdx.x / kCflGroup;
    const unsigned ngrp = (nwg + kCflGroup - 1) / kCflGroup;
    const unsigned gsize = min((unsigned)kCflGroup, nwg - grp * kCflGroup);
    unsigned long long* gs = cflo.ws + (size_t)kCflSlot * (grp + 1);  // group slots
    unsigned long long* ts = cflo.ws;                                 // top slots
    constexpr int kC = 0, kL = kCflWord, kH = 2 * kCflWord;  // count, max lambda, max (inf - h)
    if (lead) {
      const unsigned long long o1 = __hip_atomic_fetch_max(
          &gs[kL], (unsigned long long)__double_as_longlong(lam_b), __ATOMIC_RELAXED,
          __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long o2 = __hip_atomic_fetch_max(
          &gs[kH], kInfBits - (unsigned long long)__double_as_longlong(hmin),
          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // never true (no maximum reaches all ones); it only ties the arrival
      // below to the two results above
      dep_s[slot] = (o1 == ~0ull || o2 == ~0ull) ? 1ull : 0ull;
    }
    phase_sync<G::NT>();
    if (tid == 0) {
      unsigned long long dep = 0;
#pragma unroll
      for (int k = 0; k < G::PPW; ++k)
        if (wgi * G::PPW + k < count) dep |= dep_s[k];
      const unsigned long long before =
          __hip_atomic_fetch_add(&gs[kC], 1ull + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int l = 0;
      if (before == gsize - 1) {
        // last of its group: every fold of the group has been performed
        __hip_atomic_store(&gs[kC], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long tb =
            __hip_atomic_fetch_add(&ts[kC], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        l = tb == ngrp - 1;
        if (l) __hip_atomic_store(&ts[kC], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      last = l;
    }
    phase_sync<G::NT>();
    if (last && tid < 64) {
      // every group has counted its arrival: read and clear all their slots
      unsigned long long Lb = 0, Hb = 0;
      for (unsigned g = tid; g < ngrp; g += 64) {
        unsigned long long* s = cflo.ws + (size_t)kCflSlot * (g + 1);
        Lb = max(Lb, __hip_atomic_exchange(&s[kL], 0ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
        Hb = max(Hb, __hip_atomic_exchange(&s[kH], 0ull, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT));
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        Lb = max(Lb, (unsigned long long)__shfl_xor(Lb, o, 64));
        Hb = max(Hb, (unsigned long long)__shfl_xor(Hb, o, 64));
      }
      if (tid == 0) {
        const double L = __longlong_as_double((long long)Lb);
        const double h = __longlong_as_double((long long)(kInfBits - Hb));
        *cflo.dt_next = cflo.cfl * h / ((double)D * L);
        if (cflo.lambda_out) *cflo.lambda_out = L;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Uneven batches: one persistent launch over a size-sorted list of work units.
// A unit fills one 256-thread workgroup with patches of one size (one 16^3,
// four 8^3 or sixteen 4^3 patches); workgroups take units round-robin
// (unit u -> workgroup u mod gridDim.x), biggest units first, so the launch
// needs no atomics and its schedule is fixed.  Every patch takes its own
// time step (local time stepping, kLocalDt).
// ---------------------------------------------------------------------------
constexpr int kMixedNT = 256;
// A unit of 8^3 or 4^3 patches is run wave by wave: each of the four waves
// marches its own 8^3 patch, or its own four 4^3 patches, with the one-wave
// body (its LDS slot private, its phases ordered by wavefront fences, its
// patch values in scalar registers); a 16^3 patch takes the whole
// workgroup.
template <int P>
using MixedGeo = Geo<3, P, P == 16 ? kMixedNT : 64, 1>;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// Wave w owns LDS elements [w W, (w + 1) W) and reduction entries
// [w R, (w + 1) R) for both per-wave sizes (W, R the larger of their needs),
// so a wave may go on from its 8^3 units to 4^3 units while the others still
// march: no region of one wave overlaps another's.
constexpr int kMixedWaveLds = cmax(MixedGeo<8>::PPW * MixedGeo<8>::SLOT,
                                   MixedGeo<4>::PPW * MixedGeo<4>::SLOT);
constexpr int kMixedWaveRed = cmax(MixedGeo<8>::NRED, MixedGeo<4>::NRED);
constexpr int kMixedLds = cmax(MixedGeo<16>::SLOT, (kMixedNT / 64) * kMixedWaveLds);
constexpr int kMixedRed = cmax(MixedGeo<16>::NRED, (kMixedNT / 64) * kMixedWaveRed);

// The work list holds the 16^3 units first, then the 8^3 ones, then the 4^3
// ones (u8 and u4: the first unit of each of the two later classes, from the
// host plan).  Each size has its own loop: with the three bodies in one loop
// the kernel needed 209 registers (two waves per SIMD); in three loops it
// fits three waves per SIMD (167 registers, a few bytes of spills).  A unit
// whose size or run does not match its range is skipped.
template <typename T, bool NTS>
__global__ void __launch_bounds__(kMixedNT) __attribute__((amdgpu_waves_per_eu(3)))
fv_mixed_kernel(const fv_patch* __restrict__ patches, int64_t n,
                const int64_t* __restrict__ neighbours, const T* __restrict__ qin,
                int64_t qin_len, T* __restrict__ qout, int64_t qout_len, T gamma, double cfl,
                double* __restrict__ max_eig, const int64_t* __restrict__ order,
                const fv_work_unit* __restrict__ units, int64_t n_units, int64_t u8,
                int64_t u4) {
  __shared__ T lds[kMixedLds];
  __shared__ T red[kMixedRed];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  auto valid = [&](const fv_work_unit& un, int p) {
    return un.p == p && un.first >= 0 && un.count >= 0 && un.first <= n - un.count;
  };
  int64_t u = blockIdx.x;
  for (; u < u8; u += gridDim.x) {
    const fv_work_unit un = units[u];
    if (!valid(un, 16)) continue;  // the same for the whole workgroup
    const int64_t b = un.count > 0 ? order[un.first] : -1;
    update_body<T, 3, 16, kMixedNT, 1, true, kLocalDt, NTS>(
        patches, n, neighbours, qin, qin_len, qout, qout_len, 0, gamma, nullptr, max_eig, cfl,
        b, lds, red, tid);
    __syncthreads();  // the next unit reuses the LDS
  }
  // the waves of the later units march separately, each in its own LDS and
  // reduction region (the last 16^3 unit ended with a barrier)
  for (; u < u4; u += gridDim.x) {
    const fv_work_unit un = units[u];
    if (!valid(un, 8)) continue;
    const int64_t b = wave < un.count ? order[un.first + wave] : -1;
    update_body<T, 3, 8, 64, 1, true, kLocalDt, NTS>(
        patches, n, neighbours, qin, qin_len, qout, qout_len, 0, gamma, nullptr, max_eig, cfl,
        b, lds + wave * kMixedWaveLds, red + wave * kMixedWaveRed, lane);
  }
  for (; u < n_units; u += gridDim.x) {
    const fv_work_unit un = units[u];
    if (!valid(un, 4)) continue;
    using G = MixedGeo<4>;
    const int k = wave * G::PPW + lane / G::TPP;  // patch of the unit
    const int64_t b = k < un.count ? order[un.first + k] : -1;
    update_body<T, 3, 4, 64, 1, true, kLocalDt, NTS>(
        patches, n, neighbours, qin, qin_len, qout, qout_len, 0, gamma, nullptr, max_eig, cfl,
        b, lds + wave * kMixedWaveLds, red + wave * kMixedWaveRed, lane);
  }
}

// Outputs written per launch above this many bytes use non-temporal stores.
// MI355X keeps up to 256 MB in its Infinity Cache: a step whose input and
// output fit there together is read back from it by the next step, and
// streaming stores would send the output to HBM (a 4096 x 8^3 FP64 step, 84 MB
// out, is 27 % slower with them); larger steps cannot keep their output
// anyway, and streaming it leaves the caches to the face layers (5 % faster
// at 32768 x 8^3).
constexpr double kStreamingOutBytes = 128.0 * (1 << 20);
inline bool streaming_output(double bytes) { return bytes > kStreamingOutBytes; }

template <typename T, int D, int P, bool GATHER, int MODE, bool NTS, bool PUSH>
int launch(const fv_patch* patches, int64_t n, const int64_t* nbr, const T* qin, int64_t qin_len,
           T* qout, int64_t qout_len, int out_halo, T gamma, const double* dt_dev,
           double* max_eig, const CflOut& cflo, const int64_t* order, int64_t order_base,
           int64_t count, hipStream_t st) {
  using G = Geo<D, P>;
  static_assert(G::PPW * G::TPP <= G::NT, "workgroup too small");
  const int64_t blocks = (count + G::PPW - 1) / G::PPW;
  if (blocks == 0) return 0;
  const LaunchEvents& ev = launch_events();
  auto kernel = fv_update_kernel<T, D, P, GATHER, MODE, NTS, PUSH>;
  // The progress-based issue priority needs every workgroup resident at once
  // (later workgroups would start at the top priority and starve older
  // ones): workgroups per CU of this instance, queried once, times the CUs.
  static std::atomic<int> per_cu{-1};
  int wpc = per_cu.load(std::memory_order_relaxed);
  if (wpc < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kernel),
                                                     G::NT, 0) != hipSuccess)
      nb = 0;
    per_cu.store(nb, std::memory_order_relaxed);
    wpc = nb;
  }
  const int cus = device_cu_count();
  const int prio = wpc > 0 && cus > 0 && blocks <= (int64_t)wpc * cus;
  // with caller events the dispatch packet itself records them, so they time
  // the kernel's execution and nothing around it
  hipExtLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(G::NT), 0, st, ev.start, ev.stop, 0,
                        patches, n, nbr, qin, qin_len, qout, qout_len, out_halo, gamma, dt_dev,
                        max_eig, cflo, order, order_base, count, prio);
  return 0;
}

template <typename T, bool GATHER, int MODE, bool PUSH = false>
int dispatch(const fv_patch* patches, int64_t n, const int64_t* nbr, const T* qin,
             int64_t qin_len, T* qout, int64_t qout_len, int out_halo, int dim, int p,
             double gamma, const double* dt_dev, double* max_eig, const CflOut& cflo,
             const int64_t* order, int64_t order_base, int64_t count, hipStream_t st) {
  const bool nts = streaming_output((double)count * (dim + 2) * ipow(p, dim) * sizeof(T));
#define FV_CASE(DD, PP)                                                                        \
  if (dim == DD && p == PP)                                                                    \
    return nts ? launch<T, DD, PP, GATHER, MODE, true, PUSH>(                                 \
                     patches, n, nbr, qin, qin_len, qout, qout_len, out_halo, T(gamma), dt_dev, \
                     max_eig, cflo, order, order_base, count, st)                              \
               : launch<T, DD, PP, GATHER, MODE, false, PUSH>(                                \
                     patches, n, nbr, qin, qin_len, qout, qout_len, out_halo, T(gamma), dt_dev, \
                     max_eig, cflo, order, order_base, count, st);
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

}  // namespace

template <typename T>
int launch_update(const fv_patch* patches, int64_t n, const T* qin, int64_t qin_len, T* qout,
                  int64_t qout_len, int out_halo, int dim, int p, double gamma,
                  const double* dt_dev, double* max_eig, hipStream_t st) {
  return dispatch<T, false, kPlain>(patches, n, nullptr, qin, qin_len, qout, qout_len, out_halo,
                                    dim, p, gamma, dt_dev, max_eig, CflOut{}, nullptr, 0, n, st);
}

template <typename T>
int launch_update_gather(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                         const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int out_halo,
                         int dim, int p, double gamma, const double* dt_dev, double* max_eig,
                         hipStream_t st) {
  return dispatch<T, true, kPlain>(patches, n, neighbours, qin, qin_len, qout, qout_len,
                                   out_halo, dim, p, gamma, dt_dev, max_eig, CflOut{}, nullptr, 0,
                                   n, st);
}

template <typename T>
int launch_step_gather(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                       const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int dim, int p,
                       double gamma, const double* dt_dev, double* max_eig, const CflOut& cflo,
                       hipStream_t st) {
  return dispatch<T, true, kGlobalCfl>(patches, n, neighbours, qin, qin_len, qout, qout_len, 0,
                                       dim, p, gamma, dt_dev, max_eig, cflo, nullptr, 0, n, st);
}

template <typename T>
int launch_step_pipelined(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                          const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int dim,
                          int p, double gamma, double* max_eig, const CflOut& cflo,
                          hipStream_t st) {
  return dispatch<T, true, kPipelinedCfl>(patches, n, neighbours, qin, qin_len, qout, qout_len, 0,
                                          dim, p, gamma, cflo.dt_in, max_eig, cflo, nullptr, 0, n,
                                          st);
}

template <typename T>
int launch_step_halo(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                     const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int dim, int p,
                     double gamma, const double* dt_dev, double* max_eig, const CflOut& cflo,
                     hipStream_t st) {
  return dispatch<T, false, kGlobalCfl, true>(patches, n, neighbours, qin, qin_len, qout,
                                              qout_len, 1, dim, p, gamma, dt_dev, max_eig, cflo,
                                              nullptr, 0, n, st);
}
template <typename T>
int launch_step_local(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                      const fv_mixed_plan& plan, const T* qin, int64_t qin_len, T* qout,
                      int64_t qout_len, double gamma, double cfl, double* max_eig, int schedule,
                      int grid, hipStream_t st) {
  const LaunchEvents& ev = launch_events();
  // the whole step's output decides the store kind, for every launch of it
  double out_bytes = 0.0;
  for (int c = 0; c < 3; ++c)
    out_bytes += (double)plan.class_count[c] * 5.0 * ipow(plan.class_p[c], 3) * sizeof(T);
  const bool nts = streaming_output(out_bytes);
  if (schedule == FV_SCHED_PERSISTENT) {
    int64_t g = grid > 0 ? grid : plan.n_units;
    if (g > plan.n_units) g = plan.n_units;
    if (g < 1) return 0;
    // unit ranges of the size classes, as fv_plan_mixed lays them out
    int64_t bounds[3], acc = 0;
    for (int c = 0; c < 3; ++c) {
      const int ppu = mixed_patches_per_unit(plan.class_p[c]);
      acc += ppu > 0 ? (plan.class_count[c] + ppu - 1) / ppu : 0;
      bounds[c] = acc;
    }
    const int64_t u8 = bounds[0], u4 = bounds[1];
    if (nts)
      hipExtLaunchKernelGGL((fv_mixed_kernel<T, true>), dim3((unsigned)g), dim3(kMixedNT), 0, st,
                            ev.start, ev.stop, 0, patches, n, neighbours, qin, qin_len, qout,
                            qout_len, T(gamma), cfl, max_eig, plan.order, plan.units,
                            plan.n_units, u8, u4);
    else
      hipExtLaunchKernelGGL((fv_mixed_kernel<T, false>), dim3((unsigned)g), dim3(kMixedNT), 0,
                            st, ev.start, ev.stop, 0, patches, n, neighbours, qin, qin_len, qout,
                            qout_len, T(gamma), cfl, max_eig, plan.order, plan.units,
                            plan.n_units, u8, u4);
    return 0;
  }
  // per size: one launch over each class's contiguous range of the sorted
  // order; patch-wise: one launch per patch
  CflOut co;
  co.cfl = cfl;
  for (int c = 0; c < 3; ++c) {
    const int64_t first = plan.class_first[c], count = plan.class_count[c];
    if (count <= 0) continue;
    const int64_t per = schedule == FV_SCHED_PATCHWISE ? 1 : count;
    for (int64_t k = 0; k < count; k += per) {
      int rc = FV_EUNSUPPORTED;
#define FV_CLASS(PP)                                                                          \
  if (plan.class_p[c] == PP)                                                                  \
    rc = nts ? launch<T, 3, PP, true, kLocalDt, true, false>(patches, n, neighbours, qin, qin_len, \
                                                      qout, qout_len, 0, T(gamma), nullptr,   \
                                                      max_eig, co, plan.order, first + k,     \
                                                      per, st)                                \
             : launch<T, 3, PP, true, kLocalDt, false, false>(patches, n, neighbours, qin, qin_len, \
                                                       qout, qout_len, 0, T(gamma), nullptr,  \
                                                       max_eig, co, plan.order, first + k,    \
                                                       per, st);
      FV_CLASS(4)
      FV_CLASS(8)
      FV_CLASS(16)
#undef FV_CLASS
      if (rc) return rc;
    }
  }
  return 0;
}

#define FV_INSTANTIATE(T)                                                                     \
  template int launch_update<T>(const fv_patch*, int64_t, const T*, int64_t, T*, int64_t, int,  \
                                int, int, double, const double*, double*, hipStream_t);        \
  template int launch_update_gather<T>(const fv_patch*, int64_t, const int64_t*, const T*,      \
                                       int64_t, T*, int64_t, int, int, int, double,             \
                                       const double*, double*, hipStream_t);                    \
  template int launch_step_gather<T>(const fv_patch*, int64_t, const int64_t*, const T*,        \
                                     int64_t, T*, int64_t, int, int, double, const double*,     \
                                     double*, const CflOut&, hipStream_t);                      \
  template int launch_step_pipelined<T>(const fv_patch*, int64_t, const int64_t*, const T*,     \
                                        int64_t, T*, int64_t, int, int, double, double*,        \
                                        const CflOut&, hipStream_t);                            \
  template int launch_step_local<T>(const fv_patch*, int64_t, const int64_t*,                   \
                                    const fv_mixed_plan&, const T*, int64_t, T*, int64_t,       \
                                    double, double, double*, int, int, hipStream_t);

}  // namespace fvk
