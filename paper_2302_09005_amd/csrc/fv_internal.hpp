// Internal declarations shared by the translation units of libfv (not part of
// the C ABI): patch geometry constants and the per-kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fv.h"

#ifndef FV_LDS_CPAD
#define FV_LDS_CPAD 0
#endif
#ifndef FV_LDS_FPAD
#define FV_LDS_FPAD 0
#endif
#ifndef FV_ZSPLIT_3D8
#define FV_ZSPLIT_3D8 1
#endif

namespace fvk {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Chunks along the marching axis per patch in the single-size update
// kernels: each chunk marches ceil(P / ZS) planes (the last one fewer when ZS
// does not divide P), in a wave of its own when a plane has 64 volumes, else
// in its own group of lanes of the patch's wave.  2-D patches of 16^2, 17^2
// and 32^2 fill one wave that way (4, 3 and 2 chunks), so a patch is marched
// in 4, 6 or 16 rows instead of 16, 17 or 32.
template <int D, int P>
constexpr int zsplit() {
  return D == 3 && P == 8    ? FV_ZSPLIT_3D8
         : D == 2 && P == 16 ? 4
         : D == 2 && P == 17 ? 3
         : D == 2 && P == 32 ? 2
                             : 1;
}

// Geometry of a D-dimensional patch of P^D volumes with a halo of one volume,
// and of the plane-marching update that processes it.
//
// The update walks the last axis (z in 3-D, y in 2-D): one lane owns one
// column of volumes along that axis, so a patch chunk occupies P^(D-1) lanes
// ("LANES").  A patch is marched in ZS chunks of P / ZS planes each, side by
// side, so it takes TPP = ZS * LANES threads, and PPW patches share one
// workgroup of NTW threads when TPP < NTW (NTW = 64 for the single-size
// kernels, 256 in the mixed-size persistent kernel).
template <int D, int P, int NTW = 64, int ZS = zsplit<D, P>()>
struct Geo {
  static constexpr int S = D + 2;                    // unknowns
  static constexpr int W = P + 2;                    // volumes per axis incl. halo
  static constexpr int VIN = ipow(W, D);             // volumes of a halo'd block
  static constexpr int VOUT = ipow(P, D);            // volumes of a compact block
  static constexpr int SM = ipow(W, D - 1);          // halo'd stride of the marching axis
  static constexpr int SMO = ipow(P, D - 1);         // compact stride of the marching axis
  static constexpr int LANES = ipow(P, D - 1);       // lanes per chunk (one column each)
  static constexpr int CHUNKS = ZS;                  // chunks per patch
  static constexpr int PC = (P + ZS - 1) / ZS;       // planes per chunk (the last: P - (ZS-1) PC)
  static constexpr int TPP = ZS * LANES;             // threads per patch
  static constexpr int PPW = TPP >= NTW ? 1 : NTW / TPP;  // patches per workgroup
  static constexpr int NT = ((PPW * TPP + 63) / 64) * 64; // workgroup size
  static constexpr int RING = D == 3 ? 4 * P : 2;    // face-halo volumes around one plane
  static constexpr int NEXTRA = D == 3 ? 2 * P : 1;  // in-plane faces on the high boundary
  static constexpr int NCELL = LANES + RING;         // volumes of one plane incl. its ring
  static constexpr int NV = S + 3;                   // values kept per volume: q, 1/rho, p, c
  static constexpr int NF = LANES + (D == 3 ? P : 1);  // in-plane faces per axis and plane
  // LDS strides of one value across a plane's volumes and faces (padded so
  // that the two halves of a paired 64-bit access fall in different banks)
  static constexpr int CST = NCELL + FV_LDS_CPAD;
  static constexpr int FST = NF + FV_LDS_FPAD;
  static constexpr int CELLBUF = NV * CST;
  static constexpr int FACEBUF = (D - 1) * S * FST;
  static constexpr int SLOT = CELLBUF > FACEBUF ? CELLBUF : FACEBUF;  // LDS elements per chunk
  // reduction slots: one per wave of the workgroup, or one per chunk
  static constexpr int NRED = NT / 64 > PPW * ZS ? NT / 64 : PPW * ZS;
  static_assert(RING <= LANES, "every ring volume needs its own lane");
  static_assert(ZS == 1 || LANES == 64 || ZS * LANES <= 64,
                "chunks are whole waves, or lane groups of one wave");
  static_assert(P % ZS == 0 || ZS * LANES <= 64, "uneven chunks only as lane groups of one wave");
  static_assert((ZS - 1) * PC < P, "every chunk has a plane");
  static_assert(NEXTRA <= LANES, "every high-boundary face needs its own lane");
};

// Outputs of the CFL step fused into the update (see fv_step_gather).  The
// workspace holds (1 + groups) slot sets of kCflSlot words: words 0,
// kCflWord and 2 kCflWord of a set = arrival count, max lambda bits, max
// (inf - h) bits; set 0 is the top of the reduction tree (its count only),
// set g+1 serves group g of kCflGroup consecutive workgroups.
constexpr int kCflGroup = 64;
constexpr int kCflWord = 32;  // each word on a 256-byte line of its own
constexpr int kCflSlot = 3 * kCflWord;
struct CflOut {
  double cfl = 0.0;
  double* dt_next = nullptr;
  double* lambda_out = nullptr;
  unsigned long long* ws = nullptr;
  // pipelined step (kPipelinedCfl): slot sets 0..2 of kPipeSlots slots each;
  // this launch reads set (phase + 2) % 3 (unless dt_in is given), folds into
  // set phase and clears set (phase + 1) % 3; dt_used receives the step it took
  int phase = 0;
  const double* dt_in = nullptr;
  double* dt_used = nullptr;
};

// Workgroups of the update launch and the workspace words fv_step_gather needs.
int64_t update_workgroups(int dim, int p, int64_t n);
inline int64_t step_workspace_words(int64_t workgroups) {
  return (int64_t)kCflSlot * (1 + (workgroups + kCflGroup - 1) / kCflGroup);
}
// The pipelined step's three slot sets: workgroup w folds into slot
// w mod kPipeSlots of a set (no arrival counting, so a slot only needs to
// keep up with the rate at which workgroups finish), and every wave of the
// next launch reads the kPipeSlots slots of that set: a fixed cost per wave
// whatever the batch size.
constexpr int kPipeSlots = 16;
inline int64_t pipelined_workspace_words() { return (int64_t)3 * kPipeSlots * kCflSlot; }

// Events recorded by the dispatch of the next update launches (set through
// fv_set_launch_events; null = not recorded).  Per calling thread.
struct LaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
LaunchEvents& launch_events();

// Compute units of the current device (queried once per device and kept; 0
// if the query fails).
int device_cu_count();

// Time-step handling of an update launch.
enum StepMode : int {
  kPlain = 0,      // dt from dt_dev or the descriptor; nothing else
  kGlobalCfl = 1,  // plus the next global CFL step (fv_step_gather)
  kLocalDt = 2,    // per-patch dt from the descriptor; the launch advances the
                   // descriptor's t by it and stores the patch's next local
                   // CFL step in its dt (local time stepping)
  kPipelinedCfl = 3,  // dt from the maxima the previous launch folded (or a
                      // given dt); this launch's maxima folded for the next
                      // one, with no wait for the fold at the end
};

// Status for launchers: 0 ok, FV_EUNSUPPORTED when (dim, p) has no instance.
// Update launchers, instantiated for double and float state.
template <typename T>
int launch_update(const fv_patch* patches, int64_t n, const T* qin, int64_t qin_len, T* qout,
                  int64_t qout_len, int out_halo, int dim, int p, double gamma,
                  const double* dt_dev, double* max_eig, hipStream_t st);
template <typename T>
int launch_update_gather(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                         const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int out_halo,
                         int dim, int p, double gamma, const double* dt_dev, double* max_eig,
                         hipStream_t st);
template <typename T>
int launch_step_gather(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                       const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int dim, int p,
                       double gamma, const double* dt_dev, double* max_eig, const CflOut& cflo,
                       hipStream_t st);
template <typename T>
int launch_step_pipelined(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                          const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int dim,
                          int p, double gamma, double* max_eig, const CflOut& cflo,
                          hipStream_t st);

// One whole step of the paper's layout (halo'd input and output blocks): the
// update, its face-halo exchange pushed into the output halos, and the next
// CFL step (double state only).
template <typename T>
int launch_step_halo(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                     const T* qin, int64_t qin_len, T* qout, int64_t qout_len, int dim, int p,
                     double gamma, const double* dt_dev, double* max_eig, const CflOut& cflo,
                     hipStream_t st);

// Uneven batches (3-D, p in {4, 8, 16}): patches per 256-thread work unit,
// and one step with local time stepping under the given schedule.
int mixed_patches_per_unit(int p);
template <typename T>
int launch_step_local(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                      const fv_mixed_plan& plan, const T* qin, int64_t qin_len, T* qout,
                      int64_t qout_len, double gamma, double cfl, double* max_eig, int schedule,
                      int grid, hipStream_t st);

template <typename T>
int launch_patch_max(const fv_patch* patches, int64_t n, const T* q, int64_t q_len, int q_halo,
                     int which, int dim, int p, double gamma, double* per_patch, hipStream_t st);

template <typename T>
int launch_totals(const fv_patch* patches, int64_t n, const T* q, int64_t q_len, int q_halo,
                  int which, int dim, int p, double* per_patch, double* totals, hipStream_t st);

int launch_reduce_cfl(const fv_patch* patches, int64_t n, const double* per_patch, int dim,
                      double cfl, double* lambda_out, double* dt_out, hipStream_t st);

int launch_local_dt(fv_patch* patches, int64_t n, const double* per_patch, int dim, double cfl,
                    hipStream_t st);

int launch_fill_halo_f64(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                         double* q, int64_t q_len, int which, int dim, int p, hipStream_t st);

bool update_supported(int dim, int p);

// Learned face-flux correction (2-D): training data, training, inference.
int launch_face_flux_accumulate(const double* qf, int npx, int npy, int p, int r, int bc,
                                double gamma, double weight, double* accx, double* accy,
                                hipStream_t st);
int launch_coarse_grain(const double* qf, int npx, int npy, int p, int r, double* qc,
                        hipStream_t st);
int launch_face_samples(const double* qc, int npx, int npy, int p, int bc, double gamma,
                        const double* accx, const double* accy, float* feats, float* targ,
                        float* ind, hipStream_t st);
int launch_column_stats(const float* x, int64_t x_rows, int64_t n, int cols, int mode,
                        const int64_t* rows, float* mean, float* scale, hipStream_t st);
int mlp_blob_words();
int mlp_trained_words();
int mlp_workspace_words(int batch);
int launch_mlp_train_step(float* blob, float* adam, int step, float lr, const float* feats,
                          const float* targ, int64_t n_rows, const int64_t* idx, int batch,
                          float* ws, float* grad_out, hipStream_t st);
int launch_mlp_forward(const float* blob, const float* feats, int64_t n, float* out,
                       hipStream_t st);
int launch_update_learned_2d(const fv_patch* patches, int64_t n, const int64_t* neighbours,
                             const double* qin, int64_t qin_len, double* qout, int64_t qout_len,
                             double gamma, const double* dt_dev, const float* blob,
                             double threshold, double* max_eig, hipStream_t st);

}  // namespace fvk
