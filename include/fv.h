/*
 * fv.h -- C ABI of the MI355X (gfx950) batched Finite Volume patch update.
 *
 * The operation is the patch kernel of "GPU Offloading in ExaHyPE Through C++
 * Standard Algorithms" (arXiv 2302.09005): for a batch of N small Cartesian
 * patches, each stored with a halo layer of one volume, advance the first-order
 * hyperbolic system dq/dt + sum_j d f^j(q)/dx_j = 0 (Section 2, eq. (1)) by one
 * explicit Euler step with the Rusanov flux (Section 2, eqs. (3)-(5)), for the
 * compressible Euler equations (Section 2, eq. (2); s = d + 2 unknowns), and
 * return each patch's largest eigenvalue (Algorithm 1, last step; Section 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Unknowns: (rho, j_x, j_y[, j_z], E), s = d + 2.  Ideal gas,
 *    p = (gamma - 1)(E - |j|^2 / (2 rho)); energy flux (E + p) j_dir / rho.
 *  * Patch block layout: unknown-major, x fastest, [s][z][y][x].  A block with
 *    halo covers (p + 2)^d volumes, a block without covers p^d volumes.  Only
 *    the 2d face-halo layers are ever read; edge and corner halo volumes are
 *    never read and may hold anything (NaN included).
 *  * Buffers: one flat array per role; patches sit at element offsets given by
 *    their descriptors.  Lengths (`*_len`) are in elements and bound every
 *    access: a descriptor whose block does not fit is skipped (see below).
 *  * Pointers named `*_dev` or documented as device pointers are HIP device
 *    memory owned by the caller; the library never allocates, frees, copies
 *    to the host or synchronises.  Every call is asynchronous on `stream`
 *    (a hipStream_t; NULL = the null stream); outputs are valid once the
 *    stream has reached the call.
 *  * Return value: FV_OK (0) or a negative FV_E* code.  Argument errors are
 *    detected on the host before anything is launched; a launch failure
 *    returns FV_EHIP.  fv_last_error() describes the last failure of the
 *    calling thread.  No C++ exception crosses this interface, and there is
 *    no CPU fallback: without a usable HIP device every compute call fails.
 *  * NaN propagation: negative pressure or density, or NaN input, is not
 *    checked per volume; it shows up as NaN in the per-patch and global
 *    maxima (all maxima propagate NaN).
 */
#ifndef FV_H
#define FV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FV_OK            0
#define FV_EINVAL       -1   /* invalid argument (null pointer, bad sizes, s != d + 2, ...) */
#define FV_EUNSUPPORTED -2   /* valid but not built: (dim, p) without a kernel instance     */
#define FV_EHIP         -3   /* HIP runtime error while launching                           */

/* Offsets selector for calls that read or write one buffer of a batch. */
#define FV_OFFSETS_IN    0   /* use fv_patch.q_in  */
#define FV_OFFSETS_OUT   1   /* use fv_patch.q_out */

/*
 * One patch of a batch: the device-side counterpart of the paper's per-patch
 * data (Appendix A: cell centre and size, QIn/QOut pointers, t, dt; the
 * paper's "cell" is the spacetree cube that hosts a patch).  64 bytes.
 */
typedef struct fv_patch {
  int64_t q_in;    /* element offset of this patch's input block [s][(p+2)^d]      */
  int64_t q_out;   /* element offset of this patch's output block                  */
  int32_t p;       /* volumes per axis; must equal the batch-wide p of the call    */
  int32_t flags;   /* reserved, 0                                                  */
  double  dx[3];   /* volume width per axis (cube size / p); unused axes ignored   */
  double  dt;      /* time-step size of this patch (local time stepping)           */
  double  t;       /* time stamp; not used by the Euler update                     */
} fv_patch;

/* Description of the last failure on the calling thread ("" if none). */
const char* fv_last_error(void);

/* ABI version (increments on incompatible change). */
int fv_abi_version(void);

/* 1 if kernels for (dim, p) are built into this library, else 0. */
int fv_supported(int dim, int p);

/*
 * Kernel timing: until called again, every update launch of the calling
 * thread (fv_batch_update, fv_batch_update_gather, fv_step_gather,
 * fv_step_gather_pipelined, fv_step_halo, fv_step_local, the learned
 * update, and their _f32 forms) has its
 * dispatch record start_event when the kernel begins and stop_event when it
 * ends (hipEvent_t handles created by the caller), so the elapsed time
 * between them is the kernel's execution alone.  Pass two NULLs to stop.
 * Returns FV_EINVAL if exactly one is NULL.
 */
int fv_set_launch_events(void* start_event, void* stop_event);

/*
 * Host-side validation of a descriptor array (a HOST copy), for callers that
 * build descriptors themselves.  Checks p, finite positive dx and dt >= 0,
 * that every input/output block lies inside [0, len) (q_in_halo/q_out_halo:
 * 1 for blocks [s][(p+2)^d], 0 for [s][p^d]), and that output blocks do not
 * overlap each other.  Returns FV_OK or FV_EINVAL (with the first
 * offending patch named by fv_last_error()).  Touches no device.
 */
int fv_check_patches(const fv_patch* host_patches, int64_t n_patches,
                     int dim, int p, int q_in_halo, int q_out_halo,
                     int64_t q_in_len, int64_t q_out_len);

/*
 * fv_batch_update -- one explicit Euler step of every patch (Section 2,
 * eqs. (3)-(5); Algorithm 1 without its non-conservative-product step, which
 * is zero for Euler).  For each patch b and interior volume i:
 *
 *   Q_out[i] = Q_in[i] - sum_{j=x,y[,z]} (dt_b / dx_{b,j}) (F_j(i+1/2) - F_j(i-1/2)),
 *   F_j(L, R) = 1/2 [ f^j(L) + f^j(R) - max(|u_j(L)| + c(L), |u_j(R)| + c(R)) (R - L) ],
 *
 * the sum taken in axis order.  Each face flux is computed once and used by
 * both adjacent volumes.
 *
 * patches     device array [n_patches] of descriptors (read only)
 * n_patches   >= 0; 0 is a no-op
 * q_in        device, input blocks [s][(p+2)^d] at patches[b].q_in (read only)
 * q_out       device, output blocks at patches[b].q_out: [s][p^d] when
 *             q_out_halo == 0, or [s][(p+2)^d] when q_out_halo == 1 (then only
 *             interior volumes are written; the halo is left untouched).
 *             Must not overlap q_in.
 * dim, p      2 or 3; volumes per axis (fv_supported(dim, p) must hold)
 * halo        halo width; must be 1
 * s           number of unknowns; must be dim + 2
 * gamma       ratio of specific heats (> 1)
 * dt_dev      device pointer to one double overriding every patch's dt, or
 *             NULL to use patches[b].dt (lets a CFL step stay on the device)
 * max_eig     device array [n_patches]: largest eigenvalue max_j(|u_j| + c)
 *             over the interior of the NEW state of each patch, or NULL.
 *             A patch whose descriptor fails the device-side check (p differs
 *             from the call's p, or a block outside its buffer) is not
 *             updated and gets NaN here.
 */
int fv_batch_update(const fv_patch* patches, int64_t n_patches,
                    const double* q_in, int64_t q_in_len,
                    double* q_out, int64_t q_out_len, int q_out_halo,
                    int dim, int p, int halo, int s, double gamma,
                    const double* dt_dev, double* max_eig, void* stream);

/*
 * fv_batch_update_gather -- the same step as fv_batch_update, with the
 * face-halo exchange fused into the gather (Section 2: keeping the halo
 * consistent is the engine's job; here it is done while the tiles are read).
 * Patch blocks carry NO halo: q_in holds [s][p^d] at patches[b].q_in, and
 * each face-halo volume the update needs is read from the facing interior
 * volume of the neighbouring patch.  The result equals fv_fill_halo followed
 * by fv_batch_update on the same data stored with halos.
 *
 * neighbours  device int64 [n_patches][2*dim], face order -x, +x, -y, +y,
 *             -z, +z; entries in [0, n_patches) (periodic domains use
 *             wrapped indices) or -1 for a transmissive (zero-gradient)
 *             boundary, where the patch's own boundary volume is used.
 * q_out       [s][p^d] (q_out_halo == 0) or [s][(p+2)^d] (== 1, interior
 *             written) at patches[b].q_out; must not overlap q_in.
 * Other arguments as for fv_batch_update.  A patch whose own or neighbour
 * descriptors fail the device-side check (p mismatch, block outside q_in,
 * neighbour index outside [-1, n_patches)) is not updated and gets NaN in
 * max_eig.
 */
int fv_batch_update_gather(const fv_patch* patches, int64_t n_patches,
                           const int64_t* neighbours,
                           const double* q_in, int64_t q_in_len,
                           double* q_out, int64_t q_out_len, int q_out_halo,
                           int dim, int p, int s, double gamma,
                           const double* dt_dev, double* max_eig, void* stream);

/*
 * fv_step_gather -- one whole explicit step of the batch in ONE launch: the
 * update of fv_batch_update_gather (compact blocks, halo exchange fused into
 * the gather) and the CFL time step of the next step, computed from the
 * per-patch maxima of the new state exactly as fv_cfl_timestep does
 * (Lambda = max_b max_eig[b], dt = cfl * min dx / (dim * Lambda)).
 *
 * dt_dev      device [1]: the time step of THIS step (required)
 * max_eig     device [n_patches] or NULL: per-patch maxima of the new state
 * dt_next     device [1]: the time step for the next step (required; must not
 *             alias dt_dev -- alternate two buffers between steps)
 * lambda_out  device [1] or NULL: Lambda of the new state
 * workspace   device uint64 [workspace_words], at least
 *             fv_step_workspace_words(n_patches, dim, p) words (FV_EINVAL
 *             otherwise), all zero before the first call; every call leaves
 *             it zero again.  Calls that overlap in time (different streams)
 *             must use different workspaces.
 * q_out is [s][p^d] (compact).  Other arguments as for
 * fv_batch_update_gather.  The reduction is an integer maximum of IEEE bit
 * patterns (all values are >= 0 or NaN), so the result does not depend on the
 * order in which workgroups finish; a NaN maximum gives a NaN time step.
 */
int fv_step_gather(const fv_patch* patches, int64_t n_patches, const int64_t* neighbours,
                   const double* q_in, int64_t q_in_len, double* q_out, int64_t q_out_len,
                   int dim, int p, int s, double gamma, double cfl,
                   const double* dt_dev, double* max_eig, double* dt_next,
                   double* lambda_out, uint64_t* workspace, int64_t workspace_words,
                   void* stream);

/* Size in uint64 words of the workspace fv_step_gather needs (0 on bad
 * arguments).  A few words per 64 workgroups: small, allocate once. */
int64_t fv_step_workspace_words(int64_t n_patches, int dim, int p);

/*
 * fv_step_gather_pipelined -- the step of fv_step_gather in ONE launch, with
 * the CFL reduction moved across the launch boundary: a call takes the time
 * step from the per-patch maxima the PREVIOUS call folded (Lambda = max_b of
 * the previous new state's maxima, dt = cfl * min dx / (dim * Lambda), the
 * same value fv_step_gather writes to dt_next, bit for bit), and folds the
 * maxima of its own new state for the next call with atomic maxima that
 * nothing waits for.  The fused step's arrival counting at the end of the
 * launch (four dependent device-scope round trips after the last patch) is
 * gone; the previous maxima are loaded with the descriptors and reduced in
 * the wave before the first update.  Same update (Section 2, eqs. (3)-(5),
 * Algorithm 1), same CFL rule (Section 4: the step size comes from the
 * maximal eigenvalue), same results as a run of fv_step_gather.
 *
 * phase       0, 1 or 2: the calls of one run pass 0, 1, 2, 0, 1, ... (the
 *             workspace holds three slot sets: a call reads set (phase+2)%3,
 *             folds into set `phase` and clears set (phase+1)%3)
 * dt_in       device [1] or NULL: the time step to take; given on the FIRST
 *             call of a run (there are no previous maxima), NULL afterwards
 * dt_used     device [1] or NULL: receives the time step this call took
 * lambda_out  device [1] or NULL: receives the Lambda that time step came
 *             from (not written when dt_in is given)
 * max_eig     device [n_patches] or NULL: per-patch maxima of the new state
 * workspace   device uint64 [workspace_words], at least
 *             fv_step_pipelined_workspace_words(n_patches, dim, p) words
 *             (FV_EINVAL otherwise), all zero before the first call of a run
 *             (a run that continues the phase sequence of an earlier one may
 *             reuse it as that run left it); every call of a run passes the
 *             same batch (patches, n_patches).  Calls that overlap in time
 *             must use different workspaces.
 * The other arguments are as for fv_step_gather; NaN maxima give a NaN time
 * step, as there.  The time step for a call after the last one, if wanted, is
 * fv_cfl_timestep over max_eig.
 */
int fv_step_gather_pipelined(const fv_patch* patches, int64_t n_patches,
                             const int64_t* neighbours, const double* q_in, int64_t q_in_len,
                             double* q_out, int64_t q_out_len, int dim, int p, int s,
                             double gamma, double cfl, int phase, const double* dt_in,
                             double* dt_used, double* max_eig, double* lambda_out,
                             uint64_t* workspace, int64_t workspace_words, void* stream);

/* Size in uint64 words of the workspace fv_step_gather_pipelined needs (0 on
 * bad arguments): three sets of 16 slots, 4608 words for any batch size. */
int64_t fv_step_pipelined_workspace_words(int64_t n_patches, int dim, int p);

/*
 * fv_step_gather_noalloc -- fv_step_gather for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc): the same kernel and results, bit for bit, with the
 * workspace taken from a buffer inside the library instead of an argument.
 *
 * The buffer is a static device array of FV_NOALLOC_SCRATCH_WORDS uint64
 * words (3 MiB) that every GPU the library runs on holds until the process
 * ends.  The first call on a device looks up its address there and clears it
 * with a kernel on `stream`; nothing is allocated, freed or synchronised on
 * any call.  A batch whose workspace need, fv_step_workspace_words(n_patches,
 * dim, p), exceeds FV_NOALLOC_SCRATCH_WORDS is refused with FV_EINVAL (e.g.
 * 3-D 8^3: at most 262 080 patches).  Every call leaves the words it used at
 * zero again.  All calls on one GPU share the one array: calls that overlap in
 * time on one GPU (different streams, or different host threads) race and
 * give wrong time steps; serialise them, or use fv_step_gather with a
 * workspace per stream.  Arguments and outputs otherwise as for
 * fv_step_gather (FP64 state).
 */
#define FV_NOALLOC_SCRATCH_WORDS 393216
int fv_step_gather_noalloc(const fv_patch* patches, int64_t n_patches, const int64_t* neighbours,
                           const double* q_in, int64_t q_in_len, double* q_out, int64_t q_out_len,
                           int dim, int p, int s, double gamma, double cfl,
                           const double* dt_dev, double* max_eig, double* dt_next,
                           double* lambda_out, void* stream);

/*
 * fv_step_halo -- one whole explicit step of the paper's layout in ONE launch:
 * the update of fv_batch_update (input and output blocks both with halo,
 * [s][(p+2)^d]), the face-halo exchange of the NEW state (what fv_fill_halo
 * on q_out would do next) and the CFL time step of the next step (as in
 * fv_step_gather).  The exchange is pushed: when a patch has computed its new
 * boundary volumes it also stores them into the face halos that read them,
 * so the next step's input is complete when the launch ends, and no separate
 * halo pass reads the state again (Section 2: the engine keeps halos
 * consistent; here it is done while the update writes).
 *
 * neighbours  device int64 [n_patches][2*dim], as for fv_fill_halo; the table
 *             must be mutual: if neighbours[b][f] = a >= 0, then
 *             neighbours[a][f^1] = b (every conforming patch grid, periodic
 *             or not, has this property).  -1 = transmissive: the face halo
 *             repeats the patch's own boundary volume.  A patch with an entry
 *             that is not mutual, out of range, or names a patch whose
 *             descriptor fails the check, is not updated, pushes nothing and
 *             gets NaN in max_eig (so Lambda and dt_next are NaN too).
 * q_out       blocks [s][(p+2)^d] at patches[b].q_out: interior and face
 *             halo written, edge and corner halo volumes untouched.
 * Other arguments (dt_dev, max_eig, dt_next, lambda_out, workspace) as for
 * fv_step_gather.  Results equal fv_batch_update (q_out_halo = 1), then
 * fv_fill_halo on q_out, then fv_cfl_timestep, bit for bit.  FP64 state.
 */
int fv_step_halo(const fv_patch* patches, int64_t n_patches, const int64_t* neighbours,
                 const double* q_in, int64_t q_in_len, double* q_out, int64_t q_out_len,
                 int dim, int p, int halo, int s, double gamma, double cfl,
                 const double* dt_dev, double* max_eig, double* dt_next,
                 double* lambda_out, uint64_t* workspace, int64_t workspace_words,
                 void* stream);

/*
 * FP32 state (bulk flux and update arithmetic in single precision): the same
 * operations on float blocks.  The time step, the per-patch maxima written to
 * max_eig, Lambda and the CFL reduction stay FP64 (double outputs; the FP32
 * per-volume wave speeds are folded into FP64 maxima).  Arguments as for the
 * FP64 entry points above.
 */
int fv_batch_update_f32(const fv_patch* patches, int64_t n_patches,
                        const float* q_in, int64_t q_in_len,
                        float* q_out, int64_t q_out_len, int q_out_halo,
                        int dim, int p, int halo, int s, double gamma,
                        const double* dt_dev, double* max_eig, void* stream);
int fv_batch_update_gather_f32(const fv_patch* patches, int64_t n_patches,
                               const int64_t* neighbours,
                               const float* q_in, int64_t q_in_len,
                               float* q_out, int64_t q_out_len, int q_out_halo,
                               int dim, int p, int s, double gamma,
                               const double* dt_dev, double* max_eig, void* stream);
int fv_step_gather_f32(const fv_patch* patches, int64_t n_patches, const int64_t* neighbours,
                       const float* q_in, int64_t q_in_len, float* q_out, int64_t q_out_len,
                       int dim, int p, int s, double gamma, double cfl,
                       const double* dt_dev, double* max_eig, double* dt_next,
                       double* lambda_out, uint64_t* workspace, int64_t workspace_words,
                       void* stream);
int fv_step_gather_pipelined_f32(const fv_patch* patches, int64_t n_patches,
                                 const int64_t* neighbours, const float* q_in, int64_t q_in_len,
                                 float* q_out, int64_t q_out_len, int dim, int p, int s,
                                 double gamma, double cfl, int phase, const double* dt_in,
                                 double* dt_used, double* max_eig, double* lambda_out,
                                 uint64_t* workspace, int64_t workspace_words, void* stream);
int fv_max_eigenvalue_f32(const fv_patch* patches, int64_t n_patches,
                          const float* q, int64_t q_len, int q_halo, int which_offsets,
                          int dim, int p, int s, double gamma,
                          double* per_patch, double* global, void* stream);

/*
 * fv_conserved_totals / _f32 -- totals of the conserved unknowns (mass,
 * momentum, energy: the quantities eq. (3) conserves on a periodic domain)
 * over the interior volumes of all patches, accumulated in FP64 whatever the
 * state's precision, in a fixed order (deterministic for a given batch).
 * per_patch   device double [n_patches * s], required: per-patch totals
 * totals      device double [s] or NULL: sum over patches
 * q_halo, which_offsets as for fv_max_eigenvalue.  n_patches >= 1.  A patch
 * that fails the device-side check gets NaN totals.
 */
int fv_conserved_totals(const fv_patch* patches, int64_t n_patches,
                        const double* q, int64_t q_len, int q_halo, int which_offsets,
                        int dim, int p, int s, double* per_patch, double* totals, void* stream);
int fv_conserved_totals_f32(const fv_patch* patches, int64_t n_patches,
                            const float* q, int64_t q_len, int q_halo, int which_offsets,
                            int dim, int p, int s, double* per_patch, double* totals,
                            void* stream);

/*
 * Uneven batches with local time stepping (3-D, patches of 4^3, 8^3 and 16^3
 * volumes mixed in one batch; compact blocks; halo gathered from neighbours,
 * which must have the same p).  The paper's engine offloads N patches at a
 * time whatever their AMR level (Section 2, enclave tasking) and keeps a
 * time step per patch (Section 4, local adaptive time stepping; App. A
 * per-patch t and dt).
 *
 * A plan groups the patches by size: `order` lists the patch indices sorted
 * by p (16, 8, 4; stable), and each work unit is a run of `order` of one size
 * that fills one 256-thread workgroup (1 x 16^3, 4 x 8^3 or 16 x 4^3).
 * fv_plan_mixed builds it on the host from a HOST copy of the descriptors;
 * the caller uploads `order` and `units` and fills the device pointers.
 */
#define FV_SCHED_PER_SIZE   0   /* one launch per size class (batched loops)    */
#define FV_SCHED_PERSISTENT 1   /* one persistent launch over all work units    */
#define FV_SCHED_PATCHWISE  2   /* one launch per patch (the paper's patch-wise
                                   loop order, Section 3; for comparison only)  */

typedef struct fv_work_unit {
  int32_t p;       /* volumes per axis of the unit's patches          */
  int32_t count;   /* patches in the unit                             */
  int64_t first;   /* position of its first patch in `order`          */
} fv_work_unit;

typedef struct fv_mixed_plan {
  const int64_t* order;        /* device [n_patches]                                 */
  const fv_work_unit* units;   /* device [n_units]                                   */
  int64_t n_units;
  int32_t class_p[3];          /* sizes present, descending; 0 = unused class        */
  int64_t class_first[3];      /* first position in `order` of each class            */
  int64_t class_count[3];      /* patches of each class                              */
} fv_mixed_plan;

/*
 * Host: fill order[n_patches] and units[<= n_patches] (host arrays) and the
 * class fields of *plan (its device pointers are left for the caller).
 * Rejects p outside {4, 8, 16} and dim != 3.  Touches no device.
 */
int fv_plan_mixed(const fv_patch* host_patches, int64_t n_patches, int dim,
                  int64_t* order, fv_work_unit* units, fv_mixed_plan* plan);

/*
 * One step of every patch of an uneven batch with local time stepping: each
 * patch advances by its own descriptor dt (its t grows by dt) and stores its
 * next CFL step, dt = cfl * min dx / (dim * lambda_patch), from its new
 * state; max_eig (device [n_patches] or NULL) gets the per-patch maxima.
 * patches is written (t and dt only).  schedule: one of FV_SCHED_*;
 * persistent_workgroups: grid of the persistent launch (0 = one workgroup
 * per unit).  Every schedule gives bit-identical results.  Other arguments as for
 * fv_batch_update_gather with q_out compact.
 */
int fv_step_local(fv_patch* patches, int64_t n_patches, const int64_t* neighbours,
                  const fv_mixed_plan* plan,
                  const double* q_in, int64_t q_in_len, double* q_out, int64_t q_out_len,
                  int dim, int s, double gamma, double cfl, double* max_eig,
                  int schedule, int persistent_workgroups, void* stream);
int fv_step_local_f32(fv_patch* patches, int64_t n_patches, const int64_t* neighbours,
                      const fv_mixed_plan* plan,
                      const float* q_in, int64_t q_in_len, float* q_out, int64_t q_out_len,
                      int dim, int s, double gamma, double cfl, double* max_eig,
                      int schedule, int persistent_workgroups, void* stream);

/*
 * Local time steps from per-patch maxima: patches[b].dt = cfl * min dx /
 * (dim * per_patch[b]) for every patch (the first step of a run with local
 * time stepping).  patches is written (dt only).
 */
int fv_local_timestep(fv_patch* patches, int64_t n_patches, const double* per_patch,
                      int dim, double cfl, void* stream);

/*
 * ---------------------------------------------------------------------------
 * Learned face-flux correction (2-D Euler, s = 4).  Not in the paper: an
 * extension of its Rusanov update (Section 2, eqs. (2)-(5)) in which a small
 * network adds a correction to each face flux.
 *
 * Face frame: a face with normal along axis k lies between volumes i-1 (L)
 * and i (R) along k; states are read as (rho, j_n, j_t, E).  Features: the
 * volumes i-2, i-1, i, i+1 in that frame, 16 values, normalised as
 * (x - x_mean) * x_scale.  Network 16 -> 64 -> 64 -> 4 with tanh on the
 * hidden layers; the products take bfloat16 operands (weights and
 * activations rounded to nearest even) with float32 sums.  Correction
 * dF = o * y_scale + y_mean in the face frame, rotated back; 0 where
 * |rho_R - rho_L| / min(rho_L, rho_R) > threshold (plain Rusanov there).
 *
 * Parameter blob: device float32[5548]: x_mean[16], x_scale[16], W1[64][16],
 * b1[64], W2[64][64], b2[64], W3[4][64], b3[4], y_scale[4], y_mean[4]
 * (float32 master values; inference rounds the weights to bfloat16).
 *
 * Regular patch grids (training-data entry points): npx x npy patches of
 * p x p volumes, compact blocks [4][p][p] back to back in patch order (x
 * fastest); bc 0 periodic, 1 transmissive (zero gradient).
 * ---------------------------------------------------------------------------
 */
#define FV_MLP_BLOB_WORDS 5548
#define FV_MLP_TRAINED_WORDS 5508   /* W1, b1, W2, b2, W3, b3 */

/* acc_x[4][ncy][ncx+1] and acc_y[4][ncy+1][ncx] (device float64, coarse grid
 * ncx = npx*p/r, ncy = npy*p/r) += weight * (mean over the r fine faces of
 * each coarse face of the fine Rusanov flux of q_fine).  Called once per fine
 * step with weight 1/r, it builds the time- and face-averaged fine flux of
 * one coarse step (r fine steps).  r must divide p. */
int fv_learned_flux_accumulate(const double* q_fine, int npx, int npy, int p, int r, int bc,
                               double gamma, double weight, double* acc_x, double* acc_y,
                               void* stream);

/* Conservative r x r averages: q_coarse is the regular grid of npx/r x npy/r
 * patches of the same p (npx, npy multiples of r). */
int fv_learned_coarse_grain(const double* q_fine, int npx, int npy, int p, int r,
                            double* q_coarse, void* stream);

/* One sample per face of the coarse grid (x faces [ncy][ncx+1] then y faces
 * [ncy+1][ncx], row-major): features[n][16], targets[n][4] (face-frame
 * acc - Rusanov flux of the coarse state) and indicator[n], all float32. */
int fv_learned_face_samples(const double* q_coarse, int npx, int npy, int p, int bc,
                            double gamma, const double* acc_x, const double* acc_y,
                            float* features, float* targets, float* indicator, void* stream);

/* Per-column mean and spread of x[x_rows][cols] over the n_rows rows listed
 * in rows (device int64; NULL: all x_rows rows; a listed row outside
 * [0, x_rows) counts as zeros): mean_out[c]; scale_out[c] = 1/std (mode 0,
 * features) or std (mode 1, targets).  Pointers may address the blob's
 * x_mean/x_scale or y_mean/y_scale slots. */
int fv_mlp_fit_normalization(const float* x, int64_t x_rows, int cols, int mode,
                             const int64_t* rows, int64_t n_rows, float* mean_out,
                             float* scale_out, void* stream);

/* One Adam step (lr, step >= 1 counts steps) on the minibatch of rows
 * batch_idx[batch] (in [0, n_rows); other indices contribute nothing) of
 * (features[n_rows][16], targets[n_rows][4]): float32 forward and backward of
 * the mean-squared error of normalised targets, gradients summed in a fixed
 * order (deterministic).  adam: device float32[2 * 5508] moments (zero at
 * step 1); workspace: float32[fv_mlp_workspace_words(batch)] or more, of which
 * on return the words [W - batch, W), W = fv_mlp_workspace_words(batch), hold
 * the per-sample mean squared errors of the minibatch (0 for a row index
 * outside [0, n_rows)); grad_out: float32[5508] or NULL (the gradient of
 * W1..b3). */
int fv_mlp_workspace_words(int batch);
int fv_mlp_train_step(float* blob, float* adam, int step, float lr, const float* features,
                      const float* targets, int64_t n_rows, const int64_t* batch_idx, int batch,
                      float* workspace, int64_t workspace_words, float* grad_out, void* stream);

/* Network outputs o[n][4] (before y_scale / y_mean) for raw features[n][16],
 * computed the way the fused update does (bfloat16 matrix-core products). */
int fv_mlp_forward(const float* blob, const float* features, int64_t n, float* out,
                   void* stream);

/* One explicit step of 2-D patches of 16 x 16 volumes with corrected face
 * fluxes.  Compact blocks, halo of two volumes read from the face neighbours
 * (neighbours[n][4]: -x, +x, -y, +y; -1 = transmissive, which repeats the
 * boundary volume).  dt from dt_dev (device) or, when NULL, each descriptor.
 * max_eig (device, optional): largest |u_k| + c of each new patch. */
int fv_batch_update_learned_2d(const fv_patch* patches, int64_t n_patches,
                               const int64_t* neighbours, const double* q_in, int64_t q_in_len,
                               double* q_out, int64_t q_out_len, double gamma,
                               const double* dt_dev, const float* blob, double threshold,
                               double* max_eig, void* stream);

/*
 * fv_max_eigenvalue -- largest eigenvalue of a given state (Section 2,
 * eq. (5); Algorithm 1 last step), for the first CFL step of a run.
 *
 * q, q_len       device buffer holding one block per patch
 * q_halo         1: blocks are [s][(p+2)^d] (interior read), 0: [s][p^d]
 * which_offsets  FV_OFFSETS_IN or FV_OFFSETS_OUT: which descriptor offset
 *                locates each patch's block in q
 * per_patch      device [n_patches], required: max over interior volumes and
 *                axes of |u_j| + c (NaN for a patch that fails the check)
 * global         device [1] or NULL: NaN-propagating max over patches
 *                (0 for n_patches == 0)
 */
int fv_max_eigenvalue(const fv_patch* patches, int64_t n_patches,
                      const double* q, int64_t q_len, int q_halo, int which_offsets,
                      int dim, int p, int s, double gamma,
                      double* per_patch, double* global, void* stream);

/*
 * fv_cfl_timestep -- global time step from per-patch maxima, on the device:
 *   Lambda = max_b per_patch[b]            (NaN-propagating)
 *   dt     = cfl * min_{b, j < dim} patches[b].dx[j] / (dim * Lambda)
 * The paper states no formula (Section 4 only uses per-patch maxima for
 * adaptive stepping); the 1/dim factor keeps the unsplit update stable.
 * lambda_out, dt_out: device [1] each; either may be NULL.  n_patches >= 1.
 */
int fv_cfl_timestep(const fv_patch* patches, int64_t n_patches,
                    const double* per_patch, int dim, double cfl,
                    double* lambda_out, double* dt_out, void* stream);

/*
 * fv_fill_halo -- face-halo exchange (the engine's job in Section 2: keep
 * halo data consistent).  For patch b and face f = 2*axis + side (side 0 =
 * low, 1 = high; axes x, y, z):
 *   nb = neighbours[2*dim*b + f] >= 0: the face-halo layer takes the
 *        interior layer of patch nb that touches this face (periodic
 *        domains are expressed by wrapped neighbour indices);
 *   nb == -1: transmissive (zero-gradient): the halo layer takes this
 *        patch's own boundary layer.
 * Edge and corner halo volumes are untouched.  Reads interior volumes and
 * writes face-halo volumes only, so patches may be processed in any order.
 *
 * neighbours     device int64 [n_patches][2*dim], entries in [-1, n_patches)
 * q, q_len       device buffer of blocks [s][(p+2)^d]
 * which_offsets  FV_OFFSETS_IN or FV_OFFSETS_OUT
 * Faces whose block or neighbour fails the device-side bounds check are
 * skipped.
 */
int fv_fill_halo(const fv_patch* patches, int64_t n_patches,
                 const int64_t* neighbours, double* q, int64_t q_len,
                 int which_offsets, int dim, int p, int halo, int s, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FV_H */
