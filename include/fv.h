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
 * Host-side validation of a descriptor array (a HOST copy), for callers that
 * build descriptors themselves.  Checks p, finite positive dx and dt >= 0,
 * that every input/output block lies inside [0, len), and that output blocks
 * do not overlap each other.  Returns FV_OK or FV_EINVAL (with the first
 * offending patch named by fv_last_error()).  Touches no device.
 */
int fv_check_patches(const fv_patch* host_patches, int64_t n_patches,
                     int dim, int p, int q_out_halo,
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
