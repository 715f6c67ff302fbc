/*
 * Plain FP64 CPU oracle for the batched Finite Volume patch update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that the GPU library can be
 * checked against an implementation that a reader can compare with the paper
 * by eye.  It shares no code, header, table or constant with the GPU path and
 * must never be linked into, loaded by or called from the product; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Paper: "GPU Offloading in ExaHyPE Through C++ Standard Algorithms"
 * (Gomez, Brito Gadeschi, Weinzierl, arXiv 2302.09005).
 *
 *   - PDE, Section 2, eq. (1):  dq/dt + sum_j d/dx_j f^j(q) = 0, q in R^s.
 *   - Euler flux, Section 2, eq. (2): (rho, j, E_t) with fluxes
 *     j,  j (x) j / rho + p I,  (E_t + p) j / rho.
 *     The printed energy entry lacks the factor j; the standard Euler flux
 *     (E_t + p) u is used.  The equation of state is not printed; the ideal
 *     gas law p = (gamma - 1)(E_t - |j|^2 / (2 rho)) is used.
 *   - Update, Section 2, eq. (3): explicit Euler in time, flux difference over
 *     the faces of each volume; in d dimensions the fluxes of all 2d faces
 *     of a volume enter its update, each difference scaled by dt/dx
 *     (Algorithm 1, step 7), one dx per axis, axes in the order x, y, z.
 *   - Rusanov flux, Section 2, eq. (4): F = 1/2 [f(L) + f(R) - a (R - L)].
 *   - Wave speed, Section 2, eq. (5): a = max |lambda_k|; read as the larger of
 *     the two one-sided directional values |u_j| + c (the sup over the state
 *     segment is not evaluated).
 *   - Per-patch maximum eigenvalue of the new solution, Algorithm 1 (last
 *     step) and Section 4 (local adaptive time stepping needs it per patch).
 *   - Halo layer, Section 2 (mesh paragraph): keeping it consistent is the
 *     engine's job; face-neighbour copy, periodic or transmissive.
 *
 * Layout (Section 3 loop order, x innermost): each patch block is
 * unknown-major [s][z][y][x] over (p + 2)^d volumes when it carries a halo of
 * width one, or over p^d volumes without halo.  A patch is addressed by an
 * element offset into one flat array.
 *
 * Arithmetic follows the definitions literally: every face flux is evaluated
 * from its two adjacent states each time a volume needs it (so a face is
 * evaluated twice, once per side); no reordering, no blocking, no fusion.
 * Build with -O2 -ffp-contract=off and without fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXS 5

/* Larger of two values; a NaN in either argument is returned (so a blow-up
 * anywhere reaches the patch and global maxima).  The paper replaces
 * std::max by a hand-written comparison (Section 3); NaN behaviour is not
 * stated there, this propagating choice is ours. */
static double or_nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return (a > b) ? a : b;
}

/* Pressure of the ideal gas from conserved variables (reading of Section 2,
 * eq. (2), where the equation of state is not printed). */
static double or_pressure(const double* q, int d, double gamma) {
  double rho = q[0];
  double jj = 0.0;
  for (int k = 0; k < d; ++k) jj = jj + q[1 + k] * q[1 + k];
  double E = q[d + 1];
  return (gamma - 1.0) * (E - 0.5 * jj / rho);
}

/* Physical flux f^dir(q), Section 2 eq. (2): mass row j_dir, momentum rows
 * j_dir j_k / rho + p delta_{dir,k}, energy row (E + p) j_dir / rho. */
void oracle_flux(const double* q, int d, int dir, double gamma, double* f) {
  double rho = q[0];
  double p = or_pressure(q, d, gamma);
  double jd = q[1 + dir];
  f[0] = jd;
  for (int k = 0; k < d; ++k) {
    f[1 + k] = jd * q[1 + k] / rho;
    if (k == dir) f[1 + k] = f[1 + k] + p;
  }
  f[d + 1] = (q[d + 1] + p) * jd / rho;
}

/* Largest eigenvalue magnitude of the flux Jacobian along axis dir:
 * |u_dir| + c with c = sqrt(gamma p / rho) (Section 2, eq. (5)). */
double oracle_eigenvalue(const double* q, int d, int dir, double gamma) {
  double rho = q[0];
  double p = or_pressure(q, d, gamma);
  double c = sqrt(gamma * p / rho);
  double u = q[1 + dir] / rho;
  return fabs(u) + c;
}

/* Largest directional eigenvalue over all axes (what a patch or the CFL
 * condition needs). */
double oracle_max_eigenvalue_state(const double* q, int d, double gamma) {
  double m = oracle_eigenvalue(q, d, 0, gamma);
  for (int j = 1; j < d; ++j) m = or_nanmax(m, oracle_eigenvalue(q, d, j, gamma));
  return m;
}

/* Rusanov face flux between left state L and right state R along axis dir,
 * Section 2 eq. (4) with a from eq. (5). */
void oracle_rusanov(const double* L, const double* R, int d, int dir,
                    double gamma, double* F) {
  int s = d + 2;
  double fL[OR_MAXS], fR[OR_MAXS];
  oracle_flux(L, d, dir, gamma, fL);
  oracle_flux(R, d, dir, gamma, fR);
  double a = or_nanmax(oracle_eigenvalue(L, d, dir, gamma),
                       oracle_eigenvalue(R, d, dir, gamma));
  for (int k = 0; k < s; ++k)
    F[k] = 0.5 * ((fL[k] + fR[k]) - a * (R[k] - L[k]));
}

/* Number of volumes per axis of a block with halo width h. */
static int64_t or_vol(int d, int w) {
  int64_t v = 1;
  for (int j = 0; j < d; ++j) v *= w;
  return v;
}

/* Read the s unknowns of the volume with (halo-including) coordinates
 * (x, y, z) from an unknown-major block of width w. */
static void or_get(const double* blk, int d, int w, int x, int y, int z,
                   double* q) {
  int64_t vol = or_vol(d, w);
  int64_t idx = (int64_t)x + (int64_t)w * y + (d == 3 ? (int64_t)w * w * z : 0);
  for (int k = 0; k < d + 2; ++k) q[k] = blk[k * vol + idx];
}

static void or_put(double* blk, int d, int w, int x, int y, int z,
                   const double* q) {
  int64_t vol = or_vol(d, w);
  int64_t idx = (int64_t)x + (int64_t)w * y + (d == 3 ? (int64_t)w * w * z : 0);
  for (int k = 0; k < d + 2; ++k) blk[k * vol + idx] = q[k];
}

/*
 * One explicit Euler step of every patch (Section 2 eqs. (3)-(5), Algorithm 1).
 *
 * n              number of patches
 * d, p           dimension (2 or 3) and volumes per axis; s = d + 2, halo 1
 * in_off[n]      element offset of each input block [s][(p+2)^d] in q_in
 * out_off[n]     element offset of each output block in q_out
 * out_halo       0: output block is [s][p^d]; 1: [s][(p+2)^d], interior written
 * dx[n*3]        volume width per axis and patch
 * dt[n]          time step per patch
 * max_eig[n]     per-patch largest eigenvalue of the new state, or NULL
 * nthreads       OpenMP threads over patches (<= 0: runtime default)
 *
 * Returns 0, or -1 for unsupported arguments.
 */
int oracle_fv_step(int64_t n, int d, int p, double gamma,
                   const int64_t* in_off, const int64_t* out_off, int out_halo,
                   const double* dx, const double* dt,
                   const double* q_in, double* q_out, double* max_eig,
                   int nthreads) {
  if ((d != 2 && d != 3) || p < 1 || n < 0) return -1;
  int s = d + 2;
  int w = p + 2;
  int wo = out_halo ? p + 2 : p;
  int o = out_halo ? 1 : 0;
  int pz = (d == 3) ? p : 1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int64_t b = 0; b < n; ++b) {
    const double* in = q_in + in_off[b];
    double* out = q_out + out_off[b];
    double lam = 0.0;
    int first = 1;
    for (int z = 0; z < pz; ++z)
      for (int y = 0; y < p; ++y)
        for (int x = 0; x < p; ++x) {
          int zc = (d == 3) ? z + 1 : 0;
          double qc[OR_MAXS], qn[OR_MAXS];
          or_get(in, d, w, x + 1, y + 1, zc, qc);
          for (int k = 0; k < s; ++k) qn[k] = qc[k];
          for (int j = 0; j < d; ++j) {
            int ex = (j == 0), ey = (j == 1), ez = (j == 2);
            double qm[OR_MAXS], qp[OR_MAXS], Fm[OR_MAXS], Fp[OR_MAXS];
            or_get(in, d, w, x + 1 - ex, y + 1 - ey, zc - ez, qm);
            or_get(in, d, w, x + 1 + ex, y + 1 + ey, zc + ez, qp);
            oracle_rusanov(qm, qc, d, j, gamma, Fm);
            oracle_rusanov(qc, qp, d, j, gamma, Fp);
            double r = dt[b] / dx[3 * b + j];
            for (int k = 0; k < s; ++k) qn[k] = qn[k] - r * (Fp[k] - Fm[k]);
          }
          or_put(out, d, wo, x + o, y + o, (d == 3) ? z + o : 0, qn);
          double l = oracle_max_eigenvalue_state(qn, d, gamma);
          lam = first ? l : or_nanmax(lam, l);
          first = 0;
        }
    if (max_eig) max_eig[b] = lam;
  }
  return 0;
}

/*
 * The same step evaluated in the step order of Algorithm 1 instead of one
 * flux difference per face (reading of its garbled steps 2-7: the Rusanov
 * flux of eq. (4) split into its dissipative and central parts, each scaled
 * by dt/dx).  For every patch:
 *   step 1      Q_new = Q_old on the interior;
 *   steps 2-4   for each axis j: a at the low and high face of each volume
 *               (eq. (5) on the two adjacent old states) and the dissipative
 *               part D = -1/2 a (Q_R - Q_L) of both face fluxes;
 *               Q_new -= dt/dx_j (D(i+1/2) - D(i-1/2));
 *   steps 5-7   for each axis j: the central part C = 1/2 (f^j(Q_L) + f^j(Q_R))
 *               of both face fluxes; Q_new -= dt/dx_j (C(i+1/2) - C(i-1/2));
 *   step 8      non-conservative product: zero for the Euler equations;
 *   step 10     per-patch maximum eigenvalue of Q_new.
 * D + C is the face flux of eq. (4), so the result equals oracle_fv_step's
 * up to rounding.  Arguments and return value as for oracle_fv_step.
 */
int oracle_fv_step_alg1(int64_t n, int d, int p, double gamma,
                        const int64_t* in_off, const int64_t* out_off, int out_halo,
                        const double* dx, const double* dt,
                        const double* q_in, double* q_out, double* max_eig,
                        int nthreads) {
  if ((d != 2 && d != 3) || p < 1 || n < 0) return -1;
  int s = d + 2;
  int w = p + 2;
  int wo = out_halo ? p + 2 : p;
  int o = out_halo ? 1 : 0;
  int pz = (d == 3) ? p : 1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int64_t b = 0; b < n; ++b) {
    const double* in = q_in + in_off[b];
    double* out = q_out + out_off[b];
    /* step 1: copy */
    for (int z = 0; z < pz; ++z)
      for (int y = 0; y < p; ++y)
        for (int x = 0; x < p; ++x) {
          int zc = (d == 3) ? z + 1 : 0;
          double qc[OR_MAXS];
          or_get(in, d, w, x + 1, y + 1, zc, qc);
          or_put(out, d, wo, x + o, y + o, (d == 3) ? z + o : 0, qc);
        }
    /* steps 2-4 (part = 0, dissipative), then steps 5-7 (part = 1, central) */
    for (int part = 0; part < 2; ++part)
      for (int z = 0; z < pz; ++z)
        for (int y = 0; y < p; ++y)
          for (int x = 0; x < p; ++x) {
            int zc = (d == 3) ? z + 1 : 0;
            int zo = (d == 3) ? z + o : 0;
            double qc[OR_MAXS], qn[OR_MAXS];
            or_get(in, d, w, x + 1, y + 1, zc, qc);
            or_get(out, d, wo, x + o, y + o, zo, qn);
            for (int j = 0; j < d; ++j) {
              int ex = (j == 0), ey = (j == 1), ez = (j == 2);
              double qm[OR_MAXS], qp[OR_MAXS], Fm[OR_MAXS], Fp[OR_MAXS];
              or_get(in, d, w, x + 1 - ex, y + 1 - ey, zc - ez, qm);
              or_get(in, d, w, x + 1 + ex, y + 1 + ey, zc + ez, qp);
              if (part == 0) {
                double am = or_nanmax(oracle_eigenvalue(qm, d, j, gamma),
                                      oracle_eigenvalue(qc, d, j, gamma));
                double ap = or_nanmax(oracle_eigenvalue(qc, d, j, gamma),
                                      oracle_eigenvalue(qp, d, j, gamma));
                for (int k = 0; k < s; ++k) {
                  Fm[k] = -0.5 * am * (qc[k] - qm[k]);
                  Fp[k] = -0.5 * ap * (qp[k] - qc[k]);
                }
              } else {
                double fm[OR_MAXS], fc[OR_MAXS], fp[OR_MAXS];
                oracle_flux(qm, d, j, gamma, fm);
                oracle_flux(qc, d, j, gamma, fc);
                oracle_flux(qp, d, j, gamma, fp);
                for (int k = 0; k < s; ++k) {
                  Fm[k] = 0.5 * (fm[k] + fc[k]);
                  Fp[k] = 0.5 * (fc[k] + fp[k]);
                }
              }
              double r = dt[b] / dx[3 * b + j];
              for (int k = 0; k < s; ++k) qn[k] = qn[k] - r * (Fp[k] - Fm[k]);
            }
            or_put(out, d, wo, x + o, y + o, zo, qn);
          }
    /* step 8: the non-conservative product of the Euler equations is zero;
     * step 10: maximum eigenvalue of the new state */
    if (max_eig) {
      double lam = 0.0;
      int first = 1;
      for (int z = 0; z < pz; ++z)
        for (int y = 0; y < p; ++y)
          for (int x = 0; x < p; ++x) {
            double qn[OR_MAXS];
            or_get(out, d, wo, x + o, y + o, (d == 3) ? z + o : 0, qn);
            double l = oracle_max_eigenvalue_state(qn, d, gamma);
            lam = first ? l : or_nanmax(lam, l);
            first = 0;
          }
      max_eig[b] = lam;
    }
  }
  return 0;
}

/*
 * Largest eigenvalue over the interior volumes of every patch of q
 * (Algorithm 1, last step, applied to a given state; Section 4).
 * halo: 1 if q's blocks are [s][(p+2)^d], 0 if [s][p^d].
 * per_patch[n] may be NULL; *global receives the NaN-propagating maximum
 * (0 for n == 0).
 */
int oracle_max_eigenvalue(int64_t n, int d, int p, double gamma,
                          const int64_t* off, int halo, const double* q,
                          double* per_patch, double* global) {
  if ((d != 2 && d != 3) || p < 1 || n < 0) return -1;
  int w = halo ? p + 2 : p;
  int o = halo ? 1 : 0;
  int pz = (d == 3) ? p : 1;
  double g = 0.0;
  for (int64_t b = 0; b < n; ++b) {
    double lam = 0.0;
    int first = 1;
    for (int z = 0; z < pz; ++z)
      for (int y = 0; y < p; ++y)
        for (int x = 0; x < p; ++x) {
          double qc[OR_MAXS];
          or_get(q + off[b], d, w, x + o, y + o, (d == 3) ? z + o : 0, qc);
          double l = oracle_max_eigenvalue_state(qc, d, gamma);
          lam = first ? l : or_nanmax(lam, l);
          first = 0;
        }
    if (per_patch) per_patch[b] = lam;
    g = (b == 0) ? lam : or_nanmax(g, lam);
  }
  if (global) *global = g;
  return 0;
}

/*
 * Time step from the CFL condition: Lambda = max over patches of
 * max_eig[b]; dt = cfl * (smallest dx of any patch and axis) / (d * Lambda).
 * The paper gives no formula (Section 4 only says per-patch maxima drive
 * adaptive time stepping); the factor 1/d keeps the unsplit update within
 * its stability bound.  Writes Lambda to *lambda_out when non-NULL.
 */
double oracle_cfl_dt(int64_t n, int d, const double* dx,
                     const double* max_eig, double cfl, double* lambda_out) {
  double lam = 0.0, h = INFINITY;
  for (int64_t b = 0; b < n; ++b) {
    lam = (b == 0) ? max_eig[b] : or_nanmax(lam, max_eig[b]);
    for (int j = 0; j < d; ++j) h = (dx[3 * b + j] < h) ? dx[3 * b + j] : h;
  }
  if (lambda_out) *lambda_out = lam;
  return cfl * h / ((double)d * lam);
}

/*
 * Local time stepping (Section 4; per-patch t and dt of the patch data in
 * Appendix A): every patch takes its own step from its own maximum,
 * dt[b] = cfl * (smallest dx of patch b) / (d * max_eig[b]), the CFL rule of
 * oracle_cfl_dt applied to patch b alone.
 */
void oracle_local_dt(int64_t n, int d, const double* dx, const double* max_eig,
                     double cfl, double* dt) {
  for (int64_t b = 0; b < n; ++b) {
    double h = INFINITY;
    for (int j = 0; j < d; ++j) h = (dx[3 * b + j] < h) ? dx[3 * b + j] : h;
    dt[b] = cfl * h / ((double)d * max_eig[b]);
  }
}

/*
 * Face-halo fill (the engine's consistency step, Section 2).  For patch b and
 * face f = 2*axis + side (side 0: low, 1: high), nb = neighbours[2*d*b + f]:
 *   nb >= 0: the halo layer takes the neighbour's interior layer that touches
 *            this face (neighbour's high layer for a low face and vice versa);
 *   nb <  0: transmissive (zero-gradient) -- the halo layer takes this
 *            patch's own boundary layer on that face.
 * Edge and corner halo volumes are not touched.  Blocks are [s][(p+2)^d] at
 * off[b].  Reads only interior volumes and writes only face-halo volumes, so
 * the result does not depend on the order of patches.
 */
int oracle_fill_halo(int64_t n, int d, int p, const int64_t* off,
                     const int64_t* neighbours, double* q) {
  if ((d != 2 && d != 3) || p < 1 || n < 0) return -1;
  int w = p + 2;
  int pz = (d == 3) ? p : 1;
  for (int64_t b = 0; b < n; ++b) {
    for (int ax = 0; ax < d; ++ax)
      for (int side = 0; side < 2; ++side) {
        int64_t nb = neighbours[2 * d * b + 2 * ax + side];
        int64_t src = (nb >= 0) ? nb : b;
        int dst_c = side ? p + 1 : 0;  /* halo coordinate along ax */
        int src_c;                       /* interior coordinate along ax */
        if (nb >= 0) src_c = side ? 1 : p;
        else         src_c = side ? p : 1;
        /* loop over the other coordinates of the face (interior only) */
        for (int c2 = 0; c2 < pz; ++c2)
          for (int c1 = 0; c1 < p; ++c1) {
            int t[3] = {0, 0, 0}, u[3] = {0, 0, 0};
            /* the two tangential coordinates in increasing axis order */
            int k = 0, tang[2] = {c1 + 1, c2 + 1};
            for (int a = 0; a < d; ++a) {
              if (a == ax) { t[a] = dst_c; u[a] = src_c; }
              else { t[a] = tang[k]; u[a] = tang[k]; ++k; }
            }
            double qs[OR_MAXS];
            or_get(q + off[src], d, w, u[0], u[1], u[2], qs);
            or_put(q + off[b], d, w, t[0], t[1], t[2], qs);
          }
      }
  }
  return 0;
}

/*
 * Totals of the conserved unknowns over the interior volumes of all patches,
 * summed in patch order then volume order (plain FP64 accumulation; the tests
 * use exactly rounded sums where they need them).  tot[s].
 */
int oracle_totals(int64_t n, int d, int p, const int64_t* off, int halo,
                  const double* q, double* tot) {
  if ((d != 2 && d != 3) || p < 1 || n < 0) return -1;
  int s = d + 2, w = halo ? p + 2 : p, o = halo ? 1 : 0;
  int pz = (d == 3) ? p : 1;
  for (int k = 0; k < s; ++k) tot[k] = 0.0;
  for (int64_t b = 0; b < n; ++b)
    for (int z = 0; z < pz; ++z)
      for (int y = 0; y < p; ++y)
        for (int x = 0; x < p; ++x) {
          double qc[OR_MAXS];
          or_get(q + off[b], d, w, x + o, y + o, (d == 3) ? z + o : 0, qc);
          for (int k = 0; k < s; ++k) tot[k] = tot[k] + qc[k];
        }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
