// Device-side pieces of the compressible Euler equations used by every kernel:
// state decoding, physical flux, directional wave speed and the Rusanov face
// flux (Section 2, eqs. (2), (4), (5) of arXiv 2302.09005).
//
// Unknowns (rho, j_x, j_y[, j_z], E), s = D + 2; ideal gas
// p = (gamma - 1)(E - |j|^2 / (2 rho)).  The energy flux is (E + p) j_dir / rho
// (the printed eq. (2) drops the factor j).  The face wave speed is the larger
// of the two one-sided values |u_dir| + c (eq. (5) evaluated at the two
// adjacent states).
//
// Rounding.  The library is built without implicit floating-point contraction;
// the fused multiply-adds below are written out and each is invariant under a
// sign flip of its momentum operands and under swapping the two sides of a
// face.  Mirroring a state field therefore mirrors the result bit for bit.
#pragma once

#include <hip/hip_runtime.h>

namespace fvk {

// Larger of a and b; NaN in either argument wins, so a blow-up reaches every
// maximum it feeds.
template <typename T>
__device__ __forceinline__ T nanmax(T a, T b) {
  return (a > b || a != a) ? a : b;
}

// The same for operands that are +0, positive or NaN (wave speeds, |u|): for
// those the IEEE bit patterns order like unsigned integers, NaN above +inf,
// so one integer compare does it.
__device__ __forceinline__ double nanmax_pos(double a, double b) {
  return (unsigned long long)__double_as_longlong(a) > (unsigned long long)__double_as_longlong(b)
             ? a
             : b;
}
__device__ __forceinline__ float nanmax_pos(float a, float b) {
  return (unsigned)__float_as_uint(a) > (unsigned)__float_as_uint(b) ? a : b;
}

// 1/x from the hardware estimate refined by two Newton steps (about 1 ulp;
// the textbook formulas divide by rho d + 2 times, this kernel once per
// volume).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Square root from the hardware reciprocal-square-root estimate y ~ 1/sqrt(x)
// by one step of Goldschmidt's iteration on g ~ sqrt(x), h ~ 1/(2 sqrt(x))
// (relative error e of y becomes about 1.5 e^2) followed by one Newton
// correction g += (x - g^2) h (error squared again, far below an ulp for any
// estimate better than 2^-20; the last fused multiply-add rounds once, so
// the result is within about half an ulp).  Without the range scaling of the
// library routine, which normal arguments do not need.  Zeros and +inf map
// to themselves, negative arguments and NaN to NaN.
__device__ __forceinline__ double sqrt_fast(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = 0.5 * y;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, x);
  g = fma(d, h, g);
  // -0, +0 and +inf (class bits 5, 6 and 9): the iteration would give NaN
  return __builtin_amdgcn_class(x, 0x260) ? x : g;
}
// Single precision: the hardware square root alone, within one ulp.  The
// correctly rounded library routine wraps it in range scaling and a
// correction step, about 15 more instructions per call (13 % of the float
// update's instructions).  +-0, +inf and NaN pass through, negative arguments
// give NaN.
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// What a face needs from one adjacent volume besides its conserved state:
// 1/rho, pressure and sound speed.  Computing 1/rho once per volume replaces
// the d + 2 divisions of the textbook formulas.
template <typename T>
struct Prim {
  T ir, p, c;
};

template <typename T, int D>
__device__ __forceinline__ Prim<T> decode(const T (&q)[D + 2], T gamma) {
  Prim<T> w;
  w.ir = recip(q[0]);
  T jj = q[1] * q[1];
#pragma unroll
  for (int k = 1; k < D; ++k) jj = fma(q[1 + k], q[1 + k], jj);
  w.p = (gamma - T(1)) * fma(T(-0.5) * jj, w.ir, q[D + 1]);
  w.c = sqrt_fast(gamma * w.p * w.ir);
  return w;
}

// max_j (|u_j| + c) of one volume (patch maxima and the CFL condition), as
// max_j |j_j| * |1/rho| + c: |u_j| = |j_j| |1/rho| holds for either sign of
// rho, so a state with rho < 0 (and p < 0, where c is real) still gives a
// non-negative speed, as eq. (5) does.
template <typename T, int D>
__device__ __forceinline__ T max_wave_speed(const T (&q)[D + 2], const Prim<T>& w) {
  T m = fabs(q[1]);
#pragma unroll
  for (int k = 1; k < D; ++k) m = nanmax_pos(m, T(fabs(q[1 + k])));
  return fma(m, T(fabs(w.ir)), w.c);
}

// Rusanov flux across a face normal to axis K between left state L and right
// state R (Section 2, eq. (4)):
//   F = 1/2 [ f^K(L) + f^K(R) - a (R - L) ],  a = max(|u_K(L)| + c_L, |u_K(R)| + c_R).
// Twice the Rusanov flux across a face with normal along axis K, 2F =
// f(L) + f(R) - a (R - L) (eq. (4)); the caller folds the factor 1/2 into
// dt/dx, which is exact in binary floating point and so changes no bit of
// the update.
template <typename T, int D, int K>
__device__ __forceinline__ void rusanov(const T (&qL)[D + 2], const Prim<T>& wL,
                                        const T (&qR)[D + 2], const Prim<T>& wR,
                                        T (&F)[D + 2]) {
  constexpr int S = D + 2;
  const T uL = qL[1 + K] * wL.ir;
  const T uR = qR[1 + K] * wR.ir;
  const T a = nanmax_pos(T(fabs(uL)) + wL.c, T(fabs(uR)) + wR.c);
  T fL[S], fR[S];
  fL[0] = qL[1 + K];
  fR[0] = qR[1 + K];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    fL[1 + k] = k == K ? fma(qL[1 + k], uL, wL.p) : qL[1 + k] * uL;
    fR[1 + k] = k == K ? fma(qR[1 + k], uR, wR.p) : qR[1 + k] * uR;
  }
  fL[D + 1] = (qL[D + 1] + wL.p) * uL;
  fR[D + 1] = (qR[D + 1] + wR.p) * uR;
#pragma unroll
  for (int m = 0; m < S; ++m) F[m] = fma(-a, qR[m] - qL[m], fL[m] + fR[m]);
}

}  // namespace fvk
