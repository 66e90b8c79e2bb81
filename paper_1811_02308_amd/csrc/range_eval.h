// Per-pixel range stage shared by the range kernel and the fused
// moments-and-range kernels: Algorithm 1's per-pixel steps (eqs. inv, sub,
// I_0, I_1, F_forward, BFfinal) for one pixel whose
// bounds alpha != beta and Legendre coefficients are known (see range.hip for
// the method and the choice between the paper's recursion and quadrature).
#pragma once

#include "abf_internal.h"
#include "erfcx_weideman.h"

namespace abf {

constexpr double kSqrtPi = 1.7724538509055160273;

// The fit c = A^-1 mu of eq. inv in the Legendre form: p(t) = sum_k (2k+1)
// a~_k P_k(2t - 1). fit.ell[k][r] = (2k+1) ell[k][r] gives p's coefficients
// in powers of t from the Legendre moments a~_k, fit.leg[k][r] = (2k+1)
// L[k][r] in powers of x = 2t - 1 (products of small integers and dyadic
// rationals: exact, so folding the factor in changes no result bit).
struct FitTables {
  double ell[kNMax + 1][kNMax + 1];
  double leg[kNMax + 1][kNMax + 1];
  constexpr FitTables() : ell{}, leg{} {
    const ShiftedLegTable SL;
    const LegTable LT;
    for (int k = 0; k <= kNMax; ++k)
      for (int r = 0; r <= kNMax; ++r) {
        ell[k][r] = (2.0 * k + 1.0) * SL.ell[k][r];
        leg[k][r] = (2.0 * k + 1.0) * LT.L[k][r];
      }
  }
};

// Smallest lambda at which the forward recursion is used, per degree N.
// The recursion's rounding grows roughly like N!/(2 lambda)^N; these limits
// keep its error in F below ~1e-10 (FP64 path) and ~1e-6 (mixed path),
// measured against 60-digit evaluations of the integrals.
__host__ __device__ constexpr double lam_split(int N, bool mixed) {
  return mixed ? (N <= 6 ? 0.05 : (N == 7 ? 0.12 : 0.25))
               : (N <= 4 ? 0.1 : (N == 5 ? 0.2 : (N == 6 ? 0.5 : (N == 7 ? 1.0 : 2.0))));
}
// The recursion multiplies errors by about |t0| per step, so it is used only
// while t0 is within outside_limit/sqrt(lambda) of [0, 1].
__host__ __device__ constexpr double outside_limit(bool mixed) { return mixed ? 1.5 : 0.5; }
constexpr double kSupport = 30.0;

// exp(x) for x <= 0 (arguments here never exceed 0): Cody-Waite reduction
// x = n ln2 + r, |r| <= ln2/2, with ln2 split in a high part exact to 32
// bits and a low part; e^r by its Taylor series to r^13/13! (truncation
// below 2^-55 relative); 2^n applied with ldexp. Results below the FP64
// range flush to 0. A few ulp, i.e. far inside the FP64 path's tolerance.
__device__ __forceinline__ double exp_neg(double x) {
  if (x < -745.0) return 0.0;
  const double n = rint(x * 1.4426950408889634074);
  const double r = fma(n, -6.93147180369123816490e-01, x);
  const double rr = fma(n, -1.90821492927058770002e-10, r);
  double p = 1.0 / 6227020800.0;                    // 1/13!
  p = fma(p, rr, 1.0 / 479001600.0);
  p = fma(p, rr, 1.0 / 39916800.0);
  p = fma(p, rr, 1.0 / 3628800.0);
  p = fma(p, rr, 1.0 / 362880.0);
  p = fma(p, rr, 1.0 / 40320.0);
  p = fma(p, rr, 1.0 / 5040.0);
  p = fma(p, rr, 1.0 / 720.0);
  p = fma(p, rr, 1.0 / 120.0);
  p = fma(p, rr, 1.0 / 24.0);
  p = fma(p, rr, 1.0 / 6.0);
  p = fma(p, rr, 0.5);
  p = fma(p, rr, 1.0);
  p = fma(p, rr, 1.0);
  return ldexp(p, (int)n);
}

// 1/x from the hardware reciprocal estimate and two Newton steps (a few ulp;
// used for parameters and the final ratio, never for exact quantities).
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// erfcx(x) = exp(x^2) erfc(x) for x >= 0 by Weideman's rational expansion
// of the Faddeeva function on the real axis (SIAM J. Numer. Anal. 31(5),
// 1994): with r = 1/(L + x) and Z = (L - x)/(L + x) = 2 L r - 1,
// erfcx(x) = r (2 r p(Z) + 1/sqrt(pi)), p of degree kErfcxTerms - 1
// (coefficients from gen_erfcx.py). Relative error below 1.3e-15 for
// finite x >= 0 (checked against 40-digit values), tending to the
// function's own limit 1/(sqrt(pi) x). About 45 instructions, against
// about 130 for the library's erfcx (used by the FP64 path). This takes r;
// erfcx_w2 below forms it.
__device__ __forceinline__ double erfcx_w_r(double r) {
  const double z = fma(2.0 * kErfcxL, r, -1.0);
  double p = kErfcxA[0];
#pragma unroll
  for (int n = 1; n < kErfcxTerms; ++n) p = fma(p, z, kErfcxA[n]);
  return r * fma(2.0 * r, p, 0.56418958354775628695);     // 1/sqrt(pi)
}

// erfcx at two arguments x0, x1 >= 0, with one reciprocal for both r = 1/(L + x):
// 1/(u v) times v and times u (a few ulp, far below the expansion's error;
// u v stays finite for every argument the range stage passes).
__device__ __forceinline__ void erfcx_w2(double x0, double x1, double& e0, double& e1) {
  const double u = kErfcxL + x0, v = kErfcxL + x1;
  const double ruv = rcp(u * v);
  e0 = erfcx_w_r(v * ruv);
  e1 = erfcx_w_r(u * ruv);
}

// g^ = a + (b - a) F for one pixel and the interval [a, b] (a < b; the
// window bounds alpha, beta in Algorithm 1). at[k] = a~_k, the Legendre
// moments, with at[0] = 1; th = theta, sg = sigma at the pixel.
// kMixed selects the mixed-precision thresholds, the 12-node rule (else 16)
// and FP32 quadrature exponentials.
template <int N, bool kMixed>
__device__ __forceinline__ double range_eval(double a, double b, const double (&at)[N + 1], double th,
                                             double sg, unsigned flags) {
  constexpr FitTables FT{};
  constexpr int Q = kMixed ? kGLNodesMixed : kGLNodes;
  constexpr GLRule gl(Q);
  const double da = a, delta = b - da;
  double t0, lam, sl;
  if (kMixed) {
    // Mixed path: t0 and sqrt(lambda) = (beta - alpha) / (sigma sqrt 2) in
    // FP32 (relative errors of a few 1e-8 move g^ by far less than the
    // mixed tolerance), and lambda taken as the exact FP64 square of that
    // FP32 root, so that every later step works on one consistent
    // (t0, lambda) pair. sigma = +inf gives sqrt(lambda) = 0; the root is
    // capped at 1e15 (sigma -> 0).
    const float d32 = (float)b - (float)a;
    const float t32 = ((float)th - (float)a) * __builtin_amdgcn_rcpf(d32);
    const float s32 = fminf(d32 * __builtin_amdgcn_rcpf((float)sg) * 0.70710678118654752f, 1e15f);
    t0 = t32;
    sl = s32;
    lam = sl * sl;
  } else {
    t0 = (th - da) * rcp(delta);
    lam = isinf(sg) ? 0.0 : delta * delta * rcp(2.0 * sg * sg);
    sl = sqrt(lam);
  }

  const double ts = fmin(fmax(t0, 0.0), 1.0);
  const double dist = fabs(t0 - ts);
  // T1, T2 and the N = 0 estimate's ratio f0n / f0d, which is evaluated
  // only where the fit's ratio fails
  double T1, T2, f0n, f0d;
  if (lam >= lam_split(N, kMixed) && dist * sl < outside_limit(kMixed)) {
    double c[N + 1];
#pragma unroll
    for (int r = 0; r <= N; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = r; k <= N; ++k) acc = fma(at[k], FT.ell[k][r], acc);
      c[r] = acc;
    }
    const double A = -sl * t0, B = sl * (1.0 - t0);
    const double dd = t0 - ts;
    const double s = lam * dd * dd;
    const double E0 = exp_neg(s - A * A);    // exp(-lam t0^2) * e^s
    const double E1 = exp_neg(s - B * B);    // exp(-lam (1-t0)^2) * e^s
    // (erf(B) - erf(A)) * e^s from erfc of |A| and |B| (A < B):
    //   A <= 0 <= B:  2 - erfc(B) - erfc(-A)
    //   0 < A:        erfc(A) - erfc(B)
    //   B < 0:        erfc(-B) - erfc(-A)
    // with erfc(|z|) = erfcx(|z|) exp(-z^2), the e^s folded into E0 and E1.
    // Two erfcx calls per pixel in every case, so a wave whose lanes fall in
    // different cases does not run several inlined copies one after another.
    // (the mixed path takes the shorter expansion: measured 7% faster there,
    // with a margin of ~1e3 to the mixed tolerance; the FP64 path keeps the
    // library function's last ulps)
    double X0, X1;
    if (kMixed) {
      erfcx_w2(fabs(A), fabs(B), X0, X1);
    } else {
      X0 = erfcx(fabs(A));
      X1 = erfcx(fabs(B));
    }
    X0 *= E0;
    X1 *= E1;
    const bool straddle = A <= 0.0 && B >= 0.0;
    const double diff = (straddle ? 2.0 - X1 : (A > 0.0 ? -X1 : X1)) + (A > 0.0 ? X0 : -X0);
    // (mixed path: lambda is the exact square of sqrt(lambda), so 1/lambda
    // is taken as (1/sqrt(lambda))^2, one reciprocal instead of two)
    const double isl = rcp(sl);
    const double i2l = kMixed ? 0.5 * (isl * isl) : 0.5 * rcp(lam);
    double Im2 = 0.5 * kSqrtPi * isl * diff;         // I_0
    double Im1 = fma(t0, Im2, (E0 - E1) * i2l);      // I_1
    f0n = Im1;
    f0d = Im2;
    T2 = c[0] * Im2;
    T1 = c[0] * Im1;
    const double e1l = E1 * i2l;
#pragma unroll
    for (int k = 2; k <= N + 1; ++k) {
      const double Ik = fma(t0, Im1, fma((k - 1) * i2l, Im2, -e1l));
      T1 = fma(c[k - 1], Ik, T1);
      T2 = fma(c[k - 1], Im1, T2);
      Im2 = Im1;
      Im1 = Ik;
    }
  } else {
    // support of the scaled Gaussian exp(-lam ((t-t0)^2 - dist^2)) above e^-kSupport
    // (a bound, not an exact quantity: reciprocal estimate and, on the
    // mixed path, the hardware square root)
    const double L = lam > 0.0
                         ? (kMixed ? (double)__builtin_amdgcn_sqrtf((float)fma(kSupport, rcp(lam), dist * dist))
                                   : sqrt(fma(kSupport, rcp(lam), dist * dist))) - dist
                         : 2.0;
    const double lo = fmax(0.0, ts - L), hi = fmin(1.0, ts + L);
    const double span = hi - lo;
    // p in powers of x = 2t - 1: bx[r] = sum_k (2k+1) a~_k L[k][r]
    // (coefficients of moderate size, so Horner in x on [-1, 1] is well
    // conditioned)
    double bx[N + 1];
#pragma unroll
    for (int r = 0; r <= N; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = r; k <= N; k += 2) acc = fma(at[k], FT.leg[k][r], acc);
      bx[r] = acc;
    }
    T1 = T2 = 0.0;
    double J0 = 0.0, J1 = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const double t = fma(span, gl.t[q], lo);
      const double x = 2.0 * t - 1.0;
      double p = bx[N];
#pragma unroll
      for (int r = N - 1; r >= 0; --r) p = fma(p, x, bx[r]);
      const double e = -lam * (t - ts) * (t + ts - 2.0 * t0);
      double psi;
      if (kMixed) {
        psi = (double)__expf((float)fmax(e, -80.0));
      } else {
        psi = exp_neg(e);
      }
      const double wpsi = span * gl.w[q] * psi;
      J0 += wpsi;
      J1 = fma(wpsi, t, J1);
      T2 = fma(wpsi, p, T2);
      T1 = fma(wpsi * t, p, T1);
    }
    f0n = J1;
    f0d = J0;
  }
  double F = T1 * rcp(T2);
  if (!(T2 > 0.0) || !isfinite(F)) F = f0n * rcp(f0d);
  if (flags & 1u) F = fmin(fmax(F, 0.0), 1.0);
  return fma(delta, F, da);
}

}  // namespace abf
