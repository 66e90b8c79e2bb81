// Range stage: Algorithm 1 lines 10-20 from the moment stack, one thread
// per pixel, all arithmetic in FP64 registers.
//
//   p(t) = sum_k c_k t^k is the degree-N polynomial whose moments on [0,1]
//   match those of the stretched histogram (eq. match); with the stored
//   Legendre moments it is p(t) = sum_k (2k+1) a~_k P_k(2t-1), and its
//   monomial coefficients are c = A^-1 mu = sum_k (2k+1) a~_k ell_k
//   (eq. inv; A^-1 = sum_k (2k+1) ell_k ell_k^T exactly).
//   t0 = (theta - alpha)/(beta - alpha), lambda = (beta-alpha)^2/(2 sigma^2)
//   (eq. sub), T1 = int_0^1 t p psi, T2 = int_0^1 p psi with
//   psi = exp(-lambda (t - t0)^2), and g^ = alpha + (beta-alpha) T1/T2
//   (eq. BFfinal).
//
// Two evaluations of T1, T2, chosen per pixel by lambda and by how far t0
// lies outside [0, 1] (d = dist(t0, [0,1])):
//   lambda >= lam_split(N) and d sqrt(lambda) < outside_limit: the paper's route. I_0 from two error functions
//     (eq. I_0), I_1 (eq. I_1), I_2..I_{N+1} by the integration-by-parts
//     recursion (eq. F_forward), T1 = sum c_k I_{k+1}, T2 = sum c_k I_k.
//     Every I_k is scaled by exp(lambda d^2), d = dist(t0, [0,1]), so that
//     theta far outside [alpha, beta] cannot underflow; with that scaling
//     the erf difference is written with erfcx (scaled complementary error
//     function), which has no cancellation when both arguments share a
//     sign. The common factor cancels in T1/T2.
//   otherwise: the recursion divides by 2 lambda and loses accuracy as
//     lambda -> 0, and it multiplies errors by about t0 per step when t0 is
//     far outside [0,1]. There T1 and T2 are integrated directly with a
//     Gauss-Legendre rule (16 nodes FP64 path, 12 nodes mixed path) on the
//     part of [0,1] where the scaled Gaussian exceeds e^-kSupport (all of
//     [0,1] for small lambda; a short interval next to the nearer end when
//     t0 is far outside), p evaluated by Horner in x = 2t - 1, whose
//     coefficients (from the Legendre moments) stay moderate, unlike the
//     monomial coefficients c on [0,1].
// Post-rules: if T2 <= 0 or T1/T2 is not finite, F = I_1/I_0 (the N = 0
// estimate); ABF_FLAG_CLAMP clips F to [0,1]. alpha == beta gives f(i).
#include "abf_internal.h"

namespace abf {
namespace {

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
constexpr double kSqrtPi = 1.7724538509055160273;

struct GLArgs {
  double t[kGLNodes];
  double w[kGLNodes];
};

template <int N, typename TS, typename TO>
__global__ __launch_bounds__(256) void range_kernel(
    const float* __restrict__ alpha, const float* __restrict__ beta, long long sp,
    const TS* __restrict__ mom, long long plane, const float* __restrict__ theta,
    long long tpitch, const float* __restrict__ sigma, long long spitch, int H, int W,
    unsigned flags, TO* __restrict__ out, long long opitch, GLArgs gl, Batch bt) {
  constexpr ShiftedLegTable SL{};
  constexpr LegTable LT{};
  // mixed path: 12-node rule and single-precision exponentials for the
  // quadrature weights (their 1e-7 relative error is far below the FP32
  // output's own resolution of the 0.05 tolerance); FP64 path: 16 nodes.
  constexpr bool kMixed = sizeof(TO) == 4;
  constexpr int Q = kMixed ? kGLNodesMixed : kGLNodes;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  {
    const long long z = blockIdx.z;
    alpha = byte_offset(alpha, z * bt.stack);
    beta = byte_offset(beta, z * bt.stack);
    mom = byte_offset(mom, z * bt.stack);
    theta += z * bt.img;
    sigma += z * bt.img;
    out += z * bt.out;
  }
  const long long idx = (long long)y * sp + x;
  const float a = alpha[idx], b = beta[idx];
  TO* o = out + (long long)y * opitch + x;
  if (a == b) {
    *o = TO(a);
    return;
  }
  const double da = a, delta = (double)b - da;
  const double th = theta[(long long)y * tpitch + x];
  const double sg = sigma[(long long)y * spitch + x];
  const double t0 = (th - da) * rcp(delta);
  const double lam = isinf(sg) ? 0.0 : delta * delta * rcp(2.0 * sg * sg);

  double ak[N + 1];                      // (2k+1) a~_k
  ak[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= N; ++k) ak[k] = (2.0 * k + 1.0) * (double)mom[(k - 1) * plane + idx];

  const double ts = fmin(fmax(t0, 0.0), 1.0);
  const double dist = fabs(t0 - ts);
  double T1, T2, F0;
  if (lam >= lam_split(N, kMixed) && dist * sqrt(lam) < outside_limit(kMixed)) {
    double c[N + 1];
#pragma unroll
    for (int r = 0; r <= N; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = r; k <= N; ++k) acc = fma(ak[k], SL.ell[k][r], acc);
      c[r] = acc;
    }
    const double sl = sqrt(lam);
    const double A = -sl * t0, B = sl * (1.0 - t0);
    const double dd = t0 - ts;
    const double s = lam * dd * dd;
    const double E0 = exp_neg(s - A * A);    // exp(-lam t0^2) * e^s
    const double E1 = exp_neg(s - B * B);    // exp(-lam (1-t0)^2) * e^s
    double diff;                          // (erf(B) - erf(A)) * e^s
    if (A <= 0.0 && B >= 0.0) {
      diff = 2.0 - erfcx(B) * E1 - erfcx(-A) * E0;
    } else if (A > 0.0) {
      diff = erfcx(A) * E0 - erfcx(B) * E1;
    } else {
      diff = erfcx(-B) * E1 - erfcx(-A) * E0;
    }
    const double i2l = 0.5 * rcp(lam);
    double Im2 = 0.5 * kSqrtPi * rcp(sl) * diff;     // I_0
    double Im1 = fma(t0, Im2, (E0 - E1) * i2l);      // I_1
    F0 = Im1 * rcp(Im2);
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
    const double L = lam > 0.0 ? sqrt(dist * dist + kSupport / lam) - dist : 2.0;
    const double lo = fmax(0.0, ts - L), hi = fmin(1.0, ts + L);
    const double span = hi - lo;
    // p in powers of x = 2t - 1: bx[r] = sum_k ak[k] L[k][r] (coefficients of
    // moderate size, so Horner in x on [-1, 1] is well conditioned)
    double bx[N + 1];
#pragma unroll
    for (int r = 0; r <= N; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int k = r; k <= N; k += 2) acc = fma(ak[k], LT.L[k][r], acc);
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
    F0 = J1 * rcp(J0);
  }
  double F = T1 * rcp(T2);
  if (!(T2 > 0.0) || !isfinite(F)) F = F0;
  if (flags & 1u) F = fmin(fmax(F, 0.0), 1.0);
  *o = TO(fma(delta, F, da));
}

template <int N, typename TS, typename TO>
hipError_t launch_t(const float* alpha, const float* beta, long long sp, const void* mom,
                    long long plane, const float* theta, long long tpitch, const float* sigma,
                    long long spitch, int h, int w, unsigned flags, void* out, long long opitch,
                    hipStream_t stream, const Batch& b) {
  GLArgs gl;
  const GLRule& r = gl_rule(sizeof(TO) == 4 ? kGLNodesMixed : kGLNodes);
  for (int q = 0; q < kGLNodes; ++q) {
    gl.t[q] = r.t[q];
    gl.w[q] = r.w[q];
  }
  dim3 grid((w + 63) / 64, (h + 3) / 4, b.n);
  hipLaunchKernelGGL((range_kernel<N, TS, TO>), grid, dim3(256), 0, stream, alpha, beta, sp,
                     static_cast<const TS*>(mom), plane, theta, tpitch, sigma, spitch, h, w,
                     flags, static_cast<TO*>(out), opitch, gl, b);
  return hipGetLastError();
}

template <typename TS, typename TO>
hipError_t dispatch(int N, const float* alpha, const float* beta, long long sp, const void* mom,
                    long long plane, const float* theta, long long tpitch, const float* sigma,
                    long long spitch, int h, int w, unsigned flags, void* out, long long opitch,
                    hipStream_t stream, const Batch& b) {
  switch (N) {
#define ABF_CASE(n)                                                                           \
  case n:                                                                                     \
    return launch_t<n, TS, TO>(alpha, beta, sp, mom, plane, theta, tpitch, sigma, spitch, h, \
                               w, flags, out, opitch, stream, b);
    ABF_CASE(0) ABF_CASE(1) ABF_CASE(2) ABF_CASE(3) ABF_CASE(4) ABF_CASE(5) ABF_CASE(6)
    ABF_CASE(7) ABF_CASE(8)
#undef ABF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_range(const float* alpha, const float* beta, long long sp,
                        const void* mom, long long plane_elems,
                        const float* theta_or_img, long long tpitch,
                        const float* sigma, long long spitch, int h, int w,
                        int N, int prec, unsigned flags, void* out, long long opitch,
                        hipStream_t stream, const Batch& b) {
  if (prec == 0)
    return dispatch<double, double>(N, alpha, beta, sp, mom, plane_elems, theta_or_img, tpitch,
                                    sigma, spitch, h, w, flags, out, opitch, stream, b);
  return dispatch<float, float>(N, alpha, beta, sp, mom, plane_elems, theta_or_img, tpitch,
                                sigma, spitch, h, w, flags, out, opitch, stream, b);
}

}  // namespace abf
