// Range stage: the per-pixel steps of Algorithm 1 (eqs. inv, sub,
// I_0, I_1, F_forward, BFfinal) from the moment stack, one thread
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
#include "range_eval.h"

namespace abf {
namespace {

template <int N, typename TS, typename TO>
__global__ __launch_bounds__(256) void range_kernel(
    const float* __restrict__ alpha, const float* __restrict__ beta, long long sp,
    const TS* __restrict__ mom, long long plane, const float* __restrict__ theta,
    long long tpitch, const float* __restrict__ sigma, long long spitch, int H, int W,
    unsigned flags, TO* __restrict__ out, long long opitch, Batch bt) {
  // mixed path: 12-node rule and single-precision exponentials for the
  // quadrature weights (their 1e-7 relative error is far below the FP32
  // output's own resolution of the 0.05 tolerance); FP64 path: 16 nodes.
  constexpr bool kMixed = sizeof(TO) == 4;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  // a wave is one row segment: its row and every row pointer below are
  // wave-uniform (scalar registers), and each lane adds its byte offset
  const int y = blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  {
    const BatchOffsets o = bt.at(blockIdx.z, sizeof(TO));
    alpha = byte_offset(alpha, o.stack);
    beta = byte_offset(beta, o.stack);
    mom = byte_offset(mom, o.stack);
    theta = byte_offset(theta, o.theta);
    sigma = byte_offset(sigma, o.sigma);
    out = byte_offset(out, o.out);
  }
  // every row base is wave-uniform: buffer resources in scalar registers,
  // one 32-bit byte offset per lane
  const long long row = (long long)y * sp;
  const unsigned bx4 = (unsigned)x * 4u;
  const float a = buf_ld_f32(buf_rsrc(alpha + row), bx4), b = buf_ld_f32(buf_rsrc(beta + row), bx4);
  const BufRsrc orow = buf_rsrc(out + (long long)y * opitch);
  const unsigned bxo = (unsigned)x * (unsigned)sizeof(TO);
  if (a == b) {
    buf_st(orow, bxo, TO(a));
    return;
  }
  double at[N + 1];                      // a~_k
  at[0] = 1.0;
  const unsigned bxs = (unsigned)x * (unsigned)sizeof(TS);
#pragma unroll
  for (int k = 1; k <= N; ++k) at[k] = buf_ld(buf_rsrc(mom + (k - 1) * plane + row), bxs, mom);
  const double th = buf_ld_f32(buf_rsrc(theta + (long long)y * tpitch), bx4);
  const double sg = buf_ld_f32(buf_rsrc(sigma + (long long)y * spitch), bx4);
  buf_st(orow, bxo, TO(range_eval<N, kMixed>(a, b, at, th, sg, flags)));
}


// Uniform-prior variant (Sec. III-B comparison): the N = 0 estimator on
// [f(i), 2 fbar(i) - f(i)] (ordered), fbar the window mean under the
// filter's spatial kernel, recovered from the stack's first Legendre
// moment: fbar = mid + half a~_1 (a~_1 is the mean of z in [-1, 1]). A point
// interval (f = fbar, which includes alpha = beta) gives f(i).
template <typename TS, typename TO>
__global__ __launch_bounds__(256) void uniform_kernel(
    const float* __restrict__ alpha, const float* __restrict__ beta, long long sp,
    const TS* __restrict__ mom1, const float* __restrict__ img, long long ipitch,
    const float* __restrict__ theta, long long tpitch, const float* __restrict__ sigma,
    long long spitch, int H, int W, unsigned flags, TO* __restrict__ out, long long opitch) {
  constexpr bool kMixed = sizeof(TO) == 4;
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  const long long idx = (long long)y * sp + x;
  const double a = alpha[idx], b = beta[idx];
  const double f = img[(long long)y * ipitch + x] + 0.0f;
  const double fbar = a == b ? a : fma(0.5 * (b - a), (double)mom1[idx], 0.5 * (a + b));
  const double other = 2.0 * fbar - f;
  const double lo = fmin(f, other), hi = fmax(f, other);
  TO* o = out + (long long)y * opitch + x;
  if (!(hi > lo)) {
    *o = TO(f);
    return;
  }
  const double ak[1] = {1.0};
  *o = TO(range_eval<0, kMixed>(lo, hi, ak, (double)theta[(long long)y * tpitch + x],
                                (double)sigma[(long long)y * spitch + x], flags));
}

template <int N, typename TS, typename TO>
hipError_t launch_t(const float* alpha, const float* beta, long long sp, const void* mom,
                    long long plane, const float* theta, long long tpitch, const float* sigma,
                    long long spitch, int h, int w, unsigned flags, void* out, long long opitch,
                    hipStream_t stream, const Batch& b) {
  dim3 grid((w + 63) / 64, (h + 3) / 4, b.n);
  hipLaunchKernelGGL((range_kernel<N, TS, TO>), grid, dim3(256), 0, stream, alpha, beta, sp,
                     static_cast<const TS*>(mom), plane, theta, tpitch, sigma, spitch, h, w,
                     flags, static_cast<TO*>(out), opitch, b);
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

hipError_t launch_range_uniform(const float* alpha, const float* beta, long long sp,
                                const void* mom1, const float* img, long long ipitch,
                                const float* theta_or_img, long long tpitch, const float* sigma,
                                long long spitch, int h, int w, int prec, unsigned flags,
                                void* out, long long opitch, hipStream_t stream) {
  dim3 grid((w + 63) / 64, (h + 3) / 4);
  if (prec == 0)
    hipLaunchKernelGGL((uniform_kernel<double, double>), grid, dim3(256), 0, stream, alpha, beta,
                       sp, static_cast<const double*>(mom1), img, ipitch, theta_or_img, tpitch,
                       sigma, spitch, h, w, flags, static_cast<double*>(out), opitch);
  else
    hipLaunchKernelGGL((uniform_kernel<float, float>), grid, dim3(256), 0, stream, alpha, beta,
                       sp, static_cast<const float*>(mom1), img, ipitch, theta_or_img, tpitch,
                       sigma, spitch, h, w, flags, static_cast<float*>(out), opitch);
  return hipGetLastError();
}

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
