// Device helpers shared by the moment kernels (moments.hip) and the
// recursive kernel (recursive.hip): the per-pixel epilogue that turns window
// moments about an origin into shifted-Legendre moments (Prop. 3), the
// stack store and fused range stage of a finished pixel, and the direct
// recompute of pixels whose shift is ill-conditioned.
#pragma once

#include "abf_internal.h"
#include "range_eval.h"

namespace abf {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-pixel epilogue: m[1..N] are the window moments of u = f - c (m[0] = 1).
// Computes a~_1..a~_N into m[1..N] and returns false, or returns true when
// the binomial shift is too ill-conditioned for the requested precision
// (the caller then recomputes the pixel directly). alpha == beta gives 0s.
template <int N>
__device__ __forceinline__ bool legendre_from_moments(double (&m)[N + 1], float a, float b,
                                                      double c, double cond_max) {
  constexpr LegTable LT{};
  if (a == b) {
#pragma unroll
    for (int k = 1; k <= N; ++k) m[k] = 0.0;
    return false;
  }
  const double mid = 0.5 * ((double)a + (double)b) - c;
  const double half = 0.5 * ((double)b - (double)a);
  const double ih = rcp(half);      // (a few ulp; a scale, not an exact quantity)
  // The shift below amplifies the rounding of m_r by about
  // rho^k, rho = (|mid| + half) / half.
  const double rho = fma(fabs(mid), ih, 1.0);
  double rn = rho;
#pragma unroll
  for (int k = 1; k < N; ++k) rn *= rho;
  if (!(rn <= cond_max)) return true;
  // binomial shift of the moments to the origin mid (Prop. 3):
  // nu_k = sum_r C(k, r) (-mid)^(k-r) m_r, by repeated synthetic steps
  const double s = -mid;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int k = N; k > j; --k) m[k] = fma(s, m[k - 1], m[k]);
  // scale to z in [-1, 1]
  double sc = ih;
#pragma unroll
  for (int k = 1; k <= N; ++k) {
    m[k] *= sc;
    sc *= ih;
  }
  // Legendre moments a~_k = sum_r L[k][r] nu_r (only r = k, k-2, ... are non-zero)
  double out[N + 1];
#pragma unroll
  for (int k = 1; k <= N; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int r = k; r >= 0; r -= 2) acc = fma(LT.L[k][r], m[r], acc);
    out[k] = acc;
  }
#pragma unroll
  for (int k = 1; k <= N; ++k) m[k] = out[k];
  return false;
}

// Fused range stage: theta (or f), sigma and the output for kernels that
// finish each pixel's filter right after its moments (the range half of
// Algorithm 1 in registers). keep_stack also stores the moments in the
// stack.
struct FuseArgs {
  const float* theta;
  const float* sigma;
  long long tpitch;
  void* out;
  long long opitch;
  unsigned flags;
  int keep_stack;
};

// Completes pixel (y, x) from its Legendre moments m[1..N]: stores them
// (stack path, or fused with keep_stack) and, when fused, evaluates the
// range stage and writes the output. The moments enter the range stage
// rounded to the stack's type, so the fused result equals the stack path's.
template <int N, typename TS, bool FUSED>
__device__ __forceinline__ void finish_pixel(const double (&m)[N + 1], float a, float b, int y,
                                             int x, long long idx, TS* __restrict__ mom,
                                             long long plane, const FuseArgs& fz) {
  if (!FUSED || fz.keep_stack) {
#pragma unroll
    for (int k = 1; k <= N; ++k) mom[(k - 1) * plane + idx] = TS(m[k]);
  }
  if (FUSED) {
    TS* o = static_cast<TS*>(fz.out) + (long long)y * fz.opitch + x;
    if (a == b) {
      *o = TS(a);
    } else {
      double ak[N + 1];                  // a~_k as stored in the stack
      ak[0] = 1.0;
#pragma unroll
      for (int k = 1; k <= N; ++k) ak[k] = (double)TS(m[k]);
      const long long ti = (long long)y * fz.tpitch + x;
      *o = TS(range_eval<N, sizeof(TS) == 4>(a, b, ak, (double)fz.theta[ti], (double)fz.sigma[ti],
                                              fz.flags));
    }
  }
}

// finish_pixel's fused path for a pixel of a wave-uniform row, theta and
// sigma already loaded: the output goes through a buffer resource (row base
// in scalar registers, the lane's 32-bit byte offset xb); the same values.
// The stack planes (keep_stack only) take plain stores: eight more buffer
// resources would hold 32 scalar registers across the row, which the
// compiler then spills to vector lanes on the default path as well.
template <int N, typename TS>
__device__ __forceinline__ void fused_pixel(const double (&m)[N + 1], float a, float b, float th,
                                            float sg, TS* __restrict__ mrow, long long plane,
                                            unsigned xb, BufRsrc orow, const FuseArgs& fz) {
  if (fz.keep_stack) {
    TS* p = mrow + xb / (unsigned)sizeof(TS);
#pragma unroll
    for (int k = 1; k <= N; ++k, p += plane) *p = TS(m[k]);
  }
  if (a == b) {
    buf_st(orow, xb, TS(a));
    return;
  }
  double ak[N + 1];                    // a~_k as stored in the stack
  ak[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= N; ++k) ak[k] = (double)TS(m[k]);
  buf_st(orow, xb, TS(range_eval<N, sizeof(TS) == 4>(a, b, ak, (double)th, (double)sg,
                                                     fz.flags)));
}

// P_k(z) = a_k z P_{k-1}(z) - b_k P_{k-2}(z), a_k = (2k-1)/k, b_k = (k-1)/k
// (the three-term recurrence with its divisions folded into constants).
struct LegRec {
  double a[kNMax + 1];
  double b[kNMax + 1];
  constexpr LegRec() : a{}, b{} {
    for (int k = 2; k <= kNMax; ++k) {
      a[k] = (2.0 * k - 1.0) / k;
      b[k] = (k - 1.0) / k;
    }
  }
};

// Adds wt * P_k(z), k = 1..N, to acc[1..N].
template <int N>
__device__ __forceinline__ void add_legendre(double z, double wt, double (&acc)[N + 1]) {
  constexpr LegRec LR{};
  double p0 = 1.0, p1 = z;
  acc[1] = fma(wt, p1, acc[1]);
#pragma unroll
  for (int k = 2; k <= N; ++k) {
    const double p2 = fma(LR.a[k] * z, p1, -LR.b[k] * p0);
    acc[k] = fma(wt, p2, acc[k]);
    p0 = p1;
    p1 = p2;
  }
}

// Direct evaluation of a~_k = sum_j omega_j P_k(z_j) for one pixel (y, x),
// z_j = (f(i-j) - mid) / half, by the whole wave: lanes split the window's
// taps, each evaluates P_1..P_N by the three-term recurrence, and the
// partial sums are reduced across the wave. Used for the rare pixels whose
// shift is ill-conditioned. wts == nullptr means box weights.
template <int N>
__device__ __forceinline__ void direct_legendre(const float* __restrict__ img, long long pitch,
                                                int H, int W, int R, int y, int x, float a,
                                                float b, const double* __restrict__ wts,
                                                double norm, int lane, double (&acc)[N + 1]) {
  const double mid = 0.5 * ((double)a + (double)b);
  const double ih = 2.0 / ((double)b - (double)a);
  const int w = 2 * R + 1;
  const int n = w * w;
#pragma unroll
  for (int k = 1; k <= N; ++k) acc[k] = 0.0;
  for (int t = lane; t < n; t += kWave) {
    const int dy = t / w - R, dx = t - (t / w) * w - R;
    const int yy = min(max(y + dy, 0), H - 1), xx = min(max(x + dx, 0), W - 1);
    const double z = ((double)img[(long long)yy * pitch + xx] - mid) * ih;
    add_legendre<N>(z, wts ? wts[dy + R] * wts[dx + R] : 1.0, acc);
  }
#pragma unroll
  for (int k = 1; k <= N; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    acc[k] = v * norm;
  }
}

// The same sum evaluated by one lane for its own pixel (used when most of a
// wave's pixels need the recompute, so that all lanes work at once).
template <int N>
__device__ __forceinline__ void direct_legendre_lane(const float* __restrict__ img, long long pitch,
                                                     int H, int W, int R, int y, int x, float a,
                                                     float b, const double* __restrict__ wts,
                                                     double norm, double (&acc)[N + 1]) {
  const double mid = 0.5 * ((double)a + (double)b);
  const double ih = 2.0 / ((double)b - (double)a);
#pragma unroll
  for (int k = 1; k <= N; ++k) acc[k] = 0.0;
  for (int dy = -R; dy <= R; ++dy) {
    const float* row = img + (long long)min(max(y + dy, 0), H - 1) * pitch;
    const double wy = wts ? wts[dy + R] : 1.0;
    for (int dx = -R; dx <= R; ++dx) {
      const double z = ((double)row[min(max(x + dx, 0), W - 1)] - mid) * ih;
      add_legendre<N>(z, wts ? wy * wts[dx + R] : 1.0, acc);
    }
  }
#pragma unroll
  for (int k = 1; k <= N; ++k) acc[k] *= norm;
}

// Recompute the flagged pixels of a wave: one pixel at a time by the whole
// wave when few are flagged, every flagged lane its own pixel when many are.
template <int N, typename TS, bool FUSED>
__device__ __forceinline__ void recompute_flagged(unsigned long long mask, bool mine, int y, int x,
                                                  float a, float b, const float* __restrict__ img,
                                                  long long pitch, int H, int W, int R,
                                                  const double* __restrict__ wts, double norm,
                                                  TS* __restrict__ mom, long long plane,
                                                  long long sp, int lane, const FuseArgs& fz) {
  if (__popcll(mask) > 24) {
    if (mine) {
      double acc[N + 1];
      direct_legendre_lane<N>(img, pitch, H, W, R, y, x, a, b, wts, norm, acc);
      finish_pixel<N, TS, FUSED>(acc, a, b, y, x, (long long)y * sp + x, mom, plane, fz);
    }
    return;
  }
  while (mask) {
    const int l = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    const int yl = __shfl(y, l, kWave), xl = __shfl(x, l, kWave);
    const float al = __shfl(a, l, kWave), bl = __shfl(b, l, kWave);
    double acc[N + 1];
    direct_legendre<N>(img, pitch, H, W, R, yl, xl, al, bl, wts, norm, lane, acc);
    if (lane == 0)
      finish_pixel<N, TS, FUSED>(acc, al, bl, yl, xl, (long long)yl * sp + xl, mom, plane, fz);
  }
}

// Shift amplification tolerated by the FP64 path, by degree.
constexpr double fp64_cond_max(int N) { return N <= 5 ? 1e8 : (N == 6 ? 1e6 : 1e4); }

}  // namespace
}  // namespace abf
