// Brute-force adaptive bilateral filter, eqs. (BF_adaptive1), (BF_adaptive2)
// with the Gaussian range kernel of eq. (r_kernel): O((2R+1)^2) per pixel.
//
// One thread per output pixel; the workgroup stages its (16+2R)^2 padded
// input tile in LDS when it fits (R <= 48), otherwise taps are read from
// global memory (cached). Two sweeps over the window: the first finds the
// smallest range exponent (f(i-j) - theta(i))^2 / (2 sigma(i)^2), the second
// accumulates with every exponent shifted by it; the common factor cancels
// in the ratio and keeps the largest weight at 1, so nothing underflows.
// Box weights are uniform; Gaussian weights exp(-|j|^2/(2 sigma_s^2)) are
// folded into the exponent (normalisation cancels in the ratio).
#include "abf_internal.h"

namespace abf {
namespace {

constexpr int kT = 16;
constexpr int kLdsR = 48;

template <typename T>
__device__ __forceinline__ T dexp(T x);
template <>
__device__ __forceinline__ double dexp<double>(double x) { return exp(x); }
template <>
__device__ __forceinline__ float dexp<float>(float x) { return expf(x); }

template <typename T, bool LDS>
__global__ __launch_bounds__(kT* kT) void brute_kernel(
    const float* __restrict__ img, const float* __restrict__ theta,
    const float* __restrict__ sigma, long long pitch, int H, int W, int R, int gauss,
    T inv2ss, T* __restrict__ out, long long opitch) {
  extern __shared__ float tile[];
  const int E = kT + 2 * R;
  const int bx = blockIdx.x * kT, by = blockIdx.y * kT;
  if (LDS) {
    for (int i = threadIdx.x; i < E * E; i += kT * kT) {
      const int r = i / E, cc = i - r * E;
      const int gy = min(max(by - R + r, 0), H - 1);
      const int gx = min(max(bx - R + cc, 0), W - 1);
      tile[i] = img[(long long)gy * pitch + gx] + 0.0f;
    }
    __syncthreads();
  }
  const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
  const int x = bx + tx, y = by + ty;
  if (x >= W || y >= H) return;
  const T th = theta ? (T)theta[(long long)y * pitch + x] : (T)(img[(long long)y * pitch + x] + 0.0f);
  const T sg = sigma[(long long)y * pitch + x];
  const T irr = T(1) / (T(2) * sg * sg);           // 0 when sigma = +inf
  auto tap = [&](int dy, int dx) -> T {
    if (LDS) return (T)tile[(ty + R + dy) * E + (tx + R + dx)];
    const int gy = min(max(y + dy, 0), H - 1);
    const int gx = min(max(x + dx, 0), W - 1);
    return (T)(img[(long long)gy * pitch + gx] + 0.0f);
  };
  T emin = T(INFINITY);
  for (int dy = -R; dy <= R; ++dy) {
    const T ey = gauss ? (T)(dy * dy) * inv2ss : T(0);
    for (int dx = -R; dx <= R; ++dx) {
      const T v = tap(dy, dx) - th;
      const T e = fma(v * v, irr, gauss ? fma((T)(dx * dx), inv2ss, ey) : T(0));
      emin = fmin(emin, e);
    }
  }
  T num = 0, den = 0;
  for (int dy = -R; dy <= R; ++dy) {
    const T ey = gauss ? (T)(dy * dy) * inv2ss : T(0);
    for (int dx = -R; dx <= R; ++dx) {
      const T f = tap(dy, dx);
      const T v = f - th;
      const T e = fma(v * v, irr, gauss ? fma((T)(dx * dx), inv2ss, ey) : T(0));
      const T wgt = dexp<T>(emin - e);
      num = fma(wgt, f, num);
      den += wgt;
    }
  }
  out[(long long)y * opitch + x] = num / den;
}

template <typename T>
hipError_t launch_t(const float* img, const float* theta, const float* sigma, long long pitch,
                    int h, int w, int kind, double sigma_s, int R, void* out, long long opitch,
                    hipStream_t stream) {
  const double s = sigma_s > 0 ? sigma_s : (R > 0 ? R / 3.0 : 1.0);
  const T inv2ss = (T)(1.0 / (2.0 * s * s));
  dim3 grid((w + kT - 1) / kT, (h + kT - 1) / kT);
  const int gauss = kind == 1;
  if (R <= kLdsR) {
    const size_t lds = (size_t)(kT + 2 * R) * (kT + 2 * R) * sizeof(float);
    hipLaunchKernelGGL((brute_kernel<T, true>), grid, dim3(kT * kT), lds, stream, img, theta,
                       sigma, pitch, h, w, R, gauss, inv2ss, static_cast<T*>(out), opitch);
  } else {
    hipLaunchKernelGGL((brute_kernel<T, false>), grid, dim3(kT * kT), 0, stream, img, theta,
                       sigma, pitch, h, w, R, gauss, inv2ss, static_cast<T*>(out), opitch);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_brute(const float* img, const float* theta, const float* sigma,
                        long long pitch, int h, int w, int kernel_kind, double sigma_s,
                        int rho, int prec, void* out, long long opitch, hipStream_t stream) {
  if (prec == 0)
    return launch_t<double>(img, theta, sigma, pitch, h, w, kernel_kind, sigma_s, rho, out,
                            opitch, stream);
  return launch_t<float>(img, theta, sigma, pitch, h, w, kernel_kind, sigma_s, rho, out, opitch,
                         stream);
}

}  // namespace abf
