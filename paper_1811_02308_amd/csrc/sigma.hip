// Per-pixel range-kernel width from local contrast, for the texture
// workload: sigma(i) = clamp(scale * sd(i), lo, hi), where sd(i) is the
// population standard deviation of f over the clamp-to-edge window
// [-r, r]^2 of i. (The paper sets sigma from a local texture measure, mRTV,
// through an affine map, Sec. IV-C; this is the simpler contrast rule of
// the texture benchmark.)
//
// One thread per output pixel of a 16 x 16 tile; the padded tile is staged
// in LDS. The window's values are taken in FP64 as differences d = f - c
// from the tile's central input value c, and the sums of d and d^2 are
// separable: horizontal sums over 2r + 1 columns for every padded row (in
// LDS), then vertical sums over 2r + 1 rows. var = S2/n - (S1/n)^2 then
// carries an absolute error of a few 1e-16 max|d|^2 (rounding of the sums
// and their cancellation): below 1e-10 on data in [0, 255], far below the
// FP32 output's resolution.
#include "abf_internal.h"

namespace abf {
namespace {

constexpr int kST = 16;
constexpr int kSigmaRMax = 32;

__global__ __launch_bounds__(kST* kST) void sigma_std_kernel(
    const float* __restrict__ img, long long pitch, int H, int W, int r, double scale, double lo,
    double hi, float* __restrict__ out, long long op, Batch bt) {
  // dynamic LDS: the E x E tile (floats, E = 16 + 2r), then the E x 16
  // horizontal sums of d and of d^2 (doubles, 8-byte aligned)
  extern __shared__ __attribute__((aligned(8))) float tile[];
  img += blockIdx.z * bt.img;
  out += blockIdx.z * bt.out;
  const int E = kST + 2 * r;
  double* const hs1 = reinterpret_cast<double*>(tile + ((E * E + 1) & ~1));
  double* const hs2 = hs1 + E * kST;
  const int bx = blockIdx.x * kST, by = blockIdx.y * kST;
  for (int i = threadIdx.x; i < E * E; i += kST * kST) {
    const int rr = i / E, cc = i - rr * E;
    const int gy = min(max(by - r + rr, 0), H - 1);
    const int gx = min(max(bx - r + cc, 0), W - 1);
    tile[i] = img[(long long)gy * pitch + gx];
  }
  __syncthreads();
  const double c = (double)tile[(r + kST / 2) * E + r + kST / 2];
  const int w = 2 * r + 1;
  // horizontal: padded row rr, output column cc
  for (int i = threadIdx.x; i < E * kST; i += kST * kST) {
    const int rr = i / kST, cc = i - rr * kST;
    const float* t = tile + rr * E + cc;
    double s1 = 0.0, s2 = 0.0;
    for (int dx = 0; dx < w; ++dx) {
      const double d = (double)t[dx] - c;
      s1 += d;
      s2 = fma(d, d, s2);
    }
    hs1[i] = s1;
    hs2[i] = s2;
  }
  __syncthreads();
  const int tx = threadIdx.x % kST, ty = threadIdx.x / kST;
  const int x = bx + tx, y = by + ty;
  if (x >= W || y >= H) return;
  double s1 = 0.0, s2 = 0.0;
  for (int dy = 0; dy < w; ++dy) {
    s1 += hs1[(ty + dy) * kST + tx];
    s2 += hs2[(ty + dy) * kST + tx];
  }
  const double inv_n = 1.0 / ((double)w * (double)w);
  const double m1 = s1 * inv_n;
  const double var = fmax(fma(-m1, m1, s2 * inv_n), 0.0);
  out[(long long)y * op + x] = (float)fmin(fmax(scale * sqrt(var), lo), hi);
}

}  // namespace

hipError_t launch_sigma_std(const float* img, long long pitch, int h, int w, int r,
                            double scale, double lo, double hi, float* out, long long opitch,
                            hipStream_t stream, const Batch& b) {
  if (r > kSigmaRMax) return hipErrorInvalidValue;
  dim3 grid((w + kST - 1) / kST, (h + kST - 1) / kST, b.n);
  const int E = kST + 2 * r;
  const size_t lds = (size_t)((E * E + 1) & ~1) * sizeof(float) + 2 * (size_t)E * kST * sizeof(double);
  hipLaunchKernelGGL(sigma_std_kernel, grid, dim3(kST * kST), lds, stream, img, pitch, h, w, r,
                     scale, lo, hi, out, opitch, b);
  return hipGetLastError();
}

}  // namespace abf
