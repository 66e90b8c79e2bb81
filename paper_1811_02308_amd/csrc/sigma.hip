// Per-pixel range-kernel width from local contrast, for the texture
// workload: sigma(i) = clamp(scale * sd(i), lo, hi), where sd(i) is the
// population standard deviation of f over the clamp-to-edge window
// [-r, r]^2 of i. (The paper sets sigma from a local texture measure, mRTV,
// through an affine map, Sec. IV-C; this is the simpler contrast rule of
// the texture benchmark.)
//
// One thread per output pixel of a 16 x 16 tile; the padded tile is staged
// in LDS. Two FP64 passes over the window (mean, then squared deviations),
// so no cancellation between a sum and a sum of squares.
#include "abf_internal.h"

namespace abf {
namespace {

constexpr int kST = 16;
constexpr int kSigmaRMax = 32;

__global__ __launch_bounds__(kST* kST) void sigma_std_kernel(
    const float* __restrict__ img, long long pitch, int H, int W, int r, double scale, double lo,
    double hi, float* __restrict__ out, long long op, Batch bt) {
  extern __shared__ float tile[];
  img += blockIdx.z * bt.img;
  out += blockIdx.z * bt.out;
  const int E = kST + 2 * r;
  const int bx = blockIdx.x * kST, by = blockIdx.y * kST;
  for (int i = threadIdx.x; i < E * E; i += kST * kST) {
    const int rr = i / E, cc = i - rr * E;
    const int gy = min(max(by - r + rr, 0), H - 1);
    const int gx = min(max(bx - r + cc, 0), W - 1);
    tile[i] = img[(long long)gy * pitch + gx];
  }
  __syncthreads();
  const int tx = threadIdx.x % kST, ty = threadIdx.x / kST;
  const int x = bx + tx, y = by + ty;
  if (x >= W || y >= H) return;
  const int w = 2 * r + 1;
  double sum = 0.0;
  for (int dy = 0; dy < w; ++dy)
    for (int dx = 0; dx < w; ++dx) sum += (double)tile[(ty + dy) * E + tx + dx];
  const double inv_n = 1.0 / ((double)w * (double)w);
  const double mean = sum * inv_n;
  double ss = 0.0;
  for (int dy = 0; dy < w; ++dy)
    for (int dx = 0; dx < w; ++dx) {
      const double d = (double)tile[(ty + dy) * E + tx + dx] - mean;
      ss = fma(d, d, ss);
    }
  const double sd = sqrt(ss * inv_n);
  out[(long long)y * op + x] = (float)fmin(fmax(scale * sd, lo), hi);
}

}  // namespace

hipError_t launch_sigma_std(const float* img, long long pitch, int h, int w, int r,
                            double scale, double lo, double hi, float* out, long long opitch,
                            hipStream_t stream, const Batch& b) {
  if (r > kSigmaRMax) return hipErrorInvalidValue;
  dim3 grid((w + kST - 1) / kST, (h + kST - 1) / kST, b.n);
  const size_t lds = (size_t)(kST + 2 * r) * (kST + 2 * r) * sizeof(float);
  hipLaunchKernelGGL(sigma_std_kernel, grid, dim3(kST * kST), lds, stream, img, pitch, h, w, r,
                     scale, lo, hi, out, opitch, b);
  return hipGetLastError();
}

}  // namespace abf
