// Parameter maps of the applications (Sec. IV), computed on the GPU next to
// the filter:
//   sharpening (Sec. IV-A): theta = f + zeta, zeta = f - fbar with fbar the
//     mean over the (2r+1)^2 window, and sigma from an affine map of
//     |LoG * f| (low values -> high sigma);
//   texture filtering (Sec. IV-C): sigma from an affine map of
//     mRTV = Delta max|grad f| / (sum|grad f| + eps) over the window W_i,
//     Delta the window's intensity range, on a grey version of the image.
// The paper leaves the constants open; the kernels take them as arguments:
// the LoG is the sum over both axes of the second derivative of a sampled
// Gaussian (std s, radius q = round(4 s), normalised to sum 1) along one axis
// times the Gaussian along the other; gradients are central differences;
// the affine map is sigma = hi - (hi - lo) min(v / v_ref, 1); every border
// is clamp-to-edge; sums are FP64.
//
// Each kernel: one thread per output pixel of a 16 x 16 tile, the padded
// input tile staged in LDS; the image index is the grid's z.
#include "abf_internal.h"

namespace abf {
namespace {

constexpr int kMT = 16;              // output tile side
constexpr int kMapsHaloMax = 32;     // largest halo (window radius, LoG radius)

__device__ __forceinline__ void load_tile(const float* __restrict__ img, long long pitch, int H,
                                          int W, int bx, int by, int h, float* tile) {
  const int E = kMT + 2 * h;
  for (int i = threadIdx.x; i < E * E; i += kMT * kMT) {
    const int rr = i / E, cc = i - rr * E;
    const int gy = min(max(by - h + rr, 0), H - 1);
    const int gx = min(max(bx - h + cc, 0), W - 1);
    tile[i] = img[(long long)gy * pitch + gx] + 0.0f;
  }
}

__device__ __forceinline__ double affine_sigma(double v, double lo, double hi, double v_ref) {
  return hi - (hi - lo) * fmin(v / v_ref, 1.0);
}

// theta = 2 f - fbar and sigma = affine(|LoG f|); h = max(r, q). Both are
// separable: phase A forms, for every padded row of the tile and every
// output column, the row's box sum over 2r+1 columns and its convolutions
// with g and d2 over 2q+1 columns; phase B sums those down the columns.
__global__ __launch_bounds__(kMT* kMT) void sharpen_maps_kernel(
    const float* __restrict__ img, long long pitch, int H, int W, int r, double s, int q,
    double lo, double hi, double v_ref, float* __restrict__ theta, float* __restrict__ sigma,
    long long op, Batch bt) {
  extern __shared__ double rows[];                   // hbox, hg, hd2: E x kMT each; then the tile
  __shared__ double g[2 * kMapsHaloMax + 1], d2[2 * kMapsHaloMax + 1];
  img += blockIdx.z * bt.img;
  theta += blockIdx.z * bt.out;
  sigma += blockIdx.z * bt.out;
  const int h = max(r, q);
  const int E = kMT + 2 * h;
  double* hbox = rows;
  double* hg = rows + E * kMT;
  double* hd2 = rows + 2 * E * kMT;
  float* tile = reinterpret_cast<float*>(rows + 3 * E * kMT);
  const int bx = blockIdx.x * kMT, by = blockIdx.y * kMT;
  if (threadIdx.x == 0) {
    // sampled Gaussian normalised to sum 1, and its second derivative
    double z = 0.0;
    for (int i = 0; i <= 2 * q; ++i) {
      const double x = (double)(i - q);
      g[i] = exp(-0.5 * x * x / (s * s));
      z += g[i];
    }
    for (int i = 0; i <= 2 * q; ++i) {
      const double x = (double)(i - q);
      g[i] /= z;
      d2[i] = (x * x / (s * s * s * s) - 1.0 / (s * s)) * g[i];
    }
  }
  load_tile(img, pitch, H, W, bx, by, h, tile);
  __syncthreads();
  // phase A: item = (padded row, output column), columns fastest
  for (int it = threadIdx.x; it < E * kMT; it += kMT * kMT) {
    const int row = it / kMT, col = it - row * kMT;
    const float* t = tile + row * E + col + h;
    double sb = 0.0, sg_ = 0.0, sd = 0.0;
    for (int dx = -r; dx <= r; ++dx) sb += (double)t[dx];
    for (int dx = -q; dx <= q; ++dx) {
      const double v = t[dx];
      sg_ = fma(g[dx + q], v, sg_);
      sd = fma(d2[dx + q], v, sd);
    }
    hbox[it] = sb;
    hg[it] = sg_;
    hd2[it] = sd;
  }
  __syncthreads();
  const int tx = threadIdx.x % kMT, ty = threadIdx.x / kMT;
  const int x = bx + tx, y = by + ty;
  if (x >= W || y >= H) return;
  double sum = 0.0;
  for (int dy = -r; dy <= r; ++dy) sum += hbox[(ty + h + dy) * kMT + tx];
  double L = 0.0;
  for (int dy = -q; dy <= q; ++dy) {
    const int k = (ty + h + dy) * kMT + tx;
    L = fma(d2[dy + q], hg[k], fma(g[dy + q], hd2[k], L));
  }
  const double w = 2.0 * r + 1.0;
  const double f = tile[(ty + h) * E + tx + h];
  const double fbar = sum / (w * w);
  theta[(long long)y * op + x] = (float)(2.0 * f - fbar);
  sigma[(long long)y * op + x] = (float)affine_sigma(fabs(L), lo, hi, v_ref);
}

// sigma = affine(mRTV) over the (2r+1)^2 window; the tile's halo is r + 1
// (the gradients at the window's edge need one more pixel).
__global__ __launch_bounds__(kMT* kMT) void mrtv_sigma_kernel(
    const float* __restrict__ img, long long pitch, int H, int W, int r, double eps, double lo,
    double hi, double v_ref, float* __restrict__ sigma, long long op, Batch bt) {
  extern __shared__ float tile[];                    // (kMT + 2r + 2)^2 floats, then gradients
  img += blockIdx.z * bt.img;
  sigma += blockIdx.z * bt.out;
  const int h = r + 1;
  const int E = kMT + 2 * h;
  const int G = kMT + 2 * r;                         // gradient tile side
  double* gn = reinterpret_cast<double*>(tile + ((E * E + 1) & ~1));
  const int bx = blockIdx.x * kMT, by = blockIdx.y * kMT;
  load_tile(img, pitch, H, W, bx, by, h, tile);
  __syncthreads();
  // |grad f| at the G x G pixels within r of the output tile; the clamp to
  // the image applies to the differenced pixels, as on the padded image
  for (int i = threadIdx.x; i < G * G; i += kMT * kMT) {
    const int gy = i / G, gx = i - gy * G;
    const int py = by - r + gy, px = bx - r + gx;             // image position
    const int cy = min(max(py, 0), H - 1), cx = min(max(px, 0), W - 1);
    const int ty0 = cy - (by - h), tx0 = cx - (bx - h);        // its tile position
    const int xm = min(max(cx - 1, 0), W - 1) - (bx - h), xp = min(max(cx + 1, 0), W - 1) - (bx - h);
    const int ym = min(max(cy - 1, 0), H - 1) - (by - h), yp = min(max(cy + 1, 0), H - 1) - (by - h);
    const double ddx = 0.5 * ((double)tile[ty0 * E + xp] - (double)tile[ty0 * E + xm]);
    const double ddy = 0.5 * ((double)tile[yp * E + tx0] - (double)tile[ym * E + tx0]);
    gn[i] = sqrt(ddx * ddx + ddy * ddy);
  }
  __syncthreads();
  const int tx = threadIdx.x % kMT, ty = threadIdx.x / kMT;
  const int x = bx + tx, y = by + ty;
  if (x >= W || y >= H) return;
  float fmin_ = INFINITY, fmax_ = -INFINITY;
  double gmax = 0.0, gsum = 0.0;
  for (int dy = -r; dy <= r; ++dy)
    for (int dx = -r; dx <= r; ++dx) {
      const float v = tile[(ty + h + dy) * E + tx + h + dx];
      fmin_ = fminf(fmin_, v);
      fmax_ = fmaxf(fmax_, v);
      const double gv = gn[(ty + r + dy) * G + tx + r + dx];
      gmax = fmax(gmax, gv);
      gsum += gv;
    }
  const double m = ((double)fmax_ - (double)fmin_) * gmax / (gsum + eps);
  sigma[(long long)y * op + x] = (float)affine_sigma(m, lo, hi, v_ref);
}

// grey = 0.299 R + 0.587 G + 0.114 B of planar colour images
__global__ __launch_bounds__(256) void grey_kernel(const float* __restrict__ rgb, long long pitch,
                                                   long long cstride, int H, int W,
                                                   float* __restrict__ out, long long op,
                                                   Batch bt) {
  const int x = blockIdx.x * 64 + (threadIdx.x & 63);
  const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (x >= W || y >= H) return;
  const float* p = rgb + blockIdx.z * bt.img + (long long)y * pitch + x;
  const float v = 0.299f * p[0] + 0.587f * p[cstride] + 0.114f * p[2 * cstride];
  out[blockIdx.z * bt.out + (long long)y * op + x] = v;
}

}  // namespace

bool maps_params_ok(int r, double s) {
  const int q = (int)(4.0 * s + 0.5);
  return r >= 0 && r <= kMapsHaloMax && s > 0.0 && q <= kMapsHaloMax;
}

hipError_t launch_sharpen_maps(const float* img, long long pitch, int h, int w, int r, double s,
                               double lo, double hi, double v_ref, float* theta, float* sigma,
                               long long op, hipStream_t stream, const Batch& b) {
  const int q = (int)(4.0 * s + 0.5);
  const int halo = r > q ? r : q;
  const int E = kMT + 2 * halo;
  dim3 grid((w + kMT - 1) / kMT, (h + kMT - 1) / kMT, b.n);
  const size_t lds = (size_t)3 * E * kMT * sizeof(double) + (size_t)E * E * sizeof(float);
  hipLaunchKernelGGL(sharpen_maps_kernel, grid, dim3(kMT * kMT), lds, stream, img, pitch, h, w, r,
                     s, q, lo, hi, v_ref, theta, sigma, op, b);
  return hipGetLastError();
}

hipError_t launch_mrtv_sigma(const float* img, long long pitch, int h, int w, int r, double eps,
                             double lo, double hi, double v_ref, float* sigma, long long op,
                             hipStream_t stream, const Batch& b) {
  const int E = kMT + 2 * (r + 1), G = kMT + 2 * r;
  dim3 grid((w + kMT - 1) / kMT, (h + kMT - 1) / kMT, b.n);
  const size_t lds = (size_t)((E * E + 1) & ~1) * sizeof(float) + (size_t)G * G * sizeof(double);
  hipLaunchKernelGGL(mrtv_sigma_kernel, grid, dim3(kMT * kMT), lds, stream, img, pitch, h, w, r,
                     eps, lo, hi, v_ref, sigma, op, b);
  return hipGetLastError();
}

hipError_t launch_grey(const float* rgb, long long pitch, long long cstride, int h, int w,
                       float* out, long long op, hipStream_t stream, const Batch& b) {
  dim3 grid((w + 63) / 64, (h + 3) / 4, b.n);
  hipLaunchKernelGGL(grey_kernel, grid, dim3(256), 0, stream, rgb, pitch, cstride, h, w, out, op,
                     b);
  return hipGetLastError();
}

}  // namespace abf
