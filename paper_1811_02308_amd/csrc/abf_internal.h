// Internal declarations shared by the HIP translation units of libabf.
// Device helpers, compile-time coefficient tables and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace abf {

constexpr int kNMax = 8;
constexpr int kRhoMax = 96;
constexpr int kWave = 64;

// Minimum and maximum of two finite floats in one instruction each: the
// median of (a, b, -inf) and of (a, b, +inf). fminf and fmaxf must also
// quiet signalling NaNs, which costs two more instructions per call on
// values loaded from memory. The kernels' inputs are finite (a documented
// precondition) and carry no -0 (they add +0.0f on load), so both forms
// give the same bits. A kernel makes one FinMinMax at its start: the two
// infinities pass once through an empty asm statement (no instruction;
// they stay in scalar registers), so that the optimizer neither turns the
// median back into fminf / fmaxf nor rebuilds the constants at every use.
struct FinMinMax {
  float lo, hi;
  __device__ FinMinMax() : lo(-INFINITY), hi(INFINITY) { asm("" : "+s"(lo), "+s"(hi)); }
  __device__ float min(float a, float b) const { return __builtin_amdgcn_fmed3f(a, b, lo); }
  __device__ float max(float a, float b) const { return __builtin_amdgcn_fmed3f(a, b, hi); }
};

// Gauss-Legendre rules on [0, 1] used by the range stage: 16 nodes for the
// FP64 path, 12 for the mixed path.
constexpr int kGLNodes = 16;
constexpr int kGLNodesMixed = 12;

// cos(x) for 0 <= x <= pi by its Taylor series (terms to x^58/58!, far
// below FP64 rounding there); only the starting guess of the root search.
__host__ __device__ constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}

// Nodes t and weights w of the Q-node rule on [0, 1] (entries beyond Q are
// 0): the roots z of P_Q by Newton's iteration from the starting guess
// cos(pi (i + 3/4) / (Q + 1/2)), with the three-term recurrence for P_Q and
// P_Q' = Q (z P_Q - P_{Q-1}) / (z^2 - 1); mapped by t = (1 - z)/2, weight
// 1 / ((1 - z^2) P_Q'(z)^2) (half the weight on [-1, 1]). Evaluated at
// compile time, so kernels take the rule as literal constants.
struct GLRule {
  double t[kGLNodes];
  double w[kGLNodes];
  __host__ __device__ constexpr explicit GLRule(int Q) : t{}, w{} {
    for (int i = 0; i < Q; ++i) {
      double z = cos_series(3.14159265358979323846 * (i + 0.75) / (Q + 0.5));
      double p0 = 1.0, p1 = z, dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= Q; ++k) {
          const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = Q * (z * p1 - p0) / (z * z - 1.0);
        const double dz = p1 / dp;
        z -= dz;
        if ((dz < 0.0 ? -dz : dz) < 1e-17) break;
      }
      p0 = 1.0;
      p1 = z;
      for (int k = 2; k <= Q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = Q * (z * p1 - p0) / (z * z - 1.0);
      t[i] = 0.5 * (1.0 - z);
      w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

// Coefficients of the Legendre polynomial P_k(z) = sum_r L[k][r] z^r
// (three-term recurrence (k+1) P_{k+1} = (2k+1) z P_k - k P_{k-1}).
struct LegTable {
  double L[kNMax + 2][kNMax + 2];
  constexpr LegTable() : L{} {
    L[0][0] = 1.0;
    L[1][1] = 1.0;
    for (int k = 1; k <= kNMax; ++k)
      for (int r = 0; r <= k + 1; ++r) {
        double v = 0.0;
        if (r >= 1) v += (2.0 * k + 1.0) * L[k][r - 1];
        v -= k * L[k - 1][r];
        L[k + 1][r] = v / (k + 1.0);
      }
  }
};

// Coefficients of the shifted Legendre polynomial P_k(2t - 1) in powers of
// t: ell[k][r] = (-1)^(k+r) C(k, r) C(k+r, r) (integers, exact in FP64).
struct ShiftedLegTable {
  double ell[kNMax + 1][kNMax + 1];
  constexpr ShiftedLegTable() : ell{} {
    for (int k = 0; k <= kNMax; ++k)
      for (int r = 0; r <= k; ++r) {
        double c1 = 1.0, c2 = 1.0;  // C(k, r), C(k+r, r)
        for (int i = 1; i <= r; ++i) {
          c1 = c1 * (k - r + i) / i;
          c2 = c2 * (k + i) / i;
        }
        ell[k][r] = (((k + r) & 1) ? -1.0 : 1.0) * c1 * c2;
      }
  }
};

// Byte offsets of one image's planes from image 0's: the image, the plane
// the range stage reads as theta (theta, or the image where theta = f), sigma,
// the stack, the output.
struct BatchOffsets {
  long long img, theta, sigma, stack, out;
};

// A batch of images of one shape and one parameter set. Kernels take the
// image index z from the last grid dimension, so a whole batch is one launch
// per stage. Image z is found either at fixed strides -- img + z*img
// (elements; also theta and sigma), the stack at byte offset z*stack, out +
// z*out (elements) -- or, where `tab` is set, at the byte offsets tab[z]
// (device memory, filled before the launch; `host_tab` is the same table in
// host memory for launchers that loop over the images on the host). n = 1
// with zero strides and no table is a single image.
struct Batch {
  int n = 1;
  long long img = 0;
  long long stack = 0;
  long long out = 0;
  const BatchOffsets* tab = nullptr;
  const BatchOffsets* host_tab = nullptr;

  // offsets of image z (out_size: bytes per output element)
  __device__ __forceinline__ BatchOffsets at(long long z, int out_size) const {
    if (tab) return tab[z];
    return BatchOffsets{z * img * 4, z * img * 4, z * img * 4, z * stack, z * out * out_size};
  }
  BatchOffsets at_host(long long z, int out_size) const {
    if (host_tab) return host_tab[z];
    return BatchOffsets{z * img * 4, z * img * 4, z * img * 4, z * stack, z * out * out_size};
  }
};

// Copies n offset records from host memory into `dev` (device, 8-byte
// aligned) in stream order (the records travel as kernel arguments, so the
// host array may be freed when this returns).
hipError_t launch_write_offsets(BatchOffsets* dev, const BatchOffsets* host, int n,
                                hipStream_t stream);

// p[i] for a wave-uniform base p and a per-lane 32-bit byte offset (the
// load then takes the base from scalar registers and the offset from one
// vector register, with no 64-bit address arithmetic per lane).
template <typename T>
__device__ __forceinline__ T at_byte(const T* p, unsigned byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
}

// Raw buffer access for a wave-uniform base address: the resource holds the
// base in scalar registers (stride 0, the largest record count, so nothing
// within 4 GiB of the base is clipped) and each lane supplies a 32-bit byte
// offset, so no lane does 64-bit address arithmetic. Loads and stores go
// through the vector memory path (buffer_load / buffer_store).
typedef __amdgpu_buffer_rsrc_t BufRsrc;
__device__ __forceinline__ BufRsrc buf_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
__device__ __forceinline__ float buf_ld_f32(BufRsrc r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double buf_ld_f64(BufRsrc r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ float4 buf_ld_f32x4(BufRsrc r, unsigned off) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ double buf_ld(BufRsrc r, unsigned off, const float*) {
  return buf_ld_f32(r, off);
}
__device__ __forceinline__ double buf_ld(BufRsrc r, unsigned off, const double*) {
  return buf_ld_f64(r, off);
}
__device__ __forceinline__ void buf_st(BufRsrc r, unsigned off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)off, 0, 0);
}
typedef unsigned int BufU32x2 __attribute__((__vector_size__(8)));
__device__ __forceinline__ void buf_st(BufRsrc r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(BufU32x2, v), r, (int)off, 0, 0);
}

// p[i] = v for a wave-uniform base p and a per-lane 32-bit byte offset.
template <typename T>
__device__ __forceinline__ void st_byte(T* p, unsigned byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + byte_off) = v;
}

template <typename T>
__host__ __device__ __forceinline__ T* byte_offset(T* p, long long bytes) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(const_cast<void*>(static_cast<const void*>(p))) + bytes);
}

// Launchers (all asynchronous on `stream`; return hipGetLastError()).
// alpha/beta of image z are at byte offset z*b.stack (b.stack = 0 for n = 1).
hipError_t launch_minmax(const float* img, long long pitch, int h, int w, int rho,
                         float* alpha, float* beta, long long out_pitch,
                         void* scratch, hipStream_t stream, const Batch& b = Batch());

// Range-stage operands for a moments launch that also finishes the filter
// (theta and sigma share tpitch; out has the stack's element type). With
// keep_stack = 0 the moment planes are not written.
struct FuseSpec {
  const float* theta = nullptr;
  const float* sigma = nullptr;
  long long tpitch = 0;
  void* out = nullptr;
  long long opitch = 0;
  unsigned flags = 0;
  int keep_stack = 0;
};

// prec: 0 = FP64 stack, 1 = FP32 stack. N >= 1. Unless `bounds`, the
// alpha/beta planes of the stack must already hold the window bounds.
// fuse != nullptr also evaluates the range stage per pixel and writes the
// filtered output (only where moments_fusable() holds); the result equals
// launch_range() on the stack. bounds = true (only where
// moments_take_bounds() holds) computes the window bounds in the same
// kernel and writes them to alpha/beta; the stack (and, with fuse, the
// output) is then identical to launch_minmax() followed by launch_moments().
hipError_t launch_moments(const float* img, long long pitch, int h, int w,
                          int kernel_kind, double sigma_s, int rho, int N, int prec,
                          float* alpha, float* beta, long long sp,
                          void* mom, long long plane_elems, hipStream_t stream,
                          const Batch& b = Batch(), const FuseSpec* fuse = nullptr,
                          bool bounds = false);

bool moments_fusable(int kernel_kind, int rho, int N, long long h, long long w);

// Whether abf_fast runs the moment and range stages fused (launch_moments
// with a FuseSpec after launch_minmax) rather than the stack path; prec 1 =
// mixed. The box kernel's segment geometry follows the same choice.
// (Measured faster than the stack path at rho 5 and 20, every N; up to
// rho 32 its strips still hold three full 64-column chunks of outputs.)
constexpr int kFuseRhoMax = 32;
bool fast_fuses(int kernel_kind, int rho, int N, int prec);

// Moment planes for the recursive approximation of the Gaussian (kernel kind
// 2): the alpha/beta planes must hold the window bounds; `scratch` (device,
// 256-byte aligned) >= recursive_scratch_bytes(h, w, N).
hipError_t launch_recursive_moments(const float* img, long long pitch, int h, int w,
                                   double sigma_s, int rho, int N, int prec, const float* alpha,
                                   const float* beta, long long sp, void* mom,
                                   long long plane_elems, void* scratch, hipStream_t stream);
size_t recursive_scratch_bytes(int h, int w, int N);
// Which moment kernel builds the stack (values of abf_stack_kernel); prec 0 =
// FP64 stack, 1 = FP32; -1 if no kernel covers the arguments.
enum { kStackBoundsOnly = 0, kStackBox = 1, kStackTile = 2, kStackTileWide = 3, kStackMfma = 4 };
int stack_kernel_id(int kernel_kind, int rho, int N, int prec, long long h, long long w);
bool moments_take_bounds(int kernel_kind, int rho, int N, long long h, long long w);

hipError_t launch_range(const float* alpha, const float* beta, long long sp,
                        const void* mom, long long plane_elems,
                        const float* theta_or_img, long long tpitch,
                        const float* sigma, long long spitch, int h, int w,
                        int N, int prec, unsigned flags, void* out, long long opitch,
                        hipStream_t stream, const Batch& b = Batch());

// Uniform-prior variant from a stack's bounds and first moment plane.
hipError_t launch_range_uniform(const float* alpha, const float* beta, long long sp,
                                const void* mom1, const float* img, long long ipitch,
                                const float* theta_or_img, long long tpitch, const float* sigma,
                                long long spitch, int h, int w, int prec, unsigned flags,
                                void* out, long long opitch, hipStream_t stream);

// sigma(i) = clamp(scale * std of f over the (2r+1)^2 clamp-to-edge window,
// lo, hi), population standard deviation, FP64.
hipError_t launch_sigma_std(const float* img, long long pitch, int h, int w, int r,
                            double scale, double lo, double hi, float* out, long long opitch,
                            hipStream_t stream, const Batch& b = Batch());

// Application parameter maps (maps.hip). maps_params_ok: window radius r
// and LoG std s within the kernels' halo limit.
bool maps_params_ok(int r, double s);
hipError_t launch_sharpen_maps(const float* img, long long pitch, int h, int w, int r, double s,
                               double lo, double hi, double v_ref, float* theta, float* sigma,
                               long long op, hipStream_t stream, const Batch& b);
hipError_t launch_mrtv_sigma(const float* img, long long pitch, int h, int w, int r, double eps,
                             double lo, double hi, double v_ref, float* sigma, long long op,
                             hipStream_t stream, const Batch& b);
hipError_t launch_grey(const float* rgb, long long pitch, long long cstride, int h, int w,
                       float* out, long long op, hipStream_t stream, const Batch& b);

hipError_t launch_brute(const float* img, const float* theta, const float* sigma,
                        long long pitch, int h, int w, int kernel_kind, double sigma_s,
                        int rho, int prec, void* out, long long opitch,
                        hipStream_t stream);

}  // namespace abf
