// C ABI of libabf: argument validation, workspace layout and dispatch to the
// HIP kernels (see include/abf.h for the contract of every entry point).
#include "../../include/abf.h"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "abf_internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

bool shape_ok(int h, int w, long long pitch) { return h >= 1 && w >= 1 && pitch >= w; }

abf_status hip_status(hipError_t e) { return e == hipSuccess ? ABF_OK : ABF_E_HIP; }

size_t elem_bytes(int prec) { return prec == ABF_PREC_FP64 ? 8 : 4; }

bool prec_ok(int p) { return p == ABF_PREC_FP64 || p == ABF_PREC_MIXED; }
bool kind_ok(int k) { return k == ABF_KERNEL_BOX || k == ABF_KERNEL_GAUSSIAN; }
// abf_fast and abf_moment_stack also take the recursive kernel
bool stack_kind_ok(int k) { return kind_ok(k) || k == ABF_KERNEL_RECURSIVE; }
// the recursive kernel: mixed path only (see abf.h)
bool rec_supported(int, int precision) { return precision == ABF_PREC_MIXED; }

}  // namespace

extern "C" {

const char* abf_status_string(int s) {
  switch (s) {
    case ABF_OK: return "ok";
    case ABF_E_INVALID: return "invalid argument";
    case ABF_E_NOMEM: return "out of memory";
    case ABF_E_HIP: return "HIP runtime error";
    case ABF_E_UNSUPPORTED: return "unsupported parameter (N or rho out of the built range)";
    case ABF_E_WORKSPACE: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}

int abf_version(void) { return 100; }

long long abf_stack_pitch(int w) { return w < 1 ? 0 : ((long long)w + 63) / 64 * 64; }

size_t abf_stack_plane_offset(int h, int w, int N, int precision, int plane) {
  (void)N;
  const size_t P = (size_t)abf_stack_pitch(w) * (size_t)(h < 0 ? 0 : h);
  if (plane <= 0) return 0;
  if (plane == 1) return P * 4;
  return P * 8 + (size_t)(plane - 2) * P * elem_bytes(precision);
}

size_t abf_stack_bytes(int h, int w, int N, int precision) {
  if (h < 1 || w < 1 || N < 0) return 0;
  return align_up(abf_stack_plane_offset(h, w, N, precision, N + 2));
}

size_t abf_scratch_bytes(int h, int w, int rho) {
  (void)rho;
  if (h < 1 || w < 1) return 0;
  // transposed (min, max) intermediate of the separable window bounds
  return align_up((size_t)w * (size_t)(((long long)h + 63) / 64 * 64) * 8);
}

size_t abf_workspace_bytes(int h, int w, int rho, int N, int precision) {
  if (h < 1 || w < 1 || N < 0) return 0;
  return abf_stack_bytes(h, w, N, precision) + abf_scratch_bytes(h, w, rho);
}

size_t abf_kernel_scratch_bytes(int h, int w, int rho, int N, int kernel_kind) {
  if (h < 1 || w < 1 || N < 0 || rho < 0) return 0;
  const size_t bounds = abf_scratch_bytes(h, w, rho);
  if (kernel_kind != ABF_KERNEL_RECURSIVE || N == 0) return bounds;
  const size_t rec = align_up(abf::recursive_scratch_bytes(h, w, N));
  return rec > bounds ? rec : bounds;
}

size_t abf_kernel_workspace_bytes(int h, int w, int rho, int N, int precision, int kernel_kind) {
  if (h < 1 || w < 1 || N < 0) return 0;
  return abf_stack_bytes(h, w, N, precision) + abf_kernel_scratch_bytes(h, w, rho, N, kernel_kind);
}

// Window bounds and moment planes of one stack or of a strided batch of
// stacks (arguments checked by the caller): one launch where the moment
// kernel takes the bounds as well, else the bounds kernel and then the
// moment kernel; N = 0 writes the bounds only. The stack is the same either
// way.
static hipError_t bounds_and_moments(const float* img, int h, int w, long long pitch,
                                     int kernel_kind, double sigma_s, int rho, int N,
                                     int precision, char* stack, void* scratch, hipStream_t s,
                                     const abf::Batch& b) {
  const long long sp = abf_stack_pitch(w);
  float* alpha = reinterpret_cast<float*>(stack);
  float* beta = reinterpret_cast<float*>(stack + abf_stack_plane_offset(h, w, N, precision, 1));
  void* mom = stack + abf_stack_plane_offset(h, w, N, precision, 2);
  const int pc = precision == ABF_PREC_FP64 ? 0 : 1;
  if (N > 0 && abf::moments_take_bounds(kernel_kind, rho, N, h, w))
    return abf::launch_moments(img, pitch, h, w, kernel_kind, sigma_s, rho, N, pc, alpha, beta,
                               sp, mom, sp * h, s, b, nullptr, true);
  hipError_t e = abf::launch_minmax(img, pitch, h, w, rho, alpha, beta, sp, scratch, s, b);
  if (e != hipSuccess || N == 0) return e;
  if (kernel_kind == ABF_KERNEL_RECURSIVE)   // one image (the caller checks b.n == 1)
    return abf::launch_recursive_moments(img, pitch, h, w, sigma_s, rho, N, pc, alpha, beta, sp,
                                         mom, sp * h, scratch, s);
  return abf::launch_moments(img, pitch, h, w, kernel_kind, sigma_s, rho, N, pc, alpha, beta, sp,
                             mom, sp * h, s, b);
}

// Range stage of one stack or a strided batch of stacks.
static abf_status range_batch(const float* img, const float* theta, const float* sigma, int h,
                              int w, long long pitch, int N, int precision, unsigned flags,
                              const char* stack, void* out, long long out_pitch, hipStream_t s,
                              const abf::Batch& b) {
  const long long sp = abf_stack_pitch(w);
  const float* alpha = reinterpret_cast<const float*>(stack);
  const float* beta =
      reinterpret_cast<const float*>(stack + abf_stack_plane_offset(h, w, N, precision, 1));
  const void* mom = stack + abf_stack_plane_offset(h, w, N, precision, 2);
  return hip_status(abf::launch_range(alpha, beta, sp, mom, sp * h, theta ? theta : img, pitch,
                                      sigma, pitch, h, w, N, precision == ABF_PREC_FP64 ? 0 : 1,
                                      flags & ABF_FLAG_CLAMP, out, out_pitch, s, b));
}

abf_status abf_minmax(const float* img, int h, int w, long long pitch, int rho, float* alpha,
                      float* beta, long long out_pitch, void* workspace, size_t workspace_bytes,
                      void* stream) {
  if (!img || !alpha || !beta || !shape_ok(h, w, pitch) || out_pitch < w || rho < 0)
    return ABF_E_INVALID;
  if (rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (!workspace || !aligned(workspace) || workspace_bytes < abf_scratch_bytes(h, w, rho))
    return ABF_E_WORKSPACE;
  return hip_status(abf::launch_minmax(img, pitch, h, w, rho, alpha, beta, out_pitch, workspace,
                                       static_cast<hipStream_t>(stream)));
}

abf_status abf_stack_moments(const float* img, int h, int w, long long pitch, int kernel_kind,
                             double sigma_s, int rho, int N, int precision, void* stack,
                             size_t stack_bytes, void* stream) {
  if (!img || !stack || !shape_ok(h, w, pitch) || rho < 0 || N < 0 || !prec_ok(precision) ||
      !kind_ok(kernel_kind) || !std::isfinite(sigma_s))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX || rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (!aligned(stack) || stack_bytes < abf_stack_bytes(h, w, N, precision)) return ABF_E_WORKSPACE;
  if (N == 0) return ABF_OK;
  const long long sp = abf_stack_pitch(w);
  char* base = static_cast<char*>(stack);
  float* alpha = reinterpret_cast<float*>(base);
  float* beta = reinterpret_cast<float*>(base + abf_stack_plane_offset(h, w, N, precision, 1));
  void* mom = base + abf_stack_plane_offset(h, w, N, precision, 2);
  return hip_status(abf::launch_moments(img, pitch, h, w, kernel_kind, sigma_s, rho, N,
                                        precision == ABF_PREC_FP64 ? 0 : 1, alpha, beta, sp, mom,
                                        sp * h, static_cast<hipStream_t>(stream)));
}

abf_status abf_moment_stack(const float* img, int h, int w, long long pitch, int kernel_kind,
                            double sigma_s, int rho, int N, int precision, void* stack,
                            size_t stack_bytes, void* workspace, size_t workspace_bytes,
                            void* stream) {
  if (!img || !stack || !shape_ok(h, w, pitch) || rho < 0 || N < 0 || !prec_ok(precision) ||
      !stack_kind_ok(kernel_kind) || !std::isfinite(sigma_s))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX || rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (kernel_kind == ABF_KERNEL_RECURSIVE && !rec_supported(N, precision)) return ABF_E_UNSUPPORTED;
  if (!aligned(stack) || stack_bytes < abf_stack_bytes(h, w, N, precision)) return ABF_E_WORKSPACE;
  if (!workspace || !aligned(workspace) ||
      workspace_bytes < abf_kernel_scratch_bytes(h, w, rho, N, kernel_kind))
    return ABF_E_WORKSPACE;
  return hip_status(bounds_and_moments(img, h, w, pitch, kernel_kind, sigma_s, rho, N, precision,
                                       static_cast<char*>(stack), workspace,
                                       static_cast<hipStream_t>(stream), abf::Batch()));
}

int abf_stack_single_pass(int h, int w, int kernel_kind, int rho, int N) {
  if (h < 1 || w < 1 || rho < 0 || rho > ABF_RHO_MAX || N < 1 || N > ABF_N_MAX ||
      !kind_ok(kernel_kind))
    return 0;
  return abf::moments_take_bounds(kernel_kind, rho, N, h, w) ? 1 : 0;
}

int abf_stack_kernel(int h, int w, int kernel_kind, int rho, int N, int precision) {
  if (h < 1 || w < 1 || rho < 0 || rho > ABF_RHO_MAX || N < 0 || N > ABF_N_MAX ||
      !kind_ok(kernel_kind) || !prec_ok(precision))
    return -1;
  return abf::stack_kernel_id(kernel_kind, rho, N, precision == ABF_PREC_FP64 ? 0 : 1, h, w);
}

abf_status abf_range(const void* stack, size_t stack_bytes, const float* img, const float* theta,
                     const float* sigma, int h, int w, long long pitch, int N, int precision,
                     unsigned flags, void* out, long long out_pitch, void* stream) {
  if (!stack || !sigma || !out || !shape_ok(h, w, pitch) || out_pitch < w || N < 0 ||
      !prec_ok(precision) || (!theta && !img))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX) return ABF_E_UNSUPPORTED;
  if (!aligned(stack) || stack_bytes < abf_stack_bytes(h, w, N, precision)) return ABF_E_WORKSPACE;
  const long long sp = abf_stack_pitch(w);
  const char* base = static_cast<const char*>(stack);
  const float* alpha = reinterpret_cast<const float*>(base);
  const float* beta = reinterpret_cast<const float*>(base + abf_stack_plane_offset(h, w, N, precision, 1));
  const void* mom = base + abf_stack_plane_offset(h, w, N, precision, 2);
  return hip_status(abf::launch_range(alpha, beta, sp, mom, sp * h, theta ? theta : img, pitch,
                                      sigma, pitch, h, w, N, precision == ABF_PREC_FP64 ? 0 : 1,
                                      flags, out, out_pitch, static_cast<hipStream_t>(stream)));
}

// Moments and range stage of one image or a strided batch, alpha/beta
// already in the stack(s). fused: one kernel where the moment kernel
// supports it; otherwise (or fused = false) the stack path: the moment
// kernel writes the stack, then the range kernel reads it.
static abf_status moments_range_batch(const float* img, const float* theta, const float* sigma,
                                      int h, int w, long long pitch, int kernel_kind,
                                      double sigma_s, int rho, int N, int precision,
                                      unsigned flags, char* stack, void* out, long long out_pitch,
                                      hipStream_t s, const abf::Batch& b, bool fused) {
  const long long sp = abf_stack_pitch(w);
  float* alpha = reinterpret_cast<float*>(stack);
  float* beta = reinterpret_cast<float*>(stack + abf_stack_plane_offset(h, w, N, precision, 1));
  void* mom = stack + abf_stack_plane_offset(h, w, N, precision, 2);
  const int pc = precision == ABF_PREC_FP64 ? 0 : 1;
  const float* th = theta ? theta : img;
  const unsigned rflags = flags & ABF_FLAG_CLAMP;
  if (fused && N > 0 && abf::moments_fusable(kernel_kind, rho, N, h, w)) {
    abf::FuseSpec fs;
    fs.theta = th;
    fs.sigma = sigma;
    fs.tpitch = pitch;
    fs.out = out;
    fs.opitch = out_pitch;
    fs.flags = rflags;
    fs.keep_stack = (flags & ABF_FLAG_KEEP_STACK) ? 1 : 0;
    return hip_status(abf::launch_moments(img, pitch, h, w, kernel_kind, sigma_s, rho, N, pc,
                                          alpha, beta, sp, mom, sp * h, s, b, &fs));
  }
  if (N > 0) {
    const hipError_t e = abf::launch_moments(img, pitch, h, w, kernel_kind, sigma_s, rho, N, pc,
                                             alpha, beta, sp, mom, sp * h, s, b);
    if (e != hipSuccess) return ABF_E_HIP;
  }
  return hip_status(abf::launch_range(alpha, beta, sp, mom, sp * h, th, pitch, sigma, pitch, h, w,
                                      N, pc, rflags, out, out_pitch, s, b));
}

abf_status abf_moments_range(const float* img, const float* theta, const float* sigma, int h,
                             int w, long long pitch, int kernel_kind, double sigma_s, int rho,
                             int N, int precision, unsigned flags, void* stack,
                             size_t stack_bytes, void* out, long long out_pitch, void* stream) {
  if (!img || !sigma || !out || !stack || !shape_ok(h, w, pitch) || out_pitch < w || rho < 0 ||
      N < 0 || !prec_ok(precision) || !kind_ok(kernel_kind) || !std::isfinite(sigma_s))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX || rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (!aligned(stack) || stack_bytes < abf_stack_bytes(h, w, N, precision)) return ABF_E_WORKSPACE;
  return moments_range_batch(img, theta, sigma, h, w, pitch, kernel_kind, sigma_s, rho, N,
                             precision, flags, static_cast<char*>(stack), out, out_pitch,
                             static_cast<hipStream_t>(stream), abf::Batch(), true);
}

// Algorithm 1 on one image or a batch (arguments checked by the caller):
// the window bounds, then the moment and range stages fused where
// abf::fast_fuses() holds, else the stack path (moment stack, then range
// stage). `stack` holds the image's (or batch's) stacks, `scratch` the
// bounds scratch.
// The Gaussian tile kernel on the mixed path, where it takes the window
// bounds itself: one kernel for the whole filter (bounds, moments and the
// range stage), its output equal to the stack path's bit for bit.
static bool fast_one_kernel(int kernel_kind, int rho, int N, int precision, int h, int w) {
  return kernel_kind == ABF_KERNEL_GAUSSIAN && precision == ABF_PREC_MIXED && N >= 1 &&
         abf::moments_take_bounds(kernel_kind, rho, N, h, w) &&
         abf::moments_fusable(kernel_kind, rho, N, h, w);
}

static abf_status fast_stages(const float* img, const float* theta, const float* sigma, int h,
                              int w, long long pitch, int kernel_kind, double sigma_s, int rho,
                              int N, int precision, unsigned flags, char* stack, void* scratch,
                              void* out, long long out_pitch, hipStream_t s,
                              const abf::Batch& b) {
  const unsigned rflags = flags & ABF_FLAG_CLAMP;
  if (fast_one_kernel(kernel_kind, rho, N, precision, h, w)) {
    const long long sp = abf_stack_pitch(w);
    float* alpha = reinterpret_cast<float*>(stack);
    float* beta = reinterpret_cast<float*>(stack + abf_stack_plane_offset(h, w, N, precision, 1));
    void* mom = stack + abf_stack_plane_offset(h, w, N, precision, 2);
    abf::FuseSpec fs;
    fs.theta = theta ? theta : img;
    fs.sigma = sigma;
    fs.tpitch = pitch;
    fs.out = out;
    fs.opitch = out_pitch;
    fs.flags = rflags;
    return hip_status(abf::launch_moments(img, pitch, h, w, kernel_kind, sigma_s, rho, N, 1,
                                          alpha, beta, sp, mom, sp * h, s, b, &fs, true));
  }
  if (N > 0 && abf::fast_fuses(kernel_kind, rho, N, precision == ABF_PREC_MIXED ? 1 : 0)) {
    const long long sp = abf_stack_pitch(w);
    float* alpha = reinterpret_cast<float*>(stack);
    float* beta = reinterpret_cast<float*>(stack + abf_stack_plane_offset(h, w, N, precision, 1));
    if (abf::launch_minmax(img, pitch, h, w, rho, alpha, beta, sp, scratch, s, b) != hipSuccess)
      return ABF_E_HIP;
    return moments_range_batch(img, theta, sigma, h, w, pitch, kernel_kind, sigma_s, rho, N,
                               precision, rflags, stack, out, out_pitch, s, b, true);
  }
  const hipError_t e = bounds_and_moments(img, h, w, pitch, kernel_kind, sigma_s, rho, N,
                                          precision, stack, scratch, s, b);
  if (e != hipSuccess) return ABF_E_HIP;
  return range_batch(img, theta, sigma, h, w, pitch, N, precision, rflags, stack, out, out_pitch,
                     s, b);
}

int abf_fast_fused(int h, int w, int kernel_kind, int rho, int N, int precision) {
  if (h < 1 || w < 1 || rho < 0 || rho > ABF_RHO_MAX || N < 1 || N > ABF_N_MAX ||
      !stack_kind_ok(kernel_kind) || !prec_ok(precision))
    return 0;
  return (abf::fast_fuses(kernel_kind, rho, N, precision == ABF_PREC_MIXED ? 1 : 0) ||
          fast_one_kernel(kernel_kind, rho, N, precision, h, w))
             ? 1
             : 0;
}

abf_status abf_fast(const float* img, const float* theta, const float* sigma, int h, int w,
                    long long pitch, int kernel_kind, double sigma_s, int rho, int N,
                    int precision, unsigned flags, void* out, long long out_pitch,
                    void* workspace, size_t workspace_bytes, void* stream) {
  if (!img || !sigma || !out || !shape_ok(h, w, pitch) || out_pitch < w || rho < 0 || N < 0 ||
      !prec_ok(precision) || !stack_kind_ok(kernel_kind) || !std::isfinite(sigma_s))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX || rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (kernel_kind == ABF_KERNEL_RECURSIVE && !rec_supported(N, precision)) return ABF_E_UNSUPPORTED;
  if (!workspace || !aligned(workspace) ||
      workspace_bytes < abf_kernel_workspace_bytes(h, w, rho, N, precision, kernel_kind))
    return ABF_E_WORKSPACE;
  const size_t sb = abf_stack_bytes(h, w, N, precision);
  char* ws = static_cast<char*>(workspace);
  return fast_stages(img, theta, sigma, h, w, pitch, kernel_kind, sigma_s, rho, N, precision,
                     flags, ws, ws + sb, out, out_pitch, static_cast<hipStream_t>(stream),
                     abf::Batch());
}

abf_status abf_range_uniform(const void* stack, size_t stack_bytes, const float* img,
                             const float* theta, const float* sigma, int h, int w, long long pitch,
                             int N, int precision, unsigned flags, void* out, long long out_pitch,
                             void* stream) {
  if (!stack || !img || !sigma || !out || !shape_ok(h, w, pitch) || out_pitch < w || N < 1 ||
      !prec_ok(precision))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX) return ABF_E_UNSUPPORTED;
  if (!aligned(stack) || stack_bytes < abf_stack_bytes(h, w, N, precision)) return ABF_E_WORKSPACE;
  const long long sp = abf_stack_pitch(w);
  const char* base = static_cast<const char*>(stack);
  const float* alpha = reinterpret_cast<const float*>(base);
  const float* beta = reinterpret_cast<const float*>(base + abf_stack_plane_offset(h, w, N, precision, 1));
  const void* mom1 = base + abf_stack_plane_offset(h, w, N, precision, 2);
  return hip_status(abf::launch_range_uniform(
      alpha, beta, sp, mom1, img, pitch, theta ? theta : img, pitch, sigma, pitch, h, w,
      precision == ABF_PREC_FP64 ? 0 : 1, flags & ABF_FLAG_CLAMP, out, out_pitch,
      static_cast<hipStream_t>(stream)));
}

abf_status abf_uniform_prior(const float* img, const float* theta, const float* sigma, int h,
                             int w, long long pitch, int kernel_kind, double sigma_s, int rho,
                             int precision, unsigned flags, void* out, long long out_pitch,
                             void* workspace, size_t workspace_bytes, void* stream) {
  if (!img || !sigma || !out || !shape_ok(h, w, pitch) || out_pitch < w || rho < 0 ||
      !prec_ok(precision) || !kind_ok(kernel_kind) || !std::isfinite(sigma_s))
    return ABF_E_INVALID;
  if (rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (!workspace || !aligned(workspace) ||
      workspace_bytes < abf_workspace_bytes(h, w, rho, 1, precision))
    return ABF_E_WORKSPACE;
  const size_t sb = abf_stack_bytes(h, w, 1, precision);
  char* ws = static_cast<char*>(workspace);
  abf_status st = abf_moment_stack(img, h, w, pitch, kernel_kind, sigma_s, rho, 1, precision, ws,
                                   sb, ws + sb, workspace_bytes - sb, stream);
  if (st != ABF_OK) return st;
  return abf_range_uniform(ws, sb, img, theta, sigma, h, w, pitch, 1, precision, flags, out,
                           out_pitch, stream);
}

abf_status abf_bruteforce(const float* img, const float* theta, const float* sigma, int h, int w,
                          long long pitch, int kernel_kind, double sigma_s, int rho,
                          int precision, void* out, long long out_pitch, void* stream) {
  if (!img || !sigma || !out || !shape_ok(h, w, pitch) || out_pitch < w || rho < 0 ||
      !prec_ok(precision) || !kind_ok(kernel_kind))
    return ABF_E_INVALID;
  if (rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  return hip_status(abf::launch_brute(img, theta, sigma, pitch, h, w, kernel_kind, sigma_s, rho,
                                      precision == ABF_PREC_FP64 ? 0 : 1, out, out_pitch,
                                      static_cast<hipStream_t>(stream)));
}

// Requests that share launches in abf_fast_batched: one shape and pitch,
// one output pitch, one kernel, radius and degree, theta given by all or by
// none (the recursive kernel takes one image per launch).
static bool same_group(const abf_request& a, const abf_request& b) {
  return a.kernel_kind != ABF_KERNEL_RECURSIVE && a.h == b.h && a.w == b.w &&
         a.pitch == b.pitch && a.out_pitch == b.out_pitch && a.kernel_kind == b.kernel_kind &&
         a.rho == b.rho && a.N == b.N &&
         std::memcmp(&a.sigma_s, &b.sigma_s, sizeof(double)) == 0 && !a.theta == !b.theta;
}

static long long byte_diff(const void* a, const void* b) {
  return static_cast<long long>(reinterpret_cast<uintptr_t>(a) - reinterpret_cast<uintptr_t>(b));
}

static size_t request_bytes(const abf_request& r, int precision) {
  return align_up(abf_kernel_workspace_bytes(r.h, r.w, r.rho, r.N, precision, r.kernel_kind));
}

size_t abf_batched_workspace_bytes(const abf_request* reqs, int n, int precision) {
  if (!reqs || n < 0) return 0;
  size_t tot = align_up((size_t)n * sizeof(abf::BatchOffsets));
  for (int i = 0; i < n; ++i) tot += request_bytes(reqs[i], precision);
  return tot;
}

abf_status abf_fast_batched(const abf_request* reqs, int n, int precision, unsigned flags,
                            void* workspace, size_t workspace_bytes, void* stream) {
  if (!reqs || n < 0 || !prec_ok(precision)) return ABF_E_INVALID;
  for (int i = 0; i < n; ++i) {
    const abf_request& r = reqs[i];
    if (!r.img || !r.sigma || !r.out || !shape_ok(r.h, r.w, r.pitch) || r.out_pitch < r.w ||
        r.rho < 0 || r.N < 0 || !stack_kind_ok(r.kernel_kind) || !std::isfinite(r.sigma_s))
      return ABF_E_INVALID;
    if (r.N > ABF_N_MAX || r.rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
    if (r.kernel_kind == ABF_KERNEL_RECURSIVE && !rec_supported(r.N, precision))
      return ABF_E_UNSUPPORTED;
  }
  if (n == 0) return ABF_OK;
  if (!workspace || !aligned(workspace) ||
      workspace_bytes < abf_batched_workspace_bytes(reqs, n, precision))
    return ABF_E_WORKSPACE;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // workspace: the offset table, then one slice per request (its stack,
  // then its scratch)
  char* ws = static_cast<char*>(workspace);
  abf::BatchOffsets* dev_tab = reinterpret_cast<abf::BatchOffsets*>(ws);
  char* slices = ws + align_up((size_t)n * sizeof(abf::BatchOffsets));
  std::vector<size_t> slice(n);
  for (size_t i = 0, off = 0; i < (size_t)n; off += request_bytes(reqs[i], precision), ++i)
    slice[i] = off;
  // groups in order of first appearance (at most 65535 images per launch)
  std::vector<std::vector<int>> groups;
  for (int i = 0; i < n; ++i) {
    size_t g = 0;
    while (g < groups.size() &&
           !(groups[g].size() < 65535 && same_group(reqs[groups[g][0]], reqs[i])))
      ++g;
    if (g == groups.size()) groups.emplace_back();
    groups[g].push_back(i);
  }
  // offsets of every member from its group's first, group after group
  std::vector<abf::BatchOffsets> host(n);
  std::vector<int> first(groups.size());
  bool shared = false;
  for (size_t g = 0, pos = 0; g < groups.size(); ++g) {
    first[g] = (int)pos;
    shared = shared || groups[g].size() > 1;
    const abf_request& r0 = reqs[groups[g][0]];
    const void* th0 = r0.theta ? static_cast<const void*>(r0.theta) : r0.img;
    for (int j : groups[g]) {
      const abf_request& r = reqs[j];
      const void* th = r.theta ? static_cast<const void*>(r.theta) : r.img;
      host[pos++] = abf::BatchOffsets{byte_diff(r.img, r0.img), byte_diff(th, th0),
                                      byte_diff(r.sigma, r0.sigma),
                                      (long long)(slice[j] - slice[groups[g][0]]),
                                      byte_diff(r.out, r0.out)};
    }
  }
  if (shared && abf::launch_write_offsets(dev_tab, host.data(), n, s) != hipSuccess)
    return ABF_E_HIP;
  for (size_t g = 0; g < groups.size(); ++g) {
    const int i0 = groups[g][0];
    const abf_request& r = reqs[i0];
    char* base = slices + slice[i0];
    if (groups[g].size() == 1) {
      const abf_status st = abf_fast(r.img, r.theta, r.sigma, r.h, r.w, r.pitch, r.kernel_kind,
                                     r.sigma_s, r.rho, r.N, precision, flags, r.out, r.out_pitch,
                                     base, request_bytes(r, precision), stream);
      if (st != ABF_OK) return st;
      continue;
    }
    abf::Batch b;
    b.n = (int)groups[g].size();
    b.tab = dev_tab + first[g];
    b.host_tab = host.data() + first[g];
    const abf_status st = fast_stages(r.img, r.theta, r.sigma, r.h, r.w, r.pitch, r.kernel_kind,
                                      r.sigma_s, r.rho, r.N, precision, flags, base,
                                      base + abf_stack_bytes(r.h, r.w, r.N, precision), r.out,
                                      r.out_pitch, s, b);
    if (st != ABF_OK) return st;
  }
  return ABF_OK;
}

size_t abf_strided_workspace_bytes(int n, int h, int w, int rho, int N, int precision) {
  if (n < 1 || h < 1 || w < 1 || N < 0) return 0;
  return (size_t)n * abf_stack_bytes(h, w, N, precision) + abf_scratch_bytes(h, w, rho);
}

abf_status abf_fast_strided(const float* img, const float* theta, const float* sigma, int n,
                            int h, int w, long long pitch, long long image_stride,
                            int kernel_kind, double sigma_s, int rho, int N, int precision,
                            unsigned flags, void* out, long long out_pitch,
                            long long out_image_stride, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!img || !sigma || !out || !shape_ok(h, w, pitch) || out_pitch < w || rho < 0 || N < 0 ||
      !prec_ok(precision) || !kind_ok(kernel_kind) || n < 1 || n > 65535 ||
      (n > 1 && (image_stride < pitch * (long long)(h - 1) + w ||
                 out_image_stride < out_pitch * (long long)(h - 1) + w)) ||
      !std::isfinite(sigma_s))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX || rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  if (!workspace || !aligned(workspace) ||
      workspace_bytes < abf_strided_workspace_bytes(n, h, w, rho, N, precision))
    return ABF_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t sb = abf_stack_bytes(h, w, N, precision);
  const long long sp = abf_stack_pitch(w);
  char* base = static_cast<char*>(workspace);
  void* scratch = base + (size_t)n * sb;
  abf::Batch b;
  b.n = n;
  b.img = n > 1 ? image_stride : 0;
  b.stack = n > 1 ? (long long)sb : 0;
  b.out = n > 1 ? out_image_stride : 0;
  return fast_stages(img, theta, sigma, h, w, pitch, kernel_kind, sigma_s, rho, N, precision,
                     flags, base, scratch, out, out_pitch, s, b);
}

// shared checks of the strided map entry points
static bool strided_ok(const float* img, const void* out, int n, int h, int w, long long pitch,
                       long long image_stride, long long out_pitch, long long out_image_stride) {
  return img && out && shape_ok(h, w, pitch) && out_pitch >= w && n >= 1 && n <= 65535 &&
         (n == 1 || (image_stride >= pitch * (long long)(h - 1) + w &&
                     out_image_stride >= out_pitch * (long long)(h - 1) + w));
}

static abf::Batch map_batch(int n, long long image_stride, long long out_image_stride) {
  abf::Batch b;
  b.n = n;
  b.img = n > 1 ? image_stride : 0;
  b.out = n > 1 ? out_image_stride : 0;
  return b;
}

static bool affine_ok(double lo, double hi, double v_ref) {
  return std::isfinite(lo) && std::isfinite(hi) && lo <= hi && v_ref > 0.0 && std::isfinite(v_ref);
}

abf_status abf_sharpen_maps(const float* img, int n, int h, int w, long long pitch,
                            long long image_stride, int radius, double log_sigma, double lo,
                            double hi, double v_ref, float* theta, float* sigma,
                            long long out_pitch, long long out_image_stride, void* stream) {
  if (!sigma || !strided_ok(img, theta, n, h, w, pitch, image_stride, out_pitch, out_image_stride) ||
      radius < 0 || !(log_sigma > 0.0) || !affine_ok(lo, hi, v_ref))
    return ABF_E_INVALID;
  if (!abf::maps_params_ok(radius, log_sigma)) return ABF_E_UNSUPPORTED;
  return hip_status(abf::launch_sharpen_maps(img, pitch, h, w, radius, log_sigma, lo, hi, v_ref,
                                             theta, sigma, out_pitch,
                                             static_cast<hipStream_t>(stream),
                                             map_batch(n, image_stride, out_image_stride)));
}

abf_status abf_mrtv_sigma(const float* img, int n, int h, int w, long long pitch,
                          long long image_stride, int radius, double eps, double lo, double hi,
                          double v_ref, float* sigma, long long out_pitch,
                          long long out_image_stride, void* stream) {
  if (!strided_ok(img, sigma, n, h, w, pitch, image_stride, out_pitch, out_image_stride) ||
      radius < 0 || !(eps > 0.0) || !affine_ok(lo, hi, v_ref))
    return ABF_E_INVALID;
  if (!abf::maps_params_ok(radius + 1, 1.0)) return ABF_E_UNSUPPORTED;
  return hip_status(abf::launch_mrtv_sigma(img, pitch, h, w, radius, eps, lo, hi, v_ref, sigma,
                                           out_pitch, static_cast<hipStream_t>(stream),
                                           map_batch(n, image_stride, out_image_stride)));
}

abf_status abf_grey(const float* rgb, int n, int h, int w, long long pitch,
                    long long channel_stride, long long image_stride, float* out,
                    long long out_pitch, long long out_image_stride, void* stream) {
  if (!strided_ok(rgb, out, n, h, w, pitch, image_stride, out_pitch, out_image_stride) ||
      channel_stride < pitch * (long long)(h - 1) + w ||
      (n > 1 && image_stride < 2 * channel_stride + pitch * (long long)(h - 1) + w))
    return ABF_E_INVALID;
  return hip_status(abf::launch_grey(rgb, pitch, channel_stride, h, w, out, out_pitch,
                                     static_cast<hipStream_t>(stream),
                                     map_batch(n, image_stride, out_image_stride)));
}

abf_status abf_sigma_local_std(const float* img, int n, int h, int w, long long pitch,
                               long long image_stride, int radius, double scale, double lo,
                               double hi, float* out, long long out_pitch,
                               long long out_image_stride, void* stream) {
  if (!img || !out || !shape_ok(h, w, pitch) || out_pitch < w || radius < 0 || n < 1 ||
      n > 65535 || !(lo <= hi) || !std::isfinite(scale) ||
      (n > 1 && (image_stride < pitch * (long long)(h - 1) + w ||
                 out_image_stride < out_pitch * (long long)(h - 1) + w)))
    return ABF_E_INVALID;
  if (radius > 32) return ABF_E_UNSUPPORTED;
  abf::Batch b;
  b.n = n;
  b.img = n > 1 ? image_stride : 0;
  b.out = n > 1 ? out_image_stride : 0;
  return hip_status(abf::launch_sigma_std(img, pitch, h, w, radius, scale, lo, hi, out, out_pitch,
                                          static_cast<hipStream_t>(stream), b));
}

}  // extern "C"
