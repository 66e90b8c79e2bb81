// Host-only stand-ins for libabf's kernel launchers, for the sanitizer build
// of the C ABI (api.cpp) on a machine without a GPU. Each stub launches
// nothing; it checks that every plane the real kernel would read or write
// (rows of `pitch` elements, h of them, times the batch) lies inside a
// buffer the driver registered, so the ABI's workspace and stack
// arithmetic is checked for overruns, and counts the call.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../paper_1811_02308_amd/csrc/abf_internal.h"
#include "stub_registry.h"

namespace {
struct Span {
  uintptr_t lo, hi;
};
std::vector<Span> g_spans;
int g_bad = 0;
int g_calls = 0;

// [p, p + bytes) must lie inside one registered buffer.
void need(const void* p, unsigned long long bytes, const char* what) {
  if (!p || bytes == 0) return;
  const uintptr_t a = reinterpret_cast<uintptr_t>(p), b = a + bytes;
  for (const Span& s : g_spans)
    if (a >= s.lo && b <= s.hi) return;
  std::fprintf(stderr, "stub: %s [%p, +%llu) is outside every registered buffer\n", what, p, bytes);
  ++g_bad;
}

enum Field { kImg, kTheta, kSigma, kStack, kOut };

// A plane of h rows of `pitch` elements of `elem` bytes (its last row needs
// only w elements), for each of the batch's images at the byte offset the
// batch gives for `field` (its strides, or its host offset table).
void plane(const void* p, long long pitch, int h, int w, size_t elem, const abf::Batch& b,
           Field field, const char* what) {
  if (h < 1 || w < 1) return;
  const unsigned long long bytes = ((unsigned long long)(h - 1) * pitch + w) * elem;
  for (int z = 0; z < b.n; ++z) {
    const abf::BatchOffsets o = b.at_host(z, (int)elem);
    const long long off[] = {o.img, o.theta, o.sigma, o.stack, o.out};
    need(static_cast<const char*>(p) + off[field], bytes, what);
  }
}
}  // namespace

void stub_register(const void* p, size_t bytes) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  g_spans.push_back({a, a + bytes});
}
void stub_clear() { g_spans.clear(); }
int stub_violations() { return g_bad; }
int stub_calls() { return g_calls; }

namespace abf {

hipError_t launch_minmax(const float* img, long long pitch, int h, int w, int rho, float* alpha,
                         float* beta, long long out_pitch, void* scratch, hipStream_t,
                         const Batch& b) {
  ++g_calls;
  plane(img, pitch, h, w, 4, b, kImg, "minmax img");
  plane(alpha, out_pitch, h, w, 4, b, kStack, "minmax alpha");
  plane(beta, out_pitch, h, w, 4, b, kStack, "minmax beta");
  if (rho > 24) need(scratch, (unsigned long long)w * ((h + 63) / 64 * 64) * 8, "minmax scratch");
  return hipSuccess;
}

hipError_t launch_moments(const float* img, long long pitch, int h, int w, int, double, int,
                          int N, int prec, float* alpha, float* beta, long long sp, void* mom,
                          long long plane_elems, hipStream_t, const Batch& b, const FuseSpec* fz,
                          bool) {
  ++g_calls;
  plane(img, pitch, h, w, 4, b, kImg, "moments img");
  plane(alpha, sp, h, w, 4, b, kStack, "moments alpha");
  plane(beta, sp, h, w, 4, b, kStack, "moments beta");
  const size_t e = prec == 0 ? 8 : 4;
  if (!fz || fz->keep_stack)
    for (int k = 0; k < N; ++k)
      plane(static_cast<const char*>(mom) + (size_t)k * plane_elems * e, sp, h, w, e, b, kStack, "moments plane");
  if (fz) {
    plane(fz->theta, fz->tpitch, h, w, 4, b, kTheta, "fused theta");
    plane(fz->sigma, fz->tpitch, h, w, 4, b, kSigma, "fused sigma");
    plane(fz->out, fz->opitch, h, w, e, b, kOut, "fused out");
  }
  return hipSuccess;
}

hipError_t launch_recursive_moments(const float* img, long long pitch, int h, int w, double, int,
                                   int N, int prec, const float* alpha, const float* beta,
                                   long long sp, void* mom, long long plane_elems, void* scratch,
                                   hipStream_t) {
  ++g_calls;
  const size_t e = prec == 0 ? 8 : 4;
  plane(img, pitch, h, w, 4, abf::Batch(), kImg, "recursive img");
  plane(alpha, sp, h, w, 4, abf::Batch(), kImg, "recursive alpha");
  plane(beta, sp, h, w, 4, abf::Batch(), kImg, "recursive beta");
  for (int k = 0; k < N; ++k)
    plane(static_cast<const char*>(mom) + (size_t)k * plane_elems * e, sp, h, w, e, abf::Batch(), kImg,
          "recursive plane");
  need(scratch, recursive_scratch_bytes(h, w, N), "recursive scratch");
  return hipSuccess;
}

size_t recursive_scratch_bytes(int h, int w, int N) {
  return 256 + 1792 + (size_t)2 * N * (size_t)h * (size_t)w * sizeof(double);
}

bool fast_fuses(int kernel_kind, int rho, int N, int prec) {
  return kernel_kind == 0 && prec == 1 && N >= 1 && rho <= kFuseRhoMax;
}

bool moments_fusable(int kernel_kind, int rho, int N, long long, long long) {
  return N >= 1 && N <= 8 && (kernel_kind == 0 || rho <= 40);
}
int stack_kernel_id(int kernel_kind, int, int N, int, long long, long long) {
  return N < 1 ? kStackBoundsOnly : (kernel_kind == 0 ? kStackBox : kStackTile);
}
bool moments_take_bounds(int kernel_kind, int, int N, long long, long long) {
  return kernel_kind == 1 && N >= 1;
}

hipError_t launch_range(const float* alpha, const float* beta, long long sp, const void* mom,
                        long long plane_elems, const float* theta_or_img, long long tpitch,
                        const float* sigma, long long spitch, int h, int w, int N, int prec,
                        unsigned, void* out, long long opitch, hipStream_t, const Batch& b) {
  ++g_calls;
  const size_t e = prec == 0 ? 8 : 4;
  plane(alpha, sp, h, w, 4, b, kStack, "range alpha");
  plane(beta, sp, h, w, 4, b, kStack, "range beta");
  for (int k = 0; k < N; ++k)
    plane(static_cast<const char*>(mom) + (size_t)k * plane_elems * e, sp, h, w, e, b, kStack,
          "range plane");
  plane(theta_or_img, tpitch, h, w, 4, b, kTheta, "range theta");
  plane(sigma, spitch, h, w, 4, b, kSigma, "range sigma");
  plane(out, opitch, h, w, e, b, kOut, "range out");
  return hipSuccess;
}

hipError_t launch_range_uniform(const float* alpha, const float* beta, long long sp,
                                const void* mom1, const float* img, long long ipitch,
                                const float* theta_or_img, long long tpitch, const float* sigma,
                                long long spitch, int h, int w, int prec, unsigned, void* out,
                                long long opitch, hipStream_t) {
  ++g_calls;
  const size_t e = prec == 0 ? 8 : 4;
  plane(alpha, sp, h, w, 4, abf::Batch(), kImg, "uniform alpha");
  plane(beta, sp, h, w, 4, abf::Batch(), kImg, "uniform beta");
  plane(mom1, sp, h, w, e, abf::Batch(), kImg, "uniform plane 1");
  plane(img, ipitch, h, w, 4, abf::Batch(), kImg, "uniform img");
  plane(theta_or_img, tpitch, h, w, 4, abf::Batch(), kImg, "uniform theta");
  plane(sigma, spitch, h, w, 4, abf::Batch(), kImg, "uniform sigma");
  plane(out, opitch, h, w, e, abf::Batch(), kImg, "uniform out");
  return hipSuccess;
}

hipError_t launch_sigma_std(const float* img, long long pitch, int h, int w, int, double, double,
                            double, float* out, long long opitch, hipStream_t, const Batch& b) {
  ++g_calls;
  plane(img, pitch, h, w, 4, b, kImg, "sigma img");
  plane(out, opitch, h, w, 4, b, kOut, "sigma out");
  return hipSuccess;
}

bool maps_params_ok(int r, double s) { return r >= 0 && r <= 32 && s > 0 && s <= 8; }

hipError_t launch_sharpen_maps(const float* img, long long pitch, int h, int w, int, double,
                               double, double, double, float* theta, float* sigma, long long op,
                               hipStream_t, const Batch& b) {
  ++g_calls;
  plane(img, pitch, h, w, 4, b, kImg, "sharpen img");
  plane(theta, op, h, w, 4, b, kOut, "sharpen theta");
  plane(sigma, op, h, w, 4, b, kOut, "sharpen sigma");
  return hipSuccess;
}

hipError_t launch_mrtv_sigma(const float* img, long long pitch, int h, int w, int, double, double,
                             double, double, float* sigma, long long op, hipStream_t,
                             const Batch& b) {
  ++g_calls;
  plane(img, pitch, h, w, 4, b, kImg, "mrtv img");
  plane(sigma, op, h, w, 4, b, kOut, "mrtv sigma");
  return hipSuccess;
}

hipError_t launch_grey(const float* rgb, long long pitch, long long cstride, int h, int w,
                       float* out, long long op, hipStream_t, const Batch& b) {
  ++g_calls;
  for (int c = 0; c < 3; ++c)
    plane(rgb + c * cstride, pitch, h, w, 4, b, kImg, "grey rgb");
  plane(out, op, h, w, 4, b, kOut, "grey out");
  return hipSuccess;
}

hipError_t launch_brute(const float* img, const float* theta, const float* sigma, long long pitch,
                        int h, int w, int, double, int, int prec, void* out, long long opitch,
                        hipStream_t) {
  ++g_calls;
  plane(img, pitch, h, w, 4, abf::Batch(), kImg, "brute img");
  plane(theta, pitch, h, w, 4, abf::Batch(), kImg, "brute theta");
  plane(sigma, pitch, h, w, 4, abf::Batch(), kImg, "brute sigma");
  plane(out, opitch, h, w, prec == 0 ? 8 : 4, abf::Batch(), kImg, "brute out");
  return hipSuccess;
}

hipError_t launch_write_offsets(BatchOffsets* dev, const BatchOffsets* host, int n,
                                hipStream_t) {
  ++g_calls;
  need(dev, (unsigned long long)n * sizeof(BatchOffsets), "offset table");
  for (int i = 0; i < n; ++i) {    // every member's planes must be reachable from its group's first
    const BatchOffsets& o = host[i];
    if ((o.img | o.theta | o.sigma | o.out) % 4 != 0 || o.stack % 256 != 0) {
      std::fprintf(stderr, "stub: offset record %d is misaligned\n", i);
      ++g_bad;
    }
  }
  return hipSuccess;
}

}  // namespace abf
