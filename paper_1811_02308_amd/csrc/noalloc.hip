// abf_fast_noalloc: abf_fast with its workspace (the moment stack and the
// window-bounds scratch) in a fixed device array of this library instead of
// caller memory, for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` is a file-scope __device__ object: every GPU the
// library runs on holds its own copy, at its own address, until the process
// ends. In host code the name `scratch` is only a host-side stand-in, so
// host code never passes it to a kernel: on the first call on a device (that
// device current) its device address is taken with hipGetSymbolAddress and
// kept per device, and only that address is used. Nothing here allocates.
// Calls on one GPU share its array and keep the last call's contents (every
// byte the filter reads there is written first in the same call, so nothing
// is cleared); calls that overlap on one GPU, on any streams, race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abf.h"

namespace {

__device__ __align__(256) unsigned char scratch[ABF_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's `scratch`, looked up once per
// device; nullptr if the lookup fails.
void* device_scratch(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

}  // namespace

extern "C" abf_status abf_fast_noalloc(const float* img, const float* theta, const float* sigma,
                                       int h, int w, long long pitch, int kernel_kind,
                                       double sigma_s, int rho, int N, int precision,
                                       unsigned flags, void* out, long long out_pitch,
                                       void* stream) {
  // the arguments abf_fast checks, except the workspace, before any HIP call
  if (!img || !sigma || !out || h < 1 || w < 1 || pitch < w || out_pitch < w || rho < 0 ||
      N < 0 || (precision != ABF_PREC_FP64 && precision != ABF_PREC_MIXED) ||
      (kernel_kind != ABF_KERNEL_BOX && kernel_kind != ABF_KERNEL_GAUSSIAN))
    return ABF_E_INVALID;
  if (N > ABF_N_MAX || rho > ABF_RHO_MAX) return ABF_E_UNSUPPORTED;
  const size_t need = abf_workspace_bytes(h, w, rho, N, precision);
  if (need == 0 || need > (size_t)ABF_NOALLOC_BYTES) return ABF_E_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return ABF_E_HIP;
  void* ws = device_scratch(dev);
  if (!ws) return ABF_E_HIP;
  return abf_fast(img, theta, sigma, h, w, pitch, kernel_kind, sigma_s, rho, N, precision, flags,
                  out, out_pitch, ws, (size_t)ABF_NOALLOC_BYTES, stream);
}
