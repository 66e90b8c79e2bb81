// Offset tables of batched launches (struct Batch with `tab`): the records
// are copied into device memory by a small kernel that receives them as
// kernel arguments, so the copy is ordered on the caller's stream and needs
// neither pinned host memory nor a host buffer that outlives the call.
#include <hip/hip_runtime.h>

#include "abf_internal.h"

namespace abf {
namespace {

constexpr int kChunk = 32;     // records per launch (32 x 40 bytes of kernel arguments)

struct OffsetChunk {
  int n;
  BatchOffsets rec[kChunk];
};

__global__ __launch_bounds__(64) void write_offsets(BatchOffsets* __restrict__ dst, OffsetChunk c) {
  const int i = threadIdx.x;
  if (i < c.n) dst[i] = c.rec[i];
}

}  // namespace

hipError_t launch_write_offsets(BatchOffsets* dev, const BatchOffsets* host, int n,
                                hipStream_t stream) {
  for (int i0 = 0; i0 < n; i0 += kChunk) {
    OffsetChunk c;
    c.n = n - i0 < kChunk ? n - i0 : kChunk;
    for (int i = 0; i < c.n; ++i) c.rec[i] = host[i0 + i];
    hipLaunchKernelGGL(write_offsets, dim3(1), dim3(64), 0, stream, dev + i0, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace abf
