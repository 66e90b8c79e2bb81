// Window bounds alpha_i, beta_i (eq. bounds; Prop. 1; first step of Algorithm 1).
//
// The min (max) over the (2R+1)^2 clamp-to-edge window is separable: a
// 1-D sliding min along rows followed by a 1-D sliding min along columns.
// Each 1-D pass uses the van Herk / Gil-Werman scheme, O(1) comparisons per
// pixel for any R: split the padded row into blocks of w = 2R+1; the
// window [x, x+2R] is the tail of one block plus the head of the next, so
//     min = min(suffix_min(x), prefix_min(x + 2R)).
//
// For R <= 24 a single tiled kernel does both passes in LDS (below). For
// larger R, one kernel does a row pass and writes its result TRANSPOSED, so the
// column pass is the same row kernel run on the transposed intermediate
// (both passes read and write rows, coalesced). A workgroup stages
// ROWS padded rows in LDS; phase 1 writes the block suffixes into the
// result tile, phase 2 folds in the block prefixes, phase 3 writes the
// tile transposed. min and max are carried together as a float2.
#include "abf_internal.h"

namespace abf {
namespace {

constexpr int kTX = 64;        // output columns per workgroup
constexpr int kThreads = 256;

template <bool FIRST>
__global__ __launch_bounds__(kThreads) void vh_rows(
    const void* __restrict__ in, long long in_pitch, int rows, int cols, int R, int ROWS,
    float2* __restrict__ out_t, long long out_pitch,   // FIRST: transposed float2
    float* __restrict__ out_a, float* __restrict__ out_b, long long ab_pitch) {
  const FinMinMax fm;
  extern __shared__ float2 smem[];
  const int E = kTX + 2 * R;
  float2* ext = smem;                 // ROWS x E
  float2* res = smem + ROWS * E;      // ROWS x kTX
  const int row0 = blockIdx.y * ROWS;
  const int col0 = blockIdx.x * kTX;

  for (int i = threadIdx.x; i < ROWS * E; i += kThreads) {
    const int r = i / E, e = i - r * E;
    const int gr = min(row0 + r, rows - 1);
    const int gc = min(max(col0 - R + e, 0), cols - 1);
    float2 v;
    if (FIRST) {
      const float f = static_cast<const float*>(in)[(long long)gr * in_pitch + gc] + 0.0f;
      v = make_float2(f, f);
    } else {
      v = static_cast<const float2*>(in)[(long long)gr * in_pitch + gc];
    }
    ext[i] = v;
  }
  __syncthreads();

  const int w = 2 * R + 1;
  const int nb = (E + w - 1) / w;
  // phase 1: block suffixes, needed at e in [0, kTX)
  const int nb1 = min(nb, (kTX + w - 1) / w);
  for (int it = threadIdx.x; it < ROWS * nb1; it += kThreads) {
    const int r = it % ROWS, b = it / ROWS;
    const int s = b * w, e_end = min(s + w, E);
    float mn = INFINITY, mx = -INFINITY;
    const float2* er = ext + r * E;
    for (int e = e_end - 1; e >= s; --e) {
      const float2 v = er[e];
      mn = fm.min(mn, v.x);
      mx = fm.max(mx, v.y);
      if (e < kTX) res[r * kTX + e] = make_float2(mn, mx);
    }
  }
  __syncthreads();
  // phase 2: block prefixes, needed at e in [2R, 2R + kTX)
  const int b0 = (2 * R) / w;
  const int nb2 = nb - b0;
  for (int it = threadIdx.x; it < ROWS * nb2; it += kThreads) {
    const int r = it % ROWS, b = b0 + it / ROWS;
    const int s = b * w, e_end = min(s + w, E);
    float mn = INFINITY, mx = -INFINITY;
    const float2* er = ext + r * E;
    for (int e = s; e < e_end; ++e) {
      const float2 v = er[e];
      mn = fm.min(mn, v.x);
      mx = fm.max(mx, v.y);
      if (e >= 2 * R) {
        float2* o = res + r * kTX + (e - 2 * R);
        const float2 p = *o;
        *o = make_float2(fm.min(p.x, mn), fm.max(p.y, mx));
      }
    }
  }
  __syncthreads();
  // phase 3: transposed store; consecutive threads take consecutive rows so
  // each output row (an input column) is written contiguously.
  for (int i = threadIdx.x; i < ROWS * kTX; i += kThreads) {
    const int r = i % ROWS, x = i / ROWS;
    const int gr = row0 + r, gc = col0 + x;
    if (gr < rows && gc < cols) {
      const float2 v = res[r * kTX + x];
      if (FIRST) {
        out_t[(long long)gc * out_pitch + gr] = v;
      } else {
        out_a[(long long)gc * ab_pitch + gr] = v.x;
        out_b[(long long)gc * ab_pitch + gr] = v.y;
      }
    }
  }
}

// Single-pass tiled variant for R <= kTileRMax: a workgroup loads the
// (kMTY + 2R) x (kMTX + 2R) padded tile of f into LDS once, then
//   horizontal: a thread takes 8 adjacent outputs of one padded row. The
//     8 windows [v, v+2R] (v = 0..7) share the core [7, 2R], so the thread
//     takes the core's min/max once, a suffix over [v, 6] and a prefix over
//     [2R+1, 2R+v]: about (2R + 30) comparisons per 8 outputs.
//   vertical: the same on columns of the horizontal result, 8 output rows
//     per thread, written straight to alpha/beta.
// No intermediate leaves the workgroup; f is read once (+ halo from L2).
// Output tile MTX x MTY: 64 x 32, or 32 x 32 where the wider tile's LDS
// would exceed kTileLdsSmall (rho >= 8): a bounds kernel of that size
// still fits on a CU beside the fused box kernel's eight waves (17 KiB of
// LDS each), so the two images in flight overlap it instead of queueing it.
constexpr int kTileRMax = 24;
constexpr size_t kTileLdsSmall = 24 * 1024;
// horizontal items per thread: (MTY + 2 kTileRMax) MTX / 8 <= kHItems kThreads
constexpr int kHItems = 3;
static_assert((32 + 2 * kTileRMax) * (64 / 8) <= kHItems * kThreads, "horizontal items per thread");
template <int MTX>
__host__ __device__ constexpr int tile_hs() { return MTX + 1; }
template <int MTX, int MTY>
size_t tile_lds_bytes(int R) {
  const int EX = MTX + 2 * R, EY = MTY + 2 * R, XS = EX | 1;
  const size_t tile_b = (size_t)EY * XS * sizeof(float);
  const size_t hres_b = (size_t)EY * tile_hs<MTX>() * sizeof(float2);
  return tile_b > hres_b ? tile_b : hres_b;
}

template <typename Get>
__device__ __forceinline__ void slide8(Get get, int R, float (&mn)[8], float (&mx)[8],
                                       const FinMinMax& fm) {
  // windows [v, v + 2R] of the sequence get(0 .. 7 + 2R). For 2R >= 6 each
  // window is [v, 6] + [7, 2R] (the shared core, empty at 2R = 6) +
  // [2R + 1, 2R + v]; smaller windows are taken directly.
  if (2 * R < 6) {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      float lo = INFINITY, hi = -INFINITY;
      for (int i = 0; i <= 2 * R; ++i) {
        const float2 q = get(v + i);
        lo = fm.min(lo, q.x);
        hi = fm.max(hi, q.y);
      }
      mn[v] = lo;
      mx[v] = hi;
    }
    return;
  }
  float clo = INFINITY, chi = -INFINITY;
  for (int i = 7; i <= 2 * R; ++i) {
    const float2 q = get(i);
    clo = fm.min(clo, q.x);
    chi = fm.max(chi, q.y);
  }
  // suffixes over [v, 6], v = 6 .. 0
  float slo = clo, shi = chi;
#pragma unroll
  for (int v = 6; v >= 0; --v) {
    const float2 q = get(v);
    slo = fm.min(slo, q.x);
    shi = fm.max(shi, q.y);
    mn[v] = slo;
    mx[v] = shi;
  }
  mn[7] = clo;
  mx[7] = chi;
  // prefixes over [2R+1, 2R+v], v = 1 .. 7
  float plo = INFINITY, phi = -INFINITY;
#pragma unroll
  for (int v = 1; v < 8; ++v) {
    const float2 q = get(2 * R + v);
    plo = fm.min(plo, q.x);
    phi = fm.max(phi, q.y);
    mn[v] = fm.min(mn[v], plo);
    mx[v] = fm.max(mx[v], phi);
  }
}

template <int kMTX, int kMTY>
__global__ __launch_bounds__(kThreads) void minmax_tile(
    const float* __restrict__ img, long long pitch, int H, int W, int R,
    float* __restrict__ out_a, float* __restrict__ out_b, long long op, Batch bt) {
  const FinMinMax fm;
  extern __shared__ float lds[];
  {
    const BatchOffsets o = bt.at(blockIdx.z, 4);
    img = byte_offset(img, o.img);
    out_a = byte_offset(out_a, o.stack);
    out_b = byte_offset(out_b, o.stack);
  }
  // LDS row strides: odd for the padded tile and kMTX + 1 for the
  // horizontal result, so that threads walking different rows hit
  // different banks. The horizontal result takes the tile's place once the
  // tile has been read (it is held in registers across a barrier), so the
  // LDS footprint is the larger of the two, not their sum.
  constexpr int kHS = tile_hs<kMTX>();
  const int EX = kMTX + 2 * R, EY = kMTY + 2 * R;
  const int XS = EX | 1;
  float* tile = lds;                                       // EY x XS
  float2* hres = reinterpret_cast<float2*>(lds);           // EY x kHS, after the tile
  const int x0 = blockIdx.x * kMTX, y0 = blockIdx.y * kMTY;
  for (int i = threadIdx.x; i < EY * EX; i += kThreads) {
    const int r = i / EX, c = i - r * EX;
    const int gy = min(max(y0 - R + r, 0), H - 1);
    const int gx = min(max(x0 - R + c, 0), W - 1);
    tile[r * XS + c] = img[(long long)gy * pitch + gx] + 0.0f;
  }
  __syncthreads();
  // horizontal: item = (padded row, group of 8 outputs); rows vary fastest;
  // EY * kMTX / 8 <= kHItems * kThreads items
  const int n_items = EY * (kMTX / 8);
  float hmn[kHItems][8], hmx[kHItems][8];
#pragma unroll
  for (int q = 0; q < kHItems; ++q) {
    const int it = threadIdx.x + q * kThreads;
    if (it < n_items) {
      const int r = it % EY, g = it / EY;
      const float* row = tile + r * XS + 8 * g;
      slide8([&](int i) { const float v = row[i]; return make_float2(v, v); }, R, hmn[q], hmx[q], fm);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kHItems; ++q) {
    const int it = threadIdx.x + q * kThreads;
    if (it < n_items) {
      const int r = it % EY, g = it / EY;
#pragma unroll
      for (int v = 0; v < 8; ++v) hres[r * kHS + 8 * g + v] = make_float2(hmn[q][v], hmx[q][v]);
    }
  }
  __syncthreads();
  // vertical: item = (output column, group of 8 output rows); columns fastest
  for (int it = threadIdx.x; it < kMTX * (kMTY / 8); it += kThreads) {
    const int c = it % kMTX, g = it / kMTX;
    const float2* col = hres + (8 * g) * kHS + c;
    float mn[8], mx[8];
    slide8([&](int i) { return col[i * kHS]; }, R, mn, mx, fm);
    const int x = x0 + c;
    if (x < W) {
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int y = y0 + 8 * g + v;
        if (y < H) {
          out_a[(long long)y * op + x] = mn[v];
          out_b[(long long)y * op + x] = mx[v];
        }
      }
    }
  }
}

int rows_per_block(int R) {
  // keep the LDS footprint ROWS * (2*kTX + 2R) * 8 bytes within 64 KiB
  int rows = 64;
  while (rows > 1 && (size_t)rows * (2 * kTX + 2 * R) * 8 > 65536) rows >>= 1;
  return rows;
}

}  // namespace

hipError_t launch_minmax(const float* img, long long pitch, int h, int w, int rho,
                         float* alpha, float* beta, long long out_pitch,
                         void* scratch, hipStream_t stream, const Batch& b) {
  if (rho <= kTileRMax) {
    // clamping of the padded tile makes any radius exact; use rho itself.
    // The padded tile, then the horizontal result in the same bytes.
    const size_t lds_wide = tile_lds_bytes<64, 32>(rho);
    if (lds_wide <= kTileLdsSmall) {
      dim3 grid((w + 63) / 64, (h + 31) / 32, b.n);
      hipLaunchKernelGGL((minmax_tile<64, 32>), grid, dim3(kThreads), lds_wide, stream, img, pitch,
                         h, w, rho, alpha, beta, out_pitch, b);
    } else {
      dim3 grid((w + 31) / 32, (h + 31) / 32, b.n);
      const size_t lds_small = tile_lds_bytes<32, 32>(rho);
      hipLaunchKernelGGL((minmax_tile<32, 32>), grid, dim3(kThreads), lds_small, stream, img, pitch,
                         h, w, rho, alpha, beta, out_pitch, b);
    }
    return hipGetLastError();
  }
  // The window clipped to the image is the same for any radius >= dim - 1.
  const int Rh = rho < w - 1 ? rho : w - 1;
  const int Rv = rho < h - 1 ? rho : h - 1;
  const long long tp = ((long long)h + 63) / 64 * 64;   // pitch of transposed rows
  float2* t = static_cast<float2*>(scratch);
  for (int z = 0; z < b.n; ++z) {    // large radii: one image at a time through the scratch
    const BatchOffsets o = b.at_host(z, 4);
    const float* im = byte_offset(img, o.img);
    float* az = byte_offset(alpha, o.stack);
    float* bz = byte_offset(beta, o.stack);
    {
      const int ROWS = rows_per_block(Rh);
      dim3 grid((w + kTX - 1) / kTX, (h + ROWS - 1) / ROWS);
      size_t lds = (size_t)ROWS * (2 * kTX + 2 * Rh) * sizeof(float2);
      hipLaunchKernelGGL(vh_rows<true>, grid, dim3(kThreads), lds, stream,
                         im, pitch, h, w, Rh, ROWS, t, tp, nullptr, nullptr, 0LL);
    }
    {
      const int ROWS = rows_per_block(Rv);
      dim3 grid((h + kTX - 1) / kTX, (w + ROWS - 1) / ROWS);
      size_t lds = (size_t)ROWS * (2 * kTX + 2 * Rv) * sizeof(float2);
      hipLaunchKernelGGL(vh_rows<false>, grid, dim3(kThreads), lds, stream,
                         (const void*)t, tp, w, h, Rv, ROWS, nullptr, 0LL, az, bz, out_pitch);
    }
  }
  return hipGetLastError();
}

}  // namespace abf
