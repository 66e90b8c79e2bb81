// Moment stack: the moment steps of Algorithm 1 (Props. 2 and 3), fused with the
// change of basis to shifted-Legendre moments.
//
// For every pixel i the kernels form the window moments of the power images
// (Prop. 2: sum_t t^k h_i(t) = (omega * f^k)(i)) and turn them into the
// moments of the histogram stretched to [alpha_i, beta_i] (Prop. 3), kept as
// a~_k = sum_j omega_j P_k(z_j), z_j = (f(i-j) - mid_i) / half_i in [-1, 1],
// mid_i = (alpha_i + beta_i)/2, half_i = (beta_i - alpha_i)/2. This equals
// sum_r ell_kr mu_r for the mu_r of eq. (hist_moments_new).
//
// Numerics. Power sums are FP64 and taken about a local origin c instead
// of 0 (box and matrix-core kernels: the mid-range of the window bounds
// sampled over the wave's region; tile kernel: the tile's central input
// value), which shrinks the binomial shift's cancellation: its error grows
// like rho^k, rho = (|mid_i - c| + half_i) / half_i, times the rounding of
// the sums. A pixel whose rho^N exceeds a limit set by the stack's precision
// and the degree (nearly flat windows far from c) is finished about another
// origin (the tile kernel's later passes, FP64 at N >= 7) or recomputed
// directly from its window, so the stack is accurate for every input.
//
// Work decomposition (box kernel). One wave owns a strip of 256 padded
// columns (4 consecutive columns per lane) and a segment of TH output rows.
// It slides a vertical running sum down the segment (add the entering row,
// subtract the leaving row: O(1) per pixel in R), then forms the
// horizontal window sums from a wave-wide inclusive prefix of the vertical
// sums held in LDS: sum over [x-R, x+R] = P(x+R) - P(x-R-1). Outputs are
// the 256 - R - Rpad columns whose window lies inside the strip; strips
// overlap by the halo. The per-pixel epilogue (shift, scale, Legendre)
// reads the prefix from LDS with lanes mapped to consecutive output
// columns, so alpha/beta loads and moment stores are coalesced.
//
// Gaussian kernel: a 2-D tile with register-blocked separable weighted sums
// (O(R) per pixel), at least 64 output columns wide for every radius up to
// ABF_RHO_MAX. With unit weights it also serves the FP64 box path at
// N >= 7, where the box kernel's running sums are not accurate enough.
#include <algorithm>
#include <cmath>
#include <complex>

#include "abf_internal.h"
#include "moments_common.h"
#include "range_eval.h"

namespace abf {
namespace {

constexpr int kV = 4;                    // columns per lane
constexpr int kStrip = kWave * kV;       // padded columns per wave
constexpr int kWaves = 4;                // waves per workgroup
// LDS layout of a strip row in the box kernel: padded column e = 4 l + v
// (lane l, its v-th column) sits at v * kSlotStride + l. The prefix writes
// (fixed v, consecutive lanes) are contiguous, and the epilogue's reads of
// consecutive columns step through the four v-rows, whose offset of 68
// doubles puts 16 consecutive columns in 16 different bank pairs.
constexpr int kSlotStride = kWave + 4;
constexpr int kStripSlots = kV * kSlotStride;
__device__ __forceinline__ int pidx(int e) { return (e & (kV - 1)) * kSlotStride + (e >> 2); }


// v + (value of v `ctrl` DPP positions away), 0 where the source lane is
// outside its row (row shifts: the lane reads 0 by the bound control, so no
// register has to be cleared first).
template <int CTRL>
__device__ __forceinline__ double dpp_shr_add(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(bits & 0xffffffffLL), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(bits >> 32), CTRL, 0xf, 0xf, true);
  const long long tb = ((long long)hi << 32) | (long long)(unsigned)lo;
  return v + __longlong_as_double(tb);
}

// The same for the row broadcasts, where the rows that row_mask leaves out
// keep the cleared value 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(bits & 0xffffffffLL), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROW_MASK, 0xf, false);
  const long long tb = ((long long)hi << 32) | (long long)(unsigned)lo;
  return v + __longlong_as_double(tb);
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP lane moves:
// row_shr 1, 2, 4, 8 scan each row of 16 lanes, then row_bcast 15 and 31
// carry row totals into the rows above.
__device__ __forceinline__ double wave_inclusive_scan(double v, int lane) {
  (void)lane;
  v = dpp_shr_add<0x111>(v);    // row_shr:1
  v = dpp_shr_add<0x112>(v);    // row_shr:2
  v = dpp_shr_add<0x114>(v);    // row_shr:4
  v = dpp_shr_add<0x118>(v);    // row_shr:8
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 -> rows 1, 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 -> rows 2, 3
  return v;
}

// Window bounds of one output row of a strip, lane `lane` holding output
// columns j0 + lane for the kChunks chunks j0 = 0, 64, ...: issued early so
// the loads overlap the row's other work.
constexpr int kChunks = kStrip / kWave;
static_assert(kChunks == 4, "the box epilogue selects among four bound registers");
__device__ __forceinline__ void load_bounds_row(const float* __restrict__ alpha,
                                                const float* __restrict__ beta, long long sp,
                                                int y, int xo, int O, int W, int lane,
                                                float (&pa)[kChunks], float (&pb)[kChunks]) {
  const BufRsrc ar = buf_rsrc(alpha + (long long)y * sp);
  const BufRsrc br = buf_rsrc(beta + (long long)y * sp);
#pragma unroll
  for (int q = 0; q < kChunks; ++q) {
    const unsigned x4 = (unsigned)min(xo + min(q * kWave + lane, O - 1), W - 1) * 4u;
    pa[q] = buf_ld_f32(ar, x4);
    pb[q] = buf_ld_f32(br, x4);
  }
}

// Origin of a wave's power sums: the mid-range of the window bounds sampled
// on an 8 x 8 grid over the wave's output tile.
__device__ __forceinline__ double wave_origin(const float* __restrict__ alpha,
                                              const float* __restrict__ beta, long long sp,
                                              int y0, int y1, int xo, int O, int W, int lane) {
  const int gy = lane >> 3, gx = lane & 7;
  const int yy = min(y0 + (gy * (y1 - 1 - y0)) / 7, y1 - 1);
  const int xx = min(xo + (gx * (O - 1)) / 7, W - 1);
  float lo = alpha[(long long)yy * sp + xx];
  float hi = beta[(long long)yy * sp + xx];
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, off, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, off, kWave));
  }
  return 0.5 * ((double)lo + (double)hi);
}

// Origin of the box kernel's power sums: the mid-range of the input values
// sampled on an 8 x 8 grid over the wave's output tile (their range in
// `span`). It depends on the input only, so the stack is the same whether
// the kernel takes the window bounds itself or reads them.
__device__ __forceinline__ double input_origin(const float* __restrict__ img, long long pitch,
                                               int y0, int y1, int xo, int O, int W, int lane,
                                               const FinMinMax& fm, double& span) {
  const int gy = lane >> 3, gx = lane & 7;
  const int yy = min(y0 + (gy * (y1 - 1 - y0)) / 7, y1 - 1);
  const int xx = min(xo + (gx * (O - 1)) / 7, W - 1);
  float lo = img[(long long)yy * pitch + xx] + 0.0f;
  float hi = lo;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    lo = fm.min(lo, __shfl_xor(lo, off, kWave));
    hi = fm.max(hi, __shfl_xor(hi, off, kWave));
  }
  span = (double)hi - (double)lo;
  return 0.5 * ((double)lo + (double)hi);
}

// Shift and Legendre change from raw window sums: m[1..N] are the sums of
// u^k over the window, u = f - c, and area the number of taps (box weights
// 1/area). Same steps as legendre_from_moments, with the normalisation
// folded into the final scaling (the shift is homogeneous in the sums, so
// it runs on the raw sums with m_0 = area).
//
// The conditioning test rho^N <= cond_max, rho = |mid|/half + 1, is taken as
// |mid| <= dmax half with dmax = cond_max^(1/N) - 1 (computed once per wave).
// A pixel that fails it is still accepted when wide > 0 and
// rho^N (beta - alpha) <= wide: the shift's rounding grows like rho^N, and
// it reaches the output scaled by the window's range beta - alpha (g^ =
// alpha + (beta - alpha) F), so with wide = cond_max times the range of
// the wave's input samples no pixel's error bound exceeds that of a window
// as wide as the samples at rho^N = cond_max. (Only the FP32 stack uses
// it; the rarely taken branch costs nothing on images without such
// pixels.)
template <int N>
__device__ __forceinline__ bool legendre_from_sums(double (&m)[N + 1], float a, float b,
                                                   double c, double dmax, double area,
                                                   double inv_area, double wide) {
  constexpr LegTable LT{};
  const double mid = 0.5 * ((double)a + (double)b) - c;
  const double half = 0.5 * ((double)b - (double)a);
  if (!(fabs(mid) <= dmax * half)) {
    const double rho = fabs(mid) / half + 1.0;
    double rn = rho;
#pragma unroll
    for (int k = 1; k < N; ++k) rn *= rho;
    if (!(rn * ((double)b - (double)a) <= wide)) return true;
  }
  const double ih = rcp(half);
  const double s = -mid;
  m[0] = area;
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int k = N; k > j; --k) m[k] = fma(s, m[k - 1], m[k]);
  double sc = ih * inv_area;
#pragma unroll
  for (int k = 1; k <= N; ++k) {
    m[k] *= sc;
    sc *= ih;
  }
  double out[N + 1];
#pragma unroll
  for (int k = 1; k <= N; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int r = k; r >= 1; r -= 2) acc = fma(LT.L[k][r], m[r], acc);
    // (r = 0 contributes L[k][0] nu_0 = L[k][0] for even k)
    if ((k & 1) == 0) acc += LT.L[k][0];
    out[k] = acc;
  }
#pragma unroll
  for (int k = 1; k <= N; ++k) m[k] = out[k];
  return false;
}

// Strips 0 .. n_strips-2 are O columns wide and cut into n_segs segments of
// TH rows; the last strip (the image's remaining columns, possibly far
// fewer) into n_segs_last segments of TH_last rows, so that its waves carry
// about as much work as the others. Waves: the full strips' segments
// (strip-major within a segment row), then the last strip's.
struct StripGeom {
  int O;       // output columns per strip
  int Rpad;    // R rounded up to a multiple of kV
  int TH;      // output rows per segment
  int n_strips;
  int n_segs;
  int TH_last;
  int n_segs_last;
  __host__ __device__ int waves() const { return (n_strips - 1) * n_segs + n_segs_last; }
};

// Slot of the exclusive prefix P(-1) = 0 in each power's LDS row (pidx(-1):
// a padding slot of the third column row, never written by the scan).
constexpr int kZeroSlot = 2 * kSlotStride + kSlotStride - 1;
static_assert(kZeroSlot == ((-1) & (kV - 1)) * kSlotStride + ((-1) >> 2), "pidx(-1)");

// One wave per workgroup: the LDS of a wave (its N prefix rows) then
// limits occupancy with no rounding to four-wave groups.
constexpr int kBoxWaves = 1;

template <int N, typename TS, bool FUSED>
__global__ __launch_bounds__(kBoxWaves * kWave) void moments_box(
    const float* __restrict__ img, long long pitch, int H, int W, int R,
    const float* __restrict__ alpha, const float* __restrict__ beta, long long sp,
    TS* __restrict__ mom, long long plane, StripGeom g, double cond_max, int vec4, Batch bt,
    FuseArgs fz) {
  __shared__ double sh[kBoxWaves][N][kStripSlots];
  // shift amplification limit as a bound on |mid - c| / half
  const double dmax = pow(cond_max, 1.0 / N) - 1.0;
  {
    const BatchOffsets o = bt.at(blockIdx.y, sizeof(TS));
    img = byte_offset(img, o.img);
    if (FUSED) {
      fz.theta = byte_offset(fz.theta, o.theta);
      fz.sigma = byte_offset(fz.sigma, o.sigma);
      fz.out = byte_offset(fz.out, o.out);
    }
    alpha = byte_offset(alpha, o.stack);
    beta = byte_offset(beta, o.stack);
    mom = byte_offset(mom, o.stack);
  }
  const int lane = threadIdx.x & (kWave - 1);
  // (wave-uniform, so that the strip geometry and every row base below are
  // scalar values)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int gw = blockIdx.x * kBoxWaves + wv;
  if (gw >= g.waves()) return;
  const FinMinMax fm;
  const int n_full = (g.n_strips - 1) * g.n_segs;
  const bool last = gw >= n_full;
  const int fs = max(g.n_strips - 1, 1);
  const int strip = last ? g.n_strips - 1 : gw % fs;
  const int th = last ? g.TH_last : g.TH;
  const int y0 = (last ? gw - n_full : gw / fs) * th;
  const int y1 = min(H, y0 + th);
  const int xo = strip * g.O;            // first output column of the strip
  const int ow = min(g.O, W - xo);       // its output columns
  const int xs = xo - g.Rpad;            // padded column 0
  double span;
  const double c = input_origin(img, pitch, y0, y1, xo, g.O, W, lane, fm, span);
  // width-aware acceptance of ill-conditioned shifts (FP32 stack only)
  const double wide = sizeof(TS) == 4 ? cond_max * span : 0.0;
  double (*const shw)[kStripSlots] = sh[wv];
  if (lane < N) shw[lane][kZeroSlot] = 0.0;

  int cx[kV];
#pragma unroll
  for (int v = 0; v < kV; ++v) cx[v] = min(max(xs + kV * lane + v, 0), W - 1);
  // the lane's 4 columns as one aligned float4 when they are all inside the
  // image (xs is a multiple of 4) and rows are 16-byte aligned
  const bool v4 = vec4 && xs + kV * lane >= 0 && xs + kV * lane + kV <= W;
  // (rows are wave-uniform: each load takes the row from a buffer resource
  // in scalar registers and the lane's column as a 32-bit byte offset)
  auto load4 = [&](const float* row, float (&q)[kV]) {
    const BufRsrc r = buf_rsrc(row);
    if (v4) {
      const float4 t4 = buf_ld_f32x4(r, (unsigned)(xs + kV * lane) * 4u);
      q[0] = t4.x; q[1] = t4.y; q[2] = t4.z; q[3] = t4.w;
    } else {
#pragma unroll
      for (int v = 0; v < kV; ++v) q[v] = buf_ld_f32(r, (unsigned)cx[v] * 4u);
    }
  };

  double S[N][kV];
#pragma unroll
  for (int k = 0; k < N; ++k)
#pragma unroll
    for (int v = 0; v < kV; ++v) S[k][v] = 0.0;

  for (int dy = -R; dy <= R; ++dy) {
    const float* row = img + (long long)min(max(y0 + dy, 0), H - 1) * pitch;
    float q[kV];
    load4(row, q);
#pragma unroll
    for (int v = 0; v < kV; ++v) {
      const double u = (double)q[v] - c;
      double p = u;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        S[k][v] += p;
        p *= u;
      }
    }
  }

  const double area = (double)(2 * R + 1) * (double)(2 * R + 1);
  const double inv_area = 1.0 / area;
  // the rows entering and leaving the window at y + 1, loaded one row ahead
  float qi[kV], qo[kV];
  auto load_step = [&](int yn) {
    load4(img + (long long)min(yn + R, H - 1) * pitch, qi);
    load4(img + (long long)max(yn - R - 1, 0) * pitch, qo);
  };
  if (y0 + 1 < y1) load_step(y0 + 1);
  for (int y = y0; y < y1; ++y) {
    float pa[kChunks], pb[kChunks];
    load_bounds_row(alpha, beta, sp, y, xo, g.O, W, lane, pa, pb);
    // fused: the row's theta (or f) and sigma as well, issued with the
    // bounds so that their latency overlaps the row's sums and scan
    float pt[kChunks], ps[kChunks];
    if (FUSED) {
      load_bounds_row(fz.theta, fz.sigma, fz.tpitch, y, xo, g.O, W, lane, pt, ps);
    }
    if (y > y0) {
      float ci[kV], co[kV];
#pragma unroll
      for (int v = 0; v < kV; ++v) {
        ci[v] = qi[v];
        co[v] = qo[v];
      }
      if (y + 1 < y1) load_step(y + 1);
#pragma unroll
      for (int v = 0; v < kV; ++v) {
        const double ui = (double)ci[v] - c;
        const double uo = (double)co[v] - c;
        double pi = ui, po = uo;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          S[k][v] += pi - po;
          pi *= ui;
          po *= uo;
        }
      }
    }
    // horizontal sums: inclusive prefix of the vertical sums along the strip
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double p0 = S[k][0];
      double p1 = p0 + S[k][1];
      double p2 = p1 + S[k][2];
      double p3 = p2 + S[k][3];
      const double incl = wave_inclusive_scan(p3, lane);
      const double ex = incl - p3;
      double* d = shw[k];
      d[pidx(kV * lane + 0)] = ex + p0;
      d[pidx(kV * lane + 1)] = ex + p1;
      d[pidx(kV * lane + 2)] = ex + p2;
      d[pidx(kV * lane + 3)] = incl;
    }
    wave_sync();
    TS* const mrow = mom + (long long)y * sp;
    // epilogue: lanes take consecutive output columns, chunk q = columns
    // 64 q .. 64 q + 63 of the strip's outputs. The chunks have no branch
    // between them (a flat window's zero moments are selected, and the
    // ill-conditioned pixels are only marked), so their LDS reads and
    // arithmetic overlap; the marked pixels are recomputed afterwards.
    unsigned badq = 0;                   // bit q: this lane's chunk-q pixel is marked
    auto chunk = [&](int q) {
      const int j = q * kWave + lane;
      const bool valid = j < g.O && xo + j < W;
      const int x = valid ? xo + j : xo;
      const int e = g.Rpad + (valid ? j : 0);
      const float a = q == 0 ? pa[0] : q == 1 ? pa[1] : q == 2 ? pa[2] : pa[3];
      const float b = q == 0 ? pb[0] : q == 1 ? pb[1] : q == 2 ? pb[2] : pb[3];
      double m[N + 1];
      const int eh = e + R, el = e - R - 1;
#pragma unroll
      for (int k = 0; k < N; ++k) m[k + 1] = shw[k][pidx(eh)] - shw[k][pidx(el)];
      const bool flat = a == b;
      const bool bad = legendre_from_sums<N>(m, a, b, c, dmax, area, inv_area, wide) && !flat;
      if (flat) {
#pragma unroll
        for (int k = 1; k <= N; ++k) m[k] = 0.0;
      }
      if (valid && !bad) {
        if (FUSED) {
          const float th = q == 0 ? pt[0] : q == 1 ? pt[1] : q == 2 ? pt[2] : pt[3];
          const float sg = q == 0 ? ps[0] : q == 1 ? ps[1] : q == 2 ? ps[2] : ps[3];
          fused_pixel<N, TS>(m, a, b, th, sg, mrow, plane, (unsigned)x * (unsigned)sizeof(TS),
                             buf_rsrc(static_cast<TS*>(fz.out) + (long long)y * fz.opitch), fz);
        } else {
          // the row's plane bases are wave-uniform: buffer resources in
          // scalar registers, one 32-bit byte offset per lane
          const unsigned xb = (unsigned)x * (unsigned)sizeof(TS);
#pragma unroll
          for (int k = 1; k <= N; ++k) buf_st(buf_rsrc(mrow + (k - 1) * plane), xb, TS(m[k]));
        }
      }
      if (valid && bad) badq |= 1u << q;
    };
    if (FUSED) {
      for (int q = 0; q < kChunks; ++q)
        if (q * kWave < ow) chunk(q);
    } else {
#pragma unroll
      for (int q = 0; q < kChunks; ++q)
        if (q * kWave < ow) chunk(q);
    }
    for (int q = 0; q < kChunks; ++q) {
      const bool mine = (badq >> q) & 1u;
      const unsigned long long mask = __ballot(mine);
      if (!mask) continue;
      const int j = q * kWave + lane;
      const int x = mine ? xo + j : xo;
      const float a = q == 0 ? pa[0] : q == 1 ? pa[1] : q == 2 ? pa[2] : pa[3];
      const float b = q == 0 ? pb[0] : q == 1 ? pb[1] : q == 2 ? pb[2] : pb[3];
      recompute_flagged<N, TS, FUSED>(mask, mine, y, x, a, b, img, pitch, H, W, R, nullptr,
                                      inv_area, mom, plane, sp, lane, fz);
    }
    wave_sync();
  }
}

// Gaussian kernel, tiled: a workgroup computes a kTY x TX tile of outputs.
// (Tile sizes keep the LDS tile at 30-40 KiB so that four workgroups share a
// CU.)
// Phase 1 (vertical): thread t owns padded column t, reads its kTY + 2R
// inputs once (coalesced across threads), forms the powers once per input
// and accumulates the kTY x N vertical weighted sums in registers; the sums
// go to LDS. With BOUNDS the same pass takes the column's min/max over each
// output row's 2R + 1 inputs (the rows' windows share the inputs
// kTY - 1 .. 2R). Phase 2 (horizontal): a thread owns kCB adjacent output
// columns of one row and accumulates their kCB x N horizontal weighted sums
// (with BOUNDS also the min/max, the two windows sharing 2R columns) from
// the (kCB + 2R) LDS columns they span. Phase 3: shift and Legendre basis
// per pixel (same epilogue as the box kernel, with the exact recompute for
// ill-conditioned pixels); with BOUNDS the window bounds alpha_i, beta_i
// (eq. bounds) are stored as well, so no separate bounds pass is needed.
// The power sums are taken about the tile's central input value, which the
// kernel knows before it reads anything else; the stack therefore does not
// depend on whether the bounds were computed here or read. Work per pixel
// is O(R), as for the paper's direct convolution.
constexpr int kTY = 4;   // output rows per tile
constexpr int kCB = 2;   // adjacent output columns per thread in the horizontal phase
constexpr int kPF = 8;   // input rows per prefetch chunk in the vertical phase
constexpr int kTilePasses = 4;   // origins per tile (then the direct recompute)

// doubles of LDS for the zero-padded tap weights (taps -(kTY-1) .. 2R+kTY-1),
// rounded up to an even count so that what follows stays 16-byte aligned
__host__ __device__ constexpr int tile_wext_len(int R) { return 2 * R + 2 * kTY; }
// widest tile (kTY * kTXMax / kCB <= 256 phase-2 threads) and the narrow LDS
// row stride, used while TX + 2R fits in it (else 256)
constexpr int kTXMax = 128;
constexpr int kESNarrow = 160;

// ES: the LDS row stride (>= TX + 2R), a compile-time constant so that the
// offsets of the N power planes fold into the LDS instructions' immediates.
// alpha, beta: read when !BOUNDS, written when BOUNDS.
template <int N, typename TS, bool FUSED, int ES, bool BOUNDS>
__global__ __launch_bounds__(256) void moments_gauss_tile(
    const float* __restrict__ img, long long pitch, int H, int W, int R, int TX, double inv2s2,
    float* __restrict__ alpha, float* __restrict__ beta, long long sp,
    TS* __restrict__ mom, long long plane, double cond_max, Batch bt, FuseArgs fz) {
  const FinMinMax fm;      // (window bounds)
  // dynamic LDS: [N][kTY][ES] doubles (vertical sums), the tap weights
  // (tile_wext_len(R) doubles), then (BOUNDS) [kTY][ES] float2 (min, max);
  // 16-byte aligned for the pair reads of phase 2
  extern __shared__ __attribute__((aligned(16))) double vsum[];
  double* const wext = vsum + N * kTY * ES;
  float2* const vmm = reinterpret_cast<float2*>(wext + tile_wext_len(R));
  {
    const BatchOffsets o = bt.at(blockIdx.z, sizeof(TS));
    img = byte_offset(img, o.img);
    if (FUSED) {
      fz.theta = byte_offset(fz.theta, o.theta);
      fz.sigma = byte_offset(fz.sigma, o.sigma);
      fz.out = byte_offset(fz.out, o.out);
    }
    alpha = byte_offset(alpha, o.stack);
    beta = byte_offset(beta, o.stack);
    mom = byte_offset(mom, o.stack);
  }
  // wext: 1-D weights of taps -(kTY-1) .. 2R+kTY-1 (zero outside [0, 2R]),
  // so the phases below apply every tap without a range test; wts = the
  // taps 0 .. 2R
  __shared__ double inv_z;
  double* const wts = wext + (kTY - 1);
  const int E = TX + 2 * R;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * kTY;
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1);
  // loads that depend on nothing else go out before the weights are formed:
  // the tile's central input value (the origin of the power sums; one
  // cache line for the whole workgroup) and the first rows of the column
  const int yc = min(y0 + kTY / 2, H - 1), xc = min(x0 + TX / 2, W - 1);
  const float cval = img[(long long)yc * pitch + xc];
  // Phase 1 roles: thread t sums padded column tc = t over all n_in input
  // rows. When the last, partial wave would hold at most 32 columns, it
  // takes each of them twice instead (the split wave): lanes 0..31 sum the
  // top half of the rows, lanes 32..63 the bottom half in reverse order, and
  // the halves are added across lanes, so that wave runs half the rows.
  // Reversed, the bottom half's row ii meets output row kTY-1-s at tap
  // 2R - (ii - s), whose weight equals that of tap ii - s (the weights are
  // symmetric), and it lies in that row's window exactly when the top
  // half's row ii lies in row s's: so both halves run the same wave-uniform
  // code, the bottom half holding output row rr in accumulator slot kTY-1-rr.
  static_assert(kTY % 2 == 0, "the split wave pairs slots rr and kTY-1-rr");
  const int n_in = kTY + 2 * R;      // even
  const int fw = E / kWave, tw = E - fw * kWave;
  // The split is compiled for the narrow LDS stride only (R <= 16, where the
  // tail is 2R <= 32 columns), and not into the multi-pass instantiations,
  // whose registers are already at the limit. sw is wave-uniform and taken
  // from the first lane, so the compiler branches on a scalar instead of
  // running both roles under lane masks.
  constexpr bool kSplit = ES == kESNarrow && !(sizeof(TS) == 8 && N >= 7);
  const bool sw = kSplit && __builtin_amdgcn_readfirstlane(tw > 0 && tw <= kWave / 2 &&
                                                 (fw + 1) * kWave <= (int)blockDim.x &&
                                                 t / kWave == fw) != 0;
  const int tc = sw ? fw * kWave + (lane & (kWave / 2 - 1)) : t;
  const bool rev = sw && lane >= kWave / 2;
  const bool col_ok = sw ? (lane & (kWave / 2 - 1)) < tw : t < E;
  const float* col = img + min(max(x0 - R + tc, 0), W - 1);
  // rows i0 .. i0 + PF - 1 of the thread's range (SW: the split wave, which
  // prefetches half as many rows at a time to hold fewer registers)
  auto load_chunk = [&](auto sw_c, int i0, float (&q)[kPF]) {
    constexpr bool SW = decltype(sw_c)::value;
    constexpr int PF = SW ? kPF / 2 : kPF;
    const int nr = SW ? n_in / 2 : n_in;
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int ii = min(i0 + p, nr - 1);
      const int i = (SW && rev) ? n_in - 1 - ii : ii;
      q[p] = col[(long long)min(max(y0 - R + i, 0), H - 1) * pitch];
    }
  };
  float qn[kPF];
  if constexpr (kSplit) {
    if (sw) {
      if (col_ok) load_chunk(std::true_type{}, 0, qn);
    } else {
      if (col_ok) load_chunk(std::false_type{}, 0, qn);
    }
  } else {
    if (col_ok) load_chunk(std::false_type{}, 0, qn);
  }
  for (int i = t; i < 2 * R + 2 * kTY - 1; i += blockDim.x) {
    const int tap = i - (kTY - 1);
    const double d = (double)(tap - R);
    wext[i] = (tap >= 0 && tap <= 2 * R) ? exp(-d * d * inv2s2) : 0.0;
  }
  if (t < kWave) {
    // 1-D normalisation: the taps' sum, lane l adding taps l, l + 64, ...
    double zp = 0.0;
    for (int i = lane; i <= 2 * R; i += kWave) {
      const double d = (double)(i - R);
      zp += exp(-d * d * inv2s2);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) zp += __shfl_xor(zp, off, kWave);
    if (t == 0) inv_z = 1.0 / zp;
  }
  __syncthreads();
  const double iz = inv_z;
  const double norm = iz * iz;
  double c = (double)cval;

  // phase 2/3 role: kCB adjacent output columns xl .. of output row r
  const int groups = TX / kCB;
  const int r = t / groups, gq = t - r * groups;
  const bool active = r < kTY;
  const int xl = kCB * gq;
  float pa[kCB], pb[kCB];           // the outputs' window bounds
  bool pend[kCB];                   // ill-conditioned about every origin so far
#pragma unroll
  for (int v = 0; v < kCB; ++v) {
    pa[v] = 0.f;
    pb[v] = 0.f;
    pend[v] = false;
  }
  __shared__ int next_pick;
  __shared__ double next_origin;

  // Pass p takes the power sums about origin c and finishes every pixel
  // (after the first pass: every pending pixel) whose shift is well
  // conditioned about it; the next origin is the window mid-range of the
  // first pixel still pending. Pixels still ill-conditioned in the last
  // pass are recomputed directly. Only the FP64 path at N >= 7 takes more
  // than one pass (its threshold flags many pixels on high-contrast
  // content); a single pass keeps the kernel at half the registers.
  constexpr int kPasses = (sizeof(TS) == 8 && N >= 7) ? kTilePasses : 1;
#pragma unroll 1
  for (int pass_ = 0; pass_ < kPasses; ++pass_) {
    const int pass = kPasses == 1 ? 0 : pass_;     // constants when there is one pass
    const bool first = pass == 0, last = kPasses == 1 || pass == kPasses - 1;
    // phase 1: vertical sums for padded column tc. The column's inputs are
    // read in chunks of kPF rows, the next chunk's loads issued before the
    // current chunk is used, so memory latency overlaps the arithmetic.
    auto vertical = [&](auto sw_c) {
      constexpr bool SW = decltype(sw_c)::value;
      const int nr = SW ? n_in / 2 : n_in;     // rows this thread sums
      if (!first) load_chunk(sw_c, 0, qn);
      double acc[kTY][N];
#pragma unroll
      for (int rr = 0; rr < kTY; ++rr)
#pragma unroll
        for (int k = 0; k < N; ++k) acc[rr][k] = 0.0;
      // BOUNDS (first pass): min/max of the inputs shared by every row's
      // window (cmn, cmx) and of each row's other inputs (mn, mx)
      float cmn = INFINITY, cmx = -INFINITY, mn[kTY], mx[kTY];
#pragma unroll
      for (int rr = 0; rr < kTY; ++rr) {
        mn[rr] = INFINITY;
        mx[rr] = -INFINITY;
      }
      constexpr int PF = SW ? kPF / 2 : kPF;
      for (int i0 = 0; i0 < nr; i0 += PF) {
        float q[PF];
#pragma unroll
        for (int p = 0; p < PF; ++p) q[p] = qn[p];
        if (i0 + PF < nr) load_chunk(sw_c, i0 + PF, qn);
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          const int i = i0 + p;      // (the bottom half: row n_in - 1 - i)
          if (i < nr) {
            const double u = (double)q[p] - c;
            double pw[N];
            pw[0] = u;
#pragma unroll
            for (int k = 1; k < N; ++k) pw[k] = pw[k - 1] * u;
            // output row rr takes tap i - rr (a zero weight outside [0, 2R])
#pragma unroll
            for (int rr = 0; rr < kTY; ++rr) {
              const double wv = wts[i - rr];
#pragma unroll
              for (int k = 0; k < N; ++k) acc[rr][k] = fma(wv, pw[k], acc[rr][k]);
            }
            if (BOUNDS && first) {
              const float v = q[p] + 0.0f;     // -0 -> +0, as the bounds kernel
              if (i >= kTY - 1 && i <= 2 * R) {
                cmn = fm.min(cmn, v);
                cmx = fm.max(cmx, v);
              } else {
#pragma unroll
                for (int rr = 0; rr < kTY; ++rr)
                  if (i >= rr && i <= rr + 2 * R) {
                    mn[rr] = fm.min(mn[rr], v);
                    mx[rr] = fm.max(mx[rr], v);
                  }
              }
            }
          }
        }
      }
      if constexpr (SW) {
        // Row rr's sums are the top half's slot rr plus the bottom half's
        // slot kTY-1-rr. The top lane finishes rows 0 .. kTY/2-1 and its
        // partner (lane + 32) rows kTY/2 .. kTY-1, each receiving the slot it
        // lacks from the other in one exchange per row and power.
        constexpr int kH = kWave / 2;
        float cn = 0.f, cx = 0.f;
        if (BOUNDS && first) {
          cn = fm.min(cmn, __shfl_xor(cmn, kH));
          cx = fm.max(cmx, __shfl_xor(cmx, kH));
        }
#pragma unroll
        for (int q = 0; q < kTY / 2; ++q) {
          const int row = rev ? kTY / 2 + q : q;
#pragma unroll
          for (int k = 0; k < N; ++k) {
            const double snd = rev ? acc[kTY - 1 - q][k] : acc[kTY / 2 + q][k];
            const double own = rev ? acc[kTY / 2 - 1 - q][k] : acc[q][k];
            vsum[(k * kTY + row) * ES + tc] = own + __shfl_xor(snd, kH);
          }
          if (BOUNDS && first) {
            const float sn = rev ? mn[kTY - 1 - q] : mn[kTY / 2 + q];
            const float sx = rev ? mx[kTY - 1 - q] : mx[kTY / 2 + q];
            const float on = rev ? mn[kTY / 2 - 1 - q] : mn[q];
            const float ox = rev ? mx[kTY / 2 - 1 - q] : mx[q];
            vmm[row * ES + tc] = make_float2(fm.min(fm.min(on, __shfl_xor(sn, kH)), cn),
                                             fm.max(fm.max(ox, __shfl_xor(sx, kH)), cx));
          }
        }
      } else {
#pragma unroll
        for (int rr = 0; rr < kTY; ++rr)
#pragma unroll
          for (int k = 0; k < N; ++k) vsum[(k * kTY + rr) * ES + tc] = acc[rr][k];
        if (BOUNDS && first) {
#pragma unroll
          for (int rr = 0; rr < kTY; ++rr)
            vmm[rr * ES + tc] = make_float2(fm.min(mn[rr], cmn), fm.max(mx[rr], cmx));
        }
      }
    };
    if (sw) {
      if constexpr (kSplit) {
        if (col_ok) vertical(std::true_type{});
      }
    } else if (col_ok) {
      if (!first) load_chunk(std::false_type{}, 0, qn);
      double acc[kTY][N];
#pragma unroll
      for (int rr = 0; rr < kTY; ++rr)
#pragma unroll
        for (int k = 0; k < N; ++k) acc[rr][k] = 0.0;
      // BOUNDS (first pass): min/max of the inputs shared by every row's
      // window (cmn, cmx) and of each row's other inputs (mn, mx)
      float cmn = INFINITY, cmx = -INFINITY, mn[kTY], mx[kTY];
#pragma unroll
      for (int rr = 0; rr < kTY; ++rr) {
        mn[rr] = INFINITY;
        mx[rr] = -INFINITY;
      }
      for (int i0 = 0; i0 < n_in; i0 += kPF) {
        float q[kPF];
#pragma unroll
        for (int p = 0; p < kPF; ++p) q[p] = qn[p];
        if (i0 + kPF < n_in) load_chunk(std::false_type{}, i0 + kPF, qn);
#pragma unroll
        for (int p = 0; p < kPF; ++p) {
          const int i = i0 + p;
          if (i < n_in) {
            const double u = (double)q[p] - c;
            double pw[N];
            pw[0] = u;
#pragma unroll
            for (int k = 1; k < N; ++k) pw[k] = pw[k - 1] * u;
            // output row rr takes tap i - rr (a zero weight outside [0, 2R])
#pragma unroll
            for (int rr = 0; rr < kTY; ++rr) {
              const double wv = wts[i - rr];
#pragma unroll
              for (int k = 0; k < N; ++k) acc[rr][k] = fma(wv, pw[k], acc[rr][k]);
            }
            if (BOUNDS && first) {
              const float v = q[p] + 0.0f;     // -0 -> +0, as the bounds kernel
              if (i >= kTY - 1 && i <= 2 * R) {
                cmn = fm.min(cmn, v);
                cmx = fm.max(cmx, v);
              } else {
#pragma unroll
                for (int rr = 0; rr < kTY; ++rr)
                  if (i >= rr && i <= rr + 2 * R) {
                    mn[rr] = fm.min(mn[rr], v);
                    mx[rr] = fm.max(mx[rr], v);
                  }
              }
            }
          }
        }
      }
#pragma unroll
      for (int rr = 0; rr < kTY; ++rr)
#pragma unroll
        for (int k = 0; k < N; ++k) vsum[(k * kTY + rr) * ES + tc] = acc[rr][k];
      if (BOUNDS && first) {
#pragma unroll
        for (int rr = 0; rr < kTY; ++rr)
          vmm[rr * ES + tc] = make_float2(fm.min(mn[rr], cmn), fm.max(mx[rr], cmx));
      }
    }
    __syncthreads();

    // phase 2: horizontal sums for kCB adjacent outputs of one row. The
    // (kCB + 2R) LDS columns a thread spans are read as 16-byte pairs: the
    // pairs of neighbouring lanes are contiguous, so the reads are free of
    // bank conflicts (ES, 2R and the thread's first column are even).
    // Column cc (relative to the thread's first) feeds output v at tap cc - v.
    double m4[kCB][N + 1];
    if (active) {
      // BOUNDS: window min/max of the outputs; columns kCB - 1 .. 2R are in
      // every output's window (hmn, hmx), the others in some of them
      float bmn[kCB], bmx[kCB];
#pragma unroll
      for (int v = 0; v < kCB; ++v) {
        bmn[v] = INFINITY;
        bmx[v] = -INFINITY;
      }
#pragma unroll
      for (int v = 0; v < kCB; ++v)
#pragma unroll
        for (int k = 0; k <= N; ++k) m4[v][k] = 0.0;
      float hmn = INFINITY, hmx = -INFINITY;
      const double2* vs2 = reinterpret_cast<const double2*>(vsum);
      const float4* vm4 = reinterpret_cast<const float4*>(vmm);
      auto take = [&](int cc, float lo, float hi) {
        if (cc >= kCB - 1 && cc <= 2 * R) {
          hmn = fm.min(hmn, lo);
          hmx = fm.max(hmx, hi);
        } else {
#pragma unroll
          for (int v = 0; v < kCB; ++v)
            if (cc >= v && cc <= v + 2 * R) {
              bmn[v] = fm.min(bmn[v], lo);
              bmx[v] = fm.max(bmx[v], hi);
            }
        }
      };
      for (int j = 0; j < kCB + 2 * R; j += 2) {
        double2 val[N];
#pragma unroll
        for (int k = 0; k < N; ++k) val[k] = vs2[((k * kTY + r) * ES + xl + j) >> 1];
        if (BOUNDS && first) {
          // (min, max) of columns xl + j and xl + j + 1
          const float4 qm = vm4[(r * ES + xl + j) >> 1];
          take(j, qm.x, qm.y);
          take(j + 1, qm.z, qm.w);
        }
        double wa[kCB], wb[kCB];      // taps j - v and j + 1 - v (0 outside [0, 2R])
#pragma unroll
        for (int v = 0; v < kCB; ++v) {
          wa[v] = wts[j - v];
          wb[v] = wts[j + 1 - v];
        }
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
          for (int v = 0; v < kCB; ++v) {
            m4[v][k + 1] = fma(wa[v], val[k].x, m4[v][k + 1]);
            m4[v][k + 1] = fma(wb[v], val[k].y, m4[v][k + 1]);
          }
      }
      if (first) {
#pragma unroll
        for (int v = 0; v < kCB; ++v) {
          const int y = y0 + r, x = x0 + xl + v;
          if (y < H && x < W && xl + v < TX) {
            const long long idx = (long long)y * sp + x;
            if (BOUNDS) {
              pa[v] = fm.min(bmn[v], hmn);
              pb[v] = fm.max(bmx[v], hmx);
              alpha[idx] = pa[v];
              beta[idx] = pb[v];
            } else {
              pa[v] = alpha[idx];
              pb[v] = beta[idx];
            }
          }
        }
      }
    }
    // phase 3: per-pixel epilogue (all lanes take part in the wave ballots)
    bool anyp = false;
#pragma unroll
    for (int v = 0; v < kCB; ++v) {
      const int y = y0 + r, x = x0 + xl + v;
      const bool valid = active && y < H && x < W && xl + v < TX;
      const bool want = valid && (first || pend[v]);
      const long long idx = (long long)(valid ? y : 0) * sp + (valid ? x : 0);
      bool bad = false;
      if (want) {
        double m[N + 1];
        m[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= N; ++k) m[k] = m4[v][k] * norm;
        bad = legendre_from_moments<N>(m, pa[v], pb[v], c, cond_max);
        if (!bad) finish_pixel<N, TS, FUSED>(m, pa[v], pb[v], y, x, idx, mom, plane, fz);
        pend[v] = bad && !last;
      }
      anyp = anyp || pend[v];
      const unsigned long long mask = __ballot(want && bad && last);
      if (mask)
        recompute_flagged<N, TS, FUSED>(mask, want && bad && last, y, x, pa[v], pb[v], img, pitch, H,
                                        W, R, wts, norm, mom, plane, sp, lane, fz);
    }
    if (kPasses == 1) break;
    // the next origin: the window mid-range of the first pending pixel (the
    // barrier also keeps this pass's LDS reads ahead of the next pass's writes)
    if (!__syncthreads_or(anyp)) break;
    if (t == 0) next_pick = 0x7fffffff;
    __syncthreads();
#pragma unroll
    for (int v = 0; v < kCB; ++v)
      if (pend[v]) atomicMin(&next_pick, r * TX + xl + v);
    __syncthreads();
    const int pk = next_pick;
#pragma unroll
    for (int v = 0; v < kCB; ++v)
      if (pend[v] && r * TX + xl + v == pk) next_origin = 0.5 * ((double)pa[v] + (double)pb[v]);
    __syncthreads();
    c = next_origin;
  }
}

// Gaussian kernel on the matrix cores (R <= 16): the separable weighted sums
// are banded matrix products done with v_mfma_f64_16x16x4f64 (FP64 in,
// FP64 accumulate). A wave owns a strip of 16 output columns and walks down
// it in 16-row blocks. For a 16-row block of the image, the horizontal pass
//   H_k[r][c] = sum_j (f - c0)^k[r][x0 - R + j] w(j - c),  c < 16,
// is one product per power k: A = the pixels' powers (row r = lane & 15,
// column j = 4 s + (lane >> 4) of K-step s, each lane loading one pixel per
// step), B = the band of weights. Its result stays in the MFMA output
// layout, where the 4 registers of a lane hold rows 4 v + (lane >> 4) of
// column lane & 15; each register v is exactly the B operand of a K-step
// over those 4 rows, so the vertical pass
//   G_k[r'][c] = sum_rows w(row - r' + R) H_k[row][c]
// over the three row blocks b-1, b, b+1 (R <= 16) needs no data movement.
// The wave keeps the three blocks' H in registers and computes one new
// block per output block. G is the window moment of (f - c0)^k (weights
// normalised to sum 1); the epilogue is the other kernels' (shift, Legendre
// basis, exact recompute of ill-conditioned pixels).
typedef double mfma_d4 __attribute__((ext_vector_type(4)));
constexpr int kMfmaRMax = 16;
constexpr int kKHMax = (16 + 2 * kMfmaRMax + 3) / 4;   // K-steps of the horizontal pass

__device__ __forceinline__ mfma_d4 mfma16(double a, double b, mfma_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int N, typename TS>
__global__ __launch_bounds__(kWaves * kWave, N <= 6 ? 2 : 1) void moments_gauss_mfma(
    const float* __restrict__ img, long long pitch, int H, int W, int R, double inv2s2,
    const float* __restrict__ alpha, const float* __restrict__ beta, long long sp,
    TS* __restrict__ mom, long long plane, int TH, int n_strips, int n_segs, double cond_max,
    Batch bt) {
  __shared__ double wts[2 * kMfmaRMax + 1];          // 1-D weights, normalised to sum 1
  // per-lane MFMA weight fragments, the same for every wave: fh[s][lane] the
  // horizontal pass's B operand of K-step s, fv[t][lane] the vertical pass's
  // A operand for row block b + t / 4 - 1 and register t % 4
  __shared__ double fh[kKHMax][kWave];
  __shared__ double fv[12][kWave];
  {
    const BatchOffsets o = bt.at(blockIdx.y, sizeof(TS));
    img = byte_offset(img, o.img);
    alpha = byte_offset(alpha, o.stack);
    beta = byte_offset(beta, o.stack);
    mom = byte_offset(mom, o.stack);
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int m = lane >> 4, q = lane & 15;
  if (threadIdx.x < kWave) {
    double zp = 0.0;
    for (int i = lane; i <= 2 * R; i += kWave) {
      const double d = (double)(i - R);
      zp += exp(-d * d * inv2s2);
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) zp += __shfl_xor(zp, off, kWave);
    for (int i = lane; i <= 2 * R; i += kWave) {
      const double d = (double)(i - R);
      wts[i] = exp(-d * d * inv2s2) / zp;
    }
  }
  __syncthreads();
  if (threadIdx.x < kWave) {
    // horizontal: input column 4 s + m of the K-step feeds output column q
    // with tap 4 s + m - q (zero off the band, which covers s >= KH too)
#pragma unroll
    for (int s = 0; s < kKHMax; ++s) {
      const int d = 4 * s + m - q;
      fh[s][lane] = (d >= 0 && d <= 2 * R) ? wts[d] : 0.0;
    }
    // vertical: output row q takes input row 16 dl + 4 v + m with tap
    // 16 dl + 4 v + m - q + R
#pragma unroll
    for (int t = 0; t < 12; ++t) {
      const int d = 16 * (t / 4 - 1) + 4 * (t % 4) + m - q + R;
      fv[t][lane] = (d >= 0 && d <= 2 * R) ? wts[d] : 0.0;
    }
  }
  __syncthreads();
  const int gw = blockIdx.x * kWaves + wv;
  if (gw >= n_strips * n_segs) return;
  const int strip = gw % n_strips, seg = gw / n_strips;
  const int x0 = strip * 16;
  const int y0 = seg * TH;                           // a multiple of 16
  const int y1 = min(H, y0 + TH);
  const int KH = (16 + 2 * R + 3) / 4;
  const double c = wave_origin(alpha, beta, sp, y0, y1, x0, 16, W, lane);
  const int xc = x0 - R + m;

  // pixels of the 16-row block bb this lane feeds to the horizontal pass
  // (rows and columns clamped to the image)
  auto hload = [&](int bb, float (&v)[kKHMax]) {
    const float* row = img + (long long)min(max(16 * bb + q, 0), H - 1) * pitch;
#pragma unroll
    for (int s = 0; s < kKHMax; ++s)
      v[s] = (s < KH) ? row[min(max(xc + 4 * s, 0), W - 1)] : 0.0f;
  };
  // horizontal pass of a 16-row block from its loaded pixels
  auto hpass = [&](const float (&v)[kKHMax], mfma_d4 (&Hk)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) Hk[k] = mfma_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kKHMax; ++s) {
      if (s < KH) {
        const double wf = fh[s][lane];
        const double u = (double)v[s] - c;
        double p = u;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          Hk[k] = mfma16(p, wf, Hk[k]);
          p *= u;
        }
      }
    }
  };
  // acc += (vertical weights of row-block offset t0 / 4 - 1) x Hk; a K-step
  // whose 4 rows lie outside every output row's window [-R, 15 + R] has only
  // zero weights and is skipped
  auto vpass = [&](int t0, const mfma_d4 (&Hk)[N], mfma_d4 (&acc)[N]) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row0 = 16 * (t0 / 4 - 1) + 4 * v;          // first row of the K-step
      if (row0 + 3 < -R || row0 > 15 + R) continue;
      const double wf = fv[t0 + v][lane];
#pragma unroll
      for (int k = 0; k < N; ++k) acc[k] = mfma16(wf, Hk[k][v], acc[k]);
    }
  };
  // the window moments of output block b are P_b + Wv(+1) H_{b+1} with the
  // partial sum P_b = Wv(-1) H_{b-1} + Wv(0) H_b carried from the previous
  // step; Hc = H_b, Hn receives H_{b+1}, pix holds block b+1's pixels and is
  // refilled with block b+2's
  float pix[kKHMax];
  mfma_d4 P[N];
  auto step = [&](int b, const mfma_d4 (&Hc)[N], mfma_d4 (&Hn)[N]) {
    // this block's window bounds, loaded ahead of the epilogue
    float pa[4], pb[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int y = min(16 * b + 4 * v + m, y1 - 1), x = min(x0 + q, W - 1);
      pa[v] = alpha[(long long)y * sp + x];
      pb[v] = beta[(long long)y * sp + x];
    }
    hpass(pix, Hn);
    hload(b + 2, pix);
    vpass(8, Hn, P);                                 // P = moments of block b
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int y = 16 * b + 4 * v + m, x = x0 + q;
      const bool valid = y < y1 && x < W;
      const long long idx = (long long)(valid ? y : y0) * sp + (valid ? x : x0);
      float a = 0.f, bb = 0.f;
      bool bad = false;
      if (valid) {
        double mm[N + 1];
        mm[0] = 1.0;
#pragma unroll
        for (int k = 0; k < N; ++k) mm[k + 1] = P[k][v];
        a = pa[v];
        bb = pb[v];
        bad = legendre_from_moments<N>(mm, a, bb, c, cond_max);
        if (!bad) finish_pixel<N, TS, false>(mm, a, bb, y, x, idx, mom, plane, FuseArgs{});
      }
      const unsigned long long mask = __ballot(valid && bad);
      if (mask)
        recompute_flagged<N, TS, false>(mask, valid && bad, y, x, a, bb, img, pitch, H, W, R,
                                        wts, 1.0, mom, plane, sp, lane, FuseArgs{});
    }
    // partial sum of block b + 1
#pragma unroll
    for (int k = 0; k < N; ++k) P[k] = mfma_d4{0.0, 0.0, 0.0, 0.0};
    vpass(0, Hc, P);
    vpass(4, Hn, P);
  };
  const int b0 = y0 / 16, b1 = (y1 + 15) / 16;
  mfma_d4 HA[N], HB[N];
#pragma unroll
  for (int k = 0; k < N; ++k) P[k] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  hload(b0 - 1, pix);
  hpass(pix, HA);
  vpass(0, HA, P);
  hload(b0, pix);
  hpass(pix, HB);
  vpass(4, HB, P);
  hload(b0 + 1, pix);
  // two alternating buffers for H_b and H_{b+1}
  for (int b = b0; b < b1; b += 2) {
    step(b, HB, HA);
    if (b + 1 < b1) step(b + 1, HA, HB);
  }
}

// Output columns per Gaussian tile: at most 128, with the LDS tile
// kTY x (TX + 2R) x N doubles within 64 KiB; 0 if R is too large.
int gauss_tile_tx(int R, int N) {
  int e = 65536 / (kTY * 8 * N);          // padded columns within 64 KiB of LDS
  if (e > 256) e = 256;                   // one phase-1 thread per padded column
  int tx = e - 2 * R;
  if (tx > kTXMax) tx = kTXMax;
  tx &= ~(kCB - 1);
  return tx >= kCB ? tx : 0;
}

// Segment height: the running sums pay a 2R-row warm-up per segment, so
// segments should be long; but the grid should also fill the device in
// whole rounds (a last, partly filled round of waves idles most CUs). The
// height is the smallest that makes all waves fit in `capacity` resident
// waves (one round), else two rounds, ..., capped at 64 rows. The last
// strip's rows cost (ve + its chunks) / (ve + a full strip's chunks) of a
// full strip's, ve being the cost of a row's vertical update and scan in
// units of one 64-column chunk of the row's epilogue (from instruction
// counts: about 0.8 with the fused range stage, about 3 without); its
// segments are taller by that factor (at most 64 rows as well).
StripGeom make_geom(int H, int W, int R, long long capacity, double ve) {
  StripGeom g;
  g.Rpad = (R + kV - 1) / kV * kV;
  g.O = (kStrip - R - g.Rpad) / kV * kV;
  // With the fused range stage a strip outputs three full 64-column chunks
  // (192 columns) rather than up to 240, whose fourth chunk would run the
  // expensive epilogue with a quarter of its lanes idle (measured: 4096^2,
  // rho 5, N 8: 467 -> 458 us; 128 columns: 498 us)
  if (ve < 1.0 && g.O > 3 * kWave) g.O = 3 * kWave;
  g.n_strips = (W + g.O - 1) / g.O;
  const int o_last = W - (g.n_strips - 1) * g.O;
  double r = g.n_strips == 1 ? 1.0
                              : (ve + (o_last + kWave - 1) / kWave) /
                                    (ve + (g.O + kWave - 1) / kWave);
  // (balance only a grid that fills the device: with fewer waves than
  // resident slots the kernel lasts as long as its slowest wave, and
  // shorter segments always help)
  const bool balance = (long long)g.n_strips * ((H + 1) / 2) > capacity / 2;
  if (!balance) r = 1.0;
  const double units = (g.n_strips - 1) + r;
  auto fit = [&](int th, long long budget) {
    g.TH = th;
    g.n_segs = (H + th - 1) / th;
    g.TH_last = std::min(64, std::max(th, (int)(th / r)));
    g.n_segs_last = (H + g.TH_last - 1) / g.TH_last;
    return g.waves() <= budget;
  };
  for (long long m = 1; m <= 64; ++m) {
    const long long budget = m * capacity;
    const long long segs = (long long)(budget / units);
    if (segs < 1) continue;
    for (int th = std::max(2LL, (H + segs - 1) / segs); th <= 64; ++th)
      if (fit(th, budget)) return g;
  }
  fit(64, 0);
  return g;
}

int device_cus() {
  static int cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
      n = 256;
    return n;
  }();
  return cus;
}


// The matrix-core kernel is the faster one for wide windows on large
// images on the mixed path (measured: at 2048^2 and 4096^2 with 8 <= R <= 16
// it takes 0.8-0.95 of the tile kernel's time; at 1024^2 they tie, below
// that it is slower); the FP64 path keeps the tile kernel.
// Degrees 7 and 8 stay on the tile kernel, whose re-origin passes keep
// their ill-conditioned pixels cheap.
bool gauss_on_mfma(int R, int N, long long h, long long w) {
  return R <= kMfmaRMax && R >= 8 && N <= 6 && h * w >= (1LL << 22);
}

}  // namespace

// abf_fast's path for the box kernel on the mixed path at small radii: the
// moment and range stages fused in one kernel (the moments stay in
// registers), measured faster on MI355X at rho = 5, N = 5..8 (4096^2, two
// images in flight: 0.85-0.95 of the stack path's time per image) and
// slower at rho = 20 (1.01-1.05). Elsewhere the stack path.
bool fast_fuses(int kernel_kind, int rho, int N, int prec) {
  return kernel_kind == 0 && prec == 1 && N >= 1 && rho <= kFuseRhoMax;
}

namespace {

template <int N, typename TS>
hipError_t launch_moments_t(const float* img, long long pitch, int h, int w, int kind,
                            double sigma_s, int R, float* alpha, float* beta,
                            long long sp, TS* mom, long long plane, hipStream_t stream,
                            const Batch& b, const FuseSpec* fs, bool bounds) {
  if (bounds && !moments_take_bounds(kind, R, N, h, w)) return hipErrorNotSupported;
  // resident waves of the box kernel on this device (occupancy x CUs). The
  // segment geometry depends on the image, radius and device only (not on
  // the batch size or on fusion), so an image gets bit-identical moments
  // alone, in a batch or fused with the range stage. Where abf_fast fuses
  // the stages it is sized for the lower of the stack and fused
  // instantiations' occupancies, so the fused kernel runs no partly filled
  // second round of waves; elsewhere for the stack kernel's own.
  auto occupancy = [](const void* fn) {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBoxWaves * kWave, 0) !=
            hipSuccess || blocks < 1)
      blocks = 8;
    return (long long)blocks * kBoxWaves * device_cus();
  };
  static const long long cap_stack =
      occupancy(reinterpret_cast<const void*>(moments_box<N, TS, false>));
  static const long long cap_both = std::min(
      cap_stack, occupancy(reinterpret_cast<const void*>(moments_box<N, TS, true>)));
  const bool fused_geom = fast_fuses(kind, R, N, sizeof(TS) == 4 ? 1 : 0);
  const StripGeom g = make_geom(h, w, R, fused_geom ? cap_both : cap_stack, fused_geom ? 0.8 : 3.0);
  // largest tolerated shift amplification rho^N before a pixel is taken
  // about another origin (or recomputed): the FP32 stack only needs to stay
  // below its own rounding; the FP64 path's 1e-6 bound was checked pixel
  // by pixel on 4096^2 images with clipped, high-contrast regions, where the
  // shift's rounding (amplified further by the Legendre coefficients, which
  // grow with N) needed rho^N <= 1e4 at N = 8
  const double cond_max = sizeof(TS) == 4 ? 1e12 : fp64_cond_max(N);
  const int waves = g.waves();
  // The box kernel's running sums add and remove every row of a strip
  // segment, so their rounding follows the largest values the strip holds,
  // not the pixel's window: too much for the FP64 path at N >= 7 on
  // high-contrast images. That case takes the tile kernel with unit
  // weights (direct sums over each window, and its re-origin passes).
  const bool box_tile = kind == 0 && sizeof(TS) == 8 && N >= 7;
  FuseArgs fz{};
  if (fs) {
    fz.theta = fs->theta;
    fz.sigma = fs->sigma;
    fz.tpitch = fs->tpitch;
    fz.out = fs->out;
    fz.opitch = fs->opitch;
    fz.flags = fs->flags;
    fz.keep_stack = fs->keep_stack;
  }
  if (kind == 0 && !box_tile) {
    dim3 grid((waves + kBoxWaves - 1) / kBoxWaves, b.n);
    // 16-byte loads where every image's rows start 16-byte aligned
    bool rows16 = pitch % 4 == 0 && b.img % 4 == 0 && reinterpret_cast<uintptr_t>(img) % 16 == 0;
    for (int z = 0; b.host_tab && z < b.n; ++z) rows16 = rows16 && b.host_tab[z].img % 16 == 0;
    const int vec4 = rows16 ? 1 : 0;
    if (fs)
      hipLaunchKernelGGL((moments_box<N, TS, true>), grid, dim3(kBoxWaves * kWave), 0, stream,
                         img, pitch, h, w, R, alpha, beta, sp, mom, plane, g, cond_max, vec4, b, fz);
    else
      hipLaunchKernelGGL((moments_box<N, TS, false>), grid, dim3(kBoxWaves * kWave), 0, stream,
                         img, pitch, h, w, R, alpha, beta, sp, mom, plane, g, cond_max, vec4, b, fz);
    return hipGetLastError();
  }
  const double s = sigma_s > 0 ? sigma_s : (R > 0 ? R / 3.0 : 1.0);
  // (the FP64 path takes the tile kernel there instead, reading the bounds:
  // the matrix-core kernel takes one origin per 16-column strip segment,
  // and under the FP64 path's tighter conditioning limits the pixels it
  // recomputed from their windows cost 13-40 ms per 4096^2 image at
  // R = 8-15, N = 6, on a field with wide flat regions, against about 1 ms
  // for the tile kernel, whose origin is local to a 4-row tile)
  if (!fs && !box_tile && sizeof(TS) == 4 && gauss_on_mfma(R, N, h, w)) {
    // strips of 16 columns; segment height a multiple of 16, chosen so the
    // grid has about two waves per SIMD (8 per CU)
    const int n_strips = (w + 15) / 16;
    const long long target = 4LL * device_cus();
    long long segs = (target + n_strips - 1) / n_strips;
    int TH = (int)(((h + segs - 1) / segs + 15) / 16 * 16);
    if (TH < 32) TH = 32;
    const int n_segs = (h + TH - 1) / TH;
    const int n_waves = n_strips * n_segs;
    dim3 grid((n_waves + kWaves - 1) / kWaves, b.n);
    hipLaunchKernelGGL((moments_gauss_mfma<N, TS>), grid, dim3(kWaves * kWave), 0, stream, img,
                       pitch, h, w, R, 1.0 / (2.0 * s * s), alpha, beta, sp, mom, plane, TH,
                       n_strips, n_segs, cond_max, b);
    return hipGetLastError();
  }
  const int tx = gauss_tile_tx(R, N);
  if (tx > 0) {
    dim3 tg((w + tx - 1) / tx, (h + kTY - 1) / kTY, b.n);
    // 1/(2 sigma_s^2); 0 makes every tap's weight exp(0) = 1 (box)
    const double i2 = box_tile ? 0.0 : 1.0 / (2.0 * s * s);
    // LDS row stride: kESNarrow when the padded tile fits, else 256
    // (tx + 2R <= 256 by the choice of tx)
    const bool narrow = tx + 2 * R <= kESNarrow;
    const int es = narrow ? kESNarrow : 256;
    // power sums, then (bounds) the (min, max) pairs
    const size_t lds = (size_t)(N * kTY * es + tile_wext_len(R)) * sizeof(double) +
                       (bounds ? (size_t)(kTY * es) * sizeof(float2) : 0);
#define ABF_TILE(F, S, B)                                                                       \
  hipLaunchKernelGGL((moments_gauss_tile<N, TS, F, S, B>), tg, dim3(256), lds, stream, img, pitch, \
                     h, w, R, tx, i2, alpha, beta, sp, mom, plane, cond_max, b, fz)
    if (fs && bounds) {
      if (narrow) ABF_TILE(true, kESNarrow, true); else ABF_TILE(true, 256, true);
    } else if (fs) {
      if (narrow) ABF_TILE(true, kESNarrow, false); else ABF_TILE(true, 256, false);
    } else if (bounds) {
      if (narrow) ABF_TILE(false, kESNarrow, true); else ABF_TILE(false, 256, true);
    } else {
      if (narrow) ABF_TILE(false, kESNarrow, false); else ABF_TILE(false, 256, false);
    }
#undef ABF_TILE
    return hipGetLastError();
  }
  // (the tile fits every radius up to ABF_RHO_MAX: tx >= 64 for N <= 8)
  return hipErrorInvalidValue;
}

template <typename TS>
hipError_t dispatch_n(int N, const float* img, long long pitch, int h, int w, int kind,
                      double sigma_s, int R, float* alpha, float* beta,
                      long long sp, TS* mom, long long plane, hipStream_t stream,
                      const Batch& b, const FuseSpec* fs, bool bounds) {
  switch (N) {
#define ABF_CASE(n) \
  case n: return launch_moments_t<n, TS>(img, pitch, h, w, kind, sigma_s, R, alpha, beta, sp, mom, plane, stream, b, fs, bounds);
    ABF_CASE(1) ABF_CASE(2) ABF_CASE(3) ABF_CASE(4) ABF_CASE(5) ABF_CASE(6) ABF_CASE(7) ABF_CASE(8)
#undef ABF_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_moments(const float* img, long long pitch, int h, int w,
                          int kernel_kind, double sigma_s, int rho, int N, int prec,
                          float* alpha, float* beta, long long sp,
                          void* mom, long long plane_elems, hipStream_t stream, const Batch& b,
                          const FuseSpec* fuse, bool bounds) {
  if (prec == 0)
    return dispatch_n<double>(N, img, pitch, h, w, kernel_kind, sigma_s, rho, alpha, beta, sp,
                              static_cast<double*>(mom), plane_elems, stream, b, fuse, bounds);
  return dispatch_n<float>(N, img, pitch, h, w, kernel_kind, sigma_s, rho, alpha, beta, sp,
                           static_cast<float*>(mom), plane_elems, stream, b, fuse, bounds);
}

bool moments_take_bounds(int kernel_kind, int rho, int N, long long h, long long w) {
  // the Gaussian tile kernel (its LDS, the power sums and the (min, max)
  // pairs, (N + 1) kTY ES 8 bytes, plus the weights, is at most 74 KiB, so
  // two workgroups still share a CU's 160 KiB, as without the pairs); the
  // box and matrix-core kernels read the bounds from the stack
  if (kernel_kind != 1 || N < 1 || N > 8 || gauss_on_mfma(rho, N, h, w)) return false;
  const int tx = gauss_tile_tx(rho, N);
  const int es = tx + 2 * rho <= kESNarrow ? kESNarrow : 256;
  return tx > 0 && ((N + 1) * kTY * es + tile_wext_len(rho)) * 8 + 64 <= 81920;
}

int stack_kernel_id(int kernel_kind, int rho, int N, int prec, long long h, long long w) {
  if (N < 1) return kStackBoundsOnly;
  // the FP64 box path at N >= 7 takes the tile kernel with unit weights
  const bool box_tile = kernel_kind == 0 && prec == 0 && N >= 7;
  if (kernel_kind == 0 && !box_tile) return kStackBox;
  if (!box_tile && prec == 1 && gauss_on_mfma(rho, N, h, w)) return kStackMfma;
  const int tx = gauss_tile_tx(rho, N);
  if (tx <= 0) return -1;
  return tx + 2 * rho <= kESNarrow ? kStackTile : kStackTileWide;
}

bool moments_fusable(int kernel_kind, int rho, int N, long long h, long long w) {
  // The fused variant has no matrix-core form; where abf_stack_moments uses
  // the matrix-core kernel the fused call takes the stack path, so that its
  // output stays identical to abf_stack_moments + abf_range.
  return N >= 1 && N <= 8 &&
         (kernel_kind == 0 || (!gauss_on_mfma(rho, N, h, w) && gauss_tile_tx(rho, N) > 0));
}

}  // namespace abf
