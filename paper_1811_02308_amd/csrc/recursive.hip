// Moment stack for the recursive approximation of the Gaussian spatial
// kernel (ABF_KERNEL_RECURSIVE): the convolutions of Algorithm 1 (Prop. 2)
// by first-order recursions whose cost does not depend on the radius, then
// the shift and Legendre change shared with the other moment kernels.
#include <cmath>
#include <complex>

#include "abf_internal.h"
#include "moments_common.h"

namespace abf {
namespace {

// ------------------------------------------------------------ recursive kernel
// Moments for the recursive approximation of the Gaussian (Sec. II-D names
// recursive filters, Deriche's and Young and van Vliet's, as a way to make the
// convolutions of Algorithm 1 cost O(1) per pixel for any width): Deriche's
// fourth-order sum of two damped complex exponentials, g(t) = Re sum_m A_m
// z_m^|t| (constants in rec_const), taken on the window j in [-R, R] only,
// so that every weight lies inside the (2R+1)^2 window of alpha_i, beta_i.
// Per axis, sum_{|j|<=R} g(j) u(x-j) = Re sum_m A_m (q_m(x) + z_m p_m(x)),
//   causal     q_m(x) = z_m q_m(x-1) + u(x)   - z_m^(R+1) u(x-R-1),
//   anticausal p_m(x) = z_m p_m(x+1) + u(x+1) - z_m^R     u(x+R+1),
// the last term removing the sample that leaves the truncated window: O(1)
// per sample and power. The power sums are taken about one origin c for the
// image (rec_prep: the mid-range of sampled inputs), since a pass runs along
// whole rows and columns. rec_rows (a lane per row, a wave per row segment)
// writes the horizontal sums of (f - c)^k, k = 1..N, as FP64 planes Hk;
// rec_cols (a lane per column, a wave per column segment) runs the causal
// vertical recursion down the segment into FP64 planes Ck, then the
// anticausal one back up, adds the two halves and finishes each pixel with the
// shift and Legendre change of the other kernels (ill-conditioned pixels,
// where one origin for the image is far from a narrow window, are recomputed
// directly from their window with the kernel's weights). A segment starts R
// samples early (and the anticausal pass R samples late) from a zero state,
// so every output is the exact truncated sum, whatever the segment length.
struct RecConst {
  double zr[2], zi[2];     // poles z_m
  double ar[2], ai[2];     // A_m
  double bzr[2], bzi[2];   // A_m z_m (anticausal output)
  double z1r[2], z1i[2];   // z_m^(R+1)
  double zRr[2], zRi[2];   // z_m^R
  double inv_norm2;        // 1 / (sum_{|j|<=R} g(j))^2 (both axes)
};

// The kernel's normalised 1-D weights g(j) / sum g, j = -R..R, by value.
struct RecWeights {
  double v[2 * kRhoMax + 1];
};

// mid-range of the input on a 64 x 64 grid of samples -> c[0]; the kernel's
// normalised 1-D weights (for the exact recompute) -> wts[0 .. 2R].
__global__ __launch_bounds__(256) void rec_prep(const float* __restrict__ img, long long pitch,
                                                int H, int W, int R, RecWeights w_host,
                                                double* __restrict__ c, double* __restrict__ wts) {
  __shared__ float smin[256], smax[256];
  const FinMinMax fm;
  float lo = INFINITY, hi = -INFINITY;
  for (int i = threadIdx.x; i < 64 * 64; i += 256) {
    const int yy = (int)(((long long)(i >> 6) * (H - 1)) / 63);
    const int xx = (int)(((long long)(i & 63) * (W - 1)) / 63);
    const float v = img[(long long)yy * pitch + xx] + 0.0f;
    lo = fm.min(lo, v);
    hi = fm.max(hi, v);
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = fm.min(smin[threadIdx.x], smin[threadIdx.x + s]);
      smax[threadIdx.x] = fm.max(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) c[0] = 0.5 * ((double)smin[0] + (double)smax[0]);
  for (int j = threadIdx.x; j <= 2 * R; j += 256) wts[j] = w_host.v[j];
}

// Outputs per row (column) segment: every segment pays R warm-up samples
// in each direction, shorter segments give more waves. Measured at 4096^2,
// N = 6: rows 256 (5-13% faster than 512 for R = 8..96, 128 and 64 no
// faster), columns 128 (2-9% faster than 256; 64 slower at R = 96).
int rec_segment(int R) { (void)R; return 256; }
int rec_col_segment(int R) { (void)R; return 128; }
constexpr size_t kRecWtsBytes = ((2 * kRhoMax + 1) * sizeof(double) + 255) / 256 * 256;

// Row pass: a wave takes 64 rows (a lane per row) of one row segment. The
// recursion runs along the row in each lane; the inputs and outputs go
// through LDS in chunks of kRecCW columns so that every global access is
// coalesced: the chunk's inputs (u at the entering and at the leaving
// column of each step) are loaded row-contiguous by the whole wave, and the
// chunk's N output planes are written (causal pass) or read, added to and
// written back (anticausal pass) row-contiguous likewise.
constexpr int kRecCW = 8;                  // columns per staged chunk
constexpr int kRecLS = kWave + 1;          // LDS stride of a staged column (conflict-free reads)

template <int N>
__global__ __launch_bounds__(kWave) void rec_rows(const float* __restrict__ img, long long pitch,
                                                  int H, int W, int R, int seg, RecConst k,
                                                  const double* __restrict__ cptr,
                                                  double* __restrict__ hp, long long plane) {
  __shared__ float tin[kRecCW * kRecLS], tout[kRecCW * kRecLS];
  __shared__ double tres[N * kRecCW * kRecLS];
  const int lane = threadIdx.x;
  const int yb = blockIdx.y * kWave;
  const int x0 = blockIdx.x * seg, x1 = min(W, x0 + seg);
  const double c = *cptr;
  // staging roles: element (row yb + sr + 8 q, column sc) for q = 0..7
  const int sc = lane % kRecCW, sr = lane / kRecCW;
  // the inputs of columns xs .. xs + kRecCW - 1 (clamped to the image) into t
  auto stage = [&](float* t, int xs) {
    const unsigned xb = (unsigned)min(max(xs + sc, 0), W - 1) * 4u;
#pragma unroll
    for (int q = 0; q < kWave / 8; ++q) {
      const int r = sr + 8 * q;
      const float* row = img + (long long)min(yb + r, H - 1) * pitch;
      t[sc * kRecLS + r] = at_byte(row, xb) + 0.0f;
    }
  };
  // the chunk's results: out-of-range rows and columns are not written
  auto flush = [&](int xs, bool add) {
    const int x = xs + sc;
#pragma unroll
    for (int q = 0; q < kWave / 8; ++q) {
      const int r = sr + 8 * q;
      if (x >= x0 && x < x1 && yb + r < H) {
        double* d = hp + (long long)(yb + r) * W + x;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const double v = tres[(i * kRecCW + sc) * kRecLS + r];
          d[i * plane] = add ? d[i * plane] + v : v;
        }
      }
    }
  };
  auto powers = [&](float f, double (&p)[N]) {
    const double u = (double)f - c;
    double q = u;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      p[i] = q;
      q *= u;
    }
  };
  double sr_[2][N], si_[2][N];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < N; ++i) sr_[m][i] = si_[m][i] = 0.0;
  // causal: x = x0 - R .. x1 - 1, chunk by chunk
  for (int xs = x0 - R; xs < x1; xs += kRecCW) {
    stage(tin, xs);
    stage(tout, xs - R - 1);
    wave_sync();
    for (int cc = 0; cc < kRecCW; ++cc) {
      const int x = xs + cc;
      double pin[N], pout[N];
      powers(tin[cc * kRecLS + lane], pin);
      const bool sub = x > x0;                  // u(x-R-1) was added
      powers(tout[cc * kRecLS + lane], pout);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double o = 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          double nr = fma(k.zr[m], sr_[m][i], fma(-k.zi[m], si_[m][i], pin[i]));
          double ni = fma(k.zr[m], si_[m][i], k.zi[m] * sr_[m][i]);
          if (sub) {
            nr = fma(-k.z1r[m], pout[i], nr);
            ni = fma(-k.z1i[m], pout[i], ni);
          }
          sr_[m][i] = nr;
          si_[m][i] = ni;
          o = fma(k.ar[m], nr, fma(-k.ai[m], ni, o));
        }
        tres[(i * kRecCW + cc) * kRecLS + lane] = o;
      }
    }
    wave_sync();
    flush(xs, false);
    wave_sync();
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < N; ++i) sr_[m][i] = si_[m][i] = 0.0;
  // anticausal: x = x1 + R - 2 .. x0, chunk by chunk from the right; the
  // chunk [xs, xs + kRecCW) runs its columns right to left. Its flushes add
  // to the causal pass's results, which other lanes stored: make those
  // stores complete and visible first.
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const int xtop = x1 + R - 2;
  for (int xe = xtop; xe >= x0; xe -= kRecCW) {
    const int xs = xe - kRecCW + 1;
    stage(tin, xs + 1);                         // u(x + 1)
    stage(tout, xs + R + 1);                    // u(x + R + 1)
    wave_sync();
    for (int cc = kRecCW - 1; cc >= 0; --cc) {
      const int x = xs + cc;
      double pin[N], pout[N];
      powers(tin[cc * kRecLS + lane], pin);
      const bool sub = x <= x1 - 2;             // u(x+R+1) was added
      powers(tout[cc * kRecLS + lane], pout);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double o = 0.0;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          double nr = fma(k.zr[m], sr_[m][i], fma(-k.zi[m], si_[m][i], pin[i]));
          double ni = fma(k.zr[m], si_[m][i], k.zi[m] * sr_[m][i]);
          if (sub) {
            nr = fma(-k.zRr[m], pout[i], nr);
            ni = fma(-k.zRi[m], pout[i], ni);
          }
          sr_[m][i] = nr;
          si_[m][i] = ni;
          o = fma(k.bzr[m], nr, fma(-k.bzi[m], ni, o));
        }
        tres[(i * kRecCW + cc) * kRecLS + lane] = o;
      }
    }
    wave_sync();
    flush(xs, true);
    wave_sync();
  }
}

template <int N, typename TS>
__global__ __launch_bounds__(kWave) void rec_cols(
    const float* __restrict__ img, long long pitch, int H, int W, int R, int seg, RecConst k,
    const double* __restrict__ cptr, const double* __restrict__ wts,
    const double* __restrict__ hp, double* __restrict__ cp, long long plane,
    const float* __restrict__ alpha, const float* __restrict__ beta, long long sp,
    TS* __restrict__ mom, long long mplane, double cond_max) {
  const int lane = threadIdx.x;
  const int x = blockIdx.x * kWave + lane;
  const bool live = x < W;
  const int xc = live ? x : W - 1;
  const int y0 = blockIdx.y * seg, y1 = min(H, y0 + seg);
  const double c = *cptr;
  auto hv = [&](int y, double (&v)[N]) {
    const double* p = hp + (long long)min(max(y, 0), H - 1) * W + xc;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i * plane];
  };
  double sr[2][N], si[2][N];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < N; ++i) sr[m][i] = si[m][i] = 0.0;
  for (int y = y0 - R; y < y1; ++y) {           // causal, down
    double vin[N], vout[N];
    hv(y, vin);
    const bool sub = y > y0;
    if (sub) hv(y - R - 1, vout);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double o = 0.0;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        double nr = fma(k.zr[m], sr[m][i], fma(-k.zi[m], si[m][i], vin[i]));
        double ni = fma(k.zr[m], si[m][i], k.zi[m] * sr[m][i]);
        if (sub) {
          nr = fma(-k.z1r[m], vout[i], nr);
          ni = fma(-k.z1i[m], vout[i], ni);
        }
        sr[m][i] = nr;
        si[m][i] = ni;
        o = fma(k.ar[m], nr, fma(-k.ai[m], ni, o));
      }
      if (y >= y0 && live) cp[(long long)i * plane + (long long)y * W + x] = o;
    }
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < N; ++i) sr[m][i] = si[m][i] = 0.0;
  for (int y = y1 + R - 2; y >= y0; --y) {      // anticausal, up, then each pixel
    double vin[N], vout[N];
    hv(y + 1, vin);
    const bool sub = y <= y1 - 2;
    if (sub) hv(y + R + 1, vout);
    double m_[N + 1];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double o = 0.0;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        double nr = fma(k.zr[m], sr[m][i], fma(-k.zi[m], si[m][i], vin[i]));
        double ni = fma(k.zr[m], si[m][i], k.zi[m] * sr[m][i]);
        if (sub) {
          nr = fma(-k.zRr[m], vout[i], nr);
          ni = fma(-k.zRi[m], vout[i], ni);
        }
        sr[m][i] = nr;
        si[m][i] = ni;
        o = fma(k.bzr[m], nr, fma(-k.bzi[m], ni, o));
      }
      m_[i + 1] = o;
    }
    if (y >= y1) continue;
    bool bad = false;
    float a = 0.f, b = 0.f;
    if (live) {
      const long long idx = (long long)y * sp + x;
      a = alpha[idx];
      b = beta[idx];
      m_[0] = 1.0;
#pragma unroll
      for (int i = 0; i < N; ++i)
        m_[i + 1] = (m_[i + 1] + cp[(long long)i * plane + (long long)y * W + x]) * k.inv_norm2;
      bad = legendre_from_moments<N>(m_, a, b, c, cond_max);
      if (!bad) finish_pixel<N, TS, false>(m_, a, b, y, x, idx, mom, mplane, FuseArgs{});
    }
    const unsigned long long mask = __ballot(live && bad);
    if (mask)
      recompute_flagged<N, TS, false>(mask, live && bad, y, x, a, b, img, pitch, H, W, R, wts, 1.0,
                                      mom, mplane, sp, lane, FuseArgs{});
  }
}

// Deriche's constants for the Gaussian (order 0), scaled by sigma_s: poles
// z_m = exp(-(b_m - i w_m) / s), weights A_m = a_m - i a'_m.
constexpr double kDerA[2] = {1.680, -0.6803}, kDerAp[2] = {3.735, -0.2598};
constexpr double kDerB[2] = {1.783, 1.723}, kDerW[2] = {0.6318, 1.997};

double rec_sigma(int R, double sigma_s) {
  const double s = sigma_s > 0 ? sigma_s : R / 3.0;
  return s > 0 ? s : 1.0;
}

void rec_setup(int R, double sigma_s, RecConst& k, RecWeights& wt) {
  const double s = rec_sigma(R, sigma_s);
  double norm = 0.0;
  for (int j = -R; j <= R; ++j) {
    double g = 0.0;
    for (int m = 0; m < 2; ++m) {
      const double t = std::fabs((double)j) / s;
      g += (kDerA[m] * std::cos(kDerW[m] * t) + kDerAp[m] * std::sin(kDerW[m] * t)) *
           std::exp(-kDerB[m] * t);
    }
    wt.v[j + R] = g;
    norm += g;
  }
  for (int j = 0; j <= 2 * R; ++j) wt.v[j] /= norm;
  for (int m = 0; m < 2; ++m) {
    const std::complex<double> z = std::exp(std::complex<double>(-kDerB[m], kDerW[m]) / s);
    const std::complex<double> A(kDerA[m], -kDerAp[m]);
    const std::complex<double> bz = A * z, z1 = std::pow(z, R + 1), zR = std::pow(z, R);
    k.zr[m] = z.real();
    k.zi[m] = z.imag();
    k.ar[m] = A.real();
    k.ai[m] = A.imag();
    k.bzr[m] = bz.real();
    k.bzi[m] = bz.imag();
    k.z1r[m] = z1.real();
    k.z1i[m] = z1.imag();
    k.zRr[m] = zR.real();
    k.zRi[m] = zR.imag();
  }
  k.inv_norm2 = 1.0 / (norm * norm);
}

template <int N, typename TS>
hipError_t launch_rec_t(const float* img, long long pitch, int h, int w, double sigma_s, int R,
                        const float* alpha, const float* beta, long long sp, TS* mom,
                        long long plane, void* scratch, hipStream_t stream) {
  RecConst k;
  RecWeights wt;
  rec_setup(R, sigma_s, k, wt);
  char* base = static_cast<char*>(scratch);
  double* c = reinterpret_cast<double*>(base);
  double* wts = reinterpret_cast<double*>(base + 256);
  double* hp = reinterpret_cast<double*>(base + 256 + kRecWtsBytes);
  double* cp = hp + (long long)N * h * w;
  const long long hplane = (long long)h * w;
  const double cond_max = sizeof(TS) == 4 ? 1e12 : fp64_cond_max(N);
  hipLaunchKernelGGL(rec_prep, dim3(1), dim3(256), 0, stream, img, pitch, h, w, R, wt, c, wts);
  const int seg = rec_segment(R), cseg = rec_col_segment(R);
  hipLaunchKernelGGL((rec_rows<N>), dim3((w + seg - 1) / seg, (h + kWave - 1) / kWave),
                     dim3(kWave), 0, stream, img, pitch, h, w, R, seg, k, c, hp, hplane);
  hipLaunchKernelGGL((rec_cols<N, TS>), dim3((w + kWave - 1) / kWave, (h + cseg - 1) / cseg),
                     dim3(kWave), 0, stream, img, pitch, h, w, R, cseg, k, c, wts, hp, cp, hplane,
                     alpha, beta, sp, mom, plane, cond_max);
  return hipGetLastError();
}

template <typename TS>
hipError_t dispatch_rec(int N, const float* img, long long pitch, int h, int w, double sigma_s,
                        int R, const float* alpha, const float* beta, long long sp, TS* mom,
                        long long plane, void* scratch, hipStream_t stream) {
  switch (N) {
#define ABF_CASE(n) \
  case n: return launch_rec_t<n, TS>(img, pitch, h, w, sigma_s, R, alpha, beta, sp, mom, plane, scratch, stream);
    ABF_CASE(1) ABF_CASE(2) ABF_CASE(3) ABF_CASE(4) ABF_CASE(5) ABF_CASE(6) ABF_CASE(7) ABF_CASE(8)
#undef ABF_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_recursive_moments(const float* img, long long pitch, int h, int w,
                                   double sigma_s, int rho, int N, int prec, const float* alpha,
                                   const float* beta, long long sp, void* mom,
                                   long long plane_elems, void* scratch, hipStream_t stream) {
  if (N < 1 || N > kNMax || rho < 0 || rho > kRhoMax) return hipErrorInvalidValue;
  if (prec == 0)
    return dispatch_rec<double>(N, img, pitch, h, w, sigma_s, rho, alpha, beta, sp,
                                static_cast<double*>(mom), plane_elems, scratch, stream);
  return dispatch_rec<float>(N, img, pitch, h, w, sigma_s, rho, alpha, beta, sp,
                             static_cast<float*>(mom), plane_elems, scratch, stream);
}

size_t recursive_scratch_bytes(int h, int w, int N) {
  return 256 + kRecWtsBytes + (size_t)2 * N * (size_t)h * (size_t)w * sizeof(double);
}

}  // namespace abf
