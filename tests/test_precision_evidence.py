"""Why the GPU path keeps the power sums and the integral recursion in FP64.

A tempting precision split for Algorithm 1 runs the convolution step (the
power images omega * f^k of Prop. 2) as FP32 running sums with Kahan
compensation on intensities rescaled to [0, 1], and the forward recursion
of eq. (F_forward) in FP32, keeping FP64 only for the binomial shift of
Prop. 3 and the Hilbert-inverse fit of eq. (inv). This module emulates that
split on the CPU, step by step in the paper's order (NumPy float32 where
the split says FP32), on a crop of the 4096 x 4096 Voronoi workload (256
cells, noise 15, sigma constant per 16 x 16 block, box kernel), and compares
it with the value-of-record oracle for N = 5..8 and rho in {5, 20}:

* with FP32 sums and the FP32 recursion the mixed tolerance of 0.05 on
  [0, 255] fails at every N >= 6 for both radii, and already at N = 5 for
  rho = 5 (both halves of the split fail it on their own);
* the same steps with FP64 sums and the FP64 recursion (and the same
  post-rules as the oracle) stay within 1e-3.

Each emulation applies the oracle's post-rules (T2 <= 0 or a non-finite
ratio falls back to I_1/I_0; the ratio is clipped to [0, 1]) so that only
the arithmetic differs.
"""
from math import comb

import numpy as np
import pytest
from scipy.special import erf

import oracle
from oracle.hilbert import hilbert_inverse
from oracle.spatial import convolve_powers, window_minmax
from synth import workload

F32 = np.float32
BAR = 0.05


@pytest.fixture(scope="module")
def crop():
    wl = workload("voronoi4096_box5_n5")
    ys, xs = slice(1000, 1096), slice(2000, 2096)       # several cells and their borders
    return wl["f"][ys, xs].copy(), wl["sigma"][ys, xs].copy()


def _kadd(s, c, x):
    """One Kahan-compensated FP32 addition of x into (sum s, compensation c)."""
    y = (x - c).astype(F32)
    t = (s + y).astype(F32)
    return t, ((t - s) - y).astype(F32)


def kahan_box_sums(plane, R):
    """Box window sums (clamp-to-edge) of an FP32 plane as FP32 running sums
    with Kahan compensation: down the columns (add the entering row, remove
    the leaving row), then along the rows."""
    H, W = plane.shape
    pad = np.pad(plane, R, mode="edge")
    s = np.zeros(W + 2 * R, F32)
    c = np.zeros_like(s)
    for r in range(2 * R + 1):
        s, c = _kadd(s, c, pad[r])
    V = np.empty((H, W + 2 * R), F32)
    V[0] = s
    for y in range(1, H):
        s, c = _kadd(s, c, pad[y + 2 * R])
        s, c = _kadd(s, c, -pad[y - 1])
        V[y] = s
    s = np.zeros(H, F32)
    c = np.zeros_like(s)
    for x in range(2 * R + 1):
        s, c = _kadd(s, c, V[:, x])
    out = np.empty((H, W), F32)
    out[:, 0] = s
    for x in range(1, W):
        s, c = _kadd(s, c, V[:, x + 2 * R])
        s, c = _kadd(s, c, -V[:, x - 1])
        out[:, x] = s
    return out


def integrals(lam, t0, K, dt):
    """I_0..I_K by eqs. (I_0), (I_1), (F_forward), every operation rounded
    to ``dt`` (the error functions themselves correctly rounded to dt)."""
    lam, t0 = lam.astype(dt), t0.astype(dt)
    e0 = np.exp(-lam * t0 * t0).astype(dt)
    e1 = np.exp(-lam * (dt(1) - t0) ** 2).astype(dt)
    sl = np.sqrt(lam).astype(dt)
    I = np.empty(lam.shape + (K + 1,), dt)
    erfs = erf((sl * (dt(1) - t0)).astype(np.float64)) + erf((sl * t0).astype(np.float64))
    I[..., 0] = (dt(0.5) * np.sqrt(dt(np.pi)) / sl * erfs.astype(dt)).astype(dt)
    i2l = (dt(1) / (dt(2) * lam)).astype(dt)
    I[..., 1] = (t0 * I[..., 0] + (e0 - e1) * i2l).astype(dt)
    for k in range(2, K + 1):
        I[..., k] = (t0 * I[..., k - 1] + dt(k - 1) * i2l * I[..., k - 2] - e1 * i2l).astype(dt)
    return I.astype(np.float64)


def split_filter(f, sg, R, N, fp32):
    """Algorithm 1 on [0, 1] intensities (Sec. III) with the power sums and
    the recursion in FP32 (fp32=True) or FP64; shift and fit in FP64."""
    H, W = f.shape
    u = f.astype(np.float64) / 255.0
    if fp32:
        u32 = (f.astype(F32) / F32(255)).astype(F32)
        area = F32((2 * R + 1) ** 2)
        m, p = [np.ones((H, W))], np.ones_like(u32)
        for _ in range(N):
            p = (p * u32).astype(F32)
            m.append((kahan_box_sums(p, R) / area).astype(F32).astype(np.float64))
    else:
        m = convolve_powers(u, "box", R, None, N)
    a, b = window_minmax(u, R)
    live = a != b
    d = np.where(live, b - a, 1.0)
    mu = np.empty((N + 1, H, W))
    for k in range(N + 1):                                   # Prop. 3, FP64
        acc = np.zeros((H, W))
        for r in range(k + 1):
            acc += comb(k, r) * (-a) ** (k - r) * m[r]
        mu[k] = acc / d ** k
    c = np.moveaxis(np.tensordot(np.array(hilbert_inverse(N), dtype=np.float64), mu, axes=1), 0, -1)
    t0 = (u - a) / d                                         # eq. (sub)
    lam = 0.5 * d * d / (sg.astype(np.float64) / 255.0) ** 2
    I = integrals(lam, t0, N + 1, F32 if fp32 else np.float64)
    T1 = np.sum(c * I[..., 1:], axis=-1)
    T2 = np.sum(c * I[..., :-1], axis=-1)
    with np.errstate(all="ignore"):
        F = T1 / T2
        F = np.where(~np.isfinite(F) | (T2 <= 0), I[..., 1] / I[..., 0], F)
    return np.where(live, 255.0 * (a + d * np.clip(F, 0.0, 1.0)), f.astype(np.float64))


@pytest.mark.parametrize("R", [5, 20])
@pytest.mark.parametrize("N", [5, 6, 7, 8])
def test_fp32_sums_and_recursion_fail_the_mixed_bar(crop, R, N):
    f, sg = crop
    ref = oracle.fast_abf(f, None, sg, "box", R, N)
    err32 = float(np.max(np.abs(split_filter(f, sg, R, N, fp32=True) - ref)))
    err64 = float(np.max(np.abs(split_filter(f, sg, R, N, fp32=False) - ref)))
    print(f"R={R} N={N}: FP32 sums + FP32 recursion {err32:.3g}, FP64 {err64:.3g}")
    assert err64 < 1e-3
    if N >= 6 or R == 5:
        assert err32 > BAR
