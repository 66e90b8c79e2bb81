"""Pins for the spatial-stage definitions: bounds, weights, moments, shift."""
from fractions import Fraction
from math import comb

import numpy as np
import pytest

from oracle.spatial import (convolve_powers, gather_windows, legendre_moments,
                            spatial_weights, spatial_weights_1d,
                            stretched_moments, window_minmax)
from oracle.hilbert import shifted_legendre


def _naive_minmax(f, R):
    H, W = f.shape
    lo = np.empty_like(f)
    hi = np.empty_like(f)
    for i in range(H):
        for j in range(W):
            vals = [f[min(H - 1, max(0, i + a)), min(W - 1, max(0, j + b))]
                    for a in range(-R, R + 1) for b in range(-R, R + 1)]
            lo[i, j], hi[i, j] = min(vals), max(vals)
    return lo, hi


@pytest.mark.parametrize("shape,R", [((7, 9), 0), ((7, 9), 1), ((6, 5), 2), ((5, 11), 4), ((3, 4), 6), ((1, 8), 2), ((9, 1), 3)])
def test_window_minmax_matches_loops(shape, R):
    rng = np.random.default_rng(R * 31 + shape[0])
    f = rng.integers(0, 20, size=shape).astype(np.float32) * np.float32(3.5)
    lo, hi = window_minmax(f, R)
    nlo, nhi = _naive_minmax(f, R)
    assert np.array_equal(lo, nlo) and np.array_equal(hi, nhi)


def test_window_minmax_negative_zero():
    f = np.array([[0.0, -0.0, 1.0]], dtype=np.float32)
    lo, hi = window_minmax(f, 1)
    assert not np.any(np.signbit(lo))


@pytest.mark.parametrize("kind", ["box", "gaussian"])
def test_weights_normalised_and_symmetric(kind):
    for R in (0, 1, 3, 15):
        w = spatial_weights(kind, R, 5.0)
        assert abs(w.sum() - 1) < 1e-14
        assert np.allclose(w, w[::-1, ::-1]) and np.allclose(w, w.T)
    w1 = spatial_weights_1d("gaussian", 6, 2.0)
    assert np.isclose(w1[6 + 2] / w1[6], np.exp(-4 / 8.0), rtol=1e-14)
    assert np.isclose(spatial_weights_1d("gaussian", 6)[6 + 2] / spatial_weights_1d("gaussian", 6)[6],
                      np.exp(-4 / 8.0), rtol=1e-14)  # default sigma_s = R/3 = 2


@pytest.mark.parametrize("kind,R", [("box", 1), ("box", 3), ("gaussian", 2)])
def test_prop2_convolution_equals_window_sums(kind, R):
    # Prop. 2: sum_t t^k h_i(t) = (omega * f^k)(i)
    rng = np.random.default_rng(5)
    u = rng.random((9, 8))
    N = 4
    gam = convolve_powers(u, kind, R, None, N)
    ys, xs = np.meshgrid(np.arange(9), np.arange(8), indexing="ij")
    win = gather_windows(u, R, ys.ravel(), xs.ravel())
    w = spatial_weights(kind, R).ravel()
    for k in range(N + 1):
        direct = (win ** k) @ w
        assert np.allclose(gam[k].ravel(), direct, rtol=1e-13, atol=1e-15)


def test_prop3_shift_exact_in_rationals():
    # Prop. 3: mu_k = (beta-alpha)^-k sum_r C(k,r) (-alpha)^(k-r) m_r
    rng = np.random.default_rng(9)
    for trial in range(20):
        n = int(rng.integers(2, 12))
        vals = [Fraction(int(v), 7) for v in rng.integers(-50, 300, size=n)]
        if min(vals) == max(vals):
            continue
        wts = [Fraction(int(v)) for v in rng.integers(1, 9, size=n)]
        a, b = min(vals), max(vals)
        for k in range(9):
            m = [sum(wj * v ** r for wj, v in zip(wts, vals)) for r in range(k + 1)]
            shifted = sum(comb(k, r) * (-a) ** (k - r) * m[r] for r in range(k + 1)) / (b - a) ** k
            direct = sum(wj * ((v - a) / (b - a)) ** k for wj, v in zip(wts, vals))
            assert shifted == direct


def test_legendre_moments_equal_ell_times_mu():
    rng = np.random.default_rng(11)
    win = rng.random((50, 25)) * 255
    w = spatial_weights("box", 2).ravel()
    a, b = win.min(1), win.max(1)
    N = 8
    mu = stretched_moments(win, w, a, b, N)
    am = legendre_moments(win, w, a, b, N)
    ell = np.array(shifted_legendre(N), dtype=float)
    assert np.allclose(am, mu @ ell.T, atol=1e-9)
    assert np.allclose(am[:, 0], 1.0, atol=1e-15)
    assert np.all(np.abs(am) <= 1 + 1e-12)      # |P_k| <= 1 on [-1, 1]


def test_local_std_sigma_matches_library_filter():
    from scipy.ndimage import generic_filter
    from oracle.spatial import local_std_sigma
    rng = np.random.default_rng(3)
    f = (rng.random((13, 17)) * 120).astype(np.float32)
    for r in (0, 1, 4):
        ref = np.clip(3.0 * generic_filter(f.astype(np.float64), np.std, size=2 * r + 1, mode="nearest"), 5, 80)
        assert np.allclose(local_std_sigma(f, r), ref, rtol=1e-12, atol=1e-12)
