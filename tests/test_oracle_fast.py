"""Pins for the oracle's Algorithm 1 and brute force (closed forms,
invariants, 60-digit evaluation of the printed algorithm, convergence)."""
import math
import os

import numpy as np
import pytest

from oracle import brute_abf, fast_abf, fast_abf_literal
from oracle.integrals import I_quadrature
from oracle.mpref import fast_abf_mp
from oracle.spatial import gather_windows, spatial_weights, window_minmax
from synth import rect_scene, smooth_field

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed=5, h=9, w=11):
    f = rect_scene(seed, h, w, n_rect=3, noise=10, side_lo=3, side_hi=6)
    sg = smooth_field(np.random.default_rng(seed + 1), h, w, 10, 30)
    return f, sg


@pytest.mark.parametrize("N", [0, 1, 2, 4, 6, 8])
@pytest.mark.parametrize("kind,R", [("box", 1), ("gaussian", 2)])
def test_stable_route_matches_60_digit_algorithm1(N, kind, R):
    f, sg = _tiny()
    ref = fast_abf_mp(f, None, sg, kind, R, N)
    got = fast_abf(f, None, sg, kind, R, N, clamp=False)
    assert np.max(np.abs(got - ref)) < 1e-9


def test_stable_route_theta_offset_matches_60_digit():
    # sharpening-style theta = f + zeta puts t0 outside [0, 1]
    f, sg = _tiny(7)
    zeta = smooth_field(np.random.default_rng(2), *f.shape, -20, 20)
    th = (f + zeta).astype(np.float32)
    for N in (3, 6):
        ref = fast_abf_mp(f, th, sg, "box", 1, N)
        got = fast_abf(f, th, sg, "box", 1, N, clamp=False)
        ok = np.isfinite(ref)
        assert np.max(np.abs(got[ok] - ref[ok])) < 1e-9


def test_literal_route_agrees_at_low_degree():
    f, sg = _tiny(3, 16, 16)
    for N in (1, 3, 5):
        a = fast_abf_literal(f, None, sg, "box", 2, N)
        b = fast_abf(f, None, sg, "box", 2, N, clamp=False)
        assert np.max(np.abs(a - b)) < 1e-5


def test_constant_image_is_fixed():
    f = np.full((6, 7), 42.25, dtype=np.float32)
    g = fast_abf(f, None, np.full(f.shape, 20.0), "box", 2, 5)
    assert np.array_equal(g, f.astype(np.float64))


def test_flat_window_passthrough_and_range():
    f, sg = _tiny(11, 20, 20)
    f[:8, :8] = 77.0                       # a flat patch: alpha = beta inside it
    lo, hi = window_minmax(f, 2)
    g, aux = fast_abf(f, None, sg, "box", 2, 6, aux=True)
    flat = lo == hi
    assert flat.sum() > 0
    assert np.array_equal(g[flat], f[flat].astype(np.float64))
    assert np.all(g >= lo - 1e-9) and np.all(g <= hi + 1e-9)


def test_sigma_infinite_gives_spatial_mean():
    # lambda = 0: psi = 1, and moment matching of mu_1 makes the ratio the
    # window mean (any N >= 1).
    f, _ = _tiny(13)
    for kind, R in (("box", 1), ("gaussian", 2)):
        w = spatial_weights(kind, R).ravel()
        ys, xs = np.meshgrid(np.arange(f.shape[0]), np.arange(f.shape[1]), indexing="ij")
        mean = (gather_windows(f, R, ys.ravel(), xs.ravel()) @ w).reshape(f.shape)
        for N in (1, 4, 8):
            g = fast_abf(f, None, np.full(f.shape, np.inf), kind, R, N)
            assert np.max(np.abs(g - mean)) < 1e-9
        gb = brute_abf(f, None, np.full(f.shape, np.inf), kind, R)
        assert np.max(np.abs(gb - mean)) < 1e-9


def test_degree_zero_is_I1_over_I0():
    # N = 0: p is a constant, so g^ = alpha + (beta-alpha) I_1/I_0 whatever the
    # histogram (Sec. III discussion of the N = 0 case).
    f, sg = _tiny(17)
    g, aux = fast_abf(f, None, sg, "box", 1, 0, aux=True)
    live = aux["alpha"] != aux["beta"]
    I, _ = I_quadrature(aux["lam"][live], aux["t0"][live], 1)
    expect = aux["alpha"][live] + (aux["beta"] - aux["alpha"])[live] * np.clip(I[:, 1] / I[:, 0], 0, 1)
    assert np.max(np.abs(g[live] - expect)) < 1e-10


def test_affine_equivariance():
    f, sg = _tiny(19)
    f = (np.round(f * 8) / 8).astype(np.float32)   # dyadic, so 2f+3 is exact in FP32
    g = fast_abf(f, None, sg, "box", 1, 5)
    g2 = fast_abf((2 * f + 3).astype(np.float32), None, 2 * sg, "box", 1, 5)
    assert np.max(np.abs(g2 - (2 * g + 3))) < 1e-9
    gneg = fast_abf((-f).astype(np.float32), None, sg, "box", 1, 5)
    assert np.max(np.abs(gneg + g)) < 1e-9


def test_converges_to_brute_force():
    f, sg = _tiny(23, 14, 14)
    gb = brute_abf(f, None, sg, "box", 2)
    errs = [np.max(np.abs(fast_abf(f, None, sg, "box", 2, N) - gb)) for N in range(0, 13, 2)]
    assert errs[-1] < 0.05 * errs[0]
    assert all(b <= a * 1.05 for a, b in zip(errs, errs[1:]))


def test_psnr_trend_rises_with_degree():
    # Table 1 (parity unpinned: the paper's image is not available); only the
    # trend is checked on a synthetic scene: PSNR vs brute force rises with N.
    f = rect_scene(31, 48, 48, n_rect=6, noise=10, side_lo=6, side_hi=24)
    sg = np.full(f.shape, 40.0)
    gb = brute_abf(f, None, sg, "box", 3)
    psnr = []
    for N in range(0, 7):
        mse = np.mean((fast_abf(f, None, sg, "box", 3, N) - gb) ** 2)
        psnr.append(10 * math.log10(255 ** 2 / mse))
    assert all(b > a for a, b in zip(psnr, psnr[1:]))


def _golden(name):
    vals = {}
    for line in open(os.path.join(GOLD, name)):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_brute_force_hand_example():
    f = np.zeros((3, 3), dtype=np.float32)
    f[1, 1] = 10
    g = brute_abf(f, None, np.full((3, 3), 10.0), "box", 1)
    gold = _golden("brute_3x3.txt")
    assert abs(g[1, 1] - gold["centre"]) < 1e-13
    assert abs(g[0, 0] - gold["corner"]) < 1e-13


def test_brute_force_small_sigma_returns_centre():
    f, _ = _tiny(29)
    g = brute_abf(f, None, np.full(f.shape, 1e-3), "box", 1)
    # with theta = f the centre pixel dominates as sigma -> 0 unless a
    # neighbour has exactly the same value (then the two average; same value)
    assert np.max(np.abs(g - f)) < 1e-6


def test_sampled_pixels_equal_full_evaluation():
    f, sg = _tiny(37, 12, 13)
    full = fast_abf(f, None, sg, "gaussian", 2, 6)
    ys = np.array([0, 3, 11, 5])
    xs = np.array([0, 12, 7, 5])
    part = fast_abf(f, None, sg, "gaussian", 2, 6, pixels=(ys, xs))
    assert np.array_equal(part, full[ys, xs])
