"""Pins of the recursive approximation of the Gaussian spatial kernel
(oracle/recursive.py; Sec. II-D's O(1) option for the convolutions of
Algorithm 1, with Deriche's fourth-order sum of damped complex exponentials
truncated to the window):

* the weights are those of a Gaussian of the same sigma_s to within the
  approximation's own accuracy (Deriche's profile is within 1e-3 of
  exp(-t^2/2) on [0, 6]);
* the truncated recursions equal direct correlation with those weights
  (clamp-to-edge borders), for radii from 0 to beyond the row length;
* the 2-D power sums by the recursion equal convolve_powers with the kernel
  (the value of record's definition, Prop. 2);
* the route a recursive GPU pass takes -- power sums about one origin for
  the whole image, then the binomial shift of Prop. 3 to every window --
  stays within the FP64 bar on the workloads' content at wide radii (the
  conditioning worry that one origin is far from narrow windows costs at
  most rho^N ~ 2e8 here, times FP64 rounding).
"""
from math import comb

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg
from scipy.ndimage import correlate1d

import oracle
from oracle.integrals import J_quadrature
from oracle.recursive import (deriche_profile, deriche_weights_1d, recursive_filter_1d,
                              recursive_power_sums)
from oracle.spatial import canon, convolve_powers, spatial_weights_1d, window_minmax
from synth import rect_scene, smooth_field, workload


def test_profile_is_deriches_gaussian():
    t = np.linspace(0.0, 6.0, 6001)
    g = deriche_profile(t, 1.0)
    assert abs(g[0] - 0.9997) < 1e-12                 # a0 + c0
    assert np.max(np.abs(g / g[0] - np.exp(-t * t / 2))) < 1e-3


@pytest.mark.parametrize("R,s", [(1, None), (5, None), (15, 5.0), (30, None), (60, 12.0)])
def test_weights_close_to_gaussian(R, s):
    w = deriche_weights_1d(R, s)
    g = spatial_weights_1d("gaussian", R, s)
    assert w.shape == (2 * R + 1,) and abs(w.sum() - 1.0) < 1e-14
    assert np.allclose(w, w[::-1], rtol=0, atol=1e-17)
    assert np.max(np.abs(w - g)) < 1e-3 * g.max()
    assert np.array_equal(spatial_weights_1d("recursive", R, s), w)


@pytest.mark.parametrize("R", [0, 1, 3, 8, 40, 90])
def test_recursion_equals_direct_correlation(R):
    rng = np.random.default_rng(R)
    u = rng.random((4, 53)) * 255.0
    for axis in (0, 1):
        ref = correlate1d(u, deriche_weights_1d(R), axis=axis, mode="nearest")
        got = recursive_filter_1d(u, R, None, axis=axis)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_power_sums_equal_convolution():
    rng = np.random.default_rng(7)
    f = rng.random((29, 37)) * 255.0
    R, s, N, c = 6, 2.5, 5, 100.0
    rec = recursive_power_sums(f, R, s, N, c)
    ref = convolve_powers(f - c, "recursive", R, s, N)
    for k in range(N + 1):
        assert np.max(np.abs(rec[k] - ref[k])) <= 1e-11 * np.max(np.abs(ref[k]))


def _shifted_route(f, sg, R, N, origin):
    """Algorithm 1 with the power sums of one origin from the recursion, the
    shift of Prop. 3 per window, Legendre moments and the value of record's
    range integrals; post-rules as the oracle."""
    f64 = canon(np.asarray(f, np.float32)).astype(np.float64)
    m = recursive_power_sums(f64, R, None, N, origin)
    a, b = window_minmax(f64, R)
    live = a != b
    mid, half = 0.5 * (a + b), np.where(live, 0.5 * (b - a), 1.0)
    nu = np.zeros((N + 1,) + f64.shape)
    for k in range(N + 1):
        for r in range(k + 1):
            nu[k] += comb(k, r) * (origin - mid) ** (k - r) * m[r]
        nu[k] /= half ** k
    L = np.zeros((N + 1, N + 1))
    for k in range(N + 1):
        e = np.zeros(k + 1)
        e[k] = 1.0
        L[k, :k + 1] = npleg.leg2poly(e)
    am = np.tensordot(L, nu, axes=1)
    coef = np.moveaxis(am, 0, -1) * (2 * np.arange(N + 1) + 1)
    t0 = (f64 - a) / np.where(live, b - a, 1.0)
    lam = (b - a) ** 2 / (2.0 * sg.astype(np.float64) ** 2)
    idx = np.nonzero(live)
    J, Jt, _ = J_quadrature(lam[idx], t0[idx], N)
    T2, T1 = np.sum(coef[idx] * J, axis=1), np.sum(coef[idx] * Jt, axis=1)
    with np.errstate(all="ignore"):
        F = T1 / T2
    F = np.where(~np.isfinite(F) | (T2 <= 0), Jt[:, 0] / J[:, 0], F)
    out = f64.copy()
    out[idx] = a[idx] + (b - a)[idx] * np.clip(F, 0.0, 1.0)
    return out


@pytest.mark.parametrize("case", ["voronoi", "rects"])
def test_one_origin_route_meets_fp64_bar(case):
    if case == "voronoi":
        wl = workload("voronoi4096_box5_n5")
        f, sg = wl["f"][1000:1080, 2000:2080], wl["sigma"][1000:1080, 2000:2080]
    else:
        f = rect_scene(77, 80, 80, n_rect=8, noise=2.0, side_lo=12, side_hi=60)
        sg = smooth_field(np.random.default_rng(3), 80, 80, 10, 30)
    R, N = 25, 6
    origin = 0.5 * (float(f.min()) + float(f.max()))
    ref = oracle.fast_abf(f, None, sg, "recursive", R, N)
    err = np.max(np.abs(_shifted_route(f, sg, R, N, origin) - ref))
    assert err < 1e-6, err
