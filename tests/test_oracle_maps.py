"""Pins for the application parameter maps (oracle/maps.py) against SciPy's
own filters, which implement the same definitions independently."""
import numpy as np
import pytest
from scipy import ndimage as ndi

from oracle import maps
from synth import rect_scene


@pytest.fixture(scope="module")
def img():
    return rect_scene(5, 37, 53, n_rect=5, noise=8, side_lo=5, side_hi=25)


def test_box_mean(img):
    for r in (0, 1, 3):
        ref = ndi.uniform_filter(img.astype(np.float64), 2 * r + 1, mode="nearest")
        assert np.max(np.abs(maps.box_mean(img, r) - ref)) < 1e-10


@pytest.mark.parametrize("s", [0.7, 1.0, 2.0])
def test_laplacian_of_gaussian_matches_scipy(img, s):
    ref = ndi.gaussian_laplace(img.astype(np.float64), s, mode="nearest")
    assert np.max(np.abs(maps.laplacian_of_gaussian(img, s) - ref)) < 1e-9


def test_log_of_quadratic_is_nearly_constant():
    # away from the border the LoG of (x^2 + y^2)/10 is 0.4 for the
    # continuous kernel; the sampled one misses by its moment errors
    # (sum d2 = -7e-5, sum d2 x^2 = 1.998 at s = 1), i.e. by < 5e-3 here
    y, x = np.mgrid[0:40, 0:40].astype(np.float64)
    q = ((x - 20) ** 2 + (y - 20) ** 2) / 10.0
    L = maps.laplacian_of_gaussian(q.astype(np.float32), 1.0)
    assert np.max(np.abs(L[8:-8, 8:-8] - 0.4)) < 5e-3


def test_gradient_norm(img):
    a = img.astype(np.float64)
    gx = ndi.correlate1d(a, [-0.5, 0.0, 0.5], axis=1, mode="nearest")
    gy = ndi.correlate1d(a, [-0.5, 0.0, 0.5], axis=0, mode="nearest")
    assert np.max(np.abs(maps.gradient_norm(img) - np.hypot(gx, gy))) < 1e-10


@pytest.mark.parametrize("r", [1, 2, 4])
def test_mrtv_matches_library_window_filters(img, r):
    a = img.astype(np.float64)
    g = maps.gradient_norm(img)
    k = 2 * r + 1
    delta = ndi.maximum_filter(a, k, mode="nearest") - ndi.minimum_filter(a, k, mode="nearest")
    ref = delta * ndi.maximum_filter(g, k, mode="nearest") / (
        ndi.uniform_filter(g, k, mode="nearest") * k * k + 0.5)
    assert np.allclose(maps.mrtv(img, r, 0.5), ref, rtol=1e-12, atol=1e-12)


def test_mrtv_of_step_edge_and_flat():
    # a single step edge: inside the window the gradient is concentrated at
    # the edge, so max/sum is large and mRTV ~ Delta * max/sum; a flat image
    # has Delta = 0
    f = np.zeros((20, 20), np.float32)
    f[:, 10:] = 100
    m = maps.mrtv(f, 2, 1e-3)
    assert np.all(maps.mrtv(np.full((8, 8), 3, np.float32), 2, 1e-3) == 0)
    # at the edge column the window holds two gradient columns of 50 each
    # along 5 rows: max 50, sum 500 -> mRTV = 100 * 50 / 500 = 10
    assert abs(m[10, 9] - 100 * 50 / (500 + 1e-3)) < 1e-9


def test_affine_sigma_and_sharpen_theta(img):
    v = np.array([0.0, 5.0, 10.0, 50.0])
    assert np.allclose(maps.affine_sigma(v, 5, 45, 10), [45, 25, 5, 5])
    th, sg = maps.sharpen_maps(img, 2, 1.0, 5, 45, 20)
    assert np.allclose(th, 2 * img.astype(np.float64) - maps.box_mean(img, 2))
    assert sg.min() >= 5 and sg.max() <= 45


def test_grey():
    c = np.random.default_rng(0).uniform(0, 255, (3, 4, 5)).astype(np.float32)
    assert np.allclose(maps.grey(c), 0.299 * c[0] + 0.587 * c[1] + 0.114 * c[2], rtol=1e-6)
