"""Parameter maps of the applications in Sec. IV (TEST INFRASTRUCTURE ONLY:
used by tests/, __graft_entry__.smoke() and bench.py's CPU baseline, never by
the product path).

Sharpening and noise removal (Sec. IV-A): theta = f + zeta with
zeta = f - fbar, fbar the average intensity over the Omega-neighbourhood,
and sigma from an affine map of |LoG * f| that sends low values to high
sigma. Texture filtering (Sec. IV-C): sigma from an affine map of

    mRTV(i) = Delta(i) max_{j in W_i} |grad f(j)| / (sum_{j in W_i} |grad f(j)| + eps),
    Delta(i) = max_{j in W_i} f(j) - min_{j in W_i} f(j),

high sigma where mRTV is low, computed on a grey version of a colour image.
The paper leaves the constants open; the readings taken here (and in the
GPU kernels) are:

  fbar          unweighted mean over the (2r+1)^2 window, clamp-to-edge
  LoG           sum over the two axes of the second derivative of a sampled
                Gaussian of std s along one axis and the sampled Gaussian
                along the other, both on [-q, q], q = round(4 s), the
                Gaussian normalised to sum 1, the derivative kernel
                (x^2/s^4 - 1/s^2) g(x); clamp-to-edge
  grad f        central differences (f(x+1) - f(x-1)) / 2 per axis on the
                clamp-to-edge image; |grad f| its Euclidean norm
  W_i           the (2r+1)^2 clamp-to-edge window
  affine map    sigma = hi - (hi - lo) min(v / v_ref, 1): sigma = hi at
                v = 0, falling linearly to lo at v >= v_ref
  grey          0.299 R + 0.587 G + 0.114 B
"""
from __future__ import annotations

import numpy as np

from .spatial import canon, padded


def _window_reduce(a: np.ndarray, r: int, op) -> np.ndarray:
    """op over the (2r+1)^2 clamp-to-edge window of each pixel (loops over
    the window offsets; plain and slow)."""
    H, W = a.shape
    p = padded(a, r)
    out = None
    for dy in range(2 * r + 1):
        for dx in range(2 * r + 1):
            v = p[dy:dy + H, dx:dx + W]
            out = v.copy() if out is None else op(out, v)
    return out


def box_mean(f: np.ndarray, r: int) -> np.ndarray:
    """fbar: unweighted mean of f over the (2r+1)^2 window (FP64)."""
    a = canon(np.asarray(f, np.float32)).astype(np.float64)
    return _window_reduce(a, r, np.add) / float((2 * r + 1) ** 2)


def affine_sigma(v: np.ndarray, lo: float, hi: float, v_ref: float) -> np.ndarray:
    """hi at v = 0, falling linearly to lo at v >= v_ref."""
    return hi - (hi - lo) * np.minimum(np.asarray(v, np.float64) / v_ref, 1.0)


def log_kernels(s: float):
    """The sampled Gaussian g (sum 1) and its second derivative
    d2 = (x^2/s^4 - 1/s^2) g on [-q, q], q = round(4 s)."""
    q = int(4.0 * s + 0.5)
    x = np.arange(-q, q + 1, dtype=np.float64)
    g = np.exp(-0.5 * x * x / (s * s))
    g /= g.sum()
    d2 = (x * x / s ** 4 - 1.0 / (s * s)) * g
    return g, d2, q


def laplacian_of_gaussian(f: np.ndarray, s: float) -> np.ndarray:
    """LoG * f by the separable sum (d2 along y, g along x) + (g along y,
    d2 along x), clamp-to-edge, FP64, each tap written out."""
    a = canon(np.asarray(f, np.float32)).astype(np.float64)
    H, W = a.shape
    g, d2, q = log_kernels(s)
    p = padded(a, q)
    out = np.zeros((H, W))
    for dy in range(2 * q + 1):
        for dx in range(2 * q + 1):
            out += (d2[dy] * g[dx] + g[dy] * d2[dx]) * p[dy:dy + H, dx:dx + W]
    return out


def sharpen_maps(f: np.ndarray, r: int, s_log: float, lo: float, hi: float, v_ref: float):
    """(theta, sigma) of the sharpening application: theta = 2 f - fbar,
    sigma = affine_sigma(|LoG * f|)."""
    a = canon(np.asarray(f, np.float32)).astype(np.float64)
    theta = 2.0 * a - box_mean(f, r)
    sigma = affine_sigma(np.abs(laplacian_of_gaussian(f, s_log)), lo, hi, v_ref)
    return theta, sigma


def gradient_norm(f: np.ndarray) -> np.ndarray:
    """|grad f| from central differences on the clamp-to-edge image."""
    a = canon(np.asarray(f, np.float32)).astype(np.float64)
    p = padded(a, 1)
    H, W = a.shape
    gx = 0.5 * (p[1:H + 1, 2:W + 2] - p[1:H + 1, 0:W])
    gy = 0.5 * (p[2:H + 2, 1:W + 1] - p[0:H, 1:W + 1])
    return np.sqrt(gx * gx + gy * gy)


def mrtv(f: np.ndarray, r: int, eps: float) -> np.ndarray:
    """mRTV over the (2r+1)^2 window (module docstring)."""
    a = canon(np.asarray(f, np.float32)).astype(np.float64)
    gn = gradient_norm(f)
    delta = _window_reduce(a, r, np.maximum) - _window_reduce(a, r, np.minimum)
    return delta * _window_reduce(gn, r, np.maximum) / (_window_reduce(gn, r, np.add) + eps)


def mrtv_sigma(f: np.ndarray, r: int, eps: float, lo: float, hi: float, v_ref: float):
    """sigma of the texture application: affine_sigma(mRTV)."""
    return affine_sigma(mrtv(f, r, eps), lo, hi, v_ref)


def grey(rgb: np.ndarray) -> np.ndarray:
    """0.299 R + 0.587 G + 0.114 B of a (3, H, W) image, in FP32 as the
    kernels see it."""
    c = np.asarray(rgb, np.float32)
    return (np.float32(0.299) * c[0] + np.float32(0.587) * c[1] + np.float32(0.114) * c[2]).astype(np.float32)
