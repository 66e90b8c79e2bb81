"""Brute-force adaptive bilateral filter, eqs. (BF_adaptive1), (BF_adaptive2):

    g(i) = sum_j omega(j) phi_i(f(i-j) - theta(i)) f(i-j) / eta(i),
    eta(i) = sum_j omega(j) phi_i(f(i-j) - theta(i)),
    phi_i(t) = exp(-t^2 / (2 sigma(i)^2))            (eq. r_kernel),

over the clamp-to-edge window [-R, R]^2 with the normalised spatial weights
of ``spatial.spatial_weights``. FP64. Every exponent of a window is shifted
by the window's smallest exponent before exponentiation; the common factor
cancels in the ratio and keeps the largest range weight at exactly 1, so
the ratio is defined for every sigma > 0. sigma = +inf gives the spatial
mean.
"""
from __future__ import annotations

import numpy as np

from .spatial import canon, gather_windows, spatial_weights


def brute_abf(f, theta=None, sigma=None, kernel: str = "box", R: int = 3,
              sigma_s: float | None = None, pixels=None, chunk: int = 8192):
    f = canon(np.asarray(f, dtype=np.float32))
    H, W = f.shape
    th = f if theta is None else canon(np.asarray(theta, dtype=np.float32))
    sg = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (H, W))
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
    else:
        ys, xs = np.asarray(pixels[0]), np.asarray(pixels[1])
    w = spatial_weights(kernel, R, sigma_s).ravel()
    f64 = f.astype(np.float64)
    out = np.empty(len(ys))
    step = max(1, min(chunk, (1 << 24) // ((2 * R + 1) ** 2)))
    for s0 in range(0, len(ys), step):
        sl = slice(s0, min(len(ys), s0 + step))
        win = gather_windows(f64, R, ys[sl], xs[sl])
        t = th[ys[sl], xs[sl]].astype(np.float64)[:, None]
        s = sg[ys[sl], xs[sl]][:, None]
        with np.errstate(divide="ignore", invalid="ignore"):
            e = (win - t) ** 2 / (2.0 * s * s)
        e = np.where(np.isfinite(s), e, 0.0)
        e = e - e.min(axis=1, keepdims=True)
        wt = w[None, :] * np.exp(-e)
        out[sl] = np.sum(wt * win, axis=1) / np.sum(wt, axis=1)
    return out.reshape(H, W) if pixels is None else out
