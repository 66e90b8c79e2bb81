"""The uniform-prior comparison variant (TEST INFRASTRUCTURE ONLY: imported by
tests/, __graft_entry__.smoke() and bench.py's CPU baseline, never by the
product path).

Sec. III-B compares Algorithm 1 with the earlier uniform-prior method for the
classical filter. With N = 0, Algorithm 1 fits a constant to the local
histogram on [alpha_i, beta_i]; the earlier method fits a constant on
[f(i), 2 fbar(i) - f(i)], fbar the smoothed image. The constant's height
cancels in eq. (BFfinal), so both reduce to

    g^(i) = lo + (hi - lo) I_1 / I_0,   t0 = (theta(i) - lo) / (hi - lo),
                                        lambda = (hi - lo)^2 / (2 sigma(i)^2),

with I_k of eq. (integrals) and [lo, hi] the respective interval. Readings
(listed in the design notes): fbar is the window mean under the filter's own
spatial kernel (same window, weights and clamp-to-edge border);
lo = min(f, 2 fbar - f), hi = max(f, 2 fbar - f), since f(i) may lie on either
side of fbar; where the interval is a point (f(i) = fbar(i)) the output is
f(i), as for alpha_i = beta_i in Algorithm 1. I_0, I_1 come from the same
quadrature as the fast oracle (pinned against mpmath in
test_oracle_integrals.py); the ratio is in [0, 1], so clamping changes
nothing.
"""
from __future__ import annotations

import numpy as np

from .integrals import I_quadrature
from .spatial import canon, gather_windows, spatial_weights


def window_mean(f, kernel: str = "box", R: int = 3, sigma_s: float | None = None, pixels=None):
    """fbar: the spatially weighted window mean of f (FP64)."""
    f64 = canon(np.asarray(f, dtype=np.float32)).astype(np.float64)
    H, W = f64.shape
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
    else:
        ys, xs = np.asarray(pixels[0]), np.asarray(pixels[1])
    w = spatial_weights(kernel, R, sigma_s).ravel()
    out = np.empty(len(ys))
    step = max(1, (1 << 24) // ((2 * R + 1) ** 2))
    for s0 in range(0, len(ys), step):
        sl = slice(s0, min(len(ys), s0 + step))
        out[sl] = gather_windows(f64, R, ys[sl], xs[sl]) @ w
    return out.reshape(H, W) if pixels is None else out


def uniform_prior_abf(f, theta=None, sigma=None, kernel: str = "box", R: int = 3,
                      sigma_s: float | None = None, pixels=None):
    """g^ of the uniform-prior variant (module docstring); H x W, or 1-D at
    ``pixels`` = (ys, xs)."""
    f = canon(np.asarray(f, dtype=np.float32))
    H, W = f.shape
    th = f if theta is None else canon(np.asarray(theta, dtype=np.float32))
    sg = np.asarray(sigma, dtype=np.float64)
    if sg.ndim == 0:
        sg = np.full((H, W), float(sg))
    if pixels is None:
        ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
    else:
        ys, xs = np.asarray(pixels[0]), np.asarray(pixels[1])
    fbar = window_mean(f, kernel, R, sigma_s, pixels=(ys, xs))
    fi = f.astype(np.float64)[ys, xs]
    other = 2.0 * fbar - fi
    lo, hi = np.minimum(fi, other), np.maximum(fi, other)
    out = fi.copy()
    live = hi > lo
    if np.any(live):
        d = hi[live] - lo[live]
        t0 = (th.astype(np.float64)[ys[live], xs[live]] - lo[live]) / d
        s = sg[ys[live], xs[live]]
        lam = d * d / (2.0 * s * s)
        I, _ = I_quadrature(lam, t0, 1)
        out[live] = lo[live] + d * np.clip(I[:, 1] / I[:, 0], 0.0, 1.0)
    return out.reshape(H, W) if pixels is None else out
