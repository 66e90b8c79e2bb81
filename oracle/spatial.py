"""Spatial-stage definitions: windows, bounds, weights and moments.

Border rule: the paper does not say how windows that cross the image border
are treated. It states that gamma_0 = omega * f^0 equals 1 everywhere
(Sec. II-D), which rules out zero padding; we read the window as
clamp-to-edge (replicate) in every stage, brute force included.

Window: the API radius R gives Omega = [-R, R]^2. For the Gaussian kernel of
eq. (sp_kernel) the paper uses Omega = [-3 rho, 3 rho]^2; our Gaussian weight
has its own width sigma_s (default R/3, which reproduces that window).
Weights are normalised to sum to one (gamma_0 = 1).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def canon(a: np.ndarray) -> np.ndarray:
    """-0.0 -> +0.0 (x + 0.0), so that equal values compare and hash equal."""
    return np.asarray(a) + np.asarray(0.0, dtype=np.asarray(a).dtype)


def spatial_weights_1d(kind: str, R: int, sigma_s: float | None = None) -> np.ndarray:
    """1-D factor of the separable spatial kernel on [-R, R], normalised.

    box:       constant (the paper allows any spatial kernel, Sec. I and V).
    gaussian:  exp(-j^2 / (2 sigma_s^2)), eq. (sp_kernel), sigma_s = R/3 by
               default.
    recursive: Deriche's sum-of-exponentials approximation of that Gaussian
               (Sec. II-D's recursive option), truncated to [-R, R]
               (oracle.recursive).
    """
    j = np.arange(-R, R + 1, dtype=np.float64)
    if kind == "box":
        w = np.ones_like(j)
    elif kind == "gaussian":
        s = (R / 3.0) if (sigma_s is None or sigma_s <= 0) else float(sigma_s)
        w = np.exp(-(j * j) / (2.0 * s * s))
    elif kind == "recursive":
        # Deriche's recursive approximation of the Gaussian, truncated to the
        # window (oracle.recursive); sigma_s as for the Gaussian
        from .recursive import deriche_weights_1d
        return deriche_weights_1d(R, sigma_s)
    else:
        raise ValueError(kind)
    return w / w.sum()


def spatial_weights(kind: str, R: int, sigma_s: float | None = None) -> np.ndarray:
    """2-D weights omega(j) on Omega = [-R, R]^2 (outer product of 1-D factors,
    which for the Gaussian is exp(-||j||^2 / (2 sigma_s^2)) up to the
    normalising constant)."""
    w1 = spatial_weights_1d(kind, R, sigma_s)
    return np.outer(w1, w1)


def padded(f: np.ndarray, R: int) -> np.ndarray:
    return np.pad(np.asarray(f), R, mode="edge")


def window_minmax(f: np.ndarray, R: int):
    """Eq. (bounds): alpha_i, beta_i = min, max of f over the window of i.

    The min over a rectangle is the min over its rows of the min over each
    row, so the definition is evaluated as two 1-D sliding minima (exact: no
    arithmetic, only comparisons). Returns float arrays of f's dtype.
    """
    f = canon(np.asarray(f))
    p = padded(f, R)
    h = sliding_window_view(p, 2 * R + 1, axis=1)          # (H+2R, W, 2R+1)
    hmin, hmax = h.min(axis=-1), h.max(axis=-1)
    vmin = sliding_window_view(hmin, 2 * R + 1, axis=0).min(axis=-1)
    vmax = sliding_window_view(hmax, 2 * R + 1, axis=0).max(axis=-1)
    return vmin, vmax


def gather_windows(f: np.ndarray, R: int, ys: np.ndarray, xs: np.ndarray) -> np.ndarray:
    """Windows (clamp-to-edge) of the pixels (ys[n], xs[n]), flattened row-major
    to shape (n, (2R+1)^2), in float64."""
    p = padded(np.asarray(f, dtype=np.float64), R)
    dy, dx = np.meshgrid(np.arange(2 * R + 1), np.arange(2 * R + 1), indexing="ij")
    return p[ys[:, None] + dy.ravel()[None, :], xs[:, None] + dx.ravel()[None, :]]


def stretched_moments(win: np.ndarray, w: np.ndarray, alpha, beta, N: int) -> np.ndarray:
    """Eq. (hist_moments_new): mu_k = sum_t t^k H_i(t) = sum_j omega_j y_j^k,
    where y_j = (f(i-j) - alpha_i) / (beta_i - alpha_i) (eqs. Lambda_tilde,
    mhist). ``win``: (n, |Omega|) window values; returns (n, N+1)."""
    y = (win - alpha[:, None]) / (beta - alpha)[:, None]
    out = np.empty((win.shape[0], N + 1))
    yk = np.ones_like(y)
    for k in range(N + 1):
        out[:, k] = yk @ w
        yk = yk * y
    return out


def legendre_moments(win: np.ndarray, w: np.ndarray, alpha, beta, N: int) -> np.ndarray:
    """a~_k = sum_j omega_j P_k(2 y_j - 1) = sum_r ell_kr mu_r (shifted Legendre
    moments of the stretched histogram), k = 0..N; returns (n, N+1).

    P_k is evaluated with the three-term recurrence
    (k+1) P_{k+1}(x) = (2k+1) x P_k(x) - k P_{k-1}(x)."""
    x = 2.0 * (win - alpha[:, None]) / (beta - alpha)[:, None] - 1.0
    out = np.empty((win.shape[0], N + 1))
    p_prev, p = np.zeros_like(x), np.ones_like(x)
    for k in range(N + 1):
        out[:, k] = p @ w
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return out


def convolve_powers(u: np.ndarray, kind: str, R: int, sigma_s, N: int):
    """Prop. 2 / Algorithm 1, convolution line: gamma_k = omega * u^k for
    k = 0..N with clamp-to-edge borders (the kernel is symmetric, so
    correlation and convolution coincide). Separable, FP64."""
    from scipy.ndimage import correlate1d
    w1 = spatial_weights_1d(kind, R, sigma_s)
    out = []
    uk = np.ones_like(u, dtype=np.float64)
    for k in range(N + 1):
        g = correlate1d(uk, w1, axis=1, mode="nearest")
        g = correlate1d(g, w1, axis=0, mode="nearest")
        out.append(g)
        uk = uk * u
    return out


def local_std_sigma(f: np.ndarray, r: int = 4, scale: float = 3.0, lo: float = 5.0,
                    hi: float = 80.0) -> np.ndarray:
    """sigma(i) = clip(scale * sd(i), lo, hi), sd(i) the population standard
    deviation of f over the clamp-to-edge window [-r, r]^2 of i (the contrast
    rule of the texture benchmark; the paper's texture filter maps a local
    texture measure to sigma, Sec. IV-C). FP64."""
    f = np.asarray(f, dtype=np.float64)
    H, W = f.shape
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    out = np.empty(H * W)
    yr, xr = ys.ravel(), xs.ravel()
    step = 1 << 15
    for s0 in range(0, H * W, step):
        win = gather_windows(f, r, yr[s0:s0 + step], xr[s0:s0 + step])
        out[s0:s0 + step] = np.clip(scale * win.std(axis=1), lo, hi)
    return out.reshape(H, W)
