"""Algorithm 1 (Sec. II-D): the fast adaptive bilateral filter, two routes.

``fast_abf``          value of record. It takes Algorithm 1's steps in order,
                      with every step evaluated so that FP64 rounding stays
                      far below the 1e-6 parity bound:
    1. alpha_i, beta_i = window min/max (eq. bounds, Algorithm 1);
       pixels with alpha_i = beta_i output f(i) (Algorithm 1's flat-window case).
    2. the moments of the stretched histogram H_i (eqs. Lambda_tilde, mhist,
       hist_moments_new), taken directly from the window. Props. 2 and 3
       reach the same mu_k through convolutions and a binomial shift; the
       direct sum is that result without the cancellation of the shift.
       They are kept as shifted-Legendre moments
       a~_k = sum_j omega_j P_k(2 y_j - 1) = sum_r ell_kr mu_r.
    3. c = A^-1 mu (eq. inv). Because A^-1 = sum_k (2k+1) ell_k
       ell_k^T (an exact integer identity, pinned in tests),
       c = sum_k (2k+1) a~_k ell_k.
    4. t0 = (theta - alpha)/(beta - alpha), lambda = (beta-alpha)^2/(2 sigma^2)
       (eq. sub).
    5. T1 = sum_k c_k I_{k+1}, T2 = sum_k c_k I_k (Algorithm 1) and
       g^ = alpha + (beta - alpha) T1/T2 (eq. BFfinal). With c from step 3
       these sums equal sum_k (2k+1) a~_k Jt_k and sum_k (2k+1) a~_k J_k,
       where J_k, Jt_k are the Legendre-basis combinations of the I_k,
       evaluated by accurate quadrature of the definite integrals
       (``integrals.J_quadrature``).
    6. post-rules for what the paper leaves open (it drops the
       non-negativity of the fitted polynomial, Sec. II-B): if T2 <= 0 or
       the ratio is not finite, use I_1/I_0 (the N = 0 estimate); with
       ``clamp`` (default) the ratio is clipped to [0, 1], i.e. g^ to
       [alpha, beta].

``fast_abf_literal``  the same algorithm exactly as printed, in FP64: f
                      rescaled to [0,1] (Sec. III), gamma_k = omega * f^k by
                      convolution (Prop. 2), the binomial shift of
                      Prop. 3, c = A^-1 mu with the integer A^-1 of eq. (inv),
                      I_0, I_1 and the forward recursion (eqs. I_0, I_1,
                      F_forward). It shows the precision the paper's own
                      evaluation order reaches; it is not the value of
                      record.

Working range: the paper runs on f/255 with sigma/255 (Sec. III). The
method is exactly equivariant under f -> a f + b, theta -> a theta + b,
sigma -> |a| sigma (alpha, beta move affinely; mu, c, t0, lambda do not
change), so ``fast_abf`` works in the input's own units.
"""
from __future__ import annotations

import numpy as np

from .hilbert import hilbert_inverse, shifted_legendre
from .integrals import I_paper, J_quadrature
from .spatial import (canon, convolve_powers, gather_windows, legendre_moments,
                      spatial_weights, window_minmax)
from math import comb


def _all_pixels(H, W):
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    return ys.ravel(), xs.ravel()


def fast_abf(f, theta=None, sigma=None, kernel: str = "box", R: int = 3, N: int = 5,
             sigma_s: float | None = None, clamp: bool = True, pixels=None,
             chunk: int = 8192, aux: bool = False):
    """Value-of-record fast ABF (see module docstring). ``f``, ``theta``,
    ``sigma``: H x W arrays (theta None means theta = f). ``pixels``: optional
    (ys, xs) index arrays to evaluate only those outputs. Returns FP64 values
    (H x W, or 1-D for ``pixels``); with ``aux`` also a dict of per-pixel
    intermediates (alpha, beta, legendre moments, t0, lam, T1, T2, flags)."""
    f = canon(np.asarray(f, dtype=np.float32))
    H, W = f.shape
    th = f if theta is None else canon(np.asarray(theta, dtype=np.float32))
    sg = np.asarray(sigma, dtype=np.float64)
    if sg.ndim == 0:
        sg = np.full((H, W), float(sg))
    ys, xs = _all_pixels(H, W) if pixels is None else (np.asarray(pixels[0]), np.asarray(pixels[1]))
    w = spatial_weights(kernel, R, sigma_s).ravel()
    f64 = f.astype(np.float64)
    n = len(ys)
    out = np.empty(n)
    extra = {k: np.empty(n) for k in ("alpha", "beta", "t0", "lam", "T1", "T2")} if aux else None
    if aux:
        extra["amom"] = np.zeros((n, N + 1))
        extra["fallback"] = np.zeros(n, dtype=bool)
    step = max(1, min(chunk, (1 << 24) // ((2 * R + 1) ** 2)))
    for s0 in range(0, n, step):
        sl = slice(s0, min(n, s0 + step))
        py, px = ys[sl], xs[sl]
        win = gather_windows(f64, R, py, px)
        alpha = win.min(axis=1)
        beta = win.max(axis=1)
        res = f64[py, px].copy()
        live = alpha != beta
        if aux:
            extra["alpha"][sl], extra["beta"][sl] = alpha, beta
            for k in ("t0", "lam", "T1", "T2"):
                extra[k][sl] = np.nan
        if np.any(live):
            a_, b_ = alpha[live], beta[live]
            delta = b_ - a_
            am = legendre_moments(win[live], w, a_, b_, N)           # a~_k
            coef = am * (2.0 * np.arange(N + 1) + 1.0)[None, :]     # (2k+1) a~_k
            t0 = (th[py[live], px[live]].astype(np.float64) - a_) / delta
            sgl = sg[py[live], px[live]]
            lam = delta * delta / (2.0 * sgl * sgl)
            J, Jt, _ = J_quadrature(lam, t0, N)
            T2 = np.sum(coef * J, axis=1)
            T1 = np.sum(coef * Jt, axis=1)
            with np.errstate(divide="ignore", invalid="ignore"):
                F = T1 / T2
            bad = ~np.isfinite(F) | (T2 <= 0)
            F = np.where(bad, Jt[:, 0] / J[:, 0], F)
            if clamp:
                F = np.clip(F, 0.0, 1.0)
            res[live] = a_ + delta * F
            if aux:
                idx = np.arange(s0, sl.stop)[live]
                extra["amom"][idx] = am
                extra["t0"][idx], extra["lam"][idx] = t0, lam
                extra["T1"][idx], extra["T2"][idx] = T1, T2
                extra["fallback"][idx] = bad
        out[sl] = res
    if pixels is None:
        out = out.reshape(H, W)
        if aux:
            for k, v in extra.items():
                extra[k] = v.reshape((H, W) + v.shape[1:])
    return (out, extra) if aux else out


def fast_abf_literal(f, theta=None, sigma=None, kernel: str = "box", R: int = 3,
                     N: int = 5, sigma_s: float | None = None):
    """Algorithm 1 as printed, FP64 (see module docstring). No post-rules."""
    f = canon(np.asarray(f, dtype=np.float32)).astype(np.float64)
    th = f if theta is None else canon(np.asarray(theta, dtype=np.float32)).astype(np.float64)
    sg = np.broadcast_to(np.asarray(sigma, dtype=np.float64), f.shape)
    u, tu, su = f / 255.0, th / 255.0, sg / 255.0                  # Sec. III rescale
    alpha, beta = window_minmax(u, R)                               # eq. bounds
    Ainv = np.array(hilbert_inverse(N), dtype=np.float64)          # eq. inv
    gam = convolve_powers(u, kernel, R, sigma_s, N)                 # Prop. 2
    live = alpha != beta                                            # flat windows
    out = f.copy()                                                  # keep f(i) there
    a, b = alpha[live], beta[live]
    d = b - a
    m = [g[live] for g in gam]
    mu = np.empty((N + 1, a.size))
    for k in range(N + 1):                                          # Prop. 3
        acc = np.zeros(a.size)
        for r in range(k + 1):
            acc += comb(k, r) * (-a) ** (k - r) * m[r]
        mu[k] = acc / d ** k
    c = Ainv @ mu                                                   # eq. inv
    t0 = (tu[live] - a) / d                                         # eq. sub
    lam = 0.5 * d * d / (su[live] ** 2)                            # eq. sub
    I = I_paper(lam, t0, N + 1)                                     # eqs. I_0, I_1, F_forward
    T1 = np.sum(c.T * I[:, 1:], axis=1)
    T2 = np.sum(c.T * I[:, :-1], axis=1)
    out[live] = 255.0 * (a + d * T1 / T2)
    return out


def legendre_to_monomial(N: int) -> np.ndarray:
    """The (N+1) x (N+1) integer matrix ell (row k: coefficients of P_k(2t-1))."""
    return np.array(shifted_legendre(N), dtype=np.float64)
