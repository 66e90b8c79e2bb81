"""The range integrals of eq. (integrals), Sec. II-C:

    I_k(lambda, t0) = int_0^1 t^k exp(-lambda (t - t0)^2) dt,   k = 0..N+1.

Two evaluations of the same definite integrals:

``I_paper``       the paper's closed forms and recursion: eq. (I_0) with two
                  error functions, eq. (I_1), and the integration-by-parts
                  recursion eq. (F_forward). Exact in exact arithmetic; in
                  FP64 the recursion loses accuracy as lambda -> 0 because it
                  divides by 2 lambda.

``quad_rule``     composite Gauss-Legendre quadrature of the definition over
``I_quadrature``  the part of [0,1] where the Gaussian is not negligible.
``J_quadrature``  The Gaussian is scaled by exp(lambda d^2), d = dist(t0, [0,1]),
                  so that its largest value on [0,1] is 1; every returned
                  integral carries that common factor, which cancels in the
                  ratio of eq. (BFfinal). Accurate for every lambda >= 0 and
                  every t0; pinned against 50-digit ``mpmath.quad``.

``I_mpmath``      50-digit reference (tests only, slow).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


def I_paper(lam, t0, K: int) -> np.ndarray:
    """Eqs. (I_0), (I_1) and (F_forward) in FP64; returns shape (n, K+1).

    I_0 = 1/2 sqrt(pi/lam) [erf(sqrt(lam)(1-t0)) - erf(-sqrt(lam) t0)]
    I_1 = t0 I_0 + (exp(-lam t0^2) - exp(-lam (1-t0)^2)) / (2 lam)
    I_k = t0 I_{k-1} + (k-1)/(2 lam) I_{k-2} - exp(-lam (1-t0)^2)/(2 lam)
    """
    from scipy.special import erf
    lam = np.asarray(lam, dtype=np.float64)
    t0 = np.asarray(t0, dtype=np.float64)
    sl = np.sqrt(lam)
    out = np.empty(lam.shape + (K + 1,))
    e0 = np.exp(-lam * t0 * t0)
    e1 = np.exp(-lam * (1.0 - t0) ** 2)
    out[..., 0] = 0.5 * np.sqrt(np.pi / lam) * (erf(sl * (1.0 - t0)) - erf(-sl * t0))
    if K >= 1:
        out[..., 1] = t0 * out[..., 0] + (e0 - e1) / (2.0 * lam)
    for k in range(2, K + 1):
        out[..., k] = (t0 * out[..., k - 1] + (k - 1) / (2.0 * lam) * out[..., k - 2]
                       - e1 / (2.0 * lam))
    return out


@lru_cache(maxsize=None)
def _gl(q: int):
    x, w = np.polynomial.legendre.leggauss(q)
    return x, w


def quad_rule(lam, t0, panels: int = 8, q: int = 20):
    """Nodes and weights for int_0^1 g(t) psi~(t) dt, per pixel.

    psi~(t) = exp(-lam ((t - t0)^2 - d^2)), d = |t0 - clip(t0, 0, 1)|, so
    psi = exp(-lam d^2) psi~. The exponent is formed as
    lam (t - t*) (t + t* - 2 t0) with t* = clip(t0, 0, 1), which equals
    lam ((t-t0)^2 - d^2) without cancellation (nodes are generated as offsets
    s = t - t*, and the exponent is lam s (s + 2 (t* - t0))). The integral is restricted to
    the interval around t* where the exponent stays below 80 (the rest
    contributes less than e^-80 relative), split into ``panels`` equal
    panels of ``q`` Gauss-Legendre nodes each.

    Returns (t, wpsi, log_scale): t and wpsi of shape (n, panels*q) with
    wpsi = weight * psi~(t), and log_scale = lam d^2 (so that
    int g psi = exp(-log_scale) * sum wpsi g(t)).
    """
    lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
    t0 = np.atleast_1d(np.asarray(t0, dtype=np.float64))
    ts = np.clip(t0, 0.0, 1.0)
    d = np.abs(t0 - ts)
    with np.errstate(divide="ignore", invalid="ignore"):
        L = np.where(lam > 0, np.sqrt(d * d + 80.0 / np.where(lam > 0, lam, 1.0)) - d, np.inf)
    a = np.maximum(0.0, ts - L)
    b = np.minimum(1.0, ts + L)
    x, w = _gl(q)
    # panels are laid out as offsets s = t - t* so that a short interval next
    # to t* keeps full relative precision in s (and in the exponent)
    sa = np.maximum(-ts, -L)
    sb = np.minimum(1.0 - ts, L)
    edges = sa[:, None] + (sb - sa)[:, None] * (np.arange(panels + 1) / panels)[None, :]
    lo, hi = edges[:, :-1], edges[:, 1:]
    half = 0.5 * (hi - lo)
    s = (0.5 * (hi + lo))[:, :, None] + half[:, :, None] * x[None, None, :]
    wt = half[:, :, None] * w[None, None, :]
    s = s.reshape(len(lam), -1)
    wt = wt.reshape(len(lam), -1)
    expo = lam[:, None] * s * (s + 2.0 * (ts - t0)[:, None])
    return ts[:, None] + s, wt * np.exp(-expo), lam * d * d


def I_quadrature(lam, t0, K: int, panels: int = 8, q: int = 20):
    """Scaled I_k, k = 0..K: returns (I (n, K+1), log_scale) with
    I_k = exp(-log_scale) * I[:, k]."""
    t, wp, ls = quad_rule(lam, t0, panels, q)
    out = np.empty((t.shape[0], K + 1))
    tk = np.ones_like(t)
    for k in range(K + 1):
        out[:, k] = np.sum(wp * tk, axis=1)
        tk = tk * t
    return out, ls


def J_quadrature(lam, t0, N: int, panels: int = 8, q: int = 20):
    """Scaled Legendre-basis integrals J_k = int_0^1 P_k(2t-1) psi dt and
    Jt_k = int_0^1 t P_k(2t-1) psi dt, k = 0..N. These are fixed linear
    combinations of the I_k of eq. (integrals): J_k = sum_r ell_kr I_r,
    Jt_k = sum_r ell_kr I_{r+1}. Returns (J, Jt, log_scale)."""
    t, wp, ls = quad_rule(lam, t0, panels, q)
    x = 2.0 * t - 1.0
    J = np.empty((t.shape[0], N + 1))
    Jt = np.empty((t.shape[0], N + 1))
    p_prev, p = np.zeros_like(x), np.ones_like(x)
    for k in range(N + 1):
        J[:, k] = np.sum(wp * p, axis=1)
        Jt[:, k] = np.sum(wp * t * p, axis=1)
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return J, Jt, ls


def I_mpmath(lam: float, t0: float, K: int, dps: int = 50):
    """I_k by adaptive mpmath quadrature at ``dps`` digits (tests only).

    The integrand is multiplied by exp(lam d^2), d = dist(t0, [0,1]), inside
    the quadrature (mpmath's error control is absolute, so a tiny integrand
    would otherwise lose its relative accuracy) and the factor is divided out
    afterwards; [0,1] is split at t0 and at t0 +- m/sqrt(lam) so that narrow
    Gaussians are resolved."""
    import mpmath as mp
    with mp.workdps(dps):
        lam_, t0_ = mp.mpf(lam), mp.mpf(t0)
        ts = min(max(t0_, mp.mpf(0)), mp.mpf(1))
        sc = lam_ * (t0_ - ts) ** 2
        pts = {mp.mpf(0), mp.mpf(1)}
        if lam > 0:
            for m in (-8, -4, -2, -1, 1, 2, 4, 8):
                for c in (ts + m / mp.sqrt(2 * lam_), ts + m / (2 * lam_ * (abs(t0_ - ts) + 1))):
                    if 0 < c < 1:
                        pts.add(c)
        if 0 < t0 < 1:
            pts.add(t0_)
        pts = sorted(pts)
        vals = [mp.quad(lambda t, k=k: t ** k * mp.e ** (sc - lam_ * (t - t0_) ** 2), pts)
                for k in range(K + 1)]
        return [v * mp.e ** (-sc) for v in vals]
