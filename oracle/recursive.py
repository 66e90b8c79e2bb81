"""O(1)-per-pixel recursive approximation of the Gaussian spatial kernel.

Sec. II-D notes that the Gaussian convolutions of Algorithm 1 (the power
images of Prop. 2) can be computed with recursive filters whose cost does
not grow with the kernel width (Deriche; Young and van Vliet), while the
authors used direct convolution. This module is the CPU reference for such
a kernel, written from Deriche's fourth-order approximation of the Gaussian
(R. Deriche, "Recursively implementing the Gaussian and its derivatives",
INRIA research report 1893, 1993): for t >= 0

    g(t) = (a0 cos(w0 t/s) + a1 sin(w0 t/s)) e^(-b0 t/s)
         + (c0 cos(w1 t/s) + c1 sin(w1 t/s)) e^(-b1 t/s),      s = sigma_s,

with the published constants below (g(0) = 0.9997, |g - e^(-t^2/(2 s^2))| <
1e-3). The kernel used here is g(|j|) on the window j in [-R, R] only,
normalised to sum 1 per axis, so that, like the paper's Gaussian on
Omega = [-3 rho, 3 rho]^2, its weights vanish outside the (2R+1)^2 window
whose min and max are alpha_i and beta_i.

Each half of the 1-D filter is a sum of two complex first-order recursions:
with z_m = e^(-(b_m - i w_m)/s) and A_m = a_m - i a'_m (a'_0 = a1, a'_1 = c1),

    sum_{j=0}^{R} g(j) u(x - j) = Re sum_m A_m q_m(x),
    q_m(x) = z_m q_m(x - 1) + u(x) - z_m^(R+1) u(x - R - 1),

where the last term removes the sample that leaves the truncated window,
so every output costs O(1) for any R (the anticausal half, j < 0, is the
same recursion run backwards). ``deriche_weights_1d`` is the definition;
``recursive_filter_1d`` the recursion; the tests pin one against the other
and the weights against the sampled Gaussian. Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

# Deriche's coefficients for the Gaussian (order 0)
A0, A1, B0, W0 = 1.680, 3.735, 1.783, 0.6318
C0, C1, B1, W1 = -0.6803, -0.2598, 1.723, 1.997


def _poles(sigma_s: float):
    z = np.array([np.exp(-(B0 - 1j * W0) / sigma_s), np.exp(-(B1 - 1j * W1) / sigma_s)])
    A = np.array([A0 - 1j * A1, C0 - 1j * C1])
    return z, A


def deriche_profile(t, sigma_s: float):
    """g(|t|) of the module docstring (unnormalised)."""
    t = np.abs(np.asarray(t, dtype=np.float64)) / sigma_s
    return ((A0 * np.cos(W0 * t) + A1 * np.sin(W0 * t)) * np.exp(-B0 * t) +
            (C0 * np.cos(W1 * t) + C1 * np.sin(W1 * t)) * np.exp(-B1 * t))


def deriche_weights_1d(R: int, sigma_s: float | None = None) -> np.ndarray:
    """The kernel's 1-D weights on j = -R..R, normalised to sum 1
    (sigma_s <= 0 or None means R/3, as for the Gaussian kernel)."""
    s = (R / 3.0) if (sigma_s is None or sigma_s <= 0) else float(sigma_s)
    s = s if s > 0 else 1.0
    w = deriche_profile(np.arange(-R, R + 1), s)
    return w / w.sum()


def recursive_filter_1d(u: np.ndarray, R: int, sigma_s: float | None = None, axis: int = -1):
    """sum_{|j| <= R} w_j u(x - j) along ``axis`` (clamp-to-edge borders,
    w = deriche_weights_1d) by the truncated first-order recursions, FP64."""
    s = (R / 3.0) if (sigma_s is None or sigma_s <= 0) else float(sigma_s)
    s = s if s > 0 else 1.0
    z, A = _poles(s)
    norm = deriche_profile(np.arange(-R, R + 1), s).sum()
    u = np.moveaxis(np.asarray(u, dtype=np.float64), axis, -1)
    n = u.shape[-1]
    pad = np.concatenate([np.repeat(u[..., :1], R + 1, axis=-1), u,
                          np.repeat(u[..., -1:], R + 1, axis=-1)], axis=-1)   # clamp-to-edge
    L = pad.shape[-1]
    causal = np.zeros(u.shape[:-1] + (n,))
    anti = np.zeros(u.shape[:-1] + (n,))
    for m in range(2):
        zr = z[m] ** (R + 1)
        # causal: q(x) = z q(x-1) + u(x) - z^(R+1) u(x-R-1), from the first padded sample
        q = np.zeros(u.shape[:-1], dtype=np.complex128)
        qs = np.empty(u.shape[:-1] + (L,), dtype=np.complex128)
        for x in range(L):
            q = z[m] * q + pad[..., x] - (zr * pad[..., x - R - 1] if x >= R + 1 else 0.0)
            qs[..., x] = q
        causal += np.real(A[m] * qs[..., R + 1:R + 1 + n])
        # anticausal, j = 1..R: p(x) = z p(x+1) + u(x+1) - z^R u(x+R+1)
        zr1 = z[m] ** R
        p = np.zeros(u.shape[:-1], dtype=np.complex128)
        ps = np.empty(u.shape[:-1] + (L,), dtype=np.complex128)
        for x in range(L - 1, -1, -1):
            nxt = pad[..., x + 1] if x + 1 < L else 0.0
            far = pad[..., x + R + 1] if x + R + 1 < L else 0.0
            p = z[m] * p + nxt - zr1 * far
            ps[..., x] = p
        anti += np.real(A[m] * z[m] * ps[..., R + 1:R + 1 + n])
    return np.moveaxis((causal + anti) / norm, -1, axis)


def recursive_power_sums(f: np.ndarray, R: int, sigma_s: float | None, N: int, origin: float):
    """m_k = omega * (f - origin)^k, k = 0..N, omega the 2-D separable kernel,
    each by the recursion along rows then columns, FP64 (the form a
    recursive GPU pass would take: one origin for every window)."""
    u = np.asarray(f, dtype=np.float64) - origin
    out = []
    p = np.ones_like(u)
    for _ in range(N + 1):
        out.append(recursive_filter_1d(recursive_filter_1d(p, R, sigma_s, axis=1), R, sigma_s,
                                       axis=0))
        p = p * u
    return out
